"""Closed forms and deterministic quadratures used to pin the oracle.

None of this shares arithmetic with the estimator: irradiance comes from
Lambert's polygon formula (Lambert 1760, in the vector form given by Arvo,
"Applications of Irradiance Tensors", SIGGRAPH 1995), visible parts of a
light from convex polygon clipping (Sutherland-Hodgman 1974), and pixel
integrals from tensor Gauss-Legendre quadrature.
"""
from __future__ import annotations

import math

import numpy as np


def projected_solid_angle(x, n, poly) -> float:
    """Integral of cos(theta) d(omega) over a planar polygon seen from x.

    Lambert: Phi = 1/2 * sum_k Theta_k (n . g_k), Theta_k the angle between
    consecutive vertex directions and g_k the unit normal of their plane.
    The polygon must lie entirely above x's tangent plane.
    """
    x = np.asarray(x, float)
    n = np.asarray(n, float)
    u = [np.asarray(p, float) - x for p in poly]
    u = [a / np.linalg.norm(a) for a in u]
    tot = 0.0
    for k in range(len(u)):
        a, b = u[k], u[(k + 1) % len(u)]
        c = np.cross(a, b)
        s = np.linalg.norm(c)
        if s == 0:
            continue
        theta = math.atan2(s, float(a @ b))
        tot += theta * float(n @ (c / s))
    return abs(0.5 * tot)


def clip_convex(subject, clip):
    """Sutherland-Hodgman: subject polygon clipped by a convex polygon, both
    planar and coplanar (3D points); returns the intersection polygon."""
    clip = [np.asarray(p, float) for p in clip]
    nrm = np.cross(clip[1] - clip[0], clip[2] - clip[0])
    out = [np.asarray(p, float) for p in subject]
    for k in range(len(clip)):
        a, b = clip[k], clip[(k + 1) % len(clip)]
        inward = np.cross(nrm, b - a)            # points into the clip polygon
        inp, out = out, []
        if not inp:
            break
        for i in range(len(inp)):
            p, q = inp[i], inp[(i + 1) % len(inp)]
            dp, dq = float((p - a) @ inward), float((q - a) @ inward)
            if dp >= 0:
                out.append(p)
            if (dp >= 0) != (dq >= 0):
                t = dp / (dp - dq)
                out.append(p + t * (q - p))
    return out


def quad_corners(geom):
    g = np.asarray(geom, float)
    c, e1, e2 = g[0:3], g[3:6], g[6:9]
    return [c - e1 / 2 - e2 / 2, c + e1 / 2 - e2 / 2, c + e1 / 2 + e2 / 2, c - e1 / 2 + e2 / 2]


def project_to_plane(x, pts, plane_point, plane_normal):
    """Central projection from x of points onto a plane."""
    x = np.asarray(x, float)
    out = []
    for p in pts:
        d = np.asarray(p, float) - x
        t = float((plane_point - x) @ plane_normal) / float(d @ plane_normal)
        out.append(x + t * d)
    return out


def gauss_pixel(px, py, n=8):
    """Gauss-Legendre nodes/weights over the unit pixel square at (px, py)."""
    z, w = np.polynomial.legendre.leggauss(n)
    z = (z + 1) / 2
    w = w / 2
    pts = [(px + a, py + b, wa * wb) for a, wa in zip(z, w) for b, wb in zip(z, w)]
    return pts


def camera_plane_point(qx, qy, W, H, cam, ps, z0):
    """Where the pinhole ray through screen point (qx, qy) meets plane z = z0."""
    d = np.array([(qx - W / 2) * ps, (H / 2 - qy) * ps, -1.0])
    t = (z0 - cam[2]) / d[2]
    return np.asarray(cam, float) + t * d
