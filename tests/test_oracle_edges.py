"""Pins of the oracle's edge-sampling terms against deterministic integrals.

Edge sampling estimates the part of a gradient that comes from visibility
discontinuities moving (the Face Modeling paragraph uses a differentiable ray
tracer with this property).  Ground truth here is a central finite
difference of the exact integral, computed without Monte Carlo:

* camera silhouettes: the whole-image integral of the radiance of one lit
  triangle = polygon clip of its projection against the image rectangle and
  Gauss quadrature of Lambert's polygon irradiance over it; the mean of the
  interior + camera-silhouette estimator over many seeds must match its
  derivative with respect to every vertex coordinate;
* shadow boundaries: one narrow pixel sees one receiver point; its radiance
  is Lambert's formula over the light polygon minus the occluder's central
  projection; derivatives with respect to the occluder's vertices (shadow
  term only) and to a rigid motion of the receiver (interior + shadow term,
  through the shading point) must match.
"""
import math

import numpy as np
import pytest

from paper_1910_05200_amd import synth
import closed_forms as cf

N_SEEDS = 400


def _mesh(tris, albedo):
    tri = np.asarray(tris, np.float64)
    pos = np.ascontiguousarray(tri.reshape(-1, 3).T.astype(np.float32))
    faces = np.arange(tri.shape[0] * 3, dtype=np.int32).reshape(-1, 3)
    alb = np.full((3, pos.shape[1]), albedo, np.float32)
    return synth.Mesh(pos, faces, alb, np.full((2, pos.shape[1]), 0.5, np.float32))


def _tri_gauss(P, n=12):
    """Gauss points/weights on triangle P (3x2) via the collapsed square."""
    z, w = np.polynomial.legendre.leggauss(n)
    z = (z + 1) / 2
    w = w / 2
    u, v = np.meshgrid(z, z, indexing="ij")
    wu, wv = np.meshgrid(w, w, indexing="ij")
    P0, P1, P2 = (np.asarray(p, float) for p in P)
    pts = P0 + u[..., None] * (P1 - P0) + (u * v)[..., None] * (P2 - P1)
    e, f = P1 - P0, P2 - P1
    jac = abs(e[0] * f[1] - e[1] * f[0])
    return pts.reshape(-1, 2), (wu * wv * u * jac).ravel()


def _clip_rect(poly, W, H):
    """Clip a 2D polygon to [0, W] x [0, H]."""
    def clip(pts, inside, inter):
        out = []
        for i in range(len(pts)):
            p, q = pts[i], pts[(i + 1) % len(pts)]
            if inside(p):
                out.append(p)
            if inside(p) != inside(q):
                out.append(inter(p, q))
        return out
    pts = [np.asarray(p, float) for p in poly]
    for ax, lim, keep_low in ((0, 0.0, False), (0, W, True), (1, 0.0, False), (1, H, True)):
        if not pts:
            break
        def inside(p, ax=ax, lim=lim, keep_low=keep_low):
            return p[ax] <= lim if keep_low else p[ax] >= lim
        def inter(p, q, ax=ax, lim=lim):
            t = (lim - p[ax]) / (q[ax] - p[ax])
            return p + t * (q - p)
        pts = clip(pts, inside, inter)
    return pts


def _image_integral(tri, light, rgb, albedo, W, H, cam, ps):
    """Exact sum over pixels of the box-filtered radiance of one triangle."""
    cam = np.asarray(cam, float)
    tri = np.asarray(tri, float)
    n = np.cross(tri[1] - tri[0], tri[2] - tri[0])
    n /= np.linalg.norm(n)
    if n @ (cam - tri[0]) < 0:
        n = -n
    scr = []
    for x in tri:
        r = x - cam
        scr.append([W / 2 + (r[0] / -r[2]) / ps, H / 2 - (r[1] / -r[2]) / ps])
    poly = _clip_rect(scr, W, H)
    corners = cf.quad_corners(light)
    total = 0.0
    for k in range(1, len(poly) - 1):
        pts, wts = _tri_gauss([poly[0], poly[k], poly[k + 1]])
        for (qx, qy), w in zip(pts, wts):
            d = np.array([(qx - W / 2) * ps, (H / 2 - qy) * ps, -1.0])
            t = ((tri[0] - cam) @ n) / (d @ n)
            x = cam + t * d
            total += w * albedo / math.pi * cf.projected_solid_angle(x, n, corners)
    return total * np.asarray(rgb, float)


def test_camera_silhouette_term_matches_fd_of_exact_integral(orc):
    W = H = 16
    ps = np.float32(0.01)
    cam = np.array([0.0, 0.0, 0.5])
    tri = np.array([[-0.021, -0.016, 0.0], [0.026, -0.011, 0.004], [0.002, 0.022, -0.003]], np.float32)
    light = synth.quad_light([0.05, 0.03, 0.4], [0.2, 0, 0], [0, -0.2, 0])
    rgb = np.array([[0.9, 0.6, 0.3]])
    rho = 0.7
    osc = orc.scene_from_mesh(_mesh([tri], rho), W, H, cam, ps, light, rgb, np.zeros(1024))
    dL = np.ones((H, W, 3))
    samples = []
    for s in range(N_SEEDS):
        g = orc.backward(osc, 5000 + s, 1, dL, flags=orc.FLAG_INTERIOR | orc.FLAG_PRIMARY, threads=1)
        samples.append(g["d_pos"].copy())
    samples = np.array(samples)
    mean, sem = samples.mean(0), samples.std(0, ddof=1) / math.sqrt(N_SEEDS)
    # ground truth: d/dv of sum_c integral_c (all channels weighted 1)
    h = 1e-6
    tri64 = tri.astype(np.float64)
    worst = 0.0
    for k in range(3):
        for c in range(3):
            tp, tm = tri64.copy(), tri64.copy()
            tp[k, c] += h
            tm[k, c] -= h
            fd = (_image_integral(tp, light, rgb[0], rho, W, H, cam, float(ps)).sum()
                  - _image_integral(tm, light, rgb[0], rho, W, H, cam, float(ps)).sum()) / (2 * h)
            z = abs(mean[c, k] - fd) / sem[c, k]
            worst = max(worst, z)
            assert z < 5.0, (k, c, mean[c, k], fd, sem[c, k])
    # the silhouette term carries the gradient: without it the x/y
    # derivatives of the covered area are badly wrong
    g0 = np.mean([orc.backward(osc, 5000 + s, 1, dL, flags=orc.FLAG_INTERIOR, threads=1)["d_pos"]
                  for s in range(20)], axis=0)
    assert np.abs(g0 - mean).max() > 20 * sem.max()


def _visible_phi(x, n, light, occ):
    corners = cf.quad_corners(light)
    phi = cf.projected_solid_angle(x, n, corners)
    lp, ln = np.asarray(light[:3], float), np.asarray(light[9:12], float)
    sh = cf.clip_convex(cf.project_to_plane(x, occ, lp, ln), corners)
    if len(sh) >= 3:
        phi -= cf.projected_solid_angle(x, n, sh)
    return phi


def test_shadow_boundary_term_matches_fd_of_clipped_lambert(orc):
    cam = np.array([0.0, 0.0, 0.5])
    ps = np.float32(1e-7)
    light = synth.quad_light([0.35, 0.0, 0.6], [0.15, 0, 0], [0, -0.15, 0])
    occ = np.array([[0.15, -0.05, 0.3], [0.21, 0.06, 0.31], [0.16, 0.04, 0.33]], np.float32)
    rec = np.array([[[-0.01, -0.01, 0.0], [0.01, -0.01, 0.0], [0.01, 0.01, 0.0]],
                    [[-0.01, -0.01, 0.0], [0.01, 0.01, 0.0], [-0.01, 0.01, 0.0]]], np.float32)
    rho, l = 0.8, np.array([[1.0, 1.0, 1.0]])
    osc = orc.scene_from_mesh(_mesh([rec[0], rec[1], occ], rho), 1, 1, cam, ps, light, l, np.zeros(1024))
    x0 = np.zeros(3)
    nz = np.array([0, 0, 1.0])
    # the occluder really half-shadows the point
    full = cf.projected_solid_angle(x0, nz, cf.quad_corners(light))
    vis = _visible_phi(x0, nz, light, occ.astype(float))
    assert 0.2 * full < vis < 0.9 * full
    spp = 4096
    dL = np.ones((1, 1, 3))
    gs, gi = [], []
    for s in range(N_SEEDS // 4):
        g = orc.backward(osc, 7000 + s, spp, dL, flags=orc.FLAG_INTERIOR | orc.FLAG_SECONDARY, threads=4)
        gs.append(g["d_pos_secondary"].copy())
        gi.append(g["d_pos_interior"].copy())
    gs, gi = np.array(gs), np.array(gi)
    n = gs.shape[0]
    mean, sem = gs.mean(0), gs.std(0, ddof=1) / math.sqrt(n)
    h = 1e-6
    occ64 = occ.astype(np.float64)
    for k in range(3):
        for c in range(3):
            op, om = occ64.copy(), occ64.copy()
            op[k, c] += h
            om[k, c] -= h
            fd = 3 * rho / math.pi * (_visible_phi(x0, nz, light, op) - _visible_phi(x0, nz, light, om)) / (2 * h)
            vi = 6 + k
            z = abs(mean[c, vi] - fd) / max(sem[c, vi], 1e-12)
            assert z < 5.0, (k, c, mean[c, vi], fd, sem[c, vi])
    # rigid lift of the receiver along z: the shading point slides along the
    # camera ray; interior and shadow terms together give the derivative
    tot = gs + gi
    lift = tot[:, 2, :6].sum(axis=1)
    m, se = lift.mean(), lift.std(ddof=1) / math.sqrt(n)
    e = np.array([0, 0, h])
    fd = 3 * rho / math.pi * (_visible_phi(x0 + e, nz, light, occ64) - _visible_phi(x0 - e, nz, light, occ64)) / (2 * h)
    assert abs(m - fd) < 5 * se + 1e-6 * abs(fd), (m, fd, se)
