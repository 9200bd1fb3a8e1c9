"""Pins of the oracle's auxiliary buffers (the denoiser's albedo, normal and
depth inputs) against closed forms.

A plane seen through a pinhole has every quantity in closed form for each
camera sample: the sample's screen point comes from the Philox words (pinned
against the published known-answer vectors), its hit point is where the
pixel ray meets the plane, the albedo is a linear ramp across the plane
(which barycentric interpolation reproduces exactly), the normal is the
plane's, turned toward the camera, and the depth is the hit point's distance
from the pinhole.  Pixels whose samples all miss must read zero.
"""
import math

import numpy as np
import pytest

from paper_1910_05200_amd import synth


def _u01(w):
    return np.float32(int(w) >> 8) * np.float32(1.0 / 16777216.0)


def _plane_scene(orc, W, H, ps, cam_z, rot_deg, flip, shift_x, ramp):
    mesh = synth.flat_grid(9, 0.05, z=0.0)
    pos = mesh.pos.astype(np.float64)
    pos[0] += shift_x
    # albedo ramp along the plane's own x axis
    alb = np.stack([ramp[c][0] + ramp[c][1] * pos[0] for c in range(3)])
    a = math.radians(rot_deg)
    R = np.array([[1, 0, 0], [0, math.cos(a), -math.sin(a)], [0, math.sin(a), math.cos(a)]])
    pos = R @ pos
    pos[2] -= 0.05
    faces = mesh.faces[:, ::-1].copy() if flip else mesh.faces
    m = synth.Mesh(np.ascontiguousarray(pos.astype(np.float32)), np.ascontiguousarray(faces),
                   alb.astype(np.float32), mesh.uv)
    light = synth.quad_light([0.0, 0.0, 0.6], [0.1, 0, 0], [0, -0.1, 0])
    osc = orc.scene_from_mesh(m, W, H, [0, 0, cam_z], ps, light, [[1.0, 1.0, 1.0]], np.zeros(1024))
    n = R @ np.array([0, 0, 1.0])
    return osc, m, R, n


@pytest.mark.parametrize("rot_deg,flip,shift_x", [(0.0, False, 0.0), (20.0, False, 0.0), (-25.0, True, 0.0),
                                                  (10.0, False, -0.06)])
def test_aov_plane_closed_form(orc, rot_deg, flip, shift_x):
    W, H, ps, spp, seed, cam_z = 12, 10, np.float32(0.01), 3, 77, 0.5
    ramp = [(0.5, 2.0), (0.3, -1.0), (0.2, 0.5)]
    osc, mesh, R, n = _plane_scene(orc, W, H, ps, cam_z, rot_deg, flip, shift_x, ramp)
    got = orc.aov(osc, seed, spp)
    cam = np.array([0, 0, cam_z], float)
    plane_pt = R @ np.array([0, 0, 0.0]) + np.array([0, 0, -0.05])
    # plane extent in its own x (after the shift) for the coverage test
    x_lo, x_hi = -0.05 + shift_x, 0.05 + shift_x
    checked = zeros = 0
    for py in range(H):
        for px in range(W):
            want = np.zeros(7)
            inside = []
            for k in range(spp):
                s = (py * W + px) * spp + k
                w = orc.philox(seed, (s, 0, 0, 0))
                qx = np.float32(px) + _u01(w[0])
                qy = np.float32(py) + _u01(w[1])
                d = np.array([(qx - np.float32(W / 2)) * ps, (np.float32(H / 2) - qy) * ps, -1.0], np.float32)
                d = d.astype(np.float64)
                t = ((plane_pt - cam) @ n) / (d @ n)
                p = cam + t * d
                xl = (R.T @ (p - plane_pt))[0]          # plane-frame x of the hit
                inside.append(x_lo < xl < x_hi)
                if not inside[-1]:
                    continue
                want[:3] += [ramp[c][0] + ramp[c][1] * xl for c in range(3)]
                nn = n if n @ (cam - p) > 0 else -n
                want[3:6] += nn
                want[6] += np.linalg.norm(p - cam)
            want /= spp
            # a pixel is compared when its whole footprint is on one side of the
            # plane's border (samples near the border are fp32 decisions)
            corners = []
            for cx, cy in ((px, py), (px + 1, py), (px, py + 1), (px + 1, py + 1)):
                d = np.array([(cx - W / 2) * float(ps), (H / 2 - cy) * float(ps), -1.0])
                p = cam + ((plane_pt - cam) @ n) / (d @ n) * d
                corners.append((R.T @ (p - plane_pt))[0])
            if min(corners) > x_lo + 1e-3 and max(corners) < x_hi - 1e-3:
                assert all(inside)
                np.testing.assert_allclose(got[py, px], want, rtol=1e-6, atol=1e-9)   # fp32 scene inputs
                checked += 1
            elif max(corners) < x_lo - 1e-3 or min(corners) > x_hi + 1e-3:
                assert not any(inside)
                assert np.all(got[py, px] == 0)
                zeros += 1
    assert checked >= 20
    if shift_x != 0.0:
        assert zeros >= 10


def test_aov_selected_pixels_match_full(orc):
    model, scene, params, spp = synth.workload("tiny")
    osc, _, _ = orc.scene_from_model(model, scene, params)
    full = orc.aov(osc, 1234, spp)
    pix = np.array([0, 17, 2050, 4095, 1000])
    sel = orc.aov(osc, 1234, spp, pixels=pix)
    np.testing.assert_array_equal(sel, full.reshape(-1, 7)[pix])
    # hit pixels have unit normals toward the camera (spp samples averaged:
    # norm <= 1) and a depth near the camera-to-face distance
    hit = full[..., 6] > 0
    assert hit.sum() > 1000
    nrm = np.linalg.norm(full[..., 3:6], axis=-1)
    assert np.all(nrm[hit] <= 1 + 1e-12) and np.median(nrm[hit]) > 0.99
