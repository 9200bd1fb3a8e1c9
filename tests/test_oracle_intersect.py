"""Pins of the oracle's ray/triangle decisions: exact rational arithmetic and
brute force over all triangles."""
import ctypes as C
from fractions import Fraction

import numpy as np

from paper_1910_05200_amd import synth


def _exact_hit(o, d, v0, v1, v2):
    """Exact (rational) ray/plane solve: (t, b1, b2) or None if parallel."""
    o, d, v0, v1, v2 = ([Fraction(float(x)) for x in a] for a in (o, d, v0, v1, v2))
    e1 = [a - b for a, b in zip(v1, v0)]
    e2 = [a - b for a, b in zip(v2, v0)]
    # solve v0 + b1 e1 + b2 e2 = o + t d  (Cramer)
    M = [[-d[i], e1[i], e2[i]] for i in range(3)]
    rhs = [o[i] - v0[i] for i in range(3)]

    def det3(m):
        return (m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1])
                - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
                + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]))
    D = det3(M)
    if D == 0:
        return None
    sol = []
    for c in range(3):
        Mc = [row[:] for row in M]
        for i in range(3):
            Mc[i][c] = rhs[i]
        sol.append(det3(Mc) / D)
    return sol


def test_ray_tri_agrees_with_exact_away_from_edges(orc):
    rng = np.random.default_rng(11)
    checked = 0
    for _ in range(400):
        v = rng.uniform(-1, 1, (3, 3)).astype(np.float32)
        o = rng.uniform(-2, 2, 3).astype(np.float32) + np.array([0, 0, 3], np.float32)
        tgt = v.mean(0) + rng.uniform(-0.6, 0.6, 3)
        d = (tgt - o).astype(np.float32)
        ex = _exact_hit(o, d, *v)
        if ex is None:
            continue
        t, b1, b2 = ex
        margin = min(b1, b2, 1 - b1 - b2)
        if abs(float(margin)) < 1e-3:
            continue          # too close to an edge for a single-precision verdict
        want = margin > 0 and t > 0
        out = [np.zeros(1, np.float32) for _ in range(4)]
        hit = orc.lib().orc_ray_tri(*(orc._p(np.ascontiguousarray(a)) for a in (o, d, v[0], v[1], v[2])),
                                    C.c_float(0.0), C.c_float(np.inf), *(orc._p(a) for a in out))
        assert bool(hit) == bool(want)
        if hit:
            assert abs(out[0][0] - float(t)) <= 1e-5 * max(1.0, abs(float(t)))
            assert abs(out[1][0] - float(b1)) < 1e-4 and abs(out[2][0] - float(b2)) < 1e-4
        checked += 1
    assert checked > 300


def _rays_at_features(osc, rng, n):
    """Rays from above aimed at random points, vertices and edge midpoints."""
    pos = osc.pos.T.astype(np.float64)
    faces = osc.faces
    rays = []
    for i in range(n):
        kind = i % 3
        if kind == 0:
            tgt = pos[rng.integers(len(pos))]
        elif kind == 1:
            f = faces[rng.integers(len(faces))]
            tgt = (pos[f[0]] + pos[f[1]]) / 2
        else:
            tgt = pos.min(0) + rng.uniform(0, 1, 3) * (pos.max(0) - pos.min(0))
        o = tgt + rng.normal(0, 1, 3) * np.array([0.2, 0.2, 0.1]) + np.array([0, 0, 0.5])
        rays.append((o.astype(np.float32), (tgt - o).astype(np.float32)))
    return rays


def _closest(orc, st, use_bvh, o, d):
    out = [np.zeros(1, np.float32) for _ in range(4)]
    f = orc.lib().orc_closest_hit(C.byref(st), use_bvh, orc._p(o), orc._p(d), *(orc._p(a) for a in out))
    return (f, *(float(a[0]) for a in out))


def test_bvh_equals_brute_force(orc):
    rng = np.random.default_rng(5)
    model = synth.make_model(24, 20)
    scene = synth.make_scene(32, 32)
    osc, _, _ = orc.scene_from_model(model, scene, synth.make_params(3))
    st = osc.struct()
    hits = 0
    for o, d in _rays_at_features(osc, rng, 3000):
        a = _closest(orc, st, 0, o, d)
        b = _closest(orc, st, 1, o, d)
        assert a == b
        hits += a[0] >= 0
        # any-hit on the segment toward the target, skipping the closest triangle
        seg = (d * np.float32(1.5)).astype(np.float32)
        x0 = orc.lib().orc_any_hit(C.byref(st), 0, orc._p(o), orc._p(seg), a[0])
        x1 = orc.lib().orc_any_hit(C.byref(st), 1, orc._p(o), orc._p(seg), a[0])
        assert x0 == x1
    assert hits > 1000


def test_closest_hit_tie_breaks_to_lowest_index(orc):
    # two coincident triangles: the lower index must win
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)
    pos = np.ascontiguousarray(np.concatenate([v, v]).T)
    faces = np.array([[3, 4, 5], [0, 1, 2]], np.int32)
    m = synth.Mesh(pos, faces, np.ones((3, 6), np.float32), np.zeros((2, 6), np.float32))
    osc = orc.scene_from_mesh(m, 4, 4, [0, 0, 1], 0.01, synth.quad_light([0, 0, 2], [0.1, 0, 0], [0, -0.1, 0]),
                              [[1, 1, 1]], np.zeros(1024))
    st = osc.struct()
    o = np.array([0.2, 0.2, 1], np.float32)
    d = np.array([0, 0, -1], np.float32)
    for bvh in (0, 1):
        f, t, b1, b2, det = _closest(orc, st, bvh, o, d)
        assert f == 0 and t == 1.0
