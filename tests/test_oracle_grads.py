"""Pins of the oracle's interior adjoint by central finite differences.

The loss is L = sum (I - T)^2 (E_data of Eq. 1).  For fixed random numbers the
estimator is linear in the light intensities, the vertex albedo and the
specular texels, so L is quadratic in them and a central difference is exact
up to rounding.  For vertex positions and the morphable/pose parameters the
decisions (hit triangle, shadow bits, sides) are frozen and the value path is
differenced, which isolates the interior term of the gradient.
"""
import numpy as np
import pytest

from paper_1910_05200_amd import synth

SEED, SPP = 1000, 4


@pytest.fixture(scope="module")
def setup(orc):
    model, scene, params, spp = synth.workload("tiny")
    tosc, _, _ = orc.scene_from_model(model, scene, synth.make_params(synth.TARGET_SCENE_SEED))
    target = orc.render(tosc, synth.TARGET_RENDER_SEED, 16)
    osc, vm, R = orc.scene_from_model(model, scene, params)
    img = orc.render(osc, SEED, SPP)
    dLdI = 2 * (img - target)
    return model, scene, params, osc, vm, R, target, dLdI


def _loss(img, target):
    return float(((img - target) ** 2).sum())


def _check(fd, an, group_max, rel=1e-6):
    fd, an = np.asarray(fd), np.asarray(an)
    tol = rel * np.maximum(np.abs(fd), 1e-3 * group_max)
    assert np.all(np.abs(fd - an) <= tol), np.c_[fd, an]


def test_light_grads_exact(orc, setup):
    model, scene, params, osc, vm, R, target, dLdI = setup
    g = orc.backward(osc, SEED, SPP, dLdI, flags=orc.FLAG_INTERIOR)
    h = 1e-3
    fd = np.zeros_like(osc.light_rgb)
    base = osc.light_rgb.copy()
    for j in range(base.shape[0]):
        for c in range(3):
            osc.light_rgb[:] = base; osc.light_rgb[j, c] += h
            lp = _loss(orc.render(osc, SEED, SPP), target)
            osc.light_rgb[:] = base; osc.light_rgb[j, c] -= h
            lm = _loss(orc.render(osc, SEED, SPP), target)
            fd[j, c] = (lp - lm) / (2 * h)
    osc.light_rgb[:] = base
    _check(fd, g["d_light"], np.abs(fd).max(), 1e-7)
    assert np.abs(fd).max() > 0


def test_albedo_and_spec_grads_exact(orc, setup):
    model, scene, params, osc, vm, R, target, dLdI = setup
    g = orc.backward(osc, SEED, SPP, dLdI, flags=orc.FLAG_INTERIOR)
    rng = np.random.default_rng(0)
    h = 1e-3
    nz = np.flatnonzero(np.abs(g["d_alb"]).ravel() > 0)
    pick = rng.choice(nz, 12, replace=False)
    fd, an = [], []
    for e in pick:
        base = osc.alb.ravel()[e]
        osc.alb.ravel()[e] = base + h; lp = _loss(orc.render(osc, SEED, SPP), target)
        osc.alb.ravel()[e] = base - h; lm = _loss(orc.render(osc, SEED, SPP), target)
        osc.alb.ravel()[e] = base
        fd.append((lp - lm) / (2 * h)); an.append(g["d_alb"].ravel()[e])
    _check(fd, an, np.abs(g["d_alb"]).max(), 1e-7)
    nz = np.flatnonzero(np.abs(g["d_spec"]) > 0)
    pick = rng.choice(nz, min(12, nz.size), replace=False)
    fd, an = [], []
    for e in pick:
        base = osc.spec[e]
        osc.spec[e] = base + h; lp = _loss(orc.render(osc, SEED, SPP), target)
        osc.spec[e] = base - h; lm = _loss(orc.render(osc, SEED, SPP), target)
        osc.spec[e] = base
        fd.append((lp - lm) / (2 * h)); an.append(g["d_spec"][e])
    _check(fd, an, np.abs(g["d_spec"]).max(), 1e-7)


def test_vertex_grads_frozen_fd(orc, setup):
    model, scene, params, osc, vm, R, target, dLdI = setup
    rec = orc.record(osc, SEED, SPP)
    base_img = orc.render_frozen(osc, SEED, SPP, rec)
    assert np.array_equal(base_img, orc.render(osc, SEED, SPP))
    g = orc.backward_frozen(osc, SEED, SPP, rec, dLdI)
    gi = g["d_pos_interior"]
    flat = np.abs(gi).ravel()
    rng = np.random.default_rng(1)
    pick = np.concatenate([np.argsort(flat)[-8:], rng.choice(np.flatnonzero(flat > 0), 12, replace=False)])
    h = 1e-7
    fd, an = [], []
    for e in pick:
        base = osc.pos_d.ravel()[e]
        osc.pos_d.ravel()[e] = base + h; lp = _loss(orc.render_frozen(osc, SEED, SPP, rec), target)
        osc.pos_d.ravel()[e] = base - h; lm = _loss(orc.render_frozen(osc, SEED, SPP, rec), target)
        osc.pos_d.ravel()[e] = base
        fd.append((lp - lm) / (2 * h)); an.append(gi.ravel()[e])
    _check(fd, an, flat.max(), 2e-5)
    # the frozen adjoint is the interior term of the full backward
    full = orc.backward(osc, SEED, SPP, dLdI, flags=orc.FLAG_INTERIOR)
    assert np.allclose(full["d_pos_interior"], gi, rtol=1e-12, atol=1e-12 * flat.max())


def test_parameter_grads_frozen_fd(orc, setup):
    """alpha, beta, delta and pose gradients against central differences taken
    in double precision (the blend is linear, so v(alpha + h e_k) =
    v + h R B_id[k] exactly; the pose uses scipy's rotation, itself pinned)."""
    from scipy.spatial.transform import Rotation
    model, scene, params, osc, vm, R, target, dLdI = setup
    rec = orc.record(osc, SEED, SPP)
    g = orc.backward_frozen(osc, SEED, SPP, rec, dLdI)
    pg = orc.parameter_grads(model, params, vm, R, g["d_pos_interior"], g["d_alb"])
    pos0, alb0 = osc.pos_d.copy(), osc.alb.copy()

    def loss_with(pos=None, alb=None):
        osc.pos_d[:] = pos0 if pos is None else pos
        osc.alb[:] = alb0 if alb is None else alb
        return _loss(orc.render_frozen(osc, SEED, SPP, rec), target)

    try:
        for key, basis, idx, h in (("d_alpha", model.b_id, [0, 7, 33, 79], 1e-5),
                                   ("d_beta", model.b_exp, [0, 12, 55, 89], 1e-5)):
            fd = []
            for k in idx:
                dv = R @ basis[k].astype(np.float64)
                fd.append((loss_with(pos=pos0 + h * dv) - loss_with(pos=pos0 - h * dv)) / (2 * h))
            _check(fd, pg[key][idx], np.abs(pg[key]).max(), 1e-5)
        fd = []
        for k in [0, 5, 41, 79]:
            dA = model.b_alb[k].astype(np.float64)
            fd.append((loss_with(alb=alb0 + 1e-3 * dA) - loss_with(alb=alb0 - 1e-3 * dA)) / 2e-3)
        _check(fd, pg["d_delta"][[0, 5, 41, 79]], np.abs(pg["d_delta"]).max(), 1e-7)
        ang = params.pose[:3].astype(np.float64)
        # near-grazing hits make the frozen estimator strongly curved: a
        # rigid motion must stay ~1e-9 m for the central difference to settle
        fd = []
        h = 1e-8
        for k in range(3):
            e = np.zeros(3); e[k] = h
            R0 = Rotation.from_euler("xyz", ang).as_matrix()
            vp = pos0 + (Rotation.from_euler("xyz", ang + e).as_matrix() - R0) @ vm
            vmn = pos0 + (Rotation.from_euler("xyz", ang - e).as_matrix() - R0) @ vm
            fd.append((loss_with(pos=vp) - loss_with(pos=vmn)) / (2 * h))
        h = 1e-9
        for k in range(3):
            e = np.zeros((3, 1)); e[k] = h
            fd.append((loss_with(pos=pos0 + e) - loss_with(pos=pos0 - e)) / (2 * h))
        _check(fd, pg["d_pose"], np.abs(pg["d_pose"]).max(), 1e-5)
    finally:
        osc.pos_d[:] = pos0
        osc.alb[:] = alb0
