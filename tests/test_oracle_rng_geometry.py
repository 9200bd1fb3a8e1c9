"""Pins of the oracle's RNG, morphable blend, pose, normals and edge table."""
import math
import os

import numpy as np
import pytest

from paper_1910_05200_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers(orc):
    rows = [l.split() for l in open(os.path.join(GOLD, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        c = [int(x, 16) for x in r[:4]]
        k = [int(x, 16) for x in r[4:6]]
        want = [int(x, 16) for x in r[6:10]]
        got = orc.philox(k[0] | (k[1] << 32), c)
        assert list(got) == want


def test_philox_uniformity(orc):
    # chi^2 of the top byte over 4096 blocks: 256 bins, 16384 words
    words = np.concatenate([orc.philox(12345, (i, 3, 0, 0)) for i in range(4096)])
    hist = np.bincount(words >> 24, minlength=256)
    exp = words.size / 256
    chi2 = float(((hist - exp) ** 2 / exp).sum())
    assert 180 < chi2 < 340       # ~ N(255, 22.6): outside is > 3.5 sigma
    # distinct counters give distinct outputs
    assert len(set(words.tolist())) > 0.999 * words.size


def test_rotation_matches_scipy(orc):
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(3)
    for _ in range(20):
        pose = rng.uniform(-1, 1, 6).astype(np.float32)
        R = orc.rotation(pose)
        # extrinsic x, then y, then z  ==  Rz @ Ry @ Rx
        ref = Rotation.from_euler("xyz", pose[:3].astype(np.float64)).as_matrix()
        assert np.allclose(R, ref, atol=1e-15)


def test_blend_matches_float64_matmul(orc):
    model = synth.make_model(12, 10)
    params = synth.make_params(4)
    vm, v, A, R = orc.blend(model, params)
    V = model.n_vertices
    ref_m = model.mean.astype(np.float64).reshape(-1) \
        + model.b_id.reshape(80, -1).T.astype(np.float64) @ params.alpha.astype(np.float64) \
        + model.b_exp.reshape(90, -1).T.astype(np.float64) @ params.beta.astype(np.float64)
    ref_m = ref_m.reshape(3, V)
    assert np.allclose(vm, ref_m, rtol=0, atol=1e-15)
    ref_v = R @ ref_m + params.pose[3:].astype(np.float64)[:, None]
    assert np.allclose(v, ref_v, rtol=0, atol=1e-15)
    ref_A = model.alb_mean.astype(np.float64).reshape(-1) \
        + model.b_alb.reshape(80, -1).T.astype(np.float64) @ params.delta.astype(np.float64)
    assert np.allclose(A.reshape(-1), ref_A, rtol=0, atol=1e-15)


def test_normals_flat_grid_exact(orc):
    m = synth.flat_grid(7, 0.3, z=0.1)
    n = orc.vertex_normals(m.faces, m.pos.astype(np.float64))
    assert np.array_equal(n, np.tile(np.array([[0.0], [0.0], [1.0]]), (1, 49)))


def test_normals_sphere_converge_to_radial(orc):
    # vertices on a unit sphere cap: normals -> radial as O(h^2)
    errs = []
    for nx in (9, 17, 33):
        xs = np.linspace(-0.4, 0.4, nx)
        gx, gy = np.meshgrid(xs, xs, indexing="xy")
        gz = np.sqrt(1 - gx ** 2 - gy ** 2)
        pos = np.stack([gx.ravel(), gy.ravel(), gz.ravel()])
        n = orc.vertex_normals(synth.grid_faces(nx, nx), pos)
        # interior vertices only (boundary stencils are one-sided)
        inner = np.zeros((nx, nx), bool)
        inner[1:-1, 1:-1] = True
        err = np.abs(n - pos)[:, inner.ravel()].max()
        errs.append(err)
    assert errs[1] < errs[0] / 3 and errs[2] < errs[1] / 3
    assert errs[2] < 5e-4


def test_edge_table_topology(orc):
    nx, ny = 9, 6
    faces = synth.grid_faces(nx, ny)
    E = orc.build_edges(faces, nx * ny)
    V, F = nx * ny, faces.shape[0]
    assert V - E.shape[0] + F == 1                        # a disk
    assert (E[:, 0] < E[:, 1]).all()
    key = E[:, 0].astype(np.int64) * V + E[:, 1]
    assert (np.diff(key) > 0).all()                       # sorted, unique
    boundary = (E[:, 3] < 0).sum()
    assert boundary == 2 * (nx - 1) + 2 * (ny - 1)
    # every row's faces really contain the edge
    for a, b, f1, f2 in E:
        for f in (f1, f2):
            if f >= 0:
                assert a in faces[f] and b in faces[f]
        assert f2 < 0 or f1 < f2


def test_edge_counts_match_configs(orc):
    for name, (V, F, E, nb) in {"tiny": (1024, 1922, 2945, 124),
                               "paper": (20000, 39432, 59431, 566)}.items():
        c = synth.CONFIGS[name]
        faces = synth.grid_faces(c["nx"], c["ny"])
        assert faces.shape[0] == F
        ed = orc.build_edges(faces, c["nx"] * c["ny"])
        assert ed.shape[0] == E and (ed[:, 3] < 0).sum() == nb


def test_oracle_pins_clean_under_address_and_ub_sanitizers():
    """The oracle's C code, built with -fsanitize=address,undefined, passes
    its estimator pins with no sanitizer report (oracle/sanitize.py)."""
    import os
    import subprocess
    import sys
    if os.environ.get("LD_PRELOAD") or os.environ.get("FACERT_ORACLE_SANITIZE"):
        import pytest
        pytest.skip("a preload is already set, or this is the sanitized run itself")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-m", "oracle.sanitize", "-x", "-k",
                        "not unet and not sanitizers"], cwd=root, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert " passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr + r.stdout
