"""Shared helpers for GPU-vs-oracle parity tests."""
import numpy as np

# Parity rule: |gpu - ref| <= REL * max(|ref|, floor), with floor = 0 for
# pixels and FLOOR_FRAC * max|ref| over a gradient group (the floor absorbs
# fp32 atomic-order noise in components that cancel).
REL = 1e-4
FLOOR_FRAC = 1e-2


def rel_excess(gpu, ref, floor=0.0):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.maximum(np.abs(ref), floor)
    err = np.abs(gpu - ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(scale > 0, err / scale, np.where(err > 0, np.inf, 0.0))
    return r


def assert_image_parity(gpu, ref, rel=REL, what="image"):
    r = rel_excess(gpu, ref)
    bad = np.argwhere(r > rel)
    assert bad.size == 0, (f"{what}: {len(bad)} of {r.size} values exceed {rel}; worst {r.max():.3g} at "
                           f"{tuple(bad[np.argmax(r[tuple(bad.T)])])}")
    return float(r.max())


def assert_group_parity(gpu, ref, name, rel=REL, floor_frac=FLOOR_FRAC):
    ref = np.asarray(ref, np.float64)
    floor = floor_frac * float(np.abs(ref).max()) if ref.size else 0.0
    r = rel_excess(gpu, ref, floor)
    bad = np.argwhere(r > rel)
    if bad.size:
        order = np.argsort(r.ravel())[::-1][:6]
        worst = [(int(i), float(np.ravel(gpu)[i]), float(ref.ravel()[i])) for i in order]
    assert bad.size == 0, (f"{name}: {len(bad)} of {r.size} components exceed {rel} "
                           f"(group floor {floor:.3g}); worst {r.max():.3g}: {worst}")
    return float(r.max()), float(rel_excess(gpu, ref).max())
