"""Host-side checks of the C-ABI library (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "facert.h")).read()
    return sorted(set(re.findall(r"^(?:int|int32_t|void|const char \*)\s*\*?\s*(fr_\w+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("fr_create", "fr_set_stream", "fr_blend", "fr_render", "fr_backward", "fr_stats",
              "fr_last_error", "fr_destroy", "fr_loss_l2", "fr_set_terms", "fr_set_chunk",
              "fr_batch_create", "fr_batch_render", "fr_batch_backward", "fr_batch_tune", "fr_batch_capture_begin",
              "fr_batch_capture_end", "fr_batch_graph_launch", "fr_batch_num_kinds"):
        assert n in names
    from paper_1910_05200_amd import facert
    assert set(names) == set(facert.EXPORTS)


def test_library_loads_and_exports_every_declared_symbol():
    from paper_1910_05200_amd import facert
    lib = facert.load()
    for n in _declared():
        assert hasattr(lib, n), n
        assert getattr(lib, n) is not None


def test_null_context_and_argument_errors_without_gpu():
    """Calls that fail before touching the device return their codes."""
    from paper_1910_05200_amd import facert
    lib = facert.load()
    assert lib.fr_create(None, None, 0, None) == -1
    out = C.c_void_p()
    assert lib.fr_create(None, None, 0, C.byref(out)) == -1 and not out.value
    assert lib.fr_set_stream(None, None) == -1
    assert lib.fr_render(None, None, 0, 1, None) == -1
    assert lib.fr_backward(None, None, None) == -1
    assert lib.fr_set_chunk(None, 1024) == -1
    assert lib.fr_last_error(None) == b"no context"
    lib.fr_destroy(None)
    # the context-free loss rejects its arguments before touching a device
    assert lib.fr_loss_l2_noalloc(None, None, None, 12, None, None) == -1
    assert b"null" in lib.fr_last_error(None)
    buf = (C.c_float * 4)()
    assert lib.fr_loss_l2_noalloc(None, buf, buf, 0, None, None) == -1
    assert lib.fr_loss_l2_noalloc(None, buf, buf, (1 << 24) + 1, None, None) == -1
    assert b"FR_LOSS_NOALLOC_MAX" in lib.fr_last_error(None)
    # invalid model: zero vertices
    md = facert.fr_model_desc()
    sd = facert.fr_scene_desc()
    assert lib.fr_create(C.byref(md), C.byref(sd), 0, C.byref(out)) == -1


def test_create_rejects_unknown_flags_without_gpu():
    """A valid model and scene with a flag bit the header does not define:
    FR_EINVAL before any device call.  The binding's flag values are the
    header's."""
    from paper_1910_05200_amd import facert, synth
    hdr = open(os.path.join(ROOT, "include", "facert.h")).read()
    for name in ("FR_TIMING", "FR_REFIT", "FR_DEVICE_PTRS"):
        m = re.search(r"#define %s\s+(\d+)u" % name, hdr)
        assert m and int(m.group(1)) == getattr(facert, name), name
    lib = facert.load()
    model, scene = synth.make_model(4, 4), synth.make_scene(8, 8)
    k = {n: np.ascontiguousarray(getattr(model, n), np.float32) for n in ("mean", "b_id", "b_exp", "alb_mean", "b_alb", "uv")}
    faces = np.ascontiguousarray(model.faces, np.int32)
    lg = np.ascontiguousarray(scene.light_geom, np.float32)
    md = facert.fr_model_desc(model.n_vertices, model.n_faces, k["b_id"].shape[0], k["b_exp"].shape[0], k["b_alb"].shape[0],
                              faces.ctypes.data, *(k[n].ctypes.data for n in ("mean", "b_id", "b_exp", "alb_mean", "b_alb", "uv")))
    sd = facert.fr_scene_desc(scene.width, scene.height, (C.c_float * 3)(*[float(x) for x in scene.cam]),
                              float(scene.pix_scale), lg.shape[0], lg.ctypes.data, scene.spec_res)
    out = C.c_void_p()
    for bad in (8, 1 << 31, facert.FR_DEVICE_PTRS | 16):
        assert lib.fr_create(C.byref(md), C.byref(sd), bad, C.byref(out)) == -1 and not out.value


def test_batch_argument_errors_without_gpu():
    from paper_1910_05200_amd import facert
    lib = facert.load()
    out = C.c_void_p()
    assert lib.fr_batch_create(0, None, 0, C.byref(out)) == -1 and not out.value
    assert lib.fr_batch_create(1, None, 0, C.byref(out)) == -1
    ctxs = (C.c_void_p * 2)(None, None)
    assert lib.fr_batch_create(2, ctxs, 0, C.byref(out)) == -1
    assert lib.fr_batch_render(None, None, None, None, None) == -1
    assert lib.fr_batch_backward(None, None, None) == -1
    assert lib.fr_batch_tune(None, 1, None) == -1
    assert lib.fr_batch_capture_begin(None) == -1
    assert lib.fr_batch_last_error(None) == b"no context"
    n = lib.fr_batch_num_kinds()
    names = [lib.fr_batch_kind_name(k).decode() for k in range(n)]
    assert len(set(names)) == n and "sh_trace" in names and "render_adj" in names
    assert lib.fr_batch_kind_name(n) is None and lib.fr_batch_kind_name(-1) is None
    lib.fr_batch_destroy(None)


def test_denoiser_batch_arguments_without_gpu():
    """fd_create_batch refuses its sizes before any device call: n < 1, a
    height that is not a multiple of 64 with n > 1, more pixels than the
    network's 32-bit indexing allows."""
    from paper_1910_05200_amd import denoise
    lib = denoise.load()
    out = C.c_void_p()
    for H, W, n in ((64, 64, 0), (72, 64, 2), (512, 512, 100), (60, 64, 1)):
        assert lib.fd_create_batch(H, W, n, C.byref(out)) == -1 and not out.value, (H, W, n)


def test_denoiser_header_declares_what_the_library_exports():
    src = open(os.path.join(ROOT, "include", "fadenoise.h")).read()
    names = set(re.findall(r"^(?:int|int64_t|void|const char \*)\s*\*?\s*(fd_\w+)\s*\(", src, re.M))
    from paper_1910_05200_amd import denoise
    assert names == set(denoise.EXPORTS), names ^ set(denoise.EXPORTS)
    lib = denoise.load()
    for n in names:
        assert getattr(lib, n) is not None, n
