"""fr_loss_l2_noalloc (no context, no device allocation: its block partials
live in a fixed device array) against fr_loss_l2 on a context, through the
C-ABI: two calls in a row, the second on a smaller input, must each give
fr_loss_l2's image gradient and loss exactly (the same kernels over the same
blocks) and E_data's definition within 1e-4."""
import ctypes as C

import numpy as np
import pytest

from paper_1910_05200_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no HIP device")
    return T


def _pair(orc, W, H, seed):
    rng = np.random.default_rng(seed)
    I = rng.gamma(0.5, 0.05, (H, W, 3)).astype(np.float32)
    T = rng.gamma(0.5, 0.05, (H, W, 3)).astype(np.float32)
    return I, T


def test_noalloc_loss_matches_the_context_loss(torch, orc):
    from paper_1910_05200_amd import facert
    lib = facert.load()
    for W, H, seed in ((256, 256, 1), (37, 23, 2), (256, 256, 3)):
        I, T = _pair(orc, W, H, seed)
        r = facert.Renderer(synth.make_model(4, 4), synth.make_scene(W, H))
        dI, dT = torch.from_numpy(I).cuda(), torch.from_numpy(T).cuda()
        g_ref, l_ref = r.loss_l2(dI, dT)
        g, l = facert.loss_l2_noalloc(dI, dT)
        torch.cuda.synchronize()
        assert torch.equal(g, g_ref) and torch.equal(l, l_ref), (W, H)
        L, gd = orc.loss_l2(I, T)
        assert abs(float(l) - L) <= 1e-4 * L
        np.testing.assert_array_equal(g.cpu().numpy(), (2 * (I.astype(np.float64) - T)).astype(np.float32))
        r.close()


def test_noalloc_loss_outputs_are_optional_and_sizes_checked(torch):
    from paper_1910_05200_amd import facert
    lib = facert.load()
    a = torch.rand(1000, device="cuda")
    b = torch.rand(1000, device="cuda")
    _, l = facert.loss_l2_noalloc(a, b, want_dL=False)
    torch.cuda.synchronize()
    ref = float(((a.double() - b.double()) ** 2).sum())
    assert abs(float(l) - ref) <= 1e-4 * ref
    g = torch.empty_like(a)
    code = lib.fr_loss_l2_noalloc(torch.cuda.current_stream().cuda_stream, a.data_ptr(), b.data_ptr(), 1000,
                                  g.data_ptr(), None)
    torch.cuda.synchronize()
    assert code == 0 and torch.equal(g, 2 * (a - b))
    big = (1 << 24) + 1
    assert lib.fr_loss_l2_noalloc(None, a.data_ptr(), b.data_ptr(), big, None, None) == -1
    assert b"FR_LOSS_NOALLOC_MAX" in lib.fr_last_error(None)
