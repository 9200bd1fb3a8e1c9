"""Pins of the oracle's fitting arithmetic (E_light and Adam)."""
import numpy as np
import pytest

from oracle import fitting


def test_light_reg_closed_forms():
    # gray lights carry no penalty
    e, g = fitting.light_reg(np.full((20, 3), 0.37), 1e-3)
    assert abs(e) < 1e-30 and np.abs(g).max() < 1e-15    # (0.37 * 3) / 3 rounds
    # a pure red light: m = 1/3, deviations (2/3, -1/3, -1/3), E = 6/9
    e, g = fitting.light_reg([[1.0, 0.0, 0.0]], 1.0)
    assert e == pytest.approx(2.0 / 3.0, rel=1e-15)
    np.testing.assert_allclose(g, [[4 / 3, -2 / 3, -2 / 3]], rtol=1e-15)
    # scales with w2 and sums over lights
    e2, _ = fitting.light_reg([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]], 0.5)
    assert e2 == pytest.approx(2.0 / 3.0, rel=1e-15)


def test_light_reg_gradient_is_the_derivative():
    rng = np.random.default_rng(3)
    L = rng.uniform(0, 1, (20, 3))
    e0, g = fitting.light_reg(L, 1e-3)
    h = 1e-6
    for j, c in [(0, 0), (5, 2), (19, 1)]:
        Lp, Lm = L.copy(), L.copy()
        Lp[j, c] += h
        Lm[j, c] -= h
        fd = (fitting.light_reg(Lp, 1e-3)[0] - fitting.light_reg(Lm, 1e-3)[0]) / (2 * h)
        assert fd == pytest.approx(g[j, c], rel=1e-6, abs=1e-12)


def test_adam_first_step_is_a_signed_lr_step():
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    p, m, v = fitting.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.1)
    # m_hat = g, v_hat = g^2: the step is lr * g / (|g| + eps)
    np.testing.assert_allclose(p, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-14)


def test_adam_matches_torch_optim():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(11)
    p0 = rng.normal(size=37)
    grads = rng.normal(size=(6, 37)) * np.array([1e-3, 1, 10, 0.1, 5, 1e-2])[:, None]
    w = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([w], lr=0.03, betas=(0.85, 0.995), eps=1e-7)
    p, m, v = p0.copy(), np.zeros(37), np.zeros(37)
    for t, g in enumerate(grads, start=1):
        opt.zero_grad()
        w.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = fitting.adam(p, g, m, v, t, 0.03, 0.85, 0.995, 1e-7)
    np.testing.assert_allclose(p, w.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_loss_l2_against_its_definition_and_fd():
    """E_data (Eq. 1): the sum over pixels and channels of squared
    differences, checked by an explicit loop on a small ragged image, and its
    gradient by central differences (exact: the loss is quadratic)."""
    import oracle
    rng = np.random.default_rng(3)
    I, T = rng.uniform(0, 0.2, (3, 5, 3)), rng.uniform(0, 0.2, (3, 5, 3))
    L, g = oracle.loss_l2(I, T)
    brute = 0.0
    for y in range(3):
        for x in range(5):
            for c in range(3):
                brute += (I[y, x, c] - T[y, x, c]) ** 2
    assert abs(L - brute) <= 1e-15 * brute
    h = 1e-4
    for idx in [(0, 0, 0), (2, 4, 2), (1, 3, 1)]:
        Ip, Im = I.copy(), I.copy()
        Ip[idx] += h
        Im[idx] -= h
        fd = (oracle.loss_l2(Ip, T)[0] - oracle.loss_l2(Im, T)[0]) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-9 * max(1.0, abs(g[idx]))
