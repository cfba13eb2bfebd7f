"""Pins of the U-Net oracle (learned continuation predictor): each part is
checked against a definition or identity computed another way."""
import numpy as np
import pytest

from oracle import unet as U


def rng(seed):
    return np.random.default_rng(seed)


def test_parameter_count_of_the_4_level_32_channel_net():
    # 9 (6*32 + 32*32 + 32*64 + 64^2 + 64*128 + 128^2 + 128*256 + 256^2
    #    + 384*128 + 128^2 + 192*64 + 64^2 + 96*32 + 32^2) + 32*2 + biases
    w = 9 * (6 * 32 + 32 * 32 + 32 * 64 + 64 * 64 + 64 * 128 + 128 * 128 + 128 * 256 + 256 * 256
             + 384 * 128 + 128 * 128 + 192 * 64 + 64 * 64 + 96 * 32 + 32 * 32) + 32 * 2
    b = 32 + 32 + 64 + 64 + 128 + 128 + 256 + 256 + 128 + 128 + 64 + 64 + 32 + 32 + 2
    assert U.num_params(U.layer_specs(4, 32)) == w + b


def test_conv_matches_direct_sum():
    r = rng(0)
    x = r.standard_normal((3, 5, 4))
    W = r.standard_normal((2, 3, 3, 3))
    b = r.standard_normal(2)
    out = U.conv(x, W, b)
    for co in range(2):
        for y in range(5):
            for xx in range(4):
                s = b[co]
                for ky in range(3):
                    for kx in range(3):
                        yy, xs = y + ky - 1, xx + kx - 1
                        if 0 <= yy < 5 and 0 <= xs < 4:
                            s += W[co, ky, kx] @ x[:, yy, xs]
                assert out[co, y, xx] == pytest.approx(s, abs=1e-12)


def test_up_reproduces_affine_functions_and_transfers_are_adjoint():
    n = 5
    yc, xc = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    f = (1.5 + 0.25 * xc - 0.75 * yc)[None].astype(float)
    yf, xf = np.meshgrid(np.arange(2 * n - 1) / 2, np.arange(2 * n - 1) / 2, indexing="ij")
    assert np.allclose(U.up(f)[0], 1.5 + 0.25 * xf - 0.75 * yf, atol=1e-14)
    r = rng(1)
    a, b = r.standard_normal((2, n, n)), r.standard_normal((2, 2 * n - 1, 2 * n - 1))
    assert np.sum(U.up(a) * b) == pytest.approx(np.sum(a * U.up_backward(b)), rel=1e-13)
    assert np.sum(U.down(b) * a) == pytest.approx(np.sum(b * U.down_backward(a, b.shape)), rel=1e-13)


def test_silu_derivative():
    z = np.linspace(-6, 6, 41)
    eps = 1e-6
    fd = (U.silu(z + eps) - U.silu(z - eps)) / (2 * eps)
    assert np.allclose(U.silu_grad(z), fd, atol=1e-9)


@pytest.mark.parametrize("levels,base,N", [(3, 4, 9), (2, 8, 5), (1, 4, 4)])
def test_gradient_matches_finite_differences(levels, base, N):
    r = rng(2)
    specs = U.layer_specs(levels, base)
    theta = 0.3 * r.standard_normal(U.num_params(specs))
    psi = r.standard_normal(N * N) + 1j * r.standard_normal(N * N)
    psb = psi + 0.02 * (r.standard_normal(N * N) + 1j * r.standard_normal(N * N))
    tgt = psi + 0.02 * (r.standard_normal(N * N) + 1j * r.standard_normal(N * N))
    vol = U.volumes(N, 4.0)
    L, g = U.loss_and_grad(theta, specs, levels, psi, psb, 0.7, 0.02, tgt, vol, N)
    idx = r.choice(theta.size, 60, replace=False)
    eps = 1e-6
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += eps
        tm[k] -= eps
        Lp, _ = U.loss_and_grad(tp, specs, levels, psi, psb, 0.7, 0.02, tgt, vol, N)
        Lm, _ = U.loss_and_grad(tm, specs, levels, psi, psb, 0.7, 0.02, tgt, vol, N)
        fd = (Lp - Lm) / (2 * eps)
        assert g[k] == pytest.approx(fd, rel=1e-5, abs=1e-8 * max(1.0, abs(L)))


def test_loss_zero_at_exact_correction_and_prediction_form():
    N = 5
    r = rng(3)
    psi = r.standard_normal(N * N) + 1j * r.standard_normal(N * N)
    psb = psi + 0.02 * (0.5 - 1j)
    tgt = psb + 0.02 * (1 + 2j)
    o = np.stack([np.full((N, N), 1.0), np.full((N, N), 2.0)])
    L, do = U.loss_and_grad_output(o, psi, psb, tgt, 0.02, U.volumes(N, 2.0), N)
    assert L == pytest.approx(0.0, abs=1e-20) and np.abs(do).max() < 1e-12
    specs = U.layer_specs(2, 4)
    theta = np.zeros(U.num_params(specs))
    # a zero network returns the base step (the secant predictor); its loss is
    # S / (S + EPS |Omega|), S = sum d |w|^2 with w = 1 + 2i here
    assert np.array_equal(U.predict(theta, specs, 2, psi, psb, 0.3, 0.02, N), psb)
    L0, _ = U.loss_and_grad(theta, specs, 2, psi, psb, 0.3, 0.02, tgt, U.volumes(N, 2.0), N)
    S = 5.0 * 4.0
    assert L0 == pytest.approx(S / (S + U.EPS * 4.0), rel=1e-13)


def test_adam_first_step_and_bias_correction():
    g = np.array([0.5, -2.0, 1e-3])
    th = np.zeros(3)
    m, v = np.zeros(3), np.zeros(3)
    U.adam_step(th, m, v, g, 1, lr=0.1, eps=0.0)
    # m_hat = g, v_hat = g^2 after bias correction: a step of lr * sign(g)
    assert np.allclose(th, -0.1 * np.sign(g), rtol=1e-12)
    # second step with the same gradient: still lr * sign(g)
    U.adam_step(th, m, v, g, 2, lr=0.1, eps=0.0)
    assert np.allclose(th, -0.2 * np.sign(g), rtol=1e-12)


def test_volumes_sum_to_the_area():
    assert U.volumes(9, 8.0).sum() == pytest.approx(64.0, rel=1e-15)
