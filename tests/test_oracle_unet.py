"""Pins of the FP64 reference network and of the guess planes (CPU only).

The convolution is checked against scipy's 2-D correlation, pooling and
upsampling against their adjoints, the hand-written reverse pass against
central finite differences, Adam against its closed-form first step, and the
guess formulation against a dense solve: with the exact correction as network
output the guess is the exact solution.
"""
import numpy as np
import pytest
from scipy import signal

from oracle import fit, guess, precond, stencil
from oracle import operator as op
from oracle import unet
from paper_2410_17446_amd import inputs


def test_conv3_is_a_zero_padded_correlation():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 7, 9))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = unet.conv3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = sum(signal.correlate2d(x[n, c], w[o, c], mode="same", boundary="fill") for c in range(3)) + b[o]
            assert np.allclose(y[n, o], ref, atol=1e-12)


def test_pool_and_upsample_adjoints():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 3, 8, 6))
    z = rng.standard_normal((2, 3, 4, 3))
    assert np.isclose(np.sum(unet.pool(x) * z), np.sum(x * unet.pool_backward(z)))
    assert np.isclose(np.sum(unet.up(z) * x), np.sum(z * unet.up_backward(x)))
    assert np.allclose(unet.pool(np.ones((1, 1, 4, 4))), 1.0)


def _tiny(levels=3, base=2, cin=3, cout=2, seed=0):
    *_, n = unet.layout(levels, base, cin, cout)
    rng = np.random.default_rng(seed)
    return unet.UNet(levels, base, cin, cout, 0.5 * rng.standard_normal(n))


def test_layout_sizes():
    enc_a, enc_b, dec_a, dec_b, out, n = unet.layout(4, 32, 7, 2)
    assert [c.ci for c in enc_a] == [7, 32, 64, 128]
    assert [c.ci for c in dec_a] == [96, 192, 384]
    assert out.ci == 32 and out.co == 2 and out.k == 1
    assert n == out.b + 2


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_gradient_matches_central_differences(levels):
    net = _tiny(levels=levels)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 3, 8, 8))
    t = rng.standard_normal((2, 2, 8, 8))
    loss, g = net.loss_and_grad(x, t)
    p0 = net.p.copy()
    h = 1e-6

    def f(p):
        net.p = p
        y, _ = net.forward(x)
        return np.mean((y - t) ** 2)
    idx = rng.choice(len(p0), size=min(40, len(p0)), replace=False)
    for i in idx:
        e = np.zeros_like(p0)
        e[i] = h
        fd = (f(p0 + e) - f(p0 - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])
    d = rng.standard_normal(len(p0))
    fd = (f(p0 + h * d) - f(p0 - h * d)) / (2 * h)
    assert abs(fd - g @ d) <= 1e-6 * max(1.0, abs(g @ d))
    net.p = p0
    assert np.isclose(f(p0), loss)


def test_adam_first_step_is_a_signed_step():
    rng = np.random.default_rng(4)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p1, m, v = unet.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-3, eps=1e-12)
    assert np.allclose(p1, p - 1e-3 * np.sign(g), atol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_exact_correction_gives_the_exact_solution():
    """With net output = target (-P x / sigma), M^-1 (w + sigma net) = x for the dense solution x."""
    N, W = 20, 6
    c, d = stencil.stencils()
    g = op.Grid(N=N, dx=0.25, dy=0.25, k0=2 * np.pi, n0=1.0, c=c, d=d, W=W, eta_max=0.0)
    n2 = inputs.sine_product_n2(N, 0.25, 0.05, 2.0)
    co = op.coefficients(g, n2, False)
    co0 = op.coefficients(g, np.ones_like(n2), False)
    w = inputs.random_field(N, 1, seed=5)
    w[:, 0, :] = 0
    w[:, :, 0] = 0
    b = fit.fit_exp_sqrt(2 * np.pi, 6)["poles"][2]
    A = op.dense_zbar(g, co, 1) - b * np.eye((N - 1) ** 2)
    x = op.unpack(np.linalg.solve(A, op.pack(w)), 1, N)
    px = op.apply_zbar(g, co, x) - op.apply_zbar(g, co0, x)
    y = precond.apply_minv(g, w, b)
    scal = guess.stats(w, [y], n2, 1.0, W)
    tgt = guess.target(px[None], scal)
    t = guess.unpack(w, tgt, scal)
    x0 = precond.apply_minv(g, t[0], b)
    assert np.linalg.norm(x0 - x) < 1e-10 * np.linalg.norm(x)
    # the zero correction is the free-space solution
    t0 = guess.unpack(w, np.zeros_like(tgt), scal)
    assert np.allclose(precond.apply_minv(g, t0[0], b), y)
    # input planes: unit rms field planes, V plane, constant pole planes
    xin = guess.pack(w, [y], n2, scal, [(0.3, -0.7)], 1.0, W)
    assert xin.shape == (1, 7, N, N)
    assert np.isclose(np.sqrt(np.mean(xin[0, 0, 1:, 1:] ** 2 + xin[0, 1, 1:, 1:] ** 2)), 1.0)
    assert np.isclose(np.sqrt(np.mean(xin[0, 2, 1:, 1:] ** 2 + xin[0, 3, 1:, 1:] ** 2)), 1.0)
    assert np.all(xin[0, 5, 1:, 1:] == 0.3) and np.all(xin[0, 6, 1:, 1:] == -0.7)
