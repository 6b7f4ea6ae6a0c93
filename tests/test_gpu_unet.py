"""The U-Net kernels (forward, reverse pass, Adam, guess planes) against the FP64
reference network and guess planes of the oracle, through the C ABI, and the
learned guess end to end.

Tolerances: float32 weights, activations and accumulation against float64:
forward 1e-5 relative L2, gradients 1e-4 (a ReLU whose input rounds to the
other side of 0 changes a few terms), Adam 1e-5; guess planes 1e-6 (float32
rounding of planes computed in FP64).  The bf16 matrix-core convolutions
(8 significant bits per operand, float32 accumulation): forward 2e-2,
gradients 5e-2, and bit-exact against float32 where every operand and sum is
exact.
"""
import numpy as np
import pytest

from oracle import guess as oguess
from oracle import precond
from oracle import operator as op
from oracle import unet as ounet
from paper_2410_17446_amd import inputs

from helpers import gpu_plan, oracle_grid, rel_l2, to_gpu, workload

pytestmark = pytest.mark.gpu


def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _net(levels=3, base=4, cin=7, cout=2, seed=1):
    from paper_2410_17446_amd.unet import UNet
    return UNet(levels, base, cin, cout, seed=seed)


def _data(B=2, cin=7, cout=2, H=32, W=32, seed=0):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((B, cin, H, W)).astype(np.float32),
            rng.standard_normal((B, cout, H, W)).astype(np.float32))


@pytest.mark.parametrize("levels,base,H,W", [(3, 4, 32, 32), (1, 8, 16, 24), (4, 2, 24, 40)])
def test_forward_matches_oracle(levels, base, H, W):
    torch = _cuda()
    net = _net(levels, base)
    x, _ = _data(H=H, W=W)
    y = net.forward(to_gpu(x)).cpu().numpy()
    ref, _ = ounet.UNet(levels, base, 7, 2, net.state()["params"].astype(np.float64)).forward(x.astype(np.float64))
    assert rel_l2(y, ref) < 1e-5


@pytest.mark.parametrize("levels", [1, 3])
def test_gradients_match_oracle(levels):
    torch = _cuda()
    net = _net(levels, 4)
    x, t = _data()
    loss = net.grad(to_gpu(x), to_gpu(t))
    s = net.state()
    ref = ounet.UNet(levels, 4, 7, 2, s["params"].astype(np.float64))
    rloss, rg = ref.loss_and_grad(x.astype(np.float64), t.astype(np.float64))
    assert abs(loss - rloss) <= 1e-6 * rloss
    assert rel_l2(s["grads"], rg) < 1e-4


def test_bf16_convolutions_exact_on_small_integers():
    """Integer weights and inputs small enough that every bf16 operand and every float32 sum is
    exact: the matrix-core convolutions (cin 7 and 48: one and two channel chunks; cout 48: a
    partial channel tile; 40 x 24 pixels: partial pixel tiles) equal the float32 ones bit for bit."""
    torch = _cuda()
    from paper_2410_17446_amd.unet import HP_UNET_BF16, UNet
    rng = np.random.default_rng(3)
    a = UNet(1, 48, 7, 2, seed=0)
    p = rng.integers(-1, 2, size=a.nparam).astype(np.float32)
    a.load_state(p)
    b = UNet(1, 48, 7, 2, seed=0, precision=HP_UNET_BF16)
    b.load_state(p)
    x = to_gpu(rng.integers(-2, 3, size=(2, 7, 40, 24)).astype(np.float32))
    ya, yb = a.forward(x).cpu().numpy(), b.forward(x).cpu().numpy()
    assert np.abs(ya).max() > 10
    assert np.array_equal(ya, yb)


@pytest.mark.parametrize("H,W", [(32, 16), (128, 4)])
def test_bf16_gradients_exact_on_small_integers(H, W):
    """The same with the reverse pass: sparse integer weights, integer inputs, and a target that
    differs from the output by small integers, over B * cout * H * W = 2^11 outputs, so that every
    gradient the matrix cores see is a small integer times 2^-10 and every sum is exact.  The
    gradients (matrix-core weight gradients summed over pixel-segment splits, and data gradients)
    then equal the float32 ones bit for bit.  W = 4: rows shorter than one lane group, scalar
    loads; W = 16: half-filled 32-pixel segments, vector loads."""
    torch = _cuda()
    from paper_2410_17446_amd.unet import HP_UNET_BF16, UNet
    rng = np.random.default_rng(4)
    a = UNet(1, 40, 7, 2, seed=0)
    p = (rng.integers(-1, 2, size=a.nparam) * (rng.random(a.nparam) < 0.25)).astype(np.float32)
    a.load_state(p)
    b = UNet(1, 40, 7, 2, seed=0, precision=HP_UNET_BF16)
    b.load_state(p)
    x = to_gpu(rng.integers(-2, 3, size=(2, 7, H, W)).astype(np.float32))
    y = a.forward(x).cpu().numpy()
    t = to_gpu(y - rng.integers(-2, 3, size=y.shape).astype(np.float32))
    la, lb = a.grad(x, t), b.grad(x, t)
    ga, gb = a.state()["grads"], b.state()["grads"]
    assert np.count_nonzero(ga) > ga.size // 10
    assert la == lb and np.array_equal(ga, gb)


@pytest.mark.parametrize("levels", [1, 3])
def test_bf16_forward_and_gradients_near_oracle(levels):
    """bf16 operands (8 significant bits), float32 accumulation: forward within 2e-2 and the
    gradient (whose data-gradient convolutions also run on the matrix cores) within 5e-2
    relative L2 of the FP64 reference."""
    torch = _cuda()
    from paper_2410_17446_amd.unet import HP_UNET_BF16
    net = _net(levels, 8)
    net.set_precision(HP_UNET_BF16)
    x, t = _data()
    y = net.forward(to_gpu(x)).cpu().numpy()
    ref = ounet.UNet(levels, 8, 7, 2, net.state()["params"].astype(np.float64))
    ry, _ = ref.forward(x.astype(np.float64))
    assert rel_l2(y, ry) < 2e-2
    net.grad(to_gpu(x), to_gpu(t))
    _, rg = ref.loss_and_grad(x.astype(np.float64), t.astype(np.float64))
    assert rel_l2(net.state()["grads"], rg) < 5e-2


def test_adam_matches_oracle_and_checkpoint_resumes_exactly():
    torch = _cuda()
    net = _net()
    x, t = _data()
    xg, tg = to_gpu(x), to_gpu(t)
    p0 = net.state()["params"].astype(np.float64)
    net.grad(xg, tg)
    g = net.state()["grads"].astype(np.float64)
    net.adam(1e-3)
    s = net.state()
    p1, m1, v1 = ounet.adam_step(p0, g, np.zeros_like(p0), np.zeros_like(p0), 1, 1e-3)
    assert rel_l2(s["params"] - p0, p1 - p0) < 1e-5
    assert rel_l2(s["m"], m1) < 1e-6 and rel_l2(s["v"], v1) < 1e-5 and s["step"] == 1
    # resume from the saved state: two more steps on both nets give identical parameters
    twin = _net(seed=99)
    twin.load_state(s["params"], s["m"], s["v"], s["step"])
    for n in (net, twin):
        for _ in range(2):
            n.grad(xg, tg)
            n.adam(1e-3)
    assert np.array_equal(net.state()["params"], twin.state()["params"])


@pytest.mark.parametrize("ncomp", [1, 2])
def test_guess_planes_match_oracle(ncomp):
    torch = _cuda()
    N, W = 64, 8
    wl = workload(N=N, ncomp=ncomp, W=W)
    g = oracle_grid(wl)
    n2 = inputs.grf_n2(N, 0.25, 0.01, 2.0, seed=3)
    w = inputs.random_beam(N, 0.25, ncomp, seed=4)
    poles = wl["fit"]["poles"][:3]
    ys = np.stack([precond.apply_minv(g, w, b) for b in poles])
    net = _net(cin=4 * ncomp + 3, cout=2 * ncomp)
    feats = np.stack([np.arcsinh(poles.real), np.arcsinh(poles.imag)], axis=1)
    scal = net.guess_stats(to_gpu(w), to_gpu(ys), to_gpu(n2), 1.0, W)
    rs = oguess.stats(w, list(ys), n2, 1.0, W)
    assert np.allclose(scal.cpu().numpy(), rs, rtol=1e-12)
    xin = net.guess_pack(to_gpu(w), to_gpu(ys), to_gpu(n2), scal, feats, 1.0, W)
    assert rel_l2(xin.cpu().numpy(), oguess.pack(w, list(ys), n2, rs, feats, 1.0, W)) < 1e-6
    out = np.random.default_rng(5).standard_normal((3, 2 * ncomp, N, N)).astype(np.float32)
    t = net.guess_unpack(to_gpu(w), to_gpu(out), scal)
    assert rel_l2(t.cpu().numpy(), oguess.unpack(w, out.astype(np.float64), rs)) < 1e-12
    co = op.coefficients(g, n2, ncomp == 2)
    co0 = op.coefficients(g, np.ones_like(n2), ncomp == 2)
    px = np.stack([op.apply_zbar(g, co, y) - op.apply_zbar(g, co0, y) for y in ys])
    tgt = net.guess_target(to_gpu(px), scal)
    assert rel_l2(tgt.cpu().numpy(), oguess.target(px, rs)) < 1e-6


def test_learned_guess_end_to_end():
    """Train on solve pairs the propagator makes (64 x 64, random media and beams), then step
    held-out problems with the learned guesses: the net beats the free-space guess on held-out
    pairs, every solve still meets tol, and the step equals the zero-start step to tolerance.
    The trained net's guesses take fewer GMRES iterations in total than the zero start on the
    held-out steps (both counts printed)."""
    torch = _cuda()
    from paper_2410_17446_amd import learn
    from paper_2410_17446_amd.unet import UNet
    N, W, tol = 64, 8, 1e-10
    wl = workload(N=N, W=W, npoles=8, tol=tol)
    f = wl["fit"]
    net = UNet(3, 16, 7, 2, seed=2)
    X, T = learn.generate(net, f, wl["c"], wl["d"], N, 1, count=48, seed=1, tol=1e-11)
    Xv, Tv = learn.generate(net, f, wl["c"], wl["d"], N, 1, count=6, seed=2, tol=1e-11)
    losses = learn.train(net, X, T, steps=400, batch=8, lr=2e-3, seed=0)
    mse, mse0 = learn.evaluate(net, Xv, Tv)
    print(f"held-out mse {mse:.3e} vs free-space guess {mse0:.3e}; train loss {losses[0]:.3e} -> "
          f"{np.mean(losses[-20:]):.3e}")
    assert mse < 0.5 * mse0
    plan = gpu_plan(wl)
    lg = learn.LearnedGuess(plan, net)
    plain = gpu_plan(wl)
    tot_l = tot_p = 0
    for i in range(3):
        n2 = to_gpu(inputs.random_medium(N, 0.25, 777 + i))
        w = to_gpu(inputs.random_beam(N, 0.25, 1, 888 + i))
        out_l, acc = lg.step(w, n2)
        it_l, rr_l = plan.stats()
        out_p = plain.step(w, n2)
        it_p, _ = plain.stats()
        assert max(rr_l) <= tol
        assert rel_l2(out_l.cpu().numpy(), out_p.cpu().numpy()) < 1e-8
        print(f"held-out step {i}: accepted {acc}, iterations learned {it_l} vs plain {it_p}")
        tot_l += sum(it_l)
        tot_p += sum(it_p)
    print(f"total iterations: learned {tot_l}, plain {tot_p}")
    assert tot_l < tot_p, (tot_l, tot_p)
