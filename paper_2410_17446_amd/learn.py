"""Learned initial guesses: the guess step, data generation from the propagator,
and training, all driven through the library (hp.h, hp_unet.h).

The network's job and the fallback are described in include/hp_unet.h: for
pole k it predicts the correction u_k - w = -P x_k, the guess is
x0_k = M_k^{-1}(w + sigma_k net_k), and the step keeps the zero start for any
pole whose guess has a larger FP64 residual than the zero start.  The guess
step itself is the plan's HP_GUESS_LEARNED mode (the library orders its own
calls); every arithmetic step of data generation and training (preconditioner
solves, feature planes, forward and reverse passes, Adam, the GMRES solves
that make the training pairs) runs in the library's HIP kernels; this module
only orders those calls and holds tensors.
"""
from __future__ import annotations

import time

import numpy as np

from . import hp, inputs
from .unet import UNet


def pole_features(poles) -> np.ndarray:
    """(K, 2): asinh of the real and imaginary parts of each pole."""
    p = np.asarray(poles, dtype=np.complex128)
    return np.stack([np.arcsinh(p.real), np.arcsinh(p.imag)], axis=1)


class LearnedGuess:
    """The plan's learned-guess mode: the net is attached with hp_set_guess_net and the mode set
    to HP_GUESS_LEARNED, so the library itself computes every pole's starting point at the start
    of each step (preconditioner solves, feature planes, forward passes on `chunk` poles at a
    time); this class only makes those two calls and steps."""

    def __init__(self, plan: hp.Plan, net: UNet, chunk: int = 8):
        self.plan, self.net = plan, net
        plan.set_guess_net(net, chunk)
        plan.set_guess(hp.HP_GUESS_LEARNED)

    def step(self, w, n2=None, E_out=None):
        """One step from learned guesses: (E_out, accepted flags)."""
        return self.plan.step_guess(w, None, n2=n2, E_out=E_out)


def plan_for(N, ncomp, poles, residues, r_inf, d2, d1, W, tol, precision=hp.HP_FP64, eta=0.25, dz=1.0):
    return hp.Plan(nx=N, ny=N, dx=0.25, dy=0.25, k0=inputs.K0, n0=1.0, dz=dz, ncomp=ncomp, poles=poles,
                   residues=residues, r_inf=r_inf, d2=d2, d1=d1, edge_width=W, edge_eta=eta, tol=tol,
                   restart=30, max_cycles=20, precision=precision)


def generate(net: UNet, fit, d2, d1, N, ncomp, count, seed, tol=1e-10, W=None, fields_per_medium=2,
             poles_per_field=None):
    """Training pairs (X_in, T) as float32 device tensors (S, 4 ncomp + 3, N, N) and
    (S, 2 ncomp, N, N): `count` (medium, field) draws from inputs.random_medium and
    inputs.random_beam (seeded), each solved in FP64 for every pole (or a seeded subset of
    poles_per_field poles) by hp_solve; the target is -P x / sigma (hp_apply_medium,
    hp_guess_target)."""
    import torch
    W = W if W is not None else N // 8
    poles = np.asarray(fit["poles"])
    K = len(poles)
    feats = pole_features(poles)
    plan = plan_for(N, ncomp, poles, fit["residues"], fit["r_inf"], d2, d1, W, tol)
    rng = np.random.Generator(np.random.PCG64(seed))
    X, T = [], []
    for i in range(count):
        if i % fields_per_medium == 0:
            n2 = torch.from_numpy(inputs.random_medium(N, 0.25, seed * 100003 + i)).cuda()
            plan.set_medium(n2)
        w = torch.from_numpy(inputs.random_beam(N, 0.25, ncomp, seed * 100019 + i)).cuda()
        ks = np.arange(K) if poles_per_field is None else np.sort(rng.choice(K, poles_per_field, replace=False))
        Y = torch.empty((len(ks), ncomp, N, N), dtype=torch.complex128, device="cuda")
        PX = torch.empty_like(Y)
        for j, k in enumerate(ks):
            plan.apply_preconditioner(int(k), w, Y[j])
            x = plan.solve(int(k), w)
            plan.apply_medium(x, PX[j])
        scal = net.guess_stats(w, Y, n2, 1.0, W)
        X.append(net.guess_pack(w, Y, n2, scal, feats[ks], 1.0, W))
        T.append(net.guess_target(PX, scal))
    plan.close()
    return torch.cat(X), torch.cat(T)


def train(net: UNet, X, T, steps, batch=8, lr=1e-3, seed=0, log_every=0, lr_final=None):
    """Adam on mean squared error over shuffled mini-batches; returns the loss per step.
    lr decays geometrically to lr_final (default lr / 10) over the run."""
    import torch
    S = X.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    losses = []
    lr_final = lr / 10 if lr_final is None else lr_final
    perm = torch.randperm(S, generator=g)
    pos = 0
    t0 = time.perf_counter()
    for s in range(steps):
        if pos + batch > S:
            perm = torch.randperm(S, generator=g)
            pos = 0
        idx = perm[pos:pos + batch].cuda()
        pos += batch
        xb = X.index_select(0, idx).contiguous()
        tb = T.index_select(0, idx).contiguous()
        losses.append(net.grad(xb, tb))
        net.adam(lr * (lr_final / lr) ** (s / max(1, steps - 1)))
        if log_every and (s + 1) % log_every == 0:
            print(f"# train step {s + 1}/{steps}: loss {np.mean(losses[-log_every:]):.4e} "
                  f"({time.perf_counter() - t0:.1f} s)", flush=True)
    return losses


def evaluate(net: UNet, X, T, batch=8):
    """Mean squared error of the net on (X, T) and of the zero output (the free-space guess)."""
    import torch
    se, se0, n = 0.0, 0.0, 0
    for i in range(0, X.shape[0], batch):
        y = net.forward(X[i:i + batch].contiguous())
        t = T[i:i + batch]
        se += float(torch.sum((y.double() - t.double()) ** 2))
        se0 += float(torch.sum(t.double() ** 2))
        n += t.numel()
    return se / n, se0 / n
