"""One propagation step and the propagation loop (oracle; test infrastructure).

Sec. 2, eqs. Wk_define / approx_prop / W_k_def: with the partial fractions
r(z) = r_inf + sum_k a_k/(z - b_k) of exp(iK sqrt(1+z)) and K = k0 n0 dz,
    w(z + dz) = e^{-iK} [ r_inf w + sum_k a_k x_k ],   (Zbar - b_k I) x_k = w.
(The paper solves with right-hand side e^{-iK} a_k w; the solves are linear,
so solving with w and weighting afterwards gives the same field, and the
relative tolerance is unchanged.)  Each solve is the right-preconditioned
GMRES of oracle.gmres with the free-space preconditioner of oracle.precond.
Between steps n^2 (and with it Zbar) may change (Sec. 2, after eq. expop_prop).
The loss of the edge layer is applied to the stepped field as the factor
oracle.operator.absorber_mask (1 outside the layer).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import operator as op
from .gmres import gmres
from .precond import apply_minv


@dataclass
class PFTable:
    poles: np.ndarray       # b_k
    residues: np.ndarray    # a_k
    r_inf: complex          # alpha_NN / beta_NN


@dataclass
class StepStats:
    iters: list             # GMRES iterations per pole
    relres: list            # true relative residual per pole
    cycle_iters: list


def solve_pole(g: op.Grid, co: op.Coefficients, w: np.ndarray, b_k: complex, tol: float,
               restart: int = 30, schedule=None, workers: int = -1, x0: np.ndarray | None = None):
    """(Zbar - b_k I) x = w by preconditioned GMRES; x0 (ncomp, N, N) an optional start."""
    ncomp, N = w.shape[0], g.N
    A = lambda x: op.pack(op.apply_shifted(g, co, op.unpack(x, ncomp, N), b_k))
    Minv = lambda v: op.pack(apply_minv(g, op.unpack(v, ncomp, N), b_k, workers))
    return gmres(A, Minv, op.pack(w), tol, restart=restart, schedule=schedule,
                 x0=None if x0 is None else op.pack(x0))


def judge_guess(g: op.Grid, co: op.Coefficients, w: np.ndarray, b_k: complex, x0) -> bool:
    """The fallback rule for an initial guess: use x0 only when its residual is below that of
    the zero start, ||w - (Zbar - b_k I) x0|| < ||w||."""
    if x0 is None:
        return False
    r0 = w - op.apply_shifted(g, co, x0, b_k)
    return bool(np.linalg.norm(r0) < np.linalg.norm(w))


def step(g: op.Grid, co: op.Coefficients, w: np.ndarray, pf: PFTable, dz: float, tol: float,
         restart: int = 30, schedules=None, workers: int = -1, guesses=None):
    """Advance the envelope field w (ncomp, N, N) by one step dz.  guesses: None or one
    initial guess (or None) per pole, each used only if judge_guess accepts it."""
    K = g.k0 * g.n0 * dz
    ncomp, N = w.shape[0], g.N
    acc = pf.r_inf * op.pack(w)
    iters, relres, cyc = [], [], []
    for k, (b_k, a_k) in enumerate(zip(pf.poles, pf.residues)):
        x0 = None if guesses is None else guesses[k]
        if not judge_guess(g, co, w, b_k, x0):
            x0 = None
        res = solve_pole(g, co, w, b_k, tol, restart,
                         schedule=None if schedules is None else schedules[k], workers=workers, x0=x0)
        acc = acc + a_k * res.x
        iters.append(res.iters)
        relres.append(res.relres)
        cyc.append(res.cycle_iters)
    out = op.unpack(np.exp(-1j * K) * acc, ncomp, N) * op.absorber_mask(g, dz)[None]
    return out, StepStats(iters=iters, relres=relres, cycle_iters=cyc)


def propagate(g: op.Grid, n2_steps, w: np.ndarray, pf: PFTable, dz: float, nsteps: int, tol: float,
              restart: int = 30, schedules=None, workers: int = -1):
    """nsteps steps; n2_steps is one real (N, N) array (z-independent) or a list of them."""
    vector = w.shape[0] == 2
    stats = []
    co = None
    for s in range(nsteps):
        if isinstance(n2_steps, (list, tuple)):
            co = op.coefficients(g, n2_steps[s], vector)
        elif co is None:
            co = op.coefficients(g, n2_steps, vector)
        w, st = step(g, co, w, pf, dz, tol, restart,
                     None if schedules is None else schedules[s], workers)
        stats.append(st)
    return w, stats
