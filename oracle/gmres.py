"""Right-preconditioned GMRES(m) with Householder Arnoldi (oracle; test infrastructure).

Sec. 4.2 solves each shifted system with the generic right-preconditioned
GMRES of Saad (2003, Sec. 9.5) and keeps the Krylov basis orthogonal with
Householder reflections (Saad 2003, Algorithm 6.10 carried over to the
right-preconditioned operator A M^-1).

Reading of the stopping rule: relative residual ||b - A x|| / ||b||; the inner
cycle stops on the least-squares residual estimate, the cycle's iterate is
then checked with the true residual, and the solve restarts from it if the
true residual is still above tol.  `schedule` forces the number of Arnoldi
steps of each cycle (used to replay the same iteration counts elsewhere).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class GmresResult:
    x: np.ndarray
    iters: int
    cycles: int
    relres: float                       # true relative residual of x
    cycle_iters: list = field(default_factory=list)
    converged: bool = True


def _householder(z: np.ndarray, k: int) -> np.ndarray | None:
    """Unit w (zero above index k) with (I - 2 w w^H) z zero below index k; None if nothing to do."""
    x = z[k:]
    nx = np.linalg.norm(x)
    if nx == 0.0:
        return None
    x0 = x[0]
    phase = x0 / abs(x0) if x0 != 0 else 1.0
    alpha = -phase * nx
    u = x.copy()
    u[0] -= alpha
    nu = np.linalg.norm(u)
    if nu == 0.0:
        return None
    w = np.zeros_like(z)
    w[k:] = u / nu
    return w


def _reflect(w, v):
    if w is None:
        return v
    return v - 2.0 * w * np.vdot(w, v)


def _lsq(Hbar: np.ndarray, beta: complex):
    rhs = np.zeros(Hbar.shape[0], dtype=complex)
    rhs[0] = beta
    y, *_ = np.linalg.lstsq(Hbar, rhs, rcond=None)
    return y, float(np.linalg.norm(rhs - Hbar @ y))


def gmres(A, Minv, b: np.ndarray, tol: float, restart: int = 30, max_cycles: int = 20,
          schedule: list | None = None, x0: np.ndarray | None = None) -> GmresResult:
    """Solve A x = b with right preconditioner Minv (both callables on flat vectors), starting
    from x0 (zero when None).  The iterate of a cycle started at x is x + Minv(V y), V the
    cycle's Arnoldi basis of A Minv from r = b - A x (Saad 2003, Algorithm 9.5); the
    stopping test stays relative to ||b||, whatever the start."""
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=complex)
    if bnorm == 0.0:
        return GmresResult(x=np.zeros_like(b), iters=0, cycles=0, relres=0.0)
    total = 0
    cycle_iters = []
    relres = 1.0
    if x0 is not None:
        relres = float(np.linalg.norm(b - A(x)) / bnorm)
        if schedule is None and relres <= tol:
            return GmresResult(x=x, iters=0, cycles=0, relres=relres)
    ncycles = len(schedule) if schedule is not None else max_cycles
    for cyc in range(ncycles):
        m = schedule[cyc] if schedule is not None else restart
        r0 = b - A(x) if (cyc > 0 or x0 is not None) else b.copy()
        z = r0
        Ws = []
        H = np.zeros((m + 1, m), dtype=complex)
        beta = 0.0
        k = 0
        for j in range(m + 1):
            w = _householder(z, j)
            Ws.append(w)
            hz = _reflect(w, z)
            if j == 0:
                beta = hz[0]
            else:
                H[:j + 1, j - 1] = hz[:j + 1]
                k = j
                _, est = _lsq(H[:k + 1, :k], beta)
                if schedule is None and (est <= tol * bnorm or abs(H[j, j - 1]) == 0.0):
                    break
            if j == m:
                break
            v = np.zeros_like(b)
            v[j] = 1.0
            for i in reversed(range(j + 1)):
                v = _reflect(Ws[i], v)
            z = A(Minv(v))
            for i in range(j + 1):
                z = _reflect(Ws[i], z)
        y, _ = _lsq(H[:k + 1, :k], beta)
        u = np.zeros_like(b)
        for i in reversed(range(k)):
            u[i] += y[i]
            u = _reflect(Ws[i], u)
        x = x + Minv(u)
        total += k
        cycle_iters.append(k)
        relres = float(np.linalg.norm(b - A(x)) / bnorm)
        if schedule is None and relres <= tol:
            return GmresResult(x=x, iters=total, cycles=cyc + 1, relres=relres, cycle_iters=cycle_iters)
    return GmresResult(x=x, iters=total, cycles=len(cycle_iters), relres=relres,
                       cycle_iters=cycle_iters, converged=(schedule is not None or relres <= tol))
