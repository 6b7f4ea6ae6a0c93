"""Pseudo-differential form of the propagator (oracle; test infrastructure).

Sec. 2, eqs. eq_barZfactor / eq_barZfactor2: the one-way equation
    dw/dz = i k0 n0 (sqrt(I + Zbar) - I) w.
Sec. 3.2 (eqs. Mobius, Cauchy, pf_sqrt_exp) and Appendix A approximate
sqrt(1 + zeta) by partial fractions built from a Cauchy integral:
  * the Moebius map w(zeta) = (zeta + 1 + i alpha)/(zeta + 1 - i alpha) sends the
    branch point at zeta = -inf to w = 1, and the cut is put on w in [-1, 1];
  * g(w) = c_alpha (1 - (1/pi) int_{-1}^{1} sqrt((1+eta)/(1-eta)) / (eta - w) deta),
    c_alpha = sqrt(alpha) e^{i pi/4};
  * the integral is replaced by the N-point Gauss-Jacobi rule (eta_j, omega_j) of
    the weight (1 - eta)^(-1/2) (1 + eta)^(1/2);
  * mapping back to zeta and dividing each term out gives
        sqrt(1 + zeta) ~ (c_alpha + sum_j wt_j) - sum_j i alpha wt_j (1 + sigma_j) / (zeta + 1 + i alpha sigma_j),
    wt_j = (c_alpha/pi) omega_j/(1 - eta_j), sigma_j = (1 + eta_j)/(1 - eta_j),
    i.e. poles b_j = -(1 + i alpha sigma_j), residues a_j = -i alpha wt_j (1 + sigma_j),
    constant r_inf = c_alpha + sum_j wt_j.  The solves are those of eq. Auxiliary_W.

The paper leaves the z-integrator open (eq. ApproxPropagator_W is an ODE in z).
Reading used here: the classical fourth-order Runge-Kutta method with step
h = dz / substeps, each stage one application of
    L(v) = i k0 n0 (r(Zbar) v - v),   r(Zbar) v = r_inf v + sum_j a_j (Zbar - b_j I)^{-1} v,
every shifted solve by the right-preconditioned GMRES of oracle.gmres.  The loss
of the edge layer is applied after every substep as the factor
oracle.operator.absorber_mask(grid, h), as the exponential form applies it
after every step.
"""
from __future__ import annotations

import numpy as np
from scipy.special import roots_jacobi

from . import operator as op
from .step import PFTable, solve_pole


def gauss_jacobi_sqrt(N: int):
    """Nodes and weights of the N-point Gauss rule for int_{-1}^{1} f(eta) sqrt((1+eta)/(1-eta)) deta."""
    eta, omega = roots_jacobi(N, -0.5, 0.5)
    return eta, omega


def cauchy_sqrt_pf(N: int, alpha: float = 1.0) -> PFTable:
    """Partial fractions of sqrt(1 + zeta) from the Cauchy integral (Sec. 3.2, eq. pf_sqrt_exp)."""
    eta, omega = gauss_jacobi_sqrt(N)
    c_alpha = np.sqrt(alpha) * np.exp(1j * np.pi / 4)
    wt = c_alpha / np.pi * omega / (1.0 - eta)
    sigma = (1.0 + eta) / (1.0 - eta)
    poles = -(1.0 + 1j * alpha * sigma)
    residues = -1j * alpha * wt * (1.0 + sigma)
    return PFTable(poles, residues, complex(c_alpha + wt.sum()))


def sqrt_principal(zeta: np.ndarray) -> np.ndarray:
    """sqrt(1 + zeta) on the real axis: i sqrt(-1 - zeta) below the branch point."""
    zeta = np.asarray(zeta, dtype=float)
    s = 1.0 + zeta
    return np.where(s >= 0, np.sqrt(np.abs(s)) + 0j, 1j * np.sqrt(np.abs(s)))


def apply_r(g: op.Grid, co: op.Coefficients, v: np.ndarray, pf: PFTable, tol: float, restart: int = 30,
            workers: int = -1):
    """r(Zbar) v (packed), with every shifted solve by GMRES; also the iterations per pole."""
    acc = pf.r_inf * op.pack(v)
    iters = []
    for b_k, a_k in zip(pf.poles, pf.residues):
        res = solve_pole(g, co, v, b_k, tol, restart, workers=workers)
        acc = acc + a_k * res.x
        iters.append(res.iters)
    return acc, iters


def rk4_step(g: op.Grid, co: op.Coefficients, w: np.ndarray, pf: PFTable, dz: float, substeps: int, tol: float,
             restart: int = 30, workers: int = -1):
    """Advance w (ncomp, N, N) by dz: `substeps` classical RK4 steps of dw/dz = L(w)."""
    ncomp, N = w.shape[0], g.N
    h = dz / substeps
    ik = 1j * g.k0 * g.n0
    mask = op.absorber_mask(g, h)[None]
    total = np.zeros(len(pf.poles), dtype=int)

    def L(v):
        rv, it = apply_r(g, co, v, pf, tol, restart, workers)
        total[:] += it
        return ik * (op.unpack(rv, ncomp, N) - v)

    u = w.copy()
    for _ in range(substeps):
        k1 = L(u)
        k2 = L(u + 0.5 * h * k1)
        k3 = L(u + 0.5 * h * k2)
        k4 = L(u + h * k3)
        u = (u + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)) * mask
    return u, total


def propagate(g: op.Grid, n2_steps, w: np.ndarray, pf: PFTable, dz: float, nsteps: int, substeps: int, tol: float,
              restart: int = 30, workers: int = -1):
    """nsteps steps of dz; n2_steps is one real (N, N) array or a list with one per step."""
    vector = w.shape[0] == 2
    co = None
    for s in range(nsteps):
        if isinstance(n2_steps, (list, tuple)):
            co = op.coefficients(g, n2_steps[s], vector)
        elif co is None:
            co = op.coefficients(g, n2_steps, vector)
        w, _ = rk4_step(g, co, w, pf, dz, substeps, tol, restart, workers)
    return w


def rk4_amplification(z: np.ndarray) -> np.ndarray:
    """Stability polynomial of classical RK4: the factor one step applies to y' = lambda y, z = h lambda."""
    return 1.0 + z + z ** 2 / 2.0 + z ** 3 / 6.0 + z ** 4 / 24.0
