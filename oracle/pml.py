"""Perfectly matched layer by complex-coordinate stretching (oracle; test infrastructure).

Sec. 4.1: the physical domain is surrounded by PML layers, applied by modifying the
peripheral rows of the second- and first-derivative matrices that act on the transverse field
(the complex-coordinate transformation), while the n^2 and psi coefficient entries are zero
inside the layers.  The paper defers the details to earlier work; the reading taken here:

Along each axis the coordinate is stretched, d/dx -> (1/s(x)) d/dx with
    s = 1 + i sigma,   sigma(d) = sigma_max ((W + 1 - d)/W)^2 for 1 <= d <= W, 0 for d > W,
d the distance in cells to that axis's nearer Dirichlet node (0 or N).  Then
    d^2/dx~^2 = (1/s) d/dx ((1/s) d/dx) = (1/s^2) d^2/dx^2 - (s'/s^3) d/dx,
discretised node by node with the 13-point D2 and D1 of Sec. 4.1 (odd reflection at the
Dirichlet nodes) and the exact derivative s' of the profile.  Scalar operator (eq. Z_bar_eq
with the stretched derivatives):
    Zbar w = (1/(k0 n0)^2) (D2x~ + D2y~) w + V w,   V = (n^2 - n0^2)/n0^2, zero where d <= W
on either axis.  The free-space operator (eq. Z_bar_fs_def) is separable,
    Zbar_fs = (1/(k0 n0)^2) (D2x~ (x) I + I (x) D2y~),
and the preconditioner of pole b_k is the Sylvester equation of eq. fs_sylvester with the
stretched matrices, solved here by Bartels-Stewart (scipy.linalg.solve_sylvester), the route the
paper names.  A step is w(z + dz) = e^{-iK}(r_inf w + sum_k a_k x_k) with no separate loss: the
layers absorb.  With s = 1 + i sigma a mode ~ exp(i kx x~) that travels outward decays in the
layer, and the free-space eigenvalues move into the upper half plane, where the rational
function has no poles.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from . import operator as op
from .gmres import gmres


@dataclass
class PMLGrid:
    N: int                # nodes 0..N-1 per axis; 0 and N Dirichlet, unknowns 1..N-1
    h: float              # spacing (both axes)
    k0: float
    n0: float
    c: np.ndarray         # D2 stencil c0..c6
    d: np.ndarray         # D1 stencil d1..d6
    W: int                # PML width (cells)
    sigma_max: float

    @property
    def s(self) -> float:
        return 1.0 / (self.k0 * self.n0) ** 2


def stretch(g: PMLGrid):
    """(s, ds/dx) at the nodes 0..N-1 of one axis."""
    i = np.arange(g.N)
    left = i <= g.N - i                       # the nearer Dirichlet node is 0
    dist = np.minimum(i, g.N - i)
    t = np.where((dist >= 1) & (dist <= g.W), (g.W + 1 - dist) / g.W, 0.0)
    sigma = g.sigma_max * t ** 2
    # d sigma/dx: sigma falls toward the interior; distance grows with x on the left side
    dsig_dd = -2.0 * g.sigma_max * t / g.W    # d sigma / d(dist), per cell
    dsig_dx = np.where(left, dsig_dd, -dsig_dd) / g.h
    return 1.0 + 1j * sigma, 1j * dsig_dx


def d2_stretched_matrix(g: PMLGrid) -> np.ndarray:
    """Dense (N-1) x (N-1) matrix of d^2/dx~^2 on the unknowns 1..N-1 of one axis."""
    n = g.N - 1
    D2 = np.zeros((n, n))
    D1 = np.zeros((n, n))
    for j in range(1, g.N):
        for m in range(-6, 7):
            k = j + m
            sign = 1.0
            if k < 0:
                k, sign = -k, -1.0
            elif k > g.N:
                k, sign = 2 * g.N - k, -1.0
            if not 1 <= k <= g.N - 1:
                continue
            c2 = g.c[abs(m)]
            c1 = 0.0 if m == 0 else (g.d[abs(m) - 1] if m > 0 else -g.d[abs(m) - 1])
            D2[j - 1, k - 1] += sign * c2
            D1[j - 1, k - 1] += sign * c1
    s, ds = stretch(g)
    s, ds = s[1:], ds[1:]
    return (D2 / g.h ** 2) / (s ** 2)[:, None] - (ds / s ** 3)[:, None] * (D1 / g.h)


def medium(g: PMLGrid, n2: np.ndarray) -> np.ndarray:
    """V on the N x N grid: (n^2 - n0^2)/n0^2, zero in the layers and on the Dirichlet nodes."""
    dist = op.edge_distance(g.N)
    V = np.where(dist > g.W, (np.asarray(n2, float) - g.n0 ** 2) / g.n0 ** 2, 0.0).astype(complex)
    V[0, :] = 0.0
    V[:, 0] = 0.0
    return V


def apply_shifted(g: PMLGrid, V: np.ndarray, w: np.ndarray, b: complex, D=None) -> np.ndarray:
    """(Zbar - b I) w for a scalar field w (N, N); row/column 0 of the result are zero."""
    D = d2_stretched_matrix(g) if D is None else D
    u = w[1:, 1:]
    out = np.zeros_like(w, dtype=complex)
    out[1:, 1:] = g.s * (u @ D.T + D @ u) + V[1:, 1:] * u - b * u
    return out


def apply_minv(g: PMLGrid, y: np.ndarray, b: complex, D=None) -> np.ndarray:
    """(Zbar_fs - b I)^-1 y by the Sylvester equation of eq. fs_sylvester (Bartels-Stewart):
    (s D2y~ - b/2) W + W (s D2x~ - b/2)^T = y on the unknowns (axis 0 is y, axis 1 is x)."""
    D = d2_stretched_matrix(g) if D is None else D
    A = g.s * D - 0.5 * b * np.eye(D.shape[0])
    out = np.zeros_like(y, dtype=complex)
    out[1:, 1:] = sla.solve_sylvester(A, A.T, y[1:, 1:])
    return out


def solve_pole(g: PMLGrid, V, w, b_k, tol, restart=30, schedule=None, D=None):
    D = d2_stretched_matrix(g) if D is None else D
    N = g.N
    A = lambda x: op.pack(apply_shifted(g, V, op.unpack(x, 1, N)[0], b_k, D)[None])
    Minv = lambda v: op.pack(apply_minv(g, op.unpack(v, 1, N)[0], b_k, D)[None])
    return gmres(A, Minv, op.pack(w[None]), tol, restart=restart, schedule=schedule)


def step(g: PMLGrid, V, w, poles, residues, r_inf, dz, tol, restart=30, schedules=None):
    """One step of eq. approx_prop with the PML operator; returns (w_out, per-pole results)."""
    D = d2_stretched_matrix(g)
    K = g.k0 * g.n0 * dz
    acc = r_inf * op.pack(w[None])
    res = []
    for k, (b, a) in enumerate(zip(poles, residues)):
        r = solve_pole(g, V, w, b, tol, restart, None if schedules is None else schedules[k], D)
        acc = acc + a * r.x
        res.append(r)
    return np.exp(-1j * K) * op.unpack(acc, 1, g.N)[0], res


# ---------------------------------------------------------------- vector fields (E_x, E_y)

def vector_grid(g: PMLGrid) -> op.Grid:
    """The plain operator's grid with its edge region set to the PML width (and no loss): the
    coefficient planes V and psi of eq. Z_bar_eq are then zero inside the layers."""
    return op.Grid(N=g.N, dx=g.h, dy=g.h, k0=g.k0, n0=g.n0, c=g.c, d=g.d, W=g.W, eta_max=0.0)


def apply_shifted_vector(g: PMLGrid, co, w: np.ndarray, b: complex, D=None, D0=None) -> np.ndarray:
    """(Zbar~ - b I) w for a vector field w (2, N, N): eq. Z_bar_eq with the stretched transverse
    second derivatives.  co: op.coefficients(vector_grid(g), n2, True).  The psi terms and V vanish
    in the layers, the only rows whose first derivatives the stretching changes; elsewhere g = 1, so
    the plain operator's psi terms are the stretched operator's, and only its Laplacian rows change:
    the plain s (D2x + D2y) is replaced by s (D2x~ + D2y~) in each component."""
    D = d2_stretched_matrix(g) if D is None else D
    if D0 is None:
        D0 = d2_stretched_matrix(PMLGrid(g.N, g.h, g.k0, g.n0, g.c, g.d, g.W, 0.0))
    out = op.apply_shifted(vector_grid(g), co, w, b)
    for c in range(2):
        u = w[c, 1:, 1:]
        out[c, 1:, 1:] += g.s * ((u @ D.T + D @ u) - (u @ D0.T + D0 @ u))
    return out


def solve_pole_vector(g: PMLGrid, co, w, b_k, tol, restart=30, schedule=None, D=None, D0=None):
    """The shifted vector solve; the preconditioner is the Sylvester solve per component (the
    free-space operator does not couple E_x and E_y)."""
    D = d2_stretched_matrix(g) if D is None else D
    if D0 is None:
        D0 = d2_stretched_matrix(PMLGrid(g.N, g.h, g.k0, g.n0, g.c, g.d, g.W, 0.0))
    N = g.N
    A = lambda x: op.pack(apply_shifted_vector(g, co, op.unpack(x, 2, N), b_k, D, D0))

    def Minv(v):
        y = op.unpack(v, 2, N)
        return op.pack(np.stack([apply_minv(g, y[c], b_k, D) for c in range(2)]))

    return gmres(A, Minv, op.pack(w), tol, restart=restart, schedule=schedule)


def step_vector(g: PMLGrid, co, w, poles, residues, r_inf, dz, tol, restart=30, schedules=None):
    """One step of eq. approx_prop for a vector field with the PML operator."""
    D = d2_stretched_matrix(g)
    D0 = d2_stretched_matrix(PMLGrid(g.N, g.h, g.k0, g.n0, g.c, g.d, g.W, 0.0))
    K = g.k0 * g.n0 * dz
    acc = r_inf * op.pack(w)
    res = []
    for k, (b, a) in enumerate(zip(poles, residues)):
        r = solve_pole_vector(g, co, w, b, tol, restart, None if schedules is None else schedules[k], D, D0)
        acc = acc + a * r.x
        res.append(r)
    return np.exp(-1j * K) * op.unpack(acc, 2, g.N), res
