"""Operator matrix Zbar and its coefficient fields (oracle; test infrastructure).

Grid reading (the paper's grid is interior + PML layers, Sec. 4.1): an N x N
array per field component; node index i = 0..N-1 per axis, node 0 and the
virtual node N are homogeneous-Dirichlet nodes, unknowns are 1..N-1.  Axis 0
of an array is y (rows), axis 1 is x (columns).  d(i, j) = min(i, N-i, j, N-j)
is the distance in cells to the nearest Dirichlet node.

Finite differences (Sec. 4.1): 13-point stencils along one axis,
    (D2 u)_i = [c0 u_i + sum_{m=1..6} c_m (u_{i+m} + u_{i-m})] / h^2
    (D1 u)_i = sum_{m=1..6} d_m (u_{i+m} - u_{i-m}) / h
closed by odd reflection at the Dirichlet nodes (u_{-m} = -u_m,
u_{N+m} = -u_{N-m}).

Operator (Sec. 2, eq. Z_bar_eq), s = 1/(k0 n0)^2, psi = ln n^2:
    scalar:  Zbar w = s (D2x + D2y) w + V w
    vector:  (Zbar w)_1 = s[(D2x+D2y) w1 + psi_xx w1 + psi_x D1x w1
                            + psi_xy w2 + psi_y D1x w2] + V w1
             (Zbar w)_2 = s[psi_xy w1 + psi_x D1y w1 + (D2x+D2y) w2
                            + psi_yy w2 + psi_y D1y w2] + V w2
with V = k0^2 (n^2 - n0^2) s = (n^2 - n0^2)/n0^2.

Edge layer (Sec. 4.1 zeroes the n^2 and psi coefficients inside the boundary
layers): for d <= W the medium terms V, psi_* are zero, so inside the solves
the layer is free space and the free-space preconditioner is exact there.  In
place of the paper's PML the layer is a lossy medium n^2 = n0^2 + i eta(d),
eta(d) = eta_max ((W + 1 - d)/W)^2 for 1 <= d <= W, whose loss over one step
is applied to the field after the step as the factor
    m(d) = exp(-k0 dz eta(d) / (2 n0))
(the attenuation of a plane wave at normal incidence, Im k_z = k0 eta/(2 n0)).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def _shift_odd(u: np.ndarray, m: int, axis: int) -> np.ndarray:
    """Array whose entry i along `axis` is u_{i+m} under odd reflection about 0 and N.

    u has length N along axis with u_0 = 0 (node N is virtual, value 0).
    """
    N = u.shape[axis]
    idx = np.arange(N) + m
    sign = np.ones(N)
    lo = idx < 0
    idx[lo] = -idx[lo]
    sign[lo] = -1.0
    hi = idx > N
    idx[hi] = 2 * N - idx[hi]
    sign[hi] = -1.0
    at_n = idx == N
    idx[at_n] = 0          # u_N = 0 = u_0
    shape = [1] * u.ndim
    shape[axis] = N
    return np.take(u, idx, axis=axis) * sign.reshape(shape)


def d2(u: np.ndarray, c: np.ndarray, h: float, axis: int) -> np.ndarray:
    out = c[0] * u
    for m in range(1, len(c)):
        out = out + c[m] * (_shift_odd(u, m, axis) + _shift_odd(u, -m, axis))
    return _dirichlet(out / h ** 2)


def d1(u: np.ndarray, d: np.ndarray, h: float, axis: int) -> np.ndarray:
    out = np.zeros_like(u)
    for m in range(1, len(d) + 1):
        out = out + d[m - 1] * (_shift_odd(u, m, axis) - _shift_odd(u, -m, axis))
    return _dirichlet(out / h)


def _dirichlet(u: np.ndarray) -> np.ndarray:
    u = u.copy()
    u[..., 0, :] = 0.0
    u[..., :, 0] = 0.0
    return u


def edge_distance(N: int) -> np.ndarray:
    i = np.arange(N)
    di = np.minimum(i, N - i)
    return np.minimum(di[:, None], di[None, :])


@dataclass
class Coefficients:
    """Medium coefficient fields of Zbar on an N x N grid."""
    V: np.ndarray                 # complex (N, N)
    psi_x: np.ndarray | None = None
    psi_y: np.ndarray | None = None
    psi_xx: np.ndarray | None = None
    psi_yy: np.ndarray | None = None
    psi_xy: np.ndarray | None = None


@dataclass
class Grid:
    N: int
    dx: float
    dy: float
    k0: float
    n0: float
    c: np.ndarray         # D2 stencil c0..c6
    d: np.ndarray         # D1 stencil d1..d6
    W: int                # edge layer width (cells)
    eta_max: float        # peak Im(n^2) in the layer

    @property
    def s(self) -> float:
        return 1.0 / (self.k0 * self.n0) ** 2


def coefficients(g: Grid, n2: np.ndarray, vector: bool) -> Coefficients:
    """Coefficient fields from a real n^2(x, y) (Sec. 2 eq. Z_bar_eq, Sec. 4.1)."""
    n2 = np.asarray(n2, dtype=float)
    dist = edge_distance(g.N)
    inner = dist > g.W
    V = np.where(inner, (n2 - g.n0 ** 2) / g.n0 ** 2, 0.0).astype(complex)
    V[0, :] = 0.0
    V[:, 0] = 0.0
    if not vector:
        return Coefficients(V=V)
    psi = np.log(n2)
    # Each derivative of psi is evaluated only where d > W >= 6, where the
    # 13-point stencil never reaches a Dirichlet node; elsewhere it is zero.
    px = _plain_d1(psi, g.d, g.dx, axis=1)
    py = _plain_d1(psi, g.d, g.dy, axis=0)
    pxx = _plain_d2(psi, g.c, g.dx, axis=1)
    pyy = _plain_d2(psi, g.c, g.dy, axis=0)
    pxy = _plain_d1(_plain_d1(psi, g.d, g.dx, axis=1), g.d, g.dy, axis=0)
    z = lambda a: np.where(inner, a, 0.0)
    return Coefficients(V=V, psi_x=z(px), psi_y=z(py), psi_xx=z(pxx), psi_yy=z(pyy), psi_xy=z(pxy))


def _plain_d2(u, c, h, axis):
    out = c[0] * u
    for m in range(1, len(c)):
        out = out + c[m] * (np.roll(u, -m, axis) + np.roll(u, m, axis))
    return out / h ** 2


def _plain_d1(u, d, h, axis):
    out = np.zeros_like(u)
    for m in range(1, len(d) + 1):
        out = out + d[m - 1] * (np.roll(u, -m, axis) - np.roll(u, m, axis))
    return out / h


def absorber_mask(g: Grid, dz: float) -> np.ndarray:
    """Per-step loss factor m(d) of the edge layer (1 outside it, 0 on Dirichlet nodes)."""
    dist = edge_distance(g.N)
    layer = (dist >= 1) & (dist <= g.W)
    eta = np.where(layer, g.eta_max * ((g.W + 1 - dist) / g.W) ** 2, 0.0)
    m = np.exp(-g.k0 * dz * eta / (2.0 * g.n0))
    m[0, :] = 0.0
    m[:, 0] = 0.0
    return m


def apply_zbar(g: Grid, co: Coefficients, w: np.ndarray) -> np.ndarray:
    """Zbar w for w of shape (ncomp, N, N); row/column 0 of the result are zero."""
    s = g.s
    lap = lambda u: d2(u, g.c, g.dx, 1) + d2(u, g.c, g.dy, 0)
    if w.shape[0] == 1:
        return _dirichlet(s * lap(w[0]) + co.V * w[0])[None]
    w1, w2 = w[0], w[1]
    d1x = lambda u: d1(u, g.d, g.dx, 1)
    d1y = lambda u: d1(u, g.d, g.dy, 0)
    o1 = s * (lap(w1) + co.psi_xx * w1 + co.psi_x * d1x(w1) + co.psi_xy * w2 + co.psi_y * d1x(w2)) + co.V * w1
    o2 = s * (co.psi_xy * w1 + co.psi_x * d1y(w1) + lap(w2) + co.psi_yy * w2 + co.psi_y * d1y(w2)) + co.V * w2
    return np.stack([_dirichlet(o1), _dirichlet(o2)])


def apply_shifted(g: Grid, co: Coefficients, w: np.ndarray, b: complex) -> np.ndarray:
    """(Zbar - b I) w (Sec. 2 eq. W_k_def)."""
    return _dirichlet_all(apply_zbar(g, co, w) - b * w)


def _dirichlet_all(w):
    w = w.copy()
    w[:, 0, :] = 0.0
    w[:, :, 0] = 0.0
    return w


def dense_zbar(g: Grid, co: Coefficients, ncomp: int) -> np.ndarray:
    """Dense matrix of Zbar on the unknowns (brute force, tiny grids only)."""
    N = g.N
    n = ncomp * (N - 1) ** 2
    M = np.zeros((n, n), dtype=complex)
    for col in range(n):
        e = np.zeros(n, dtype=complex)
        e[col] = 1.0
        M[:, col] = pack(apply_zbar(g, co, unpack(e, ncomp, N)))
    return M


def pack(w: np.ndarray) -> np.ndarray:
    """Unknowns of a (ncomp, N, N) field as a flat vector."""
    return w[:, 1:, 1:].reshape(-1)


def unpack(v: np.ndarray, ncomp: int, N: int) -> np.ndarray:
    w = np.zeros((ncomp, N, N), dtype=complex)
    w[:, 1:, 1:] = v.reshape(ncomp, N - 1, N - 1)
    return w
