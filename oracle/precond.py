"""Free-space preconditioner (oracle; test infrastructure).

Sec. 4.2.1 (eq. Z_bar_fs_def) keeps only the scaled transverse Laplacian,
block-diagonal over the field components; the preconditioner of the shifted
system k is Zbar_fs - b_k I.  Sec. 4.2.2 (eqs. freespace_prob, shift_identity,
fs_sylvester) writes each component's free-space problem as the Sylvester
equation
    (Dx - b/2 I) W + W (Dy - b/2 I)^T = rhs,
with Dx, Dy the scaled second-derivative matrices.

With the odd-reflection closure the 13-point second-derivative matrix on the
N-1 unknowns of an axis is diagonalised exactly by the orthonormal DST-I,
    S_pj = sqrt(2/N) sin(pi p j / N),   S = S^T = S^-1,
with eigenvalues (scaled by s = 1/(k0 n0)^2)
    mu_p = s [c0 + 2 sum_m c_m cos(m pi p / N)] / h^2.
So the Sylvester solve is  W = S_y [(S_y rhs S_x) / (mu^y_p + mu^x_q - b)] S_x,
the same matrix the Bartels-Stewart route of Sec. 4.2.2 would produce.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from .operator import Grid


def dst2(u: np.ndarray, workers: int = -1) -> np.ndarray:
    """Orthonormal 2-D DST-I over the unknowns of (..., N, N) arrays (row/col 0 ignored)."""
    out = np.zeros_like(u)
    out[..., 1:, 1:] = sfft.dstn(u[..., 1:, 1:], type=1, axes=(-2, -1), norm="ortho", workers=workers)
    return out


def mu(N: int, h: float, c: np.ndarray, s: float) -> np.ndarray:
    """Eigenvalues mu_p (p = 1..N-1) of s * D2 along one axis."""
    p = np.arange(1, N)
    m = np.arange(1, len(c))
    sym = c[0] + 2.0 * np.cos(np.outer(p * np.pi / N, m)) @ c[1:]
    return s * sym / h ** 2


def spectrum(g: Grid) -> np.ndarray:
    """mu^y_p + mu^x_q on the (N-1) x (N-1) unknowns, indexed [p-1, q-1]."""
    my = mu(g.N, g.dy, g.c, g.s)
    mx = mu(g.N, g.dx, g.c, g.s)
    return my[:, None] + mx[None, :]


def apply_minv(g: Grid, y: np.ndarray, b: complex, workers: int = -1) -> np.ndarray:
    """M^-1 y = (Zbar_fs - b I)^-1 y, component by component, y of shape (ncomp, N, N)."""
    lam = spectrum(g) - b
    t = dst2(y, workers)
    t[..., 1:, 1:] = t[..., 1:, 1:] / lam
    return dst2(t, workers)


def dense_d2(N: int, c: np.ndarray, h: float) -> np.ndarray:
    """Dense (N-1) x (N-1) second-derivative matrix with odd-reflection closure."""
    D = np.zeros((N - 1, N - 1))
    for j in range(1, N):
        D[j - 1, j - 1] += c[0]
        for m in range(1, len(c)):
            for k in (j + m, j - m):
                sign = 1.0
                if k < 0:
                    k, sign = -k, -1.0
                elif k > N:
                    k, sign = 2 * N - k, -1.0
                if 1 <= k <= N - 1:
                    D[j - 1, k - 1] += sign * c[m]
    return D / h ** 2
