"""Input, output and target planes of the learned initial guess (oracle; test
infrastructure).

Not from the paper.  Around the shifted solves (Zbar - b_k I) x_k = w of Sec. 2
(eq. W_k_def) with the free-space preconditioner M_k of Sec. 4.2.2 and the
medium part P = Zbar - Zbar_fs of the operator, the solution is
x_k = M_k^{-1} u_k with u_k = w - P x_k.  The network predicts the correction
u_k - w from planes of w, y_k = M_k^{-1} w, the medium V and the pole; the
guess is x0_k = M_k^{-1}(w + sigma_k net_k), sigma_k = rms(y_k) rms(V).

Fields are (ncomp, ny, nx) complex arrays whose row 0 and column 0 are the
Dirichlet nodes; the rms values run over the unknowns (rows, columns >= 1).
"""
from __future__ import annotations

import numpy as np


def medium_v(n2: np.ndarray, n0: float, W: int) -> np.ndarray:
    """V = (n^2 - n0^2) / n0^2 where the distance to the edge exceeds W, else 0."""
    ny, nx = n2.shape
    i, j = np.arange(ny), np.arange(nx)
    d = np.minimum(np.minimum(i, ny - i)[:, None], np.minimum(j, nx - j)[None, :])
    return np.where(d > W, (n2 - n0 ** 2) / n0 ** 2, 0.0)


def _rms(a: np.ndarray) -> float:
    """rms over the unknowns of a (..., ny, nx) array (all leading entries pooled)."""
    inner = a[..., 1:, 1:]
    return float(np.sqrt(np.mean(np.abs(inner) ** 2)))


def stats(w, ys, n2, n0, W):
    """[rms w, rms V, rms y_0, rms y_1, ...], each at least 1e-300."""
    vals = [_rms(w), _rms(medium_v(n2, n0, W))] + [_rms(y) for y in ys]
    return np.maximum(np.array(vals), 1e-300)


def pack(w, ys, n2, scal, feats, n0, W):
    """(B, 4 ncomp + 3, ny, nx): per component Re, Im of w / rms w; per component Re, Im of
    y_b / rms y_b; V / rms V; the pole features feats[b] as constant planes; row 0 and
    column 0 zero."""
    ncomp, ny, nx = w.shape
    V = medium_v(n2, n0, W)
    out = np.zeros((len(ys), 4 * ncomp + 3, ny, nx))
    for b, y in enumerate(ys):
        planes = []
        for c in range(ncomp):
            planes += [w[c].real / scal[0], w[c].imag / scal[0]]
        for c in range(ncomp):
            planes += [y[c].real / scal[2 + b], y[c].imag / scal[2 + b]]
        planes += [V / scal[1], np.full((ny, nx), feats[b][0]), np.full((ny, nx), feats[b][1])]
        out[b] = np.stack(planes)
    out[:, :, 0, :] = 0.0
    out[:, :, :, 0] = 0.0
    return out


def unpack(w, net_out, scal):
    """t_b = w + sigma_b (net_out[b, 2c] + i net_out[b, 2c+1]) per component; borders zero."""
    B = net_out.shape[0]
    ncomp = w.shape[0]
    t = np.zeros((B,) + w.shape, dtype=complex)
    for b in range(B):
        sg = scal[2 + b] * scal[1]
        for c in range(ncomp):
            t[b, c] = w[c] + sg * (net_out[b, 2 * c] + 1j * net_out[b, 2 * c + 1])
    t[:, :, 0, :] = 0.0
    t[:, :, :, 0] = 0.0
    return t


def target(px, scal):
    """(B, 2 ncomp, ny, nx) = -(P x_b) / sigma_b as Re, Im planes per component."""
    B, ncomp = px.shape[:2]
    out = np.zeros((B, 2 * ncomp) + px.shape[2:])
    for b in range(B):
        v = -px[b] / (scal[2 + b] * scal[1])
        out[b, 0::2] = v.real
        out[b, 1::2] = v.imag
    return out
