"""Rational approximation of exp(iK sqrt(1+z)) and its partial fractions (oracle).

Test infrastructure only.

Sec. 2 (eq. rational approximation) replaces exp(iK sqrt(I + Zbar)) by an
(N,N) rational function of Zbar and (eq. pf_expan_eq) splits it into
    r(z) = alpha_NN/beta_NN + sum_k a_k / (z - b_k).
Sec. 3.1 builds that rational function with AAA-Lawson on Re z in [-4, 2]:
AAA (greedy support-point selection, barycentric weights from the smallest
singular vector of a Loewner matrix) followed by Lawson iteratively reweighted
least squares on the barycentric numerator/denominator weights toward minimax.

Target function, principal branch: for z >= -1, exp(iK sqrt(1+z)) (a phase);
for z < -1, sqrt(1+z) = i sqrt(-1-z) so f = exp(-K sqrt(-1-z)) (evanescent
decay).  Both are evaluated in real form, never through a complex sqrt of a
value carrying a signed zero.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def target(z: np.ndarray, K: float) -> np.ndarray:
    """f(z) = exp(iK sqrt(1+z)) on the real axis, principal branch."""
    z = np.asarray(z, dtype=float)
    out = np.empty(z.shape, dtype=complex)
    prop = z >= -1.0
    out[prop] = np.exp(1j * K * np.sqrt(1.0 + z[prop]))
    out[~prop] = np.exp(-K * np.sqrt(-1.0 - z[~prop]))
    return out


def target_complex(z: np.ndarray, K: float) -> np.ndarray:
    """f(z) = exp(iK sqrt(1+z)) for complex z, principal branch of sqrt."""
    return np.exp(1j * K * np.sqrt(np.asarray(z, dtype=complex) + 1.0))


def _cauchy(Z: np.ndarray, zj: np.ndarray) -> np.ndarray:
    return 1.0 / (Z[:, None] - zj[None, :])


def aaa(Z: np.ndarray, F: np.ndarray, mmax: int):
    """Plain AAA: returns support points zj, values fj, weights wj (mmax of each).

    Each pass adds the sample with the largest current error to the support
    set, then takes the weights as the right singular vector of the smallest
    singular value of the Loewner matrix  L_ij = (F_i - f_j)/(Z_i - z_j)
    over the non-support samples.
    """
    Z = np.asarray(Z, dtype=complex)
    F = np.asarray(F, dtype=complex)
    M = len(Z)
    support: list[int] = []
    R = np.full(M, F.mean())
    w = None
    for _ in range(mmax):
        err = np.abs(F - R)
        err[support] = -1.0
        support.append(int(np.argmax(err)))
        rest = np.setdiff1d(np.arange(M), support)
        zj, fj = Z[support], F[support]
        C = _cauchy(Z[rest], zj)
        L = F[rest, None] * C - C * fj[None, :]
        _, _, vh = np.linalg.svd(L, full_matrices=False)
        w = vh[-1].conj()
        R = F.copy()
        R[rest] = (C @ (w * fj)) / (C @ w)
    zj = Z[support]
    return zj, F[support], w


def lawson(Z: np.ndarray, F: np.ndarray, zj: np.ndarray, alpha: np.ndarray, beta: np.ndarray,
           iters: int = 40):
    """Lawson IRLS on separate numerator/denominator barycentric weights.

    With the support points fixed, minimise sum_i lam_i |F_i d(Z_i) - n(Z_i)|^2
    with n(z) = sum alpha_j/(z - z_j), d(z) = sum beta_j/(z - z_j) and
    ||(alpha, beta)|| = 1 (smallest singular vector), then set
    lam_i <- lam_i |F_i - r(Z_i)| and renormalise.  The iterate with the
    smallest maximum error is returned.

    Once alpha != f_j beta, r no longer interpolates at a support point z_j,
    where r(z_j) = alpha_j/beta_j.  Each support point therefore keeps a row of
    its own, (f_j beta_j - alpha_j)/h with h the sample spacing near z_j: the
    residue of F d - n at z_j, scaled like the rows of the neighbouring samples.
    """
    Z = np.asarray(Z, dtype=complex)
    F = np.asarray(F, dtype=complex)
    keep = np.ones(len(Z), dtype=bool)
    for z in zj:
        keep &= np.abs(Z - z) > 0
    Zs, Fs = Z[keep], F[keep]
    if (~keep).sum() != len(zj):
        raise ValueError("support points must be distinct samples")
    fj = np.array([F[np.argmin(np.abs(Z - z))] for z in zj])
    spacing = np.array([np.sort(np.abs(Z - z))[1] for z in zj])
    m = len(zj)
    C = np.vstack([_cauchy(Zs, zj), np.diag(1.0 / spacing)])
    Fa = np.concatenate([Fs, fj])

    def errors(a, b):
        return np.abs(Fa - (C @ a) / (C @ b))

    e0 = errors(alpha, beta)
    best = (e0.max(), alpha, beta)
    lam = np.full(len(Fa), 1.0 / len(Fa))
    for _ in range(iters):
        s = np.sqrt(lam)[:, None]
        A = np.hstack([-s * C, s * (Fa[:, None] * C)])
        if not np.all(np.isfinite(A)):
            break
        _, _, vh = np.linalg.svd(A, full_matrices=False)
        v = vh[-1].conj()
        a, b = v[:m], v[m:]
        e = errors(a, b)
        if not np.all(np.isfinite(e)):
            break
        if e.max() < best[0]:
            best = (e.max(), a, b)
        lam = lam * np.maximum(e, 1e-300)
        lam = lam / lam.sum()
    return best[1], best[2]


def poles_residues(zj: np.ndarray, alpha: np.ndarray, beta: np.ndarray):
    """Poles b_k, residues a_k and r_inf of r = n/d (barycentric, weights alpha/beta).

    Poles: finite eigenvalues of the arrowhead pencil
        E = [[0, beta^T], [1, diag(zj)]],  B = diag(0, 1, ..., 1).
    Residues at simple poles: a_k = n(b_k) / d'(b_k), d'(z) = -sum beta_j/(z-z_j)^2.
    Value at infinity: r_inf = sum alpha / sum beta.
    """
    m = len(zj)
    E = np.zeros((m + 1, m + 1), dtype=complex)
    E[0, 1:] = beta
    E[1:, 0] = 1.0
    E[1:, 1:] = np.diag(zj)
    B = np.eye(m + 1, dtype=complex)
    B[0, 0] = 0.0
    ev = sla.eig(E, B, right=False)
    poles = ev[np.isfinite(ev)]
    poles = poles[np.abs(poles) < 1e12]
    Cp = _cauchy(poles, zj)
    n_at = Cp @ alpha
    dprime = -(Cp ** 2) @ beta
    residues = n_at / dprime
    r_inf = alpha.sum() / beta.sum()
    order = np.argsort(poles.real)
    return poles[order], residues[order], complex(r_inf)


def eval_barycentric(z, zj, alpha, beta):
    z = np.asarray(z, dtype=complex)
    C = _cauchy(z.ravel(), zj)
    return ((C @ alpha) / (C @ beta)).reshape(z.shape)


def eval_pf(z, poles, residues, r_inf):
    """r(z) = r_inf + sum_k a_k/(z - b_k)."""
    z = np.asarray(z, dtype=complex)
    return r_inf + (1.0 / (z.ravel()[:, None] - poles[None, :])) @ residues


def fit_exp_sqrt(K: float, N: int, zlo: float = -4.0, zhi: float = 2.0, nsamp: int = 4001,
                 lawson_iters: int = 40) -> dict:
    """(N,N) AAA-Lawson fit of exp(iK sqrt(1+z)) on uniform samples of [zlo, zhi].

    The default interval is the paper's Re z in [-4, 2] (Sec. 3).  The "average
    error" the paper quotes in Sec. 3.1 is read as the mean of |r - f| over the
    uniform samples; the report also gives the maximum on a 10^5-point grid,
    which sees the slow convergence at the branch point z = -1.

    Returns a dict with poles, residues, r_inf and a fit report (mean and max
    error on the samples, max error on a fine grid, min Im(-b_k)).
    """
    Z = np.linspace(zlo, zhi, nsamp)
    F = target(Z, K)
    zj, fj, w = aaa(Z.astype(complex), F, N + 1)
    alpha, beta = w * fj, w
    if lawson_iters:
        alpha, beta = lawson(Z, F, zj, alpha, beta, lawson_iters)
    poles, residues, r_inf = poles_residues(zj, alpha, beta)
    rs = eval_pf(Z, poles, residues, r_inf)
    zf = np.linspace(zlo, zhi, 100001)
    rf = eval_pf(zf, poles, residues, r_inf)
    return {
        "K": K, "N": N, "zlo": zlo, "zhi": zhi,
        "poles": poles, "residues": residues, "r_inf": r_inf,
        "support": zj, "alpha": alpha, "beta": beta,
        "mean_err": float(np.mean(np.abs(rs - F))),
        "max_err": float(np.max(np.abs(rs - F))),
        "fine_max_err": float(np.max(np.abs(rf - target(zf, K)))),
        "min_im_neg_pole": float(np.min(-poles.imag)),
    }
