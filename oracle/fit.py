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
           iters: int = 40, score=None):
    """Lawson IRLS on separate numerator/denominator barycentric weights.

    With the support points fixed, minimise sum_i lam_i |F_i d(Z_i) - n(Z_i)|^2
    with n(z) = sum alpha_j/(z - z_j), d(z) = sum beta_j/(z - z_j) and
    ||(alpha, beta)|| = 1 (smallest singular vector), then set
    lam_i <- lam_i |F_i - r(Z_i)| and renormalise.  The iterate with the
    smallest score is returned; score(alpha, beta) defaults to the maximum
    barycentric error over the rows, and a non-finite score counts as +inf
    (so a NaN never blocks the comparison).

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
        with np.errstate(divide="ignore", invalid="ignore"):
            return np.abs(Fa - (C @ a) / (C @ b))

    def worst(e):
        # a row where d vanishes (r has a pole on a sample) counts as an infinite error
        return np.inf if not np.all(np.isfinite(e)) else float(e.max())

    def scored(a, b, e):
        v = worst(e) if score is None else float(score(a, b))
        return v if np.isfinite(v) else np.inf

    best = (scored(alpha, beta, errors(alpha, beta)), alpha, beta)
    lam = np.full(len(Fa), 1.0 / len(Fa))
    for _ in range(iters):
        s = np.sqrt(lam)[:, None]
        A = np.hstack([-s * C, s * (Fa[:, None] * C)])
        _, _, vh = np.linalg.svd(A, full_matrices=False)
        v = vh[-1].conj()
        a, b = v[:m], v[m:]
        e = errors(a, b)
        sc = scored(a, b, e)
        if sc < best[0]:
            best = (sc, a, b)
        # such an iterate is not kept, but the iteration goes on: its rows with no finite
        # error are reweighted as the worst finite row (the iteration pushes them down next)
        fin = np.isfinite(e)
        if not fin.any():
            break
        e = np.where(fin, e, e[fin].max())
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


def samples(zlo: float, zhi: float, nsamp: int, grade: int = 0) -> np.ndarray:
    """nsamp uniform samples of [zlo, zhi]; with grade > 0 also -1 -+ 10^t for grade values of t
    evenly spaced in [-10, 0] on each side of the branch point (those inside the interval)."""
    Z = np.linspace(zlo, zhi, nsamp)
    if grade > 0:
        t = 10.0 ** np.linspace(-10.0, 0.0, grade)
        Z = np.unique(np.concatenate([Z, -1.0 - t, -1.0 + t]))
        Z = Z[(Z >= zlo) & (Z <= zhi)]
    return Z


def fit_exp_sqrt(K: float, N: int, zlo: float = -4.0, zhi: float = 2.0, nsamp: int = 4001,
                 lawson_iters: int = 40, grade: int = 0) -> dict:
    """(N,N) AAA-Lawson fit of exp(iK sqrt(1+z)) on uniform samples of [zlo, zhi]
    (plus, with grade > 0, samples graded toward the branch point z = -1, see samples()).

    Of the Lawson iterates (AAA's own weights included) the one whose partial
    fractions have the smallest maximum error on the samples is kept.

    The default interval is the paper's Re z in [-4, 2] (Sec. 3).  The "average
    error" the paper quotes in Sec. 3.1 is read as the mean of |r - f| over the
    uniform samples; the report also gives the maximum on a 10^5-point grid,
    which sees the slow convergence at the branch point z = -1.

    Returns a dict with poles, residues, r_inf and a fit report: mean and max
    error on the uniform samples, max error and max |r| on a fine grid that
    also approaches z = -1 to 1e-14, min Im(-b_k).
    """
    Z = samples(zlo, zhi, nsamp, grade)
    F = target(Z, K)
    zj, fj, w = aaa(Z.astype(complex), F, N + 1)
    alpha, beta = w * fj, w

    def pf_max_err(a, b):
        # what a plan consumes is the partial-fraction form: judge each iterate by it
        with np.errstate(all="ignore"):
            p, r, ri = poles_residues(zj, a, b)
            return np.max(np.abs(eval_pf(Z, p, r, ri) - F)) if len(p) == N else np.inf

    if lawson_iters:
        alpha, beta = lawson(Z, F, zj, alpha, beta, lawson_iters, score=pf_max_err)
    poles, residues, r_inf = poles_residues(zj, alpha, beta)
    Zu = np.linspace(zlo, zhi, nsamp)
    eu = np.abs(eval_pf(Zu, poles, residues, r_inf) - target(Zu, K))
    # fine grid: 10^5 uniform points and points approaching the branch point from both sides
    near = 10.0 ** np.linspace(-14.0, 0.0, 2001)
    zf = np.unique(np.concatenate([np.linspace(zlo, zhi, 100001), -1.0 - near, -1.0 + near]))
    zf = zf[(zf >= zlo) & (zf <= zhi)]
    rf = eval_pf(zf, poles, residues, r_inf)
    return {
        "K": K, "N": N, "zlo": zlo, "zhi": zhi,
        "poles": poles, "residues": residues, "r_inf": r_inf,
        "support": zj, "alpha": alpha, "beta": beta,
        "mean_err": float(np.mean(eu)),
        "max_err": float(np.max(eu)),
        "fine_max_err": float(np.max(np.abs(rf - target(zf, K)))),
        "fine_max_abs_r": float(np.max(np.abs(rf))),
        "min_im_neg_pole": float(np.min(-poles.imag)),
    }
