"""Plan tables a caller of libhp needs (host-side set-up, not on the per-step path).

* 13-point stencils (Sec. 4.1): fourth-order second and first derivatives whose
  free coefficients minimise the worst relative error of the Fourier symbol
  over a design band (83 % of [0, pi] for the second derivative, 70 % for the
  first), as a linear programme.
* The (N,N) AAA-Lawson rational fit of exp(iK sqrt(1+z)) on Re z in [-4, 2]
  (Sec. 3.1) and its partial fractions r_inf + sum a_k/(z - b_k)
  (Sec. 2, eq. pf_expan_eq): the poles/residues hp_plan_create takes.
* The Cauchy-integral partial fractions of sqrt(1+z) (Sec. 3.2, eq.
  pf_sqrt_exp, Appendix A) for the pseudo-differential form (HP_FORM_SQRT).
* A lookup table of AAA-Lawson partial fractions for one reference index n0
  and a list of k0 dz values (Sec. 3.1: the coefficients depend on K = k0 n0 dz
  only, so a table over k0 dz at fixed n0 replaces the fit at plan set-up).
"""
from __future__ import annotations

import json

import numpy as np
import scipy.linalg as sla
from scipy.optimize import linprog


def _minimax_lp(rows: np.ndarray, eq: np.ndarray, rhs: np.ndarray) -> np.ndarray:
    """min t  s.t. |rows @ x - 1| <= t, eq @ x = rhs."""
    ns, nv = rows.shape
    ones = np.ones((ns, 1))
    A_ub = np.block([[rows, -ones], [-rows, -ones]])
    b_ub = np.concatenate([np.ones(ns), -np.ones(ns)])
    A_eq = np.hstack([eq, np.zeros((eq.shape[0], 1))])
    c = np.zeros(nv + 1)
    c[-1] = 1.0
    sol = linprog(c, A_ub=A_ub, b_ub=b_ub, A_eq=A_eq, b_eq=rhs, bounds=(None, None), method="highs")
    if sol.status != 0:
        raise RuntimeError("stencil design LP failed: " + sol.message)
    return sol.x[:nv]


def stencil_d2(band_frac: float = 0.83, hw: int = 6, samples: int = 3000) -> np.ndarray:
    """c0..c_hw; symbol 4 sum_m c_m sin^2(m theta / 2) (c0 = -2 sum c_m) ~ theta^2."""
    th = np.pi * band_frac * np.arange(1, samples + 1) / samples
    m = np.arange(1, hw + 1)
    rows = 4.0 * np.sin(np.outer(th, m) / 2.0) ** 2 / th[:, None] ** 2
    eq = np.vstack([m ** 2, m ** 4]).astype(float)
    cm = _minimax_lp(rows, eq, np.array([1.0, 0.0]))
    return np.concatenate([[-2.0 * cm.sum()], cm])


def stencil_d1(band_frac: float = 0.70, hw: int = 6, samples: int = 3000) -> np.ndarray:
    """d1..d_hw; symbol 2 sum_m d_m sin(m theta) ~ theta."""
    th = np.pi * band_frac * np.arange(1, samples + 1) / samples
    m = np.arange(1, hw + 1)
    rows = 2.0 * np.sin(np.outer(th, m)) / th[:, None]
    eq = np.vstack([2.0 * m, m ** 3]).astype(float)
    return _minimax_lp(rows, eq, np.array([1.0, 0.0]))


def exp_sqrt(z: np.ndarray, K: float) -> np.ndarray:
    """exp(iK sqrt(1+z)) for real z, principal branch (decay below z = -1)."""
    z = np.asarray(z, dtype=float)
    s = 1.0 + z
    return np.where(s >= 0, np.exp(1j * K * np.sqrt(np.abs(s))), np.exp(-K * np.sqrt(np.abs(s))))


class RationalFit:
    """AAA followed by Lawson reweighting; barycentric numerator/denominator weights a, b."""

    def __init__(self, K: float, degree: int, lo: float = -4.0, hi: float = 2.0, samples: int = 4001,
                 lawson_steps: int = 40, grade: int = 0):
        """grade > 0 adds 2 grade samples at -1 -+ 10^s, s = -10..0 (evenly spaced), to the
        uniform ones: the fit then sees the branch point z = -1 closely (smaller error and
        overshoot |r| > 1 there) at the price of poles closer to the real axis."""
        self.K, self.degree = K, degree
        Z = np.linspace(lo, hi, samples)
        if grade > 0:
            off = np.logspace(-10.0, 0.0, grade)
            Z = np.union1d(Z, np.concatenate([-1.0 - off, -1.0 + off]))
            Z = Z[(Z >= lo) & (Z <= hi)]
        self.Z = Z
        self.F = exp_sqrt(self.Z, K)
        self._aaa(degree + 1)
        if lawson_steps:
            self._lawson(lawson_steps)
        self._partial_fractions()

    def _aaa(self, nsupport: int):
        Z, F = self.Z.astype(complex), self.F
        chosen = np.zeros(len(Z), dtype=bool)
        approx = np.full(len(Z), np.mean(F))
        for _ in range(nsupport):
            err = np.where(chosen, -np.inf, np.abs(F - approx))
            chosen[int(np.argmax(err))] = True
            t, ft = Z[chosen], F[chosen]
            others = ~chosen
            cauchy = 1.0 / np.subtract.outer(Z[others], t)
            loewner = cauchy * np.subtract.outer(F[others], ft)
            w = sla.svd(loewner, full_matrices=False)[2][-1].conj()
            approx = F.copy()
            approx[others] = (cauchy @ (w * ft)) / (cauchy @ w)
        self.t = Z[chosen]
        self.ft = F[chosen]
        self.a = w * self.ft
        self.b = w

    def _rows(self):
        Z, F = self.Z.astype(complex), self.F
        off = np.ones(len(Z), dtype=bool)
        idx = [int(np.argmin(np.abs(Z - t))) for t in self.t]
        off[idx] = False
        # local sample spacing at each support point (the samples may be graded)
        h = np.array([np.partition(np.abs(self.Z - t.real), 1)[1] for t in self.t])
        # sample rows: Cauchy matrix; support rows: the residue of F d - n at t_j, over h_j
        C = np.vstack([1.0 / np.subtract.outer(Z[off], self.t), np.diag(1.0 / h)])
        return C, np.concatenate([F[off], F[idx]])

    def _lawson(self, steps: int):
        C, F = self._rows()
        n = len(self.t)

        def err(a, b):
            with np.errstate(divide="ignore", invalid="ignore"):
                e = np.abs(F - (C @ a) / (C @ b))
            # NaN (0/0) and inf (d = 0 on a sample row) both mean "no finite value there"
            return np.where(np.isnan(e), np.inf, e)

        Zs = self.Z.astype(complex)

        def pf_err(a, b):
            # the iterate is judged by the form the plan receives: its partial fractions
            with np.errstate(all="ignore"):
                poles, res, rinf = self._pf_of(a, b)
                if len(poles) != self.degree:
                    return np.inf
                v = np.max(np.abs(rinf + (1.0 / np.subtract.outer(Zs, poles)) @ res - self.F))
            return v if np.isfinite(v) else np.inf

        best_err, best = pf_err(self.a, self.b), (self.a, self.b)
        wts = np.full(len(F), 1.0 / len(F))
        for _ in range(steps):
            sq = np.sqrt(wts)[:, None]
            M = np.hstack([sq * (F[:, None] * C), -sq * C])      # unknowns (b, a)
            v = sla.svd(M, full_matrices=False)[2][-1].conj()
            b, a = v[:n], v[n:]
            e = err(a, b)
            score = pf_err(a, b)
            if score < best_err:
                best_err, best = score, (a, b)
            finite = e < np.inf
            if not finite.any():
                break
            # an unbounded row takes the largest finite error as its weight factor
            wts = wts * np.maximum(np.minimum(e, e[finite].max()), 1e-300)
            wts /= wts.sum()
        self.a, self.b = best

    def _pf_of(self, a, b):
        """Poles, residues and value at infinity of the barycentric form with weights a, b."""
        n = len(self.t)
        E = np.zeros((n + 1, n + 1), dtype=complex)
        E[0, 1:] = b
        E[1:, 0] = 1.0
        E[1:, 1:] = np.diag(self.t)
        B = np.diag(np.concatenate([[0.0], np.ones(n)])).astype(complex)
        ev = sla.eigvals(E, B)
        poles = ev[np.isfinite(ev) & (np.abs(ev) < 1e12)]
        d = 1.0 / np.subtract.outer(poles, self.t)
        return poles, (d @ a) / (-(d ** 2) @ b), complex(a.sum() / b.sum())

    def _partial_fractions(self):
        self.poles, self.residues, self.r_inf = self._pf_of(self.a, self.b)

    def __call__(self, z):
        z = np.asarray(z, dtype=complex)
        return self.r_inf + (1.0 / np.subtract.outer(z.ravel(), self.poles)) @ self.residues


def plan_tables(K: float, npoles: int):
    """(poles, residues, r_inf, d2, d1) for hp_plan_create."""
    f = RationalFit(K, npoles)
    return f.poles, f.residues, f.r_inf, stencil_d2(), stencil_d1()


def pml_stretched_d2(N: int, h: float, k0: float, n0: float, W: int, sigma_max: float, d2=None, d1=None):
    """s D~: the one-axis stretched second derivative of the absorbing layers (Sec. 4.1) on the
    unknowns 1..N-1, as a dense (N-1, N-1) complex matrix, s = 1/(k0 n0)^2.

    The stretch is g = 1 + i sigma with sigma = sigma_max ((W + 1 - d)/W)^2 at distance d in
    [1, W] cells from the nearer Dirichlet node (0 beyond), and d^2/dx~^2 = (1/g^2) D2 - (g'/g^3) D1
    with the 13-point stencils (odd reflection about the Dirichlet nodes 0 and N)."""
    c = np.asarray(stencil_d2() if d2 is None else d2, float)
    dd = np.asarray(stencil_d1() if d1 is None else d1, float)
    n = N - 1
    nodes = np.arange(1, N)
    C2 = np.zeros((n, n))
    C1 = np.zeros((n, n))
    for m in range(-6, 7):
        tgt = nodes + m
        sign = np.where((tgt < 0) | (tgt > N), -1.0, 1.0)
        tgt = np.where(tgt < 0, -tgt, np.where(tgt > N, 2 * N - tgt, tgt))
        keep = (tgt >= 1) & (tgt <= N - 1)
        rows, cols = nodes[keep] - 1, tgt[keep] - 1
        np.add.at(C2, (rows, cols), sign[keep] * c[abs(m)])
        if m:
            np.add.at(C1, (rows, cols), sign[keep] * np.sign(m) * dd[abs(m) - 1])
    dist = np.minimum(nodes, N - nodes)
    t = np.where(dist <= W, (W + 1.0 - dist) / W, 0.0)
    g = 1.0 + 1j * sigma_max * t ** 2
    dsig = -2.0 * sigma_max * t / W / h            # d sigma/d(distance) per unit length
    gp = 1j * np.where(nodes <= N - nodes, dsig, -dsig)
    s = 1.0 / (k0 * n0) ** 2
    return s * ((1.0 / g ** 2)[:, None] * (C2 / h ** 2) - (gp / g ** 3)[:, None] * (C1 / h))


def pml_eigen(N: int, h: float, k0: float, n0: float, W: int, sigma_max: float, d2=None, d1=None):
    """(Q, Qinv, lam) with s D~ = Q diag(lam) Qinv (pml_stretched_d2), the tables hp_set_pml takes."""
    A = pml_stretched_d2(N, h, k0, n0, W, sigma_max, d2, d1)
    lam, Q = np.linalg.eig(A)
    return Q, np.linalg.inv(Q), lam


def cauchy_sqrt_table(N: int, alpha: float = 1.0):
    """(poles, residues, r_inf) of sqrt(1+z) ~ r_inf + sum_j a_j/(z - b_j) from the Cauchy
    integral over the cut w in [-1, 1] of the Moebius variable w = (z+1+i alpha)/(z+1-i alpha),
    discretised by the N-point Gauss rule of the weight sqrt((1+eta)/(1-eta)).  That weight is
    the Chebyshev weight of the third kind, whose Gauss rule is explicit: eta_j = cos(theta_j),
    theta_j = (2j-1) pi/(2N+1), omega_j = 4 pi cos^2(theta_j/2)/(2N+1).  With
    wt_j = (c_alpha/pi) omega_j/(1 - eta_j), sigma_j = (1+eta_j)/(1-eta_j), c_alpha = sqrt(alpha) e^{i pi/4}:
    b_j = -(1 + i alpha sigma_j), a_j = -i alpha wt_j (1 + sigma_j), r_inf = c_alpha + sum_j wt_j."""
    if N < 1 or not alpha > 0:
        raise ValueError("N >= 1 and alpha > 0 required")
    th = (2.0 * np.arange(1, N + 1) - 1.0) * np.pi / (2 * N + 1)
    half = th / 2.0
    # 1 - eta = 2 sin^2(theta/2), 1 + eta = 2 cos^2(theta/2): no cancellation near eta = +-1
    one_m, one_p = 2.0 * np.sin(half) ** 2, 2.0 * np.cos(half) ** 2
    omega = 2.0 * np.pi / (2 * N + 1) * one_p
    c_alpha = np.sqrt(alpha) * np.exp(0.25j * np.pi)
    wt = c_alpha / np.pi * omega / one_m
    sigma = one_p / one_m
    return -(1.0 + 1j * alpha * sigma), -1j * alpha * wt * (1.0 + sigma), complex(c_alpha + wt.sum())


class PFLookup:
    """AAA-Lawson partial fractions of exp(iK sqrt(1+z)) on [-4, 2] for a fixed reference index n0
    and a list of k0 dz values, K = k0 n0 dz.  Entries are whole fits: poles and residues of fits
    at neighbouring K do not interpolate (1 % apart in K, averaging them costs three orders of
    magnitude in accuracy), so a lookup must hit a tabulated k0 dz."""

    def __init__(self, n0: float, npoles: int, entries: list):
        self.n0, self.npoles, self.entries = float(n0), int(npoles), entries

    @classmethod
    def build(cls, k0dz_values, npoles: int, n0: float = 1.0003):
        entries = []
        for k0dz in k0dz_values:
            K = float(k0dz) * n0
            f = RationalFit(K, npoles)
            err = float(np.abs(f(f.Z) - exp_sqrt(f.Z, K)).max())            # on the fit's samples
            zf = np.linspace(-4.0, 2.0, 100001)
            fine = float(np.abs(f(zf) - exp_sqrt(zf, K)).max())           # between them (branch point)
            entries.append(dict(k0dz=float(k0dz), K=K, poles=f.poles, residues=f.residues, r_inf=f.r_inf,
                                max_err=err, fine_max_err=fine))
        return cls(n0, npoles, entries)

    def save(self, path: str):
        def c(a):
            a = np.asarray(a, dtype=complex)
            return [[float(v.real), float(v.imag)] for v in np.atleast_1d(a)]
        doc = dict(n0=self.n0, npoles=self.npoles, target="exp(iK sqrt(1+z)), K = k0 n0 dz, z in [-4, 2]; max_err on the 4001 fit samples, "
                          "fine_max_err on 100001 points",
                   entries=[dict(k0dz=e["k0dz"], K=e["K"], max_err=e["max_err"],
                                 fine_max_err=e["fine_max_err"], poles=c(e["poles"]),
                                 residues=c(e["residues"]), r_inf=c(e["r_inf"])[0]) for e in self.entries])
        with open(path, "w") as fh:
            json.dump(doc, fh, indent=1)

    @classmethod
    def load(cls, path: str):
        with open(path) as fh:
            doc = json.load(fh)
        def c(a):
            a = np.asarray(a, dtype=float)
            return a[..., 0] + 1j * a[..., 1]
        entries = [dict(k0dz=e["k0dz"], K=e["K"], max_err=e["max_err"], fine_max_err=e["fine_max_err"],
                        poles=c(e["poles"]),
                        residues=c(e["residues"]), r_inf=complex(c(e["r_inf"]))) for e in doc["entries"]]
        return cls(doc["n0"], doc["npoles"], entries)

    def get(self, k0: float, dz: float, n0: float, rtol: float = 1e-9):
        """(poles, residues, r_inf) of the entry for k0 dz; KeyError when n0 differs from the
        table's or k0 dz is not tabulated (to rtol)."""
        if abs(n0 - self.n0) > rtol * self.n0:
            raise KeyError(f"table is for n0 = {self.n0}, not {n0}")
        want = k0 * dz
        for e in self.entries:
            if abs(e["k0dz"] - want) <= rtol * abs(want):
                return e["poles"], e["residues"], e["r_inf"]
        raise KeyError(f"k0 dz = {want} is not in the table ({[e['k0dz'] for e in self.entries]})")


if __name__ == "__main__":
    # python -m paper_2410_17446_amd.tables OUT.json N0 NPOLES DZ... (dz in wavelengths; k0 = 2 pi)
    import sys
    out, n0, npoles = sys.argv[1], float(sys.argv[2]), int(sys.argv[3])
    dzs = [float(v) for v in sys.argv[4:]]
    PFLookup.build([2.0 * np.pi * v for v in dzs], npoles, n0=n0).save(out)
    print(f"wrote {out}: n0 = {n0}, {npoles} poles, dz = {dzs} wavelengths")
