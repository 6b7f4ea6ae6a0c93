"""The library's host-side plan tables (paper_2410_17446_amd.tables) against the oracle.

The two sides are written independently (the library's Gauss rule is the explicit
Chebyshev third-kind rule, the oracle's a general Gauss-Jacobi routine; the fits share
only their definition), so agreement checks both."""
import numpy as np
import pytest

from oracle import fit, stencil
from oracle import sqrt_form as sf
from paper_2410_17446_amd import tables


def _match(b1, a1, b2, a2):
    i, j = np.argsort(b1.imag), np.argsort(b2.imag)
    return np.abs(b1[i] / b2[j] - 1).max(), np.abs(a1[i] / a2[j] - 1).max()


@pytest.mark.parametrize("N,alpha", [(1, 1.0), (25, 1.0), (45, 0.1), (60, 1.0)])
def test_cauchy_table_matches_oracle(N, alpha):
    b, a, r = tables.cauchy_sqrt_table(N, alpha)
    o = sf.cauchy_sqrt_pf(N, alpha)
    eb, ea = _match(b, a, o.poles, o.residues)
    assert eb < 1e-12 and ea < 1e-10 and abs(r / o.r_inf - 1) < 1e-10
    assert np.all(b.imag < 0)  # the cut's images lie below the real axis


def test_cauchy_table_rejects_bad_arguments():
    with pytest.raises(ValueError):
        tables.cauchy_sqrt_table(0)
    with pytest.raises(ValueError):
        tables.cauchy_sqrt_table(5, 0.0)


@pytest.mark.parametrize("N", [8, 16])
def test_rational_fit_accuracy_matches_oracle(N):
    """Both AAA-Lawson fits of exp(iK sqrt(1+z)), K = 2 pi, reach the same accuracy on the
    uniform samples of [-4, 2] (the fits need not coincide term by term)."""
    K = 2 * np.pi
    lib = tables.RationalFit(K, N)
    ora = fit.fit_exp_sqrt(K, N)
    z = np.linspace(-4, 2, 4001)
    e_lib = np.abs(lib(z) - fit.target(z, K)).max()
    assert e_lib < 3 * ora["max_err"]
    assert len(lib.poles) == N and np.all(lib.poles.imag < 0)


def test_rational_fit_at_the_beam_step_matches_oracle():
    """The 25-term fit at dz = lambda/20, n0 = 1.0003 (the beam runs of Sec. 5.2): both fits sit
    near 1e-11..1e-10 on the samples, where the conversion from barycentric weights to poles and
    residues (residues of size ~30, so cancellation) decides the last digit, and the library's
    Lawson stage never ends worse than its own AAA start (a non-finite Lawson iterate no longer
    stops the iteration at the AAA weights)."""
    K = 2 * np.pi * 1.0003 * 0.05
    z = np.linspace(-4, 2, 4001)
    lib = tables.RationalFit(K, 25)
    start = tables.RationalFit(K, 25, lawson_steps=0)
    ora = fit.fit_exp_sqrt(K, 25)
    e_lib = np.abs(lib(z) - fit.target(z, K)).max()
    e_start = np.abs(start(z) - fit.target(z, K)).max()
    assert e_lib <= e_start
    assert e_lib < 3e-10 and ora["max_err"] < 3e-10
    assert e_lib < 15 * ora["max_err"]
    assert len(lib.poles) == 25 and np.all(lib.poles.imag < 0)


def test_graded_rational_fit_matches_oracle():
    """With samples graded toward z = -1 both fits reach the same branch-point accuracy."""
    K = 2 * np.pi
    lib = tables.RationalFit(K, 16, grade=300)
    ora = fit.fit_exp_sqrt(K, 16, grade=300)
    near = 10.0 ** np.linspace(-14, 0, 2001)
    z = np.concatenate([np.linspace(-4, 2, 100001), -1 - near, -1 + near])
    e_lib = np.abs(lib(z) - fit.target(z, K)).max()
    assert e_lib < 3 * ora["fine_max_err"] and ora["fine_max_err"] < 1e-3


def test_stencils_match_oracle_symbols():
    """Both stencil designs solve the same minimax problem: their symbols agree."""
    c_o, d_o = stencil.stencils()
    c_l, d_l = tables.stencil_d2(), tables.stencil_d1()
    th = np.linspace(0.01, 0.83 * np.pi, 500)
    s_o, s_l = stencil.d2_symbol(c_o, th), stencil.d2_symbol(c_l, th)
    assert np.abs(s_l / s_o - 1).max() < 1e-3
    th = np.linspace(0.01, 0.70 * np.pi, 500)
    s_o, s_l = stencil.d1_symbol(d_o, th), stencil.d1_symbol(d_l, th)
    assert np.abs(s_l / s_o - 1).max() < 1e-3


# ---------------------------------------------------------------- lookup table over k0 dz (Sec. 3.1)

import glob
import os

DATA = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2410_17446_amd", "data")


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(DATA, "pf_lookup_*.json"))))
def test_shipped_lookup_tables_meet_their_errors(path):
    """Every entry of a shipped table approximates the oracle's exp(iK sqrt(1+z)), K = k0 dz n0,
    within its recorded errors: on the fit's 4001 uniform samples (below 2e-5 for the 16-term
    tables up to dz = 2 lambda) and on a 100001-point grid, which sees the slow convergence at
    the branch point z = -1 between the samples.  All poles lie below the real axis."""
    t = tables.PFLookup.load(path)
    assert len(t.entries) >= 4
    for e in t.entries:
        assert abs(e["K"] - e["k0dz"] * t.n0) < 1e-12 * e["K"]
        for z, rec in ((np.linspace(-4, 2, 4001), e["max_err"]), (np.linspace(-4, 2, 100001), e["fine_max_err"])):
            r = e["r_inf"] + (1.0 / np.subtract.outer(z, e["poles"])) @ e["residues"]
            err = np.abs(r - fit.target(z, e["K"])).max()
            assert err <= 1.01 * rec + 1e-15
        assert e["max_err"] < 2e-5
        assert len(e["poles"]) == t.npoles and np.all(e["poles"].imag < 0)


def test_lookup_round_trip_and_misses(tmp_path):
    k0 = 2 * np.pi
    t = tables.PFLookup.build([k0 * 0.5, k0 * 1.0], 8, n0=1.0)
    p = tmp_path / "t.json"
    t.save(str(p))
    u = tables.PFLookup.load(str(p))
    b, a, r = u.get(k0, 1.0, 1.0)
    f = tables.RationalFit(k0, 8)
    assert np.allclose(np.sort_complex(b), np.sort_complex(f.poles), rtol=1e-12)
    assert abs(r - f.r_inf) < 1e-12
    with pytest.raises(KeyError):
        u.get(k0, 0.75, 1.0)          # k0 dz not tabulated
    with pytest.raises(KeyError):
        u.get(k0, 1.0, 1.0003)        # other reference index


# ---------------------------------------------------------------- absorbing-layer tables (Sec. 4.1)


@pytest.mark.parametrize("N,W,sm", [(32, 6, 1.0), (64, 12, 3.0)])
def test_pml_stretched_matrix_matches_oracle(N, W, sm):
    """The library's stretched one-axis operator and the oracle's (written separately from the
    same definition) agree entry by entry, and pml_eigen decomposes it."""
    from oracle import pml
    c, d = tables.stencil_d2(), tables.stencil_d1()
    g = pml.PMLGrid(N=N, h=0.25, k0=2 * np.pi, n0=1.0, c=c, d=d, W=W, sigma_max=sm)
    ref = g.s * pml.d2_stretched_matrix(g)
    A = tables.pml_stretched_d2(N, 0.25, 2 * np.pi, 1.0, W, sm, c, d)
    assert np.abs(A - ref).max() <= 1e-14 * np.abs(ref).max()
    Q, Qi, lam = tables.pml_eigen(N, 0.25, 2 * np.pi, 1.0, W, sm, c, d)
    assert np.abs(Q @ (lam[:, None] * Qi) - ref).max() < 1e-10 * np.abs(ref).max()
    assert lam.imag.min() > 0      # the layers move the spectrum above the real axis
