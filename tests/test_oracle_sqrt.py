"""Pins of the oracle's pseudo-differential propagator (Sec. 2 eq. eq_barZfactor2,
Sec. 3.2, Appendix A) against closed forms, an independent quadrature, the
paper's stated accuracy behaviour and brute force on tiny grids."""
import numpy as np
import pytest
from scipy.integrate import quad

from oracle import precond, stencil
from oracle import operator as op
from oracle import sqrt_form as sf
from paper_2410_17446_amd import inputs

K2PI = 2 * np.pi


def _eval(pf, z):
    z = np.asarray(z, dtype=complex)
    return pf.r_inf + sum(a / (z - b) for a, b in zip(pf.residues, pf.poles))


def _grid(N, W=6, eta=0.0, dx=0.25):
    c, d = stencil.stencils()
    return op.Grid(N=N, dx=dx, dy=dx, k0=K2PI, n0=1.0, c=c, d=d, W=W, eta_max=eta)


# ---------------------------------------------------------------- the quadrature rule

@pytest.mark.parametrize("N", [1, 5, 25, 45])
def test_gauss_jacobi_rule_is_chebyshev_third_kind(N):
    """The weight sqrt((1+x)/(1-x)) is that of the Chebyshev polynomials of the third
    kind, whose Gauss rule is known in closed form: nodes cos(theta_j),
    theta_j = (2j-1) pi/(2N+1), weights 2 pi (1 + cos theta_j)/(2N+1) (Mason and Handscomb)."""
    eta, om = sf.gauss_jacobi_sqrt(N)
    th = (2 * np.arange(1, N + 1) - 1) * np.pi / (2 * N + 1)
    o = np.argsort(eta)
    oc = np.argsort(np.cos(th))
    assert np.allclose(eta[o], np.cos(th)[oc], rtol=0, atol=1e-14)
    wc = 4 * np.pi / (2 * N + 1) * np.cos(th / 2) ** 2  # 1 + cos(theta) without cancellation
    assert np.allclose(om[o], wc[oc], rtol=1e-11, atol=0)  # Golub-Welsch weights: ~2e-12 at N = 45


def test_gauss_jacobi_rule_exact_on_polynomials():
    """An N-point Gauss rule integrates polynomials of degree < 2N exactly; the integrals
    come from QUADPACK's algebraic-singularity routine, not from a Gauss rule."""
    N = 6
    eta, om = sf.gauss_jacobi_sqrt(N)
    for m in range(2 * N):
        ref, _ = quad(lambda x: x ** m, -1, 1, weight="alg", wvar=(0.5, -0.5), epsabs=1e-14, epsrel=1e-14)
        assert abs(np.sum(om * eta ** m) - ref) < 1e-12


# ---------------------------------------------------------------- the partial fractions

@pytest.mark.parametrize("N,alpha", [(12, 1.0), (25, 1.0), (45, 0.1), (7, 2.5)])
def test_value_at_branch_point_closed_form(N, alpha):
    """At zeta = -1 (w = -1) sqrt(1+zeta) = 0, and with the closed-form rule
    sum_j omega_j/(1 + eta_j) = 2 pi N/(2N+1), so the partial fractions take exactly
    c_alpha (1 - 2N/(2N+1)) = c_alpha/(2N+1): the slow convergence at the branch
    point that Sec. 3.2 warns of."""
    pf = sf.cauchy_sqrt_pf(N, alpha)
    c_alpha = np.sqrt(alpha) * np.exp(1j * np.pi / 4)
    v = _eval(pf, -1.0)
    assert abs(v - c_alpha / (2 * N + 1)) < 1e-13 * (1 + abs(c_alpha))


def test_matches_sqrt_away_from_branch_point():
    """alpha = 1, N = 25 (the paper's accuracy figure): the expansion reproduces
    sqrt(1+zeta) (i sqrt(-1-zeta) below -1) to roundoff away from zeta = -1, also on
    the part of the discrete spectrum below the fit interval (to -7)."""
    pf = sf.cauchy_sqrt_pf(25, 1.0)
    z = np.linspace(-7.0, 2.0, 9001)
    e = np.abs(_eval(pf, z) - sf.sqrt_principal(z))
    away = np.abs(z + 1) >= 0.2
    assert e[away & (z >= -4.0)].max() < 1e-12
    assert e[away].max() < 1e-11  # the rate slows toward -inf (w -> 1)
    assert e.max() <= 1.0 / 51 + 1e-12  # the branch-point value is the worst


@pytest.mark.parametrize("zeta", [2.0, 1.0, -0.5, -3.0])
def test_geometric_convergence_rate(zeta):
    """Sec. 3.2: for w off the cut the Gauss-Jacobi error decays geometrically, set by
    the ellipse with foci -1, 1 through w: one more node divides the error by rho^2,
    rho = |w + sqrt(w^2 - 1)| > 1 (semi-axis sum)."""
    alpha = 1.0
    w = (zeta + 1 + 1j * alpha) / (zeta + 1 - 1j * alpha)
    s = np.sqrt(w * w - 1 + 0j)
    rho = max(abs(w + s), abs(w - s))
    e = [abs(_eval(sf.cauchy_sqrt_pf(N, alpha), zeta) - sf.sqrt_principal(zeta)) for N in range(4, 13)]
    ratios = np.array(e[1:]) / np.array(e[:-1])
    assert np.allclose(ratios, rho ** -2, rtol=2e-3)


def test_cauchy_integral_representation():
    """Appendix A: with the cut on [-1, 1], g(w) = c_alpha (1 - (1/pi) int sqrt((1+eta)/(1-eta))
    /(eta - w) deta) equals sqrt(1 + zeta(w)); the integral by QUADPACK's algebraic-weight
    routine, and the partial fractions agree with it (they are its quadrature)."""
    alpha = 1.0
    c_alpha = np.sqrt(alpha) * np.exp(1j * np.pi / 4)
    pf = sf.cauchy_sqrt_pf(40, alpha)
    for zeta in [1.7, 0.3, -0.6, -2.5, -5.0, 0.4 + 0.3j]:
        w = (zeta + 1 + 1j * alpha) / (zeta + 1 - 1j * alpha)
        re, _ = quad(lambda x: (1 / (x - w)).real, -1, 1, weight="alg", wvar=(0.5, -0.5), epsabs=1e-14)
        im, _ = quad(lambda x: (1 / (x - w)).imag, -1, 1, weight="alg", wvar=(0.5, -0.5), epsabs=1e-14)
        g = c_alpha * (1 - (re + 1j * im) / np.pi)
        exact = np.sqrt(1 + zeta) if isinstance(zeta, complex) else sf.sqrt_principal(zeta)
        assert abs(g - exact) < 1e-10
        assert abs(_eval(pf, zeta) - g) < 1e-10


def test_alpha_trade_off():
    """Sec. 3.2: alpha = 0.1 narrows the low-accuracy band at the branch point but at fixed
    N loses accuracy elsewhere; N = 45 restores it."""
    z = np.linspace(-4.0, 2.0, 60001)
    ex = sf.sqrt_principal(z)

    def err(N, a):
        return np.abs(_eval(sf.cauchy_sqrt_pf(N, a), z) - ex)

    def band(e):
        bad = z[e > 1e-6]
        return bad.max() - bad.min()

    away = np.abs(z + 1) >= 0.5
    e1, e2, e3 = err(25, 1.0), err(25, 0.1), err(45, 0.1)
    assert e2[away].max() > 1e6 * e1[away].max()
    assert e3[away].max() < 1e-9
    assert band(e3) < band(e1) / 10


# ---------------------------------------------------------------- the z-integrator

def test_rk4_homogeneous_closed_form():
    """n = n0, no layer loss: Zbar is the free-space operator, diagonal in the DST basis, so
    each mode is multiplied per substep by the RK4 polynomial of h i k0 n0 (r(mu_p + mu_q) - 1),
    and every solve takes one preconditioned iteration."""
    N, dz, sub = 48, 0.25, 2
    g = _grid(N, W=8)
    pf = sf.cauchy_sqrt_pf(12, 1.0)
    w = inputs.gaussian_beam(N, g.dx, 2.0)
    co = op.coefficients(g, np.ones((N, N)), False)
    out, iters = sf.rk4_step(g, co, w, pf, dz, sub, 1e-12)
    assert list(iters) == [4 * sub] * 12
    lam = precond.spectrum(g)
    h = dz / sub
    R = sf.rk4_amplification(h * 1j * K2PI * (_eval(pf, lam) - 1.0))
    t = precond.dst2(w)
    t[..., 1:, 1:] *= R ** sub
    ref = precond.dst2(t)
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) < 1e-12


@pytest.mark.parametrize("vector", [False, True])
def test_rk4_brute_force_tiny_grid(vector):
    """Inhomogeneous medium and a lossy layer on a tiny grid: the RK4 step equals the dense
    matrix polynomial of h L, L = i k0 n0 (r(Zbar) - I) with r(Zbar) from dense solves."""
    N, dz, sub = 16, 0.2, 2
    g = _grid(N, W=6, eta=0.25)
    nc = 2 if vector else 1
    x = inputs.coords(N, g.dx)
    X, Y = np.meshgrid(x, x)
    n2 = 1.0 + 0.15 * np.exp(-(X ** 2 + Y ** 2) / 0.5) * (1 + 0.5 * np.sin(3 * X))
    co = op.coefficients(g, n2, vector)
    w = inputs.random_field(N, nc, seed=12)
    pf = sf.cauchy_sqrt_pf(10, 1.0)
    out, _ = sf.rk4_step(g, co, w, pf, dz, sub, 1e-13)
    Z = op.dense_zbar(g, co, nc)
    n = len(Z)
    R = pf.r_inf * np.eye(n, dtype=complex)
    for bk, ak in zip(pf.poles, pf.residues):
        R = R + ak * np.linalg.inv(Z - bk * np.eye(n))
    h = dz / sub
    L = 1j * K2PI * (R - np.eye(n))
    step = np.eye(n) + h * L + (h * L) @ (h * L) / 2 + np.linalg.matrix_power(h * L, 3) / 6 \
        + np.linalg.matrix_power(h * L, 4) / 24
    mask = op.pack(np.broadcast_to(op.absorber_mask(g, h), (nc, N, N)))
    v = op.pack(w)
    for _ in range(sub):
        v = mask * (step @ v)
    assert np.linalg.norm(op.pack(out) - v) / np.linalg.norm(v) < 1e-11


def test_rk4_converges_to_exponential_propagator():
    """As the substep shrinks, the pseudo-differential form integrated by RK4 approaches
    the exponential propagator exp(iK(-1 + sqrt(1 + Zbar))) (Sec. 2 eq. expop_prop),
    here in free space where that is a per-mode phase; fourth order: halving h divides
    the error by about 16."""
    N, dz = 64, 0.5
    g = _grid(N, W=8)
    pf = sf.cauchy_sqrt_pf(25, 1.0)
    w = inputs.gaussian_beam(N, g.dx, 2.0)
    co = op.coefficients(g, np.ones((N, N)), False)
    lam = precond.spectrum(g)
    t = precond.dst2(w)
    t[..., 1:, 1:] *= np.exp(1j * K2PI * dz * (-1 + sf.sqrt_principal(lam)))
    ref = precond.dst2(t)
    errs = []
    for sub in (4, 8):
        out, _ = sf.rk4_step(g, co, w, pf, dz, sub, 1e-12)
        errs.append(np.linalg.norm(out - ref) / np.linalg.norm(ref))
    assert errs[1] < 2e-4
    assert 12 < errs[0] / errs[1] < 20
