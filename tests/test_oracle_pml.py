"""Pins of the oracle's PML (oracle/pml.py): complex-coordinate stretching of Sec. 4.1 and the
Sylvester preconditioner of eq. fs_sylvester with the stretched derivative matrices.

Each test checks the oracle against something other than itself: the analytic continuation of a
plane wave through the stretched coordinate, a dense Kronecker solve, the position of the
spectrum against the poles, and a free-space run on a domain large enough to have no boundary in
reach."""
import numpy as np
import pytest

from oracle import fit, pml, stencil
from oracle import operator as op

K2PI = 2 * np.pi


def _grid(N, W, sm, h=0.25):
    c, d = stencil.stencils()
    return pml.PMLGrid(N=N, h=h, k0=K2PI, n0=1.0, c=c, d=d, W=W, sigma_max=sm)


@pytest.mark.parametrize("kh", [0.3, 0.6, 1.2])
def test_stretched_second_derivative_of_the_continued_plane_wave(kh):
    """d^2/dx~^2 exp(i k x~) = -k^2 exp(i k x~) for x~ = x + i int sigma: with s = 1 + i sigma the
    discrete (1/s^2) D2 - (s'/s^3) D1 reproduces it to the 13-point stencils' accuracy at every
    node the odd reflection does not reach, inside the layers (where |u| varies by orders of
    magnitude) and outside.  A dropped s' term, 1/s in place of 1/s^2 or a wrong sign of s' is
    off by O(s'/k) ~ 0.1."""
    N, h, W, sm = 64, 0.25, 10, 0.5
    g = _grid(N, W, sm, h)
    D = pml.d2_stretched_matrix(g)
    x = np.arange(N) * h
    tl = np.clip(W + 1 - x / h, 0, None)           # left layer: distance-to-the-interior ramp
    tr = np.clip(W + 1 - (N - x / h), 0, None)     # right layer
    im_xt = -sm * h * tl ** 3 / (3 * W ** 2) + sm * h * tr ** 3 / (3 * W ** 2)
    k = kh / h
    u = np.exp(1j * k * (x + 1j * im_xt))
    r = D @ u[1:] + k ** 2 * u[1:]
    inner = slice(6, N - 1 - 6)
    assert np.abs(r[inner]).max() < 1e-2 * np.abs(k ** 2 * u[1:][inner]).max()
    # outside the layers the matrix is the plain 13-point D2
    D0 = pml.d2_stretched_matrix(_grid(N, W, 0.0, h))
    assert np.allclose(D[W + 6:N - W - 7], D0[W + 6:N - W - 7], atol=0, rtol=0)


def test_pml_preconditioner_is_the_dense_kronecker_solve():
    """eq. fs_sylvester by Bartels-Stewart equals the dense solve of (s (I (x) D2x~ + D2y~ (x) I) - b)
    vec(W) = vec(R) built from unit vectors (tiny grid)."""
    N = 20
    g = _grid(N, 5, 1.0)
    D = pml.d2_stretched_matrix(g)
    n = N - 1
    rng = np.random.default_rng(3)
    R = np.zeros((N, N), complex)
    R[1:, 1:] = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    b = -0.7 - 0.05j
    big = g.s * (np.kron(np.eye(n), D) + np.kron(D, np.eye(n))) - b * np.eye(n * n)
    ref = np.linalg.solve(big, R[1:, 1:].reshape(-1)).reshape(n, n)
    out = pml.apply_minv(g, R, b, D)
    assert np.abs(out[1:, 1:] - ref).max() < 1e-10 * np.abs(ref).max()
    # and the operator with V = 0 is that dense matrix
    V = pml.medium(g, np.ones((N, N)))
    Aw = pml.apply_shifted(g, V, out, b, D)
    assert np.abs(Aw[1:, 1:] - R[1:, 1:]).max() < 1e-9 * np.abs(R).max()


def test_pml_spectrum_lies_above_the_poles():
    """With s = 1 + i sigma the free-space eigenvalues move into the upper half plane, where
    exp(iK sqrt(1+z)) has modulus <= 1 and the rational approximation has no poles (all b_k lie
    below the real axis): the shifted systems stay well separated from singular, and
    |e^{-iK} r| on the spectrum stays at the fit's overshoot next to the branch point."""
    g = _grid(48, 10, 0.5)
    lam1 = np.linalg.eigvals(g.s * pml.d2_stretched_matrix(g))
    assert lam1.imag.min() > 0
    lam = (lam1[:, None] + lam1[None, :]).ravel()
    f = fit.fit_exp_sqrt(K2PI, 8)
    assert np.abs(lam[:, None] - f["poles"][None, :]).min() > 0.05
    r = np.exp(-1j * K2PI) * fit.eval_pf(lam, f["poles"], f["residues"], f["r_inf"])
    assert np.abs(r).max() < 1.01


def test_pml_absorbs_a_beam_leaving_the_domain():
    """A Gaussian beam (waist 2 lambda) tilted at 30 degrees in free space: with the PML, the field
    in the physical region after 14 steps of lambda (the beam half inside the layer) matches the
    same propagation on a twice larger Dirichlet domain, whose walls the beam never reaches, to
    1e-2 of the initial peak, and after 24 steps 1 % of the power is left; without stretching
    (sigma = 0) the walls reflect and neither holds."""
    f = fit.fit_exp_sqrt(K2PI, 8)

    def run(N, W, sm, steps):
        g = _grid(N, W, sm)
        xs = (np.arange(N) - N / 2) * g.h
        X, Y = np.meshgrid(xs, xs)
        w = np.exp(-(X ** 2 + Y ** 2) / 2.0 ** 2) * np.exp(1j * K2PI * 0.5 * X)
        w[0, :] = 0
        w[:, 0] = 0
        V = pml.medium(g, np.ones((N, N)))
        p0 = np.sum(np.abs(w) ** 2)
        for _ in range(steps):
            w, _ = pml.step(g, V, w, f["poles"], f["residues"], f["r_inf"], 1.0, 1e-10)
        return w, np.sum(np.abs(w) ** 2) / p0

    ref, _ = run(128, 1, 0.0, 14)
    phys = slice(64 - 18, 64 + 18)                 # |x|, |y| <= 4.5 lambda
    core = ref[phys, phys]
    for sm, ok in ((1.0, True), (0.0, False)):
        w, _ = run(64, 12, sm, 14)
        err = np.abs(w[32 - 18:32 + 18, 32 - 18:32 + 18] - core).max()
        assert (err < 1e-2) == ok, (sm, err)
    _, p = run(64, 12, 1.0, 24)
    assert p < 1e-2
    _, p0 = run(64, 12, 0.0, 24)
    assert p0 > 0.5


def test_vector_pml_operator_reduces_to_the_scalar_one_in_a_homogeneous_medium():
    """With n = n0 (psi = 0, V = 0) the vector operator decouples: each component is the scalar
    PML operator.  This pins the replacement of the plain Laplacian rows by the stretched ones (a
    plain Laplacian left in, or a wrong sign, fails)."""
    g = _grid(40, 8, 1.5)
    co = op.coefficients(pml.vector_grid(g), np.ones((40, 40)), True)
    rng = np.random.default_rng(11)
    w = rng.standard_normal((2, 40, 40)) + 1j * rng.standard_normal((2, 40, 40))
    w[:, 0, :] = 0
    w[:, :, 0] = 0
    b = -0.4 - 0.02j
    out = pml.apply_shifted_vector(g, co, w, b)
    V = pml.medium(g, np.ones((40, 40)))
    for c in range(2):
        ref = pml.apply_shifted(g, V, w[c], b)
        assert np.abs(out[c] - ref).max() < 1e-12 * np.abs(ref).max()


def test_vector_pml_operator_keeps_the_coupling_in_the_interior():
    """Away from the layers (every stencil point outside them) the vector PML operator is the plain
    vector operator of eq. Z_bar_eq, psi coupling included; inside the layers it is the scalar PML
    operator per component (psi and V are zero there)."""
    N, W = 48, 8
    g = _grid(N, W, 2.0)
    x = (np.arange(N) - N / 2) * g.h
    X, Y = np.meshgrid(x, x)
    n2 = (1 + 0.05 * np.sin(2 * np.pi * X / 2.0) * np.sin(2 * np.pi * Y / 2.0)) ** 2
    og = pml.vector_grid(g)
    co = op.coefficients(og, n2, True)
    rng = np.random.default_rng(12)
    w = rng.standard_normal((2, N, N)) + 1j * rng.standard_normal((2, N, N))
    w[:, 0, :] = 0
    w[:, :, 0] = 0
    b = -1.1 - 0.07j
    out = pml.apply_shifted_vector(g, co, w, b)
    plain = op.apply_shifted(og, co, w, b)
    inner = slice(W + 7, N - W - 6)
    assert np.abs(out[:, inner, inner] - plain[:, inner, inner]).max() < 1e-12 * np.abs(plain).max()
    assert np.abs(co.psi_x[inner, inner]).max() > 1e-3         # the coupling is really there
    V = pml.medium(g, n2)
    edge = (slice(1, W + 1), slice(1, N))
    for c in range(2):
        ref = pml.apply_shifted(g, V, w[c], b)
        assert np.abs(out[c][edge] - ref[edge]).max() < 1e-12 * np.abs(ref).max()


def test_vector_pml_step_of_a_decoupled_field_is_the_scalar_step():
    """In a homogeneous medium an x-polarised beam stays x-polarised and its step is the scalar
    PML step (the solves and the weighted sum per component)."""
    N, W = 32, 6
    g = _grid(N, W, 1.0)
    f = fit.fit_exp_sqrt(K2PI, 6)
    x = (np.arange(N) - N / 2) * g.h
    X, Y = np.meshgrid(x, x)
    u = np.exp(-(X ** 2 + Y ** 2) / 1.5 ** 2) * np.exp(1j * K2PI * 0.4 * X)
    u[0, :] = 0
    u[:, 0] = 0
    w = np.stack([u, np.zeros_like(u)])
    co = op.coefficients(pml.vector_grid(g), np.ones((N, N)), True)
    out, _ = pml.step_vector(g, co, w, f["poles"], f["residues"], f["r_inf"], 1.0, 1e-11)
    ref, _ = pml.step(g, pml.medium(g, np.ones((N, N))), u, f["poles"], f["residues"], f["r_inf"], 1.0, 1e-11)
    assert np.abs(out[1]).max() < 1e-12
    assert np.abs(out[0] - ref).max() < 1e-9 * np.abs(ref).max()
