"""Seeded synthetic workloads (beams, media, configurations).

This module only generates inputs: it holds none of the propagator's
arithmetic, and both the GPU library's callers and the CPU oracle's tests take
their fields from it.

Conventions: lambda = 1, k0 = 2 pi, n0 = 1; an N x N array per field
component, axis 0 = y, axis 1 = x; node j sits at x_j = (j - N/2) dx, nodes 0
and N are Dirichlet nodes, so row 0 and column 0 of every field are zero.
"""
from __future__ import annotations

import numpy as np

LAMBDA = 1.0
K0 = 2.0 * np.pi / LAMBDA
N0 = 1.0


def coords(N: int, dx: float) -> np.ndarray:
    return (np.arange(N) - N / 2) * dx


def gaussian_beam(N: int, dx: float, w0: float, ncomp: int = 1, x0: float = 0.0, y0: float = 0.0) -> np.ndarray:
    """exp(-r^2/w0^2) (1/e amplitude radius w0), x-polarised when ncomp = 2."""
    x = coords(N, dx)
    X, Y = np.meshgrid(x - x0, x - y0)
    u = np.exp(-(X ** 2 + Y ** 2) / w0 ** 2).astype(np.complex128)
    u[0, :] = 0.0
    u[:, 0] = 0.0
    out = np.zeros((ncomp, N, N), dtype=np.complex128)
    out[0] = u
    return out


def tilted_beam(N: int, dx: float, w0: float, sin_t: float, x0: float = 0.0) -> np.ndarray:
    """Gaussian beam (1/e radius w0) centred at x = x0 with the phase exp(i k0 sin_t x): travelling
    at angle asin(sin_t) to the axis in the x-z plane; (1, N, N)."""
    x = coords(N, dx)
    X, Y = np.meshgrid(x, x)
    u = np.exp(-((X - x0) ** 2 + Y ** 2) / w0 ** 2) * np.exp(1j * K0 * sin_t * X)
    u[0, :] = 0.0
    u[:, 0] = 0.0
    return u[None].astype(np.complex128)


def sine_product_n2(N: int, dx: float, amp: float, period: float) -> np.ndarray:
    """n^2 for n = 1 + amp sin(2 pi x/period) sin(2 pi y/period)."""
    x = coords(N, dx)
    X, Y = np.meshgrid(x, x)
    n = 1.0 + amp * np.sin(2 * np.pi * X / period) * np.sin(2 * np.pi * Y / period)
    return n * n


# Rotation of the sine-product medium of Sec. 5 (eq. sineprod): axis and angle.
ROT_AXIS = (0.258, 0.312, 0.914)
ROT_ANGLE = 0.128


def rotation_matrix() -> np.ndarray:
    """R of the rotated sine product: rotation by ROT_ANGLE about the unit vector along
    ROT_AXIS (axis-angle / Rodrigues form)."""
    u = np.asarray(ROT_AXIS, dtype=float)
    u = u / np.linalg.norm(u)
    c, s = np.cos(ROT_ANGLE), np.sin(ROT_ANGLE)
    ux = np.array([[0.0, -u[2], u[1]], [u[2], 0.0, -u[0]], [-u[1], u[0], 0.0]])
    return c * np.eye(3) + s * ux + (1.0 - c) * np.outer(u, u)


def rotated_sine_n2(N: int, dx: float, z: float, n0: float = 1.2, dn: float = 0.025, q: float = 1.0,
                    k0: float = 2.0 * np.pi) -> np.ndarray:
    """n^2 on the plane z of the rotated sine product of Sec. 5 (eq. sineprod):
    n = n0 + dn sin(ks x~) sin(ks y~) sin(ks z~), ks = k0 n0 / (sqrt(3) q), with
    (x~, y~, z~) = R (x, y, z) (rotation_matrix()); x, y on the grid's coordinates."""
    R = rotation_matrix()
    xs = coords(N, dx)
    X, Y = np.meshgrid(xs, xs)
    P = np.stack([X, Y, np.full_like(X, z)])
    Xt = np.tensordot(R, P, axes=1)
    ks = k0 * n0 / (np.sqrt(3.0) * q)
    n = n0 + dn * np.sin(ks * Xt[0]) * np.sin(ks * Xt[1]) * np.sin(ks * Xt[2])
    return n * n


def grf_n2(N: int, dx: float, rms: float, corr_len: float, seed: int) -> np.ndarray:
    """n^2 = 1 + delta, delta a Gaussian random field.

    White N(0,1) noise (PCG64, seed) filtered in periodic Fourier space by
    sqrt(S(k)), S(k) = exp(-k^2 corr_len^2 / 2) (correlation exp(-r^2/(2 corr_len^2))),
    real part, mean removed, rescaled to rms exactly.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    white = rng.standard_normal((N, N))
    k = 2 * np.pi * np.fft.fftfreq(N, d=dx)
    KX, KY = np.meshgrid(k, k)
    filt = np.sqrt(np.exp(-(KX ** 2 + KY ** 2) * corr_len ** 2 / 2.0))
    delta = np.real(np.fft.ifft2(np.fft.fft2(white) * filt))
    delta -= delta.mean()
    delta *= rms / np.sqrt(np.mean(delta ** 2))
    return 1.0 + delta


def random_field(N: int, ncomp: int, seed: int) -> np.ndarray:
    """Complex N(0,1) field (row/col 0 zero) for operator-level parity checks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.standard_normal((ncomp, N, N)) + 1j * rng.standard_normal((ncomp, N, N))
    u[:, 0, :] = 0.0
    u[:, :, 0] = 0.0
    return u


# Named workloads.  W is the edge-layer width in cells, eta_max the peak
# Im(n^2) of its loss, dz the step, npoles the (N,N) type of the rational fit.
CONFIGS = {
    "scalar64": dict(N=64, dx=0.25, ncomp=1, W=8, eta_max=0.25, dz=1.0, npoles=8, steps=10,
                     tol=1e-10, restart=30, medium=("sine", 0.05, 2.0), w0=4.0),
    "scalar1024": dict(N=1024, dx=0.25, ncomp=1, W=128, eta_max=0.25, dz=1.0, npoles=16, steps=200,
                       tol=1e-8, restart=30, medium=("sine", 0.02, 1.0), w0=32.0),
    "vector2048": dict(N=2048, dx=0.25, ncomp=2, W=256, eta_max=0.25, dz=1.0, npoles=24, steps=100,
                       tol=1e-8, restart=30, medium=("grf", 1e-3, 2.0, 3), w0=64.0),
}


def medium_n2(cfg: dict) -> np.ndarray:
    m = cfg["medium"]
    if m[0] == "sine":
        return sine_product_n2(cfg["N"], cfg["dx"], m[1], m[2])
    if m[0] == "grf":
        return grf_n2(cfg["N"], cfg["dx"], m[1], m[2], m[3])
    if m[0] == "uniform":
        return np.ones((cfg["N"], cfg["N"]))
    raise ValueError(m)


def beam(cfg: dict) -> np.ndarray:
    return gaussian_beam(cfg["N"], cfg["dx"], cfg["w0"], cfg["ncomp"])


def batch_configs(count: int = 64, seed: int = 4) -> list[dict]:
    """Serving-style batch: N in {256,384,512,768,1024}, poles in {8,12,16},
    sine-product (as scalar1024) or random (as vector2048, scalar) media, W = N/8,
    w0 = N dx / 8, 50 steps each; medium seed 4000 + i."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        N = int(rng.choice([256, 384, 512, 768, 1024]))
        npoles = int(rng.choice([8, 12, 16]))
        kind = "sine" if rng.random() < 0.5 else "grf"
        medium = ("sine", 0.02, 1.0) if kind == "sine" else ("grf", 1e-3, 2.0, 4000 + i)
        out.append(dict(N=N, dx=0.25, ncomp=1, W=N // 8, eta_max=0.25, dz=1.0, npoles=npoles, steps=50,
                        tol=1e-8, restart=30, medium=medium, w0=N * 0.25 / 8))
    return out


def random_beam(N: int, dx: float, ncomp: int, seed: int) -> np.ndarray:
    """A Gaussian beam with seeded waist (N dx / 16 .. N dx / 6), centre offset (within
    N dx / 10 of the middle), tilt (transverse wavenumber up to 0.15 k0 per axis) and
    curvature phase; for ncomp = 2 a seeded linear polarisation angle."""
    rng = np.random.Generator(np.random.PCG64(seed))
    L = N * dx
    w0 = rng.uniform(L / 16, L / 6)
    cx, cy = rng.uniform(-L / 10, L / 10, size=2)
    kx, ky = rng.uniform(-0.15, 0.15, size=2) * K0
    curv = rng.uniform(-0.5, 0.5) / w0 ** 2
    x = coords(N, dx)
    X, Y = np.meshgrid(x - cx, x - cy)
    r2 = X ** 2 + Y ** 2
    u = np.exp(-r2 / w0 ** 2 + 1j * (kx * X + ky * Y + curv * r2))
    u[0, :] = 0.0
    u[:, 0] = 0.0
    out = np.zeros((ncomp, N, N), dtype=np.complex128)
    if ncomp == 1:
        out[0] = u
    else:
        a = rng.uniform(0, np.pi)
        out[0], out[1] = np.cos(a) * u, np.sin(a) * u
    return out


def random_medium(N: int, dx: float, seed: int) -> np.ndarray:
    """Training media: half Gaussian random fields (rms log-uniform in [1e-3, 2e-2],
    correlation length uniform in [1, 3] lambda), half sine products (amplitude uniform
    in [0.005, 0.03], period uniform in [1, 2] lambda)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if rng.random() < 0.5:
        rms = float(np.exp(rng.uniform(np.log(1e-3), np.log(2e-2))))
        return grf_n2(N, dx, rms, float(rng.uniform(1.0, 3.0)), int(rng.integers(1 << 30)))
    return sine_product_n2(N, dx, float(rng.uniform(0.005, 0.03)), float(rng.uniform(1.0, 2.0)))
