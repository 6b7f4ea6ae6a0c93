"""Closed forms used to pin the oracle (test infrastructure).

* Plane waves in a homogeneous medium (Sec. 3, eq. exp_prop_planewave): the
  exact one-step factor of exp(i(kx x + ky y)) is
  exp(iK(-1 + sqrt(1 - (kx^2 + ky^2)/(k0 n0)^2))).
* Gaussian beams (Sec. 5.2, eq. eq_ft_gaussian): exp(-r^2/w^2) has the
  transform (w^2/2) exp(-k^2 w^2/4) under (1/2pi) int int ... e^{-i k.x}, so
  on the axis the exact field at range z is the Hankel integral
      u(0, 0, z) = int_0^inf (w^2/2) exp(-k^2 w^2/4) exp(i kz z) k dk,
  kz = sqrt((k0 n0)^2 - k^2) on the principal branch (evanescent for
  k > k0 n0).  |u| is the envelope amplitude the paper plots.
"""
from __future__ import annotations

import numpy as np
from scipy.integrate import quad


def plane_wave_factor(kx, ky, k0: float, n0: float, dz: float):
    K = k0 * n0 * dz
    zeta = -(np.asarray(kx) ** 2 + np.asarray(ky) ** 2) / (k0 * n0) ** 2
    return np.exp(1j * K * (-1.0 + np.sqrt(1.0 + zeta + 0j)))


def gaussian_axis_field(w: float, z: float, k0: float, n0: float) -> complex:
    kn = k0 * n0

    def kz(k):
        return np.sqrt(kn * kn - k * k + 0j)

    def f(k, part):
        v = 0.5 * w * w * np.exp(-k * k * w * w / 4.0) * np.exp(1j * kz(k) * z) * k
        return v.real if part == 0 else v.imag

    kmax = 12.0 / w
    pts = [kn] if kn < kmax else None
    re = quad(f, 0.0, kmax, args=(0,), points=pts, limit=400, epsabs=1e-14, epsrel=1e-12)[0]
    im = quad(f, 0.0, kmax, args=(1,), points=pts, limit=400, epsabs=1e-14, epsrel=1e-12)[0]
    return complex(re, im)
