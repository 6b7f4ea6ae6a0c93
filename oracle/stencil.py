"""13-point, 4th-order explicit finite-difference stencils (oracle; test infrastructure).

Sec. 4.1 of the paper uses fourth-order explicit 13-point schemes for the
first and second transverse derivatives, tuned for resolving efficiency: the
second derivative is accurate to 0.5 % relative error over 83 % of the grid
bandwidth [0, pi/dx], an order of magnitude more than the 3-point scheme.  The
coefficients themselves are not printed (they are cited to another paper), so
this module designs them from that description:

* a 1-D stencil of half-width 6 (13 points) along one axis;
* D2 symmetric, D1 antisymmetric;
* the Taylor conditions for 4th order;
* the remaining free coefficients chosen to minimise the maximum relative
  error of the Fourier symbol over a design band (a linear programme).

Symbols (u_j = exp(i theta j), unit spacing):
    D2:  sigma2(theta) = -(c0 + 2 sum_m c_m cos(m theta))   (exact: theta^2)
    D1:  sigma1(theta) =  2 sum_m d_m sin(m theta)          (exact: theta)
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import linprog

HALF_WIDTH = 6
D2_BAND = 0.83 * np.pi   # design band of the second derivative (Sec. 4.1: 83 %)
D1_BAND = 0.70 * np.pi   # design band of the first derivative (reading; not printed)


def d2_symbol(c: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """sigma2(theta) for coefficients c = (c0, c1..c6)."""
    m = np.arange(1, len(c))
    return -(c[0] + 2.0 * np.cos(np.outer(theta, m)) @ c[1:])


def d1_symbol(d: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """sigma1(theta) for coefficients d = (d1..d6)."""
    m = np.arange(1, len(d) + 1)
    return 2.0 * np.sin(np.outer(theta, m)) @ d


def design_d2(band: float = D2_BAND, half_width: int = HALF_WIDTH, nsamp: int = 4000) -> np.ndarray:
    """Minimax-relative-error 4th-order D2 stencil (c0..c_hw).

    Unknowns x = (c0, c1..c_hw, t).  Minimise t subject to
    |sigma2(theta_i)/theta_i^2 - 1| <= t on the band and the Taylor conditions
    c0 + 2 sum c_m = 0, sum m^2 c_m = 1, sum m^4 c_m = 0.
    """
    hw = half_width
    theta = np.linspace(band / nsamp, band, nsamp)
    m = np.arange(1, hw + 1)
    # sigma2 / theta^2 is linear in c:  row . c
    rows = -np.hstack([np.ones((nsamp, 1)), 2.0 * np.cos(np.outer(theta, m))]) / theta[:, None] ** 2
    n = hw + 2
    a_ub = np.vstack([np.hstack([rows, -np.ones((nsamp, 1))]),
                      np.hstack([-rows, -np.ones((nsamp, 1))])])
    b_ub = np.concatenate([np.ones(nsamp), -np.ones(nsamp)])
    a_eq = np.zeros((3, n))
    a_eq[0, 0] = 1.0
    a_eq[0, 1:hw + 1] = 2.0
    a_eq[1, 1:hw + 1] = m ** 2
    a_eq[2, 1:hw + 1] = m ** 4
    b_eq = np.array([0.0, 1.0, 0.0])
    cost = np.zeros(n)
    cost[-1] = 1.0
    res = linprog(cost, A_ub=a_ub, b_ub=b_ub, A_eq=a_eq, b_eq=b_eq,
                  bounds=[(None, None)] * n, method="highs")
    if not res.success:
        raise RuntimeError(res.message)
    return res.x[:hw + 1]


def design_d1(band: float = D1_BAND, half_width: int = HALF_WIDTH, nsamp: int = 4000) -> np.ndarray:
    """Minimax-relative-error 4th-order D1 stencil (d1..d_hw).

    Taylor conditions: 2 sum m d_m = 1, sum m^3 d_m = 0.
    """
    hw = half_width
    theta = np.linspace(band / nsamp, band, nsamp)
    m = np.arange(1, hw + 1)
    rows = 2.0 * np.sin(np.outer(theta, m)) / theta[:, None]
    n = hw + 1
    a_ub = np.vstack([np.hstack([rows, -np.ones((nsamp, 1))]),
                      np.hstack([-rows, -np.ones((nsamp, 1))])])
    b_ub = np.concatenate([np.ones(nsamp), -np.ones(nsamp)])
    a_eq = np.zeros((2, n))
    a_eq[0, :hw] = 2.0 * m
    a_eq[1, :hw] = m ** 3
    b_eq = np.array([1.0, 0.0])
    cost = np.zeros(n)
    cost[-1] = 1.0
    res = linprog(cost, A_ub=a_ub, b_ub=b_ub, A_eq=a_eq, b_eq=b_eq,
                  bounds=[(None, None)] * n, method="highs")
    if not res.success:
        raise RuntimeError(res.message)
    return res.x[:hw]


def resolving_efficiency(symbol, exact, tol: float = 5e-3, nsamp: int = 200001) -> float:
    """Largest fraction f of [0, pi] such that |symbol/exact - 1| <= tol on (0, f*pi]."""
    theta = np.linspace(np.pi / nsamp, np.pi, nsamp)
    bad = np.abs(symbol(theta) / exact(theta) - 1.0) > tol
    if not bad.any():
        return 1.0
    return float(theta[np.argmax(bad)] / np.pi) - 1.0 / nsamp


_CACHE: dict = {}


def stencils() -> tuple[np.ndarray, np.ndarray]:
    """The oracle's (c, d) pair: c = (c0..c6) for D2, d = (d1..d6) for D1."""
    if "cd" not in _CACHE:
        _CACHE["cd"] = (design_d2(), design_d1())
    return _CACHE["cd"]
