"""The rational fit of Sec. 3.1 computed on the device (hp_fit_exp_sqrt) against the oracle's fit.

The two fits run the same published algorithm (AAA, Lawson reweighting, partial fractions) but
not the same arithmetic (the device takes the smallest singular vector by Gram-Schmidt QR and
Jacobi, the poles by Aberth's iteration), so their support points and poles need not coincide:
what must agree is the accuracy each reaches against exp(iK sqrt(1+z)), evaluated here by the
oracle's own target function."""
import time

import numpy as np
import pytest

from oracle import fit
from oracle import operator as op
from oracle import step as st

from helpers import K0, oracle_grid, rel_l2, to_gpu, workload

pytestmark = pytest.mark.gpu


def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("K,degree", [(2 * np.pi, 8), (2 * np.pi, 16), (2 * np.pi * 1.0003 * 0.05, 25),
                                      (2 * np.pi * 0.5, 12)])
def test_device_fit_matches_oracle_accuracy(K, degree):
    _cuda()
    from paper_2410_17446_amd import hp
    t0 = time.perf_counter()
    poles, res, r_inf, emax = hp.fit_exp_sqrt(K, degree)
    dt = time.perf_counter() - t0
    ora = fit.fit_exp_sqrt(K, degree)
    z = np.linspace(-4, 2, 4001)
    e = np.abs(r_inf + (1.0 / np.subtract.outer(z, poles)) @ res - fit.target(z, K)).max()
    zf = np.linspace(-4, 2, 100001)
    ef = np.abs(r_inf + (1.0 / np.subtract.outer(zf, poles)) @ res - fit.target(zf, K)).max()
    ev = np.abs(r_inf + (1.0 / np.subtract.outer(z, poles)) @ res - fit.target(z, K))
    print(f"K={K:.4f} degree {degree}: device {e:.6e} (reported {emax:.6e}, at z = {z[np.argmax(ev)]:.4f}; "
          f"fine {ef:.3e}) in {dt * 1e3:.0f} ms; oracle {ora['max_err']:.3e} (fine {ora['fine_max_err']:.3e})")
    assert len(poles) == degree and np.all(poles.imag < 0)
    assert abs(e - emax) <= 1e-3 * e + 1e-15, (e, emax)   # the error the library reports is this one
    assert e <= 3 * ora["max_err"]
    assert ef <= 3 * ora["fine_max_err"]


def test_device_fit_drives_a_step():
    """A plan built from the device fit (16 poles, dz = lambda) steps the 64^2 workload to within
    the two fits' error of the oracle's step with its own fit."""
    torch = _cuda()
    from paper_2410_17446_amd import hp
    wl = workload(N=64, W=8, npoles=16, tol=1e-10)
    ref, _ = st.step(oracle_grid(wl), op.coefficients(oracle_grid(wl), wl["n2"], False), wl["w"],
                     st.PFTable(wl["fit"]["poles"], wl["fit"]["residues"], wl["fit"]["r_inf"]), 1.0, 1e-10)
    poles, res, r_inf, emax = hp.fit_exp_sqrt(K0, 16)
    cfg = wl["cfg"]
    plan = hp.Plan(nx=64, ny=64, dx=cfg["dx"], dy=cfg["dx"], k0=K0, n0=1.0, dz=1.0, ncomp=1, poles=poles,
                   residues=res, r_inf=r_inf, d2=wl["c"], d1=wl["d"], edge_width=8, edge_eta=cfg["eta_max"],
                   tol=1e-10, restart=30, max_cycles=20)
    out = plan.step(to_gpu(wl["w"]), to_gpu(wl["n2"]))
    err = rel_l2(out.cpu().numpy(), ref)
    assert err < 20 * (emax + wl["fit"]["max_err"]), (err, emax)


def test_device_fit_rejects_bad_arguments():
    _cuda()
    from paper_2410_17446_amd import hp
    for args in ((0.0, 8), (K0, 0), (K0, 32)):
        with pytest.raises(hp.HPError):
            hp.fit_exp_sqrt(*args)
