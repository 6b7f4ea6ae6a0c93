"""Oracle parity at the vector workload's full size (2048^2, E_x and E_y coupled, Gaussian random
medium of rms 1e-3 and correlation length 2 lambda, 24 poles) and of the batch of independent
propagations, through the C ABI.

The 2048^2 instances of the transforms (an 8 x 16 x 16 FFT per 2048-point DST-I, 131 KB of LDS per
row-pass workgroup) run only at this size, so they are compared with the oracle here: the
preconditioner in every precision, and single pole solves (the whole coupled operator, the column
and row passes, Gram-Schmidt and the least squares) with the oracle's iteration count replayed in
FP64, and at a tight tolerance in the mixed modes."""
import functools

import numpy as np
import pytest

from oracle import operator as op
from oracle import precond
from oracle import step as st
from paper_2410_17446_amd import inputs

from helpers import gpu_plan, oracle_grid, oracle_pf, rel_l2, to_gpu, workload

pytestmark = pytest.mark.gpu

N = 2048


def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _vector_workload(npoles=24, tol=1e-8):
    cfg = inputs.CONFIGS["vector2048"]
    return workload(N=N, ncomp=2, W=cfg["W"], npoles=npoles, medium=cfg["medium"], w0=cfg["w0"], tol=tol)


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_vector2048_preconditioner_matches_oracle(precision):
    """M_k^-1 on both components at 2048^2, against the oracle's DST solve: the transforms' own
    rounding (a multiple of eps log2 N) amplified by kappa_k = max|mu - b_k| / min|mu - b_k| in the
    divide, bound eps (20 kappa_k + 50 log2 N) (eps of the transform arithmetic: FP64; complex64 in
    HP_MIXED, complex64 storage in HP_MIXED64)."""
    torch = _cuda()
    wl = _vector_workload()
    g = oracle_grid(wl)
    lam = precond.spectrum(g)
    x = inputs.random_field(N, 2, seed=21)
    eps = 2.2e-16 if precision == 0 else 1.2e-7
    plan = gpu_plan(wl, precision=precision, restart=1)   # one Krylov vector per pole: 16 GB in FP64
    xd = to_gpu(x)
    for pole in (0, 11, 23):
        b = wl["fit"]["poles"][pole]
        kappa = np.abs(lam - b).max() / np.abs(lam - b).min()
        ref = precond.apply_minv(g, x, b)
        y = torch.zeros_like(xd)
        plan.apply_preconditioner(pole, xd, y)
        err = rel_l2(y.cpu().numpy(), ref)
        bound = eps * (20 * kappa + 50 * np.log2(N))
        print(f"precision {precision}, pole {pole}: relative L2 {err:.3e}, bound {bound:.3e}")
        assert err < bound, (pole, err, kappa)
    plan.close()


def _two_pole_plan(wl, poles, precision, tol):
    """A plan holding only the given poles of the 24-pole table (Krylov storage for two poles)."""
    sub = dict(wl)
    f = wl["fit"]
    sub["fit"] = dict(poles=f["poles"][list(poles)], residues=f["residues"][list(poles)], r_inf=f["r_inf"])
    sub["cfg"] = dict(wl["cfg"], npoles=len(poles))
    return gpu_plan(sub, precision=precision, tol=tol)


TOL = 1e-11


@functools.lru_cache(maxsize=None)
def _solve_case():
    """The workload, its oracle coefficients and the two poles checked: the one nearest the real
    axis (the hardest solve) and the one farthest from it."""
    wl = _vector_workload(tol=TOL)
    g = oracle_grid(wl)
    co = op.coefficients(g, wl["n2"], True)
    f = wl["fit"]
    return wl, g, co, (int(np.argmax(f["poles"].imag)), int(np.argmin(f["poles"].imag)))


@functools.lru_cache(maxsize=None)
def _oracle_solve(pole):
    """The oracle's solve of pole `pole` at TOL (about a minute of numpy per pole at 2048^2)."""
    wl, g, co, _ = _solve_case()
    return st.solve_pole(g, co, wl["w"], wl["fit"]["poles"][pole], TOL, 30)


@pytest.mark.timeout(400)
@pytest.mark.parametrize("which", [0, 1])
def test_vector2048_pole_solve_matches_oracle_fp64(which):
    """A shifted solve (Zbar - b_k I) x = w of the vector workload, FP64, with the oracle's
    iteration count replayed: 1e-10 relative L2."""
    _cuda()
    wl, g, co, picks = _solve_case()
    pole = picks[which]
    res = _oracle_solve(pole)
    assert res.cycles == 1, res.cycle_iters
    plan = _two_pole_plan(wl, picks, 0, TOL)
    plan.set_medium(to_gpu(wl["n2"]))
    iters = [1, 1]
    iters[which] = res.iters
    plan.set_fixed_iters(iters)
    x = plan.solve(which, to_gpu(wl["w"])).cpu().numpy()
    plan.close()
    err = rel_l2(x, op.unpack(res.x, 2, N))
    print(f"pole {pole} (b = {wl['fit']['poles'][pole]:.4g}): {res.iters} iterations, relative L2 {err:.3e}")
    assert err < 1e-10, (pole, err)


@pytest.mark.timeout(400)
@pytest.mark.parametrize("precision", [1, 2])
def test_vector2048_pole_solves_match_oracle_mixed(precision):
    """The same two solves in the mixed modes, each side to its own tolerance 1e-11 on the FP64
    true residual (the mixed modes refine in FP64): 1e-6 relative L2."""
    _cuda()
    wl, g, co, picks = _solve_case()
    plan = _two_pole_plan(wl, picks, precision, TOL)
    plan.set_medium(to_gpu(wl["n2"]))
    w = to_gpu(wl["w"])
    for slot, pole in enumerate(picks):
        res = _oracle_solve(pole)
        x = plan.solve(slot, w).cpu().numpy()
        it, rr = plan.stats()
        err = rel_l2(x, op.unpack(res.x, 2, N))
        print(f"precision {precision}, pole {pole}: GPU {it[slot]} / oracle {res.iters} iterations, "
              f"relative residual {rr[slot]:.2e}, relative L2 {err:.3e}")
        assert rr[slot] <= TOL and err < 1e-6, (pole, err)
    plan.close()


def test_batch_matches_oracle_steps():
    """Independent propagations of uneven sizes, pole counts and media run concurrently by the
    batch workers: each problem's field after one step against the oracle's step, both sides at
    tol 1e-12 (so the two GMRES, Householder and Gram-Schmidt, stop at iterates 1e-12 apart)."""
    torch = _cuda()
    from paper_2410_17446_amd import hp
    specs = [(64, 8, ("sine", 0.05, 2.0)), (128, 12, ("grf", 1e-3, 2.0, 5)), (64, 16, ("grf", 2e-3, 1.0, 6)),
             (192, 8, ("sine", 0.02, 1.0))]
    problems, ins, meds, refs = [], [], [], []
    for Np, npoles, med in specs:
        wl = workload(N=Np, W=Np // 8, npoles=npoles, medium=med, w0=Np * 0.25 / 8, tol=1e-12)
        f = wl["fit"]
        problems.append(dict(nx=Np, ny=Np, dx=0.25, dy=0.25, k0=2 * np.pi, n0=1.0, dz=1.0, ncomp=1,
                             poles=f["poles"], residues=f["residues"], r_inf=f["r_inf"], d2=wl["c"], d1=wl["d"],
                             edge_width=Np // 8, edge_eta=0.25, tol=1e-12))
        ins.append(to_gpu(wl["w"]))
        meds.append(to_gpu(wl["n2"]))
        g = oracle_grid(wl)
        co = op.coefficients(g, wl["n2"], False)
        ref, _ = st.step(g, co, wl["w"], oracle_pf(wl), 1.0, 1e-12)
        refs.append(ref)
    b = hp.Batch(problems, nworkers=3)
    outs = b.propagate(ins, meds, [1] * len(specs))
    torch.cuda.synchronize()
    for (Np, npoles, med), o, ref in zip(specs, outs, refs):
        err = rel_l2(o.cpu().numpy(), ref)
        print(f"{Np}^2, {npoles} poles, {med[0]}: relative L2 vs oracle {err:.3e}")
        assert err < 1e-9, (Np, npoles, err)
    b.close()
