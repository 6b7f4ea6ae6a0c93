"""Failure modes of a step, through the C ABI: a solve that cannot converge within its cycles, a
medium with a NaN (or n^2 <= 0 where the vector operator takes ln n^2), a right-hand side with a
NaN, and the plan-time stability report of an exponential table.  Every case ends normally on
the device: a pole that meets a non-finite value stops itself and the host reports it."""
import numpy as np
import pytest

from oracle import operator as op
from oracle import step as st

from helpers import gpu_plan, oracle_grid, oracle_pf, rel_l2, to_gpu, workload

pytestmark = pytest.mark.gpu


def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_max_cycles_one_warns_and_writes_the_cycle_iterate():
    """GMRES(2) with one cycle cannot reach tol 1e-10 in the 5 % sine medium: the step returns
    HP_WARN_NOCONV and writes the step built from each pole's one-cycle iterate, which equals the
    oracle's step with the same schedule (one cycle of two Arnoldi steps per pole)."""
    _cuda()
    from paper_2410_17446_amd import hp
    wl = workload(N=64, W=8, tol=1e-10)
    g = oracle_grid(wl)
    co = op.coefficients(g, wl["n2"], False)
    K = len(wl["fit"]["poles"])
    _, free = st.step(g, co, wl["w"], oracle_pf(wl), 1.0, 1e-10)
    assert min(free.iters) > 2                      # no pole converges within two steps
    ref, stats = st.step(g, co, wl["w"], oracle_pf(wl), 1.0, 1e-10, restart=2, schedules=[[2]] * K)
    assert max(stats.relres) > 1e-10
    plan = hp.Plan(nx=64, ny=64, dx=0.25, dy=0.25, k0=2 * np.pi, n0=1.0, dz=1.0, ncomp=1,
                   poles=wl["fit"]["poles"], residues=wl["fit"]["residues"], r_inf=wl["fit"]["r_inf"],
                   d2=wl["c"], d1=wl["d"], edge_width=8, edge_eta=0.25, tol=1e-10, restart=2, max_cycles=1)
    out = plan.step(to_gpu(wl["w"]), to_gpu(wl["n2"]))
    assert plan.last_status == hp.HP_WARN_NOCONV
    it, rr = plan.stats()
    assert it == [2] * K
    assert max(rr) > 1e-10
    assert rel_l2(out.cpu().numpy(), ref) < 1e-10
    plan.close()


@pytest.mark.parametrize("ncomp,bad", [(1, np.nan), (2, np.nan), (2, -1.0), (1, np.inf)])
def test_non_finite_medium_is_reported_and_the_plan_recovers(ncomp, bad):
    """A NaN or Inf in n^2 (or n^2 <= 0, whose ln the vector operator takes) at one interior node
    reaches every pole's Krylov space; each pole stops itself and hp_step returns HP_EINVAL with a
    message.  The same plan then steps a valid medium exactly as a fresh plan does."""
    torch = _cuda()
    from paper_2410_17446_amd import hp
    wl = workload(N=64, ncomp=ncomp, W=8, tol=1e-10)
    n2 = wl["n2"].copy()
    n2[32, 30] = bad
    plan = gpu_plan(wl)
    with pytest.raises(hp.HPError, match="NaN or Inf"):
        plan.step(to_gpu(wl["w"]), to_gpu(n2))
    out = plan.step(to_gpu(wl["w"]), to_gpu(wl["n2"])).cpu().numpy()
    fresh = gpu_plan(wl)
    ref = fresh.step(to_gpu(wl["w"]), to_gpu(wl["n2"])).cpu().numpy()
    assert np.array_equal(out, ref)
    plan.close()
    fresh.close()


def test_non_finite_field_is_reported():
    torch = _cuda()
    from paper_2410_17446_amd import hp
    wl = workload(N=64, W=8, tol=1e-10)
    w = wl["w"].copy()
    w[0, 20, 20] = np.nan
    plan = gpu_plan(wl, precision=hp.HP_MIXED)
    with pytest.raises(hp.HPError, match="NaN or Inf"):
        plan.step(to_gpu(w), to_gpu(wl["n2"]))
    plan.close()


def test_unstable_table_is_reported_at_plan_creation():
    """hp_plan_create measures max |r| over the free-space spectrum's interval: the 16-pole AAA
    fit of exp(2 pi i sqrt(1+z)) exceeds 1 next to the branch point (about 1.019), so the plan is
    created with HP_WARN_UNSTABLE; the same table with its residues and r_inf halved stays below 1
    and gives HP_OK."""
    _cuda()
    from paper_2410_17446_amd import hp
    wl = workload(N=128, W=16, npoles=16)
    f = wl["fit"]
    z = np.linspace(-6.8, 0.1, 200001)
    r = f["r_inf"] + (1.0 / (z[:, None] - f["poles"][None, :])) @ f["residues"]
    assert np.abs(r).max() > 1 + 1e-6
    plan = gpu_plan(wl)
    assert plan.create_status == hp.HP_WARN_UNSTABLE
    plan.close()
    half = dict(wl, fit=dict(poles=f["poles"], residues=0.5 * f["residues"], r_inf=0.5 * f["r_inf"]))
    plan = gpu_plan(half)
    assert plan.create_status == hp.HP_OK
    plan.close()
