"""hp_apply_preconditioner_noalloc (the entry point for callers that cannot allocate) against
hp_apply_preconditioner, through the C ABI: the same solve, in every precision, on two calls in a
row whose second is smaller (the static scratch keeps the first call's contents), and a field
beyond the static array is rejected on the host."""
import ctypes as C

import numpy as np
import pytest

from paper_2410_17446_amd import hp, inputs

from helpers import gpu_plan, rel_l2, to_gpu, workload

pytestmark = pytest.mark.gpu


def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _pair(plan, pole, x):
    """(existing entry point's y, no-alloc entry point's y) for one input."""
    import torch
    L = hp.lib()
    ref = torch.zeros_like(x)
    out = torch.full_like(x, complex(np.nan, np.nan))
    assert L.hp_apply_preconditioner(plan.handle, pole, C.c_void_p(x.data_ptr()), C.c_void_p(ref.data_ptr())) == 0
    rc = L.hp_apply_preconditioner_noalloc(plan.handle, pole, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()))
    assert rc == 0, L.hp_last_error(plan.handle)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_noalloc_preconditioner_matches_the_allocating_one(precision):
    """Same kernels, same arithmetic: the two entry points agree to rounding (1e-13 relative L2 in
    FP64, 1e-6 in the mixed modes; in practice bit for bit).  Call 1: 1024^2 scalar (the largest
    scalar field the array takes); call 2: 256^2 vector, smaller, right after it."""
    _cuda()
    bar = 1e-13 if precision == 0 else 1e-6
    cases = [(1024, 1, 128, 16, 3), (256, 2, 32, 8, 5)]
    for N, ncomp, W, npoles, pole in cases:
        wl = workload(N=N, ncomp=ncomp, W=W, npoles=npoles, medium=("sine", 0.02, 1.0), w0=N * 0.25 / 8)
        plan = gpu_plan(wl, precision=precision, restart=1)
        x = to_gpu(inputs.random_field(N, ncomp, seed=N + ncomp))
        for p in (pole, -1):
            ref, out = _pair(plan, p, x)
            err = rel_l2(out, ref)
            print(f"precision {precision}, {N}^2 x {ncomp}, pole {p}: relative L2 {err:.3e}")
            assert np.isfinite(out).all() and err <= bar, (N, ncomp, p, err)
            assert np.all(out[:, 0, :] == 0) and np.all(out[:, :, 0] == 0)
        plan.close()


def test_noalloc_rejects_a_field_beyond_the_static_array():
    """A 1024^2 vector field in FP64 needs three 32 MiB intermediate fields, beyond the array's
    48 MiB: HP_EINVAL on the host, nothing launched, the output untouched."""
    torch = _cuda()
    wl = workload(N=1024, ncomp=2, W=128, npoles=8, medium=("sine", 0.02, 1.0), w0=32.0)
    plan = gpu_plan(wl, restart=1)
    x = to_gpu(inputs.random_field(1024, 2, seed=1))
    y = torch.zeros_like(x)
    L = hp.lib()
    rc = L.hp_apply_preconditioner_noalloc(plan.handle, 0, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()))
    assert rc == -1 and b"static scratch" in L.hp_last_error(plan.handle)
    torch.cuda.synchronize()
    assert float(y.abs().max()) == 0.0
    plan.close()
