"""The C ABI: the library loads, exports what include/hp.h declares, and its
host-side validation answers without touching a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2410_17446_amd import hp, unet

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions(header=None):
    names = set()
    for h in ([header] if header else sorted(os.listdir(os.path.join(ROOT, "include")))):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(hp_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_binding_symbols():
    assert declared_functions("hp.h") == sorted(hp.SYMBOLS)
    assert declared_functions("hp_unet.h") == sorted(unet.SYMBOLS)
    assert declared_functions() == sorted(hp.SYMBOLS + unet.SYMBOLS)


@pytest.mark.parametrize("args", [(0, 32, 7, 2), (7, 32, 7, 2), (4, 0, 7, 2), (4, 300, 7, 2), (4, 32, 0, 2),
                                  (4, 32, 7, 65)])
def test_unet_create_rejects_bad_sizes_on_the_host(args):
    L = unet.lib()
    h = C.c_void_p()
    assert L.hp_unet_create(*args, 0, None, C.byref(h)) == -1
    assert h.value is None
    assert b"levels" in L.hp_unet_last_error(None)


def test_library_exports_every_declared_symbol():
    lib = hp.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def _desc(**kw):
    poles = (hp.hp_c128 * 2)(hp.hp_c128(-1.0, -0.1), hp.hp_c128(-2.0, -0.5))
    res = (hp.hp_c128 * 2)(hp.hp_c128(0.1, 0.0), hp.hp_c128(0.2, 0.0))
    d2 = (C.c_double * 7)(-3.2, 1.9, -0.41, 0.14, -0.055, 0.0175, -0.003)
    d1 = (C.c_double * 6)(0.93, -0.38, 0.17, -0.074, 0.025, -0.0046)
    args = dict(nx=64, ny=64, dx=0.25, dy=0.25, k0=2 * np.pi, n0=1.0, dz=1.0, ncomp=1, npoles=2,
                poles=poles, residues=res, r_inf=hp.hp_c128(0.0, 0.0), d2=d2, d1=d1, edge_width=8,
                edge_eta=0.25, tol=1e-10, restart=30, max_cycles=20, precision=0)
    args.update(kw)
    d = hp.hp_plan_desc(**args)
    d._keep = (poles, res, d2, d1)
    return d


def test_workspace_bytes_scales_with_problem():
    L = hp.lib()
    a = L.hp_workspace_bytes(C.byref(_desc()))
    b = L.hp_workspace_bytes(C.byref(_desc(nx=128, ny=128)))
    c = L.hp_workspace_bytes(C.byref(_desc(precision=1)))
    assert a > 0 and b > 3 * a and c < a


@pytest.mark.parametrize("bad", [dict(nx=100), dict(nx=32), dict(ncomp=3), dict(edge_width=5),
                                 dict(tol=0.0), dict(restart=0), dict(restart=65), dict(npoles=0),
                                 dict(precision=7), dict(dz=-1.0), dict(nx=4096, ny=4096),
                                 dict(edge_width=30)])
def test_invalid_descriptors_are_rejected_on_the_host(bad):
    L = hp.lib()
    d = _desc(**bad)
    assert L.hp_workspace_bytes(C.byref(d)) == 0
    out = C.c_void_p()
    rc = L.hp_plan_create(C.byref(d), None, None, C.byref(out))
    assert rc == -1 and not out.value
    assert L.hp_last_error(None)


def test_null_arguments():
    """Every entry point that takes a plan rejects a NULL plan with HP_EINVAL (-1) on the host,
    before any device work, and records a thread-local message."""
    L = hp.lib()
    assert L.hp_plan_create(None, None, None, None) == -1
    assert L.hp_step(None, None, None, None) == -1
    assert L.hp_set_medium(None, None) == -1
    assert L.hp_propagate(None, None, None, 0, 1, None) == -1
    assert L.hp_solve(None, 0, None, None) == -1
    assert L.hp_step_guess(None, None, None, None, None, None) == -1
    assert L.hp_set_guess(None, 0) == -1
    assert L.hp_autotune(None, None, None, 1, None, None) == -1
    assert L.hp_set_launch(None, 1) == -1
    assert L.hp_batch_set_launch(None, None) == -1
    assert L.hp_set_form(None, 1, 8) == -1
    assert L.hp_get_solution(None, 0, None) == -1
    assert L.hp_apply_medium(None, None, None) == -1
    assert L.hp_get_stats(None, None, None) == -1
    assert L.hp_set_fixed_iters(None, None) == -1
    assert L.hp_apply_operator(None, 0, None, None) == -1
    assert L.hp_apply_preconditioner(None, 0, None, None) == -1
    assert L.hp_profile(None, 0) == -1
    assert L.hp_profile_sample(None, 1) == -1
    assert L.hp_profile_read(None, None, None, None) == -1
    assert L.hp_profile_totals(None, None, None) == -1
    assert L.hp_set_pml(None, 1.0, None, None, None) == -1
    assert b"NULL" in L.hp_last_error(None)
    L.hp_plan_destroy(None)


def test_pole_on_the_free_space_spectrum_is_rejected_on_the_host():
    """A pole equal to an eigenvalue mu_p + mu_q of the free-space operator makes the preconditioner
    singular; hp_plan_create rejects it with HP_EINVAL before allocating anything.  The eigenvalue
    is formed as the library documents it: mu_q = s [c0 + 2 sum_m c_m cos(m pi q / n)] / h^2,
    s = 1/(k0 n0)^2, summed in that order."""
    import math
    L = hp.lib()
    d0 = _desc()
    c = [d0.d2[i] for i in range(7)]
    n, h, s = 64, 0.25, 1.0 / (2 * np.pi) ** 2

    def mu(q):
        sym = c[0]
        for m in range(1, 7):
            sym += 2.0 * c[m] * math.cos(m * math.pi * q / n)
        return s * sym / (h * h)

    lam = mu(3) + mu(5)
    poles = (hp.hp_c128 * 2)(hp.hp_c128(-1.0, -0.1), hp.hp_c128(lam, 0.0))
    d = _desc(poles=poles)
    d._keep = d._keep + (poles,)
    out = C.c_void_p()
    assert L.hp_plan_create(C.byref(d), None, None, C.byref(out)) == -1 and not out.value
    assert b"spectrum" in L.hp_last_error(None)


def test_device_fit_validates_on_the_host():
    """hp_fit_exp_sqrt rejects bad arguments before touching a GPU, with a message."""
    L = hp.lib()
    P = (hp.hp_c128 * 8)()
    R = (hp.hp_c128 * 8)()
    r = hp.hp_c128()
    assert L.hp_fit_exp_sqrt(0.0, 8, 40, None, P, R, C.byref(r), None) == -1
    assert b"K must be" in L.hp_last_error(None)
    assert L.hp_fit_exp_sqrt(6.28, 32, 40, None, P, R, C.byref(r), None) == -1
    assert b"degree" in L.hp_last_error(None)
    assert L.hp_fit_exp_sqrt(6.28, 8, 40, None, None, R, C.byref(r), None) == -1
