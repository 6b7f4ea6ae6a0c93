"""Thin ctypes binding of libhp.so (include/hp.h).

Argument marshalling only: every step of a propagation runs in the HIP
kernels of the library.  Fields are torch tensors on the GPU (complex128,
shape (ncomp, ny, nx); n^2 float64, shape (ny, nx)); PyTorch provides the
device memory and the stream.  There is no CPU fallback: if the library is not
built, loading it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhp.so")
_lib = None

HP_OK, HP_WARN_NOCONV, HP_WARN_UNSTABLE = 0, 1, 2
HP_FP64, HP_MIXED, HP_MIXED64 = 0, 1, 2
HP_GUESS_ZERO, HP_GUESS_PREV, HP_GUESS_LEARNED = 0, 1, 2
HP_FORM_EXP, HP_FORM_SQRT = 0, 1

SYMBOLS = ("hp_workspace_bytes", "hp_plan_create", "hp_set_medium", "hp_step", "hp_solve", "hp_propagate",
           "hp_step_guess", "hp_set_guess", "hp_autotune", "hp_set_launch", "hp_batch_set_launch", "hp_set_form", "hp_set_pml", "hp_fit_exp_sqrt", "hp_get_solution", "hp_apply_medium", "hp_get_stats",
           "hp_set_fixed_iters", "hp_apply_operator", "hp_apply_preconditioner",
           "hp_apply_preconditioner_noalloc",
           "hp_profile", "hp_profile_read", "hp_profile_sample", "hp_profile_totals", "hp_last_error",
           "hp_plan_destroy",
           "hp_batch_create", "hp_batch_propagate", "hp_batch_stats", "hp_batch_destroy")
KERNEL_CLASSES = ("row_fwd", "col", "row_apply", "update", "small", "final", "residual", "guess", "pml_gemm")


class hp_c128(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class hp_plan_desc(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("dx", C.c_double), ("dy", C.c_double),
                ("k0", C.c_double), ("n0", C.c_double), ("dz", C.c_double), ("ncomp", C.c_int),
                ("npoles", C.c_int), ("poles", C.POINTER(hp_c128)), ("residues", C.POINTER(hp_c128)),
                ("r_inf", hp_c128), ("d2", C.POINTER(C.c_double)), ("d1", C.POINTER(C.c_double)),
                ("edge_width", C.c_int), ("edge_eta", C.c_double), ("tol", C.c_double),
                ("restart", C.c_int), ("max_cycles", C.c_int), ("precision", C.c_int)]


class HPError(RuntimeError):
    pass


def lib():
    """Load libhp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise HPError(f"{_LIB_PATH} is missing: build it with python -m paper_2410_17446_amd.build")
        L = C.CDLL(_LIB_PATH)
        vp, ip, dp = C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double)
        L.hp_workspace_bytes.argtypes = [C.POINTER(hp_plan_desc)]
        L.hp_workspace_bytes.restype = C.c_size_t
        L.hp_plan_create.argtypes = [C.POINTER(hp_plan_desc), vp, vp, C.POINTER(vp)]
        L.hp_set_medium.argtypes = [vp, vp]
        L.hp_step.argtypes = [vp, vp, vp, vp]
        L.hp_propagate.argtypes = [vp, vp, vp, C.c_long, C.c_int, vp]
        L.hp_solve.argtypes = [vp, C.c_int, vp, vp]
        L.hp_step_guess.argtypes = [vp, vp, vp, C.POINTER(vp), ip, vp]
        L.hp_set_guess.argtypes = [vp, C.c_int]
        L.hp_autotune.argtypes = [vp, vp, vp, C.c_int, vp, ip]
        L.hp_set_launch.argtypes = [vp, C.c_int]
        L.hp_batch_set_launch.argtypes = [vp, ip]
        L.hp_set_pml.argtypes = [vp, C.c_double, vp, vp, vp]
        L.hp_fit_exp_sqrt.argtypes = [C.c_double, C.c_int, C.c_int, vp, C.POINTER(hp_c128), C.POINTER(hp_c128),
                                      C.POINTER(hp_c128), dp]
        L.hp_get_solution.argtypes = [vp, C.c_int, vp]
        L.hp_apply_medium.argtypes = [vp, vp, vp]
        L.hp_get_stats.argtypes = [vp, ip, dp]
        L.hp_set_fixed_iters.argtypes = [vp, ip]
        L.hp_apply_operator.argtypes = [vp, C.c_int, vp, vp]
        L.hp_apply_preconditioner.argtypes = [vp, C.c_int, vp, vp]
        L.hp_apply_preconditioner_noalloc.argtypes = [vp, C.c_int, vp, vp]
        L.hp_profile.argtypes = [vp, C.c_int]
        L.hp_profile_read.argtypes = [vp, C.POINTER(C.c_long), dp, dp]
        L.hp_profile_sample.argtypes = [vp, C.c_int]
        L.hp_profile_totals.argtypes = [vp, C.POINTER(C.c_long), dp]
        L.hp_last_error.argtypes = [vp]
        L.hp_last_error.restype = C.c_char_p
        L.hp_plan_destroy.argtypes = [vp]
        L.hp_batch_create.argtypes = [C.POINTER(hp_plan_desc), C.c_int, C.c_int, C.POINTER(vp)]
        L.hp_batch_propagate.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), ip, C.POINTER(vp)]
        L.hp_batch_stats.argtypes = [vp, C.POINTER(C.c_long), dp]
        L.hp_batch_destroy.argtypes = [vp]
        for name in SYMBOLS:
            if name not in ("hp_workspace_bytes", "hp_last_error", "hp_plan_destroy", "hp_batch_destroy"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _ptr(t) -> int | None:
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise HPError("expected a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise HPError("tensor must be contiguous")
    return t.data_ptr()


def fit_exp_sqrt(K, degree, lawson_steps=40, stream=None):
    """The rational fit of exp(iK sqrt(1+z)) computed on the GPU (hp_fit_exp_sqrt): (poles,
    residues, r_inf, max_err) as numpy complex arrays, a complex and a float."""
    L = lib()
    P = (hp_c128 * degree)()
    R = (hp_c128 * degree)()
    r = hp_c128()
    e = C.c_double()
    rc = L.hp_fit_exp_sqrt(float(K), int(degree), int(lawson_steps), stream, P, R, C.byref(r), C.byref(e))
    if rc < 0:
        raise HPError(f"hp_fit_exp_sqrt: {rc}: {L.hp_last_error(None).decode()}")
    return (np.array([complex(x.re, x.im) for x in P]), np.array([complex(x.re, x.im) for x in R]),
            complex(r.re, r.im), float(e.value))


class Plan:
    """A propagation plan (hp_plan_create).  poles/residues: complex arrays; d2 (7) and d1 (6):
    the 13-point stencil coefficients; the rest as in hp_plan_desc."""

    def __init__(self, nx, ny, dx, dy, k0, n0, dz, ncomp, poles, residues, r_inf, d2, d1,
                 edge_width, edge_eta, tol, restart=30, max_cycles=20, precision=HP_FP64,
                 stream=None, workspace=None):
        import torch
        self.L = lib()
        poles = np.asarray(poles, dtype=np.complex128)
        residues = np.asarray(residues, dtype=np.complex128)
        self._poles = (hp_c128 * len(poles))(*[hp_c128(p.real, p.imag) for p in poles])
        self._res = (hp_c128 * len(residues))(*[hp_c128(a.real, a.imag) for a in residues])
        self._d2 = (C.c_double * 7)(*np.asarray(d2, dtype=float))
        self._d1 = (C.c_double * 6)(*np.asarray(d1, dtype=float))
        r_inf = complex(r_inf)
        self.desc = hp_plan_desc(nx, ny, dx, dy, k0, n0, dz, ncomp, len(poles), self._poles, self._res,
                                 hp_c128(r_inf.real, r_inf.imag), self._d2, self._d1, edge_width, edge_eta,
                                 tol, restart, max_cycles, precision)
        self.shape = (ncomp, ny, nx)
        self.npoles = len(poles)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        self.handle = C.c_void_p()
        ws = _ptr(workspace) if workspace is not None else None
        rc = self.L.hp_plan_create(C.byref(self.desc), C.c_void_p(stream), C.c_void_p(ws), C.byref(self.handle))
        if rc < 0:
            raise HPError(f"hp_plan_create: {rc}: {self.L.hp_last_error(None).decode()}")
        self.create_status = rc

    def _check(self, rc, what):
        if rc < 0:
            raise HPError(f"{what}: {rc}: {self.L.hp_last_error(self.handle).decode()}")
        return rc

    def set_medium(self, n2):
        return self._check(self.L.hp_set_medium(self.handle, _ptr(n2)), "hp_set_medium")

    def step(self, E_in, n2=None, E_out=None):
        import torch
        if E_out is None:
            E_out = torch.empty_like(E_in)
        self.last_status = self._check(self.L.hp_step(self.handle, _ptr(E_in), _ptr(n2), _ptr(E_out)), "hp_step")
        return E_out

    def propagate(self, E_in, nsteps, n2=None, n2_step_stride=0, E_out=None):
        import torch
        if E_out is None:
            E_out = torch.empty_like(E_in)
        rc = self.L.hp_propagate(self.handle, _ptr(E_in), _ptr(n2), n2_step_stride, nsteps, _ptr(E_out))
        self.last_status = self._check(rc, "hp_propagate")
        return E_out

    def solve(self, pole, rhs, x=None):
        import torch
        if x is None:
            x = torch.empty_like(rhs)
        self.last_status = self._check(self.L.hp_solve(self.handle, pole, _ptr(rhs), _ptr(x)), "hp_solve")
        return x

    def step_guess(self, E_in, x0, n2=None, E_out=None):
        """One step with per-pole initial guesses x0 (list of tensors or None); returns
        (E_out, accepted flags)."""
        import torch
        if E_out is None:
            E_out = torch.empty_like(E_in)
        vp = C.c_void_p
        arr = None
        if x0 is not None:
            if len(x0) != self.npoles:
                raise HPError("x0 needs one entry per pole")
            arr = (vp * self.npoles)(*[vp(_ptr(g)) if g is not None else vp() for g in x0])
        acc = (C.c_int * self.npoles)()
        rc = self.L.hp_step_guess(self.handle, _ptr(E_in), _ptr(n2), arr, acc, _ptr(E_out))
        self._check(rc, "hp_step_guess")
        return E_out, list(acc)

    def autotune(self, E_in, n2=None, reps=3, E_out=None):
        """Time the column-pass variants on steps from E_in, keep the fastest; returns
        (E_out, variant)."""
        import torch
        if E_out is None:
            E_out = torch.empty_like(E_in)
        v = C.c_int(-1)
        rc = self.L.hp_autotune(self.handle, _ptr(E_in), _ptr(n2), int(reps), _ptr(E_out), C.byref(v))
        self._check(rc, "hp_autotune")
        return E_out, v.value

    def set_launch(self, col_variant):
        return self._check(self.L.hp_set_launch(self.handle, int(col_variant)), "hp_set_launch")

    def set_guess(self, mode):
        return self._check(self.L.hp_set_guess(self.handle, int(mode)), "hp_set_guess")

    def set_guess_net(self, net, chunk=8):
        """Attach a trained UNet for HP_GUESS_LEARNED (None detaches); the plan keeps a reference."""
        from . import unet as un
        L = un.lib()
        self._net = net
        rc = L.hp_set_guess_net(self.handle, net.handle if net is not None else None, int(chunk))
        return self._check(rc, "hp_set_guess_net")

    def set_form(self, form, substeps=1):
        """HP_FORM_EXP or HP_FORM_SQRT (pseudo-differential form, `substeps` RK4 substeps per
        step); returns HP_OK or HP_WARN_UNSTABLE."""
        return self._check(self.L.hp_set_form(self.handle, int(form), int(substeps)), "hp_set_form")

    def set_pml(self, sigma_max, Q=None, Qinv=None, lam=None):
        """Absorbing layers on the plan's edge_width cells (hp_set_pml): Q, Qinv (N-1, N-1) and lam
        (N-1,) the eigen-decomposition of the one-axis stretched operator (tables.pml_eigen); all
        None with sigma_max = 0 removes them."""
        if Q is None:
            return self._check(self.L.hp_set_pml(self.handle, float(sigma_max), None, None, None), "hp_set_pml")
        arrs = [np.ascontiguousarray(a, dtype=np.complex128) for a in (Q, Qinv, lam)]
        return self._check(self.L.hp_set_pml(self.handle, float(sigma_max), *(a.ctypes.data for a in arrs)),
                           "hp_set_pml")

    def solution(self, pole, x=None):
        import torch
        if x is None:
            x = torch.empty(self.shape, dtype=torch.complex128, device="cuda")
        self._check(self.L.hp_get_solution(self.handle, pole, _ptr(x)), "hp_get_solution")
        return x

    def apply_medium(self, x, y):
        return self._check(self.L.hp_apply_medium(self.handle, _ptr(x), _ptr(y)), "hp_apply_medium")

    def stats(self):
        it = (C.c_int * self.npoles)()
        rr = (C.c_double * self.npoles)()
        self._check(self.L.hp_get_stats(self.handle, it, rr), "hp_get_stats")
        return list(it), list(rr)

    def set_fixed_iters(self, iters):
        arr = None if iters is None else (C.c_int * self.npoles)(*iters)
        return self._check(self.L.hp_set_fixed_iters(self.handle, arr), "hp_set_fixed_iters")

    def apply_operator(self, pole, x, y):
        return self._check(self.L.hp_apply_operator(self.handle, pole, _ptr(x), _ptr(y)), "hp_apply_operator")

    def apply_preconditioner(self, pole, x, y):
        return self._check(self.L.hp_apply_preconditioner(self.handle, pole, _ptr(x), _ptr(y)),
                           "hp_apply_preconditioner")

    def profile(self, enable: bool, classes=None):
        """Time the launches of the given kernel classes (names of KERNEL_CLASSES; all when None)."""
        mask = 0
        if enable:
            mask = -1 if classes is None else sum(1 << KERNEL_CLASSES.index(c) for c in classes)
        return self._check(self.L.hp_profile(self.handle, mask), "hp_profile")

    def profile_sample(self, period):
        """Time every period-th launch of each timed class (1 = all)."""
        return self._check(self.L.hp_profile_sample(self.handle, int(period)), "hp_profile_sample")

    def profile_read(self):
        """{kernel class: (launches, total ms, total algorithmic bytes)}."""
        n = len(KERNEL_CLASSES)
        la, ms, by = (C.c_long * n)(), (C.c_double * n)(), (C.c_double * n)()
        self._check(self.L.hp_profile_read(self.handle, la, ms, by), "hp_profile_read")
        return {k: (la[i], ms[i], by[i]) for i, k in enumerate(KERNEL_CLASSES)}

    def profile_totals(self):
        """{kernel class: (launches, algorithmic bytes)} over every launch of the enabled classes
        since profile(True), timed or not."""
        n = len(KERNEL_CLASSES)
        la, by = (C.c_long * n)(), (C.c_double * n)()
        self._check(self.L.hp_profile_totals(self.handle, la, by), "hp_profile_totals")
        return {k: (la[i], by[i]) for i, k in enumerate(KERNEL_CLASSES)}

    def workspace_bytes(self):
        return self.L.hp_workspace_bytes(C.byref(self.desc))

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            self.L.hp_plan_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_desc(nx, ny, dx, dy, k0, n0, dz, ncomp, poles, residues, r_inf, d2, d1, edge_width, edge_eta, tol,
              restart=30, max_cycles=20, precision=HP_FP64):
    """An hp_plan_desc plus the ctypes arrays it points to (keep both alive)."""
    poles = np.asarray(poles, dtype=np.complex128)
    residues = np.asarray(residues, dtype=np.complex128)
    keep = ((hp_c128 * len(poles))(*[hp_c128(p.real, p.imag) for p in poles]),
            (hp_c128 * len(residues))(*[hp_c128(a.real, a.imag) for a in residues]),
            (C.c_double * 7)(*np.asarray(d2, dtype=float)),
            (C.c_double * 6)(*np.asarray(d1, dtype=float)))
    r_inf = complex(r_inf)
    d = hp_plan_desc(nx, ny, dx, dy, k0, n0, dz, ncomp, len(poles), keep[0], keep[1],
                     hp_c128(r_inf.real, r_inf.imag), keep[2], keep[3], edge_width, edge_eta, tol, restart,
                     max_cycles, precision)
    return d, keep


class Batch:
    """Independent propagations run concurrently by the library (hp_batch_*).
    problems: list of dicts with the Plan keyword arguments."""

    def __init__(self, problems, nworkers=8):
        self.L = lib()
        descs, self._keep = [], []
        for pr in problems:
            d, keep = make_desc(**pr)
            descs.append(d)
            self._keep.append(keep)
        self.n = len(descs)
        self._descs = (hp_plan_desc * self.n)(*descs)
        self.handle = C.c_void_p()
        rc = self.L.hp_batch_create(self._descs, self.n, nworkers, C.byref(self.handle))
        if rc < 0:
            raise HPError(f"hp_batch_create: {rc}: {self.L.hp_last_error(None).decode()}")
        self.shapes = [(pr["ncomp"], pr["ny"], pr["nx"]) for pr in problems]

    def set_launch(self, variants):
        """Column-pass launch variant per problem (0, 1 or 2; see Plan.autotune)."""
        if len(variants) != self.n:
            raise HPError("one variant per problem")
        arr = (C.c_int * self.n)(*[int(v) for v in variants])
        rc = self.L.hp_batch_set_launch(self.handle, arr)
        if rc < 0:
            raise HPError(f"hp_batch_set_launch: {rc}: {self.L.hp_last_error(None).decode()}")

    def propagate(self, E_in, n2, nsteps, E_out=None):
        import torch
        if E_out is None:
            E_out = [torch.empty_like(e) for e in E_in]
        vp = C.c_void_p
        a_in = (vp * self.n)(*[vp(_ptr(e)) for e in E_in])
        a_n2 = (vp * self.n)(*[vp(_ptr(m)) for m in n2])
        a_out = (vp * self.n)(*[vp(_ptr(e)) for e in E_out])
        a_st = (C.c_int * self.n)(*nsteps)
        rc = self.L.hp_batch_propagate(self.handle, a_in, a_n2, a_st, a_out)
        if rc < 0:
            raise HPError(f"hp_batch_propagate: {rc}: {self.L.hp_last_error(None).decode()}")
        self.status = rc
        return E_out

    def stats(self):
        it = (C.c_long * self.n)()
        sec = (C.c_double * self.n)()
        self.L.hp_batch_stats(self.handle, it, sec)
        return list(it), list(sec)

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            self.L.hp_batch_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
