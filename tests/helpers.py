"""Shared set-up of the parity tests: one workload, the oracle on one side and
the HIP library on the other, fed the same inputs (fields, medium, pole table,
stencils).  Tables come from the oracle; nothing flows from the GPU side into
the oracle."""
from __future__ import annotations

import numpy as np

from oracle import fit, stencil
from oracle import operator as op
from oracle import step as st
from paper_2410_17446_amd import inputs

K0 = inputs.K0


def workload(N=64, ncomp=1, W=8, eta=0.25, npoles=8, dz=1.0, medium=("sine", 0.05, 2.0), w0=4.0,
             dx=0.25, tol=1e-10, restart=30, ny=None):
    ny = ny or N
    c, d = stencil.stencils()
    f = fit.fit_exp_sqrt(K0 * dz, npoles)
    cfg = dict(N=N, dx=dx, ncomp=ncomp, W=W, eta_max=eta, dz=dz, npoles=npoles, tol=tol,
               restart=restart, medium=medium, w0=w0)
    if ny == N:
        n2 = inputs.medium_n2(cfg) if medium[0] != "uniform" else np.ones((N, N))
        w = inputs.beam(cfg)
    else:
        n2 = np.ones((ny, N))
        xs, ys = inputs.coords(N, dx), inputs.coords(ny, dx)
        X, Y = np.meshgrid(xs, ys)
        n2 = (1 + medium[1] * np.sin(2 * np.pi * X / medium[2]) * np.sin(2 * np.pi * Y / medium[2])) ** 2
        w = np.zeros((ncomp, ny, N), dtype=complex)
        w[0] = np.exp(-(X ** 2 + Y ** 2) / w0 ** 2)
        w[:, 0, :] = 0
        w[:, :, 0] = 0
    return dict(cfg=cfg, c=c, d=d, fit=f, n2=n2, w=w, ny=ny, nx=N)


def oracle_grid(wl):
    cfg = wl["cfg"]
    assert wl["nx"] == wl["ny"], "the oracle grid is square"
    return op.Grid(N=cfg["N"], dx=cfg["dx"], dy=cfg["dx"], k0=K0, n0=1.0, c=wl["c"], d=wl["d"],
                   W=cfg["W"], eta_max=cfg["eta_max"])


def oracle_pf(wl):
    f = wl["fit"]
    return st.PFTable(f["poles"], f["residues"], f["r_inf"])


def gpu_plan(wl, precision=0, tol=None, restart=None):
    from paper_2410_17446_amd import hp
    cfg, f = wl["cfg"], wl["fit"]
    return hp.Plan(nx=wl["nx"], ny=wl["ny"], dx=cfg["dx"], dy=cfg["dx"], k0=K0, n0=1.0, dz=cfg["dz"],
                   ncomp=cfg["ncomp"], poles=f["poles"], residues=f["residues"], r_inf=f["r_inf"],
                   d2=wl["c"], d1=wl["d"], edge_width=cfg["W"], edge_eta=cfg["eta_max"],
                   tol=tol if tol is not None else cfg["tol"],
                   restart=restart if restart is not None else cfg["restart"], max_cycles=20,
                   precision=precision)


def to_gpu(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
