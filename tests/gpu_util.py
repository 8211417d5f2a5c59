"""Helpers for GPU tests: run a workload through libsfrde via torch tensors."""
import numpy as np
import torch

from paper_2003_13569_amd.torch_api import Plan

TD = {"f32": torch.float32, "f64": torch.float64}


def plan_for(wl, dtype, scheme=None, alpha=None, kappa=None, params=None):
    return Plan(wl.shape, wl.bc, wl.h, wl.alpha if alpha is None else alpha,
                wl.kappa if kappa is None else kappa, wl.dt, wl.reaction,
                wl.params if params is None else params, dtype,
                wl.scheme if scheme is None else scheme)


def run(wl, u0, nsteps, dtype, scheme=None, plan=None, t0=0.0):
    p = plan or plan_for(wl, dtype, scheme)
    u = torch.tensor(np.asarray(u0), dtype=TD[dtype], device="cuda")
    p.integrate(u, nsteps, t0)
    torch.cuda.synchronize()
    out = u.double().cpu().numpy()
    if plan is None:
        p.close()
    return out
