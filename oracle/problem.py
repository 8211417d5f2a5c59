"""Run a seeded workload (``workloads.Workload``) through the O2 oracle."""
from __future__ import annotations

import numpy as np

from . import reactions
from .separable import SeparableScheme


def scheme(wl, alpha=None, kappa=None, scheme_name=None, periodic_basis="lapack"):
    return SeparableScheme(wl.bc, wl.shape, wl.h,
                           wl.alpha if alpha is None else alpha,
                           wl.kappa if kappa is None else kappa,
                           wl.dt, wl.scheme if scheme_name is None else scheme_name,
                           periodic_basis)


def nonlinearity(wl, params=None):
    p = wl.params if params is None else params
    return lambda U, t: reactions.f(wl.reaction, p, U, t)


def run(wl, U0, nsteps=None, t0=0.0, **kw):
    """FP64 fields after ``nsteps`` steps of eq. ETDRK4P13."""
    sch = scheme(wl, **kw)
    n = wl.nsteps if nsteps is None else nsteps
    return sch.integrate(U0, n, nonlinearity(wl), t0)


def gradients(wl, U0, nsteps, grad_uT, t0=0.0, **kw):
    """Discrete adjoint: d<grad_uT, u_T>/d(u0, kappa, alpha, params)."""
    sch = scheme(wl, **kw)
    kind, p = wl.reaction, wl.params
    jacT = lambda U, G, t: reactions.jacT(kind, p, U, G)
    dpar = lambda U, G, t: reactions.dparams(kind, p, U, G)
    return sch.gradients(U0, nsteps, nonlinearity(wl), jacT, dpar, grad_uT, t0,
                         nparams=reactions.nparams(kind, wl.nspecies))


def rel_err(x, ref):
    """max over species of ||x - ref||_inf / ||ref||_inf."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    out = 0.0
    for s in range(ref.shape[0]):
        den = np.max(np.abs(ref[s]))
        num = np.max(np.abs(x[s] - ref[s]))
        out = max(out, num / den if den > 0 else num)
    return out
