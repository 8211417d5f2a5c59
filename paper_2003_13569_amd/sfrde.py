"""ctypes binding of libsfrde (include/sfrde.h), with the same entry-point
names. Argument marshalling only: every step of the method runs in the HIP
library. Pointers are integers (device addresses, e.g. ``tensor.data_ptr()``).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsfrde.so")

OK, EINVAL, ENOMEM, EDEVICE, ENONFINITE, EUNSUPPORTED, ESTATE = 0, -1, -2, -3, -4, -5, -6
BC = {"periodic": 0, "dirichlet": 1, "neumann": 2}
DTYPE = {"f32": 0, "f64": 1}
SCHEME = {"p13": 0, "exp": 1}
REACTION = {"linear": 0, "fhn": 1, "gray_scott": 2, "schnakenberg": 3, "gierer_meinhardt": 4,
            "huxley_mms": 5, "fisher_mms": 6}
CKPT_HEADER_BYTES = 256
MAX_PARAMS = 16

EXPORTS = ("sfrde_plan", "sfrde_plan_batch", "sfrde_step", "sfrde_integrate", "sfrde_ckpt_bytes", "sfrde_resume",
           "sfrde_backward", "sfrde_backward_noalloc", "sfrde_destroy", "sfrde_last_error", "sfrde_workspace_bytes",
           "sfrde_axis_eigenvalues", "sfrde_eval_coefficients", "sfrde_profile",
           "sfrde_profile_read", "sfrde_amplification", "sfrde_stability_boundary")
KERNEL_CLASSES = ("X", "Y", "Z", "XADJ", "ZADJ", "OTHER")


class SfrdeError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """Load libsfrde.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first "
                           "(python -m paper_2003_13569_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    pd = ctypes.POINTER(ctypes.c_double)
    L.sfrde_plan.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(i64), i32, pd, i32, pd, pd, d,
                             i32, i32, pd, i32, i32, vp]
    L.sfrde_plan.restype = ctypes.c_int
    L.sfrde_plan_batch.argtypes = [ctypes.POINTER(vp), i32, i32, ctypes.POINTER(i64), i32, pd,
                                   i32, pd, pd, d, i32, i32, pd, i32, i32, vp]
    L.sfrde_plan_batch.restype = ctypes.c_int
    L.sfrde_step.argtypes = [vp, vp, d]
    L.sfrde_step.restype = ctypes.c_int
    L.sfrde_integrate.argtypes = [vp, vp, i64, d, i64, vp]
    L.sfrde_integrate.restype = ctypes.c_int
    L.sfrde_ckpt_bytes.argtypes = [vp, i64, i64]
    L.sfrde_ckpt_bytes.restype = i64
    L.sfrde_resume.argtypes = [vp, vp, i64, vp, i64, d, i64, vp]
    L.sfrde_resume.restype = ctypes.c_int
    L.sfrde_backward.argtypes = [vp, vp, i64, i64, d, vp, vp, pd, pd, pd]
    L.sfrde_backward.restype = ctypes.c_int
    L.sfrde_backward_noalloc.argtypes = [vp, vp, i64, i64, d, vp, vp, pd, pd, pd]
    L.sfrde_backward_noalloc.restype = ctypes.c_int
    L.sfrde_destroy.argtypes = [vp]
    L.sfrde_destroy.restype = ctypes.c_int
    L.sfrde_last_error.argtypes = []
    L.sfrde_last_error.restype = ctypes.c_char_p
    L.sfrde_workspace_bytes.argtypes = [vp]
    L.sfrde_workspace_bytes.restype = i64
    L.sfrde_profile.argtypes = [vp, i32]
    L.sfrde_profile.restype = ctypes.c_int
    L.sfrde_profile_read.argtypes = [vp, pd, ctypes.POINTER(i64)]
    L.sfrde_profile_read.restype = ctypes.c_int
    L.sfrde_axis_eigenvalues.argtypes = [i32, i64, d, pd]
    L.sfrde_axis_eigenvalues.restype = ctypes.c_int
    L.sfrde_eval_coefficients.argtypes = [i32, d, d, i32, pd]
    L.sfrde_eval_coefficients.restype = ctypes.c_int
    L.sfrde_amplification.argtypes = [i32, i64, vp, vp, vp, vp]
    L.sfrde_amplification.restype = ctypes.c_int
    L.sfrde_stability_boundary.argtypes = [i32, i64, vp, i64, vp, vp, vp]
    L.sfrde_stability_boundary.restype = ctypes.c_int
    _lib = L
    return L


def sfrde_last_error() -> str:
    return lib().sfrde_last_error().decode()


def _check(rc: int, where: str) -> int:
    if rc < 0:
        raise SfrdeError(int(rc), where, sfrde_last_error())
    return rc


def _darr(vals):
    vals = list(vals)
    return (ctypes.c_double * max(1, len(vals)))(*vals)


def sfrde_plan(ndim, n, bc, h, nspecies, alpha, kappa, dt, reaction, nparams, params,
               dtype, scheme, hip_stream=0) -> int:
    """Create a plan; returns the handle. n and h are x-first."""
    out = ctypes.c_void_p()
    n_arr = (ctypes.c_int64 * max(1, len(n)))(*[int(v) for v in n])
    rc = lib().sfrde_plan(ctypes.byref(out), int(ndim), n_arr, int(bc), _darr(h), int(nspecies),
                          _darr(alpha), _darr(kappa), float(dt), int(reaction), int(nparams),
                          _darr(params), int(dtype), int(scheme),
                          ctypes.c_void_p(int(hip_stream) if hip_stream else None))
    _check(rc, "sfrde_plan")
    return out.value


def sfrde_plan_batch(batch, ndim, n, bc, h, nspecies, alpha, kappa, dt, reaction, nparams,
                     params, dtype, scheme, hip_stream=0) -> int:
    """Ensemble plan; alpha, kappa are [batch][nspecies] and params [batch][nparams],
    flattened. Returns the handle."""
    out = ctypes.c_void_p()
    n_arr = (ctypes.c_int64 * max(1, len(n)))(*[int(v) for v in n])
    rc = lib().sfrde_plan_batch(ctypes.byref(out), int(batch), int(ndim), n_arr, int(bc),
                                _darr(h), int(nspecies), _darr(alpha), _darr(kappa), float(dt),
                                int(reaction), int(nparams), _darr(params), int(dtype),
                                int(scheme),
                                ctypes.c_void_p(int(hip_stream) if hip_stream else None))
    _check(rc, "sfrde_plan_batch")
    return out.value


def sfrde_step(plan, state, t) -> int:
    return _check(lib().sfrde_step(plan, state, float(t)), "sfrde_step")


def sfrde_integrate(plan, state, nsteps, t0, ckpt_every=0, ckpt=None) -> int:
    return _check(lib().sfrde_integrate(plan, state, int(nsteps), float(t0), int(ckpt_every),
                                        ckpt), "sfrde_integrate")


def sfrde_ckpt_bytes(plan, nsteps, ckpt_every) -> int:
    return _check(lib().sfrde_ckpt_bytes(plan, int(nsteps), int(ckpt_every)), "sfrde_ckpt_bytes")


def sfrde_resume(plan, ckpt, slot, state, nsteps, t0, ckpt_every=0, ckpt_out=None) -> int:
    return _check(lib().sfrde_resume(plan, ckpt, int(slot), state, int(nsteps), float(t0),
                                     int(ckpt_every), ckpt_out), "sfrde_resume")


def _backward(fn, plan, ckpt, nsteps, ckpt_every, t0, grad_uT, grad_u0, nspecies, nparams,
              want_kappa, want_alpha, want_params, batch):
    gk = (ctypes.c_double * (batch * nspecies))() if want_kappa else None
    ga = (ctypes.c_double * (batch * nspecies))() if want_alpha else None
    gp = ((ctypes.c_double * max(1, batch * nparams))() if (want_params and nparams > 0)
          else None)
    rc = getattr(lib(), fn)(plan, ckpt, int(nsteps), int(ckpt_every), float(t0), grad_uT,
                            grad_u0, gk, ga, gp)
    _check(rc, fn)
    return (list(gk) if gk is not None else None, list(ga) if ga is not None else None,
            list(gp)[:batch * nparams] if gp is not None else None)


def sfrde_backward(plan, ckpt, nsteps, ckpt_every, t0, grad_uT, grad_u0=None, nspecies=2,
                   nparams=0, want_kappa=True, want_alpha=True, want_params=True, batch=1):
    """Returns (grad_kappa, grad_alpha, grad_params) as flat lists, [batch][...]
    for ensemble plans (None if not asked)."""
    return _backward("sfrde_backward", plan, ckpt, nsteps, ckpt_every, t0, grad_uT, grad_u0,
                     nspecies, nparams, want_kappa, want_alpha, want_params, batch)


def sfrde_backward_noalloc(plan, ckpt, nsteps, ckpt_every, t0, grad_uT, grad_u0=None,
                           nspecies=2, nparams=0, want_kappa=True, want_alpha=True,
                           want_params=True, batch=1):
    """sfrde_backward without device allocation (static scratch); same returns."""
    return _backward("sfrde_backward_noalloc", plan, ckpt, nsteps, ckpt_every, t0, grad_uT,
                     grad_u0, nspecies, nparams, want_kappa, want_alpha, want_params, batch)


def sfrde_destroy(plan) -> int:
    return _check(lib().sfrde_destroy(plan), "sfrde_destroy")


def sfrde_workspace_bytes(plan) -> int:
    return _check(lib().sfrde_workspace_bytes(plan), "sfrde_workspace_bytes")


def sfrde_profile(plan, enable) -> int:
    """enable = 0 stops; enable = k >= 1 clears and reserves events for k launches."""
    return _check(lib().sfrde_profile(plan, int(enable)), "sfrde_profile")


def sfrde_profile_read(plan):
    """{class: (total ms, launches)} for the launches recorded since enabling."""
    ms = (ctypes.c_double * len(KERNEL_CLASSES))()
    cnt = (ctypes.c_int64 * len(KERNEL_CLASSES))()
    _check(lib().sfrde_profile_read(plan, ms, cnt), "sfrde_profile_read")
    return {k: (ms[i], cnt[i]) for i, k in enumerate(KERNEL_CLASSES)}


def sfrde_axis_eigenvalues(bc, n, h):
    out = (ctypes.c_double * int(n))()
    _check(lib().sfrde_axis_eigenvalues(int(bc), int(n), float(h), out), "sfrde_axis_eigenvalues")
    return list(out)


def sfrde_eval_coefficients(scheme, L, dt, deriv=False):
    out = (ctypes.c_double * 6)()
    _check(lib().sfrde_eval_coefficients(int(scheme), float(L), float(dt), int(bool(deriv)), out),
           "sfrde_eval_coefficients")
    return list(out)


def sfrde_amplification(scheme, count, x, y, r, hip_stream=0) -> int:
    """x, y, r: device addresses (x and r hold complex pairs)."""
    return _check(lib().sfrde_amplification(int(scheme), int(count), x, y, r,
                                            hip_stream or None), "sfrde_amplification")


def sfrde_stability_boundary(scheme, ny, y, ntheta, roots, poly=None, hip_stream=0) -> int:
    """y, roots, poly: device addresses (poly may be None)."""
    return _check(lib().sfrde_stability_boundary(int(scheme), int(ny), y, int(ntheta), roots,
                                                 poly, hip_stream or None),
                  "sfrde_stability_boundary")
