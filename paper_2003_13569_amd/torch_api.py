"""PyTorch-facing wrappers: a plan bound to torch tensors and the current
HIP stream, and a ``torch.autograd.Function`` over the whole integration
whose backward is the library's hand-written adjoint. PyTorch provides device
memory and streams only; every step runs in libsfrde.
"""
from __future__ import annotations

import torch

from . import sfrde as C

_TORCH_DTYPE = {"f32": torch.float32, "f64": torch.float64}


class Plan:
    """A libsfrde plan for fields shaped ``[S, (nz,) ny, nx]``, or an ensemble
    plan (``batch`` members, fields ``[batch, S, ...]``) when ``batch`` is given:
    then ``alpha`` and ``kappa`` are ``[batch][S]`` and ``params`` ``[batch][np]``.

    ``shape`` and ``h`` are in tensor order (slowest axis first); the C ABI
    takes them x-first, which this wrapper handles.
    """

    def __init__(self, shape, bc, h, alpha, kappa, dt, reaction, params, dtype="f32",
                 scheme="p13", stream=None, batch=None):
        self.shape = tuple(int(v) for v in shape)
        self.ndim = len(self.shape)
        self.batch = batch
        self.dtype = dtype
        self.torch_dtype = _TORCH_DTYPE[dtype]
        self.dt = float(dt)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        n_xyz, h_xyz = list(reversed(self.shape)), list(reversed(list(h)))
        if batch is None:
            self.S = len(alpha)
            self.nparams = len(params)
            self.handle = C.sfrde_plan(self.ndim, n_xyz, C.BC[bc], h_xyz, self.S, alpha, kappa,
                                       dt, C.REACTION[reaction], len(params), params,
                                       C.DTYPE[dtype], C.SCHEME[scheme], stream.cuda_stream)
        else:
            if not (len(alpha) == len(kappa) == len(params) == batch):
                raise ValueError("alpha, kappa and params need one entry per member")
            self.S = len(alpha[0])
            self.nparams = len(params[0])
            flat = lambda rows: [float(v) for r in rows for v in r]  # noqa: E731
            self.handle = C.sfrde_plan_batch(batch, self.ndim, n_xyz, C.BC[bc], h_xyz, self.S,
                                             flat(alpha), flat(kappa), dt, C.REACTION[reaction],
                                             self.nparams, flat(params), C.DTYPE[dtype],
                                             C.SCHEME[scheme], stream.cuda_stream)

    @property
    def field_shape(self):
        lead = (self.S,) if self.batch is None else (self.batch, self.S)
        return lead + self.shape

    def _check_field(self, u):
        if not (u.is_cuda and u.is_contiguous() and u.dtype == self.torch_dtype
                and tuple(u.shape) == self.field_shape):
            raise ValueError(f"expected a contiguous {self.torch_dtype} CUDA tensor of shape "
                             f"{self.field_shape}, got {u.dtype} {tuple(u.shape)}")

    def ckpt_bytes(self, nsteps, ckpt_every):
        return C.sfrde_ckpt_bytes(self.handle, nsteps, ckpt_every)

    def new_ckpt(self, nsteps, ckpt_every):
        nbytes = self.ckpt_bytes(nsteps, ckpt_every)
        return torch.empty(nbytes, dtype=torch.uint8, device="cuda")

    def integrate(self, u, nsteps, t0=0.0, ckpt_every=0, ckpt=None):
        """Advance ``u`` in place; returns the checkpoint tensor if asked."""
        self._check_field(u)
        if ckpt_every and ckpt is None:
            ckpt = self.new_ckpt(nsteps, ckpt_every)
        C.sfrde_integrate(self.handle, u.data_ptr(), nsteps, t0, ckpt_every,
                          ckpt.data_ptr() if ckpt is not None else None)
        return ckpt

    def step(self, u, t=0.0):
        self._check_field(u)
        C.sfrde_step(self.handle, u.data_ptr(), t)

    def resume(self, ckpt, slot, u, nsteps, t0=0.0, ckpt_every=0, ckpt_out=None):
        self._check_field(u)
        C.sfrde_resume(self.handle, ckpt.data_ptr(), slot, u.data_ptr(), nsteps, t0, ckpt_every,
                       ckpt_out.data_ptr() if ckpt_out is not None else None)

    def backward(self, ckpt, nsteps, ckpt_every, grad_uT, t0=0.0, grad_u0=None, kappa=True,
                 alpha=True, params=True):
        self._check_field(grad_uT)
        if grad_u0 is not None:
            self._check_field(grad_u0)
        return C.sfrde_backward(self.handle, ckpt.data_ptr(), nsteps, ckpt_every, t0,
                                grad_uT.data_ptr(),
                                grad_u0.data_ptr() if grad_u0 is not None else None,
                                self.S, self.nparams, kappa, alpha, params, self.batch or 1)

    def workspace_bytes(self):
        return C.sfrde_workspace_bytes(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            C.sfrde_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SFRDEFunction(torch.autograd.Function):
    """u_T = integrate(u0; kappa, alpha, params) with the discrete adjoint.

    ``spec`` is a dict: shape, bc, h, dt, reaction, nsteps, ckpt_every,
    dtype, scheme (t0 optional). With ``spec["batch"] = B`` it runs an
    ensemble plan: u0 is [B, S, ...], kappa and alpha [B, S], params [B, np].
    """

    @staticmethod
    def forward(ctx, u0, kappa, alpha, params, spec):
        batch = spec.get("batch")
        plan = Plan(spec["shape"], spec["bc"], spec["h"], alpha.tolist(), kappa.tolist(),
                    spec["dt"], spec["reaction"], params.tolist(), spec.get("dtype", "f32"),
                    spec.get("scheme", "p13"), batch=batch)
        n, K = int(spec["nsteps"]), int(spec.get("ckpt_every") or spec["nsteps"])
        u = u0.detach().clone().contiguous()
        ckpt = plan.integrate(u, n, spec.get("t0", 0.0), K)
        ctx.plan, ctx.ckpt, ctx.n, ctx.K = plan, ckpt, n, K
        ctx.t0 = spec.get("t0", 0.0)
        ctx.param_dtypes = (kappa.dtype, alpha.dtype, params.dtype)
        ctx.param_shapes = (kappa.shape, alpha.shape, params.shape)
        return u

    @staticmethod
    def backward(ctx, gout):
        plan = ctx.plan
        g = gout.contiguous()
        gu0 = torch.empty_like(g)
        gk, ga, gp = plan.backward(ctx.ckpt, ctx.n, ctx.K, g, ctx.t0, gu0)
        kd, ad, pd = ctx.param_dtypes
        ks, as_, ps = ctx.param_shapes
        return (gu0, torch.tensor(gk, dtype=kd).reshape(ks), torch.tensor(ga, dtype=ad).reshape(as_),
                torch.tensor(gp if gp else [], dtype=pd).reshape(ps), None)


def amplification(x, y, scheme="p13"):
    """Amplification factor r(x, y) of one step on the linear test equation
    (Section 4.2.2) for complex128 CUDA tensors x and float64 y of one shape;
    returns a complex128 tensor."""
    x = x.to(torch.complex128).contiguous()
    y = y.to(torch.float64).contiguous()
    if not (x.is_cuda and y.is_cuda and x.shape == y.shape):
        raise ValueError("x and y must be CUDA tensors of one shape")
    r = torch.empty_like(x)
    C.sfrde_amplification(C.SCHEME[scheme], x.numel(), x.data_ptr(), y.data_ptr(), r.data_ptr(),
                          torch.cuda.current_stream().cuda_stream)
    return r


def stability_boundary(y, ntheta, scheme="p13"):
    """Points of |r(x, y)| = 1 for each y in a float64 CUDA tensor:
    (roots [ny, ntheta, 4] complex128, quartic coefficients [ny, 5])."""
    y = y.to(torch.float64).contiguous()
    if not y.is_cuda or y.dim() != 1:
        raise ValueError("y must be a 1D CUDA tensor")
    ny = y.numel()
    roots = torch.empty((ny, ntheta, 4), dtype=torch.complex128, device=y.device)
    poly = torch.empty((ny, 5), dtype=torch.float64, device=y.device)
    C.sfrde_stability_boundary(C.SCHEME[scheme], ny, y.data_ptr(), ntheta, roots.data_ptr(),
                               poly.data_ptr(), torch.cuda.current_stream().cuda_stream)
    return roots, poly
