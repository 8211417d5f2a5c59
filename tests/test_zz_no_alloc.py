"""sfrde_backward_noalloc (the allocation-free backward, through the C ABI)
against sfrde_backward on the same plans and checkpoints: two calls in a
row, the second on a smaller problem, so that the static scratch array still
holds the first call's data when the second runs."""
import numpy as np
import pytest
import torch

import workloads as W
from paper_2003_13569_amd import sfrde as C
from tests.gpu_util import TD, plan_for
from tests.test_gpu_parity import CASES, VEC_CASES

pytestmark = pytest.mark.gpu


def _grads(fn, p, wl, ckpt, M, K, wbar, dtype):
    g_uT = torch.tensor(wbar, dtype=TD[dtype], device="cuda")
    g_u0 = torch.full_like(g_uT, float("nan"))
    gk, ga, gp = fn(p.handle, ckpt.data_ptr(), M, K, 0.0, g_uT.data_ptr(), g_u0.data_ptr(),
                    p.S, p.nparams, True, True, True, 1)
    torch.cuda.synchronize()
    return g_u0.double().cpu().numpy(), np.array(gk), np.array(ga), np.array(gp)


def _compare(wl, M, K, dtype, seed):
    p = plan_for(wl, dtype)
    u0 = W.initial_fields(wl)
    u = torch.tensor(u0, dtype=TD[dtype], device="cuda")
    ckpt = p.integrate(u, M, 0.0, ckpt_every=K)
    wbar = np.random.default_rng(seed).standard_normal(u0.shape)
    a = _grads(C.sfrde_backward_noalloc, p, wl, ckpt, M, K, wbar, dtype)
    b = _grads(C.sfrde_backward, p, wl, ckpt, M, K, wbar, dtype)
    p.close()
    tol = 1e-10 if dtype == "f64" else 2e-5
    for x, y in zip(a, b):
        assert np.all(np.isfinite(x))
        scale = max(float(np.max(np.abs(y))), 1e-300)
        assert float(np.max(np.abs(x - y))) <= tol * scale
        # same kernels, same fixed summation orders: identical results
        assert np.array_equal(x, y)


# (larger, smaller) pairs: FP32 vector path (kappa/alpha partials in the Z
# kernels), FP64 per-point path (FP64 accumulator and derivative tables)
PAIRS = [
    ((VEC_CASES[0], 4, 2, "f32"), (W.small(VEC_CASES[0], (64, 32, 64)), 3, 3, "f32")),
    ((CASES[0], 5, 2, "f64"), (W.small(CASES[0], (20, 24)), 3, 3, "f64")),
]


@pytest.mark.parametrize("first,second", PAIRS, ids=["f32-vector", "f64-generic"])
def test_noalloc_backward_matches_backward_twice(first, second):
    _compare(*first, seed=1)
    _compare(*second, seed=2)


def test_noalloc_backward_rejects_what_does_not_fit():
    # 256^3 FP32 with 32 steps per segment needs ~40 GB of segment store
    wl = W.C5_SCHNAK_NEU
    p = plan_for(wl, "f32")
    u = torch.tensor(W.initial_fields(wl), dtype=torch.float32, device="cuda")
    ckpt = p.integrate(u, 2, 0.0, ckpt_every=32)
    g = torch.zeros_like(u)
    with pytest.raises(C.SfrdeError) as ei:
        C.sfrde_backward_noalloc(p.handle, ckpt.data_ptr(), 2, 32, 0.0, g.data_ptr(),
                                 g.data_ptr(), p.S, p.nparams)
    assert ei.value.code == C.EINVAL
    assert "allocation-free" in C.sfrde_last_error()
    p.close()
