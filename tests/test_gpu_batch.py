"""Ensemble plans (sfrde_plan_batch through the C ABI): several members of one
grid with their own orders, diffusion coefficients and reaction parameters,
advanced by the same launches. Each member must match the FP64 oracle run of
that member alone (FP64 1e-10, FP32 2e-5), and the adjoint of each member its
own oracle adjoint."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import problem
from paper_2003_13569_amd.torch_api import Plan
from tests.gpu_util import TD
from tests.test_gpu_parity import CASES, DENSE_CASES, FFT_CASES, VEC_CASES

pytestmark = pytest.mark.gpu


def _members(wl, B):
    """B variants of a workload: orders, diffusion and parameters shifted per member."""
    out = []
    for b in range(B):
        alpha = tuple(min(2.0, a - 0.07 * b) for a in wl.alpha)
        kappa = tuple(k * (1.0 + 0.3 * b) for k in wl.kappa)
        params = tuple(p * (1.0 + 0.02 * b) for p in wl.params)
        out.append(wl.replace(alpha=alpha, kappa=kappa, params=params, seed=wl.seed + b))
    return out


def _batch_plan(members, dtype):
    wl = members[0]
    return Plan(wl.shape, wl.bc, wl.h, [m.alpha for m in members], [m.kappa for m in members],
                wl.dt, wl.reaction, [m.params for m in members], dtype, wl.scheme,
                batch=len(members))


# ..., a dense-kernel axis, an FFT axis
BATCH_CASES = [CASES[2], CASES[3], CASES[6], DENSE_CASES[1], FFT_CASES[0]]


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 2e-5)])
@pytest.mark.parametrize("wl", BATCH_CASES, ids=[c.name for c in BATCH_CASES])
def test_batch_members_match_oracle(wl, dtype, tol):
    members = _members(wl, 3)
    u0 = np.stack([W.initial_fields(m) for m in members])
    p = _batch_plan(members, dtype)
    u = torch.tensor(u0, dtype=TD[dtype], device="cuda")
    p.integrate(u, 5, 0.0)
    torch.cuda.synchronize()
    got = u.double().cpu().numpy()
    p.close()
    for b, m in enumerate(members):
        ref = problem.run(m, u0[b], 5)
        assert problem.rel_err(got[b], ref) <= tol, (b, problem.rel_err(got[b], ref))


@pytest.mark.parametrize("dtype,tol", [("f32", 2e-5), ("f64", 1e-10)])
@pytest.mark.parametrize("wl", VEC_CASES[:3], ids=[c.name for c in VEC_CASES[:3]])
def test_batch_vector_paths_match_oracle(wl, dtype, tol):
    """Members on the FP32 vector paths and the FP64 register tiles (each
    member's fields at its own offset)."""
    members = _members(wl, 2)
    u0 = np.stack([W.initial_fields(m) for m in members])
    p = _batch_plan(members, dtype)
    u = torch.tensor(u0, dtype=TD[dtype], device="cuda")
    p.integrate(u, 3, 0.0)
    torch.cuda.synchronize()
    got = u.double().cpu().numpy()
    p.close()
    for b, m in enumerate(members):
        ref = problem.run(m, u0[b], 3)
        assert problem.rel_err(got[b], ref) <= tol


def test_batch_adjoint_matches_oracle_per_member():
    wl = CASES[2]  # Gierer-Meinhardt, Neumann, per-species orders
    members = _members(wl, 3)
    u0 = np.stack([W.initial_fields(m) for m in members])
    wbar = np.random.default_rng(5).standard_normal(u0.shape)
    M, K = 5, 2
    p = _batch_plan(members, "f64")
    u = torch.tensor(u0, device="cuda")
    ck = p.integrate(u, M, 0.0, K)
    g_u0 = torch.empty_like(u)
    gk, ga, gp = p.backward(ck, M, K, torch.tensor(wbar, device="cuda"), 0.0, g_u0)
    torch.cuda.synchronize()
    g_u0 = g_u0.cpu().numpy()
    S, npar = wl.nspecies, len(wl.params)
    for b, m in enumerate(members):
        ref = problem.gradients(m, u0[b], M, wbar[b])
        assert problem.rel_err(g_u0[b], ref["u0"]) <= 1e-10
        for key, got in (("kappa", gk[b * S:(b + 1) * S]), ("alpha", ga[b * S:(b + 1) * S]),
                         ("params", gp[b * npar:(b + 1) * npar])):
            r = ref[key]
            assert np.max(np.abs(np.array(got) - r)) <= 1e-10 * max(np.max(np.abs(r)), 1e-300), \
                (b, key, got, r)
    p.close()


@pytest.mark.parametrize("params", [True, False], ids=["params", "no-params"])
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 1e-3)])
def test_batch_adjoint_on_vector_paths_matches_oracle_per_member(dtype, tol, params):
    """Ensemble adjoint on a grid whose axes take the vector paths (the
    ensemble's z adjoint accumulates the kappa/alpha terms per point;
    without reaction-parameter gradients the FP32 adjoint x kernel folds its
    input from registers)."""
    wl = VEC_CASES[2]  # Gierer-Meinhardt 256 x 128, Neumann
    members = _members(wl, 2)
    u0 = np.stack([W.initial_fields(m) for m in members])
    wbar = np.random.default_rng(6).standard_normal(u0.shape)
    M, K = 4, 2
    p = _batch_plan(members, dtype)
    u = torch.tensor(u0, dtype=TD[dtype], device="cuda")
    ck = p.integrate(u, M, 0.0, K)
    g_u0 = torch.empty_like(u)
    gk, ga, gp = p.backward(ck, M, K, torch.tensor(wbar, dtype=TD[dtype], device="cuda"), 0.0,
                            g_u0, params=params)
    torch.cuda.synchronize()
    assert (gp is None) == (not params)
    g_u0 = g_u0.double().cpu().numpy()
    S, npar = wl.nspecies, len(wl.params)
    for b, m in enumerate(members):
        ref = problem.gradients(m, u0[b], M, wbar[b])
        assert problem.rel_err(g_u0[b], ref["u0"]) <= (1e-10 if dtype == "f64" else 1e-4)
        checks = [("kappa", gk[b * S:(b + 1) * S]), ("alpha", ga[b * S:(b + 1) * S])]
        if params:
            checks.append(("params", gp[b * npar:(b + 1) * npar]))
        for key, got in checks:
            r = ref[key]
            assert np.max(np.abs(np.array(got) - r)) <= tol * max(np.max(np.abs(r)), 1e-300), \
                (b, key, got, r)
    p.close()


def test_batch_exponential_scheme_matches_oracle():
    wl = CASES[4].replace(scheme="exp")  # 3D Dirichlet, Cox-Matthews coefficients
    members = _members(wl, 2)
    u0 = np.stack([W.initial_fields(m) for m in members])
    p = _batch_plan(members, "f64")
    u = torch.tensor(u0, device="cuda")
    p.integrate(u, 4, 0.0)
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    p.close()
    for b, m in enumerate(members):
        assert problem.rel_err(got[b], problem.run(m, u0[b], 4)) <= 1e-10


def test_batch_checkpoint_resume_continues_every_member():
    wl = CASES[6]
    members = _members(wl, 2)
    u0 = np.stack([W.initial_fields(m) for m in members])
    p = _batch_plan(members, "f64")
    u = torch.tensor(u0, device="cuda")
    ck = p.integrate(u, 6, 0.0, 3)
    v = torch.empty_like(u)
    p.resume(ck, 1, v, 3, 3 * wl.dt)
    torch.cuda.synchronize()
    assert torch.equal(u, v)
    p.close()


def test_batch_of_example2_members_reproduces_table2_rows():
    """Two Example 2 members (orders 2.0 and 1.4) in one plan, 1/h = 20."""
    inv_h, n = 20, 20
    h = 1.0 / inv_h
    tau = 0.1 * h
    M = int(round(1.0 / tau))
    p = Plan((n, n), "periodic", (h, h), [(2.0,), (1.4,)], [(1.0,), (1.0,)], tau, "huxley_mms",
             [(), ()], "f64", batch=2)
    u = torch.zeros((2, 1, n, n), dtype=torch.float64, device="cuda")
    p.integrate(u, M, 0.0)
    torch.cuda.synchronize()
    C = np.cos(2 * np.pi * np.arange(n) * h) ** 3
    for b, (alpha, printed) in enumerate(((2.0, 1.4159e-03), (1.4, 9.8009e-04))):
        exact = (M * tau) ** alpha * np.outer(C, C)
        err = float(np.max(np.abs(u[b, 0].cpu().numpy() - exact)))
        assert abs(err - printed) <= 0.6e-4 * printed, (alpha, err)
    p.close()


def test_autograd_function_on_an_ensemble_matches_members():
    """SFRDEFunction with spec["batch"]: gradients of every member equal those
    of that member run alone through the same function."""
    from paper_2003_13569_amd.torch_api import SFRDEFunction
    wl = CASES[2]
    members = _members(wl, 2)
    u0 = np.stack([W.initial_fields(m) for m in members])
    wbar = np.random.default_rng(8).standard_normal(u0.shape)
    base = dict(shape=wl.shape, bc=wl.bc, h=wl.h, dt=wl.dt, reaction=wl.reaction, nsteps=4,
                ckpt_every=2, dtype="f64", scheme="p13")

    def grads(x0, kap, alp, par, spec, w):
        x0 = torch.tensor(x0, device="cuda", requires_grad=True)
        kap = torch.tensor(kap, dtype=torch.float64, requires_grad=True)
        alp = torch.tensor(alp, dtype=torch.float64, requires_grad=True)
        par = torch.tensor(par, dtype=torch.float64, requires_grad=True)
        uT = SFRDEFunction.apply(x0, kap, alp, par, spec)
        (uT * torch.tensor(w, device="cuda")).sum().backward()
        return x0.grad.cpu().numpy(), kap.grad.numpy(), alp.grad.numpy(), par.grad.numpy()

    gb = grads(u0, [m.kappa for m in members], [m.alpha for m in members],
               [m.params for m in members], dict(base, batch=2), wbar)
    for b, m in enumerate(members):
        g1 = grads(u0[b], m.kappa, m.alpha, m.params, base, wbar[b])
        for x, y in zip((gb[0][b], gb[1][b], gb[2][b], gb[3][b]), g1):
            assert np.max(np.abs(x - y)) <= 1e-10 * max(np.max(np.abs(y)), 1e-300)


def test_large_fp64_ensemble_of_small_grids_matches_oracle():
    """48 members of a small 2D FP64 problem in one plan. A single member's
    strided-axis tiles hold one species (too few blocks otherwise); with 48
    members the launch has enough blocks and the tiles hold both species. Both
    layouts must give each member's oracle result."""
    wl = CASES[0]  # FitzHugh-Nagumo, Neumann, 37 x 45
    B = 48
    members = [wl.replace(alpha=(1.2 + 0.8 * b / (B - 1),) * 2,
                          kappa=(wl.kappa[0] * (1.0 + 0.05 * b), wl.kappa[1]), seed=wl.seed + b)
               for b in range(B)]
    u0 = np.stack([W.initial_fields(m) for m in members])
    p = _batch_plan(members, "f64")
    u = torch.tensor(u0, device="cuda")
    p.integrate(u, 3, 0.0)
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    p.close()
    for b in range(0, B, 6):
        ref = problem.run(members[b], u0[b], 3)
        assert problem.rel_err(got[b], ref) <= 1e-10, (b, problem.rel_err(got[b], ref))
    # the same members alone (species-split tiles) agree with the ensemble
    for b in (0, B - 1):
        m = members[b]
        q = Plan(m.shape, m.bc, m.h, m.alpha, m.kappa, m.dt, m.reaction, m.params, "f64", m.scheme)
        v = torch.tensor(u0[b], device="cuda")
        q.integrate(v, 3, 0.0)
        torch.cuda.synchronize()
        assert problem.rel_err(v.cpu().numpy(), got[b]) <= 1e-12
        q.close()
