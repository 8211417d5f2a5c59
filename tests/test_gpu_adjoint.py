"""GPU adjoint (sfrde_backward through the C ABI) against the FP64 oracle's
discrete adjoint, with segment recomputation from checkpoints."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import problem
from paper_2003_13569_amd.torch_api import SFRDEFunction
from tests.gpu_util import TD, plan_for
from tests.test_gpu_parity import CASES, DENSE_CASES, FFT_CASES, PATH_MATRIX, VEC_CASES

pytestmark = pytest.mark.gpu

M, K = 5, 2


def _rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _gpu_grads(wl, u0, wbar, dtype, scheme=None, params=True):
    p = plan_for(wl, dtype, scheme)
    u = torch.tensor(u0, dtype=TD[dtype], device="cuda")
    ckpt = p.integrate(u, M, 0.0, ckpt_every=K)
    g_uT = torch.tensor(wbar, dtype=TD[dtype], device="cuda")
    g_u0 = torch.empty_like(g_uT)
    gk, ga, gp = p.backward(ckpt, M, K, g_uT, 0.0, g_u0, params=params)
    torch.cuda.synchronize()
    out = dict(uT=u.double().cpu().numpy(), u0=g_u0.double().cpu().numpy(), kappa=np.array(gk),
               alpha=np.array(ga), params=None if gp is None else np.array(gp))
    p.close()
    return out


@pytest.mark.parametrize("scheme", ["p13", "exp"])
@pytest.mark.parametrize("wl", CASES, ids=[c.name for c in CASES])
def test_fp64_adjoint_matches_oracle(wl, scheme):
    wl = wl.replace(scheme=scheme)
    u0 = W.initial_fields(wl)
    wbar = np.random.default_rng(11).standard_normal(u0.shape)
    ref = problem.gradients(wl, u0, M, wbar)
    got = _gpu_grads(wl, u0, wbar, "f64")
    assert _rel(got["uT"], ref["uT"]) <= 1e-10
    assert _rel(got["u0"], ref["u0"]) <= 1e-10
    for key in ("kappa", "alpha", "params"):
        r, g = ref[key], got[key]
        scale = max(np.max(np.abs(r)), 1e-300)
        assert np.max(np.abs(g - r)) <= 1e-10 * scale, (key, g, r)


@pytest.mark.parametrize("wl", CASES[:4], ids=[c.name for c in CASES[:4]])
def test_fp32_adjoint_matches_oracle(wl):
    u0 = W.initial_fields(wl)
    wbar = np.random.default_rng(12).standard_normal(u0.shape)
    ref = problem.gradients(wl, u0, M, wbar)
    got = _gpu_grads(wl, u0, wbar, "f32")
    assert _rel(got["u0"], ref["u0"]) <= 1e-4
    for key in ("kappa", "alpha", "params"):
        r, g = ref[key], got[key]
        assert np.max(np.abs(g - r)) <= 1e-3 * max(np.max(np.abs(r)), 1e-300), (key, g, r)


@pytest.mark.parametrize("wl", [VEC_CASES[0], VEC_CASES[2]], ids=["sch3d-neu-vec", "gm2d-neu-vec"])
def test_fp32_adjoint_vector_paths_match_oracle(wl):
    u0 = W.initial_fields(wl)
    wbar = np.random.default_rng(13).standard_normal(u0.shape)
    ref = problem.gradients(wl, u0, M, wbar)
    got = _gpu_grads(wl, u0, wbar, "f32")
    assert _rel(got["u0"], ref["u0"]) <= 1e-4
    for key in ("kappa", "alpha", "params"):
        r, g = ref[key], got[key]
        assert np.max(np.abs(g - r)) <= 1e-3 * max(np.max(np.abs(r)), 1e-300), (key, g, r)


# Two species, DCT-I / DST-I x axes of 64, 128 or 256 points, FP32, no
# reaction-parameter gradients: the adjoint x kernel folds its input straight
# from registers (launches with parameter partials take the LDS-staged one).
RF_CASES = [wl for wl in PATH_MATRIX + VEC_CASES
            if wl.name in ("lin2-neu-64x128", "lin2-dir-64x128", "sch3d-neu-vec", "sch3d-dir-vec",
                           "gm2d-neu-vec", "sch3d-dir-vec128")]


@pytest.mark.parametrize("wl", RF_CASES, ids=[c.name for c in RF_CASES])
def test_fp32_adjoint_without_parameter_gradients_matches_oracle(wl):
    u0 = W.initial_fields(wl)
    wbar = np.random.default_rng(15).standard_normal(u0.shape)
    ref = problem.gradients(wl, u0, M, wbar)
    got = _gpu_grads(wl, u0, wbar, "f32", params=False)
    assert got["params"] is None
    assert _rel(got["u0"], ref["u0"]) <= 1e-4
    for key in ("kappa", "alpha"):
        r, g = ref[key], got[key]
        assert np.max(np.abs(g - r)) <= 1e-3 * max(np.max(np.abs(r)), 1e-300), (key, g, r)


# The adjoint's instances by species count (one, two, three species) and
# boundary condition on the 2D grid whose axes take the vector paths and on
# the 1D grids, in both precisions (the periodic references in the exact
# circulant basis).
ADJ_MATRIX = [wl for wl in PATH_MATRIX if len(wl.shape) != 3]


@pytest.mark.parametrize("scheme", ["p13", "exp"])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("wl", ADJ_MATRIX, ids=[c.name for c in ADJ_MATRIX])
def test_adjoint_species_count_and_boundary_matrix_matches_oracle(wl, dtype, scheme):
    wl = wl.replace(scheme=scheme)
    u0 = W.initial_fields(wl)
    wbar = np.random.default_rng(14).standard_normal(u0.shape)
    ref = problem.gradients(wl, u0, M, wbar, periodic_basis="hartley")
    got = _gpu_grads(wl, u0, wbar, dtype)
    t_u, t_p = (1e-10, 1e-10) if dtype == "f64" else (1e-4, 1e-3)
    assert _rel(got["u0"], ref["u0"]) <= t_u
    for key in ("kappa", "alpha", "params"):
        r, g = ref[key], got[key]
        assert np.max(np.abs(g - r)) <= t_p * max(np.max(np.abs(r)), 1e-300), (key, g, r)


def test_checkpoint_spacing_does_not_change_gradients():
    wl = CASES[1]
    u0 = W.initial_fields(wl)
    wbar = np.random.default_rng(2).standard_normal(u0.shape)
    outs = []
    for k in (1, 2, 5):
        p = plan_for(wl, "f64")
        u = torch.tensor(u0, dtype=torch.float64, device="cuda")
        ckpt = p.integrate(u, M, 0.0, ckpt_every=k)
        g0 = torch.empty_like(u)
        gk, ga, gp = p.backward(ckpt, M, k, torch.tensor(wbar, device="cuda"), 0.0, g0)
        outs.append((g0.cpu().numpy(), gk, ga, gp))
        p.close()
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0])
        assert o[1] == outs[0][1] and o[2] == outs[0][2] and o[3] == outs[0][3]


def test_autograd_function_gives_oracle_gradients():
    wl = CASES[2]
    u0 = W.initial_fields(wl)
    wbar = np.random.default_rng(4).standard_normal(u0.shape)
    ref = problem.gradients(wl, u0, M, wbar)
    spec = dict(shape=wl.shape, bc=wl.bc, h=wl.h, dt=wl.dt, reaction=wl.reaction, nsteps=M,
                ckpt_every=K, dtype="f64", scheme="p13")
    x0 = torch.tensor(u0, dtype=torch.float64, device="cuda", requires_grad=True)
    kap = torch.tensor(wl.kappa, dtype=torch.float64, requires_grad=True)
    alp = torch.tensor(wl.alpha, dtype=torch.float64, requires_grad=True)
    par = torch.tensor(wl.params, dtype=torch.float64, requires_grad=True)
    uT = SFRDEFunction.apply(x0, kap, alp, par, spec)
    loss = (uT * torch.tensor(wbar, device="cuda")).sum()
    loss.backward()
    assert _rel(x0.grad.cpu().numpy(), ref["u0"]) <= 1e-10
    assert _rel(kap.grad.numpy(), ref["kappa"]) <= 1e-10
    assert _rel(alp.grad.numpy(), ref["alpha"]) <= 1e-10
    assert _rel(par.grad.numpy(), ref["params"]) <= 1e-10


def test_incompatible_checkpoint_is_rejected():
    from paper_2003_13569_amd import sfrde as C
    wl = CASES[0]
    p = plan_for(wl, "f64")
    u = torch.tensor(W.initial_fields(wl), dtype=torch.float64, device="cuda")
    ckpt = p.integrate(u, 4, 0.0, ckpt_every=2)
    with pytest.raises(C.SfrdeError) as ei:
        p.backward(ckpt, 4, 3, torch.zeros_like(u))
    assert ei.value.code == C.ESTATE
    with pytest.raises(C.SfrdeError) as ei:
        p.backward(ckpt, 6, 2, torch.zeros_like(u))
    assert ei.value.code == C.ESTATE
    p.close()


LONG_CASES = DENSE_CASES + FFT_CASES[:3] + FFT_CASES[-2:]  # the last two: one species


@pytest.mark.parametrize("wl", LONG_CASES, ids=[c.name for c in LONG_CASES])
def test_fp64_adjoint_long_axes_match_oracle(wl):
    # axes past the matrix-core engine (dense LDS kernels, FFT kernels). On
    # long periodic axes the oracle takes the exact circulant eigenbasis:
    # LAPACK's eigenvectors of a 1024-point axis move the kappa gradient by
    # 2e-10 relative (dL/dkappa weighs the top modes up to 1e5).
    u0 = W.initial_fields(wl)
    wbar = np.random.default_rng(13).standard_normal(u0.shape)
    ref = problem.gradients(wl, u0, M, wbar, periodic_basis="hartley")
    got = _gpu_grads(wl, u0, wbar, "f64")
    assert _rel(got["u0"], ref["u0"]) <= 1e-10
    for key in ("kappa", "alpha", "params"):
        r, g = ref[key], got[key]
        assert np.max(np.abs(g - r)) <= 1e-10 * max(np.max(np.abs(r)), 1e-300), (key, g, r)


def _c4_loss_and_grads(dtype, kappa, alpha, params, u0, target, with_grads):
    """Config 4 (Gierer-Meinhardt 256^2 Neumann, 200 steps of dt = 0.05):
    loss = mean over points of sum over species of (u_T - u*)^2."""
    wl = W.C4_GM_ADJ
    p = plan_for(wl, dtype, alpha=alpha, kappa=kappa, params=params)
    u = torch.tensor(u0, dtype=TD[dtype], device="cuda")
    npts = wl.npoints
    if not with_grads:
        p.integrate(u, wl.nsteps)
        d = u.double() - target
        loss = float((d * d).sum()) / npts
        p.close()
        return loss
    ck = p.integrate(u, wl.nsteps, 0.0, ckpt_every=wl.ckpt_every)
    d = u.double() - target
    loss = float((d * d).sum()) / npts
    g_uT = (2.0 / npts * d).to(TD[dtype]).contiguous()
    g_u0 = torch.empty_like(g_uT)
    gk, ga, gp = p.backward(ck, wl.nsteps, wl.ckpt_every, g_uT, 0.0, g_u0)
    torch.cuda.synchronize()
    p.close()
    return loss, g_u0.double(), np.array(gk), np.array(ga), np.array(gp)


C4_FD_TOL = 1e-8


def test_config4_adjoint_full_size_matches_central_differences():
    # Config 4 as specified: MSE after 200 steps against a target run with
    # perturbed parameters, gradients of u0, kappa, alpha and the reaction
    # constants with checkpoints every 20 steps, against central differences
    # in FP64 (steps of 1e-4 relative, at least 1e-6); the FP32 adjoint against
    # the FP64 one.
    wl = W.C4_GM_ADJ
    tg = wl.extra["target"]
    u0 = W.initial_fields(wl)
    pt = plan_for(wl, "f64", alpha=tg["alpha"], kappa=tg["kappa"], params=tg["params"])
    target = torch.tensor(u0, dtype=torch.float64, device="cuda")
    pt.integrate(target, wl.nsteps)
    pt.close()
    kap, alp, par = list(wl.kappa), list(wl.alpha), list(wl.params)
    loss, gu0, gk, ga, gp = _c4_loss_and_grads("f64", kap, alp, par, u0, target, True)
    assert loss > 0

    def central(which, i, rel):
        vals = {"kappa": kap, "alpha": alp, "params": par}
        out = []
        for sgn in (1.0, -1.0):
            v = {k: list(x) for k, x in vals.items()}
            step = rel * max(abs(v[which][i]), 1e-2)
            v[which][i] += sgn * step
            out.append(_c4_loss_and_grads("f64", v["kappa"], v["alpha"], v["params"], u0,
                                          target, False))
        return (out[0] - out[1]) / (2 * step)

    def fd(which, i):
        # central differences at steps h and h/2 (h = 1e-4 relative, at least
        # 1e-6), Richardson-extrapolated: error O(h^4) instead of O(h^2)
        d1, d2 = central(which, i, 1e-4), central(which, i, 5e-5)
        return (4.0 * d2 - d1) / 3.0

    for which, g in (("kappa", gk), ("alpha", ga), ("params", gp)):
        for i in range(len(g)):
            ref = fd(which, i)
            print(f"config4 FD {which}[{i}]: adjoint {g[i]:.12e} central {ref:.12e} "
                  f"rel {abs(g[i] - ref) / abs(ref):.2e}")
            assert abs(g[i] - ref) <= C4_FD_TOL * abs(ref), (which, i, g[i], ref)
    # u0 along a random direction
    v = torch.tensor(np.random.default_rng(17).standard_normal(u0.shape), device="cuda")

    def central_u0(eps):
        lp = _c4_loss_and_grads("f64", kap, alp, par, (torch.tensor(u0, device="cuda") + eps * v)
                                .cpu().numpy(), target, False)
        lm = _c4_loss_and_grads("f64", kap, alp, par, (torch.tensor(u0, device="cuda") - eps * v)
                                .cpu().numpy(), target, False)
        return (lp - lm) / (2 * eps)

    fdu = (4.0 * central_u0(5e-5) - central_u0(1e-4)) / 3.0
    ad = float((gu0 * v).sum())
    print(f"config4 FD u0: adjoint {ad:.12e} central {fdu:.12e} rel {abs(ad - fdu) / abs(fdu):.2e}")
    assert abs(ad - fdu) <= C4_FD_TOL * abs(fdu), (ad, fdu)
    # the FP32 path (the configuration's precision) against the FP64 adjoint
    _, gu0_32, gk32, ga32, gp32 = _c4_loss_and_grads("f32", kap, alp, par, u0, target, True)
    assert _rel(gu0_32.cpu().numpy(), gu0.cpu().numpy()) <= 1e-3
    for a, b in ((gk32, gk), (ga32, ga), (gp32, gp)):
        assert np.max(np.abs(a - b)) <= 1e-3 * np.max(np.abs(b)), (a, b)


@pytest.mark.gpu
def test_checkpoint_of_another_shape_or_bc_is_rejected():
    # same point count, species and dtype: a transposed grid and another
    # boundary condition have other spectral bases
    from paper_2003_13569_amd import sfrde as C
    import workloads as Wk
    base = Wk.small(Wk.C1_FHN, (24, 32), nsteps=4)
    tr = Wk.small(Wk.C1_FHN, (32, 24), nsteps=4)
    bc = base.replace(bc="dirichlet")
    pa = plan_for(base, "f64")
    u = torch.tensor(W.initial_fields(base), dtype=torch.float64, device="cuda")
    ckpt = pa.integrate(u, 4, 0.0, ckpt_every=2)
    for other in (tr, bc):
        pb = plan_for(other, "f64")
        v = torch.zeros(pb.field_shape, dtype=torch.float64, device="cuda")
        with pytest.raises(C.SfrdeError) as ei:
            pb.backward(ckpt, 4, 2, v)
        assert ei.value.code == C.ESTATE
        with pytest.raises(C.SfrdeError) as ei:
            pb.resume(ckpt, 1, v, 2)
        assert ei.value.code == C.ESTATE
        pb.close()
    # the writer itself resumes fine
    pa.resume(ckpt, 1, u, 2, 2 * base.dt)
    pa.close()


def _c5_loss_and_grads(alpha, kappa, u0, target, M, K, with_grads):
    """Configuration 5 (3D Schnakenberg Neumann 256^3, dt 0.005) over M steps
    in FP64: loss = mean over points and species of (u_M - u*)^2 with u* the
    run from perturbed orders and diffusion (the configuration's loss)."""
    wl = W.C5_SCHNAK_NEU
    p = plan_for(wl, "f64", alpha=alpha, kappa=kappa)
    u = torch.tensor(u0, dtype=torch.float64, device="cuda")
    if not with_grads:
        p.integrate(u, M)
        d = u - target
        loss = float((d * d).sum()) / d.numel()
        p.close()
        return loss
    ck = p.integrate(u, M, 0.0, ckpt_every=K)
    d = u - target
    loss = float((d * d).sum()) / d.numel()
    g = (2.0 / d.numel()) * d
    gk, ga, _ = p.backward(ck, M, K, g.contiguous(), 0.0, None, params=False)
    torch.cuda.synchronize()
    p.close()
    return loss, np.array(gk), np.array(ga)


# alpha_v and kappa_v have gradients of ~4e-13 on this loss: their central
# differences carry ~1e-7 of rounding noise (they converge as h^2 down to it)
C5_FD_TOL = 1e-6


def test_config5_fp64_adjoint_matches_central_differences():
    # The benchmark workload at full size (256^3) over a bounded horizon
    # (64 steps, checkpoints every 8) with its loss (MSE against a run with
    # alpha + 0.05 and kappa_v 1.1 times): FP64 gradients of alpha_u, alpha_v
    # and kappa_v against Richardson-extrapolated central differences (steps
    # of 1e-4 and 5e-5 relative).
    wl = W.C5_SCHNAK_NEU
    tg = wl.extra["target"]
    M, K = 64, 8
    u0 = W.initial_fields(wl)
    pt = plan_for(wl, "f64", alpha=tuple(a + tg["alpha_shift"] for a in wl.alpha),
                  kappa=(wl.kappa[0], wl.kappa[1] * tg["kappa_v_scale"]))
    target = torch.tensor(u0, dtype=torch.float64, device="cuda")
    pt.integrate(target, M)
    pt.close()
    alp, kap = list(wl.alpha), list(wl.kappa)
    loss, gk, ga = _c5_loss_and_grads(alp, kap, u0, target, M, K, True)
    assert loss > 0
    for which, i, g in (("alpha", 0, ga[0]), ("alpha", 1, ga[1]), ("kappa", 1, gk[1])):
        cds = []
        for rel in (1e-4, 5e-5):
            out = []
            for sgn in (1.0, -1.0):
                a, k = list(alp), list(kap)
                v = a if which == "alpha" else k
                step = rel * abs(v[i])
                v[i] += sgn * step
                out.append(_c5_loss_and_grads(a, k, u0, target, M, K, False))
            cds.append((out[0] - out[1]) / (2 * step))
        # Richardson extrapolation of the two central differences (O(h^4))
        ref = (4.0 * cds[1] - cds[0]) / 3.0
        err = abs(g - ref) / abs(ref)
        print(f"config5 FD {which}[{i}]: central h {abs(g - cds[0]) / abs(ref):.2e}, "
              f"h/2 {abs(g - cds[1]) / abs(ref):.2e}")
        print(f"config5 FD {which}[{i}]: adjoint {g:.12e} central {ref:.12e} rel {err:.2e}")
        assert err <= C5_FD_TOL, (which, i, g, ref)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("wl", [CASES[2], VEC_CASES[0]], ids=["gm2d-neu", "sch3d-neu-vec"])
def test_u0_only_backward_matches_full_backward(wl, dtype):
    # without kappa/alpha gradients the recompute stores 4 fields per step
    # (no u_hat, no f_hat) and runs on the plan's own u_hat
    u0 = W.initial_fields(wl)
    wbar = np.random.default_rng(31).standard_normal(u0.shape)
    p = plan_for(wl, dtype)
    u = torch.tensor(u0, dtype=TD[dtype], device="cuda")
    ck = p.integrate(u, M, 0.0, ckpt_every=K)
    g = torch.tensor(wbar, dtype=TD[dtype], device="cuda")
    a, b = torch.empty_like(g), torch.empty_like(g)
    full_bytes = None
    p.backward(ck, M, K, g, 0.0, a)
    full_bytes = p.workspace_bytes()
    gk, ga, gp = p.backward(ck, M, K, g, 0.0, b, kappa=False, alpha=False, params=False)
    assert gk is None and ga is None and gp is None
    torch.cuda.synchronize()
    tol = 1e-12 if dtype == "f64" else 1e-5
    assert _rel(b.double().cpu().numpy(), a.double().cpu().numpy()) <= tol
    # a fresh plan asked for u0 only holds the smaller store
    q = plan_for(wl, dtype)
    v = torch.tensor(u0, dtype=TD[dtype], device="cuda")
    ck2 = q.integrate(v, M, 0.0, ckpt_every=K)
    c = torch.empty_like(g)
    q.backward(ck2, M, K, g, 0.0, c, kappa=False, alpha=False, params=False)
    torch.cuda.synchronize()
    assert torch.equal(c, b)
    assert q.workspace_bytes() < full_bytes
    p.close()
    q.close()
