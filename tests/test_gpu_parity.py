"""GPU parity: libsfrde (through the C ABI) against the FP64 oracle.

FP64 results must agree with the oracle to 1e-10 and FP32 results to 2e-5
(max over species of ||x - x_ref||_inf / ||x_ref||_inf) after the stated
number of steps. Grids are small enough for the oracle but span several tiles
with ragged tails.
"""
import functools

import numpy as np
import pytest
import torch

import workloads as W
from oracle import problem
from paper_2003_13569_amd import sfrde as C
from paper_2003_13569_amd.torch_api import Plan
from tests.gpu_util import TD, plan_for, run

pytestmark = pytest.mark.gpu

FHN = (0.1, 0.01, 0.5, 1.0, 0.0)
GS = (0.04, 0.06)
SCH = (1.0, 0.1305, 0.7695)
GM = (0.1, 1.0, 1.0, 1.0, 1.0)


@functools.lru_cache(maxsize=32)
def oracle_run(wl, nsteps):
    """The oracle's fields after nsteps from the workload's initial fields
    (several tests share a reference; the exponential scheme's coefficients
    on 10^5-10^6 modes take tens of seconds)."""
    return problem.run(wl, W.initial_fields(wl), nsteps)


def _wl(name, bc, shape, reaction, params, alpha, kappa, dt, init, domain, scheme="p13"):
    return W.Workload(name=name, bc=bc, shape=shape, domain=domain, alpha=alpha, kappa=kappa,
                      reaction=reaction, params=params, dt=dt, nsteps=5, seed=7, init=init,
                      scheme=scheme)


CASES = [
    _wl("fhn2d-neu", "neumann", (37, 45), "fhn", FHN, (1.5, 1.5), (1e-2, 0.0), 0.1,
        "fhn_noise", (0.0, 2.5)),
    _wl("gs2d-per", "periodic", (40, 36), "gray_scott", GS, (1.7, 1.7), (2e-3, 1e-3), 1.0,
        "gs_square", (-1.0, 1.0)),
    _wl("gm2d-neu", "neumann", (33, 30), "gierer_meinhardt", GM, (1.6, 1.4), (1e-3, 0.05),
        0.05, "gm_noise", (0.0, 2.0)),
    _wl("sch2d-dir", "dirichlet", (31, 20), "schnakenberg", SCH, (1.8, 1.8), (0.05, 1.0), 0.01,
        "schnak_noise", (0.0, 1.0)),
    _wl("sch3d-dir", "dirichlet", (11, 13, 17), "schnakenberg", SCH, (1.8, 1.8), (0.05, 1.0),
        0.01, "schnak_noise", (0.0, 1.0)),
    _wl("sch3d-neu", "neumann", (9, 12, 10), "schnakenberg", SCH, (1.5, 1.2), (0.05, 1.0),
        0.005, "schnak_noise", (0.0, 1.0)),
    _wl("gs3d-per", "periodic", (8, 10, 12), "gray_scott", GS, (1.7, 1.9), (2e-3, 1e-3), 0.5,
        "gs_square", (-1.0, 1.0)),
]
IDS = [c.name for c in CASES]

# Shapes that take the FP32 vector tile paths: x tiles of 32 lines with
# n_x in {64, 128, 256}; strided axes with 32-lane tiles and 64 | n; the
# per-stage Z kernels (last axes of 64 to 256 points, L formed in the kernel).
VEC_CASES = [
    _wl("sch3d-neu-vec", "neumann", (256, 32, 64), "schnakenberg", SCH, (1.5, 1.2), (0.05, 1.0),
        0.005, "schnak_noise", (0.0, 1.0)),
    _wl("sch3d-dir-vec", "dirichlet", (64, 64, 128), "schnakenberg", SCH, (1.8, 1.8),
        (0.05, 1.0), 0.01, "schnak_noise", (0.0, 1.0)),
    _wl("gm2d-neu-vec", "neumann", (256, 128), "gierer_meinhardt", GM, (1.6, 1.4), (1e-3, 0.05),
        0.05, "gm_noise", (0.0, 2.0)),
    _wl("gs3d-per-vec", "periodic", (64, 64, 64), "gray_scott", GS, (1.7, 1.9), (2e-3, 1e-3), 0.5,
        "gs_square", (-1.0, 1.0)),
    # per-stage Z kernels on last axes of 128 and 192 points
    _wl("sch3d-dir-vec128", "dirichlet", (128, 32, 64), "schnakenberg", SCH, (1.8, 1.6),
        (0.05, 1.0), 0.01, "schnak_noise", (0.0, 1.0)),
    _wl("sch3d-neu-vec192", "neumann", (192, 32, 64), "schnakenberg", SCH, (1.5, 1.2),
        (0.05, 1.0), 0.005, "schnak_noise", (0.0, 1.0)),
]
VEC_IDS = [c.name for c in VEC_CASES]


@pytest.mark.parametrize("scheme", ["p13", "exp"])
@pytest.mark.parametrize("wl", CASES, ids=IDS)
def test_fp64_matches_oracle(wl, scheme):
    wl = wl.replace(scheme=scheme)
    u0 = W.initial_fields(wl)
    ref = problem.run(wl, u0, 5)
    got = run(wl, u0, 5, "f64")
    assert problem.rel_err(got, ref) <= 1e-10


@pytest.mark.parametrize("wl", CASES, ids=IDS)
def test_fp32_matches_oracle(wl):
    u0 = W.initial_fields(wl)
    ref = problem.run(wl, u0, 5)
    got = run(wl, u0, 5, "f32")
    assert problem.rel_err(got, ref) <= 2e-5


@pytest.mark.parametrize("scheme", ["p13", "exp"])
@pytest.mark.parametrize("wl", VEC_CASES, ids=VEC_IDS)
def test_fp32_vector_paths_match_oracle(wl, scheme):
    wl = wl.replace(scheme=scheme)
    u0 = W.initial_fields(wl)
    ref = oracle_run(wl, 5)
    got = run(wl, u0, 5, "f32")
    assert problem.rel_err(got, ref) <= 2e-5


# The FP64 engine moves full tiles through registers (x axes of 64, 128 or
# 256 points; strided axes of multiples of 64, with one or both species per
# tile); an x axis of 192 points takes its generic in-place loads.
X192 = _wl("sch2d-neu-x192", "neumann", (64, 192), "schnakenberg", SCH, (1.5, 1.2), (0.05, 1.0),
           0.005, "schnak_noise", (0.0, 1.0))
F64_TILE_CASES = VEC_CASES + [X192]


@pytest.mark.parametrize("scheme", ["p13", "exp"])
@pytest.mark.parametrize("wl", F64_TILE_CASES, ids=[c.name for c in F64_TILE_CASES])
def test_fp64_register_tile_paths_match_oracle(wl, scheme):
    wl = wl.replace(scheme=scheme)
    u0 = W.initial_fields(wl)
    ref = oracle_run(wl, 5)
    got = run(wl, u0, 5, "f64")
    assert problem.rel_err(got, ref) <= 1e-10


def test_fp32_x_axis_of_192_points_matches_oracle():
    u0 = W.initial_fields(X192)
    ref = problem.run(X192, u0, 5)
    assert problem.rel_err(run(X192, u0, 5, "f32"), ref) <= 2e-5


# One species on x axes the vector paths take (64, 128, 256 points,
# non-periodic): the x-axis transforms before and after the steps run on
# tiles of that one species.
ONE_SPECIES_CASES = [
    _wl("lin1-neu-x256", "neumann", (32, 256), "linear", (-0.5,), (1.6,), (1e-3,), 0.5,
        "normal", (0.0, 1.0)),
    _wl("lin1-dir-x128", "dirichlet", (8, 32, 128), "linear", (0.25,), (1.8,), (2e-3,), 0.2,
        "normal", (0.0, 1.0)),
]


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 2e-5)])
@pytest.mark.parametrize("wl", ONE_SPECIES_CASES, ids=[c.name for c in ONE_SPECIES_CASES])
def test_one_species_on_vector_x_axes_matches_oracle(wl, dtype, tol):
    u0 = W.initial_fields(wl)
    ref = problem.run(wl, u0, 5)
    assert problem.rel_err(run(wl, u0, 5, dtype), ref) <= tol


# The engine's paths are chosen by precision, species count, boundary
# condition and axis lengths: the linear reaction (any species count) on a
# 2D grid with x = 128 and y = 64 points, a 3D one with 64-point x and y
# axes, and 1D grids of 256 points (matrix cores) and 1024 (FFT for the
# periodic one, dense kernels otherwise), for one to three species and every
# boundary condition.
def _lin(S, bc, shape):
    return _wl(f"lin{S}-{bc[:3]}-{'x'.join(map(str, shape))}", bc, shape, "linear",
               (-0.5, 0.25, -1.0)[:S], (1.6, 1.8, 1.2)[:S], (1e-3, 2e-3, 5e-4)[:S], 0.3,
               "normal", (0.0, 1.0))


PATH_MATRIX = [_lin(S, bc, shape) for shape in ((64, 128), (32, 64, 64), (256,), (1024,))
               for bc in ("neumann", "dirichlet", "periodic") for S in (1, 2, 3)]


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 2e-5)])
@pytest.mark.parametrize("wl", PATH_MATRIX, ids=[c.name for c in PATH_MATRIX])
def test_species_count_and_boundary_matrix_matches_oracle(wl, dtype, tol):
    u0 = W.initial_fields(wl)
    ref = problem.run(wl, u0, 4)
    assert problem.rel_err(run(wl, u0, 4, dtype), ref) <= tol


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-13), ("f32", 1e-6)])
def test_fields_off_16_byte_boundaries_match_aligned_ones(dtype, tol):
    """A caller's field 8 (FP64) or 4 (FP32) bytes past a 16-byte boundary:
    the launches that read or write it take the element-wise tile paths
    instead of the 16-byte vector ones, with the same arithmetic."""
    wl = VEC_CASES[1]  # every axis on the vector / register tile paths
    u0 = W.initial_fields(wl)
    p = plan_for(wl, dtype, None)
    a = torch.tensor(u0, dtype=TD[dtype], device="cuda")
    big = torch.zeros(a.numel() + 1, dtype=TD[dtype], device="cuda")
    b = big[1:].view(a.shape)
    b.copy_(a)
    assert b.data_ptr() % 16 != 0
    p.integrate(a, 3, 0.0)
    p.integrate(b, 3, 0.0)
    torch.cuda.synchronize()
    got, ref = b.double().cpu().numpy(), a.double().cpu().numpy()
    p.close()
    assert problem.rel_err(got, ref) <= tol
    assert problem.rel_err(ref, problem.run(wl, u0, 3)) <= (1e-10 if dtype == "f64" else 2e-5)


# Axes the matrix-core engine and the FFT kernels do not take (n > 256, and
# periodic n >= 256 that is not 256, 512 or 1024) run the dense LDS kernels,
# with tiles narrowed to fill the device.
DENSE_CASES = [
    _wl("gs2d-per-dense", "periodic", (24, 300), "gray_scott", GS, (1.7, 1.7), (2e-3, 1e-3), 1.0,
        "gs_square", (-1.0, 1.0)),
    _wl("sch2d-dir-dense", "dirichlet", (270, 20), "schnakenberg", SCH, (1.8, 1.6), (0.05, 1.0),
        0.01, "schnak_noise", (0.0, 1.0)),
]


@pytest.mark.parametrize("scheme", ["p13", "exp"])
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 2e-5)])
@pytest.mark.parametrize("wl", DENSE_CASES, ids=[c.name for c in DENSE_CASES])
def test_dense_axes_match_oracle(wl, dtype, tol, scheme):
    wl = wl.replace(scheme=scheme)
    u0 = W.initial_fields(wl)
    ref = problem.run(wl, u0, 5)
    assert problem.rel_err(run(wl, u0, 5, dtype), ref) <= tol


# Long periodic axes of 256, 512 and 1024 points take the FFT kernels: on x
# (every species per tile), on the middle and last axes (one species per
# tile), with ragged partners, and with an odd line count per tile (three
# species, one x line per tile).
FFT_CASES = [
    _wl("gs2d-per-fft-x", "periodic", (24, 512), "gray_scott", GS, (1.7, 1.5), (2e-3, 1e-3), 1.0,
        "gs_square", (-1.0, 1.0)),
    _wl("gs2d-per-fft-y", "periodic", (256, 40), "gray_scott", GS, (1.7, 1.9), (2e-3, 1e-3), 1.0,
        "gs_square", (-1.0, 1.0)),
    _wl("sch3d-per-fft-mid", "periodic", (6, 256, 10), "schnakenberg", SCH, (1.8, 1.6),
        (0.05, 1.0), 0.01, "schnak_noise", (0.0, 1.0)),
    _wl("sch3d-per-fft-xz", "periodic", (512, 3, 256), "schnakenberg", SCH, (1.5, 1.2),
        (0.05, 1.0), 0.01, "schnak_noise", (0.0, 1.0)),
    _wl("lin3-per-fft-x", "periodic", (5, 512), "linear", (-0.5, 0.25, -1.0), (1.6, 1.8, 1.2),
        (1e-3, 2e-3, 5e-4), 0.5, "normal", (0.0, 1.0)),
    # one species: x tiles of two lines, strided tiles of four
    _wl("lin1-per-fft-x", "periodic", (6, 1024), "linear", (-0.5,), (1.6,), (1e-3,), 0.5,
        "normal", (0.0, 1.0)),
    _wl("lin1-per-fft-y", "periodic", (256, 12), "linear", (0.25,), (1.8,), (2e-3,), 0.5,
        "normal", (0.0, 1.0)),
]


@pytest.mark.parametrize("scheme", ["p13", "exp"])
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 2e-5)])
@pytest.mark.parametrize("wl", FFT_CASES, ids=[c.name for c in FFT_CASES])
def test_fft_axes_match_oracle(wl, dtype, tol, scheme):
    wl = wl.replace(scheme=scheme)
    u0 = W.initial_fields(wl)
    ref = problem.run(wl, u0, 5)
    assert problem.rel_err(run(wl, u0, 5, dtype), ref) <= tol


# The benchmark configurations at their full sizes, a few steps.
FULL = [W.C2_GS, W.C3_SCHNAK_DIR, W.C4_GM_ADJ]


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 2e-5)])
@pytest.mark.parametrize("wl", FULL, ids=[c.name for c in FULL])
def test_configs_full_size_match_oracle(wl, dtype, tol):
    u0 = W.initial_fields(wl)
    ref = problem.run(wl, u0, 3)
    assert problem.rel_err(run(wl, u0, 3, dtype), ref) <= tol


# The paper's own applications (Section 5.2) at its grids, constants and
# deterministic initial data; GM with different orders per species.
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 2e-5)])
@pytest.mark.parametrize("wl", W.PAPER, ids=[c.name for c in W.PAPER])
def test_paper_applications_match_oracle(wl, dtype, tol):
    u0 = W.initial_fields(wl)
    ref = problem.run(wl, u0, 5)
    assert problem.rel_err(run(wl, u0, 5, dtype), ref) <= tol


_C5_REF = {}


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 2e-5)])
def test_config5_full_size_one_step_matches_oracle(dtype, tol):
    # 3D Schnakenberg Neumann 256^3 (the benchmark workload), one step; the
    # oracle's step takes seconds on the host cores.
    wl = W.C5_SCHNAK_NEU
    u0 = W.initial_fields(wl)
    if "ref" not in _C5_REF:
        _C5_REF["ref"] = problem.run(wl, u0, 1)
    assert problem.rel_err(run(wl, u0, 1, dtype), _C5_REF["ref"]) <= tol


@pytest.mark.parametrize("wl,alpha,nsteps", [(W.C2_GS, 1.7, 500), (W.C3_SCHNAK_DIR, 1.8, None),
                                             (W.C5_SCHNAK_NEU, 1.2, None),
                                             (W.C5_SCHNAK_NEU, 1.9, None)],
                         ids=["c2-500", "c3-500", "c5-a1.2-1000", "c5-a1.9-1000"])
def test_fp32_full_horizon_matches_fp64_gpu(wl, alpha, nsteps):
    # FP32 against the FP64 GPU path (itself pinned to the oracle above) over
    # the configuration's whole horizon. The Gray-Scott run forms spots that
    # amplify any perturbation: an FP64 run whose state is rounded to FP32
    # once per step leaves FP64 by 2.9e-5 after its 2000 steps (6e-7 after
    # 500), so no FP32 computation holds 2e-5 over the full horizon; it is
    # held to it over 500 steps.
    wl = wl.replace(alpha=(alpha, alpha))
    nsteps = nsteps or wl.nsteps
    u0 = W.initial_fields(wl)
    a = run(wl, u0, nsteps, "f32")
    b = run(wl, u0, nsteps, "f64")
    assert problem.rel_err(a, b) <= 2e-5


# The largest axes a plan accepts (1024 unknowns), on each kind of axis:
# contiguous x, strided middle and strided last (dense kernels; periodic x on
# the FFT kernels), ragged partners on the other axes.
MAX_CASES = [
    _wl("max2d-neu", "neumann", (1024, 700), "gray_scott", GS, (1.7, 1.5), (2e-3, 1e-3), 0.5,
        "gs_square", (-1.0, 1.0)),
    _wl("max3d-dir-z", "dirichlet", (1024, 6, 5), "schnakenberg", SCH, (1.8, 1.6), (0.05, 1.0),
        0.01, "schnak_noise", (0.0, 1.0)),
    _wl("max3d-per-x", "periodic", (5, 6, 1024), "schnakenberg", SCH, (1.8, 1.6), (0.05, 1.0),
        0.01, "schnak_noise", (0.0, 1.0)),
]


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 2e-5)])
@pytest.mark.parametrize("wl", MAX_CASES, ids=[c.name for c in MAX_CASES])
def test_largest_axes_match_oracle(wl, dtype, tol):
    u0 = W.initial_fields(wl)
    ref = problem.run(wl, u0, 2)
    assert problem.rel_err(run(wl, u0, 2, dtype), ref) <= tol


def test_linear_reaction_many_species():
    wl = W.Workload(name="lin4", bc="dirichlet", shape=(14, 19), domain=(0.0, 1.0),
                    alpha=(1.2, 1.5, 1.8, 2.0), kappa=(0.01, 0.02, 0.0, 0.05),
                    reaction="linear", params=(0.3, -0.2, 1.0, 0.0), dt=0.02, nsteps=4, seed=3,
                    init="normal", extra={"mean": [0.5, 0.4, 0.3, 0.2], "sd": 0.2})
    u0 = W.initial_fields(wl)
    ref = problem.run(wl, u0, 4)
    assert problem.rel_err(run(wl, u0, 4, "f64"), ref) <= 1e-10


def test_config1_fhn_full_size_fp64():
    # 2D FitzHugh-Nagumo, Neumann, 64x64, FP64, 100 steps of dt = 0.1.
    wl = W.C1_FHN
    u0 = W.initial_fields(wl)
    ref = problem.run(wl, u0, wl.nsteps)
    got = run(wl, u0, wl.nsteps, "f64")
    assert problem.rel_err(got, ref) <= 1e-10


@pytest.mark.parametrize("bc", ["periodic", "dirichlet", "neumann"])
def test_minimum_grid_two_unknowns(bc):
    wl = _wl("tiny", bc, (2, 3), "schnakenberg", SCH, (1.5, 1.5), (0.05, 1.0), 0.01,
             "schnak_noise", (0.0, 1.0))
    u0 = W.initial_fields(wl)
    ref = problem.run(wl, u0, 3)
    assert problem.rel_err(run(wl, u0, 3, "f64"), ref) <= 1e-10


def test_zero_steps_leave_state_untouched():
    wl = CASES[0]
    u0 = W.initial_fields(wl)
    p = plan_for(wl, "f64")
    u = torch.tensor(u0, dtype=torch.float64, device="cuda")
    p.integrate(u, 0)
    torch.cuda.synchronize()
    assert np.array_equal(u.cpu().numpy(), u0)
    p.close()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("wl", [CASES[4], VEC_CASES[1], FFT_CASES[1]],
                         ids=["small", "vector-paths", "fft"])
def test_runs_are_bitwise_deterministic(wl, dtype):
    u0 = W.initial_fields(wl)
    a = run(wl, u0, 6, dtype)
    b = run(wl, u0, 6, dtype)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("wl", [CASES[2], VEC_CASES[1], FFT_CASES[1]],
                         ids=["small", "vector-paths", "fft"])
def test_resume_from_checkpoint_is_bitwise_identical(dtype, wl):
    u0 = W.initial_fields(wl)
    p = plan_for(wl, dtype)
    u = torch.tensor(u0, dtype=TD[dtype], device="cuda")
    ckpt = p.integrate(u, 9, 0.0, ckpt_every=3)
    v = torch.tensor(u0, dtype=TD[dtype], device="cuda")
    p.resume(ckpt, 1, v, 6, t0=3 * wl.dt)
    torch.cuda.synchronize()
    assert torch.equal(u, v)
    p.close()


@pytest.mark.parametrize("bc", ["periodic", "dirichlet", "neumann"])
def test_single_eigenmode_decays_by_R13_power(bc):
    # f = 0: M steps multiply an eigenmode by R13(L)^M (closed form).
    ny, nx, tau, kappa, alpha, M = 10, 12, 0.02, 0.7, 1.3, 7

    def mode(n, k):
        jj = np.arange(n)
        if bc == "periodic":
            return np.cos(2 * np.pi * k * jj / n), np.sin(np.pi * k / n)
        if bc == "dirichlet":
            N = n + 1
            return np.sin(np.pi * (jj + 1) * k / N), np.sin(np.pi * k / (2 * N))
        N = n - 1
        return np.cos(np.pi * jj * k / N), np.sin(np.pi * k / (2 * N))

    wl = W.Workload(name="mode", bc=bc, shape=(ny, nx), domain=(0.0, 1.0), alpha=(alpha,),
                    kappa=(kappa,), reaction="linear", params=(0.0,), dt=tau, nsteps=M, seed=0,
                    init="normal")
    hy, hx = wl.h
    my, sy = mode(ny, 2)
    mx, sx = mode(nx, 3)
    lam = sum(4 * s * s / (hh * hh * (1 - s * s / 3)) for s, hh in ((sy, hy), (sx, hx)))
    L = kappa * tau * lam ** (alpha / 2)
    R = (24 - 6 * L) / (24 + 18 * L + 6 * L ** 2 + L ** 3)
    u0 = np.outer(my, mx)[None]
    p = plan_for(wl, "f64")
    got = run(wl, u0, M, "f64", plan=p)
    p.close()
    assert np.max(np.abs(got - R ** M * u0)) <= 1e-12


@pytest.mark.parametrize("bc", ["periodic", "neumann"])
@pytest.mark.parametrize("dtype,tol", [("f32", 1e-6), ("f64", 1e-13)])
def test_mean_mode_is_not_damped(bc, dtype, tol):
    # f = 0 and a constant field: L = 0 on the constant mode, where R13 = 1
    # exactly (Section 4), so the field stays constant over any number of
    # steps. A multiplier off by one rounding of 1 would drift by 500 ulps.
    wl = W.Workload(name="mean", bc=bc, shape=(20, 24, 28), domain=(0.0, 1.0), alpha=(1.5,),
                    kappa=(0.7,), reaction="linear", params=(0.0,), dt=0.005, nsteps=500, seed=0,
                    init="normal")
    c = 0.9359
    u0 = np.full((1,) + wl.shape, c)
    got = run(wl, u0, wl.nsteps, dtype)
    assert np.max(np.abs(got - c)) <= tol * c


def test_nonfinite_reaction_is_reported():
    wl = CASES[2]
    u0 = W.initial_fields(wl)
    # Gierer-Meinhardt u^2/v with v = 0. The whole field is zeroed: the
    # initial fields pass through the spectral state, which returns zeros
    # exactly but not an isolated zero among non-zeros.
    u0[1] = 0.0
    p = plan_for(wl, "f64")
    u = torch.tensor(u0, dtype=torch.float64, device="cuda")
    with pytest.raises(C.SfrdeError) as ei:
        p.integrate(u, 2)
    assert ei.value.code == C.ENONFINITE
    # the plan stays usable
    u = torch.tensor(W.initial_fields(wl), dtype=torch.float64, device="cuda")
    p.integrate(u, 1)
    p.close()


def test_nonfinite_reaction_is_reported_after_many_steps():
    wl = CASES[2]
    u0 = W.initial_fields(wl)
    u0[1] = 0.0
    p = plan_for(wl, "f64")
    u = torch.tensor(u0, dtype=torch.float64, device="cuda")
    with pytest.raises(C.SfrdeError) as ei:
        p.integrate(u, 20)
    assert ei.value.code == C.ENONFINITE
    p.close()


def test_null_state_is_rejected_on_a_live_plan():
    p = plan_for(CASES[0], "f64")
    assert C.lib().sfrde_integrate(p.handle, None, 1, 0.0, 0, None) == C.EINVAL
    p.close()


# 1D plans (run as 2D plans with a one-point padding axis) for every boundary
# condition, two species with different orders, forward and adjoint.
ONE_D = [
    W.Workload(name=f"sch1d-{bc}", bc=bc, shape=(n,), domain=(0.0, 1.0), alpha=(1.6, 1.3),
               kappa=(0.01, 0.1), reaction="schnakenberg", params=SCH, dt=0.01, nsteps=5,
               seed=5, init="normal", extra={"mean": [0.9, 0.9], "sd": 0.05})
    for bc, n in (("periodic", 50), ("dirichlet", 63), ("neumann", 257))
]


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 2e-5)])
@pytest.mark.parametrize("wl", ONE_D, ids=[c.name for c in ONE_D])
def test_one_dimensional_plans_match_oracle(wl, dtype, tol):
    u0 = W.initial_fields(wl)
    ref = problem.run(wl, u0, 5)
    assert problem.rel_err(run(wl, u0, 5, dtype), ref) <= tol


@pytest.mark.parametrize("wl", ONE_D, ids=[c.name for c in ONE_D])
def test_one_dimensional_adjoint_matches_oracle(wl):
    u0 = W.initial_fields(wl)
    wbar = np.random.default_rng(21).standard_normal(u0.shape)
    ref = problem.gradients(wl, u0, 5, wbar)
    p = plan_for(wl, "f64")
    u = torch.tensor(u0, dtype=torch.float64, device="cuda")
    ck = p.integrate(u, 5, 0.0, ckpt_every=2)
    g0 = torch.empty_like(u)
    gk, ga, gp = p.backward(ck, 5, 2, torch.tensor(wbar, device="cuda"), 0.0, g0)
    torch.cuda.synchronize()
    p.close()
    assert problem.rel_err(g0.cpu().numpy(), ref["u0"]) <= 1e-10
    for key, got in (("kappa", gk), ("alpha", ga), ("params", gp)):
        r = ref[key]
        assert np.max(np.abs(np.array(got) - r)) <= 1e-10 * max(np.max(np.abs(r)), 1e-300), key


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 2e-6)])
@pytest.mark.parametrize("wl", [CASES[1], VEC_CASES[1], FFT_CASES[1]],
                         ids=["small", "vector-paths", "fft"])
def test_single_steps_match_integrate(wl, dtype, tol):
    # sfrde_step is one step from physical data (forward transforms of the
    # state each call): k calls agree with one k-step integrate to rounding,
    # and a step at time t equals a one-step integrate from t0 = t.
    u0 = W.initial_fields(wl)
    p = plan_for(wl, dtype)
    a = torch.tensor(u0, dtype=TD[dtype], device="cuda")
    b = a.clone()
    for k in range(4):
        p.step(a, k * wl.dt)
    p.integrate(b, 4, 0.0)
    torch.cuda.synchronize()
    assert problem.rel_err(a.double().cpu().numpy(), b.double().cpu().numpy()) <= tol
    p.close()


def test_single_step_at_time_t_is_a_one_step_integrate_from_t():
    h = 1.0 / 20
    pm = Plan((20, 20), "periodic", (h, h), (1.5,), (1.0,), 0.1 * h, "huxley_mms", (), "f64")
    x = torch.zeros((1, 20, 20), dtype=torch.float64, device="cuda")
    y = x.clone()
    pm.step(x, 0.3)
    pm.integrate(y, 1, 0.3)
    torch.cuda.synchronize()
    assert torch.equal(x, y)
    pm.close()


def test_checkpoint_and_workspace_sizes():
    wl = CASES[6]
    p = plan_for(wl, "f32")
    field = wl.nspecies * wl.npoints * 4
    assert p.ckpt_bytes(10, 3) == C.CKPT_HEADER_BYTES + 4 * field
    assert p.ckpt_bytes(9, 3) == C.CKPT_HEADER_BYTES + 3 * field
    assert p.workspace_bytes() >= 4 * field  # P, u_hat, c_tilde, acc at least
    with pytest.raises(C.SfrdeError):
        p.ckpt_bytes(10, 0)
    p.close()
