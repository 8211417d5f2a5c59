#!/usr/bin/env python3
"""Benchmark of the fractional ETDRK4 step on one MI355X.

Workload (default): 3D Schnakenberg, homogeneous Neumann (DCT-I basis), 256^3
unknowns, two species, alpha = 1.5, kappa = (0.05, 1.0), dt = 0.005, the
paper's ETDRK4-P13 coefficients, seeded synthetic initial fields.

Reported on one JSON line:
* value: FP32 point-steps per second (Mpoint-steps/s; a point advances all
  species) over the timed steps, inputs resident in HBM;
* fp64: the same for the FP64 path on the same GPU;
* error: FP32 vs FP64 GPU after the same steps (max over species of the
  relative max-norm error);
* adjoint: backward (recompute from checkpoints + adjoint sweep, gradients
  w.r.t. u0, kappa, alpha, reaction parameters) over forward time;
* roofline: the dominant kernel's algorithmic bytes per launch over its mean
  launch time (HIP events around every launch on the plan's stream);
* cpu_baseline: the FP64 CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def src_hash() -> str:
    h = hashlib.sha256()
    cdir = os.path.join(ROOT, "paper_2003_13569_amd", "csrc")
    for name in sorted(os.listdir(cdir)):
        with open(os.path.join(cdir, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(cls: str, S: int, n: int, w: int) -> float:
    """Bytes one launch of a kernel class must move (tables excluded).

    X and Y read and write every species' field once. Z does the same and
    also touches the retained spectral arrays: 3, 3, 3 and 2 accesses in the
    four stages (u_hat, c_til, acc), 2.75 on average.
    """
    f = float(S) * n * w
    if cls in ("X", "Y"):
        return 2.0 * f
    if cls == "Z":
        return (2.0 + 2.75) * f
    raise ValueError(cls)


def bytes_per_point_step(ndim: int, S: int, w: int) -> float:
    return float(S * w * (16 * (ndim - 1) + 11))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--alpha", type=float, default=1.5)
    ap.add_argument("--fp64-steps", type=int, default=20)
    ap.add_argument("--adjoint-steps", type=int, default=16)
    ap.add_argument("--adjoint-ckpt", type=int, default=4)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (PMC scaling)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU design is described, not built).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1

    if args.copy_calibration:
        nbytes = 1 << 30
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "launches": 5}), flush=True)
        return 0

    import workloads as W
    from paper_2003_13569_amd import sfrde as C
    from paper_2003_13569_amd.torch_api import Plan

    C.lib()  # fails loudly if the HIP library is missing

    wl = W.C5_SCHNAK_NEU.replace(alpha=(args.alpha, args.alpha))
    S, n = wl.nspecies, wl.npoints
    print(f"[bench] workload {wl.name} shape={wl.shape} alpha={args.alpha} "
          f"steps={args.steps} warmup={args.warmup}", flush=True)
    u0 = W.initial_fields(wl)

    def make(dtype):
        return Plan(wl.shape, wl.bc, wl.h, wl.alpha, wl.kappa, wl.dt, wl.reaction, wl.params,
                    dtype, wl.scheme)

    def timed(plan, dtype, steps, warmup, profile):
        td = torch.float32 if dtype == "f32" else torch.float64
        u = torch.tensor(u0, dtype=td, device="cuda")
        if warmup:
            w = u.clone()
            plan.integrate(w, warmup)
            del w
        torch.cuda.synchronize()
        if profile:
            C.sfrde_profile(plan.handle, 16 * steps + 64)
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        plan.integrate(u, steps)
        stop.record()
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop)
        prof = None
        if profile:
            prof = C.sfrde_profile_read(plan.handle)
            C.sfrde_profile(plan.handle, 0)
        return u, ms, prof

    # ---------------------------------------------------------------- FP32
    p32 = make("f32")
    u32, ms32, prof = timed(p32, "f32", args.steps, args.warmup, profile=True)
    ms_step = ms32 / args.steps
    value = n * args.steps / (ms32 * 1e-3) / 1e6
    print(f"[bench] fp32: {ms_step:.3f} ms/step, {value:.1f} Mpoint-steps/s", flush=True)

    # dominant forward kernel and its roofline
    w32 = 4
    dom, dom_ms = None, -1.0
    for cls in ("X", "Y", "Z"):
        t, cnt = prof[cls]
        if cnt and t > dom_ms:
            dom, dom_ms = cls, t
    t_dom, n_dom = prof[dom]
    avg_ms = t_dom / n_dom
    achieved = algorithmic_bytes(dom, S, n, w32) / (avg_ms * 1e-3) / 1e9
    kernel_names = {"X": "k_xstage<float>", "Y": "k_single<float>", "Z": "k_zstage<float>"}
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"traffic_{dom}_{wl.name}_f32.json")
    if os.path.exists(tfile):
        with open(tfile) as fh:
            tj = json.load(fh)
        if tj.get("src_hash") == src_hash():
            traffic = tj.get("hbm_bytes_per_launch")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kernel_names[dom], "avg_launch_ms": round(avg_ms, 4),
                "launches": n_dom,
                "algorithmic_bytes_per_launch": algorithmic_bytes(dom, S, n, w32)}
    kernels = {k: {"ms_total": round(v[0], 3), "launches": v[1],
                   "avg_ms": round(v[0] / v[1], 4) if v[1] else None}
               for k, v in prof.items() if v[1]}
    step_gbs = bytes_per_point_step(wl.ndim, S, w32) * n / (ms_step * 1e-3) / 1e9

    # ---------------------------------------------------------------- FP64 + error
    fp64 = None
    err = None
    if not args.no_fp64:
        p64 = make("f64")
        k64 = args.fp64_steps
        u64, ms64, _ = timed(p64, "f64", k64, 1, profile=False)
        v64 = n * k64 / (ms64 * 1e-3) / 1e6
        fp64 = {"value": round(v64, 2), "unit": "Mpoint-steps/s", "ms_per_step": round(ms64 / k64, 3),
                "steps": k64}
        print(f"[bench] fp64: {ms64 / k64:.3f} ms/step, {v64:.1f} Mpoint-steps/s", flush=True)
        # FP32 over the same steps from the same initial fields
        ue = torch.tensor(u0, dtype=torch.float32, device="cuda")
        p32.integrate(ue, k64)
        a = ue.double().cpu().numpy()
        b = u64.cpu().numpy()
        err = max(float(np.max(np.abs(a[s] - b[s])) / np.max(np.abs(b[s]))) for s in range(S))
        print(f"[bench] fp32 vs fp64 after {k64} steps: {err:.3e}", flush=True)
        p64.close()
        del u64

    # ---------------------------------------------------------------- adjoint
    adjoint = None
    if not args.no_adjoint:
        ka, kc = args.adjoint_steps, args.adjoint_ckpt
        u = torch.tensor(u0, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p32.integrate(u.clone(), ka)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        t0 = time.perf_counter()
        ckpt = p32.integrate(u, ka, 0.0, ckpt_every=kc)
        torch.cuda.synchronize()
        t_fwd_ck = time.perf_counter() - t0
        g = torch.full_like(u, 1.0 / u.numel())
        g0 = torch.empty_like(u)
        t0 = time.perf_counter()
        p32.backward(ckpt, ka, kc, g, 0.0, g0)
        torch.cuda.synchronize()
        t_bwd = time.perf_counter() - t0
        adjoint = {"steps": ka, "ckpt_every": kc, "forward_s": round(t_fwd, 4),
                   "forward_with_ckpt_s": round(t_fwd_ck, 4), "backward_s": round(t_bwd, 4),
                   "ratio": round(t_bwd / t_fwd, 3),
                   "workspace_gb": round(p32.workspace_bytes() / 1e9, 2)}
        print(f"[bench] adjoint/forward = {t_bwd / t_fwd:.2f}", flush=True)
        del ckpt, g, g0

    # ---------------------------------------------------------------- CPU oracle
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import problem
        try:
            from threadpoolctl import threadpool_info
            cores = max(i.get("num_threads", 1) for i in threadpool_info()) if threadpool_info() else os.cpu_count()
        except Exception:
            cores = os.cpu_count()
        sch = problem.scheme(wl)
        N = problem.nonlinearity(wl)
        t0 = time.perf_counter()
        sch.step(u0, 0.0, N)
        dt_cpu = time.perf_counter() - t0
        cpu = {"value": round(n / dt_cpu / 1e6, 4), "unit": "Mpoint-steps/s", "cores": cores,
               "kind": "oracle",
               "sample": f"1 step of the same {'x'.join(map(str, wl.shape))} workload "
                         f"({dt_cpu:.1f} s), FP64, per-axis LAPACK eigenbasis"}
        print(f"[bench] cpu oracle: {dt_cpu:.1f} s for 1 step", flush=True)

    out = {
        "metric": "ETDRK4 Mpoint-steps/s FP32 vs FP64 at stated error; adjoint/forward time ratio",
        "value": round(value, 2),
        "unit": "Mpoint-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "grid": list(wl.shape), "bc": wl.bc, "species": S,
                   "alpha": args.alpha, "kappa": list(wl.kappa), "dt": wl.dt,
                   "scheme": wl.scheme, "reaction": wl.reaction,
                   "config_steps": wl.nsteps},
        "fp64": fp64,
        "error": {"fp32_vs_fp64_gpu": err, "steps": args.fp64_steps} if err is not None else None,
        "adjoint": adjoint,
        "roofline": roofline,
        "step_effective_gbs": round(step_gbs, 1),
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
