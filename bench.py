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


KERNEL_CLASSES = (("k_zstage", "Z"), ("k_xstage", "X"), ("k_single", "Y"), ("k_zadj", "ZADJ"),
                  ("k_xadj", "XADJ"))


def kernel_class(name: str):
    base = name.split("(")[0]
    for key, cls in KERNEL_CLASSES:
        if ("sfrde::" + key + "_m<") in base or ("sfrde::" + key + "<") in base:
            return cls
    return None


def _pmc_per_dispatch(path: str, counter: str):
    """Counter value (KiB) of every dispatch in a rocprofv3 counter CSV: [(name, value)]."""
    import csv
    out = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] == counter:
                out.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return out


def summarize_pmc(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, out_json, workload):
    """HBM bytes per launch for each kernel class from FETCH_SIZE / WRITE_SIZE.

    Each counter is scaled by what it reads for a plain device copy of known
    size (bench.py --copy-calibration: 1 GiB read and 1 GiB written per copy;
    the largest dispatches of that run are the copies).
    """
    nb = float(1 << 30)
    cf = sorted(v for _, v in _pmc_per_dispatch(copy_fetch_csv, "FETCH_SIZE"))[-1]
    cw = sorted(v for _, v in _pmc_per_dispatch(copy_write_csv, "WRITE_SIZE"))[-1]
    f_scale, w_scale = nb / (cf * 1024.0), nb / (cw * 1024.0)
    res = {}
    for counter, path, scale in (("fetch", fetch_csv, f_scale), ("write", write_csv, w_scale)):
        name = "FETCH_SIZE" if counter == "fetch" else "WRITE_SIZE"
        for kname, v in _pmc_per_dispatch(path, name):
            cls = kernel_class(kname)
            if cls is None:
                continue
            d = res.setdefault(cls, {"fetch": [], "write": []})
            d[counter].append(v * 1024.0 * scale)
    summary = {"workload": workload, "src_hash": src_hash(), "fetch_scale": round(f_scale, 4),
               "write_scale": round(w_scale, 4), "classes": {}}
    for cls, d in res.items():
        fb = sum(d["fetch"]) / max(len(d["fetch"]), 1)
        wb = sum(d["write"]) / max(len(d["write"]), 1)
        summary["classes"][cls] = {"launches": len(d["fetch"]), "fetch_bytes": round(fb),
                                   "write_bytes": round(wb), "hbm_bytes_per_launch": round(fb + wb)}
    with open(out_json, "w") as fh:
        json.dump(summary, fh, indent=1)
    print(json.dumps(summary, indent=1))


def summarize_stats(stats_csv):
    """Markdown table of a rocprofv3 --stats kernel summary, grouped by class."""
    import csv
    rows = []
    with open(stats_csv) as fh:
        for r in csv.DictReader(fh):
            rows.append((r["Name"], int(r["Calls"]), float(r["TotalDurationNs"]),
                         float(r["AverageNs"]), float(r["Percentage"])))
    rows.sort(key=lambda r: -r[2])
    print("| Kernel | Class | Calls | Avg (ms) | Total (ms) | Share |")
    print("|---|---|---|---|---|---|")
    for name, calls, tot, avg, pct in rows:
        short = name.split("(")[0].replace("sfrde::", "")
        print(f"| `{short}` | {kernel_class(name) or '-'} | {calls} | {avg / 1e6:.4f} | "
              f"{tot / 1e6:.3f} | {pct:.1f} % |")


def cpu_fast_alg1(wl, u0, nsteps, workers):
    """Alg. 1 on the host in FP64 with scipy.fft, all host cores: the
    fast-transform CPU counterpart of the paper's own implementation (MATLAB
    fftn/ifftn on a CPU), timed beside the oracle. A timing reference, not an
    oracle: per step and species, four forward and four inverse d-dimensional
    transforms (DCT-I for Neumann, DST-I for Dirichlet, FFT for periodic), the
    P13 coefficients (Section 4) of L = kappa tau Lambda^(alpha/2) with the
    compact eigenvalues of Section 3.1, the retained-spectral-state schedule of
    the GPU path, and the workload's reaction. Returns (fields, seconds per
    step)."""
    import numpy as np
    import scipy.fft as sf

    assert wl.reaction == "schnakenberg"
    axes = tuple(range(wl.ndim))
    if wl.bc == "neumann":
        fwd = lambda x: sf.dctn(x, type=1, axes=axes, workers=workers)  # noqa: E731
        inv = lambda x: sf.idctn(x, type=1, axes=axes, workers=workers)  # noqa: E731
    elif wl.bc == "dirichlet":
        fwd = lambda x: sf.dstn(x, type=1, axes=axes, workers=workers)  # noqa: E731
        inv = lambda x: sf.idstn(x, type=1, axes=axes, workers=workers)  # noqa: E731
    else:
        fwd = lambda x: sf.fftn(x, axes=axes, workers=workers)  # noqa: E731
        inv = lambda x: sf.ifftn(x, axes=axes, workers=workers).real  # noqa: E731
    lam = 0.0
    for ax, (n, h) in enumerate(zip(wl.shape, wl.h)):
        if wl.bc == "neumann":
            k, N = np.arange(n), n - 1
            s = np.sin(k * np.pi / (2 * N))
        elif wl.bc == "dirichlet":
            k, N = np.arange(1, n + 1), n + 1
            s = np.sin(k * np.pi / (2 * N))
        else:
            k = np.arange(n)
            s = np.sin(k * np.pi / n)
        l1 = 4 * s * s / (h * h * (1 - s * s / 3))
        shape = [1] * wl.ndim
        shape[ax] = n
        lam = lam + l1.reshape(shape)
    tau = wl.dt
    co = []
    for a, kap in zip(wl.alpha, wl.kappa):
        L = kap * tau * np.where(lam > 0, lam, 1.0) ** (0.5 * a) * (lam > 0)
        D = 24 + L * (18 + L * (6 + L))
        Dh = 192 + L * (72 + L * (12 + L))
        co.append(dict(R=(24 - 6 * L) / D, Q=24 * (8 - L) / Dh, ph=tau * (96 + L * (12 + L)) / Dh,
                       p1=tau * (4 - L) / D, p2=tau * (8 + 2 * L) / D,
                       p3=tau * (4 + L * (3 + L)) / D))
    g, a_, b_ = wl.params

    def rxn(u):
        u2v = u[0] * u[0] * u[1]
        return np.stack([g * (a_ - u[0] + u2v), g * (b_ - u2v)])

    def F(x):
        return np.stack([fwd(x[s]) for s in range(2)])

    def Fi(x):
        return np.stack([inv(x[s]) for s in range(2)])

    def c(name):
        return np.stack([co[s][name] for s in range(2)])

    R, Q, ph, p1, p2, p3 = (c(k) for k in ("R", "Q", "ph", "p1", "p2", "p3"))
    uh = F(u0)
    t0 = None
    for step in range(nsteps + 1):
        if step == 1:
            t0 = time.perf_counter()  # the first step is a warm-up
        fu = F(rxn(Fi(uh)))
        ah = Q * uh + ph * fu
        ct = Q * ah - ph * fu
        acc = R * uh + p1 * fu
        fa = F(rxn(Fi(ah)))
        bh = Q * uh + ph * fa
        acc = acc + p2 * fa
        fb = F(rxn(Fi(bh)))
        ch = ct + 2 * ph * fb
        acc = acc + p2 * fb
        fc = F(rxn(Fi(ch)))
        uh = acc + p3 * fc
    dt_step = (time.perf_counter() - t0) / nsteps
    return Fi(uh), dt_step


def time_configs(W, Plan, torch, time):
    """The remaining benchmark configurations at their full sizes (context for
    the headline; each is also a parity test case): ms per step."""
    configs = {}
    for c, dt_c, kc in ((W.C1_FHN, "f64", 200), (W.C2_GS, "f32", 100), (W.C2_GS, "f64", 50),
                        (W.C3_SCHNAK_DIR, "f32", 50), (W.C3_SCHNAK_DIR, "f64", 20),
                        (W.C4_GM_ADJ, "f32", 100)):
        pc = Plan(c.shape, c.bc, c.h, c.alpha, c.kappa, c.dt, c.reaction, c.params, dt_c,
                  c.scheme)
        uc = torch.tensor(W.initial_fields(c), dtype=torch.float32 if dt_c == "f32"
                          else torch.float64, device="cuda")
        pc.integrate(uc.clone(), 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pc.integrate(uc, kc)
        torch.cuda.synchronize()
        msc = (time.perf_counter() - t0) * 1e3 / kc
        configs[f"{c.name}_{dt_c}"] = {
            "ms_per_step": round(msc, 4), "steps": kc,
            "Mpoint_steps_per_s": round(c.npoints / (msc * 1e-3) / 1e6, 1)}
        print(f"[bench] {c.name} {dt_c}: {msc:.4f} ms/step", flush=True)
        pc.close()
        del uc
    return configs


def time_c4_adjoint(W, Plan, torch, time):
    """The Gierer-Meinhardt 256^2 Neumann adjoint workload at full size: loss =
    mean over points of the squared distance of (u, v) after 200 steps from a
    target run with perturbed orders, diffusion and source; checkpoints every
    20 steps; gradients of u0, kappa, alpha and the reaction parameters. The
    forward and the backward are timed in FP32 and FP64 (warm plans)."""
    c = W.C4_GM_ADJ
    tg = c.extra["target"]
    u0 = W.initial_fields(c)
    out, grads = {}, {}
    for dt_c in ("f32", "f64"):
        td = torch.float32 if dt_c == "f32" else torch.float64
        pt = Plan(c.shape, c.bc, c.h, tg["alpha"], tg["kappa"], c.dt, c.reaction, tg["params"],
                  dt_c, c.scheme)
        target = torch.tensor(u0, dtype=td, device="cuda")
        pt.integrate(target, c.nsteps)
        pt.close()
        pc = Plan(c.shape, c.bc, c.h, c.alpha, c.kappa, c.dt, c.reaction, c.params, dt_c,
                  c.scheme)
        u = torch.tensor(u0, dtype=td, device="cuda")
        ck = pc.integrate(u.clone(), c.nsteps, 0.0, ckpt_every=c.ckpt_every)  # warm-up
        g = torch.zeros_like(u)
        g0 = torch.empty_like(u)
        pc.backward(ck, c.nsteps, c.ckpt_every, g, 0.0, g0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pc.integrate(u.clone(), c.nsteps)
        torch.cuda.synchronize()
        t_f = time.perf_counter() - t0
        uc = u.clone()
        t0 = time.perf_counter()
        ck = pc.integrate(uc, c.nsteps, 0.0, ckpt_every=c.ckpt_every)
        torch.cuda.synchronize()
        t_fc = time.perf_counter() - t0
        g = (2.0 / c.npoints) * (uc - target)
        t0 = time.perf_counter()
        gk, ga, gp = pc.backward(ck, c.nsteps, c.ckpt_every, g, 0.0, g0)
        torch.cuda.synchronize()
        t_b = time.perf_counter() - t0
        loss = float(((uc.double() - target.double()) ** 2).sum() / c.npoints)
        grads[dt_c] = list(gk) + list(ga) + list(gp)
        out[dt_c] = {"forward_s": round(t_f, 4), "forward_with_ckpt_s": round(t_fc, 4),
                     "backward_s": round(t_b, 4), "ratio": round(t_b / t_f, 3), "loss": loss,
                     "workspace_mb": round(pc.workspace_bytes() / 1e6, 1),
                     "checkpoint_mb": round(ck.numel() / 1e6, 1)}
        print(f"[bench] {c.name} adjoint {dt_c}: forward {t_f * 1e3:.1f} ms, backward "
              f"{t_b * 1e3:.1f} ms ({t_b / t_f:.2f}x)", flush=True)
        pc.close()
        del ck, u, uc, target, g, g0
    scale = max(abs(b) for b in grads["f64"])
    out["fp32_vs_fp64_grad"] = max(abs(a - b) for a, b in zip(grads["f32"], grads["f64"])) / scale
    out["workload"] = f"{c.name}: {c.nsteps} steps, checkpoints every {c.ckpt_every}"
    return out


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
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-c4-adjoint", action="store_true",
                    help="skip the Gierer-Meinhardt 256^2 adjoint timing")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the timings of the other benchmark configurations")
    ap.add_argument("--no-c5-adjoint", action="store_true",
                    help="skip configuration 5's full FP32 adjoint (1000 steps, checkpoints "
                         "every 32: time, memory, gradients)")
    ap.add_argument("--c5-adjoint-fp64", action="store_true",
                    help="also run configuration 5's full adjoint in FP64 (about 35 s, "
                         "92 GB)")
    ap.add_argument("--configs-only", action="store_true",
                    help="time only the other configurations (one JSON line)")
    ap.add_argument("--cpu-fast-steps", type=int, default=2,
                    help="timed steps of the scipy.fft CPU implementation of Alg. 1")
    ap.add_argument("--ensemble-members", type=int, default=64)
    ap.add_argument("--ensemble-steps", type=int, default=200)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (PMC scaling)")
    ap.add_argument("--summarize-pmc", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH",
                                                          "COPY_WRITE"),
                    help="rocprofv3 counter CSVs -> per-class HBM bytes per launch (no GPU)")
    ap.add_argument("--summarize-stats", metavar="KERNEL_STATS_CSV",
                    help="rocprofv3 --stats CSV -> markdown table (no GPU)")
    ap.add_argument("--out", help="output JSON of --summarize-pmc")
    args = ap.parse_args()

    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc, args.out, "schnakenberg3d_neumann_256")
        return 0
    if args.summarize_stats:
        summarize_stats(args.summarize_stats)
        return 0

    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
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

    if args.configs_only:
        print(json.dumps({"configs": time_configs(W, Plan, torch, time)}), flush=True)
        return 0

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
    # the throughput run has no per-launch events on the stream; the same K
    # steps are then run again with a HIP event pair around every launch for
    # the per-kernel averages of the roofline
    u32, ms32, _ = timed(p32, "f32", args.steps, args.warmup, profile=False)
    ms_step = ms32 / args.steps
    value = n * args.steps / (ms32 * 1e-3) / 1e6
    _, ms32p, prof = timed(p32, "f32", args.steps, 0, profile=True)
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
    kernel_names = {"X": "k_xstage_m<float> (inverse-x, reaction, forward-x)",
                    "Y": "k_single_m<float> (y transform)",
                    "Z": "k_zstage_m<float> (forward-z, stage combine, inverse-z; four stage "
                         "kernels)"}
    traffic = None
    tfile = os.path.join(ROOT, "profiles", f"traffic_{wl.name}_f32.json")
    if os.path.exists(tfile):
        with open(tfile) as fh:
            tj = json.load(fh)
        if tj.get("src_hash") == src_hash() and dom in tj.get("classes", {}):
            traffic = tj["classes"][dom]["hbm_bytes_per_launch"]
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kernel_names[dom], "avg_launch_ms": round(avg_ms, 4),
                "launches": n_dom,
                "profiled_ms_per_step": round(ms32p / args.steps, 4),
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

    # ---------------------------------------------------------------- ensemble
    # The small 2D FitzHugh-Nagumo problem (64x64, FP64) alone and as B
    # members with orders spread over [1.2, 2.0] in one ensemble plan.
    ensemble = None
    if not args.no_ensemble:
        e = W.C1_FHN
        B, ke = args.ensemble_members, args.ensemble_steps
        e0 = W.initial_fields(e)
        single = Plan(e.shape, e.bc, e.h, e.alpha, e.kappa, e.dt, e.reaction, e.params, "f64")
        alphas = [(a, a) for a in np.linspace(1.2, 2.0, B)]
        batch = Plan(e.shape, e.bc, e.h, alphas, [e.kappa] * B, e.dt, e.reaction,
                     [e.params] * B, "f64", batch=B)

        def run_timed(plan, u):
            w = u.clone()
            plan.integrate(w, 2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.integrate(u, ke)
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) * 1e3 / ke

        ms1 = run_timed(single, torch.tensor(e0, device="cuda"))
        msb = run_timed(batch, torch.tensor(np.stack([e0] * B), device="cuda"))
        ensemble = {"workload": f"{e.name} x {B} members (alpha 1.2..2.0)", "dtype": "f64",
                    "steps": ke, "single_ms_per_step": round(ms1, 4),
                    "batch_ms_per_step": round(msb, 4),
                    "member_steps_per_s_single": round(1e3 / ms1, 1),
                    "member_steps_per_s_batch": round(B * 1e3 / msb, 1),
                    "speedup_vs_one_at_a_time": round(B * ms1 / msb, 2)}
        print(f"[bench] ensemble: single {ms1:.3f} ms/step, {B} members {msb:.3f} ms/step "
              f"({B * ms1 / msb:.1f}x)", flush=True)
        single.close()
        batch.close()

    # ---------------------------------------------------------------- config 5 adjoint
    # MSE after 1000 steps against a target run with alpha + 0.05 and
    # kappa_v * 1.1; gradients with respect to alpha (per species) and kappa_v.
    c5adj = None
    if not args.no_c5_adjoint:
        c5 = W.C5_SCHNAK_NEU.replace(alpha=(args.alpha, args.alpha))
        tg = c5.extra["target"]
        c5adj = {"workload": f"{c5.name}: {c5.nsteps} steps, checkpoints every "
                             f"{c5.ckpt_every}, gradients of alpha_u, alpha_v, kappa_v"}
        grads = {}
        for dt_c in ("f32", "f64") if args.c5_adjoint_fp64 else ("f32",):
            td = torch.float32 if dt_c == "f32" else torch.float64
            kt = (c5.kappa[0], c5.kappa[1] * tg["kappa_v_scale"])
            at = tuple(a + tg["alpha_shift"] for a in c5.alpha)
            pt = Plan(c5.shape, c5.bc, c5.h, at, kt, c5.dt, c5.reaction, c5.params, dt_c,
                      c5.scheme)
            target = torch.tensor(u0, dtype=td, device="cuda")
            pt.integrate(target, c5.nsteps)
            pt.close()
            pc = Plan(c5.shape, c5.bc, c5.h, c5.alpha, c5.kappa, c5.dt, c5.reaction, c5.params,
                      dt_c, c5.scheme)
            uc = torch.tensor(u0, dtype=td, device="cuda")
            w = uc.clone()
            pc.integrate(w, 4)  # warm-up
            del w
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pc.integrate(uc.clone(), c5.nsteps)
            torch.cuda.synchronize()
            t_f = time.perf_counter() - t0
            t0 = time.perf_counter()
            ck = pc.integrate(uc, c5.nsteps, 0.0, ckpt_every=c5.ckpt_every)
            torch.cuda.synchronize()
            t_fc = time.perf_counter() - t0
            g = (2.0 / uc.numel()) * (uc - target)
            g0 = torch.empty_like(uc)
            t0 = time.perf_counter()
            gk, ga, _ = pc.backward(ck, c5.nsteps, c5.ckpt_every, g, 0.0, g0, params=False)
            torch.cuda.synchronize()
            t_b = time.perf_counter() - t0
            loss = float(((uc.double() - target.double()) ** 2).mean())
            grads[dt_c] = [ga[0], ga[1], gk[1]]
            c5adj[dt_c] = {"forward_s": round(t_f, 3), "forward_with_ckpt_s": round(t_fc, 3),
                           "backward_s": round(t_b, 3),
                           "ratio": round(t_b / t_f, 3), "loss": loss,
                           "workspace_gb": round(pc.workspace_bytes() / 1e9, 2),
                           "checkpoint_gb": round(ck.numel() / 1e9, 2),
                           "grad_alpha_u": ga[0], "grad_alpha_v": ga[1], "grad_kappa_v": gk[1]}
            print(f"[bench] config 5 adjoint {dt_c}: forward {t_f:.2f} s, backward {t_b:.2f} s "
                  f"({t_b / t_f:.3f}x)", flush=True)
            pc.close()
            del ck, uc, target, g, g0
            torch.cuda.empty_cache()
        if "f64" in grads:
            c5adj["fp32_vs_fp64_grad_rel"] = max(
                abs(a - b) / max(abs(b), 1e-300) for a, b in zip(grads["f32"], grads["f64"]))

    # ---------------------------------------------------------------- other configs
    configs = None if args.no_configs else time_configs(W, Plan, torch, time)
    c4adj = None if args.no_c4_adjoint else time_c4_adjoint(W, Plan, torch, time)

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
        # the fast-transform CPU implementation of Alg. 1 (scipy.fft), checked
        # against the FP64 GPU path after the same steps from the same fields
        workers = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        kf = args.cpu_fast_steps
        cpu_u, dt_fast = cpu_fast_alg1(wl, u0, kf, workers)
        g64 = make("f64")
        ug = torch.tensor(u0, dtype=torch.float64, device="cuda")
        g64.integrate(ug, kf + 1)
        torch.cuda.synchronize()
        ugn = ug.cpu().numpy()
        g64.close()
        fast_err = max(float(np.max(np.abs(cpu_u[s] - ugn[s])) / np.max(np.abs(ugn[s])))
                       for s in range(S))
        cpu["fast_alg1"] = {"value": round(n / dt_fast / 1e6, 3), "unit": "Mpoint-steps/s",
                            "cores": workers, "kind": "scipy.fft Alg. 1, FP64",
                            "sample": f"{kf} steps after 1 warm-up step of the same workload "
                                      f"({dt_fast:.2f} s per step)",
                            "vs_fp64_gpu_after_steps": fast_err}
        print(f"[bench] cpu scipy.fft Alg. 1: {dt_fast:.2f} s per step on {workers} cores, "
              f"vs FP64 GPU {fast_err:.2e}", flush=True)

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
        "ensemble": ensemble,
        "config4_adjoint": c4adj,
        "config5_adjoint": c5adj,
        "configs": configs,
        "roofline": roofline,
        "step_effective_gbs": round(step_gbs, 1),
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
