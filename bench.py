"""Throughput of the SGN RK4 hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload: the 1024x512 transversely perturbed line soliton (a = 0.5,
eps = 0.01, k = 2, x0 = -10) on [-10pi, 10pi] x [-5pi, 5pi], FP64, RK4 with
dt = 0.005, GMRES tol 1e-10, restart 20, Krasny filter 1e-12.  W untimed
warm-up steps, then K timed steps (one library call), bracketed by
device synchronisations; inputs are resident on the GPU before timing.

Prints one JSON line: grid-points x RK4 steps per second, GMRES iterations
per solve, a roofline entry for the dominant kernel (algorithmic bytes per
launch / its mean duration from HIP events recorded by the library on its
stream during the timed steps), and the FP64 oracle timed on the host CPU on
a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "grid-pts×RK4 steps/s at GMRES tol; iters/solve, plain vs learned"
UNIT = "grid-pts×RK4 steps/s"
HBM_PEAK_GBS = 8000.0
WORKLOAD = "perturbed_soliton_1024x512"
PARAMS = dict(a=0.5, eps=0.01, k=2)
KRASNY = 1e-12

# The roofline entry is for the kernel class with the largest share of device
# time on this workload: the x part of the elliptic operator in the Arnoldi
# step (kernel B, k_row_matvec3: inverse x-transforms of E and G, the
# pointwise products with 1/h, forward x-transforms into P and Q).  Its
# algorithmic bytes per launch, 5 fields (E, G, h read; P, Q written), are
# summed by the library over the launches that did work.
DOMINANT = "row_matvec"
EVENT_PERIOD = 7  # launches of the timed class per launch that carries events


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=100)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--main-only", action="store_true",
                   help="time only the headline 1024x512 run (no guess, precision or batched forms; for profiler runs)")
    p.add_argument("--cpu-steps", type=int, default=5)
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="only run a plain device-to-device copy of MIB MiB, --steps times (calibrates the "
                        "FETCH_SIZE / WRITE_SIZE counters against a known byte count)")
    return p.parse_args()


def copy_calibration(mib: int, reps: int):
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(json.dumps({"copy_mib": mib, "reps": reps, "bytes_read_per_copy": n * 8, "bytes_written_per_copy": n * 8,
                      "gb_per_s": 2 * n * 8 * reps / dt / 1e9}), flush=True)


def traffic_ratio_from_profile(kernel: str):
    """Measured HBM bytes / algorithmic bytes of the kernel, from the rocprofv3
    FETCH_SIZE and WRITE_SIZE counters summarised in profiles/, if that summary
    was taken on the kernel source currently in the tree (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{WORKLOAD}_counters.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"traffic_over_algorithmic:\s*([0-9.eE+]+)", text)
    h = re.search(r"kernel_source_sha256:\s*([0-9a-f]+)", text)
    if not m or not h:
        return None
    if kernel_source_hash() != h.group(1):
        return None
    return float(m.group(1))


def kernel_source_hash() -> str:
    """sha256 of the kernel sources (the kernels and the FFT engine they inline)."""
    import hashlib
    d = hashlib.sha256()
    for name in ("sgn_kernels.hip", "sgn_fft.hpp"):
        d.update(open(os.path.join(ROOT, "paper_2306_09731_amd", "csrc", name), "rb").read())
    return d.hexdigest()


def timed_guess_run(sgn, torch, box, state, w, dev, args):
    """K timed steps (after W warm-up steps) of the same workload with
    SGN_GUESS_STAGE_INCREMENT: each RK stage starts GMRES from the previous
    stage's sigma plus that stage's increment in the previous step."""
    cfg = sgn.config_default(box.nx, box.ny, box.Lx, box.Ly, gmres_tol=w["tol"], gmres_restart=w["restart"],
                             krasny=KRASNY, guess=sgn.SGN_GUESS_STAGE_INCREMENT)
    ctx = sgn.sgn_init(cfg, dev)
    f = [torch.from_numpy(a).to(dev).contiguous() for a in state]
    if args.warmup > 0:
        sgn.sgn_rk4_step(ctx, *f, w["dt"], args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = sgn.sgn_rk4_step(ctx, *f, w["dt"], args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.close()
    return {"value": box.nx * box.ny * args.steps / el, "ms_per_step": el * 1e3 / args.steps,
            "iters_per_solve_mean": info.total_iters / max(info.solves, 1),
            "iters_per_solve_max": info.max_iters_per_solve,
            "note": "same tolerance; the first step of each call uses the plain warm start"}


def graph_form(sgn, torch, box, state, w, dev, args):
    """The same K steps (after W warm-up steps) with every RK4 step replayed as
    one captured HIP graph (sgn_rk4_step_graph, automatic iteration budget),
    beside the host-driven loop on a fresh context: bitwise the same states."""
    out = {}
    for mode in ("host", "graph"):
        cfg = sgn.config_default(box.nx, box.ny, box.Lx, box.Ly, gmres_tol=w["tol"], gmres_restart=w["restart"],
                                 krasny=KRASNY)
        ctx = sgn.sgn_init(cfg, dev)
        f = [torch.from_numpy(a).to(dev).contiguous() for a in state]
        step = (lambda n: sgn.sgn_rk4_step(ctx, *f, w["dt"], n)) if mode == "host" else \
            (lambda n: sgn.sgn_rk4_step_graph(ctx, *f, w["dt"], n)[0])
        if args.warmup > 0:
            step(args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step(args.steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[mode] = {"value": box.nx * box.ny * args.steps / el, "ms_per_step": el * 1e3 / args.steps}
        out[mode + "_state"] = [t.clone() for t in f]
        ctx.close()
    same = all(torch.equal(a, b) for a, b in zip(out.pop("host_state"), out.pop("graph_state")))
    out["identical_states"] = same
    return out


def learned_form(sgn, torch, dev, args):
    """The learned initial guess with the stored weights (trained by
    python -m paper_2306_09731_amd.learned on solver-recorded samples) against
    the paper's warm start, on the held-out oblique crossing solitons (1024^2,
    tol 1e-8) and on this benchmark's workload: ms per RK4 step, GMRES
    iterations per solve, and the network's mean squared error on recorded
    samples beside the zero and M^-1 r0 predictors."""
    import numpy as np
    from paper_2306_09731_amd import learned
    if not os.path.exists(learned.PARAMS_FILE):
        return {"error": f"missing {os.path.relpath(learned.PARAMS_FILE, ROOT)}"}
    params = np.load(learned.PARAMS_FILE)
    steps = max(1, min(args.steps, 40))
    return {"weights": os.path.relpath(learned.PARAMS_FILE, ROOT),
            "runs": [learned.evaluate(params, dev, name, steps=steps)
                     for name in ("crossing_solitons_1024x1024", WORKLOAD)]}


PRECISION_WORKLOAD = "gaussian_2048x2048"


def precision_form(sgn, torch, dev, args):
    """The 2048x2048 Gaussian (h = 1 + 0.5 exp(-r^2), v = 0) in FP64 and in the
    mixed-precision mode (FP32 fields and transforms, FP64 reductions): K
    timed steps after W warm-up steps each, the Arnoldi kernel class with the
    largest share of the FP32 run against the HBM roofline, and the FP32 - FP64
    difference after the same steps."""
    import numpy as np
    from sgn_inputs import workload
    box, state, w = workload(PRECISION_WORKLOAD)
    steps = max(1, min(args.steps, 20))
    warm = min(args.warmup, 5)
    out, final = {"workload": PRECISION_WORKLOAD, "nx": box.nx, "ny": box.ny, "steps": steps, "warmup": warm}, {}
    for name, prec, dtype in (("fp64", sgn.SGN_FP64, torch.float64), ("fp32_mixed", sgn.SGN_FP32_MIXED, torch.float32)):
        cfg = sgn.config_default(box.nx, box.ny, box.Lx, box.Ly, gmres_tol=w["tol"], gmres_restart=w["restart"],
                                 krasny=KRASNY, precision=prec)
        ctx = sgn.sgn_init(cfg, dev)
        f = [torch.from_numpy(np.ascontiguousarray(a)).to(dev).to(dtype) for a in state]
        if warm:
            sgn.sgn_rk4_step(ctx, *f, w["dt"], warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = sgn.sgn_rk4_step(ctx, *f, w["dt"], steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res = {"value": box.nx * box.ny * steps / el, "unit": UNIT, "ms_per_step": el * 1e3 / steps,
               "iters_per_solve_mean": info.total_iters / max(info.solves, 1),
               "gmres_tol_effective": max(w["tol"], 1e-6) if prec == sgn.SGN_FP32_MIXED else w["tol"]}
        final[name] = [t.double().cpu().numpy() for t in f[:2]]
        if prec == sgn.SGN_FP64:
            state_after = [t.clone() for t in f[:3]]
        if prec == sgn.SGN_FP32_MIXED:
            # time every Arnoldi kernel class over the same number of further steps
            per = {}
            for kind in (0, 1, 2, 3):
                sgn.sgn_kernel_timing(ctx, kind, True)
                sgn.sgn_rk4_step(ctx, *[t.clone() for t in f], w["dt"], steps)
                n, ms, by = sgn.sgn_kernel_time(ctx, kind)
                sgn.sgn_kernel_timing(ctx, kind, False)
                if n:
                    per[sgn.KERNEL_NAMES[kind]] = (n, ms, by)
            dom = max(per, key=lambda k: per[k][1])
            n, ms, by = per[dom]
            ach = by / (ms * 1e-3) / 1e9 if ms else None
            res["roofline"] = {"kernel_class": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": ach / HBM_PEAK_GBS if ach else None,
                               "traffic": None, "algorithmic_bytes_per_launch": by / n,
                               "mean_launch_us": ms / n * 1e3, "launches": n,
                               "share_of_arnoldi_kernel_time": ms / sum(v[1] for v in per.values())}
        out[name] = res
        ctx.close()
    out["refined_solve"] = refined_solve_form(sgn, torch, dev, box, state_after, w["tol"])
    h64, v64 = final["fp64"]
    h32, v32 = final["fp32_mixed"]
    out["fp32_vs_fp64_after_steps"] = {
        "h": float(np.abs(h32 - h64).max() / np.abs(h64 - 1.0).max()),
        "vx": float(np.abs(v32 - v64).max() / max(np.abs(v64).max(), 1e-300))}
    return out


def refined_solve_form(sgn, torch, dev, box, state, tol, reps: int = 3):
    """One elliptic solve on the state after the timed FP64 steps (b = -div v),
    from sigma = 0 to the workload's tolerance: the FP64 GMRES solve against
    the mixed-precision refinement (FP64 residuals, FP32 GMRES corrections at
    1e-6); best of a few repetitions each."""
    h, vx, vy = state
    c64 = sgn.sgn_init(sgn.config_default(box.nx, box.ny, box.Lx, box.Ly, gmres_tol=tol, krasny=KRASNY), dev)
    c32 = sgn.sgn_init(sgn.config_default(box.nx, box.ny, box.Lx, box.Ly, gmres_tol=1e-6, krasny=KRASNY,
                                          precision=sgn.SGN_FP32_MIXED), dev)
    dx, dy = torch.empty_like(h), torch.empty_like(h)
    sgn.sgn_derivative(c64, 0, vx, dx)
    sgn.sgn_derivative(c64, 1, vy, dy)
    b = -(dx + dy)
    out = {"tol": tol}
    for name in ("fp64_gmres", "fp32_refined"):
        best = None
        for _ in range(reps):
            sig = torch.zeros_like(h)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if name == "fp64_gmres":
                info = sgn.sgn_elliptic_solve(c64, h, b, sig)
                rec = {"iters": info.iters}
            else:
                info = sgn.sgn_elliptic_solve_refined(c64, c32, h, b, sig, tol, 8)
                rec = {"rounds": info.rounds, "inner_iters": info.inner_iters,
                       "rel_resid_true": info.rel_resid_true}
            torch.cuda.synchronize()
            el = (time.perf_counter() - t0) * 1e3
            if best is None or el < best["ms"]:
                best = dict(rec, ms=el)
        out[name] = best
        if name == "fp64_gmres":
            ref = sig.clone()
    out["sigma_difference"] = float((sig - ref).abs().max() / ref.abs().max())
    out["speedup"] = out["fp64_gmres"]["ms"] / out["fp32_refined"]["ms"]
    c64.close()
    c32.close()
    return out


def batched_form(sgn, torch, dev, args, per_grid: int = 16):
    """64 perturbed line solitons, 16 on each of 256x256, 512x512, 1024x512 and
    1024x1024 (dx = dy = pi/16, seeded amplitudes and transverse perturbations),
    in the mixed-precision mode: each member has its own context and stream,
    the Arnoldi schedule comes from the autotuner, and K steps of all members
    run as one sgn_rk4_step_ensemble call; the same steps run one member after
    another give the sequential rate, and with graph replays per member
    (sgn_rk4_step_ensemble_graph) the graph rate."""
    import numpy as np
    from sgn_inputs import ENSEMBLE_GRIDS, ensemble_member
    members, seed, schedules = [], 0, {}
    for nx, ny in ENSEMBLE_GRIDS:
        for _ in range(per_grid):
            box, state, p = ensemble_member(seed, nx, ny)
            seed += 1
            cfg = sgn.config_default(box.nx, box.ny, box.Lx, box.Ly, krasny=KRASNY, precision=sgn.SGN_FP32_MIXED)
            ctx = sgn.sgn_init(cfg, dev, stream=torch.cuda.Stream(dev))
            f = [torch.from_numpy(np.ascontiguousarray(a)).to(dev).to(torch.float32) for a in state]
            schedules[f"{nx}x{ny}"] = sgn.ARNOLDI_SCHEDULES[sgn.sgn_autotune(ctx)]
            members.append((ctx, f, p["dt"], nx * ny))
    ctxs, fields, dts = [m[0] for m in members], [m[1] for m in members], [m[2] for m in members]
    pts = sum(m[3] for m in members)
    steps = max(1, min(args.steps, 10))
    sgn.sgn_rk4_step_ensemble(ctxs, fields, dts, min(args.warmup, 2) or 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = sgn.sgn_rk4_step_ensemble(ctxs, fields, dts, steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # the same members with their steps replayed as captured graphs (the
    # first call captures and calibrates the iteration budgets)
    sgn.sgn_rk4_step_ensemble(ctxs, fields, dts, min(args.warmup, 2) or 1, graphs=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sgn.sgn_rk4_step_ensemble(ctxs, fields, dts, steps, graphs=True)
    torch.cuda.synchronize()
    el_graph = time.perf_counter() - t0
    t0 = time.perf_counter()
    for c, f, d in zip(ctxs, fields, dts):
        sgn.sgn_rk4_step(c, *f, d, steps)
    torch.cuda.synchronize()
    el_seq = time.perf_counter() - t0
    for c in ctxs:
        c.close()
    return {"workload": "ensemble of 64 perturbed line solitons (16 each on 256^2, 512^2, 1024x512, 1024^2)",
            "members": len(members), "points": pts, "precision": "fp32_mixed", "steps": steps,
            "value": pts * steps / el, "unit": UNIT, "ms_per_step": el * 1e3 / steps,
            "sequential_value": pts * steps / el_seq, "speedup_vs_sequential": el_seq / el,
            "graph_value": pts * steps / el_graph, "graph_ms_per_step": el_graph * 1e3 / steps,
            "iters_per_solve_mean": sum(i.total_iters for i in infos) / max(sum(i.solves for i in infos), 1),
            "schedules": schedules}


def cpu_baseline(steps: int):
    import numpy as np  # noqa: F401
    from oracle import sgn_oracle as O
    from sgn_inputs import workload
    box, (h, vx, vy, s), w = workload(WORKLOAD, **PARAMS)
    g = O.Grid(O.Config(nx=box.nx, ny=box.ny, Lx=box.Lx, Ly=box.Ly, gmres_tol=w["tol"],
                        gmres_restart=w["restart"], krasny=KRASNY))
    t0 = time.perf_counter()
    O.rk4(g, h, vx, vy, s, w["dt"], steps)
    dt = time.perf_counter() - t0
    return {"value": box.nx * box.ny * steps / dt, "unit": UNIT, "cores": 1, "kind": "oracle",
            "sample": f"{steps} RK4 step(s) of the {box.nx}x{box.ny} workload from t=0 "
                      f"(numpy FP64, single-threaded FFTs), {dt:.1f} s"}


def progress(msg: str):
    """One progress line per phase on stderr (the JSON result goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration, max(args.steps, 1))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the solver is single-GPU.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2306_09731_amd import sgn
    from sgn_inputs import workload

    box, (h, vx, vy, s), w = workload(WORKLOAD, **PARAMS)
    dev = torch.device("cuda:0")
    cfg = sgn.config_default(box.nx, box.ny, box.Lx, box.Ly, gmres_tol=w["tol"], gmres_restart=w["restart"],
                             krasny=KRASNY)
    ctx = sgn.sgn_init(cfg, dev)
    th, tvx, tvy, ts = (torch.from_numpy(a).to(dev).contiguous() for a in (h, vx, vy, s))
    if args.warmup > 0:
        sgn.sgn_rk4_step(ctx, th, tvx, tvy, ts, w["dt"], args.warmup)
    # the same run with the stage-increment initial guess (same tolerance),
    # timed first so that the headline run below is the last thing measured
    progress("warm-up done")
    alt = None if args.main_only else timed_guess_run(sgn, torch, box, (h, vx, vy, s), w, dev, args)
    progress("stage-increment guess run done")
    dominant = DOMINANT
    kind = [k for k, v in sgn.KERNEL_NAMES.items() if v == dominant][0]
    # events on every EVENT_PERIOD-th launch of the class: recording them on
    # every launch costs about 3% of the step
    sgn.sgn_kernel_timing(ctx, kind, True, EVENT_PERIOD)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = sgn.sgn_rk4_step(ctx, th, tvx, tvy, ts, w["dt"], args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    progress(f"timed run done: {elapsed * 1e3 / args.steps:.3f} ms per step")
    launches, kms, algo_total = sgn.sgn_kernel_time(ctx, kind)  # events recorded at dispatch start/end
    sgn.sgn_kernel_timing(ctx, kind, False)
    npts = box.nx * box.ny
    value = npts * args.steps / elapsed
    algo = algo_total / launches if launches else 0.0  # per launch, averaged over all timed launches
    mean_s = (kms / launches) / 1e3 if launches else float("nan")
    achieved = algo / mean_s / 1e9 if launches else None
    ratio = traffic_ratio_from_profile(dominant)
    traffic = ratio * algo if (ratio is not None and launches) else None  # HBM bytes per launch
    out = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": WORKLOAD, "nx": box.nx, "ny": box.ny, "Lx": box.Lx, "Ly": box.Ly,
            "a": PARAMS["a"], "eps": PARAMS["eps"], "k": PARAMS["k"], "dt": w["dt"],
            "gmres_tol": w["tol"], "gmres_restart": w["restart"], "krasny": KRASNY,
            "guess": "plain (warm start from the previous sigma)",
            "iters_per_solve_mean": info.total_iters / max(info.solves, 1),
            "iters_per_solve_max": info.max_iters_per_solve,
            "solves": info.solves,
            "stage_increment_guess": alt,
        },
        "roofline": {
            "kernel": f"k_row_matvec3<{box.nx}> (Arnoldi kernel B: x part of the elliptic operator, "
                      f"three transform chains per row pair)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": algo,
            "mean_launch_us": mean_s * 1e6,
            "launches": launches,
            "events_on_every": EVENT_PERIOD,
        },
    }
    if not args.main_only:
        out["graph_form"] = graph_form(sgn, torch, box, (h, vx, vy, s), w, dev, args)
        progress("graph form done")
        out["learned_form"] = learned_form(sgn, torch, dev, args)
        progress("learned form done")
        out["precision_form"] = precision_form(sgn, torch, dev, args)
        progress("precision form done")
        out["batched_form"] = batched_form(sgn, torch, dev, args)
        progress("batched form done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
