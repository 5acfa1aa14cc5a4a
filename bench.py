"""Throughput of the SGN RK4 hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload: the 1024x512 transversely perturbed line solitons on
[-10pi, 10pi] x [-5pi, 5pi] (x0 = -10, eps = 0.01), all nine runs
a in {0.2, 0.5, 1.0} x k in {1, 2, 4} advanced together as the members of one
ensemble context (every kernel launch covers the nine grids, each with its
own GMRES state), FP64, RK4 with dt = 0.005, GMRES tol 1e-10, restart 20,
Krasny filter 1e-12.  W untimed warm-up steps, then K timed steps (one
library call), bracketed by device synchronisations; inputs are resident on
the GPU before timing.

Prints one JSON line: grid-points x RK4 steps per second over the nine runs,
GMRES iterations per solve (overall and per run), a roofline entry for the
dominant kernel (algorithmic bytes per launch / its mean duration from HIP
events recorded by the library on its stream during the timed steps), the
same run one grid per context, the nine runs to t = 20 with their mass and
energy drift, the other forms of the build, and the FP64 oracle timed on the
host CPU on a bounded sample of the same workload.
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
SWEEP_WORKLOAD = "perturbed_soliton_1024x512_sweep"
PARAMS = dict(a=0.5, eps=0.01, k=2)  # the run of the nine timed alone (single_grid, cpu_baseline)
KRASNY = 1e-12

# The roofline entry is for the kernel class with the largest share of device
# time on the headline workload (rocprofv3 kernel statistics of the nine-run
# context): kernel A of the three-kernel Arnoldi step, k_col_proj, which
# finishes step j - 1 from C's block partials, forms u_j = w_{j-1} - sum_i
# c_i V_i and the inverse y-transforms E, G of it.  Its algorithmic bytes in
# step j are j + 4 fields (w_{j-1} and V_0..V_{j-1} read; u_j, E, G written),
# summed by the library over the launches that did work.  --time-class picks
# another class for profiler runs; the single grid and the 16-grid FP32 group
# report kernel B (the x part of the operator), which leads there.
DOMINANT = "col_basis"
ROW_CLASS = "row_matvec"
EVENT_PERIOD = 7  # launches of the timed class per launch that carries events


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=100)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--main-only", action="store_true",
                   help="time only the headline nine-run ensemble (no other forms; for profiler runs)")
    p.add_argument("--single-only", action="store_true",
                   help="time only the single 1024x512 grid (a = 0.5, k = 2; for profiler runs)")
    p.add_argument("--precision-only", action="store_true",
                   help="time only the 2048^2 precision form (for profiler runs)")
    p.add_argument("--c3-only", choices=("fp64", "fp32_mixed"),
                   help="time only the 2048^2 Gaussian in one precision, events on every launch of its "
                        "dominant Arnoldi kernel class (for profiler runs)")
    p.add_argument("--cnn-only", action="store_true",
                   help="time only the learned network's forward pass at 1024^2 (inference path), --steps passes")
    p.add_argument("--no-autotune", action="store_true",
                   help="keep the library's default launch choices (or those set by SGN_* variables) instead of "
                        "autotuning the member contexts; for profiler runs, whose counters would include the "
                        "autotuner's trial dispatches")
    p.add_argument("--time-class", choices=("col_basis", "row_matvec", "col_precond_dot", "gs_update"),
                   default=DOMINANT,
                   help="kernel class of the headline run (or of --c3-only) that carries HIP events and gives "
                        "the roofline entry (default: the class with the largest share of device time; "
                        "gs_update exists in the four-kernel step of --c3-only only)")
    p.add_argument("--t5-steps", type=int, default=1000,
                   help="steps of the 2048^2 precision comparison at t = 5 (dt = 0.005; 0 skips it)")
    p.add_argument("--t20-steps", type=int, default=4000,
                   help="steps of the nine-run to-t=20 leg (dt = 0.005; 0 skips it)")
    p.add_argument("--cpu-steps", type=int, default=5)
    p.add_argument("--cpu-worker", type=int, default=-1, metavar="RUN",
                   help="internal: one process of the all-core CPU baseline (the oracle on run RUN of the nine)")
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


def traffic_ratio_from_profile(kernel: str, workload: str = SWEEP_WORKLOAD):
    """Measured HBM bytes / algorithmic bytes of the kernel, from the rocprofv3
    FETCH_SIZE and WRITE_SIZE counters summarised in profiles/, if that summary
    was taken on the kernel source currently in the tree (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_counters.txt")
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


def timed_kernel_run(sgn, torch, ctx, fields, dt, steps, kind=None, period=EVENT_PERIOD):
    """steps timed RK4 steps in one call; with kind, every period-th launch of
    that kernel class carries HIP events.  Returns (elapsed s, infos list,
    (launches, total ms, algorithmic bytes) or None)."""
    if kind is not None:
        sgn.sgn_kernel_timing(ctx, kind, True, period)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = sgn.sgn_rk4_step(ctx, *fields, dt, steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kt = None
    if kind is not None:
        kt = sgn.sgn_kernel_time(ctx, kind)  # events recorded at dispatch start/end
        sgn.sgn_kernel_timing(ctx, kind, False)
    return el, (info if isinstance(info, list) else [info]), kt


def iters_summary(infos):
    return {"iters_per_solve_mean": sum(i.total_iters for i in infos) / max(sum(i.solves for i in infos), 1),
            "iters_per_solve_max": max(i.max_iters_per_solve for i in infos),
            "solves": sum(i.solves for i in infos)}


def sweep_kernel_labels(box, shape) -> dict:
    """Names of the three Arnoldi kernel classes of the nine-member context."""
    return {
        "col_basis": f"k_col_proj<{box.ny}> (Arnoldi kernel A: finishes step j-1, u_j = w_(j-1) - sum_i c_i V_i, "
                     f"inverse y-transforms E, G of u_j), nine grids per launch",
        "row_matvec": f"k_row_matvec2<{box.nx}> (Arnoldi kernel B: x part of the elliptic operator, two transform "
                      f"chains per block, {shape['row_radix'] or 4} values per thread), nine grids per launch",
        "col_precond_dot": f"k_col_precond_new<{box.ny}> (Arnoldi kernel C: forward y-transforms of P, Q, the "
                           f"preconditioner, V_j and the projections onto the basis), nine grids per launch",
    }


def roofline_entry(kernel: str, kt, workload: str, klass: str):
    launches, kms, algo_total = kt
    algo = algo_total / launches if launches else 0.0  # per launch, averaged over all timed launches
    mean_s = (kms / launches) / 1e3 if launches else float("nan")
    achieved = algo / mean_s / 1e9 if launches else None
    ratio = traffic_ratio_from_profile(klass, workload)
    traffic = ratio * algo if (ratio is not None and launches) else None  # HBM bytes per launch
    return {"kernel": kernel, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
            "algorithmic_bytes_per_launch": algo, "mean_launch_us": mean_s * 1e6, "launches": launches,
            "events_on_every": EVENT_PERIOD}


AUTOTUNE = True


def sweep_context(sgn, torch, dev, guess=None):
    """The nine runs as one ensemble context and its [9][ny][nx] fields."""
    from sgn_inputs import perturbed_soliton_sweep
    box, state, ak, w = perturbed_soliton_sweep(eps=PARAMS["eps"])
    kw = dict(gmres_tol=w["tol"], gmres_restart=w["restart"], krasny=KRASNY, batch=len(ak))
    if guess is not None:
        kw["guess"] = guess
    cfg = sgn.config_default(box.nx, box.ny, box.Lx, box.Ly, **kw)
    ctx = sgn.sgn_init(cfg, dev)
    if AUTOTUNE:
        sgn.sgn_autotune(ctx)  # schedule, launch shapes and row radix for nine members of this grid
    f = [torch.from_numpy(a).to(dev).contiguous() for a in state]
    return box, ak, w, ctx, f


STREAM_SPLIT = (3, 3, 3)


def streams_form(sgn, torch, dev, args, ref_final):
    """The nine runs as three member contexts of three runs each, on three
    streams, advanced by one sgn_rk4_step_ensemble call (a host thread per
    context inside the library), so that the kernels of one context overlap
    those of the others (memory-bound column passes beside transform-bound row
    passes, and the tails of launches): W warm-up and K timed steps, the final
    states compared bitwise with the one-context run's (ref_final, after the
    same steps)."""
    import numpy as np
    from sgn_inputs import perturbed_soliton_sweep
    box, state, ak, w = perturbed_soliton_sweep(eps=PARAMS["eps"])
    ctxs, i0 = [], 0
    for nm in STREAM_SPLIT:
        cfg = sgn.config_default(box.nx, box.ny, box.Lx, box.Ly, gmres_tol=w["tol"], gmres_restart=w["restart"],
                                 krasny=KRASNY, batch=nm)
        ctx = sgn.sgn_init(cfg, dev, stream=torch.cuda.Stream(dev))
        if AUTOTUNE:
            sgn.sgn_autotune(ctx)
        ctxs.append((ctx, [torch.from_numpy(np.ascontiguousarray(a[i0:i0 + nm])).to(dev) for a in state]))
        i0 += nm
    torch.cuda.synchronize()
    cl, fl, dts = [c for c, _ in ctxs], [f for _, f in ctxs], [w["dt"]] * len(ctxs)
    if args.warmup > 0:
        sgn.sgn_rk4_step_ensemble(cl, fl, dts, args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = sgn.sgn_rk4_step_ensemble(cl, fl, dts, args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    final = [torch.cat([fl[i] for _, fl in ctxs]) for i in range(4)]
    out = {"split": list(STREAM_SPLIT), "value": len(ak) * box.nx * box.ny * args.steps / el,
           "ms_per_step": el * 1e3 / args.steps,
           "identical_to_one_context": all(torch.equal(a, b) for a, b in zip(final, ref_final)),
           "launch_shapes": [sgn.sgn_launch_shape(c) for c, _ in ctxs]}
    out.update(iters_summary(infos))
    for c, _ in ctxs:
        c.close()
    return out


def timed_guess_run(sgn, torch, dev, args):
    """K timed steps (after W warm-up steps) of the nine runs with
    SGN_GUESS_STAGE_INCREMENT: each RK stage starts GMRES from the previous
    stage's sigma plus that stage's increment in the previous step."""
    box, ak, w, ctx, f = sweep_context(sgn, torch, dev, guess=sgn.SGN_GUESS_STAGE_INCREMENT)
    if args.warmup > 0:
        sgn.sgn_rk4_step(ctx, *f, w["dt"], args.warmup)
    el, infos, _ = timed_kernel_run(sgn, torch, ctx, f, w["dt"], args.steps)
    ctx.close()
    out = {"value": len(ak) * box.nx * box.ny * args.steps / el, "ms_per_step": el * 1e3 / args.steps}
    out.update(iters_summary(infos))
    out["note"] = "same tolerance; the first step of each call uses the plain warm start"
    return out


def single_grid_run(sgn, torch, dev, args, with_roofline=True):
    """The run a = 0.5, k = 2 alone on a context of its own (one grid per
    launch): K timed steps after W warm-up steps, kernel B timed."""
    from sgn_inputs import workload
    box, state, w = workload(WORKLOAD, **PARAMS)
    cfg = sgn.config_default(box.nx, box.ny, box.Lx, box.Ly, gmres_tol=w["tol"], gmres_restart=w["restart"],
                             krasny=KRASNY)
    ctx = sgn.sgn_init(cfg, dev)
    f = [torch.from_numpy(a).to(dev).contiguous() for a in state]
    if args.warmup > 0:
        sgn.sgn_rk4_step(ctx, *f, w["dt"], args.warmup)
    kind = [k for k, v in sgn.KERNEL_NAMES.items() if v == ROW_CLASS][0]
    el, infos, kt = timed_kernel_run(sgn, torch, ctx, f, w["dt"], args.steps, kind if with_roofline else None)
    ctx.close()
    out = {"workload": WORKLOAD, "a": PARAMS["a"], "k": PARAMS["k"],
           "value": box.nx * box.ny * args.steps / el, "ms_per_step": el * 1e3 / args.steps}
    out.update(iters_summary(infos))
    if kt:
        out["roofline"] = roofline_entry(f"k_row_matvec3<{box.nx}> (kernel B), one grid per launch", kt, WORKLOAD,
                                         ROW_CLASS)
    return out


def sweep_single(sgn, torch, dev, args):
    """Each of the nine runs on a context of its own, one after another: K
    timed steps each (after W warm-up steps)."""
    import numpy as np
    from sgn_inputs import perturbed_soliton_sweep
    box, state, ak, w = perturbed_soliton_sweep(eps=PARAMS["eps"])
    cfg = sgn.config_default(box.nx, box.ny, box.Lx, box.Ly, gmres_tol=w["tol"], gmres_restart=w["restart"],
                             krasny=KRASNY)
    runs, total = [], 0.0
    for m, (a, k) in enumerate(ak):
        ctx = sgn.sgn_init(cfg, dev)
        f = [torch.from_numpy(np.ascontiguousarray(x[m])).to(dev) for x in state]
        if args.warmup > 0:
            sgn.sgn_rk4_step(ctx, *f, w["dt"], args.warmup)
        el, infos, _ = timed_kernel_run(sgn, torch, ctx, f, w["dt"], args.steps)
        ctx.close()
        total += el
        r = {"a": a, "k": k, "value": box.nx * box.ny * args.steps / el, "ms_per_step": el * 1e3 / args.steps}
        r.update(iters_summary(infos))
        runs.append(r)
    return {"runs": runs, "value": len(ak) * box.nx * box.ny * args.steps / total,
            "ms_per_step": total * 1e3 / args.steps,
            "note": "the nine runs one after another, one grid per context; value over all nine"}


def sweep_to_t20(sgn, torch, dev, steps):
    """The nine runs from t = 0 as one ensemble context for `steps` steps of
    dt = 0.005 (4000: t = 20): wall time, iterations, and each run's mass and
    energy drift (invariants of Section 2.3 at the start and the end)."""
    box, ak, w, ctx, f = sweep_context(sgn, torch, dev)
    inv0 = sgn.sgn_invariants(ctx, *[t.clone() for t in f])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    try:
        info = sgn.sgn_rk4_step(ctx, *f, w["dt"], steps)
        status = "ok"
    except sgn.SgnError as e:
        info, status = None, str(e)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out = {"steps": steps, "t_end": steps * w["dt"], "status": status, "wall_s": el,
           "value": len(ak) * box.nx * box.ny * steps / el}
    if info is None:
        ctx.close()
        return out
    inv1 = sgn.sgn_invariants(ctx, *f)
    out.update(iters_summary(info))
    out["runs"] = [{"a": a, "k": k, "mass_drift": abs(i1["mass"] - i0["mass"]) / abs(i0["mass"]),
                    "energy_drift": abs(i1["energy"] - i0["energy"]) / abs(i0["energy"]),
                    "max_h": i1["max_h"], "spectral_tail": i1["spectral_tail"],
                    "iters_per_solve_mean": inf.total_iters / max(inf.solves, 1)}
                   for (a, k), i0, i1, inf in zip(ak, inv0, inv1, info)]
    ctx.close()
    return out


def graph_form(sgn, torch, box, state, w, dev, args):
    """The same K steps (after W warm-up steps) with every RK4 step replayed as
    one captured HIP graph (sgn_rk4_step_graph, automatic per-stage iteration
    budgets), beside the host-driven loop on a fresh context: bitwise the same
    states; steps_replayed counts the timed steps that ran as replays (the
    others were chunks redone host-driven)."""
    out = {}
    for mode in ("host", "graph"):
        cfg = sgn.config_default(box.nx, box.ny, box.Lx, box.Ly, gmres_tol=w["tol"], gmres_restart=w["restart"],
                                 krasny=KRASNY)
        ctx = sgn.sgn_init(cfg, dev)
        f = [torch.from_numpy(a).to(dev).contiguous() for a in state]
        step = (lambda n: (sgn.sgn_rk4_step(ctx, *f, w["dt"], n), n)) if mode == "host" else \
            (lambda n: sgn.sgn_rk4_step_graph(ctx, *f, w["dt"], n))
        if args.warmup > 0:
            step(args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info, nrep = step(args.steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[mode] = {"value": box.nx * box.ny * args.steps / el, "ms_per_step": el * 1e3 / args.steps,
                     "iters_per_solve_mean": info.total_iters / max(info.solves, 1)}
        if mode == "graph":
            out[mode]["steps_replayed"] = nrep
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
                     for name in ("crossing_solitons_1024x1024", WORKLOAD)],
            "forward_1024x1024": cnn_forward_run(sgn, torch, dev, 50)}


PRECISION_WORKLOAD = "gaussian_2048x2048"
_COPY_PEAK = {}


def copy_peak_gbs(torch, dev, mib: int = 1024, reps: int = 20):
    """Attainable HBM bandwidth: a device-to-device copy of 1 GiB (read and
    write counted), best of `reps`."""
    if "v" not in _COPY_PEAK:
        n = mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.copy_(a)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            best = el if best is None or el < best else best
        _COPY_PEAK["v"] = 2 * n * 8 / best / 1e9
        del a, b
    return _COPY_PEAK["v"]


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
        ratio = traffic_ratio_from_profile(dom, f"{PRECISION_WORKLOAD}_{name}")
        res["roofline"] = {"kernel_class": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": ach / HBM_PEAK_GBS if ach else None,
                           "traffic": ratio * by / n if ratio is not None else None,
                           "algorithmic_bytes_per_launch": by / n, "mean_launch_us": ms / n * 1e3, "launches": n,
                           "share_of_arnoldi_kernel_time": ms / sum(v[1] for v in per.values()),
                           "attainable_copy_gbs": copy_peak_gbs(torch, dev),
                           "classes": {k: {"launches": v[0], "mean_launch_us": v[1] / v[0] * 1e3,
                                           "achieved": v[2] / (v[1] * 1e-3) / 1e9 if v[1] else None}
                                       for k, v in per.items()}}
        out[name] = res
        ctx.close()
    out["refined_solve"] = refined_solve_form(sgn, torch, dev, box, state_after, w["tol"])
    out["refined_step"] = refined_step_form(sgn, torch, dev, box, state, w, steps, warm)
    if args.t5_steps > 0:
        out["errors_at_t5"] = t5_errors(sgn, torch, dev, box, state, w, args.t5_steps)
    h64, v64 = final["fp64"]
    h32, v32 = final["fp32_mixed"]
    out["fp32_vs_fp64_after_steps"] = {
        "h": float(np.abs(h32 - h64).max() / np.abs(h64 - 1.0).max()),
        "vx": float(np.abs(v32 - v64).max() / max(np.abs(v64).max(), 1e-300))}
    return out




# the learned network's forward pass: 6 layers of 3x3 convolutions, 32 -> 32
# channels as run (padded), 2 * 9 * 32 * 32 flop per point and layer; HBM
# bytes per point of the inference path: the FP32 input triplets (12 B) and
# the BF16 output activation (64 B) of layer 1, 64 B in and out of layers
# 2-5, 64 B in and the FP32 output (4 B) of layer 6
CNN_FLOP_PER_POINT = 6 * 2 * 9 * 32 * 32
CNN_BYTES_PER_POINT = 12 + 64 + 4 * 128 + 64 + 4
BF16_PEAK_TFLOPS = 2500.0


def cnn_forward_run(sgn, torch, dev, passes: int, H: int = 1024, W: int = 1024):
    """passes forward passes of the network at H x W on random input
    triplets: mean ms, TFLOP/s against the dense BF16 MFMA peak, GB/s."""
    import numpy as np
    net = sgn.cnn_init(H, W, dev)
    rng = np.random.default_rng(0)
    sgn.cnn_set_params(net, (0.05 * rng.standard_normal(sgn.SGN_CNN_PARAMS)).astype(np.float32))
    x = torch.from_numpy(rng.standard_normal((H, W, 3)).astype(np.float32)).to(dev)
    out = torch.empty(H, W, dtype=torch.float32, device=dev)
    for _ in range(3):
        sgn.cnn_forward(net, x, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(passes):
        sgn.cnn_forward(net, x, out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / passes
    net.close()
    n = H * W
    tflops = CNN_FLOP_PER_POINT * n / (ms * 1e-3) / 1e12
    gbs = CNN_BYTES_PER_POINT * n / (ms * 1e-3) / 1e9
    return {"grid": [H, W], "passes": passes, "ms_per_forward": ms, "tflops": tflops,
            "mfma_frac": tflops / BF16_PEAK_TFLOPS, "gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
            "flop_per_point": CNN_FLOP_PER_POINT, "bytes_per_point": CNN_BYTES_PER_POINT}


def c3_run(sgn, torch, dev, args, name):
    """K steps of the 2048^2 Gaussian in one precision after W warm-up steps,
    one Arnoldi kernel class (--time-class) timed on every launch (all its
    dispatches of the timed call): the library's algorithmic bytes over
    exactly the dispatches a profiler of this run sees when W = 0."""
    import numpy as np
    from sgn_inputs import workload
    box, state, w = workload(PRECISION_WORKLOAD)
    prec, dtype = ((sgn.SGN_FP32_MIXED, torch.float32) if name == "fp32_mixed" else (sgn.SGN_FP64, torch.float64))
    cfg = sgn.config_default(box.nx, box.ny, box.Lx, box.Ly, gmres_tol=w["tol"], gmres_restart=w["restart"],
                             krasny=KRASNY, precision=prec)
    ctx = sgn.sgn_init(cfg, dev)
    f = [torch.from_numpy(np.ascontiguousarray(a)).to(dev).to(dtype) for a in state]
    if args.warmup > 0:
        sgn.sgn_rk4_step(ctx, *f, w["dt"], args.warmup)
    kind = [k for k, v in sgn.KERNEL_NAMES.items() if v == args.time_class][0]
    el, infos, kt = timed_kernel_run(sgn, torch, ctx, f, w["dt"], args.steps, kind, period=1)
    ctx.close()
    n, ms, by = kt
    out = {"workload": PRECISION_WORKLOAD, "precision": name, "steps": args.steps,
           "ms_per_step": el * 1e3 / args.steps, "kernel_class": args.time_class, "launches": n,
           "mean_launch_us": ms / n * 1e3 if n else None, "algorithmic_bytes_total": by,
           "algorithmic_bytes_per_launch": by / n if n else None,
           "achieved": by / (ms * 1e-3) / 1e9 if ms else None}
    out.update(iters_summary(infos))
    return out


def refined_step_form(sgn, torch, dev, box, state, w, steps, warm):
    """The precision form's FP64 residual refinement inside the RK4 step
    (sgn_rk4_step_refined): FP64 state, fluxes and RK combine, every stage
    solve refined to the FP64 tolerance from FP32 GMRES corrections; K timed
    steps after the warm-up, beside the FP64 step at the same tolerance."""
    import numpy as np
    c64 = sgn.sgn_init(sgn.config_default(box.nx, box.ny, box.Lx, box.Ly, gmres_tol=w["tol"], krasny=KRASNY), dev)
    c32 = sgn.sgn_init(sgn.config_default(box.nx, box.ny, box.Lx, box.Ly, gmres_tol=1e-6, krasny=KRASNY,
                                          precision=sgn.SGN_FP32_MIXED), dev)
    f = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in state]
    if warm:
        sgn.sgn_rk4_step_refined(c64, c32, *f, w["dt"], warm, w["tol"], 8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = sgn.sgn_rk4_step_refined(c64, c32, *f, w["dt"], steps, w["tol"], 8)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    c64.close()
    c32.close()
    return {"value": box.nx * box.ny * steps / el, "unit": UNIT, "ms_per_step": el * 1e3 / steps,
            "tol": w["tol"], "rounds_per_solve": info.rounds / max(info.solves, 1),
            "fp32_iters_per_solve": info.inner_iters / max(info.solves, 1),
            "max_rel_resid_true": info.max_rel_resid}


def t5_errors(sgn, torch, dev, box, state, w, nsteps):
    """The 2048^2 Gaussian from t = 0 for nsteps steps (1000: t = 5) in FP64
    (tol 1e-10), in the mixed-precision mode (FP32 state, GMRES at 1e-6) and
    with the refined step (FP64 state, stage solves refined to 1e-10): each
    field's difference from the FP64 run, relative to max |h - 1|, to the
    velocity scale max |v| of the FP64 run and to max |sigma|, and each run's
    wall time."""
    import numpy as np
    runs = {}
    for name in ("fp64", "fp32_mixed", "fp64_refined"):
        prec = sgn.SGN_FP32_MIXED if name == "fp32_mixed" else sgn.SGN_FP64
        dtype = torch.float32 if name == "fp32_mixed" else torch.float64
        ctx = sgn.sgn_init(sgn.config_default(box.nx, box.ny, box.Lx, box.Ly, gmres_tol=w["tol"], krasny=KRASNY,
                                              precision=prec), dev)
        c32 = None
        if name == "fp64_refined":
            c32 = sgn.sgn_init(sgn.config_default(box.nx, box.ny, box.Lx, box.Ly, gmres_tol=1e-6, krasny=KRASNY,
                                                  precision=sgn.SGN_FP32_MIXED), dev)
        f = [torch.from_numpy(np.ascontiguousarray(a)).to(dev).to(dtype) for a in state]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if c32 is None:
            sgn.sgn_rk4_step(ctx, *f, w["dt"], nsteps)
        else:
            sgn.sgn_rk4_step_refined(ctx, c32, *f, w["dt"], nsteps, w["tol"], 8)
        torch.cuda.synchronize()
        runs[name] = ([t.double().cpu().numpy() for t in f], time.perf_counter() - t0)
        ctx.close()
        if c32 is not None:
            c32.close()
    ref = runs["fp64"][0]
    vs = max(np.abs(ref[1]).max(), np.abs(ref[2]).max())
    out = {"steps": nsteps, "t": nsteps * w["dt"], "wall_s": {k: v[1] for k, v in runs.items()}}
    for name in ("fp32_mixed", "fp64_refined"):
        a = runs[name][0]
        out[name] = {"h": float(np.abs(a[0] - ref[0]).max() / np.abs(ref[0] - 1.0).max()),
                     "v": float(max(np.abs(a[1] - ref[1]).max(), np.abs(a[2] - ref[2]).max()) / vs),
                     "sigma": float(np.abs(a[3] - ref[3]).max() / np.abs(ref[3]).max())}
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
    in the mixed-precision mode, K steps after a warm-up step:
      members: one ensemble context per grid size (16 members each, every
        kernel launch covers the 16 grids), the four contexts on four streams
        advanced by one sgn_rk4_step_ensemble call (a host thread each);
      members_serial: the same four contexts one after another on one stream;
      contexts: the 64 members on 64 contexts of their own (streams and host
        threads, sgn_rk4_step_ensemble), the previous form; and with their
        steps replayed as captured graphs (graph_value);
      sequential: the 64 contexts one after another.
    Kernel B of the 1024x1024 group is timed against the HBM roofline."""
    import numpy as np
    from sgn_inputs import ENSEMBLE_GRIDS, ensemble_member
    steps = max(1, min(args.steps, 10))
    groups, seed = [], 0
    for nx, ny in ENSEMBLE_GRIDS:
        states, dts = [], []
        for _ in range(per_grid):
            box, state, p = ensemble_member(seed, nx, ny)
            seed += 1
            states.append(state)
            dts.append(p["dt"])
        assert len(set(dts)) == 1
        groups.append((box, states, dts[0]))
    pts = sum(b.nx * b.ny * len(st) for b, st, _ in groups)
    out = {"workload": "ensemble of 64 perturbed line solitons (16 each on 256^2, 512^2, 1024x512, 1024^2)",
           "members": sum(len(st) for _, st, _ in groups), "points": pts, "precision": "fp32_mixed",
           "steps": steps, "unit": UNIT}
    # one ensemble context per grid size
    ctxs = []
    for box, states, dt in groups:
        cfg = sgn.config_default(box.nx, box.ny, box.Lx, box.Ly, krasny=KRASNY, precision=sgn.SGN_FP32_MIXED,
                                 batch=len(states))
        stream = torch.cuda.Stream(dev)
        ctx = sgn.sgn_init(cfg, dev, stream=stream)
        sgn.sgn_autotune(ctx)
        f = [torch.from_numpy(np.ascontiguousarray(np.stack([m[i] for m in states]))).to(dev).to(torch.float32)
             for i in range(4)]
        ctxs.append((ctx, f, dt, stream))
    def run(i, n):
        c, f, dt, _ = ctxs[i]
        sgn.sgn_rk4_step(c, *f, dt, n)

    cl, fl, dl = [c[0] for c in ctxs], [c[1] for c in ctxs], [c[2] for c in ctxs]
    sgn.sgn_rk4_step_ensemble(cl, fl, dl, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    flat = sgn.sgn_rk4_step_ensemble(cl, fl, dl, steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["value"] = pts * steps / el
    out["ms_per_step"] = el * 1e3 / steps
    out.update(iters_summary(flat))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(len(ctxs)):
        run(i, steps)
    torch.cuda.synchronize()
    el_ser = time.perf_counter() - t0
    out["members_serial"] = {"value": pts * steps / el_ser, "ms_per_step": el_ser * 1e3 / steps}
    # kernel B of the largest group against the roofline
    c, f, dt, _ = ctxs[-1]
    kind = [k for k, v in sgn.KERNEL_NAMES.items() if v == ROW_CLASS][0]
    _, _, kt = timed_kernel_run(sgn, torch, c, [t.clone() for t in f], dt, steps, kind, period=1)
    n, ms, by = kt
    ach = by / n / (ms / n * 1e-3) / 1e9 if n else None
    shp = sgn.sgn_launch_shape(c)
    kname = (f"k_row_matvec2<1024> (kernel B, two transform chains per block, {shp['row_radix'] or 4} values "
             f"per thread)" if shp["arnoldi"] == 2 else "Arnoldi x-part kernel")
    out["roofline_1024x1024_group"] = {"kernel": f"{kname}, 16 grids per launch, FP32", "launch_shape": shp,
                                       "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                       "frac": ach / HBM_PEAK_GBS if ach else None,
                                       "algorithmic_bytes_per_launch": by / n if n else None,
                                       "mean_launch_us": ms / n * 1e3 if n else None, "launches": n}
    for c, _, _, _ in ctxs:
        c.close()
    del ctxs
    # the previous form: one context (and stream and host thread) per member
    members, schedules = [], {}
    for box, states, dt in groups:
        for st in states:
            cfg = sgn.config_default(box.nx, box.ny, box.Lx, box.Ly, krasny=KRASNY, precision=sgn.SGN_FP32_MIXED)
            ctx = sgn.sgn_init(cfg, dev, stream=torch.cuda.Stream(dev))
            f = [torch.from_numpy(np.ascontiguousarray(a)).to(dev).to(torch.float32) for a in st]
            schedules[f"{box.nx}x{box.ny}"] = sgn.ARNOLDI_SCHEDULES[sgn.sgn_autotune(ctx)]
            members.append((ctx, f, dt))
    cl, fields, dts = [m[0] for m in members], [m[1] for m in members], [m[2] for m in members]
    sgn.sgn_rk4_step_ensemble(cl, fields, dts, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sgn.sgn_rk4_step_ensemble(cl, fields, dts, steps)
    torch.cuda.synchronize()
    el_ctx = time.perf_counter() - t0
    sgn.sgn_rk4_step_ensemble(cl, fields, dts, 1, graphs=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sgn.sgn_rk4_step_ensemble(cl, fields, dts, steps, graphs=True)
    torch.cuda.synchronize()
    el_graph = time.perf_counter() - t0
    t0 = time.perf_counter()
    for c, f, d in zip(cl, fields, dts):
        sgn.sgn_rk4_step(c, *f, d, steps)
    torch.cuda.synchronize()
    el_seq = time.perf_counter() - t0
    for c in cl:
        c.close()
    out["contexts"] = {"value": pts * steps / el_ctx, "ms_per_step": el_ctx * 1e3 / steps,
                       "graph_value": pts * steps / el_graph, "graph_ms_per_step": el_graph * 1e3 / steps,
                       "schedules": schedules}
    out["sequential"] = {"value": pts * steps / el_seq, "ms_per_step": el_seq * 1e3 / steps}
    out["speedup_vs_contexts"] = el_ctx / el
    out["speedup_vs_sequential"] = el_seq / el
    return out


def cpu_baseline(steps: int):
    """The FP64 oracle (numpy, one thread: numpy's FFTs are single-threaded)
    on `steps` RK4 steps of one of the nine runs (a = 0.5, k = 2) from t = 0."""
    from oracle import sgn_oracle as O
    from sgn_inputs import workload
    box, (h, vx, vy, s), w = workload(WORKLOAD, **PARAMS)
    g = O.Grid(O.Config(nx=box.nx, ny=box.ny, Lx=box.Lx, Ly=box.Ly, gmres_tol=w["tol"],
                        gmres_restart=w["restart"], krasny=KRASNY))
    t0 = time.perf_counter()
    O.rk4(g, h, vx, vy, s, w["dt"], steps)
    dt = time.perf_counter() - t0
    usable, model = host_cpu()
    return {"value": box.nx * box.ny * steps / dt, "unit": UNIT, "cores": 1, "kind": "oracle",
            "host_cores_usable": usable, "host_cpu": model,
            "sample": f"{steps} RK4 step(s) of the {box.nx}x{box.ny} run a = {PARAMS['a']}, k = {PARAMS['k']} "
                      f"from t=0 (numpy FP64, single-threaded FFTs, one of the host's {usable} usable cores), "
                      f"{dt:.1f} s"}


def cpu_worker(run: int, steps: int):
    """One process of the all-core CPU baseline: the oracle, as it stands, on
    `steps` RK4 steps of run `run` of the nine from t = 0; prints its own
    start and end times (wall clock) as one JSON line."""
    from oracle import sgn_oracle as O
    from sgn_inputs import perturbed_soliton_sweep
    box, state, ak, w = perturbed_soliton_sweep(eps=PARAMS["eps"])
    h, vx, vy, s = (a[run].copy() for a in state)
    g = O.Grid(O.Config(nx=box.nx, ny=box.ny, Lx=box.Lx, Ly=box.Ly, gmres_tol=w["tol"],
                        gmres_restart=w["restart"], krasny=KRASNY))
    t0 = time.time()
    O.rk4(g, h, vx, vy, s, w["dt"], steps)
    t1 = time.time()
    print(json.dumps({"run": run, "t0": t0, "t1": t1, "points": box.nx * box.ny, "steps": steps}), flush=True)


def cpu_baseline_all_cores(steps: int):
    """The oracle on the host's cores: the nine runs (fewer if fewer cores may
    be used), one process each with one thread, `steps` RK4 steps from t = 0,
    all started together.  Throughput = the points x steps of all of them over
    the span from the first start to the last end.  Runs before the GPU is
    touched, so that every child is started from a process without it."""
    import subprocess
    usable, model = host_cpu()
    n = min(9, usable)
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", str(i),
                               "--cpu-steps", str(steps)], stdout=subprocess.PIPE, env=env) for i in range(n)]
    outs = []
    try:
        for pr in procs:
            so, _ = pr.communicate(timeout=600)
            if pr.returncode != 0:
                raise RuntimeError(f"CPU baseline worker exited with status {pr.returncode}")
            outs.append(json.loads(so.decode().strip().splitlines()[-1]))
    finally:
        for pr in procs:  # a worker still running after an error or the time limit
            if pr.poll() is None:
                pr.kill()
                pr.wait()
    span = max(o["t1"] for o in outs) - min(o["t0"] for o in outs)
    work = sum(o["points"] * o["steps"] for o in outs)
    return {"value": work / span, "unit": UNIT, "cores": n, "kind": "oracle", "host_cores_usable": usable,
            "host_cpu": model,
            "sample": f"{steps} RK4 step(s) of each of {n} of the nine 1024x512 runs from t=0, one single-threaded "
                      f"numpy FP64 process per run, all started together, {span:.1f} s from the first start to "
                      f"the last end"}


def progress(msg: str):
    """One progress line per phase on stderr (the JSON result goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_cpu():
    """Host cores this process may use and the CPU model (for cpu_baseline)."""
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        usable = os.cpu_count()
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:  # pragma: no cover
        pass
    return usable, model


def main():
    args = parse()
    if args.cpu_worker >= 0:
        cpu_worker(args.cpu_worker, args.cpu_steps)
        return
    global AUTOTUNE
    AUTOTUNE = not args.no_autotune
    if args.copy_calibration:
        copy_calibration(args.copy_calibration, max(args.steps, 1))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the solver is single-GPU.",
              file=sys.stderr)
        sys.exit(2)
    only = (args.precision_only or args.cnn_only or args.c3_only or args.single_only or args.main_only)
    cpu_all = None
    if not args.no_cpu_baseline and not only:
        cpu_all = cpu_baseline_all_cores(args.cpu_steps)
        progress("all-core CPU baseline done")
    import torch
    from paper_2306_09731_amd import sgn

    dev = torch.device("cuda:0")
    if args.precision_only:
        print(json.dumps({"precision_form": precision_form(sgn, torch, dev, args)}), flush=True)
        return
    if args.cnn_only:
        print(json.dumps({"cnn_forward": cnn_forward_run(sgn, torch, dev, args.steps)}), flush=True)
        return
    if args.c3_only:
        print(json.dumps({"c3": c3_run(sgn, torch, dev, args, args.c3_only)}), flush=True)
        return
    if args.single_only:
        print(json.dumps({"single_grid": single_grid_run(sgn, torch, dev, args)}), flush=True)
        return
    box, ak, w, ctx, f = sweep_context(sgn, torch, dev)
    if args.warmup > 0:
        sgn.sgn_rk4_step(ctx, *f, w["dt"], args.warmup)
    progress("warm-up done")
    # the same runs with the stage-increment initial guess (same tolerance),
    # timed first so that the headline run below is the last thing measured
    alt = None if args.main_only else timed_guess_run(sgn, torch, dev, args)
    progress("stage-increment guess run done")
    shape = sgn.sgn_launch_shape(ctx)
    labels = sweep_kernel_labels(box, shape)
    # the other Arnoldi kernel classes against the roofline, each on a copy
    # of the warm state (so the headline run starts where it would alone)
    others = {}
    if not args.main_only:
        for klass in labels:
            if klass == args.time_class:
                continue
            kk = [k for k, v in sgn.KERNEL_NAMES.items() if v == klass][0]
            _, _, kto = timed_kernel_run(sgn, torch, ctx, [t.clone() for t in f], w["dt"], args.steps, kk)
            others[klass] = roofline_entry(labels[klass], kto, SWEEP_WORKLOAD, klass)
        progress("other kernel classes timed")
    kind = [k for k, v in sgn.KERNEL_NAMES.items() if v == args.time_class][0]
    # events on every EVENT_PERIOD-th launch of the class: recording them on
    # every launch costs about 3% of the step
    elapsed, infos, kt = timed_kernel_run(sgn, torch, ctx, f, w["dt"], args.steps, kind)
    progress(f"timed run done: {elapsed * 1e3 / args.steps:.3f} ms per step")
    ctx.close()
    npts = len(ak) * box.nx * box.ny
    config = {
        "workload": SWEEP_WORKLOAD, "runs": len(ak), "nx": box.nx, "ny": box.ny, "Lx": box.Lx, "Ly": box.Ly,
        "a": sorted({a for a, _ in ak}), "k": sorted({k for _, k in ak}), "eps": PARAMS["eps"], "x0": -10.0,
        "dt": w["dt"], "gmres_tol": w["tol"], "gmres_restart": w["restart"], "krasny": KRASNY,
        "guess": "plain (warm start from the previous sigma)",
        "launch": "the nine runs as members of one context: one launch per kernel for all of them "
                  "(member index in blockIdx.z), each with its own GMRES state",
        "launch_shape": shape,
    }
    config.update(iters_summary(infos))
    config["per_run"] = [dict(a=a, k=k, iters_per_solve_mean=i.total_iters / max(i.solves, 1),
                              iters_per_solve_max=i.max_iters_per_solve) for (a, k), i in zip(ak, infos)]
    config["stage_increment_guess"] = alt
    out = {
        "metric": METRIC,
        "value": npts * args.steps / elapsed,
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
        "config": config,
        "roofline": roofline_entry(labels[args.time_class], kt, SWEEP_WORKLOAD, args.time_class),
    }
    if others:
        out["roofline_other_classes"] = others
    if not args.main_only:
        out["streams_form"] = streams_form(sgn, torch, dev, args, [t.clone() for t in f])
        progress("streams form done")
        out["single_grid"] = single_grid_run(sgn, torch, dev, args)
        progress("single-grid run done")
        out["sweep_single"] = sweep_single(sgn, torch, dev, args)
        progress("sweep one grid per context done")
        if args.t20_steps > 0:
            out["sweep_to_t20"] = sweep_to_t20(sgn, torch, dev, args.t20_steps)
            progress("nine runs to t = 20 done")
        from sgn_inputs import workload
        sbox, sstate, sw = workload(WORKLOAD, **PARAMS)
        out["graph_form"] = graph_form(sgn, torch, sbox, sstate, sw, dev, args)
        progress("graph form done")
        out["learned_form"] = learned_form(sgn, torch, dev, args)
        progress("learned form done")
        out["precision_form"] = precision_form(sgn, torch, dev, args)
        progress("precision form done")
        # the measured device-to-device copy rate beside the 8 TB/s peak
        copy_gbs = copy_peak_gbs(torch, dev)
        for entry in [out["roofline"]] + list(out.get("roofline_other_classes", {}).values()):
            entry["attainable_copy_gbs"] = copy_gbs
            entry["frac_of_copy"] = entry["achieved"] / copy_gbs if entry.get("achieved") else None
        out["batched_form"] = batched_form(sgn, torch, dev, args)
        progress("batched form done")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_steps)
        if cpu_all is not None:
            out["cpu_baseline"]["all_cores"] = cpu_all
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
