"""Training recipe of the learned initial guess (argument marshalling only:
recording, training and evaluation all run in the library's kernels).

    python -m paper_2306_09731_amd.learned [--out DIR] [--epochs N]

1. Record: RK4 trajectories of the solver at grid spacing dx = dy = 2 pi / 102.4
   (the spacing of the benchmark workloads) with the recorder attached; every
   solve writes the network input of its warm start and the target
   (sigma - sigma_prev) / |r0|.  Sources (about 10^4 samples): eight of the
   nine perturbed line solitons of the 1024 x 512 sweep and two Gaussian
   humps on 1024 x 512, the 2048^2 Gaussian of the precision form (cut into
   512 x 1024 tiles), oblique crossing solitons on 512 x 512 with amplitudes
   other than the evaluation's.
2. Train: Adam over the recorded samples, one sample per step, in a seeded
   order; the parameters start from He-normal weights (seeded).
3. Evaluate on two held-out workloads: the oblique crossing solitons on
   1024 x 1024 (a = 0.4, tol 1e-8) and the 1024 x 512 perturbed soliton
   (a = 0.5, eps = 0.01, k = 2, tol 1e-10): network MSE on recorded samples
   beside the zero and M^-1 r0 predictors, GMRES iterations per solve and
   time per RK4 step with the warm start and with the learned guess.

Writes DIR/learned_guess_params.npy (float32, SGN_CNN_PARAMS values) and
DIR/learned_guess_summary.json.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

from . import sgn

DT = 0.005
PKG = os.path.dirname(os.path.abspath(__file__))
PARAMS_FILE = os.path.join(PKG, "data", "learned_guess_params.npy")


def he_params(seed: int = 0) -> np.ndarray:
    """He-normal weights (std sqrt(2 / (9 fan_in)), fan_in = 3 for the first
    layer, 32 otherwise), zero biases, in the library's padded layout."""
    rng = np.random.default_rng(seed)
    ch = sgn.SGN_CNN_CH
    out = []
    dims = [3] + [ch] * (sgn.SGN_CNN_LAYERS - 1) + [1]
    for l in range(sgn.SGN_CNN_LAYERS):
        cin, cout = dims[l], dims[l + 1]
        w = np.zeros((9, ch, ch))
        w[:, :cout, :cin] = rng.normal(0.0, np.sqrt(2.0 / (9 * cin)), size=(9, cout, cin))
        out += [w.ravel(), np.zeros(ch)]
    return np.concatenate(out).astype(np.float32)


def _tensors(state, device):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).to(device) for a in state]


def training_sources():
    """(nx, ny, Lx, Ly, state, steps) of the recorded trajectories, all at the
    grid spacing of the benchmark workloads (2 pi / 102.4), none of them the
    held-out workloads of the evaluation: eight of the nine perturbed-soliton
    runs of the 1024 x 512 sweep (a in {0.2, 0.5, 1}, k in {1, 2, 4}, without
    the evaluated a = 0.5, k = 2), two
    Gaussian humps on 1024 x 512, the 2048^2 Gaussian of the precision form, and
    oblique crossing solitons on 512 x 512 with other amplitudes.  4 samples per
    step; about 10^4 samples in all."""
    from sgn_inputs import Box, gaussian_hump, perturbed_line_soliton
    from sgn_inputs.generators import SWEEP_AMPLITUDES, SWEEP_WAVENUMBERS, oblique_crossing_solitons
    out = []
    box = Box(1024, 512, 10.0, 5.0)
    for a in SWEEP_AMPLITUDES:
        for k in SWEEP_WAVENUMBERS:
            if (a, k) != (0.5, 2):
                out.append((1024, 512, 10.0, 5.0, perturbed_line_soliton(box, a=a, eps=0.01, k=k, x0=-10.0), 220))
    X, Y = box.mesh()
    for alpha in (0.3, 0.6):
        h = 1.0 + alpha * np.exp(-X * X - Y * Y)
        z = np.zeros_like(h)
        out.append((1024, 512, 10.0, 5.0, (h, z.copy(), z.copy(), z.copy()), 100))
    big = Box(2048, 2048, 20.0, 20.0)
    out.append((2048, 2048, 20.0, 20.0, gaussian_hump(big, alpha=0.5), 50))
    sq = Box(512, 512, 5.0, 5.0)
    for a in (0.2, 0.7):
        out.append((512, 512, 5.0, 5.0, oblique_crossing_solitons(sq, a=a), 60))
    return out


def record(device, steps_scale: float = 1.0, warmup_steps: int = 10, tol: float = 1e-10, log=None):
    """Record 4 samples per step of each source (one recorder tensor per
    source); steps_scale scales every source's step count."""
    import torch
    recs = []
    for nx, ny, Lx, Ly, state, steps in training_sources():
        steps = max(1, int(round(steps * steps_scale)))
        cfg = sgn.config_default(nx, ny, Lx, Ly, gmres_tol=tol, krasny=1e-12)
        ctx = sgn.sgn_init(cfg, device)
        f = _tensors(state, device)
        sgn.sgn_rk4_step(ctx, *f, DT, warmup_steps)
        rec = torch.zeros(4 * steps, 4, ny, nx, dtype=torch.float32, device=device)
        sgn.learned_guess_attach(ctx, None, rec)
        sgn.sgn_rk4_step(ctx, *f, DT, steps)
        sgn.learned_guess_attach(ctx, None)
        torch.cuda.synchronize()
        recs.append(rec)
        ctx.close()
        if log:
            log(source=f"{nx}x{ny}", samples=4 * steps)
    return recs


TRAIN_H, TRAIN_W = 512, 1024


def training_samples(recs):
    """(input, target) pairs on the 512 x 1024 training grid: samples of 512 x
    512 sources are repeated once along x (still periodic fields of the same
    spacing, which a translation-equivariant network sees alike); samples of
    2048 x 2048 sources are cut into eight 512 x 1024 tiles (the network's
    periodic padding then meets a seam at the tile edges, a few points of each
    tile)."""
    import torch
    out = []
    for rec in recs:
        for i in range(rec.shape[0]):
            x, t = sgn.record_sample(rec, i)
            H, W = t.shape
            if W < TRAIN_W:
                reps = TRAIN_W // W
                out.append((torch.cat([x] * reps, dim=1).contiguous(), torch.cat([t] * reps, dim=1).contiguous()))
            elif H > TRAIN_H:
                for y0 in range(0, H, TRAIN_H):
                    for x0 in range(0, W, TRAIN_W):
                        out.append((x[y0:y0 + TRAIN_H, x0:x0 + TRAIN_W].contiguous(),
                                    t[y0:y0 + TRAIN_H, x0:x0 + TRAIN_W].contiguous()))
            else:
                out.append((x.contiguous(), t.contiguous()))
    return out


def train(samples, device, epochs: int = 6, seed: int = 0, params=None, log=None):
    """Adam, one sample per step, in a seeded order; lr 1e-3, then 3e-4 for the
    last third of the epochs."""
    import torch
    net = sgn.cnn_init(TRAIN_H, TRAIN_W, device)
    sgn.cnn_set_params(net, he_params(seed) if params is None else params)
    rng = np.random.default_rng(seed)
    losses = []
    for epoch in range(epochs):
        lr = 1e-3 if epoch < (2 * epochs) // 3 else 3e-4
        ep = [sgn.cnn_train_step(net, *samples[j], lr) for j in rng.permutation(len(samples))]
        torch.cuda.synchronize()
        losses.append(float(np.mean(ep)))
        if log:
            log(epoch=epoch, loss=losses[-1])
    return sgn.cnn_get_params(net), losses


def _bf16(t):
    """Round to BF16 and back (round to nearest even), the precision of the
    network's activations and weights."""
    import torch
    return t.to(torch.bfloat16).to(t.dtype)


def ideal_guess_bound(ctx, box, f):
    """GMRES iterations of one stage-1 solve at the workload's tolerance from
    (a) the warm start sigma_prev, (b) sigma_prev + BF16(sigma* - sigma_prev),
    the best a network whose output carries BF16 rounding could return, and
    (c) the exact sigma* (to 1e-13): the most iterations any BF16 guess can
    save.  f = (h, vx, vy, sigma_prev) of the current state."""
    import torch
    h, vx, vy, sp = f
    b = torch.empty_like(h)
    t = torch.empty_like(h)
    sgn.sgn_derivative(ctx, 0, vx, b)
    sgn.sgn_derivative(ctx, 1, vy, t)
    b = -(b + t)
    tight = sgn.sgn_init(sgn.config_default(box.nx, box.ny, box.Lx, box.Ly, gmres_tol=1e-13, gmres_max_iters=400),
                         h.device)
    star = sp.clone()
    sgn.sgn_elliptic_solve(tight, h, b, star)
    tight.close()
    out = {}
    for key, guess in (("warm_start", sp.clone()), ("bf16_exact_correction", sp + _bf16(star - sp)),
                       ("exact", star.clone())):
        info = sgn.sgn_elliptic_solve(ctx, h, b, guess)
        out[key] = int(info.iters)
    return out


def fgmres_time_to_solution(ctx, box, f, params, reps: int = 3):
    """One elliptic solve of the current state (b = -div v) at the context's
    tolerance, from the warm start sigma_prev and from zero: plain GMRES
    against flexible GMRES preconditioned by the network (then the plain
    judge).  ms per solve (mean of reps) and iterations."""
    import torch
    h, vx, vy, sp = f
    b = torch.empty_like(h)
    t = torch.empty_like(h)
    sgn.sgn_derivative(ctx, 0, vx, b)
    sgn.sgn_derivative(ctx, 1, vy, t)
    b = -(b + t)
    net = sgn.cnn_init(box.ny, box.nx, h.device)
    sgn.cnn_set_params(net, params)
    out = {}
    for start in ("warm_start", "zero"):
        g0 = sp if start == "warm_start" else torch.zeros_like(sp)
        res = {}
        for solver in ("plain", "fgmres_learned"):
            el, info = 0.0, None
            for rep in range(reps + 1):  # the first run is not timed
                sig = g0.clone()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = (sgn.sgn_elliptic_solve(ctx, h, b, sig) if solver == "plain"
                        else sgn.sgn_elliptic_solve_fgmres(ctx, net, h, b, sig))
                torch.cuda.synchronize()
                if rep > 0:
                    el += time.perf_counter() - t0
            r = {"ms": el * 1e3 / reps}
            if solver == "plain":
                r["iters"] = int(info.iters)
            else:
                r.update(fgmres_iters=int(info.fgmres_iters), judge_iters=int(info.gmres_iters),
                         converged=bool(info.converged))
            res[solver] = r
        out[start] = res
    net.close()
    return out


def evaluate(params, device, name: str, steps: int = 40, warmup_steps: int = 10, record_n: int = 16):
    """The paper's warm start against the stage-increment guess and the
    learned guess (every stage, and once per RK4 step), on a named workload at
    its tolerance: ms per RK4 step (time to solution per step), GMRES
    iterations per solve; the network's mean squared error on recorded samples
    beside the zero and M^-1 r0 predictors; the cost of one forward pass; and
    the iterations of one solve from an ideal BF16-accurate guess."""
    import torch
    from sgn_inputs import workload
    box, state, w = workload(name)
    out = {"workload": name, "tol": w["tol"], "steps": steps}
    modes = (("warm_start", None), ("stage_increment", None), ("learned", 0xF), ("learned_once_per_step", 0x1))
    for mode, mask in modes:
        guess = sgn.SGN_GUESS_STAGE_INCREMENT if mode == "stage_increment" else sgn.SGN_GUESS_PREVIOUS
        cfg = sgn.config_default(box.nx, box.ny, box.Lx, box.Ly, gmres_tol=w["tol"], krasny=1e-12, guess=guess)
        ctx = sgn.sgn_init(cfg, device)
        f = _tensors(state, device)
        sgn.sgn_rk4_step(ctx, *f, DT, warmup_steps)
        net = None
        if mask is not None:
            net = sgn.cnn_init(box.ny, box.nx, device)
            sgn.cnn_set_params(net, params)
            sgn.learned_guess_attach(ctx, net)
            sgn.learned_guess_stages(ctx, mask)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = sgn.sgn_rk4_step(ctx, *f, DT, steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[mode] = {"ms_per_step": el * 1e3 / steps, "iters_per_solve": info.total_iters / info.solves,
                     "value": box.nx * box.ny * steps / el}
        if mode == "warm_start":
            out["ideal_guess_iters"] = ideal_guess_bound(ctx, box, f)
            out["fgmres_learned_preconditioner"] = fgmres_time_to_solution(ctx, box, f, params)
            # network error on samples of this workload beside the zero and M^-1 r0 predictors
            rec = torch.zeros(record_n, 4, box.ny, box.nx, dtype=torch.float32, device=device)
            sgn.learned_guess_attach(ctx, None, rec)
            sgn.sgn_rk4_step(ctx, *f, DT, record_n // 4)
            sgn.learned_guess_attach(ctx, None)
            net = sgn.cnn_init(box.ny, box.nx, device)
            sgn.cnn_set_params(net, params)
            pred = torch.empty(box.ny, box.nx, dtype=torch.float32, device=device)
            e_net, e_zero, e_mr = [], [], []
            for i in range(record_n):
                x, t = sgn.record_sample(rec, i)
                sgn.cnn_forward(net, x.contiguous(), pred)
                e_net.append(float(((pred - t) ** 2).mean()))
                e_zero.append(float((t ** 2).mean()))
                e_mr.append(float(((x[..., 1] - t) ** 2).mean()))
            out["sample_mse"] = {"network": float(np.mean(e_net)), "zero": float(np.mean(e_zero)),
                                 "minv_r0": float(np.mean(e_mr))}
            # one forward pass (input packing excluded), mean of 20
            x = sgn.record_sample(rec, 0)[0].contiguous()
            sgn.cnn_forward(net, x, pred)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(20):
                sgn.cnn_forward(net, x, pred)
            torch.cuda.synchronize()
            out["forward_ms"] = (time.perf_counter() - t0) * 1e3 / 20
            # marginal cost of one GMRES iteration: the same steps at a 100x
            # tighter tolerance from the same state, time and iterations differenced
            cfg2 = sgn.config_default(box.nx, box.ny, box.Lx, box.Ly, gmres_tol=w["tol"] / 100, krasny=1e-12)
            ctx2 = sgn.sgn_init(cfg2, device)
            f2 = _tensors(state, device)
            sgn.sgn_rk4_step(ctx2, *f2, DT, warmup_steps)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info2 = sgn.sgn_rk4_step(ctx2, *f2, DT, steps)
            torch.cuda.synchronize()
            ms2 = (time.perf_counter() - t0) * 1e3 / steps
            it2 = info2.total_iters / info2.solves
            ctx2.close()
            d_it = 4 * (it2 - out[mode]["iters_per_solve"])
            out["marginal_ms_per_gmres_iteration"] = (ms2 - out[mode]["ms_per_step"]) / d_it if d_it > 0 else None
        ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.dirname(PARAMS_FILE))
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--steps-scale", type=float, default=1.0,
                    help="scales every source's recorded steps (1: about 10^4 samples)")
    ap.add_argument("--device", default="cuda:0")
    args = ap.parse_args()
    t0 = time.time()

    def log(**kw):
        kw["t"] = round(time.time() - t0, 1)
        print(json.dumps(kw), flush=True)

    recs = record(args.device, args.steps_scale, log=log)
    samples = training_samples(recs)
    log(recorded=len(samples))
    params, losses = train(samples, args.device, args.epochs, log=log)
    del samples, recs
    os.makedirs(args.out, exist_ok=True)
    np.save(os.path.join(args.out, "learned_guess_params.npy"), params)
    summary = {"losses": losses, "evaluation": []}
    for name in ("crossing_solitons_1024x1024", "perturbed_soliton_1024x512"):
        summary["evaluation"].append(evaluate(params, args.device, name))
        log(**summary["evaluation"][-1])
    with open(os.path.join(args.out, "learned_guess_summary.json"), "w") as fh:
        json.dump(summary, fh, indent=1)


if __name__ == "__main__":
    main()
