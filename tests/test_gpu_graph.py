"""The captured RK4 step (sgn_rk4_step_graph).

Each RK4 step is one replay of a captured HIP graph whose solves run a fixed
budget of predicated Arnoldi steps per RK stage.  A solve that converges within
its budget executes exactly the arithmetic of the host-driven loop, so the
graph path must end bit for bit where sgn_rk4_step ends, replay after replay
(with the program's own eager work and synchronisations between the calls).
A budget too small for a solve must be detected on the device and its chunk
of steps redone host-driven from the chunk's checkpoint, again bit for bit,
whether that chunk is the first of the call or one in the middle.  One case is
also checked against the oracle directly."""
import os

import numpy as np
import pytest
import torch

from oracle import sgn_oracle as O
from paper_2306_09731_amd import sgn
from sgn_inputs import ensemble_member, workload

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)


def make(seed, nx, ny, arnoldi=None, stream=None, **kw):
    box, state, p = ensemble_member(seed, nx, ny)
    cfg = sgn.config_default(box.nx, box.ny, box.Lx, box.Ly, krasny=1e-12)
    for k, v in kw.items():
        setattr(cfg, k, v)
    old = os.environ.pop("SGN_ARNOLDI_KERNELS", None)
    try:
        if arnoldi is not None:
            os.environ["SGN_ARNOLDI_KERNELS"] = arnoldi
        ctx = sgn.sgn_init(cfg, DEV, stream=stream)
    finally:
        os.environ.pop("SGN_ARNOLDI_KERNELS", None)
        if old is not None:
            os.environ["SGN_ARNOLDI_KERNELS"] = old
    dt = torch.float32 if cfg.precision == sgn.SGN_FP32_MIXED else torch.float64
    f = [torch.from_numpy(np.ascontiguousarray(a)).to(DEV).to(dt) for a in state]
    torch.cuda.synchronize()  # the fields are written on the default stream
    return ctx, f, p["dt"]


CASES = {
    "fp64 three-kernel": dict(seed=0, nx=128, ny=64),
    "fp64 stage-increment guess": dict(seed=1, nx=256, ny=128, guess=sgn.SGN_GUESS_STAGE_INCREMENT),
    "fp32 mixed": dict(seed=2, nx=128, ny=128, precision=sgn.SGN_FP32_MIXED),
    "fp64 serial + two-thirds": dict(seed=3, nx=128, ny=64, arnoldi="serial", dealias=1),
    "fp64 chained + guess": dict(seed=5, nx=256, ny=256, arnoldi="chained", guess=sgn.SGN_GUESS_STAGE_INCREMENT),
    "fp64 2048-point columns": dict(seed=4, nx=64, ny=2048, guess=sgn.SGN_GUESS_STAGE_INCREMENT),
}


@pytest.mark.parametrize("name", list(CASES))
def test_graph_replays_match_host_loop(name):
    kw = dict(CASES[name])
    seed, nx, ny = kw.pop("seed"), kw.pop("nx"), kw.pop("ny")
    say(f"graph vs host loop: {name} {nx}x{ny}")
    ctx_h, fh, dt = make(seed, nx, ny, **kw)
    ctx_g, fg, _ = make(seed, nx, ny, **kw)
    nsteps = 4
    total_replayed = 0
    for call in range(3):
        ih = sgn.sgn_rk4_step(ctx_h, *fh, dt, nsteps)
        ig, replayed = sgn.sgn_rk4_step_graph(ctx_g, *fg, dt, nsteps)
        torch.cuda.synchronize()
        same = all(torch.equal(a, b) for a, b in zip(fh, fg))
        say(f"  call {call}: replayed {replayed}, identical {same}, iters host {ih.total_iters} graph "
            f"{ig.total_iters}, max/solve {ih.max_iters_per_solve} / {ig.max_iters_per_solve}")
        # the first two steps of the first call calibrate the budgets host-driven;
        # a chunk whose solves need more is redone host-driven
        total_replayed += replayed
        assert same
        assert ig.total_iters == ih.total_iters and ig.max_iters_per_solve == ih.max_iters_per_solve
        assert ig.solves == 4 * nsteps and not ig.any_unconverged and ig.min_h == ih.min_h
        # eager work of the program between the calls
        for a in fg:
            a.mul_(1.0)
        _ = sum(float(a.abs().sum()) for a in fg)
        torch.cuda.synchronize()
    assert total_replayed >= 4


def test_graph_budget_too_small_falls_back():
    say("graph budget 1: every call falls back to the host loop")
    ctx_h, fh, dt = make(7, 128, 64)
    ctx_g, fg, _ = make(7, 128, 64)
    for call in range(2):
        ih = sgn.sgn_rk4_step(ctx_h, *fh, dt, 3)
        ig, replayed = sgn.sgn_rk4_step_graph(ctx_g, *fg, dt, 3, iter_budget=1)
        torch.cuda.synchronize()
        same = all(torch.equal(a, b) for a, b in zip(fh, fg))
        say(f"  call {call}: replayed {replayed}, identical {same}, iters {ig.total_iters} / {ih.total_iters}")
        assert not replayed and same and ig.total_iters == ih.total_iters
    # an explicit budget that suffices replays
    need = ih.max_iters_per_solve + 1
    ih = sgn.sgn_rk4_step(ctx_h, *fh, dt, 3)
    ig, replayed = sgn.sgn_rk4_step_graph(ctx_g, *fg, dt, 3, iter_budget=need)
    torch.cuda.synchronize()
    assert replayed and all(torch.equal(a, b) for a, b in zip(fh, fg))


@pytest.mark.parametrize("name,kw", [("plain", {}), ("stage-increment guess",
                                                   {"guess": sgn.SGN_GUESS_STAGE_INCREMENT})])
def test_graph_chunk_redone_mid_call(name, kw):
    """Fixed budgets below what some solves need: the call's chunks of sixteen
    replays either pass or are restored and redone host-driven.  The first
    solves of a call start from a poor sigma and need the most iterations, so
    a budget between the later solves' need and the first ones' makes the
    first chunk fail and later chunks pass; every outcome must equal the host
    loop bit for bit."""
    say(f"graph chunks redone mid-call: {name}")
    nsteps = 40
    ctx_h, fh, dt = make(11, 128, 64, **kw)
    ih = sgn.sgn_rk4_step(ctx_h, *fh, dt, nsteps)
    torch.cuda.synchronize()
    mixed = False
    for budget in range(ih.max_iters_per_solve, 0, -1):
        ctx_g, fg, _ = make(11, 128, 64, **kw)
        ig, nrep = sgn.sgn_rk4_step_graph(ctx_g, *fg, dt, nsteps, iter_budget=budget)
        torch.cuda.synchronize()
        same = all(torch.equal(a, b) for a, b in zip(fh, fg))
        say(f"  budget {budget}: {nrep} of {nsteps} steps replayed, identical {same}, iters {ig.total_iters} / "
            f"{ih.total_iters}")
        assert same and ig.total_iters == ih.total_iters and ig.max_iters_per_solve == ih.max_iters_per_solve
        assert ig.solves == 4 * nsteps and nrep % 8 == 0
        mixed = mixed or 0 < nrep < nsteps
        ctx_g.close()
        if nrep == 0:
            break
    assert mixed


def test_graph_automatic_budgets_grow():
    """Automatic per-stage budgets, calibrated on the first call, meet a
    harder state on the same context (a hump added to h, sigma restarted from
    zero): chunks whose solves exceed the budgets are redone host-driven and
    the budgets grow; every call equals the host loop bit for bit, and the last
    call replays."""
    say("graph automatic budgets grow")
    ctx_g, fg, dt = make(12, 128, 64)
    ctx_h, fh, _ = make(12, 128, 64)
    for call in range(3):
        ih = sgn.sgn_rk4_step(ctx_h, *fh, dt, 8)
        ig, nrep = sgn.sgn_rk4_step_graph(ctx_g, *fg, dt, 8)
        torch.cuda.synchronize()
        same = all(torch.equal(a, b) for a, b in zip(fh, fg))
        say(f"  call {call}: {nrep} replayed, identical {same}, iters {ig.total_iters} / {ih.total_iters}")
        assert same and ig.total_iters == ih.total_iters
        if call == 0:
            # a harder state: a hump added to h, sigma restarted from zero
            bump = 0.3 * torch.exp(-torch.linspace(-3, 3, fg[0].shape[1], device=DEV, dtype=fg[0].dtype) ** 2)
            for f in (fg, fh):
                f[0].add_(bump[None, :])
                f[3].zero_()
            torch.cuda.synchronize()
    assert nrep > 0


def test_graph_argument_checks_and_zero_steps():
    ctx, f, dt = make(0, 64, 64)
    with pytest.raises(sgn.SgnError):
        sgn.sgn_rk4_step_graph(ctx, *f, dt, 1, iter_budget=ctx.cfg.gmres_restart + 1)
    before = [a.clone() for a in f]
    info, replayed = sgn.sgn_rk4_step_graph(ctx, *f, dt, 0)
    torch.cuda.synchronize()
    assert not replayed and info.solves == 0
    assert all(torch.equal(a, b) for a, b in zip(f[:3], before[:3]))


def test_graph_on_a_side_stream_and_new_fields():
    """Context on a non-default stream; a second set of fields makes the
    cached graph stale and is recaptured."""
    say("graph on a side stream, two field sets")
    st = torch.cuda.Stream(DEV)
    ctx_g, fg, dt = make(9, 128, 128, stream=st)
    ctx_h, fh, _ = make(9, 128, 128)
    _, fg2, _ = make(9, 128, 128)
    with torch.cuda.stream(st):
        ig, r1 = sgn.sgn_rk4_step_graph(ctx_g, *fg, dt, 3)
        ig2, r2 = sgn.sgn_rk4_step_graph(ctx_g, *fg2, dt, 3)
        # work ordered after the call on the same stream sees its results
        sums = [a.sum() for a in fg2]
    ih = sgn.sgn_rk4_step(ctx_h, *fh, dt, 3)
    torch.cuda.synchronize()
    assert r1 and r2
    assert all(torch.equal(a, b) for a, b in zip(fh, fg))
    assert all(torch.equal(a, b) for a, b in zip(fh, fg2))
    assert all(float(s) == float(a.sum()) for s, a in zip(sums, fh))
    assert ig.total_iters == ih.total_iters == ig2.total_iters


def test_graph_line_soliton_against_oracle():
    """The 128x64 line soliton workload, 40 graph steps in two calls, against
    the oracle (the host loop's own parity gate: 1e-10 relative)."""
    box, (h, vx, vy, s), w = workload("line_soliton_128x64")
    cfg = sgn.config_default(box.nx, box.ny, box.Lx, box.Ly, gmres_tol=w["tol"], gmres_restart=w["restart"])
    ctx = sgn.sgn_init(cfg, DEV)
    f = [torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in (h, vx, vy, s)]
    i1, r1 = sgn.sgn_rk4_step_graph(ctx, *f, w["dt"], 20)
    i2, r2 = sgn.sgn_rk4_step_graph(ctx, *f, w["dt"], 20)
    torch.cuda.synchronize()
    g = O.Grid(O.Config(nx=box.nx, ny=box.ny, Lx=box.Lx, Ly=box.Ly, gmres_tol=w["tol"], gmres_restart=w["restart"]))
    oh, ovx, ovy, os_, o1 = O.rk4(g, h, vx, vy, s, w["dt"], 20)
    oh, ovx, ovy, os_, o2 = O.rk4(g, oh, ovx, ovy, os_, w["dt"], 20)
    gh, gvx = (a.cpu().numpy() for a in f[:2])
    eh = np.abs(gh - oh).max() / np.abs(oh - 1.0).max()
    ev = np.abs(gvx - ovx).max() / np.abs(ovx).max()
    say(f"graph line soliton x40: h {eh:.2e} vx {ev:.2e}; iters {i1.total_iters + i2.total_iters} "
        f"oracle {o1.total_iters + o2.total_iters}; replayed {r1} {r2}")
    assert r1 and r2 and eh < 1e-10 and ev < 1e-10
    assert abs(i1.total_iters + i2.total_iters - o1.total_iters - o2.total_iters) <= 8
