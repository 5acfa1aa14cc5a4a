"""Ensemble members in one launch (sgn_config.batch = B > 1) through the C-ABI.

Each member of a B-member context must end bitwise equal to a context with
batch = 1 run on that member's fields alone (same kernels, same arithmetic,
only the member index in blockIdx.z differs), with the same iteration counts,
restarts and status, under every Arnoldi schedule and in both precisions;
and one member per grid size is compared with the FP64 oracle (gates of the
parity tests: 1e-10 after RK4 steps at tol 1e-10 / 1e-12)."""
import os

import numpy as np
import pytest
import torch

from oracle import sgn_oracle as O
from paper_2306_09731_amd import sgn
from sgn_inputs import Box, perturbed_line_soliton, random_smooth_field, random_state

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)


def ctx_for(nx, ny, Lx, Ly, batch, arnoldi=None, **kw):
    cfg = sgn.config_default(nx, ny, Lx, Ly, batch=batch, **kw)
    old = os.environ.pop("SGN_ARNOLDI_KERNELS", None)
    try:
        if arnoldi is not None:
            os.environ["SGN_ARNOLDI_KERNELS"] = arnoldi
        return sgn.sgn_init(cfg, DEV)
    finally:
        os.environ.pop("SGN_ARNOLDI_KERNELS", None)
        if old is not None:
            os.environ["SGN_ARNOLDI_KERNELS"] = old


def soliton_members(box, params):
    """Perturbed line solitons (a, eps, k) as [B][ny][nx] arrays."""
    st = [perturbed_line_soliton(box, a=a, eps=e, k=k, x0=-0.5 * np.pi * box.Lx) for a, e, k in params]
    return [np.stack([m[i] for m in st]) for i in range(4)]


def to_dev(a, dt):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV).to(dt)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


PARAMS = [(0.2, 0.05, 1), (0.5, 0.01, 2), (1.0, 0.02, 4)]


@pytest.mark.parametrize("nx,ny", [(128, 64), (64, 16)])
@pytest.mark.parametrize("arnoldi", ["fused", "chained", "serial"])
@pytest.mark.parametrize("prec", [sgn.SGN_FP64, sgn.SGN_FP32_MIXED])
def test_members_rk4_bitwise_equal_to_single_contexts(arnoldi, prec, nx, ny):
    """128x64 takes the XCD-grouped block order of the two-chain row kernel
    (row pairs a multiple of 16), 64x16 the plain one."""
    box = Box(nx, ny, 10.0 * nx / 128, 5.0 * ny / 64)
    fields = soliton_members(box, PARAMS)
    B = len(PARAMS)
    dt = torch.float64 if prec == sgn.SGN_FP64 else torch.float32
    kw = dict(precision=prec, gmres_tol=1e-10, krasny=1e-12)
    cb = ctx_for(nx, ny, box.Lx, box.Ly, B, arnoldi, **kw)
    fb = [to_dev(a, dt) for a in fields]
    infos = sgn.sgn_rk4_step(cb, *fb, 0.01, 6)
    got = [host(t) for t in fb]
    for k in range(B):
        cs = ctx_for(nx, ny, box.Lx, box.Ly, 1, arnoldi, **kw)
        fs = [to_dev(a[k], dt) for a in fields]
        info = sgn.sgn_rk4_step(cs, *fs, 0.01, 6)
        same = all(np.array_equal(got[i][k], host(fs[i])) for i in range(4))
        say(f"members {nx}x{ny} {arnoldi} {'fp64' if prec == 0 else 'fp32'} member {k}: iters {infos[k].total_iters} "
            f"(single {info.total_iters}), bitwise equal {same}")
        assert same
        assert infos[k].total_iters == info.total_iters
        assert infos[k].max_iters_per_solve == info.max_iters_per_solve
        cs.close()
    # members converge at different counts (the test exercises the per-member exits)
    assert len({i.total_iters for i in infos}) > 1
    cb.close()


def test_members_solve_with_restarts_and_iteration_cap():
    """Restart length 3: members of different depth contrast need different
    numbers of cycles; one member hits the iteration cap.  Each member's sigma,
    iterations, restarts and convergence flag equal its single-context solve."""
    nx, ny = 64, 32
    B = 4
    rng = np.random.default_rng(3)
    amps = [0.05, 0.3, 0.6, 0.8]
    h = np.stack([1.0 + a * random_smooth_field(rng, ny, nx, kmax=4) for a in amps])
    b = np.stack([random_smooth_field(rng, ny, nx, kmax=6) for _ in amps])
    kw = dict(gmres_tol=1e-12, gmres_restart=3, gmres_max_iters=24)
    cb = ctx_for(nx, ny, 1.0, 1.0, B, **kw)
    sig = torch.zeros(B, ny, nx, dtype=torch.float64, device=DEV)
    infos = sgn.sgn_elliptic_solve(cb, to_dev(h, torch.float64), to_dev(b, torch.float64), sig)
    got = host(sig)
    conv = []
    for k in range(B):
        cs = ctx_for(nx, ny, 1.0, 1.0, 1, **kw)
        s1 = torch.zeros(ny, nx, dtype=torch.float64, device=DEV)
        i1 = sgn.sgn_elliptic_solve(cs, to_dev(h[k], torch.float64), to_dev(b[k], torch.float64), s1)
        say(f"member {k} (depth contrast {amps[k]}): iters {infos[k].iters} restarts {infos[k].restarts} "
            f"converged {infos[k].converged}; single: {i1.iters} {i1.restarts} {i1.converged}")
        assert np.array_equal(got[k], host(s1))
        assert (infos[k].iters, infos[k].restarts, infos[k].converged) == (i1.iters, i1.restarts, i1.converged)
        assert infos[k].rel_resid_true == i1.rel_resid_true
        conv.append(infos[k].converged)
        cs.close()
    assert len({i.restarts for i in infos}) > 1
    # one member against the oracle
    g = O.Grid(O.Config(nx=nx, ny=ny, Lx=1.0, Ly=1.0))
    ref, _ = O.gmres(g, h[0], b[0], np.zeros_like(b[0]), 1e-13, 20, 400)
    assert np.abs(got[0] - ref).max() / np.abs(ref).max() < 1e-10
    cb.close()


def test_members_rhs_invariants_and_guess():
    nx, ny = 64, 64
    box = Box(nx, ny, 2.0, 2.0)
    B = 3
    rng = np.random.default_rng(5)
    st = [random_state(rng, box, amp_h=0.2 + 0.1 * k, amp_v=0.2, kmax=5) for k in range(B)]
    fields = [np.stack([m[i] for m in st]) for i in range(4)]
    cb = ctx_for(nx, ny, 2.0, 2.0, B, gmres_tol=1e-12)
    outs = [torch.empty(B, ny, nx, dtype=torch.float64, device=DEV) for _ in range(3)]
    sig = to_dev(fields[3], torch.float64)
    sgn.sgn_rhs(cb, *(to_dev(a, torch.float64) for a in fields[:3]), sig, *outs)
    invs = sgn.sgn_invariants(cb, *(to_dev(a, torch.float64) for a in fields))
    g = O.Grid(O.Config(nx=nx, ny=ny, Lx=2.0, Ly=2.0, gmres_tol=1e-12))
    for k in range(B):
        cs = ctx_for(nx, ny, 2.0, 2.0, 1, gmres_tol=1e-12)
        o1 = [torch.empty(ny, nx, dtype=torch.float64, device=DEV) for _ in range(3)]
        s1 = to_dev(fields[3][k], torch.float64)
        sgn.sgn_rhs(cs, *(to_dev(a[k], torch.float64) for a in fields[:3]), s1, *o1)
        assert all(np.array_equal(host(outs[i])[k], host(o1[i])) for i in range(3))
        assert np.array_equal(host(sig)[k], host(s1))
        inv1 = sgn.sgn_invariants(cs, *(to_dev(a[k], torch.float64) for a in fields))
        assert invs[k] == inv1
        cs.close()
    r = O.rhs(g, *(a[1] for a in fields))
    e = np.abs(host(outs[0])[1] - r.dh).max() / np.abs(r.dh).max()
    say(f"members rhs: member 1 dh vs oracle {e:.1e}")
    assert e < 1e-10
    # stage-increment guess with members
    cg = ctx_for(nx, ny, 2.0, 2.0, B, gmres_tol=1e-10, guess=sgn.SGN_GUESS_STAGE_INCREMENT)
    fg = [to_dev(a, torch.float64) for a in fields]
    ig = sgn.sgn_rk4_step(cg, *fg, 0.005, 4)
    for k in range(B):
        cs = ctx_for(nx, ny, 2.0, 2.0, 1, gmres_tol=1e-10, guess=sgn.SGN_GUESS_STAGE_INCREMENT)
        f1 = [to_dev(a[k], torch.float64) for a in fields]
        i1 = sgn.sgn_rk4_step(cs, *f1, 0.005, 4)
        assert all(np.array_equal(host(fg[i])[k], host(f1[i])) for i in range(4))
        assert ig[k].total_iters == i1.total_iters
        cs.close()


def test_members_full_size_1024x512_sweep():
    """The 1024x512 workload's nine (a, k) runs as one nine-member context:
    two RK4 steps; members 0 and 8 bitwise equal to single contexts, member 4
    (a = 0.5, k = 2) against the oracle."""
    nx, ny = 1024, 512
    box = Box(nx, ny, 10.0, 5.0)
    params = [(a, 0.01, k) for a in (0.2, 0.5, 1.0) for k in (1, 2, 4)]
    st = [perturbed_line_soliton(box, a=a, eps=e, k=k, x0=-10.0) for a, e, k in params]
    fields = [np.stack([m[i] for m in st]) for i in range(4)]
    kw = dict(gmres_tol=1e-10, krasny=1e-12)
    cb = ctx_for(nx, ny, 10.0, 5.0, 9, **kw)
    fb = [to_dev(a, torch.float64) for a in fields]
    infos = sgn.sgn_rk4_step(cb, *fb, 0.005, 2)
    got = [host(t) for t in fb]
    say("nine members, iterations per member: " + " ".join(str(i.total_iters) for i in infos))
    for k in (0, 8):
        cs = ctx_for(nx, ny, 10.0, 5.0, 1, **kw)
        f1 = [to_dev(a[k], torch.float64) for a in fields]
        i1 = sgn.sgn_rk4_step(cs, *f1, 0.005, 2)
        assert all(np.array_equal(got[i][k], host(f1[i])) for i in range(4)), k
        assert infos[k].total_iters == i1.total_iters
        cs.close()
    g = O.Grid(O.Config(nx=nx, ny=ny, Lx=10.0, Ly=5.0, gmres_tol=1e-10, krasny=1e-12))
    oh, ovx, ovy, _, _ = O.rk4(g, *(a[4] for a in fields), 0.005, 2)
    eh = np.abs(got[0][4] - oh).max() / np.abs(oh - 1.0).max()
    ev = np.abs(got[1][4] - ovx).max() / np.abs(ovx).max()
    say(f"  member 4 vs oracle: h {eh:.1e} vx {ev:.1e}")
    assert eh < 1e-10 and ev < 1e-10


def test_members_refusals_and_layout():
    cfg1 = sgn.config_default(64, 64, 1.0, 1.0)
    cfg4 = sgn.config_default(64, 64, 1.0, 1.0, batch=4)
    assert sgn.sgn_workspace_bytes(cfg4) == 4 * sgn.sgn_workspace_bytes(cfg1)
    cb = sgn.sgn_init(cfg4, DEV)
    f = [torch.ones(4, 64, 64, dtype=torch.float64, device=DEV) for _ in range(4)]
    with pytest.raises(sgn.SgnError) as e:
        sgn.sgn_rk4_step_graph(cb, *f, 0.01, 1)
    assert e.value.status == sgn.SGN_ERR_UNSUPPORTED
    with pytest.raises(ValueError):
        sgn.sgn_rk4_step(cb, *[torch.ones(64, 64, dtype=torch.float64, device=DEV)] * 4, 0.01, 1)
    # a bad member is reported
    bad = torch.ones(4, 64, 64, dtype=torch.float64, device=DEV)
    bad[2, 3, 3] = -1.0
    with pytest.raises(sgn.SgnError) as e:
        sgn.sgn_rk4_step(cb, bad, f[1], f[2], f[3], 0.01, 1)
    assert e.value.status == sgn.SGN_ERR_CAVITATION and "member 2" in str(e.value)


def test_members_autotune_radix_and_results():
    """The autotuner on a four-member 1024x512 context: it may pick the radix-8
    two-chain row kernel; whatever it picks, each member's RK4 steps equal a
    single context's to the FP64 parity gate (the radix changes the rounding
    of the row transforms only), and member 1 matches the oracle."""
    nx, ny = 1024, 512
    box = Box(nx, ny, 10.0, 5.0)
    params = [(0.2, 0.01, 1), (0.5, 0.01, 2), (1.0, 0.01, 4), (0.5, 0.02, 1)]
    st = [perturbed_line_soliton(box, a=a, eps=e, k=k, x0=-10.0) for a, e, k in params]
    fields = [np.stack([m[i] for m in st]) for i in range(4)]
    kw = dict(gmres_tol=1e-10, krasny=1e-12)
    results = {}
    for rr in ("0", "8"):
        os.environ["SGN_ROW_RADIX"] = rr
        try:
            cb = ctx_for(nx, ny, 10.0, 5.0, len(params), **kw)
        finally:
            os.environ.pop("SGN_ROW_RADIX", None)
        assert sgn.sgn_launch_shape(cb)["row_radix"] == int(rr)
        fb = [to_dev(a, torch.float64) for a in fields]
        sgn.sgn_rk4_step(cb, *fb, 0.005, 2)
        results[rr] = [host(t) for t in fb]
        cb.close()
    e = max(np.abs(results["8"][i] - results["0"][i]).max() / max(np.abs(results["0"][i] - (1.0 if i == 0 else 0.0)).max(), 1e-300)
            for i in range(3))
    say(f"members radix 8 vs 4 after two steps: {e:.1e}")
    assert e < 1e-12
    g = O.Grid(O.Config(nx=nx, ny=ny, Lx=10.0, Ly=5.0, gmres_tol=1e-10, krasny=1e-12))
    oh, ovx, _, _, _ = O.rk4(g, *(a[1] for a in fields), 0.005, 2)
    assert np.abs(results["8"][0][1] - oh).max() / np.abs(oh - 1.0).max() < 1e-10
    cb = ctx_for(nx, ny, 10.0, 5.0, len(params), **kw)
    chosen = sgn.sgn_autotune(cb)
    shape = sgn.sgn_launch_shape(cb)
    say(f"members autotune: schedule {chosen}, shape {shape}")
    fb = [to_dev(a, torch.float64) for a in fields]
    infos = sgn.sgn_rk4_step(cb, *fb, 0.005, 2)
    for k in (0, 3):
        got = host(fb[0])[k]
        assert np.abs(got - results["0"][0][k]).max() / np.abs(results["0"][0][k] - 1.0).max() < 1e-12
    assert all(i.any_unconverged == 0 for i in infos)
    cb.close()


def test_member_contexts_in_one_ensemble_call():
    """Two member contexts (three and two members of a 128x64 grid) advanced by
    one sgn_rk4_step_ensemble call, each on a stream of its own, end bitwise
    equal to the same contexts stepped one after the other, with one info per
    member in order; the captured-graph ensemble refuses member contexts."""
    nx, ny = 128, 64
    box = Box(nx, ny, 2.0, 2.0)
    params = PARAMS + [(0.3, 0.02, 2), (0.7, 0.01, 1)]
    fields = soliton_members(box, params)
    splits = [(0, 3), (3, 5)]

    def make():
        cs, fs = [], []
        for a, b in splits:
            cfg = sgn.config_default(nx, ny, 2.0, 2.0, batch=b - a, gmres_tol=1e-10)
            cs.append(sgn.sgn_init(cfg, DEV, stream=torch.cuda.Stream(DEV)))
            fs.append([to_dev(x[a:b], torch.float64) for x in fields])
        torch.cuda.synchronize()
        return cs, fs

    c1, f1 = make()
    infos = sgn.sgn_rk4_step_ensemble(c1, f1, [0.005, 0.005], 3)
    c2, f2 = make()
    ref = []
    for c, f in zip(c2, f2):
        ref += sgn.sgn_rk4_step(c, *f, 0.005, 3)
    say("member contexts in one ensemble call, iterations: " + " ".join(str(i.total_iters) for i in infos))
    assert len(infos) == len(params)
    assert [i.total_iters for i in infos] == [r.total_iters for r in ref]
    for fa, fb in zip(f1, f2):
        assert all(np.array_equal(host(fa[i]), host(fb[i])) for i in range(4))
    with pytest.raises(sgn.SgnError):
        sgn.sgn_rk4_step_ensemble(c1, f1, [0.005, 0.005], 1, graphs=True)
    for c in c1 + c2:
        c.close()
