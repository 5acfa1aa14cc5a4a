"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Every comparison uses the same seeded inputs on both sides.  Errors are
relative: max |gpu - oracle| / max |oracle - background|, with background
h_inf for h and 0 otherwise.  Tolerances:
  * single spectral passes (derivatives, operator, preconditioner, Krasny):
    1e-12 (a few hundred ulps of FFT rounding, amplified by k_max);
  * GMRES solves and RHS at tol 1e-12: 1e-10 (two different Gram-Schmidt
    orders on a problem with condition number ~10);
  * 200 RK4 steps of the 128x64 line soliton at tol 1e-10: 1e-10 (the
    accuracy target for the FP64 path).
"""
import math
import os

import numpy as np
import pytest
import torch

from oracle import sgn_oracle as O
from paper_2306_09731_amd import sgn
from sgn_inputs import Box, line_soliton, perturbed_line_soliton, random_smooth_field, random_state, workload

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)


def mk(nx, ny, Lx, Ly, arnoldi=None, **kw):
    """Context + oracle grid.  arnoldi selects the Arnoldi kernel variant
    ("fused", "chained" or "serial"; None = the library default)."""
    cfg = sgn.config_default(nx, ny, Lx, Ly)
    for k, v in kw.items():
        setattr(cfg, k, v)
    old = os.environ.pop("SGN_ARNOLDI_KERNELS", None)
    try:
        if arnoldi is not None:
            os.environ["SGN_ARNOLDI_KERNELS"] = arnoldi
        ctx = sgn.sgn_init(cfg, DEV)
    finally:
        os.environ.pop("SGN_ARNOLDI_KERNELS", None)
        if old is not None:
            os.environ["SGN_ARNOLDI_KERNELS"] = old
    return ctx, O.Grid(O.Config(nx=nx, ny=ny, Lx=Lx, Ly=Ly,
                                **{k: v for k, v in kw.items() if k in O.Config.__dataclass_fields__}))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, ref, bg=0.0):
    scale = np.abs(ref - bg).max()
    return np.abs(a - ref).max() / (scale if scale > 0 else 1.0)


SIZES = [(8, 8), (16, 32), (32, 16), (128, 64), (256, 16), (512, 256), (1024, 512), (2048, 16), (16, 2048),
         (4096, 8), (8, 4096)]


@pytest.mark.parametrize("nx,ny", SIZES)
def test_derivatives(nx, ny):
    say(f"derivatives {nx}x{ny}")
    ctx, g = mk(nx, ny, 1.7, 0.9)
    rng = np.random.default_rng(nx * 7 + ny)
    f = random_smooth_field(rng, ny, nx, kmax=min(6, nx // 2 - 1, ny // 2 - 1))
    f += 0.1 * rng.standard_normal((ny, nx))   # energy up to the Nyquist modes
    out = torch.empty_like(dev(f))
    sgn.sgn_derivative(ctx, 0, dev(f), out)
    assert rel(host(out), O.d_x(g, f)) < 1e-12
    sgn.sgn_derivative(ctx, 1, dev(f), out)
    assert rel(host(out), O.d_y(g, f)) < 1e-12


@pytest.mark.parametrize("nx,ny", [(8, 8), (64, 32), (128, 64), (256, 128), (1024, 512), (16, 1024), (2048, 32),
                                   (32, 2048), (4096, 16), (16, 4096)])
def test_operator_and_preconditioner(nx, ny):
    say(f"operator {nx}x{ny}")
    ctx, g = mk(nx, ny, 2.0, 1.3)
    rng = np.random.default_rng(nx + 3 * ny)
    h, _, _, s = random_state(rng, Box(nx, ny, 2.0, 1.3), amp_h=0.4,
                              kmax=min(6, nx // 2 - 1, ny // 2 - 1))
    s = s + 0.01 * rng.standard_normal((ny, nx))
    out = torch.empty_like(dev(s))
    sgn.sgn_apply_operator(ctx, dev(h), dev(s), out, False)
    assert rel(host(out), O.apply_L(g, h, s)) < 1e-12
    sgn.sgn_apply_operator(ctx, dev(h), dev(s), out, True)
    assert rel(host(out), O.apply_Minv(g, O.apply_L(g, h, s))) < 1e-12
    sgn.sgn_apply_precond(ctx, dev(s), out)
    assert rel(host(out), O.apply_Minv(g, s)) < 1e-12


@pytest.mark.parametrize("nx,ny", [(32, 16), (128, 64), (64, 256)])
def test_krasny_filter(nx, ny):
    say(f"krasny {nx}x{ny}")
    ctx, g = mk(nx, ny, 1.0, 1.0, krasny=1e-12)
    X, Y = np.meshgrid(g.x, g.y)
    rng = np.random.default_rng(5)
    f = 1.0 + 0.3 * np.cos(X) * np.sin(2 * Y)
    # modes straddling the threshold, incl. the x- and y-Nyquist columns/rows
    for amp, kx, ky in [(3e-12, 3, 1), (1e-12, 5, 2), (8e-13, 2, 0), (2e-11, nx // 2, 0), (1e-13, nx // 2, 3),
                        (5e-12, 0, ny // 2), (1e-13, 1, ny // 2), (4e-12, 0, 3), (1.5e-12, 0, 5)]:
        f = f + amp * np.cos(kx * X + ky * Y + rng.random())
    t = dev(f)
    sgn.sgn_krasny_filter(ctx, t)
    ref = O.krasny(g, f, 1e-12)
    assert np.abs(host(t) - ref).max() < 1e-14


@pytest.mark.parametrize("krasny", [1e-12, 0.0])
@pytest.mark.parametrize("nx,ny", [(32, 16), (128, 64), (64, 256), (2048, 16)])
def test_two_thirds_filter(nx, ny, krasny):
    say(f"two-thirds filter {nx}x{ny} krasny {krasny}")
    ctx, g = mk(nx, ny, 1.0, 1.0, krasny=krasny, dealias=1)
    X, Y = np.meshgrid(g.x, g.y)
    rng = np.random.default_rng(nx + ny)
    f = 1.0 + 0.3 * np.cos(X) * np.sin(2 * Y)
    # modes on both sides of the 1/3 band edge in x and y, the Nyquist lines, small modes
    ex, ey = nx // 3, ny // 3
    for amp, kx, ky in [(0.1, ex, 0), (0.1, ex + 1, 0), (0.1, 0, ey), (0.1, 0, ey + 1), (0.1, ex, ey),
                        (0.1, ex + 1, ey), (0.1, ex, -ey - 1), (0.1, nx // 2, 0), (0.1, nx // 2, 3),
                        (0.1, 0, ny // 2), (0.1, 2, ny // 2), (3e-12, 3, 1), (8e-13, 2, 0), (1e-13, 0, 1)]:
        f = f + amp * np.cos(kx * X + ky * Y + rng.random())
    t = dev(f)
    sgn.sgn_krasny_filter(ctx, t)
    ref = O.two_thirds(g, O.krasny(g, f, krasny) if krasny > 0 else f)
    assert np.abs(host(t) - ref).max() < 1e-14


def test_rk4_two_thirds_rule():
    say("rk4 random state with Krasny and the two-thirds rule")
    nx, ny = 64, 32
    ctx, g = mk(nx, ny, 1.0, 1.0, gmres_tol=1e-12, krasny=1e-12, dealias=1)
    rng = np.random.default_rng(19)
    h, vx, vy, s = random_state(rng, Box(nx, ny, 1.0, 1.0), amp_h=0.2, amp_v=0.1, kmax=12)
    gh, gvx, gvy, gs, info = run_gpu_rk4(ctx, h, vx, vy, s, 0.005, 5)
    oh, ovx, ovy, os_, oinfo = O.rk4(g, h, vx, vy, s, 0.005, 5)
    assert rel(gh, oh, 1.0) < 1e-10 and rel(gvx, ovx) < 1e-10 and rel(gvy, ovy) < 1e-10
    # the state is band-limited after the step
    for a in (gh, gvx, gvy):
        c = np.abs(np.fft.fft2(a)) / a.size
        mx = np.abs(np.fft.fftfreq(nx) * nx)
        my = np.abs(np.fft.fftfreq(ny) * ny)
        outside = (3 * my[:, None] > ny) | (3 * mx[None, :] > nx)
        assert c[outside].max() < 1e-15


@pytest.mark.parametrize("arnoldi", ["fused", "chained", "serial"])
@pytest.mark.parametrize("nx,ny,restart", [(16, 16, 20), (64, 32, 20), (128, 64, 20), (256, 128, 20),
                                           (64, 64, 3), (1024, 512, 20), (2048, 32, 20), (32, 2048, 20),
                                           (4096, 16, 20), (16, 4096, 20)])
def test_elliptic_solve(nx, ny, restart, arnoldi):
    say(f"elliptic solve {nx}x{ny} m={restart} {arnoldi}")
    ctx, g = mk(nx, ny, 1.5, 1.5, arnoldi=arnoldi, gmres_tol=1e-12, gmres_restart=restart, gmres_max_iters=400)
    rng = np.random.default_rng(nx + ny + restart)
    h, vx, vy, s0 = random_state(rng, Box(nx, ny, 1.5, 1.5), amp_h=0.35, kmax=min(6, nx // 2 - 1, ny // 2 - 1))
    b = -(O.d_x(g, vx) + O.d_y(g, vy))
    ref, rinfo = O.gmres(g, h, b, s0, 1e-12, restart, 400)
    sig = dev(s0)
    info = sgn.sgn_elliptic_solve(ctx, dev(h), dev(b), sig)
    assert info.converged and rinfo.converged
    assert abs(info.iters - rinfo.iters) <= 1, (info.iters, rinfo.iters)
    assert info.restarts == rinfo.restarts or abs(info.iters - rinfo.iters) == 1
    assert rel(host(sig), ref) < 1e-10
    assert info.rel_resid_true < 1e-10


def test_elliptic_solve_zero_rhs_and_unit_depth():
    say("elliptic solve special cases")
    ctx, g = mk(64, 32, 1.0, 1.0, gmres_tol=1e-12)
    rng = np.random.default_rng(1)
    b = rng.standard_normal((32, 64))
    sig = dev(np.ones((32, 64)))
    info = sgn.sgn_elliptic_solve(ctx, dev(np.ones((32, 64))), dev(np.zeros((32, 64))), sig)
    assert info.converged and info.iters == 0 and np.all(host(sig) == 0.0)
    sig = dev(np.zeros((32, 64)))
    info = sgn.sgn_elliptic_solve(ctx, dev(np.ones((32, 64))), dev(b), sig)
    assert info.converged and info.iters == 1
    assert rel(host(sig), O.apply_Minv(g, b)) < 1e-12


def test_elliptic_solve_not_converged():
    say("elliptic solve max_iters")
    ctx, g = mk(32, 32, 1.0, 1.0, gmres_tol=1e-14, gmres_max_iters=2)
    rng = np.random.default_rng(2)
    h, vx, vy, _ = random_state(rng, Box(32, 32, 1.0, 1.0), amp_h=0.4, kmax=5)
    b = -(O.d_x(g, vx) + O.d_y(g, vy))
    sig = dev(np.zeros((32, 32)))
    info = sgn.sgn_elliptic_solve(ctx, dev(h), dev(b), sig)
    ref, rinfo = O.gmres(g, h, b, np.zeros((32, 32)), 1e-14, 20, 2)
    assert not info.converged and info.iters == 2 and not rinfo.converged
    assert rel(host(sig), ref) < 1e-11


@pytest.mark.parametrize("case", ["random", "soliton"])
def test_rhs(case):
    say(f"rhs {case}")
    if case == "random":
        nx, ny, L = 128, 64, (2.0, 1.0)
        ctx, g = mk(nx, ny, *L, gmres_tol=1e-12)
        rng = np.random.default_rng(3)
        h, vx, vy, s0 = random_state(rng, Box(nx, ny, *L), amp_h=0.3, amp_v=0.2, kmax=6)
    else:
        nx, ny, L = 256, 16, (10.0, 2.0)
        ctx, g = mk(nx, ny, *L, gmres_tol=1e-12)
        h, vx, vy, s0 = line_soliton(Box(nx, ny, *L), a=0.5)
        s0 = np.zeros_like(h)
    r = O.rhs(g, h, vx, vy, s0, tol=1e-12)
    dh, dvx, dvy, sig = (torch.empty((ny, nx), dtype=torch.float64, device=DEV) for _ in range(4))
    sig.copy_(dev(s0))
    info = sgn.sgn_rhs(ctx, dev(h), dev(vx), dev(vy), sig, dh, dvx, dvy)
    assert info.converged and abs(info.iters - r.info.iters) <= 1
    assert rel(host(sig), r.sigma) < 1e-10
    assert rel(host(dh), r.dh) < 1e-10
    assert rel(host(dvx), r.dvx) < 1e-10
    assert rel(host(dvy), r.dvy) < 1e-10 or np.abs(r.dvy).max() < 1e-13


def run_gpu_rk4(ctx, h, vx, vy, s, dt, n):
    th, tvx, tvy, ts = dev(h), dev(vx), dev(vy), dev(s)
    info = sgn.sgn_rk4_step(ctx, th, tvx, tvy, ts, dt, n)
    return host(th), host(tvx), host(tvy), host(ts), info


@pytest.mark.parametrize("arnoldi", ["fused", "serial"])
@pytest.mark.parametrize("nx,ny", [(128, 64), (256, 128)])
def test_rk4_stage_increment_guess(nx, ny, arnoldi):
    """guess = SGN_GUESS_STAGE_INCREMENT against the oracle with the same
    option (transversally perturbed soliton, 40 steps, two calls so that the
    increments restart at zero in the second), and against the plain warm
    start: same states to the GMRES tolerance, fewer iterations."""
    say(f"rk4 stage-increment guess {nx}x{ny} {arnoldi}")
    box = Box(nx, ny, 10.0, 5.0)
    h, vx, vy, s = perturbed_line_soliton(box, a=0.5, eps=0.01, k=2, x0=-10.0)
    dt, n = 0.01, 20
    ctx, g = mk(nx, ny, box.Lx, box.Ly, arnoldi=arnoldi, gmres_tol=1e-12, krasny=1e-12,
                guess=sgn.SGN_GUESS_STAGE_INCREMENT)
    th, tvx, tvy, ts = dev(h), dev(vx), dev(vy), dev(s)
    i1 = sgn.sgn_rk4_step(ctx, th, tvx, tvy, ts, dt, n)
    i2 = sgn.sgn_rk4_step(ctx, th, tvx, tvy, ts, dt, n)
    gh, gvx, gvy, gs = host(th), host(tvx), host(tvy), host(ts)
    oh, ovx, ovy, os_, o1 = O.rk4(g, h, vx, vy, s, dt, n)
    oh, ovx, ovy, os_, o2 = O.rk4(g, oh, ovx, ovy, os_, dt, n)
    gi, oi = i1.total_iters + i2.total_iters, o1.total_iters + o2.total_iters
    ctx0, _ = mk(nx, ny, box.Lx, box.Ly, arnoldi=arnoldi, gmres_tol=1e-12, krasny=1e-12)
    ph, pvx, pvy, ps, p = run_gpu_rk4(ctx0, h, vx, vy, s, dt, 2 * n)
    say(f"  iters gpu {gi} oracle {oi} plain warm start {p.total_iters}")
    assert not (i1.any_unconverged or i2.any_unconverged)
    assert abs(gi - oi) <= 8
    assert rel(gh, oh, 1.0) < 1e-10 and rel(gvx, ovx) < 1e-10 and rel(gvy, ovy) < 1e-10
    assert rel(gs, os_) < 1e-9
    assert rel(gh, ph, 1.0) < 1e-9 and rel(gvx, pvx) < 1e-9 and rel(gvy, pvy) < 1e-9
    assert gi < 0.9 * p.total_iters


@pytest.mark.parametrize("arnoldi", ["fused", "chained", "serial"])
def test_rk4_line_soliton_128x64_200_steps(arnoldi):
    """The 128x64 line soliton workload: a = 0.5 on [-10pi,10pi]x[-5pi,5pi],
    dt = 0.01, 200 steps, GMRES tol 1e-10, restart 20."""
    say(f"rk4 line soliton 128x64 x200 {arnoldi}")
    box, (h, vx, vy, s), w = workload("line_soliton_128x64")
    ctx, g = mk(box.nx, box.ny, box.Lx, box.Ly, arnoldi=arnoldi, gmres_tol=w["tol"], gmres_restart=w["restart"])
    gh, gvx, gvy, gs, info = run_gpu_rk4(ctx, h, vx, vy, s, w["dt"], w["steps"])
    oh, ovx, ovy, os_, oinfo = O.rk4(g, h, vx, vy, s, w["dt"], w["steps"])
    say(f"  gpu iters {info.total_iters} oracle {oinfo.total_iters}")
    assert not info.any_unconverged and info.solves == 800
    assert abs(info.total_iters - oinfo.total_iters) <= 8
    assert rel(gh, oh, 1.0) < 1e-10
    assert rel(gvx, ovx) < 1e-10
    assert np.abs(gvy).max() < 1e-12
    assert rel(gs, os_) < 1e-9
    # and the GPU result itself: translation, mass and energy
    inv0 = sgn.sgn_invariants(ctx, dev(h), dev(vx), dev(vy), dev(s))
    inv1 = sgn.sgn_invariants(ctx, dev(gh), dev(gvx), dev(gvy), dev(gs))
    assert abs(inv1["mass"] - inv0["mass"]) < 1e-12 * abs(inv0["mass"])
    assert abs(inv1["energy"] - inv0["energy"]) < 1e-9 * abs(inv0["energy"])
    p = math.sqrt(1.5)
    h_exact, *_ = line_soliton(box, a=0.5, x0=p * 2.0)
    assert np.abs(gh - h_exact).max() < 1e-6


def test_rk4_krasny_and_random_state():
    say("rk4 random state with Krasny")
    nx, ny = 64, 64
    ctx, g = mk(nx, ny, 1.0, 1.0, gmres_tol=1e-12, krasny=1e-12)
    rng = np.random.default_rng(9)
    h, vx, vy, s = random_state(rng, Box(nx, ny, 1.0, 1.0), amp_h=0.2, amp_v=0.1, kmax=5)
    gh, gvx, gvy, gs, info = run_gpu_rk4(ctx, h, vx, vy, s, 0.005, 5)
    oh, ovx, ovy, os_, oinfo = O.rk4(g, h, vx, vy, s, 0.005, 5)
    assert rel(gh, oh, 1.0) < 1e-10 and rel(gvx, ovx) < 1e-10 and rel(gvy, ovy) < 1e-10


@pytest.mark.parametrize("nx,ny", [(2048, 16), (16, 2048), (4096, 16), (16, 4096)])
def test_rk4_long_transforms(nx, ny):
    """2048-point rows and columns (eight values per thread in the transforms),
    and the largest supported length, 4096 (the four-kernel schedule: the
    chained blocks do not fit)."""
    say(f"rk4 {nx}x{ny}")
    ctx, g = mk(nx, ny, 1.0, 1.0, gmres_tol=1e-12, krasny=1e-12)
    rng = np.random.default_rng(nx + 7 * ny)
    h, vx, vy, s = random_state(rng, Box(nx, ny, 1.0, 1.0), amp_h=0.2, amp_v=0.1, kmax=5)
    gh, gvx, gvy, gs, info = run_gpu_rk4(ctx, h, vx, vy, s, 0.005, 3)
    oh, ovx, ovy, os_, oinfo = O.rk4(g, h, vx, vy, s, 0.005, 3)
    assert rel(gh, oh, 1.0) < 1e-10 and rel(gvx, ovx) < 1e-10 and rel(gvy, ovy) < 1e-10


@pytest.mark.parametrize("nx,ny", [(128, 64), (64, 128), (256, 256), (2048, 16), (16, 2048)])
def test_invariants(nx, ny):
    say(f"invariants {nx}x{ny}")
    ctx, g = mk(nx, ny, 2.0, 1.5)
    rng = np.random.default_rng(nx * ny)
    h, vx, vy, s = random_state(rng, Box(nx, ny, 2.0, 1.5), amp_h=0.3, amp_v=0.2, kmax=6)
    ref, rs = O.invariants(g, h, vx, vy, s)
    got = sgn.sgn_invariants(ctx, dev(h), dev(vx), dev(vy), dev(s))
    for k in ("mass", "px", "py", "energy", "curl_l2"):
        assert abs(got[k] - ref[k]) <= 1e-11 * max(abs(ref[k]), 1e-3), (k, got[k], ref[k])
    assert got["min_h"] == ref["min_h"] and got["max_h"] == ref["max_h"]
    assert abs(got["spectral_tail"] - ref["spectral_tail"]) <= 1e-12 * max(ref["spectral_tail"], 1e-3)


def test_full_size_1024x512_rhs_and_step():
    """The 1024x512 perturbed-soliton workload at full size, in the launch
    configuration the benchmark times: one RHS and one RK4 step vs the oracle."""
    say("full size 1024x512")
    box, (h, vx, vy, s), w = workload("perturbed_soliton_1024x512")
    ctx, g = mk(box.nx, box.ny, box.Lx, box.Ly, gmres_tol=w["tol"], gmres_restart=w["restart"])
    r = O.rhs(g, h, vx, vy, s)
    dh, dvx, dvy, sig = (torch.empty((box.ny, box.nx), dtype=torch.float64, device=DEV) for _ in range(4))
    sig.copy_(dev(s))
    info = sgn.sgn_rhs(ctx, dev(h), dev(vx), dev(vy), sig, dh, dvx, dvy)
    say(f"  rhs iters gpu {info.iters} oracle {r.info.iters}")
    assert rel(host(dh), r.dh) < 1e-9 and rel(host(dvx), r.dvx) < 1e-9 and rel(host(dvy), r.dvy) < 1e-9
    gh, gvx, gvy, gs, sinfo = run_gpu_rk4(ctx, h, vx, vy, s, w["dt"], 1)
    oh, ovx, ovy, os_, oinfo = O.rk4(g, h, vx, vy, s, w["dt"], 1)
    say(f"  step iters gpu {sinfo.total_iters} oracle {oinfo.total_iters}")
    assert rel(gh, oh, 1.0) < 1e-10 and rel(gvx, ovx) < 1e-10 and rel(gvy, ovy) < 1e-10


def test_determinism_bitwise():
    say("determinism")
    box, (h, vx, vy, s), w = workload("line_soliton_128x64")
    ctx, g = mk(box.nx, box.ny, box.Lx, box.Ly)
    a = run_gpu_rk4(ctx, h, vx, vy, s, 0.01, 5)
    b = run_gpu_rk4(ctx, h, vx, vy, s, 0.01, 5)
    for x, y in zip(a[:4], b[:4]):
        assert np.array_equal(x, y)


def test_error_paths():
    say("error paths")
    ctx, g = mk(32, 32, 1.0, 1.0)
    rng = np.random.default_rng(4)
    h, vx, vy, s = random_state(rng, Box(32, 32, 1.0, 1.0))
    bad = h.copy()
    bad[3, 5] = -0.1
    with pytest.raises(sgn.SgnError) as e:
        sgn.sgn_rk4_step(ctx, dev(bad), dev(vx), dev(vy), dev(s), 0.01, 1)
    assert e.value.status == sgn.SGN_ERR_CAVITATION
    nan = vx.copy()
    nan[0, 0] = np.nan
    with pytest.raises(sgn.SgnError) as e:
        sgn.sgn_rk4_step(ctx, dev(h), dev(nan), dev(vy), dev(s), 0.01, 1)
    assert e.value.status == sgn.SGN_ERR_NONFINITE
    with pytest.raises(ValueError):
        sgn.sgn_rk4_step(ctx, dev(h[:, :16]), dev(vx), dev(vy), dev(s), 0.01, 1)


@pytest.mark.parametrize("arnoldi", ["fused", "serial"])
@pytest.mark.parametrize("amp", [1e-9, 1e-6, 1e-3])
def test_elliptic_solve_nearly_constant_depth(amp, arnoldi):
    """h = 1 + amp * (smooth field): M^-1 L = I + O(amp), so the first Arnoldi
    step leaves a new direction of relative size ~amp.  The solve must still
    reach the tolerance in the true residual (not only in its estimate)."""
    say(f"elliptic solve, depth 1 + {amp:g} perturbation, {arnoldi}")
    nx, ny = 64, 32
    ctx, g = mk(nx, ny, 1.0, 1.0, arnoldi=arnoldi, gmres_tol=1e-12)
    rng = np.random.default_rng(17)
    h = 1.0 + amp * random_smooth_field(rng, ny, nx, kmax=4)
    b = random_smooth_field(rng, ny, nx, kmax=6)
    ref, rinfo = O.gmres(g, h, b, np.zeros_like(b), 1e-13, 20, 400)
    sig = dev(np.zeros_like(b))
    info = sgn.sgn_elliptic_solve(ctx, dev(h), dev(b), sig)
    pr = O.apply_Minv(g, b - O.apply_L(g, h, host(sig)))
    rel_pre = np.sqrt(np.sum(pr ** 2)) / np.sqrt(np.sum(O.apply_Minv(g, b) ** 2))
    say(f"  iters {info.iters} (oracle {rinfo.iters}), restarts {info.restarts}, "
        f"true preconditioned residual {rel_pre:.1e}, sigma error {rel(host(sig), ref):.1e}")
    assert info.converged and rel_pre < 1e-11
    assert rel(host(sig), ref) < 1e-10
