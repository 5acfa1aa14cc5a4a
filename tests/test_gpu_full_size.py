"""Parity with the FP64 oracle at the grid sizes the product runs, in the
launch configurations the benchmark uses.

* 2048 x 2048 FP64 (the precision-form workload's grid): default schedule for
  2048-point columns (four Arnoldi kernels, one transform chain), whose column
  passes launch 1024 blocks (four per CU), so the GMRES-status reads and the
  last-block reductions run over several waves of blocks.
* 2048 x 1024 FP64 under the default three-kernel schedule: its column passes
  launch 512 two-chain blocks, more than one wave, so the Gram-identity finish
  in kernel A and the speculative status reads are checked on a multi-wave
  grid.
* 2048 x 2048 in the mixed-precision mode: single calls against the oracle on
  FP32-rounded inputs, with the gates of the mode (1e-5 relative for sigma,
  M^-1 L, M^-1 and the RK4 state; derivative-type outputs normwise, error <=
  1e-6 k_max (input scale), because a spectral derivative multiplies the
  ~1e-7 rounding of an FP32 transform by up to k_max).
Gates of the FP64 cases are those of the 1024 x 512 full-size test: 1e-9 for
the RHS outputs (GMRES at tol 1e-10 on both sides) and 1e-10 for the state
after one RK4 step."""
import numpy as np
import pytest
import torch

from oracle import sgn_oracle as O
from paper_2306_09731_amd import sgn
from sgn_inputs import Box, random_state

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)


def rel(a, ref, bg=0.0):
    scale = np.abs(ref - bg).max()
    return np.abs(a - ref).max() / (scale if scale > 0 else 1.0)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def fp64_case(nx, ny, L, seed, expect_schedule):
    box = Box(nx, ny, L, L)
    cfg = sgn.config_default(nx, ny, L, L, gmres_tol=1e-10)
    ctx = sgn.sgn_init(cfg, DEV)
    shape = sgn.sgn_launch_shape(ctx)
    say(f"  launch shape {shape}")
    assert shape["arnoldi"] == expect_schedule
    g = O.Grid(O.Config(nx=nx, ny=ny, Lx=L, Ly=L, gmres_tol=1e-10))
    h, vx, vy, s = random_state(np.random.default_rng(seed), box, amp_h=0.3, amp_v=0.2, kmax=4)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    r = O.rhs(g, h, vx, vy, s)
    outs = [torch.empty((ny, nx), dtype=torch.float64, device=DEV) for _ in range(3)]
    sig = d(s)
    info = sgn.sgn_rhs(ctx, d(h), d(vx), d(vy), sig, *outs)
    errs = [rel(host(o), ref) for o, ref in zip(outs, (r.dh, r.dvx, r.dvy))]
    say(f"  rhs: iters gpu {info.iters} oracle {r.info.iters}; dh {errs[0]:.1e} dvx {errs[1]:.1e} "
        f"dvy {errs[2]:.1e} sigma {rel(host(sig), r.sigma):.1e}")
    assert max(errs) < 1e-9 and rel(host(sig), r.sigma) < 1e-9
    f = [d(a) for a in (h, vx, vy, s)]
    sinfo = sgn.sgn_rk4_step(ctx, *f, 0.005, 1)
    oh, ovx, ovy, os_, oinfo = O.rk4(g, h, vx, vy, s, 0.005, 1)
    eh, evx, evy = rel(host(f[0]), oh, 1.0), rel(host(f[1]), ovx), rel(host(f[2]), ovy)
    say(f"  one step: iters gpu {sinfo.total_iters} oracle {oinfo.total_iters}; h {eh:.1e} vx {evx:.1e} "
        f"vy {evy:.1e}")
    assert eh < 1e-10 and evx < 1e-10 and evy < 1e-10
    ctx.close()


def test_full_size_2048x2048_fp64_serial_schedule():
    say("full size 2048x2048 FP64, default schedule (four kernels, one chain)")
    fp64_case(2048, 2048, 20.0, 5, expect_schedule=0)


def test_full_size_2048x1024_fp64_three_kernel_schedule():
    say("full size 2048x1024 FP64, default three-kernel schedule")
    fp64_case(2048, 1024, 10.0, 6, expect_schedule=2)


def test_full_size_2048x2048_fp32_single_calls():
    """Every single call of the mixed-precision mode at 2048^2 against the FP64
    oracle on FP32-rounded inputs."""
    say("full size 2048x2048 FP32-mixed single calls")
    nx = ny = 2048
    L = 20.0
    box = Box(nx, ny, L, L)
    cfg = sgn.config_default(nx, ny, L, L, precision=sgn.SGN_FP32_MIXED)
    ctx = sgn.sgn_init(cfg, DEV)
    g = O.Grid(O.Config(nx=nx, ny=ny, Lx=L, Ly=L, gmres_tol=1e-12))
    r32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)
    h, vx, vy, s = (r32(a) for a in random_state(np.random.default_rng(9), box, amp_h=0.3, amp_v=0.2, kmax=4))
    kmax = nx / 2 / L
    out = torch.empty(ny, nx, dtype=torch.float32, device=DEV)
    # derivatives
    for axis, ref in ((0, O.d_x(g, s)), (1, O.d_y(g, s))):
        sgn.sgn_derivative(ctx, axis, d(s), out)
        e = np.abs(host(out) - ref).max() / (kmax * np.abs(s).max())
        say(f"  d/d{'xy'[axis]}: error / (k_max |f|) {e:.2e}")
        assert e < 1e-6
    # operator, preconditioned operator, preconditioner
    sgn.sgn_apply_operator(ctx, d(h), d(s), out, 0)
    e1 = np.abs(host(out) - O.apply_L(g, h, s)).max() / (kmax ** 2 * np.abs(s).max() * np.abs(1 / h).max())
    sgn.sgn_apply_operator(ctx, d(h), d(s), out, 1)
    e2 = rel(host(out), O.apply_Minv(g, O.apply_L(g, h, s)))
    sgn.sgn_apply_precond(ctx, d(s), out)
    e3 = rel(host(out), O.apply_Minv(g, s))
    say(f"  L {e1:.2e} (normwise), M^-1 L {e2:.2e}, M^-1 {e3:.2e}")
    assert e1 < 1e-6 and e2 < 1e-5 and e3 < 1e-5
    # elliptic solve from zero
    b = r32(-(O.d_x(g, vx) + O.d_y(g, vy)))
    ref, oinfo = O.gmres(g, h, b, np.zeros_like(b), 1e-12, 20, 200)
    sig = torch.zeros(ny, nx, dtype=torch.float32, device=DEV)
    info = sgn.sgn_elliptic_solve(ctx, d(h), d(b), sig)
    es = rel(host(sig), ref)
    say(f"  solve: iters {info.iters} (oracle at 1e-12: {oinfo.iters}), sigma {es:.2e}")
    assert info.converged and es < 1e-5
    # right-hand side
    outs = [torch.empty(ny, nx, dtype=torch.float32, device=DEV) for _ in range(3)]
    ts = d(s)
    sgn.sgn_rhs(ctx, d(h), d(vx), d(vy), ts, *outs)
    r = O.rhs(g, h, vx, vy, s, tol=1e-12)
    sx, sy = O.d_x(g, r.sigma), O.d_y(g, r.sigma)
    qmax = max(np.abs(h * vx - sx).max(), np.abs(h * vy - sy).max())
    bmax = np.abs(0.5 * (vx ** 2 + vy ** 2) - (sx ** 2 + sy ** 2) / (2 * h * h) + h
                  - 4.5 * r.sigma ** 2 / h ** 4).max()
    scales = (kmax * qmax, kmax * bmax, kmax * bmax)
    errs = [np.abs(host(o) - x).max() / sc for o, x, sc in zip(outs, (r.dh, r.dvx, r.dvy), scales)]
    es = rel(host(ts), r.sigma)
    say(f"  rhs: error / (k_max x input scale) dh {errs[0]:.2e} dvx {errs[1]:.2e} dvy {errs[2]:.2e}; "
        f"sigma {es:.2e}")
    assert max(errs) < 1e-6 and es < 1e-5
    # one RK4 step of the moving random state (the workload's Gaussian starts
    # at rest, where one step leaves v of size dt and its relative error
    # measures nothing of the mode)
    f = [d(a) for a in (h, vx, vy, s)]
    sinfo = sgn.sgn_rk4_step(ctx, *f, 0.005, 1)
    oh, ovx, ovy, _, _ = O.rk4(g, h, vx, vy, s, 0.005, 1)
    eh, evx, evy = rel(host(f[0]), oh, 1.0), rel(host(f[1]), ovx), rel(host(f[2]), ovy)
    say(f"  one step: h {eh:.2e} vx {evx:.2e} vy {evy:.2e}; iters {sinfo.total_iters}")
    assert eh < 1e-5 and evx < 1e-5 and evy < 1e-5
    ctx.close()
