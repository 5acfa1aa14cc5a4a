"""The context-free operator entry point (sgn_apply_operator_noalloc, fixed
device scratch, nothing allocated) against the context entry point
sgn_apply_operator on the same inputs, two calls in a row with the second on
a smaller grid, in both precisions.  The two calls differ only in the
rounding of their twiddle tables (computed on the device here, on the host
there), which the operator amplifies by up to k_max^2: M^-1 L is gated
field-relative (FP64 1e-12, FP32 1e-5), L normwise, error <= c k_max^2 |s|
|1/h| with c = 1e-13 in FP64 (a few hundred ulps of transform rounding) and
1e-6 in FP32."""
import numpy as np
import pytest
import torch

from paper_2306_09731_amd import sgn
from sgn_inputs import random_smooth_field

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)


def compare(nx, ny, prec, seed):
    Lx, Ly = 2.0, 1.5
    cfg = sgn.config_default(nx, ny, Lx, Ly, precision=prec)
    ctx = sgn.sgn_init(cfg, DEV)
    dt = sgn.field_dtype(cfg)
    rng = np.random.default_rng(seed)
    h = 1.0 + 0.3 * random_smooth_field(rng, ny, nx, kmax=5)
    s = random_smooth_field(rng, ny, nx, kmax=5)
    th = torch.from_numpy(h).to(DEV).to(dt)
    ts = torch.from_numpy(s).to(DEV).to(dt)
    kmax = max(nx / 2 / Lx, ny / 2 / Ly)
    for pre in (False, True):
        ref = torch.empty(ny, nx, dtype=dt, device=DEV)
        got = torch.full((ny, nx), float("nan"), dtype=dt, device=DEV)
        sgn.sgn_apply_operator(ctx, th, ts, ref, pre)
        sgn.sgn_apply_operator_noalloc(cfg, th, ts, got, pre)
        torch.cuda.synchronize()
        a = got.cpu().double().numpy()
        b = ref.cpu().double().numpy()
        err = np.abs(a - b).max()
        if pre:
            e, gate = err / np.abs(b).max(), (1e-12 if prec == sgn.SGN_FP64 else 1e-5)
        else:
            e = err / (kmax ** 2 * np.abs(s).max() * np.abs(1.0 / h).max())
            gate = 1e-13 if prec == sgn.SGN_FP64 else 1e-6
        say(f"noalloc {nx}x{ny} {'fp32' if prec else 'fp64'} {'M^-1 L' if pre else 'L'}: error {e:.2e} "
            f"(gate {gate:g}, bitwise equal: {bool(np.array_equal(a, b))})")
        assert np.isfinite(a).all() and e < gate
    ctx.close()


@pytest.mark.parametrize("prec", [sgn.SGN_FP64, sgn.SGN_FP32_MIXED])
def test_operator_noalloc_matches_context_call(prec):
    # the largest grid the scratch holds, then a smaller one on the same scratch
    compare(1024, 1024, prec, 1)
    compare(256, 128, prec, 2)
