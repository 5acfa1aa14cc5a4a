"""The learned initial guess inside the RK4 step, and its recorder.

The recorder's samples are checked against the oracle on the state where they
are taken (the first solve of a step starts from the given sigma): the
network input (r0 / |r0|, M^-1 r0 / |r0|, h - h_inf with r0 = b - L sigma_prev,
b = -div v) and the target (sigma - sigma_prev) / |r0| with sigma the oracle's
GMRES solution.  A network built to output exactly its second input channel
turns the guess into sigma_prev + M^-1 r0, one preconditioned Richardson
step: GMRES must converge to the same sigma in no more iterations than from
the warm start (a sign or scale error in applying the guess would cost
iterations).  A zero network changes nothing but rounding."""
import numpy as np
import pytest
import torch

from oracle import sgn_oracle as O
from paper_2306_09731_amd import sgn
from sgn_inputs import Box, perturbed_line_soliton

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
CH = sgn.SGN_CNN_CH


def say(msg):
    print(msg, flush=True)


def setup(nx=128, ny=64, **kw):
    box = Box(nx, ny, 10.0 * nx / 128, 5.0 * ny / 64)
    h, vx, vy, s = perturbed_line_soliton(box, a=0.5, eps=0.05, k=1, x0=-0.5 * np.pi * box.Lx)
    cfg = sgn.config_default(nx, ny, box.Lx, box.Ly, gmres_tol=1e-12, **kw)
    ctx = sgn.sgn_init(cfg, DEV)
    f = [torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in (h, vx, vy, s)]
    g = O.Grid(O.Config(nx=nx, ny=ny, Lx=box.Lx, Ly=box.Ly, gmres_tol=1e-13))
    return ctx, f, (h, vx, vy, s), g


def passthrough_params():
    """Output = input channel 1: layer 0 splits it into ReLU(+x) and ReLU(-x),
    the middle layers pass both on, the last layer takes their difference."""
    per = 9 * CH * CH + CH
    p = np.zeros(sgn.SGN_CNN_LAYERS * per, dtype=np.float32)
    centre = 4
    for l in range(sgn.SGN_CNN_LAYERS):
        w = p[l * per:l * per + 9 * CH * CH].reshape(9, CH, CH)
        if l == 0:
            w[centre, 0, 1], w[centre, 1, 1] = 1.0, -1.0
        elif l < sgn.SGN_CNN_LAYERS - 1:
            w[centre, 0, 0], w[centre, 1, 1] = 1.0, 1.0
        else:
            w[centre, 0, 0], w[centre, 0, 1] = 1.0, -1.0
    return p


def test_recorder_samples_match_oracle():
    ctx, f, (h, vx, vy, s), g = setup()
    rec = torch.zeros(8, 4, 64, 128, dtype=torch.float32, device=DEV)
    sgn.learned_guess_attach(ctx, None, rec)
    sgn.sgn_rk4_step(ctx, *f, 0.01, 1)
    torch.cuda.synchronize()
    assert sgn.learned_guess_recorded(ctx) == 4
    in3, target = (a.cpu().numpy().astype(np.float64) for a in sgn.record_sample(rec, 0))
    b = -(O.d_x(g, vx) + O.d_y(g, vy))
    r0 = b - O.apply_L(g, h, s)
    mr0 = O.apply_Minv(g, r0)
    scale = np.sqrt(np.mean(r0 ** 2))
    ref_in = np.stack([r0 / scale, mr0 / scale, h - 1.0], axis=-1)
    sig, _ = O.gmres(g, h, b, s, 1e-13, 20, 400)
    ref_t = (sig - s) / scale
    e_in = [np.abs(in3[..., c] - ref_in[..., c]).max() / np.abs(ref_in[..., c]).max() for c in range(3)]
    e_t = np.abs(target - ref_t).max() / np.abs(ref_t).max()
    say(f"recorder sample 0: input errors {[f'{e:.1e}' for e in e_in]}, target error {e_t:.1e}")
    assert max(e_in) < 1e-6 and e_t < 1e-6
    # later slots are filled, the unused ones untouched
    assert float(rec[3].abs().sum()) > 0 and float(rec[4:].abs().sum()) == 0


def test_passthrough_network_guess_saves_iterations():
    ctx0, f0, _, _ = setup()
    ctx1, f1, _, _ = setup()
    net = sgn.cnn_init(64, 128, DEV)
    sgn.cnn_set_params(net, passthrough_params())
    sgn.learned_guess_attach(ctx1, net)
    i0 = sgn.sgn_rk4_step(ctx0, *f0, 0.01, 5)
    i1 = sgn.sgn_rk4_step(ctx1, *f1, 0.01, 5)
    torch.cuda.synchronize()
    e = max(float((a - b).abs().max()) for a, b in zip(f0[:3], f1[:3]))
    say(f"passthrough guess: iterations {i1.total_iters} vs warm start {i0.total_iters}, state difference {e:.1e}")
    assert i1.total_iters <= i0.total_iters and e < 1e-9


def test_zero_network_changes_nothing_but_rounding():
    ctx0, f0, _, _ = setup()
    ctx1, f1, _, _ = setup()
    net = sgn.cnn_init(64, 128, DEV)
    sgn.cnn_set_params(net, np.zeros(sgn.SGN_CNN_PARAMS, dtype=np.float32))
    sgn.learned_guess_attach(ctx1, net)
    i0 = sgn.sgn_rk4_step(ctx0, *f0, 0.01, 3)
    i1 = sgn.sgn_rk4_step(ctx1, *f1, 0.01, 3)
    torch.cuda.synchronize()
    e = max(float((a - b).abs().max()) for a, b in zip(f0[:3], f1[:3]))
    say(f"zero network: iterations {i1.total_iters} vs {i0.total_iters}, state difference {e:.1e}")
    assert abs(i1.total_iters - i0.total_iters) <= 2 and e < 1e-10


def test_stage_mask_selects_the_corrected_solves():
    """Mask 0: the attached network is never applied, so the steps are bit for
    bit the warm start's.  Mask 0x1 (once per RK4 step): the passthrough guess
    corrects stage 0 only; the state agrees with the warm start's to the
    solver tolerance and costs no more iterations."""
    ctx0, f0, _, _ = setup()
    i0 = sgn.sgn_rk4_step(ctx0, *f0, 0.01, 4)
    net = sgn.cnn_init(64, 128, DEV)
    sgn.cnn_set_params(net, passthrough_params())
    res = {}
    for mask in (0x0, 0x1):
        ctx, f, _, _ = setup()
        sgn.learned_guess_attach(ctx, net)
        sgn.learned_guess_stages(ctx, mask)
        res[mask] = (sgn.sgn_rk4_step(ctx, *f, 0.01, 4), f)
    torch.cuda.synchronize()
    i_none, f_none = res[0x0]
    i_once, f_once = res[0x1]
    e = max(float((a - b).abs().max()) for a, b in zip(f0[:3], f_once[:3]))
    say(f"stage mask: none {i_none.total_iters}, once per step {i_once.total_iters}, warm start {i0.total_iters}; "
        f"once-per-step state difference {e:.1e}")
    assert all(torch.equal(a, b) for a, b in zip(f0, f_none)) and i_none.total_iters == i0.total_iters
    assert i_once.total_iters <= i0.total_iters and e < 1e-9
    with pytest.raises(sgn.SgnError):
        sgn.learned_guess_stages(ctx0, 16)


def test_attach_errors():
    ctx, f, _, _ = setup()
    with pytest.raises(sgn.SgnError):
        sgn.learned_guess_attach(ctx, sgn.cnn_init(64, 64, DEV))  # grid mismatch
    ctx2, f2, _, _ = setup(guess=sgn.SGN_GUESS_STAGE_INCREMENT)
    with pytest.raises(sgn.SgnError):
        sgn.learned_guess_attach(ctx2, sgn.cnn_init(64, 128, DEV))
    sgn.learned_guess_attach(ctx, sgn.cnn_init(64, 128, DEV))
    with pytest.raises(sgn.SgnError):
        sgn.sgn_rk4_step_graph(ctx, *f, 0.01, 2)
    sgn.learned_guess_attach(ctx, None)
    _, rep = sgn.sgn_rk4_step_graph(ctx, *f, 0.01, 4)  # two calibration steps, then replays
    assert rep


def test_stored_weights_guess_a_small_soliton():
    """The committed weights (trained at dx = dy = 2 pi / 102.4) on a 256 x 128
    perturbed soliton of the same spacing: same states as the warm start to
    the GMRES tolerance, and no more iterations."""
    from paper_2306_09731_amd import learned
    params = np.load(learned.PARAMS_FILE)
    assert params.shape == (sgn.SGN_CNN_PARAMS,) and np.all(np.isfinite(params))
    box = Box(256, 128, 2.5, 1.25)
    h, vx, vy, s = perturbed_line_soliton(box, a=0.5, eps=0.02, k=1, x0=-2.5)
    res = {}
    for mode in ("warm", "learned"):
        cfg = sgn.config_default(256, 128, 2.5, 1.25, gmres_tol=1e-10, krasny=1e-12)
        ctx = sgn.sgn_init(cfg, DEV)
        f = [torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in (h, vx, vy, s)]
        sgn.sgn_rk4_step(ctx, *f, 0.005, 5)
        if mode == "learned":
            net = sgn.cnn_init(128, 256, DEV)
            sgn.cnn_set_params(net, params)
            sgn.learned_guess_attach(ctx, net)
        info = sgn.sgn_rk4_step(ctx, *f, 0.005, 10)
        torch.cuda.synchronize()
        res[mode] = ([a.cpu().numpy() for a in f], info)
    (fw, iw), (fl, il) = res["warm"], res["learned"]
    e = max(np.abs(a - b).max() for a, b in zip(fw[:3], fl[:3]))
    say(f"stored weights, 256x128: iterations {il.total_iters} vs warm start {iw.total_iters}, state difference {e:.1e}")
    assert il.total_iters <= iw.total_iters and e < 1e-8


def test_recorder_in_fp32_mode():
    """The recorder's kernels in the mixed-precision mode: the sample of the
    first solve against the oracle on the FP32-rounded state, within the FP32
    mode's gates (1e-5; the GMRES tolerance there is 1e-6)."""
    nx, ny = 128, 64
    box = Box(nx, ny, 10.0, 5.0)
    h, vx, vy, s = (np.asarray(a, np.float32).astype(np.float64)
                    for a in perturbed_line_soliton(box, a=0.5, eps=0.05, k=1, x0=-5.0 * np.pi))
    cfg = sgn.config_default(nx, ny, box.Lx, box.Ly, gmres_tol=1e-6, precision=sgn.SGN_FP32_MIXED)
    ctx = sgn.sgn_init(cfg, DEV)
    f = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV) for a in (h, vx, vy, s)]
    rec = torch.zeros(4, 4, ny, nx, dtype=torch.float32, device=DEV)
    sgn.learned_guess_attach(ctx, None, rec)
    sgn.sgn_rk4_step(ctx, *f, 0.01, 1)
    torch.cuda.synchronize()
    g = O.Grid(O.Config(nx=nx, ny=ny, Lx=box.Lx, Ly=box.Ly, gmres_tol=1e-13))
    in3, target = (a.cpu().numpy().astype(np.float64) for a in sgn.record_sample(rec, 0))
    b = -(O.d_x(g, vx) + O.d_y(g, vy))
    r0 = b - O.apply_L(g, h, s)
    scale = np.sqrt(np.mean(r0 ** 2))
    ref_in = np.stack([r0 / scale, O.apply_Minv(g, r0) / scale, h - 1.0], axis=-1)
    sig, _ = O.gmres(g, h, b, s, 1e-13, 20, 400)
    ref_t = (sig - s) / scale
    e_in = [np.abs(in3[..., c] - ref_in[..., c]).max() / np.abs(ref_in[..., c]).max() for c in range(3)]
    e_t = np.abs(target - ref_t).max() / np.abs(ref_t).max()
    say(f"fp32 recorder sample 0: input errors {[f'{e:.1e}' for e in e_in]}, target error {e_t:.1e}")
    assert max(e_in) < 1e-5 and e_t < 1e-5
