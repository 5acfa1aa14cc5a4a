"""Host logic of the learned guess's training recipe (no GPU): the recorded
sources cover about 10^4 samples at the workloads' grid spacing and hold out
the evaluated runs, and recorded samples of other grid sizes are mapped onto
the 512 x 1024 training grid by periodic repetition or by tiling."""
import numpy as np
import torch

from paper_2306_09731_amd import learned, sgn


def test_training_sources_spacing_count_and_held_out_runs():
    src = learned.training_sources()
    spacing = 2 * np.pi / 102.4
    total = 0
    for nx, ny, Lx, Ly, state, steps in src:
        assert abs(2 * np.pi * Lx / nx - spacing) < 1e-12 and abs(2 * np.pi * Ly / ny - spacing) < 1e-12
        assert state[0].shape == (ny, nx) and np.all(state[0] > 0)
        total += 4 * steps * (nx * ny // (learned.TRAIN_H * learned.TRAIN_W) if nx * ny > 512 * 1024 else 1)
    assert 9000 <= total <= 11000
    # the evaluated 1024 x 512 run (a = 0.5, k = 2) and the 1024^2 crossing solitons are not sources
    from sgn_inputs import workload
    _, held, _ = workload("perturbed_soliton_1024x512", a=0.5, eps=0.01, k=2)
    for nx, ny, Lx, Ly, state, steps in src:
        if (nx, ny) == (1024, 512):
            assert not np.array_equal(state[0], held[0])
        assert (nx, ny) != (1024, 1024)


def _record(n, H, W, seed):
    g = torch.Generator().manual_seed(seed)
    return torch.randn(n, 4, H, W, generator=g, dtype=torch.float32)


def test_training_samples_repeat_small_and_tile_large_grids():
    H, W = learned.TRAIN_H, learned.TRAIN_W
    small = _record(2, 512, 512, 0)
    big = _record(1, 2048, 2048, 1)
    exact = _record(1, H, W, 2)
    out = learned.training_samples([small, big, exact])
    assert len(out) == 2 + 8 + 1
    for x, t in out:
        assert x.shape == (H, W, 3) and t.shape == (H, W) and x.is_contiguous() and t.is_contiguous()
    # 512 x 512: repeated once along x
    x0, t0 = sgn.record_sample(small, 0)
    assert torch.equal(out[0][0][:, :512], x0) and torch.equal(out[0][0][:, 512:], x0)
    assert torch.equal(out[0][1][:, 512:], t0)
    # 2048 x 2048: eight tiles in row-major order
    xb, tb = sgn.record_sample(big, 0)
    for k, (y0, x0_) in enumerate([(y, x) for y in range(0, 2048, H) for x in range(0, 2048, W)]):
        assert torch.equal(out[2 + k][0], xb[y0:y0 + H, x0_:x0_ + W])
        assert torch.equal(out[2 + k][1], tb[y0:y0 + H, x0_:x0_ + W])
    # the training grid itself: unchanged
    xe, te = sgn.record_sample(exact, 0)
    assert torch.equal(out[-1][0], xe) and torch.equal(out[-1][1], te)
