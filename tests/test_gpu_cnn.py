"""The learned-guess network on the GPU against the FP64 oracle.

The GPU keeps weights and activations in BF16 and accumulates in FP32.  The
reference gets the same BF16-rounded weights and input and rounds each hidden
activation to BF16 as the GPU does (test-side emulation of the storage
format), then computes in FP64; what remains is FP32 accumulation order and
the rare activation that lands on the other side of a BF16 rounding
boundary.  Gates: network output within 5e-3 of max |output| (elementwise);
loss within 1e-3 relative; weight and bias gradients per layer within 3e-2
normwise (the gradient buffers between layers are BF16 too); one Adam step
(FP32) within 2e-6 of the oracle's FP64 step from the same gradients."""
import numpy as np
import pytest
import torch

from oracle import cnn_oracle as C
from paper_2306_09731_amd import sgn

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]
DEV = "cuda:0"
CH = sgn.SGN_CNN_CH


def say(msg):
    print(msg, flush=True)


def bf16_round(a):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def pack(net: C.Net) -> np.ndarray:
    """Oracle network (true shapes) -> the library's padded FP32 parameter vector."""
    out = []
    for w, b in zip(net.w, net.b):
        wp = np.zeros((9, CH, CH))
        wp[:, :w.shape[2], :w.shape[3]] = w.reshape(9, w.shape[2], w.shape[3])
        bp = np.zeros(CH)
        bp[:b.shape[0]] = b
        out += [wp.ravel(), bp]
    return np.concatenate(out).astype(np.float32)


def unpack_grads(g: np.ndarray, net: C.Net):
    per = 9 * CH * CH + CH
    gw, gb = [], []
    for l, (w, b) in enumerate(zip(net.w, net.b)):
        blk = g[l * per:(l + 1) * per].astype(np.float64)
        wl = blk[:9 * CH * CH].reshape(3, 3, CH, CH)[:, :, :w.shape[2], :w.shape[3]]
        gw.append(wl)
        gb.append(blk[9 * CH * CH:][:b.shape[0]])
    return gw, gb


def rounded_net(net: C.Net) -> C.Net:
    return C.Net(w=[bf16_round(w) for w in net.w], b=[np.asarray(b, np.float32).astype(np.float64) for b in net.b])


def emulated_forward(net: C.Net, x):
    """The oracle's layers with each hidden activation rounded to BF16."""
    acts = [bf16_round(x)]
    n = len(net.w)
    for l in range(n):
        z = C.conv3x3(acts[-1], net.w[l], net.b[l])
        acts.append(bf16_round(np.maximum(z, 0.0)) if l < n - 1 else z)
    return acts


def make(H, W, seed):
    rng = np.random.default_rng(seed)
    net = C.init_net(rng)
    for b in net.b:
        b += rng.normal(scale=0.05, size=b.shape)
    x = rng.normal(size=(H, W, 3))
    x[..., 2] *= 0.3
    target = rng.normal(scale=0.5, size=(H, W))
    return net, x, target


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


@pytest.mark.parametrize("H,W", [(32, 32), (64, 64), (16, 128), (128, 64), (512, 1024), (1024, 1024)])
def test_cnn_forward_matches_oracle(H, W):
    net, x, _ = make(H, W, H * 7 + W)
    cn = sgn.cnn_init(H, W, DEV)
    sgn.cnn_set_params(cn, pack(net))
    out = torch.empty(H, W, dtype=torch.float32, device=DEV)
    sgn.cnn_forward(cn, dev(x), out)
    torch.cuda.synchronize()
    ref = emulated_forward(rounded_net(net), x)[-1][..., 0]
    got = out.cpu().numpy().astype(np.float64)
    e = np.abs(got - ref).max() / np.abs(ref).max()
    say(f"cnn forward {H}x{W}: max |out - ref| / max |ref| = {e:.2e}")
    assert e < 5e-3


@pytest.mark.parametrize("H,W", [(32, 32), (64, 128), (512, 1024), (1024, 1024)])
def test_cnn_gradients_match_oracle(H, W):
    net, x, target = make(H, W, 100 + H + W)
    cn = sgn.cnn_init(H, W, DEV)
    sgn.cnn_set_params(cn, pack(net))
    g, loss = sgn.cnn_gradients(cn, dev(x), dev(target))
    rnet = rounded_net(net)
    acts = emulated_forward(rnet, x)
    loss_ref, gw_ref, gb_ref = C.backward(rnet, acts, np.asarray(target, np.float32).astype(np.float64))
    gw, gb = unpack_grads(g, net)
    say(f"cnn loss {H}x{W}: gpu {loss:.6e} oracle {loss_ref:.6e}")
    assert abs(loss - loss_ref) < 1e-3 * loss_ref
    for l in range(len(net.w)):
        ew = np.linalg.norm(gw[l] - gw_ref[l]) / np.linalg.norm(gw_ref[l])
        eb = np.linalg.norm(gb[l] - gb_ref[l]) / max(np.linalg.norm(gb_ref[l]), 1e-30)
        mw = np.abs(gw[l] - gw_ref[l]).max() / np.abs(gw_ref[l]).max()
        say(f"  layer {l}: weight-gradient error {ew:.2e} (max-norm {mw:.2e}), bias-gradient error {eb:.2e}")
        assert ew < 3e-2 and eb < 3e-2
    # padded parameters get no gradient
    per = 9 * CH * CH + CH
    w0 = g[:9 * CH * CH].reshape(9, CH, CH)
    assert np.all(w0[:, :, 3:] == 0)
    last = g[5 * per:6 * per]
    assert np.all(last[:9 * CH * CH].reshape(9, CH, CH)[:, 1:, :] == 0) and np.all(last[9 * CH * CH + 1:] == 0)


def test_cnn_adam_step_matches_oracle():
    H, W = 32, 64
    net, x, target = make(H, W, 7)
    cn = sgn.cnn_init(H, W, DEV)
    p0 = pack(net)
    sgn.cnn_set_params(cn, p0)
    g, _ = sgn.cnn_gradients(cn, dev(x), dev(target))
    lr = 1e-3
    sgn.cnn_train_step(cn, dev(x), dev(target), lr)
    p1 = sgn.cnn_get_params(cn).astype(np.float64)
    opt = C.Adam(lr=lr)
    ref = [p0.astype(np.float64).copy()]
    C.adam_step(opt, ref, [g.astype(np.float64)])
    e = np.abs(p1 - ref[0]).max()
    say(f"cnn Adam step: max |p1 - ref| = {e:.2e}, max |step| = {np.abs(ref[0] - p0).max():.2e}")
    assert e < 2e-6


def test_cnn_training_reduces_the_loss():
    """A learnable target (a smoothed input channel): 60 Adam steps must cut the
    loss at least in half; the run is deterministic (same losses twice)."""
    H, W = 64, 64
    net, x, _ = make(H, W, 11)
    k = np.fft.fftfreq(W)[None, :] ** 2 + np.fft.fftfreq(H)[:, None] ** 2
    target = np.real(np.fft.ifft2(np.fft.fft2(x[..., 0]) / (1.0 + 40.0 * k)))
    runs = []
    for _ in range(2):
        cn = sgn.cnn_init(H, W, DEV)
        sgn.cnn_set_params(cn, pack(net))
        losses = [sgn.cnn_train_step(cn, dev(x), dev(target), 2e-3) for _ in range(60)]
        runs.append(losses)
    say(f"cnn training: loss {runs[0][0]:.4e} -> {runs[0][-1]:.4e}")
    assert runs[0][-1] < 0.5 * runs[0][0]
    assert runs[0] == runs[1]


def test_cnn_argument_errors():
    assert sgn.cnn_workspace_bytes(64, 16) == 0 and sgn.cnn_workspace_bytes(48, 64) == 0
    with pytest.raises(sgn.SgnError):
        sgn.cnn_init(64, 16, DEV)
    cn = sgn.cnn_init(32, 32, DEV)
    with pytest.raises(ValueError):
        sgn.cnn_forward(cn, torch.zeros(32, 32, 2, device=DEV), torch.zeros(32, 32, device=DEV))
    with pytest.raises(ValueError):
        sgn.cnn_set_params(cn, np.zeros(10, dtype=np.float32))
