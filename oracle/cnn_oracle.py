"""FP64 reference of the learned initial guess (test infrastructure).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
import this module; the GPU path never does.

The paper has no network: it starts every GMRES solve from the previous
sigma (Section 3, the warm start).  The learned guess corrects that warm
start.  With r0 = b - L sigma_prev (eq. (3): the residual of the warm start)
the exact correction is e = L^-1 r0, and a small convolutional network
predicts e / |r0| from three channels per grid point,

    r0 / |r0|,   M^-1 r0 / |r0|,   h - h_inf,

|r0| the RMS of r0 and M^-1 the spectral preconditioner of Section 3.  The
network: six 3x3 convolutions with periodic (circular) padding, 32 channels,
ReLU after the first five, none after the last (1 output channel).  It is
trained by mean squared error with Adam (Kingma & Ba, "Adam: a method for
stochastic optimization", 2015, Algorithm 1).

Layouts (the GPU path uses the same): activations [H][W][C] (channels last);
weights w[ky][kx][cout][cin], tap (ky, kx) reading the input at
(y + ky - 1, x + kx - 1) modulo the grid.  Everything here is plain numpy in
FP64: np.roll for the circular shifts, matrix products per tap.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

CHANNELS = 32
LAYERS = 6
IN_CHANNELS = 3


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray | None = None) -> np.ndarray:
    """y[p, co] = b[co] + sum_{ky,kx,ci} w[ky, kx, co, ci] x[p + (ky-1, kx-1), ci] (circular)."""
    H, W, _ = x.shape
    cout = w.shape[2]
    y = np.zeros((H, W, cout))
    for ky in range(3):
        for kx in range(3):
            xs = np.roll(x, shift=(1 - ky, 1 - kx), axis=(0, 1))  # xs[p] = x[p + (ky-1, kx-1)]
            y += xs @ w[ky, kx].T
    if b is not None:
        y += b
    return y


def conv3x3_input_grad(dy: np.ndarray, w: np.ndarray) -> np.ndarray:
    """The adjoint of conv3x3 in x: dx[q, ci] = sum_{ky,kx,co} w[ky, kx, co, ci] dy[q - (ky-1, kx-1), co]."""
    H, W, _ = dy.shape
    cin = w.shape[3]
    dx = np.zeros((H, W, cin))
    for ky in range(3):
        for kx in range(3):
            ds = np.roll(dy, shift=(ky - 1, kx - 1), axis=(0, 1))  # ds[q] = dy[q - (ky-1, kx-1)]
            dx += ds @ w[ky, kx]
    return dx


def conv3x3_weight_grad(dy: np.ndarray, x: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """dw[ky, kx, co, ci] = sum_p dy[p, co] x[p + (ky-1, kx-1), ci];  db[co] = sum_p dy[p, co]."""
    cout, cin = dy.shape[2], x.shape[2]
    dw = np.zeros((3, 3, cout, cin))
    flat_dy = dy.reshape(-1, cout)
    for ky in range(3):
        for kx in range(3):
            xs = np.roll(x, shift=(1 - ky, 1 - kx), axis=(0, 1)).reshape(-1, cin)
            dw[ky, kx] = flat_dy.T @ xs
    return dw, flat_dy.sum(axis=0)


@dataclass
class Net:
    """Weights w[l] of shape (3, 3, cout_l, cin_l) and biases b[l]."""
    w: list = field(default_factory=list)
    b: list = field(default_factory=list)


def layer_shapes(cin: int = IN_CHANNELS, ch: int = CHANNELS, layers: int = LAYERS, cout: int = 1):
    dims = [cin] + [ch] * (layers - 1) + [cout]
    return [(dims[l + 1], dims[l]) for l in range(layers)]


def init_net(rng: np.random.Generator, cin: int = IN_CHANNELS, ch: int = CHANNELS, layers: int = LAYERS,
             cout: int = 1) -> Net:
    """He-normal weights (std sqrt(2 / fan_in), fan_in = 9 cin), zero biases."""
    net = Net()
    for co, ci in layer_shapes(cin, ch, layers, cout):
        net.w.append(rng.normal(0.0, np.sqrt(2.0 / (9 * ci)), size=(3, 3, co, ci)))
        net.b.append(np.zeros(co))
    return net


def forward(net: Net, x: np.ndarray) -> list[np.ndarray]:
    """Activations a_0 = x, a_{l+1} = relu(conv(a_l)) (no ReLU after the last layer)."""
    acts = [x]
    n = len(net.w)
    for l in range(n):
        z = conv3x3(acts[-1], net.w[l], net.b[l])
        acts.append(np.maximum(z, 0.0) if l < n - 1 else z)
    return acts


def mse(pred: np.ndarray, target: np.ndarray) -> float:
    """Mean over grid points of (pred - target)^2 (pred, target: [H][W])."""
    return float(np.mean((pred - target) ** 2))


def backward(net: Net, acts: list[np.ndarray], target: np.ndarray) -> tuple[float, list, list]:
    """Loss = mse(acts[-1][..., 0], target) and its gradients in every w[l], b[l]."""
    n = len(net.w)
    pred = acts[-1][..., 0]
    H, W = pred.shape
    loss = mse(pred, target)
    d = np.zeros_like(acts[-1])
    d[..., 0] = 2.0 * (pred - target) / (H * W)
    gw, gb = [None] * n, [None] * n
    for l in range(n - 1, -1, -1):
        gw[l], gb[l] = conv3x3_weight_grad(d, acts[l])
        if l > 0:
            d = conv3x3_input_grad(d, net.w[l]) * (acts[l] > 0.0)  # through the ReLU of layer l-1
    return loss, gw, gb


@dataclass
class Adam:
    """Adam moments for a list of arrays."""
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    t: int = 0
    m: list = field(default_factory=list)
    v: list = field(default_factory=list)


def adam_step(opt: Adam, params: list, grads: list) -> None:
    """One step of Algorithm 1 of Kingma & Ba in place on params."""
    if not opt.m:
        opt.m = [np.zeros_like(p) for p in params]
        opt.v = [np.zeros_like(p) for p in params]
    opt.t += 1
    for p, g, m, v in zip(params, grads, opt.m, opt.v):
        m *= opt.beta1
        m += (1.0 - opt.beta1) * g
        v *= opt.beta2
        v += (1.0 - opt.beta2) * g * g
        mhat = m / (1.0 - opt.beta1 ** opt.t)
        vhat = v / (1.0 - opt.beta2 ** opt.t)
        p -= opt.lr * mhat / (np.sqrt(vhat) + opt.eps)


def rms(a: np.ndarray) -> float:
    return float(np.sqrt(np.mean(a * a)))


def features(r0: np.ndarray, minv_r0: np.ndarray, h: np.ndarray, h_inf: float = 1.0) -> tuple[np.ndarray, float]:
    """Network input [H][W][3] and the scale |r0| (RMS)."""
    s = rms(r0)
    inv = 1.0 / s if s > 0 else 0.0
    return np.stack([r0 * inv, minv_r0 * inv, h - h_inf], axis=-1), s


def guess(net: Net, sigma_prev: np.ndarray, r0: np.ndarray, minv_r0: np.ndarray, h: np.ndarray,
          h_inf: float = 1.0) -> np.ndarray:
    """sigma_prev + |r0| * net(features)."""
    x, s = features(r0, minv_r0, h, h_inf)
    return sigma_prev + s * forward(net, x)[-1][..., 0]
