"""Closed-form and seeded initial data for the 2D SGN equations.

Conventions (paper, Section 3, collocation grid): the torus has periods
2*pi*Lx and 2*pi*Ly, the grid is x_j = -pi*Lx + j*dx, j = 0..nx-1 with
dx = 2*pi*Lx/nx (same in y).  Fields are numpy float64 arrays of shape
(ny, nx): row index y, column index x, x contiguous.

The exact solitary wave (paper, Section 2.4, eq. (sol)):
    h_c   = h_inf + a * sech^2(kappa * xi),   xi = x - c t
    a     = (c^2 - g h_inf) / g
    kappa = sqrt(3 a g) / (2 c h_inf)
    h_c (u_c - c) = m,  m = -c h_inf
    sigma = m (h_c^2)' / 6
    v_x   = phi' = c + (m / h_c) (1 + (h_c^2)'' / 6)
All derivatives are taken analytically here.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Box:
    nx: int
    ny: int
    Lx: float
    Ly: float

    @property
    def dx(self) -> float:
        return 2.0 * math.pi * self.Lx / self.nx

    @property
    def dy(self) -> float:
        return 2.0 * math.pi * self.Ly / self.ny

    def coords(self):
        x = -math.pi * self.Lx + self.dx * np.arange(self.nx, dtype=np.float64)
        y = -math.pi * self.Ly + self.dy * np.arange(self.ny, dtype=np.float64)
        return x, y

    def mesh(self):
        x, y = self.coords()
        X, Y = np.meshgrid(x, y)  # shapes (ny, nx)
        return X, Y


@dataclasses.dataclass(frozen=True)
class SolitonParams:
    a: float
    c: float
    kappa: float
    h_inf: float
    g: float

    @property
    def m(self) -> float:
        return -self.c * self.h_inf


def soliton_params(a: float | None = None, c: float | None = None,
                   h_inf: float = 1.0, g: float = 1.0) -> SolitonParams:
    """Amplitude/speed relations of the solitary wave (Section 2.4):
    c^2 = g (h_inf + a), kappa = sqrt(3 a g) / (2 c h_inf)."""
    if (a is None) == (c is None):
        raise ValueError("give exactly one of a, c")
    if a is None:
        a = (c * c - g * h_inf) / g
    else:
        c = math.sqrt(g * (h_inf + a))
    if a <= 0:
        raise ValueError("solitary wave needs c^2 > g h_inf")
    kappa = math.sqrt(3.0 * a * g) / (2.0 * c * h_inf)
    return SolitonParams(a=a, c=c, kappa=kappa, h_inf=h_inf, g=g)


def soliton_profile(xi: np.ndarray, p: SolitonParams):
    """h, h', h'', sigma, v (=phi') and u of the solitary wave at coordinate xi,
    all analytic.  Returns a dict of float64 arrays."""
    xi = np.asarray(xi, dtype=np.float64)
    s = 1.0 / np.cosh(p.kappa * xi)
    t = np.tanh(p.kappa * xi)
    s2 = s * s
    h = p.h_inf + p.a * s2
    h1 = -2.0 * p.a * p.kappa * s2 * t
    h2 = 2.0 * p.a * p.kappa ** 2 * s2 * (3.0 * t * t - 1.0)
    hh1 = 2.0 * h * h1                       # (h^2)'
    hh2 = 2.0 * (h1 * h1 + h * h2)           # (h^2)''
    m = p.m
    sigma = m * hh1 / 6.0
    v = p.c + (m / h) * (1.0 + hh2 / 6.0)
    u = p.c * (1.0 - p.h_inf / h)
    # analytic derivative of v: v' = -(m h'/h^2)(1 + (h^2)''/6) + (m/h)(h^2)'''/6
    h3 = _h_third(xi, p)
    hh3 = 2.0 * (3.0 * h1 * h2 + h * h3)     # (h^2)'''
    v1 = -(m * h1 / (h * h)) * (1.0 + hh2 / 6.0) + (m / h) * hh3 / 6.0
    return dict(h=h, h1=h1, h2=h2, sigma=sigma, v=v, v1=v1, u=u)


def _h_third(xi, p: SolitonParams):
    # h''' of a*sech^2(kappa xi): d/dxi [2 a k^2 (3 s^2 t^2 - s^2)]
    # with (s^2)' = -2k s^2 t and t' = k s^2:
    # d(s^2 t^2) = -2k s^2 t^3 + 2k s^4 t ; d(s^2) = -2k s^2 t
    s = 1.0 / np.cosh(p.kappa * xi)
    t = np.tanh(p.kappa * xi)
    s2 = s * s
    k = p.kappa
    d = 3.0 * (-2.0 * k * s2 * t ** 3 + 2.0 * k * s2 * s2 * t) + 2.0 * k * s2 * t
    return 2.0 * p.a * k * k * d


def line_soliton(box: Box, a: float, x0: float = 0.0, h_inf: float = 1.0, g: float = 1.0,
                 along: str = "x"):
    """y-independent line solitary wave centred at x0 (exact solution).
    Returns h, vx, vy, sigma (exact sigma, usable as the first warm start)."""
    p = soliton_params(a=a, h_inf=h_inf, g=g)
    X, Y = box.mesh()
    if along == "x":
        prof = soliton_profile(_periodic_offset(X - x0, box.Lx), p)
        return prof["h"], prof["v"], np.zeros_like(X), prof["sigma"]
    prof = soliton_profile(_periodic_offset(Y - x0, box.Ly), p)
    return prof["h"], np.zeros_like(X), prof["v"], prof["sigma"]


def _periodic_offset(d, L):
    """Map a coordinate difference to [-pi L, pi L) so a profile centred
    anywhere on the torus is evaluated at its nearest image."""
    P = 2.0 * math.pi * L
    return (d + 0.5 * P) % P - 0.5 * P


def perturbed_line_soliton(box: Box, a: float, eps: float, k: int, x0: float = -10.0,
                           h_inf: float = 1.0, g: float = 1.0):
    """Transversely perturbed line soliton h = h_c(x - x0) (1 + eps cos(2 pi k y / P_y)),
    P_y = 2 pi Ly the y-period.  The velocity follows the paper's recipe for
    perturbed solitary waves (Section 4, eqs. (soldef), (solgauss)):
    v_x = c - (c/h)(1 + (h^2)_xx / 6) with the perturbed h, v_y = 0."""
    p = soliton_params(a=a, h_inf=h_inf, g=g)
    X, Y = box.mesh()
    prof = soliton_profile(_periodic_offset(X - x0, box.Lx), p)
    Py = 2.0 * math.pi * box.Ly
    f = 1.0 + eps * np.cos(2.0 * math.pi * k * Y / Py)
    h = prof["h"] * f
    hh_xx = 2.0 * (prof["h1"] ** 2 + prof["h"] * prof["h2"]) * f * f
    vx = p.c - (p.c * h_inf / h) * (1.0 + hh_xx / 6.0)
    return h, vx, np.zeros_like(h), np.zeros_like(h)


def deformed_line_soliton(box: Box, c: float = 1.7, x0: float = -10.0, amp: float = 0.1,
                          h_inf: float = 1.0, g: float = 1.0):
    """Deformed line solitary wave (Section 4.1, eq. (soldef)): the profile in
    x - x0 - amp cos(y); v_x = c - (c/h)(1 + (h^2)_xx / 6) with analytic x
    derivatives, v_y = 0."""
    p = soliton_params(c=c, h_inf=h_inf, g=g)
    X, Y = box.mesh()
    prof = soliton_profile(_periodic_offset(X - x0 - amp * np.cos(Y), box.Lx), p)
    h = prof["h"]
    hh_xx = 2.0 * (prof["h1"] ** 2 + h * prof["h2"])
    vx = c - (c * h_inf / h) * (1.0 + hh_xx / 6.0)
    return h, vx, np.zeros_like(h), np.zeros_like(h)


def soliton_plus_gaussian(box: Box, c: float = 1.7, x0: float = -20.0, sign: float = 1.0, amp: float = 0.1,
                          h_inf: float = 1.0, g: float = 1.0):
    """Line solitary wave with a localized Gaussian perturbation (Section 4.2,
    eq. (solgauss)): h = h_c(x - x0) +- amp exp(-(x - x0)^2 - y^2), v_x from
    the perturbed h as in eq. (soldef) with analytic derivatives, v_y = 0."""
    p = soliton_params(c=c, h_inf=h_inf, g=g)
    X, Y = box.mesh()
    xi = _periodic_offset(X - x0, box.Lx)
    prof = soliton_profile(xi, p)
    e = amp * sign * np.exp(-xi * xi - Y * Y)
    h = prof["h"] + e
    h1 = prof["h1"] - 2.0 * xi * e
    h2 = prof["h2"] + (4.0 * xi * xi - 2.0) * e
    hh_xx = 2.0 * (h1 * h1 + h * h2)
    vx = c - (c * h_inf / h) * (1.0 + hh_xx / 6.0)
    return h, vx, np.zeros_like(h), np.zeros_like(h)


def gaussian_hump(box: Box, alpha: float = 0.5, h_inf: float = 1.0):
    """Localized Gaussian h = h_inf + alpha exp(-x^2 - y^2), v = 0 (Section 6,
    eq. (gauss), read with the background depth h_inf added)."""
    X, Y = box.mesh()
    h = h_inf + alpha * np.exp(-X * X - Y * Y)
    z = np.zeros_like(h)
    return h, z.copy(), z.copy(), z.copy()


def crossing_solitons(box: Box, c: float = 1.7, h_inf: float = 1.0, g: float = 1.0):
    """Two crossing line solitary waves, one along x and one along y
    (Section 5, eq. (cross)), summed as the paper writes them:
    h = h_c(x) + h_c(y), so the far field is 2 h_inf; v_x is the x-wave's
    velocity and v_y the y-wave's, each built from its own h_c."""
    p = soliton_params(c=c, h_inf=h_inf, g=g)
    X, Y = box.mesh()
    px = soliton_profile(X, p)
    py = soliton_profile(Y, p)
    h = px["h"] + py["h"]
    return h, px["v"], py["v"], np.zeros_like(h)


# Ensemble of perturbed line solitons on uneven grids (the batched workload).
ENSEMBLE_GRIDS = ((256, 256), (512, 512), (1024, 512), (1024, 1024))


def ensemble_member(seed: int, nx: int, ny: int, h_inf: float = 1.0, g: float = 1.0):
    """Member `seed` of the ensemble: grid spacing dx = dy = pi/16 (L = n/32),
    a line soliton with amplitude a ~ U[0.1, 1.0] at x0 = -pi Lx / 2, times a
    transverse perturbation 1 + eps P(y), P = sum_{1<=|n|<=8} Re(z_n e^{2 pi i n
    y / P_y}) with z_n ~ CN(0, 1) exp(-n^2/16), rescaled to max |P| = 1, eps
    log-uniform in [1e-3, 1e-2]; v_x = c - (c/h)(1 + (h^2)_xx / 6), v_y = 0.
    Returns (Box, (h, vx, vy, sigma0), params)."""
    rng = np.random.default_rng(seed)
    a = float(rng.uniform(0.1, 1.0))
    eps = float(10.0 ** rng.uniform(-3.0, -2.0))
    z = (rng.standard_normal(17) + 1j * rng.standard_normal(17)) / math.sqrt(2.0)
    box = Box(nx, ny, nx / 32.0, ny / 32.0)
    X, Y = box.mesh()
    Py = 2.0 * math.pi * box.Ly
    P = np.zeros(ny)
    y = box.coords()[1]
    for i, n in enumerate([m for m in range(-8, 9) if m != 0]):
        P += np.real(z[i] * math.exp(-n * n / 16.0) * np.exp(2j * math.pi * n * y / Py))
    P /= np.abs(P).max()
    f = (1.0 + eps * P)[:, None]
    p = soliton_params(a=a, h_inf=h_inf, g=g)
    prof = soliton_profile(_periodic_offset(X + math.pi * box.Lx / 2.0, box.Lx), p)
    h = prof["h"] * f
    hh_xx = 2.0 * (prof["h1"] ** 2 + prof["h"] * prof["h2"]) * f * f
    vx = p.c - (p.c * h_inf / h) * (1.0 + hh_xx / 6.0)
    return box, (h, vx, np.zeros_like(h), np.zeros_like(h)), dict(a=a, eps=eps, dt=0.005)


def random_smooth_field(rng: np.random.Generator, ny: int, nx: int, kmax: int = 6,
                        decay: float = 0.35) -> np.ndarray:
    """Real field sum of random trigonometric modes |m_x|, |m_y| <= kmax with
    amplitudes exp(-decay (m_x^2 + m_y^2)); O(1), zero mean, smooth and
    periodic.  Built in physical space from cos/sin so no transform is used."""
    y = 2.0 * math.pi * np.arange(ny) / ny
    x = 2.0 * math.pi * np.arange(nx) / nx
    kx = min(kmax, nx // 2 - 1)
    ky = min(kmax, ny // 2 - 1)
    f = np.zeros((ny, nx))
    for my in range(-ky, ky + 1):
        for mx in range(0, kx + 1):
            if mx == 0 and my <= 0:
                continue
            amp = math.exp(-decay * (mx * mx + my * my))
            a, b = rng.standard_normal(2) * amp
            ph = my * y[:, None] + mx * x[None, :]
            f += a * np.cos(ph) + b * np.sin(ph)
    scale = np.max(np.abs(f))
    return f / scale if scale > 0 else f


def random_state(rng: np.random.Generator, box: Box, amp_h: float = 0.3, amp_v: float = 0.3,
                 kmax: int = 6):
    """Seeded smooth random state (h, vx, vy, sigma0) with h in [1-amp_h, 1+amp_h]."""
    ny, nx = box.ny, box.nx
    h = 1.0 + amp_h * random_smooth_field(rng, ny, nx, kmax)
    vx = amp_v * random_smooth_field(rng, ny, nx, kmax)
    vy = amp_v * random_smooth_field(rng, ny, nx, kmax)
    s0 = 0.05 * random_smooth_field(rng, ny, nx, kmax)
    return h, vx, vy, s0


# Named workloads of the build.  Boxes are given as (nx, ny, Lx, Ly) with the
# torus [-pi Lx, pi Lx) x [-pi Ly, pi Ly).
WORKLOADS = {
    # 128x64 line soliton a=0.5 on [-10pi,10pi]x[-5pi,5pi], dt=0.01, 200 steps
    "line_soliton_128x64": dict(nx=128, ny=64, Lx=10.0, Ly=5.0, dt=0.01, steps=200,
                                tol=1e-10, restart=20),
    # 1024x512 transversely perturbed line soliton, dt=0.005, tol 1e-10
    "perturbed_soliton_1024x512": dict(nx=1024, ny=512, Lx=10.0, Ly=5.0, dt=0.005,
                                       steps=4000, tol=1e-10, restart=20),
    # 2048x2048 Gaussian hump on [-20pi,20pi]^2, dt=0.005 to t=5
    "gaussian_2048x2048": dict(nx=2048, ny=2048, Lx=20.0, Ly=20.0, dt=0.005, steps=1000,
                               tol=1e-10, restart=20),
}


# The nine runs of the 1024x512 perturbed-soliton workload: amplitudes a and
# transverse wavenumbers k of h = h_c(x - x0) (1 + eps cos(2 pi k y / (2 pi Ly))).
SWEEP_AMPLITUDES = (0.2, 0.5, 1.0)
SWEEP_WAVENUMBERS = (1, 2, 4)


def perturbed_soliton_sweep(eps: float = 0.01, x0: float = -10.0):
    """The nine (a, k) runs of the 1024x512 workload stacked as ensemble
    members: returns (box, (h, vx, vy, sigma0) arrays of shape (9, ny, nx),
    [(a, k), ...], params)."""
    w = WORKLOADS["perturbed_soliton_1024x512"]
    box = Box(w["nx"], w["ny"], w["Lx"], w["Ly"])
    ak = [(a, k) for a in SWEEP_AMPLITUDES for k in SWEEP_WAVENUMBERS]
    st = [perturbed_line_soliton(box, a=a, eps=eps, k=k, x0=x0) for a, k in ak]
    return box, tuple(np.stack([m[i] for m in st]) for i in range(4)), ak, w


def workload(name: str, a: float = 0.5, eps: float = 0.01, k: int = 2):
    """Return (box, (h, vx, vy, sigma0), params) for a named workload."""
    w = WORKLOADS[name]
    box = Box(w["nx"], w["ny"], w["Lx"], w["Ly"])
    if name == "line_soliton_128x64":
        st = line_soliton(box, a=a, x0=0.0)
    elif name == "perturbed_soliton_1024x512":
        st = perturbed_line_soliton(box, a=a, eps=eps, k=k, x0=-10.0)
    elif name == "gaussian_2048x2048":
        st = gaussian_hump(box, alpha=0.5)
    elif name == "crossing_solitons_1024x1024":
        st = oblique_crossing_solitons(box, a=0.4)
    else:  # pragma: no cover
        raise KeyError(name)
    return box, st, w


def oblique_crossing_solitons(box: Box, a: float = 0.4, slope: float = 0.5, h_inf: float = 1.0, g: float = 1.0):
    """Two line solitary waves of amplitude a crossing at +- theta, tan theta =
    slope, on a square torus (Lx = Ly): wave +- travels along (cos theta,
    +- sin theta).  With slope = 1/2 the phase xi = x cos theta +- y sin theta
    is periodic on the box (period 2 pi Lx cos theta / 2), so each wave is
    continued periodically; h = h_inf + sum of the two excesses and v = sum of
    the two waves' v (the variable of the (h, v) system, eq. (soldef) profile)
    times their directions, so each wave alone is the exact solitary wave of
    its direction.  The superposition is initial data, not a solution."""
    if abs(box.Lx - box.Ly) > 1e-12 or abs(slope - 0.5) > 1e-12:
        raise ValueError("oblique_crossing_solitons: square box and slope 1/2 only")
    p = soliton_params(a=a, h_inf=h_inf, g=g)
    X, Y = box.mesh()
    ct, st = 2.0 / math.sqrt(5.0), 1.0 / math.sqrt(5.0)
    period = 2.0 * math.pi * box.Lx * st  # shifts by the box move xi by multiples of this
    h = np.full_like(X, h_inf)
    vx = np.zeros_like(X)
    vy = np.zeros_like(X)
    for sgn in (1.0, -1.0):
        xi = X * ct + sgn * Y * st
        xi = (xi + 0.5 * period) % period - 0.5 * period
        prof = soliton_profile(xi, p)
        h += prof["h"] - h_inf
        vx += prof["v"] * ct
        vy += sgn * prof["v"] * st
    return h, vx, vy, np.zeros_like(h)


WORKLOADS["crossing_solitons_1024x1024"] = dict(nx=1024, ny=1024, Lx=10.0, Ly=10.0, dt=0.005, steps=400,
                                                 tol=1e-8, restart=20)
