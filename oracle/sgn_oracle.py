"""FP64 CPU oracle of the 2D Serre-Green-Naghdi hot path (Gavrilyuk & Klein,
"Numerical study of the Serre-Green-Naghdi equations in 2D").

TEST INFRASTRUCTURE ONLY.  This module is imported by the tests, by the
smoke check and by the benchmark's CPU-baseline leg.  The product (the HIP
library and its Python binding) never imports or calls it, and it shares no
code, tables or helpers with the HIP path.

It is plain and slow on purpose: numpy.fft is the only library primitive used
(as the DFT step); everything else is the paper's formulas written out in
float64, in the paper's order.

Readings of the paper used here (where it is silent or garbled):
  * grid: x_j = -pi Lx + j dx, dx = 2 pi Lx / nx, j = 0..nx-1 (Section 3; the
    printed collocation formula lacks the 1/N_x, and n = 1..N is the same
    point set shifted by one period);
  * wavenumbers k = m / L for m in [-N/2, N/2) with the Nyquist mode set to 0,
    so the discrete Laplacian is D.D and the preconditioner uses the same k;
  * preconditioner M = 3/h_inf^3 + (kx^2 + ky^2)/h_inf, i.e. the operator L at
    h = h_inf (Section 3 takes the operator at unit depth, M = 3 + kx^2 + ky^2
    for h_inf = 1);
  * GMRES: restarted, left-preconditioned, modified Gram-Schmidt Arnoldi with
    Givens rotations (Saad & Schultz); stop when the preconditioned residual
    is <= tol * ||M^-1 b||;
  * warm start: every RHS evaluation starts GMRES from the sigma returned by
    the previous evaluation (Section 3);
  * optional stage-increment guess (Config.guess = 1, not in the paper): RK
    stage i of step n starts GMRES from sigma_{i-1}(n) + D_i, where D_i is the
    increment sigma_i - sigma_{i-1} of the same stage in step n - 1 (zero in
    the first step of an rk4 call); the converged sigma still meets the same
    tolerance;
  * Krasny filter: normalised 2D DFT coefficients |F f| / N below the
    threshold are set to zero in h, v_x, v_y once per completed RK4 step;
  * optional two-thirds rule (Config.dealias, off by default; Orszag's
    dealiasing, not part of the paper's scheme): in the same place, modes
    with 3 |m_x| > nx or 3 |m_y| > ny are set to zero as well;
  * h-equation written as h_t = -D.(h v - D sigma), which equals
    -D.(h v) + Laplacian(sigma) when the Laplacian is D.D (eq. (1)).
Parity pins for every function live in tests/test_oracle_pins.py.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# ---------------------------------------------------------------------------
# Configuration and grid (Section 3, collocation points and wavenumbers)
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class Config:
    nx: int
    ny: int
    Lx: float
    Ly: float
    g: float = 1.0
    h_inf: float = 1.0
    gmres_tol: float = 1e-10
    gmres_restart: int = 20
    gmres_max_iters: int = 200
    krasny: float = 0.0          # 0 disables the filter
    invariants_tol: float = 1e-13
    dealias: bool = False        # two-thirds rule after each step (not in the paper)
    guess: int = 0               # 0: previous sigma (Section 3); 1: stage-increment extrapolation


class Grid:
    """Torus [-pi Lx, pi Lx) x [-pi Ly, pi Ly) with nx x ny collocation points
    (Section 3).  Fields are arrays of shape (ny, nx), x contiguous."""

    def __init__(self, cfg: Config):
        self.cfg = cfg
        nx, ny = cfg.nx, cfg.ny
        self.nx, self.ny = nx, ny
        self.dx = 2.0 * math.pi * cfg.Lx / nx
        self.dy = 2.0 * math.pi * cfg.Ly / ny
        self.x = -math.pi * cfg.Lx + self.dx * np.arange(nx)
        self.y = -math.pi * cfg.Ly + self.dy * np.arange(ny)
        self.kx = self._wavenumbers(nx, cfg.Lx)       # shape (nx,)
        self.ky = self._wavenumbers(ny, cfg.Ly)       # shape (ny,)
        KX, KY = np.meshgrid(self.kx, self.ky)
        # preconditioner symbol: L at h = h_inf (Section 3)
        self.M = 3.0 / cfg.h_inf ** 3 + (KX * KX + KY * KY) / cfg.h_inf

    @staticmethod
    def _wavenumbers(n: int, L: float) -> np.ndarray:
        m = np.arange(n, dtype=np.float64)
        m[m >= n // 2] -= n
        k = m / L
        if n % 2 == 0:
            k[n // 2] = 0.0   # Nyquist mode of an odd derivative set to zero
        return k


# ---------------------------------------------------------------------------
# Spectral derivatives (Section 3: derivative <-> multiplication by i k)
# ---------------------------------------------------------------------------


def d_x(grid: Grid, f: np.ndarray) -> np.ndarray:
    """x-derivative of a real periodic field: Re F_x^-1 (i k_x F_x f), row-wise."""
    F = np.fft.fft(f, axis=1)
    return np.real(np.fft.ifft(1j * grid.kx[None, :] * F, axis=1))


def d_y(grid: Grid, f: np.ndarray) -> np.ndarray:
    """y-derivative: Re F_y^-1 (i k_y F_y f), column-wise."""
    F = np.fft.fft(f, axis=0)
    return np.real(np.fft.ifft(1j * grid.ky[:, None] * F, axis=0))


# ---------------------------------------------------------------------------
# Elliptic operator and preconditioner (Section 2.2 eq. (3), Section 3 eq. (sigmav))
# ---------------------------------------------------------------------------


def apply_L(grid: Grid, h: np.ndarray, s: np.ndarray) -> np.ndarray:
    """L_h[s] = 3 s / h^3 - div(grad s / h)  (eq. (3) / (sigmav))."""
    return 3.0 * s / h ** 3 - d_x(grid, d_x(grid, s) / h) - d_y(grid, d_y(grid, s) / h)


def apply_Minv(grid: Grid, r: np.ndarray) -> np.ndarray:
    """M^-1 r with M = L at h = h_inf, diagonal in Fourier space (Section 3)."""
    return np.real(np.fft.ifft2(np.fft.fft2(r) / grid.M))


# ---------------------------------------------------------------------------
# GMRES (Saad & Schultz), left-preconditioned, restarted (Section 3)
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class SolveInfo:
    iters: int = 0
    restarts: int = 0
    rel_resid_precond: float = 0.0
    rel_resid_true: float = 0.0
    converged: bool = False


def _dot(a, b):
    return float(np.sum(a * b))


def gmres(grid: Grid, h: np.ndarray, b: np.ndarray, x0: np.ndarray, tol: float,
          restart: int, max_iters: int, record: dict | None = None):
    """Solve L_h x = b by GMRES(restart) applied to M^-1 L_h x = M^-1 b.

    Arnoldi with modified Gram-Schmidt; the least-squares problem is kept
    upper triangular with Givens rotations; the stopping test is on the
    preconditioned residual relative to ||M^-1 b||.  Returns (x, SolveInfo).
    record (tests only): receives, for the first cycle, the basis "V", the
    Hessenberg matrix before rotation "Hbar" ((k+1) x k) and the residual
    estimates |g_{j+1}| / ||M^-1 b|| after each step, "resid".
    """
    info = SolveInfo()
    x = np.array(x0, dtype=np.float64, copy=True)
    pb = apply_Minv(grid, b)
    beta0 = math.sqrt(_dot(pb, pb))
    bnorm = math.sqrt(_dot(b, b))
    if beta0 == 0.0:
        x[:] = 0.0
        info.converged = True
        return x, info
    m = restart
    total = 0
    while True:
        r = apply_Minv(grid, b - apply_L(grid, h, x))
        beta = math.sqrt(_dot(r, r))
        info.rel_resid_precond = beta / beta0
        if beta <= tol * beta0:
            info.converged = True
            break
        if total >= max_iters:
            break
        V = [r / beta]
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        k = 0
        done = False
        for j in range(m):
            if total >= max_iters:
                break
            w = apply_Minv(grid, apply_L(grid, h, V[j]))
            for i in range(j + 1):                       # modified Gram-Schmidt
                H[i, j] = _dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = math.sqrt(_dot(w, w))
            if record is not None and info.restarts == 0:
                record.setdefault("Hbar", np.zeros((m + 1, m)))[:j + 2, j] = H[:j + 2, j]
            for i in range(j):                           # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            rho = math.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / rho
            sn[j] = H[j + 1, j] / rho
            H[j, j] = rho
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            k = j + 1
            info.rel_resid_precond = abs(g[j + 1]) / beta0
            if record is not None and info.restarts == 0:
                record.setdefault("resid", []).append(abs(g[j + 1]) / beta0)
            if abs(g[j + 1]) <= tol * beta0:
                done = True
                break
            hn = math.sqrt(_dot(w, w))
            if hn == 0.0:                                # happy breakdown
                done = True
                break
            V.append(w / hn)
        if record is not None and info.restarts == 0:
            record["V"] = list(V)
            record["Hbar"] = record["Hbar"][:len(V), :k]
        # back substitution for y in R y = g, then x += V y
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]
        for i in range(k):
            x = x + y[i] * V[i]
        if done:
            info.converged = True
            break
        info.restarts += 1
        if total >= max_iters:
            break
    info.iters = total
    res = b - apply_L(grid, h, x)
    info.rel_resid_true = math.sqrt(_dot(res, res)) / bnorm if bnorm > 0 else 0.0
    pr = apply_Minv(grid, res)
    info.rel_resid_precond = math.sqrt(_dot(pr, pr)) / beta0
    return x, info


# ---------------------------------------------------------------------------
# Right-hand side of the (h, v) system (Section 3 eq. (sigmav), eq. (1) and the
# gradient form of the Bernoulli equation (2))
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class RhsResult:
    dh: np.ndarray
    dvx: np.ndarray
    dvy: np.ndarray
    sigma: np.ndarray
    info: SolveInfo


def rhs(grid: Grid, h, vx, vy, sigma_guess, tol: float | None = None) -> RhsResult:
    """One evaluation of d/dt (h, v_x, v_y):
        b     = -div v
        sigma = GMRES(L_h, b; x0 = sigma_guess)
        dh    = -div(h v - grad sigma)
        B     = |v|^2/2 - |grad sigma|^2/(2 h^2) + g h - 9/2 sigma^2/h^4
        dv    = -grad B
    """
    cfg = grid.cfg
    tol = cfg.gmres_tol if tol is None else tol
    b = -(d_x(grid, vx) + d_y(grid, vy))
    sigma, info = gmres(grid, h, b, sigma_guess, tol, cfg.gmres_restart, cfg.gmres_max_iters)
    sx = d_x(grid, sigma)
    sy = d_y(grid, sigma)
    dh = -d_x(grid, h * vx - sx) - d_y(grid, h * vy - sy)
    B = 0.5 * (vx * vx + vy * vy) - (sx * sx + sy * sy) / (2.0 * h * h) + cfg.g * h \
        - 4.5 * sigma * sigma / h ** 4
    return RhsResult(dh=dh, dvx=-d_x(grid, B), dvy=-d_y(grid, B), sigma=sigma, info=info)


# ---------------------------------------------------------------------------
# Krasny filter (Section 3) and classical RK4 (Section 3)
# ---------------------------------------------------------------------------


def krasny(grid: Grid, f: np.ndarray, threshold: float) -> np.ndarray:
    """Set normalised 2D DFT coefficients with modulus below threshold to 0."""
    n = f.size
    c = np.fft.fft2(f) / n
    c[np.abs(c) < threshold] = 0.0
    return np.real(np.fft.ifft2(c * n))


def two_thirds(grid: Grid, f: np.ndarray) -> np.ndarray:
    """Orszag's two-thirds rule: keep the DFT modes with 3|m_x| <= nx and
    3|m_y| <= ny (signed indices m in [-N/2, N/2), the Nyquist index included
    in the discarded set), set the rest to zero."""
    ny, nx = f.shape
    mx = np.abs(np.fft.fftfreq(nx) * nx)
    my = np.abs(np.fft.fftfreq(ny) * ny)
    keep = (3 * my[:, None] <= ny) & (3 * mx[None, :] <= nx)
    c = np.fft.fft2(f)
    c[~keep] = 0.0
    return np.real(np.fft.ifft2(c))


@dataclasses.dataclass
class StepInfo:
    total_iters: int = 0
    max_iters_per_solve: int = 0
    solves: int = 0
    min_h: float = 0.0
    any_unconverged: bool = False
    stage_iters: list = dataclasses.field(default_factory=list)   # per solve, in order
    guess_dist: list = dataclasses.field(default_factory=list)    # max |sigma - guess| per solve


def rk4_step(grid: Grid, h, vx, vy, sigma, dt: float, info: StepInfo | None = None, incr=None):
    """One classical RK4 step of (h, v_x, v_y); sigma carries the warm start
    from one RHS evaluation to the next.  With Config.guess = 1, incr is the
    list of the four stage increments D_i (updated in place).  Returns
    (h, vx, vy, sigma)."""
    info = info if info is not None else StepInfo()
    y0 = (h, vx, vy)
    use_incr = grid.cfg.guess == 1 and incr is not None

    def ev(state, s, stage):
        guess = s + incr[stage] if use_incr else s
        r = rhs(grid, *state, guess)
        if use_incr:
            incr[stage] = incr[stage] + (r.sigma - guess)
        info.solves += 1
        info.total_iters += r.info.iters
        info.max_iters_per_solve = max(info.max_iters_per_solve, r.info.iters)
        info.any_unconverged |= not r.info.converged
        info.stage_iters.append(r.info.iters)
        info.guess_dist.append(float(np.max(np.abs(r.sigma - guess))))
        return (r.dh, r.dvx, r.dvy), r.sigma

    k1, s1 = ev(y0, sigma, 0)
    y1 = tuple(a + 0.5 * dt * k for a, k in zip(y0, k1))
    k2, s2 = ev(y1, s1, 1)
    y2 = tuple(a + 0.5 * dt * k for a, k in zip(y0, k2))
    k3, s3 = ev(y2, s2, 2)
    y3 = tuple(a + dt * k for a, k in zip(y0, k3))
    k4, s4 = ev(y3, s3, 3)
    out = tuple(a + dt / 6.0 * (q1 + 2.0 * q2 + 2.0 * q3 + q4)
                for a, q1, q2, q3, q4 in zip(y0, k1, k2, k3, k4))
    if grid.cfg.krasny > 0.0:
        out = tuple(krasny(grid, f, grid.cfg.krasny) for f in out)
    if grid.cfg.dealias:
        out = tuple(two_thirds(grid, f) for f in out)
    info.min_h = float(np.min(out[0]))
    return out[0], out[1], out[2], s4


def rk4(grid: Grid, h, vx, vy, sigma, dt: float, nsteps: int):
    """nsteps RK4 steps; returns (h, vx, vy, sigma, StepInfo)."""
    info = StepInfo()
    incr = [np.zeros_like(h) for _ in range(4)] if grid.cfg.guess == 1 else None
    for _ in range(nsteps):
        h, vx, vy, sigma = rk4_step(grid, h, vx, vy, sigma, dt, info, incr)
    return h, vx, vy, sigma, info


# ---------------------------------------------------------------------------
# Conserved quantities (Section 2.3) and monitors (Section 3, Section 4.2)
# ---------------------------------------------------------------------------


def invariants(grid: Grid, h, vx, vy, sigma_guess):
    """Mass, momentum and energy of Section 2.3 on the torus (the trapezoid
    rule, which is spectrally accurate for periodic data), with sigma solved
    tightly for the given state, plus min/max h, the L2 norm of curl v and the
    largest normalised DFT coefficient of h in the outer half of the spectrum.
    Returns (dict, sigma)."""
    cfg = grid.cfg
    b = -(d_x(grid, vx) + d_y(grid, vy))
    sigma, _ = gmres(grid, h, b, sigma_guess, cfg.invariants_tol, cfg.gmres_restart,
                     cfg.gmres_max_iters)
    dA = grid.dx * grid.dy
    sx = d_x(grid, sigma)
    sy = d_y(grid, sigma)
    ux = vx - sx / h
    uy = vy - sy / h
    mass = dA * float(np.sum(h - cfg.h_inf))
    px = dA * float(np.sum(h * ux))
    py = dA * float(np.sum(h * uy))
    energy = dA * float(np.sum(0.5 * h * (ux * ux + uy * uy) + 1.5 * sigma * sigma / h ** 3
                               + 0.5 * cfg.g * (h - cfg.h_inf) ** 2))
    curl = d_x(grid, vy) - d_y(grid, vx)
    curl_l2 = math.sqrt(dA * float(np.sum(curl * curl)))
    tail = spectral_tail(h)
    return dict(mass=mass, px=px, py=py, energy=energy, min_h=float(np.min(h)),
                max_h=float(np.max(h)), curl_l2=curl_l2, spectral_tail=tail), sigma


def spectral_tail(f: np.ndarray) -> float:
    """Largest |F f| / N over modes with |m_x| > nx/4 or |m_y| > ny/4 (the
    decay monitor of the DFT coefficients, Section 3)."""
    ny, nx = f.shape
    c = np.abs(np.fft.fft2(f)) / f.size
    mx = np.abs(np.fft.fftfreq(nx) * nx)
    my = np.abs(np.fft.fftfreq(ny) * ny)
    mask = (mx[None, :] > nx / 4) | (my[:, None] > ny / 4)
    return float(np.max(c[mask])) if np.any(mask) else 0.0
