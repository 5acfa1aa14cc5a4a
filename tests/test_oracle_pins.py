"""Pins of the FP64 oracle against facts that do not come from the oracle:
naive DFTs, Trefethen's closed-form periodic differentiation matrix, dense
direct solves, the exact solitary wave of the paper, the linear dispersion
relation, the RK4 stability polynomial, closed-form invariants and the
numbers printed in the paper (tests/golden/)."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import sgn_oracle as O
from sgn_inputs import Box, line_soliton, soliton_params, soliton_profile, random_state

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.json")


def grid(nx, ny, Lx, Ly, **kw):
    return O.Grid(O.Config(nx=nx, ny=ny, Lx=Lx, Ly=Ly, **kw))


def naive_dft(f):
    n = f.shape[-1]
    j = np.arange(n)
    W = np.exp(-2j * np.pi * np.outer(j, j) / n)
    return f @ W.T


# --- transforms and derivatives -------------------------------------------------


@pytest.mark.parametrize("n", [2, 8, 16, 64, 256])
def test_fft_primitive_matches_naive_dft(n):
    rng = np.random.default_rng(n)
    f = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    ref = naive_dft(f)
    np.testing.assert_allclose(np.fft.fft(f, axis=1), ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    np.testing.assert_allclose(np.fft.ifft(np.fft.fft(f, axis=1), axis=1), f, atol=1e-14 * n)


def trefethen_D(n, L):
    """Periodic spectral differentiation matrix (Trefethen, Spectral Methods in
    MATLAB, ch. 3), n even, on a period 2 pi L:  D_ij = 1/2 (-1)^(i-j) cot((i-j) h / 2) / L."""
    h = 2 * np.pi / n
    i = np.arange(n)
    d = i[:, None] - i[None, :]
    with np.errstate(divide="ignore"):
        D = 0.5 * (-1.0) ** d / np.tan(d * h / 2)
    D[d == 0] = 0.0
    return D / L


@pytest.mark.parametrize("nx,ny,Lx,Ly", [(16, 8, 1.0, 2.0), (32, 64, 3.0, 0.7), (8, 8, 1.0, 1.0)])
def test_derivatives_match_trefethen_matrix(nx, ny, Lx, Ly):
    g = grid(nx, ny, Lx, Ly)
    rng = np.random.default_rng(1)
    f = rng.standard_normal((ny, nx))
    np.testing.assert_allclose(O.d_x(g, f), f @ trefethen_D(nx, Lx).T, atol=1e-12)
    np.testing.assert_allclose(O.d_y(g, f), trefethen_D(ny, Ly) @ f, atol=1e-12)


def test_derivatives_exact_on_trig_polynomials():
    g = grid(64, 32, 2.0, 1.5)
    X, Y = np.meshgrid(g.x, g.y)
    f = np.zeros_like(X)
    fx = np.zeros_like(X)
    fy = np.zeros_like(X)
    rng = np.random.default_rng(7)
    for mx in range(0, 31):
        for my in range(-15, 16):
            a, b = rng.standard_normal(2)
            kx, ky = mx / 2.0, my / 1.5
            ph = kx * X + ky * Y
            f += a * np.cos(ph) + b * np.sin(ph)
            fx += kx * (-a * np.sin(ph) + b * np.cos(ph))
            fy += ky * (-a * np.sin(ph) + b * np.cos(ph))
    scale = np.abs(fx).max()
    assert np.abs(O.d_x(g, f) - fx).max() < 1e-12 * scale
    assert np.abs(O.d_y(g, f) - fy).max() < 1e-12 * np.abs(fy).max()


def test_nyquist_mode_has_zero_derivative():
    g = grid(16, 8, 1.0, 1.0)
    X, Y = np.meshgrid(g.x, g.y)
    f = np.cos(8 * X) + np.cos(4 * Y)   # Nyquist in x and in y
    assert np.abs(O.d_x(g, f)).max() < 1e-13
    assert np.abs(O.d_y(g, f)).max() < 1e-13


# --- elliptic operator, preconditioner, GMRES ------------------------------------


def dense(op, ny, nx):
    n = nx * ny
    A = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        A[:, i] = op(e.reshape(ny, nx)).ravel()
    return A


def test_L_dense_is_spd_and_equals_M_at_h1():
    g = grid(16, 16, 1.3, 0.9)
    rng = np.random.default_rng(3)
    h = 1.0 + 0.4 * np.cos(g.x)[None, :] * np.sin(2 * g.y)[:, None] + 0.1 * rng.random((16, 16))
    A = dense(lambda s: O.apply_L(g, h, s), 16, 16)
    np.testing.assert_allclose(A, A.T, atol=1e-12 * np.abs(A).max())
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0
    # h = 1: M^-1 L = I
    one = np.ones((16, 16))
    P = dense(lambda s: O.apply_Minv(g, O.apply_L(g, one, s)), 16, 16)
    np.testing.assert_allclose(P, np.eye(256), atol=1e-12)


def test_constant_depth_closed_form():
    g = grid(32, 16, 1.0, 2.0)
    h0 = 1.7
    rng = np.random.default_rng(4)
    b = rng.standard_normal((16, 32))
    KX, KY = np.meshgrid(g.kx, g.ky)
    s_exact = np.real(np.fft.ifft2(np.fft.fft2(b) / (3 / h0 ** 3 + (KX ** 2 + KY ** 2) / h0)))
    s, info = O.gmres(g, np.full((16, 32), h0), b, np.zeros_like(b), 1e-13, 20, 200)
    assert info.converged
    assert np.abs(s - s_exact).max() < 1e-11 * np.abs(s_exact).max()


def test_gmres_matches_dense_solve_16x16():
    g = grid(16, 16, 1.0, 1.0)
    rng = np.random.default_rng(5)
    h, _, _, _ = random_state(rng, Box(16, 16, 1.0, 1.0), amp_h=0.4)
    b = rng.standard_normal((16, 16))
    A = dense(lambda s: O.apply_L(g, h, s), 16, 16)
    s_ref = np.linalg.solve(A, b.ravel()).reshape(16, 16)
    s, info = O.gmres(g, h, b, np.zeros_like(b), 1e-13, 20, 400)
    assert info.converged and info.rel_resid_true < 1e-11
    assert np.abs(s - s_ref).max() < 1e-10 * np.abs(s_ref).max()
    # restarts give the same answer
    s2, info2 = O.gmres(g, h, b, np.zeros_like(b), 1e-13, 4, 400)
    assert info2.restarts > 0 and info2.converged
    assert np.abs(s2 - s_ref).max() < 1e-10 * np.abs(s_ref).max()


def test_gmres_arnoldi_relation_orthonormality_monotone_residual():
    """Within a cycle: M^-1 L V_k = V_{k+1} Hbar_k (the Arnoldi relation), the
    basis is orthonormal while the residual is far from round-off (modified
    Gram-Schmidt loses orthogonality in inverse proportion to the relative
    residual, the result of Paige, Rozloznik and Strakos, so only the vectors
    built while the residual estimate is above 1e-6 are held to 1e-9), and the
    residual estimate never grows (GMRES minimises it over a growing
    subspace)."""
    g = grid(16, 16, 1.0, 1.0)
    rng = np.random.default_rng(12)
    h, _, _, _ = random_state(rng, Box(16, 16, 1.0, 1.0), amp_h=0.5)
    b = rng.standard_normal((16, 16))
    rec = {}
    s, info = O.gmres(g, h, b, np.zeros_like(b), 1e-13, 30, 400, record=rec)
    assert info.converged and info.restarts == 0
    V = np.stack([v.ravel() for v in rec["V"]], axis=1)
    Hbar = rec["Hbar"]
    k = Hbar.shape[1]
    assert k == info.iters and V.shape[1] >= k
    AV = np.stack([O.apply_Minv(g, O.apply_L(g, h, rec["V"][j])).ravel() for j in range(k - 1)], axis=1)
    lhs, rhs_ = AV, V[:, :k] @ Hbar[:k, :k - 1]
    assert np.abs(lhs - rhs_).max() < 1e-12 * np.abs(lhs).max()
    r = np.array(rec["resid"])
    q = int(np.argmax(r < 1e-6)) + 1          # vectors V_0..V_q built while r >= 1e-6
    Vq = V[:, :q + 1]
    assert np.abs(Vq.T @ Vq - np.eye(q + 1)).max() < 1e-9
    assert len(r) == k and np.all(r[1:] <= r[:-1] * (1 + 1e-12))
    assert r[-1] <= 1e-13 and abs(r[-1] - info.rel_resid_precond) < 1e-12


def test_gmres_one_iteration_at_unit_depth_and_zero_rhs():
    g = grid(32, 16, 1.0, 1.0)
    rng = np.random.default_rng(6)
    b = rng.standard_normal((16, 32))
    s, info = O.gmres(g, np.ones((16, 32)), b, np.zeros_like(b), 1e-12, 20, 200)
    assert info.iters == 1 and info.converged
    s, info = O.gmres(g, np.ones((16, 32)), np.zeros_like(b), b, 1e-12, 20, 200)
    assert info.converged and info.iters == 0 and np.all(s == 0)


def test_gmres_not_converged_flag():
    g = grid(16, 16, 1.0, 1.0)
    rng = np.random.default_rng(8)
    h, _, _, _ = random_state(rng, Box(16, 16, 1.0, 1.0), amp_h=0.5)
    b = rng.standard_normal((16, 16))
    s, info = O.gmres(g, h, b, np.zeros_like(b), 1e-14, 20, 1)
    assert not info.converged and info.iters == 1


def soliton_grid(nx=256, ny=8, Lx=10.0, Ly=1.0, **kw):
    return grid(nx, ny, Lx, Ly, **kw), Box(nx, ny, Lx, Ly)


def test_elliptic_solve_reproduces_soliton_sigma():
    g, box = soliton_grid()
    h, vx, vy, sig = line_soliton(box, a=0.5)
    b = -(O.d_x(g, vx) + O.d_y(g, vy))
    s, info = O.gmres(g, h, b, np.zeros_like(h), 1e-13, 20, 200)
    assert info.converged
    assert np.abs(s - sig).max() < 1e-12 * np.abs(sig).max()


def test_vector_form_identity():
    """u = v - grad(sigma)/h satisfies h u - 1/3 grad(h^3 div u) = h v (eq. K_1)."""
    g = grid(64, 64, 2.0, 2.0)
    rng = np.random.default_rng(9)
    h, vx, vy, _ = random_state(rng, Box(64, 64, 2.0, 2.0), amp_h=0.3, kmax=4)
    b = -(O.d_x(g, vx) + O.d_y(g, vy))
    s, info = O.gmres(g, h, b, np.zeros_like(h), 1e-13, 30, 400)
    ux = vx - O.d_x(g, s) / h
    uy = vy - O.d_y(g, s) / h
    divu = O.d_x(g, ux) + O.d_y(g, uy)
    # sigma = -h^3 div(u) / 3
    assert np.abs(s + h ** 3 * divu / 3).max() < 1e-9
    lhs_x = h * ux - O.d_x(g, h ** 3 * divu) / 3
    lhs_y = h * uy - O.d_y(g, h ** 3 * divu) / 3
    assert np.abs(lhs_x - h * vx).max() < 1e-8
    assert np.abs(lhs_y - h * vy).max() < 1e-8


# --- right-hand side ---------------------------------------------------------------


def test_rhs_is_translation_at_exact_soliton():
    """A travelling wave satisfies d/dt f = -c f_x; derivatives taken analytically."""
    g, box = soliton_grid(gmres_tol=1e-13)
    a = 0.5
    p = soliton_params(a=a)
    h, vx, vy, sig = line_soliton(box, a=a)
    X, _ = box.mesh()
    prof = soliton_profile(X, p)
    r = O.rhs(g, h, vx, vy, np.zeros_like(h))
    assert r.info.converged
    assert np.abs(r.dh - (-p.c * prof["h1"])).max() < 1e-11
    assert np.abs(r.dvx - (-p.c * prof["v1"])).max() < 1e-11
    assert np.abs(r.dvy).max() < 1e-12
    assert np.abs(r.sigma - sig).max() < 1e-12


def _linear_wave(eps, m=3, L=1.0, n=32):
    g = grid(n, 4, L, 1.0, gmres_tol=1e-13)
    k = m / L
    X, _ = np.meshgrid(g.x, g.y)
    h = 1.0 + eps * np.cos(k * X)
    z = np.zeros_like(h)
    omega = math.sqrt(k * k / (1.0 + k * k / 3.0))
    return g, h, z, k, X, omega


def test_linear_dispersion_relation():
    """Linearising eqs. (1)-(3) about h = 1, v = 0 gives omega^2 = g h k^2 / (1 + h^2 k^2 / 3)."""
    eps = 1e-7
    g, h, z, k, X, omega = _linear_wave(eps)
    dt, n = 0.01, 100
    hh, vx, vy, s, _ = O.rk4(g, h, z, z.copy(), z.copy(), dt, n)
    exact = eps * np.cos(k * X) * math.cos(omega * dt * n)
    assert np.abs((hh - 1.0) - exact).max() < 1e-6 * eps


def test_rk4_amplification_polynomial():
    """RK4 on the linear mode multiplies the complex amplitude by
    R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24, z = i omega dt, per step."""
    eps = 1e-8
    g, h, z, k, X, omega = _linear_wave(eps)
    dt, n = 0.4, 12
    zz = 1j * omega * dt
    R = 1 + zz + zz ** 2 / 2 + zz ** 3 / 6 + zz ** 4 / 24
    hh, *_ = O.rk4(g, h, z, z.copy(), z.copy(), dt, n)
    pred = eps * np.cos(k * X) * np.real(R ** n)
    exact = eps * np.cos(k * X) * math.cos(omega * dt * n)
    assert np.abs((hh - 1.0) - pred).max() < 1e-5 * eps
    assert np.abs(pred - exact).max() > 1e-4 * eps      # the pin discriminates
    # dt halving: fourth order gives a ratio near 16 (third order would give ~8);
    # the max over x at one time mixes phase and amplitude error, hence the band
    errs = []
    for dt_, n_ in ((0.2, 20), (0.1, 40)):
        hh, *_ = O.rk4(g, h, z, z.copy(), z.copy(), dt_, n_)
        errs.append(np.abs((hh - 1.0) - eps * np.cos(k * X) * math.cos(omega * dt_ * n_)).max())
    assert 12 < errs[0] / errs[1] < 32


# --- Krasny filter --------------------------------------------------------------


def test_krasny_filter_removes_only_small_modes():
    g = grid(32, 16, 1.0, 1.0, krasny=1e-12)
    X, Y = np.meshgrid(g.x, g.y)
    keep = 1.0 + 0.5 * np.cos(Y) + 1e-11 * np.sin(2 * X)
    f = keep + 1e-12 * np.cos(3 * X + Y)   # normalised coefficients 5e-13 < 1e-12
    out = O.krasny(g, f, 1e-12)
    assert np.abs(out - keep).max() < 1e-15
    nyq = 1.0 + 1e-13 * np.cos(16 * X)     # Nyquist mode, coefficient 1e-13
    assert np.abs(O.krasny(g, nyq, 1e-12) - 1.0).max() < 1e-15


def _soliton_guess_run(guess, dt, nsteps, tol=1e-12):
    from sgn_inputs import Box, line_soliton
    box = Box(256, 16, 10.0, 1.0)
    g = grid(box.nx, box.ny, box.Lx, box.Ly, gmres_tol=tol, guess=guess)
    h, vx, vy, s = line_soliton(box, a=0.5, x0=0.0)
    return O.rk4(g, h, vx, vy, s, dt, nsteps)


def test_stage_increment_guess_is_second_order_and_leaves_the_solution():
    """The stage-increment guess predicts each stage's sigma to O(dt^2) (the
    increment of a stage changes by O(dt) per step), where the plain warm start
    is O(dt) off for the half- and full-step stages; the converged states are
    the same up to the GMRES tolerance, and the first step is identical."""
    dist = {}
    for guess in (0, 1):
        for dt in (0.02, 0.01):
            n = int(round(0.08 / dt))
            h, vx, vy, s, info = _soliton_guess_run(guess, dt, n)
            # stages of the last step
            dist[guess, dt] = np.array(info.guess_dist[-4:])
            if dt == 0.01:
                final = (h, vx)
                if guess == 0:
                    plain, plain_iters = final, info.stage_iters
                else:
                    assert info.stage_iters[:4] == plain_iters[:4]       # first step: same guesses
                    assert sum(info.stage_iters) < sum(plain_iters)      # fewer iterations overall
                    for a, b in zip(final, plain):
                        assert np.abs(a - b).max() < 1e-9
    r0 = dist[0, 0.01] / dist[0, 0.02]
    r1 = dist[1, 0.01] / dist[1, 0.02]
    # plain: stages 2 and 4 first order (ratio ~1/2)
    assert 0.4 < r0[1] < 0.6 and 0.4 < r0[3] < 0.6
    # increment guess: every stage at least second order (ratio <= ~1/4)
    assert np.all(r1 < 0.3), r1
    assert np.all(dist[1, 0.01] < dist[0, 0.01])


def test_two_thirds_rule_keeps_exactly_the_inner_band():
    # nx = 32: |m_x| <= 10 kept, 11 dropped; ny = 16: |m_y| <= 5 kept, 6 dropped.
    g = grid(32, 16, 1.0, 1.0)
    X, Y = np.meshgrid(g.x, g.y)
    kept = 0.7 + np.cos(10 * X + 5 * Y) + 0.3 * np.sin(10 * X - 5 * Y) + 0.2 * np.cos(3 * X)
    dropped = (0.5 * np.cos(11 * X) + 0.4 * np.sin(2 * X + 6 * Y) + 0.3 * np.cos(16 * X)
               + 0.2 * np.cos(8 * Y) + 0.1 * np.cos(16 * X + 8 * Y))
    out = O.two_thirds(g, kept + dropped)
    assert np.abs(out - kept).max() < 1e-14
    assert np.abs(O.two_thirds(g, dropped)).max() < 1e-14


# --- invariants -----------------------------------------------------------------


def test_invariants_closed_forms():
    g = grid(64, 32, 2.0, 1.0)
    X, Y = np.meshgrid(g.x, g.y)
    area = (2 * np.pi * 2.0) * (2 * np.pi * 1.0)
    eps = 0.1
    h = 1.2 + eps * np.cos(X)
    vx = 0.3 * np.sin(Y)
    z = np.zeros_like(h)
    inv, s = O.invariants(g, h, vx, z, z)
    assert abs(inv["mass"] - 0.2 * area) < 1e-12 * area
    assert abs(inv["curl_l2"] - math.sqrt(0.09 * area / 2)) < 1e-12
    assert abs(inv["max_h"] - 1.3) < 1e-15 and abs(inv["min_h"] - 1.1) < 1e-15
    # v with zero divergence -> sigma = 0, u = v
    assert np.abs(s).max() < 1e-14
    E = area * (0.5 * 0.04 + 0.5 * eps ** 2 / 2) + 0.5 * 0.09 * (area * 1.2 / 2)
    assert abs(inv["energy"] - E) < 1e-12 * E
    # spectral tail: a mode beyond nx/4 with amplitude 1e-3 -> coefficient 5e-4
    inv2, _ = O.invariants(g, 1.0 + 1e-3 * np.cos(20 * X), z, z, z)
    assert abs(inv2["spectral_tail"] - 5e-4) < 1e-15


def test_soliton_invariants_match_quadrature():
    """Mass, momentum and energy of the exact soliton vs adaptive quadrature of
    the analytic integrands (independent of the spectral machinery)."""
    g, box = soliton_grid(nx=512, ny=4, Lx=10.0, Ly=1.0)
    a = 0.5
    p = soliton_params(a=a)
    h, vx, vy, sig = line_soliton(box, a=a)
    inv, s = O.invariants(g, h, vx, vy, sig)
    Py = 2 * np.pi * 1.0

    def dens(x, what):
        pr = soliton_profile(np.array([x]), p)
        hh, u, sg = pr["h"][0], pr["u"][0], pr["sigma"][0]
        if what == "mass":
            return hh - 1.0
        if what == "mom":
            return hh * u
        return 0.5 * hh * u * u + 1.5 * sg * sg / hh ** 3 + 0.5 * (hh - 1.0) ** 2

    lim = np.pi * 10.0
    for key, what in (("mass", "mass"), ("px", "mom"), ("energy", "en")):
        q, _ = integrate.quad(dens, -lim, lim, args=(what,), epsabs=1e-14, epsrel=1e-13, limit=400)
        assert abs(inv[key] - q * Py) < 1e-10 * abs(q * Py), key
    assert abs(inv["mass"] - Py * 2 * a / p.kappa) < 1e-9
    assert abs(inv["px"] - p.c * inv["mass"]) < 1e-10


def test_y_soliton_momentum_matches_quadrature():
    """The y-momentum of Section 2.3 on a solitary wave travelling along y:
    P_y = integral of h u_y equals adaptive quadrature of the analytic h u
    and c times the mass (the travelling-wave flux relation of Section 2.4),
    while P_x vanishes.  A momentum that used u_x, or v_y - h d_y sigma, or
    that dropped the factor h, misses these values by O(1)."""
    g, _ = soliton_grid(nx=4, ny=512, Lx=1.0, Ly=10.0)
    box = Box(4, 512, 1.0, 10.0)
    a = 0.5
    p = soliton_params(a=a)
    h, vx, vy, sig = line_soliton(box, a=a, along="y")
    inv, _ = O.invariants(g, h, vx, vy, sig)
    Px = 2 * np.pi * 1.0

    def hu(y):
        pr = soliton_profile(np.array([y]), p)
        return pr["h"][0] * pr["u"][0]

    lim = np.pi * 10.0
    q, _ = integrate.quad(hu, -lim, lim, epsabs=1e-14, epsrel=1e-13, limit=400)
    assert abs(inv["py"] - q * Px) < 1e-10 * abs(q * Px)
    assert abs(inv["py"] - p.c * inv["mass"]) < 1e-10
    assert abs(inv["px"]) < 1e-13


def test_momentum_components_swap_under_transpose():
    """On a square torus, exchanging x and y (and v_x with v_y) exchanges P_x
    and P_y and leaves the scalars unchanged; the random state has P_x and
    P_y of different size, so a P_y built from x-quantities fails."""
    g = grid(32, 32, 1.5, 1.5, invariants_tol=1e-14)
    rng = np.random.default_rng(13)
    h, vx, vy, s0 = random_state(rng, Box(32, 32, 1.5, 1.5), amp_h=0.2, amp_v=0.3, kmax=4)
    vx = vx + 0.2
    vy = vy - 0.1
    a, _ = O.invariants(g, h, vx, vy, s0)
    b, _ = O.invariants(g, h.T.copy(), vy.T.copy(), vx.T.copy(), s0.T.copy())
    assert abs(a["px"] - a["py"]) > 0.1 * abs(a["px"])
    assert abs(a["py"] - b["px"]) < 1e-12 * abs(a["py"])
    assert abs(a["px"] - b["py"]) < 1e-12 * abs(a["px"])
    for key in ("mass", "energy", "curl_l2", "min_h", "max_h"):
        assert abs(a[key] - b[key]) <= 1e-12 * max(1.0, abs(a[key])), key


# --- whole steps -----------------------------------------------------------------


def test_line_soliton_128x64_translation_mass_energy():
    """The 128x64 correctness workload: line soliton a = 0.5 on [-10pi,10pi]x[-5pi,5pi],
    dt = 0.01, 200 steps, GMRES tol 1e-10, restart 20."""
    cfg = O.Config(nx=128, ny=64, Lx=10.0, Ly=5.0, gmres_tol=1e-10, gmres_restart=20,
                   gmres_max_iters=200)
    g = O.Grid(cfg)
    box = Box(128, 64, 10.0, 5.0)
    a = 0.5
    p = soliton_params(a=a)
    h, vx, vy, sig = line_soliton(box, a=a)
    inv0, _ = O.invariants(g, h, vx, vy, sig)
    hh, vvx, vvy, s, info = O.rk4(g, h, vx, vy, sig, 0.01, 200)
    assert not info.any_unconverged
    t = 2.0
    h_exact, *_ = line_soliton(box, a=a, x0=p.c * t)
    # 128 points on 20 pi leave the sech^2 tail at ~1e-7 of the amplitude
    assert np.abs(hh - h_exact).max() < 1e-6
    assert np.abs(vvy).max() < 1e-12 and np.abs(hh - hh[:1, :]).max() < 1e-12
    inv1, _ = O.invariants(g, hh, vvx, vvy, s)
    assert abs(inv1["mass"] - inv0["mass"]) < 1e-12 * abs(inv0["mass"])
    assert abs(inv1["energy"] - inv0["energy"]) < 1e-9 * abs(inv0["energy"])


def test_paper_exact_soliton_energy_conservation():
    """Section 3: the exact c = 1.7 line soliton conserves energy to ~1e-14
    (Lx = 10, Ly = 2, dt = 1e-3).  Run at nx = 512 (spectral tail ~1e-12; the
    data are y-independent so ny = 4 suffices) for 100 steps."""
    ref = json.load(open(GOLDEN))["exact_line_soliton_energy_conservation"]
    st = ref["setup"]
    cfg = O.Config(nx=512, ny=4, Lx=st["Lx"], Ly=st["Ly"], gmres_tol=1e-12)
    g = O.Grid(cfg)
    box = Box(512, 4, st["Lx"], st["Ly"])
    p = soliton_params(c=st["c"])
    h, vx, vy, sig = line_soliton(box, a=p.a)
    inv0, _ = O.invariants(g, h, vx, vy, sig)
    hh, vvx, vvy, s, info = O.rk4(g, h, vx, vy, sig, st["t_end"] / st["nt"], 100)
    inv1, _ = O.invariants(g, hh, vvx, vvy, s)
    drift = abs(inv1["energy"] - inv0["energy"]) / abs(inv0["energy"])
    assert drift < 10 * ref["value"]
    h_exact, *_ = line_soliton(box, a=p.a, x0=p.c * 0.1)
    assert np.abs(hh - h_exact).max() < 1e-10


def test_transpose_symmetry_square_grid():
    """On a square torus, swapping x and y (and v_x with v_y) commutes with a step."""
    g = grid(32, 32, 1.5, 1.5, gmres_tol=1e-13)
    rng = np.random.default_rng(11)
    h, vx, vy, s0 = random_state(rng, Box(32, 32, 1.5, 1.5), amp_h=0.2, amp_v=0.1, kmax=4)
    a = O.rk4_step(g, h, vx, vy, s0, 0.01)
    b = O.rk4_step(g, h.T.copy(), vy.T.copy(), vx.T.copy(), s0.T.copy(), 0.01)
    assert np.abs(a[0] - b[0].T).max() < 1e-12
    assert np.abs(a[1] - b[2].T).max() < 1e-12
    assert np.abs(a[2] - b[1].T).max() < 1e-12


def test_discrete_curl_preserved():
    g = grid(32, 32, 1.0, 1.0, gmres_tol=1e-13)
    rng = np.random.default_rng(12)
    h, vx, vy, s0 = random_state(rng, Box(32, 32, 1.0, 1.0), amp_h=0.2, amp_v=0.1, kmax=4)
    curl0 = O.d_x(g, vy) - O.d_y(g, vx)
    hh, vvx, vvy, s, _ = O.rk4(g, h, vx, vy, s0, 0.01, 5)
    curl1 = O.d_x(g, vvy) - O.d_y(g, vvx)
    assert np.abs(curl1 - curl0).max() < 1e-12
