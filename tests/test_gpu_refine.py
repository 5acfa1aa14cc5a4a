"""Mixed-precision iterative refinement of the elliptic solve against the FP64
oracle.

The residual b - L sigma is taken in FP64 and each correction is solved in the
mixed-precision mode (FP32 fields, GMRES tolerance 1e-6).  The refined sigma
must satisfy the FP64 equation to the requested tolerance: its residual,
recomputed by the oracle's operator, is below tol ||b|| (up to the oracle's own
rounding), and it agrees with the oracle's GMRES solution to within the
conditioning of the problem times tol.  A correction contracts the residual
by about the mixed mode's accuracy, so 1e-12 takes a few rounds, not one per
digit."""
import numpy as np
import pytest
import torch

from oracle import sgn_oracle as O
from paper_2306_09731_amd import sgn
from sgn_inputs import Box, perturbed_line_soliton, random_smooth_field

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)


def contexts(nx, ny, Lx, Ly, tol32=1e-6):
    c64 = sgn.sgn_init(sgn.config_default(nx, ny, Lx, Ly, gmres_tol=1e-12), DEV)
    c32 = sgn.sgn_init(sgn.config_default(nx, ny, Lx, Ly, gmres_tol=tol32, precision=sgn.SGN_FP32_MIXED), DEV)
    return c64, c32


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def problem(kind, nx, ny):
    if kind == "soliton":
        box = Box(nx, ny, 10.0 * nx / 1024, 5.0 * ny / 512)
        h, vx, vy, _ = perturbed_line_soliton(box, a=0.5, eps=0.01, k=2, x0=-0.5 * np.pi * box.Lx)
        g = O.Grid(O.Config(nx=nx, ny=ny, Lx=box.Lx, Ly=box.Ly, gmres_tol=1e-13))
        return box.Lx, box.Ly, h, -(O.d_x(g, vx) + O.d_y(g, vy)), g
    rng = np.random.default_rng(nx * 3 + ny)
    Lx, Ly = 2.0, 1.5
    h = 1.0 + 0.4 * random_smooth_field(rng, ny, nx, kmax=5)
    b = random_smooth_field(rng, ny, nx, kmax=7)
    return Lx, Ly, h, b, O.Grid(O.Config(nx=nx, ny=ny, Lx=Lx, Ly=Ly, gmres_tol=1e-13))


@pytest.mark.parametrize("kind,nx,ny", [("random", 64, 64), ("random", 256, 128), ("soliton", 1024, 512)])
def test_refined_solve_reaches_fp64_accuracy(kind, nx, ny):
    Lx, Ly, h, b, g = problem(kind, nx, ny)
    c64, c32 = contexts(nx, ny, Lx, Ly)
    sig = torch.zeros(ny, nx, dtype=torch.float64, device=DEV)
    tol = 1e-12
    info = sgn.sgn_elliptic_solve_refined(c64, c32, dev(h), dev(b), sig, tol, 8)
    torch.cuda.synchronize()
    s = sig.cpu().numpy()
    res = np.linalg.norm(b - O.apply_L(g, h, s)) / np.linalg.norm(b)
    ref, _ = O.gmres(g, h, b, np.zeros_like(b), 1e-13, 20, 400)
    e = np.abs(s - ref).max() / np.abs(ref).max()
    say(f"refined {kind} {nx}x{ny}: rounds {info.rounds}, inner iterations {info.inner_iters}, "
        f"residual {info.rel_resid_first:.1e} -> {info.rel_resid_true:.1e} (oracle {res:.1e}), "
        f"sigma error {e:.1e}")
    assert info.rel_resid_true <= tol and info.rel_resid_first == pytest.approx(1.0)
    assert 1 <= info.rounds <= 4
    assert res < 2 * tol
    assert e < 1e-10
    # the FP64 solve to the same tolerance lands on the same sigma
    s64 = torch.zeros_like(sig)
    sgn.sgn_elliptic_solve(c64, dev(h), dev(b), s64)
    torch.cuda.synchronize()
    e64 = np.abs(s - s64.cpu().numpy()).max() / np.abs(ref).max()
    say(f"  against the FP64 solve: {e64:.1e}")
    assert e64 < 1e-10


def test_refined_solve_from_the_solution_does_no_round():
    Lx, Ly, h, b, g = problem("random", 128, 64)
    c64, c32 = contexts(128, 64, Lx, Ly)
    ref, _ = O.gmres(g, h, b, np.zeros_like(b), 1e-13, 20, 400)
    sig = dev(ref)
    info = sgn.sgn_elliptic_solve_refined(c64, c32, dev(h), dev(b), sig, 1e-10, 4)
    torch.cuda.synchronize()
    say(f"refined from the solution: rounds {info.rounds}, residual {info.rel_resid_true:.1e}")
    assert info.rounds == 0 and info.inner_iters == 0 and info.rel_resid_true < 1e-10
    assert np.array_equal(sig.cpu().numpy(), ref)


def test_refined_solve_round_limit():
    """One round cannot reach 1e-13 from zero: the call reports the residual
    it reached after that round and leaves sigma at that iterate."""
    Lx, Ly, h, b, g = problem("random", 128, 128)
    c64, c32 = contexts(128, 128, Lx, Ly)
    sig = torch.zeros(128, 128, dtype=torch.float64, device=DEV)
    info = sgn.sgn_elliptic_solve_refined(c64, c32, dev(h), dev(b), sig, 1e-13, 1)
    torch.cuda.synchronize()
    res = np.linalg.norm(b - O.apply_L(g, h, sig.cpu().numpy())) / np.linalg.norm(b)
    say(f"one round: residual {info.rel_resid_true:.1e} (oracle {res:.1e})")
    assert info.rounds == 1 and info.rel_resid_true > 1e-13
    assert info.rel_resid_true == pytest.approx(res, rel=1e-6)
    assert res < 1e-4


def test_refined_solve_argument_errors():
    c64, c32 = contexts(64, 64, 2.0, 1.5)
    o64, _ = contexts(64, 64, 2.0, 1.5)
    _, w32 = contexts(64, 32, 2.0, 1.5)
    _, l32 = contexts(64, 64, 2.5, 1.5)
    z = torch.zeros(64, 64, dtype=torch.float64, device=DEV)
    h = torch.ones_like(z)
    for a, b_ in ((c64, o64), (c64, c64), (c64, w32), (c64, l32)):
        with pytest.raises(sgn.SgnError):
            sgn.sgn_elliptic_solve_refined(a, b_, h, z, z.clone(), 1e-10, 4)
    with pytest.raises(ValueError):  # FP32 fields where FP64 ones are expected
        sgn.sgn_elliptic_solve_refined(c64, c32, h.float(), z.float(), z.float(), 1e-10, 4)
    with pytest.raises(sgn.SgnError):
        sgn.sgn_elliptic_solve_refined(c64, c32, h, z, z.clone(), 0.0, 4)
    with pytest.raises(sgn.SgnError):
        sgn.sgn_elliptic_solve_refined(c64, c32, h, z, z.clone(), 1e-10, 0)


def test_refined_rk4_step_matches_oracle_and_fp64():
    """20 RK4 steps of a perturbed soliton on 256x128 with every stage solve
    refined to 1e-12 (FP32 GMRES corrections, FP64 residuals, FP64 fluxes and
    RK combine): against the oracle's 20 steps at GMRES tol 1e-12 and the FP64
    path's at the same tolerance, both within the FP64 parity gate 1e-10."""
    nx, ny = 256, 128
    box = Box(nx, ny, 10.0 * nx / 1024, 5.0 * ny / 512)
    h, vx, vy, s = perturbed_line_soliton(box, a=0.5, eps=0.01, k=2, x0=-0.5 * np.pi * box.Lx)
    c64, c32 = contexts(nx, ny, box.Lx, box.Ly)
    f = [dev(a) for a in (h, vx, vy, s)]
    info = sgn.sgn_rk4_step_refined(c64, c32, *f, 0.005, 20, 1e-12, 8)
    got = [t.cpu().numpy() for t in f]
    c64b = sgn.sgn_init(sgn.config_default(nx, ny, box.Lx, box.Ly, gmres_tol=1e-12), DEV)
    f64 = [dev(a) for a in (h, vx, vy, s)]
    sgn.sgn_rk4_step(c64b, *f64, 0.005, 20)
    ref64 = [t.cpu().numpy() for t in f64]
    g = O.Grid(O.Config(nx=nx, ny=ny, Lx=box.Lx, Ly=box.Ly, gmres_tol=1e-12))
    oh, ovx, ovy, _, _ = O.rk4(g, h, vx, vy, s, 0.005, 20)
    eh = np.abs(got[0] - oh).max() / np.abs(oh - 1.0).max()
    ev = np.abs(got[1] - ovx).max() / np.abs(ovx).max()
    e64 = max(np.abs(got[0] - ref64[0]).max() / np.abs(ref64[0] - 1.0).max(),
              np.abs(got[1] - ref64[1]).max() / np.abs(ref64[1]).max())
    say(f"refined rk4 x20 256x128: rounds {info.rounds} over {info.solves} solves "
        f"(max {info.max_rounds_per_solve}), FP32 iterations {info.inner_iters}, worst residual "
        f"{info.max_rel_resid:.1e}; vs oracle h {eh:.1e} vx {ev:.1e}; vs FP64 path {e64:.1e}")
    assert info.solves == 80 and info.max_rel_resid <= 1e-12
    assert eh < 1e-10 and ev < 1e-10 and e64 < 1e-10
