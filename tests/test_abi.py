"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every symbol include/sgn.h declares, and rejects bad arguments on the host
before any HIP call."""
import ctypes
import os
import re

import pytest

from paper_2306_09731_amd import sgn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sgn.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sgn_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = sgn.load_library()
    names = declared_functions()
    assert "sgn_init" in names and "sgn_rk4_step" in names and len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(sgn._SIGNATURES), set(names) - set(sgn._SIGNATURES)


def test_status_strings():
    lib = sgn.load_library()
    assert lib.sgn_status_string(0) == b"ok"
    assert b"converge" in lib.sgn_status_string(sgn.SGN_ERR_NOT_CONVERGED)
    assert lib.sgn_status_string(99) == b"unknown status"


def test_config_default_and_struct_layout():
    cfg = sgn.config_default(128, 64, 10.0, 5.0)
    assert (cfg.nx, cfg.ny, cfg.Lx, cfg.Ly) == (128, 64, 10.0, 5.0)
    assert cfg.g == 1.0 and cfg.h_inf == 1.0 and cfg.gmres_restart == 20
    assert cfg.gmres_tol == 1e-10 and cfg.gmres_max_iters == 200 and cfg.batch == 1
    assert cfg.krasny == 0.0 and cfg.dealias == 0 and cfg.guess == sgn.SGN_GUESS_PREVIOUS
    assert ctypes.sizeof(sgn.sgn_config) == 88


@pytest.mark.parametrize("field,value", [
    ("nx", 100), ("ny", 4), ("nx", 8192), ("gmres_restart", 65), ("precision", 2), ("batch", 0),
    ("batch", 65),
])
def test_workspace_bytes_rejects_unsupported(field, value):
    cfg = sgn.config_default(128, 64, 10.0, 5.0)
    setattr(cfg, field, value)
    assert sgn.sgn_workspace_bytes(cfg) == 0
    lib = sgn.load_library()
    h = ctypes.c_void_p()
    assert lib.sgn_init(ctypes.byref(cfg), ctypes.c_void_p(256), 1 << 30, None, ctypes.byref(h)) \
        == sgn.SGN_ERR_UNSUPPORTED


@pytest.mark.parametrize("field,value", [
    ("Lx", 0.0), ("Ly", -1.0), ("gmres_tol", 0.0), ("gmres_max_iters", 0), ("h_inf", 0.0),
    ("krasny", -1.0), ("gmres_restart", 0), ("Lx", float("nan")), ("dealias", 2), ("guess", 2), ("guess", -1),
])
def test_invalid_config(field, value):
    cfg = sgn.config_default(128, 64, 10.0, 5.0)
    setattr(cfg, field, value)
    assert sgn.sgn_workspace_bytes(cfg) == 0
    lib = sgn.load_library()
    h = ctypes.c_void_p()
    assert lib.sgn_init(ctypes.byref(cfg), ctypes.c_void_p(256), 1 << 30, None, ctypes.byref(h)) \
        == sgn.SGN_ERR_INVALID_ARG


def test_workspace_fp32_mode_halves_the_fields():
    a = sgn.sgn_workspace_bytes(sgn.config_default(256, 128, 10.0, 5.0))
    b = sgn.sgn_workspace_bytes(sgn.config_default(256, 128, 10.0, 5.0, precision=sgn.SGN_FP32_MIXED))
    nfields = 21 + 15 + 6  # basis, working fields, checkpoint of captured steps (h, vx, vy, SIG, E, G)
    # FP32 fields are half as large (both twiddle tables exist in either mode)
    assert a - b == nfields * 256 * 128 * 4


def test_workspace_stage_increment_guess_adds_eight_fields():
    # the four stage increments and their copies in the checkpoint of captured steps
    a = sgn.sgn_workspace_bytes(sgn.config_default(128, 64, 10.0, 5.0))
    b = sgn.sgn_workspace_bytes(sgn.config_default(128, 64, 10.0, 5.0, guess=sgn.SGN_GUESS_STAGE_INCREMENT))
    field = 128 * 64 * 8
    assert b - a == 8 * field


def test_workspace_size_scales_with_grid_and_restart():
    a = sgn.sgn_workspace_bytes(sgn.config_default(128, 64, 10.0, 5.0))
    b = sgn.sgn_workspace_bytes(sgn.config_default(256, 64, 10.0, 5.0))
    c = sgn.sgn_workspace_bytes(sgn.config_default(128, 64, 10.0, 5.0, gmres_restart=40))
    field = 128 * 64 * 8
    # Krylov basis: restart + 1 fields, plus 15 working fields and a 6-field checkpoint
    assert a >= 40 * field and b > a and c - a == 20 * field


def test_init_rejects_bad_workspace_without_gpu():
    lib = sgn.load_library()
    cfg = sgn.config_default(128, 64, 10.0, 5.0)
    need = sgn.sgn_workspace_bytes(cfg)
    h = ctypes.c_void_p()
    # null, misaligned, too small: all rejected on the host
    assert lib.sgn_init(ctypes.byref(cfg), None, need, None, ctypes.byref(h)) == sgn.SGN_ERR_INVALID_ARG
    assert lib.sgn_init(ctypes.byref(cfg), ctypes.c_void_p(4096 + 8), need, None, ctypes.byref(h)) \
        == sgn.SGN_ERR_INVALID_ARG
    assert lib.sgn_init(ctypes.byref(cfg), ctypes.c_void_p(4096), need - 1, None, ctypes.byref(h)) \
        == sgn.SGN_ERR_INVALID_ARG
    assert lib.sgn_init(None, ctypes.c_void_p(4096), need, None, ctypes.byref(h)) == sgn.SGN_ERR_INVALID_ARG


def test_calls_reject_null_context():
    lib = sgn.load_library()
    assert lib.sgn_rk4_step(None, None, None, None, None, 0.01, 1, None) == sgn.SGN_ERR_INVALID_ARG
    assert lib.sgn_rhs(None, None, None, None, None, None, None, None, None) == sgn.SGN_ERR_INVALID_ARG
    assert lib.sgn_elliptic_solve(None, None, None, None, None) == sgn.SGN_ERR_INVALID_ARG
    assert lib.sgn_invariants(None, None, None, None, None, None) == sgn.SGN_ERR_INVALID_ARG
    assert lib.sgn_destroy(None) == sgn.SGN_ERR_INVALID_ARG
    # no context: the message of this thread's last context-free failure
    assert isinstance(lib.sgn_last_error(None), bytes)


def test_ensemble_and_autotune_host_checks():
    lib = sgn.load_library()
    null = ctypes.POINTER(ctypes.c_void_p)()
    dts = (ctypes.c_double * 1)(0.01)
    assert lib.sgn_rk4_step_ensemble(-1, null, null, null, null, null, dts, 1, None) == sgn.SGN_ERR_INVALID_ARG
    assert lib.sgn_rk4_step_ensemble(1, null, null, null, null, null, dts, 1, None) == sgn.SGN_ERR_INVALID_ARG
    assert lib.sgn_rk4_step_ensemble(0, null, null, null, null, null, None, 1, None) == sgn.SGN_OK
    for fn in (lib.sgn_rk4_step_ensemble, lib.sgn_rk4_step_ensemble_graph):
        assert fn(-1, null, null, null, null, null, dts, 1, None) == sgn.SGN_ERR_INVALID_ARG
        assert fn(1, null, null, null, null, null, dts, 1, None) == sgn.SGN_ERR_INVALID_ARG
        assert fn(0, null, null, null, null, null, None, 1, None) == sgn.SGN_OK
    assert lib.sgn_autotune(None, None) == sgn.SGN_ERR_INVALID_ARG
    out = (ctypes.c_int32 * 8)()
    assert lib.sgn_launch_shape(None, out) == sgn.SGN_ERR_INVALID_ARG


def test_refined_solve_host_checks():
    lib = sgn.load_library()
    info = sgn.sgn_refine_info()
    assert lib.sgn_elliptic_solve_refined(None, None, None, None, None, 1e-10, 4, ctypes.byref(info)) \
        == sgn.SGN_ERR_INVALID_ARG


def test_graph_step_host_checks():
    lib = sgn.load_library()
    rep = ctypes.c_int32(7)
    assert lib.sgn_rk4_step_graph(None, None, None, None, None, 0.01, 1, 0, None, ctypes.byref(rep)) \
        == sgn.SGN_ERR_INVALID_ARG
    assert rep.value == 0  # cleared even on an argument error
    assert lib.sgn_rk4_step_graph(None, None, None, None, None, 0.01, 1, 0, None, None) == sgn.SGN_ERR_INVALID_ARG


def test_cnn_and_learned_guess_host_checks():
    lib = sgn.load_library()
    assert lib.sgn_cnn_workspace_bytes(64, 16) == 0          # W < 32
    assert lib.sgn_cnn_workspace_bytes(48, 64) == 0          # not a power of two
    assert lib.sgn_cnn_workspace_bytes(64, 64) > 0
    h = ctypes.c_void_p()
    assert lib.sgn_cnn_init(64, 64, None, 0, None, ctypes.byref(h)) == sgn.SGN_ERR_INVALID_ARG
    assert lib.sgn_cnn_init(64, 16, None, 0, None, ctypes.byref(h)) == sgn.SGN_ERR_UNSUPPORTED
    assert lib.sgn_cnn_destroy(None) == sgn.SGN_ERR_INVALID_ARG
    assert lib.sgn_learned_guess_attach(None, None, None, 0) == sgn.SGN_ERR_INVALID_ARG
    n = ctypes.c_int64()
    assert lib.sgn_learned_guess_recorded(None, ctypes.byref(n)) == sgn.SGN_ERR_INVALID_ARG
    assert lib.sgn_learned_guess_stages(None, 1) == sgn.SGN_ERR_INVALID_ARG
    assert lib.sgn_elliptic_solve_fgmres(None, None, None, None, None, 10, None) == sgn.SGN_ERR_INVALID_ARG
    assert sgn.SGN_CNN_PARAMS == 6 * (9 * 32 * 32 + 32)


def test_operator_noalloc_host_checks():
    """The context-free operator refuses grids beyond its fixed scratch, and
    bad or aliased fields, on the host before any GPU work (the pointers
    below are never dereferenced)."""
    lib = sgn.load_library()
    p, q, r = (ctypes.c_void_p(4096 * (i + 1)) for i in range(3))
    big = sgn.config_default(2048, 1024, 10.0, 5.0)
    assert big.nx * big.ny > sgn.SGN_NOALLOC_MAX_POINTS
    assert lib.sgn_apply_operator_noalloc(ctypes.byref(big), p, q, r, 0, None) == sgn.SGN_ERR_UNSUPPORTED
    assert b"exceeds" in lib.sgn_last_error(None)
    ok = sgn.config_default(1024, 1024, 10.0, 5.0)
    assert lib.sgn_apply_operator_noalloc(ctypes.byref(ok), None, q, r, 0, None) == sgn.SGN_ERR_INVALID_ARG
    assert lib.sgn_apply_operator_noalloc(ctypes.byref(ok), p, q, q, 1, None) == sgn.SGN_ERR_INVALID_ARG
    assert lib.sgn_apply_operator_noalloc(ctypes.byref(ok), p, ctypes.c_void_p(4100), r, 0, None) \
        == sgn.SGN_ERR_INVALID_ARG
    ok.batch = 2
    assert lib.sgn_apply_operator_noalloc(ctypes.byref(ok), p, q, r, 0, None) != sgn.SGN_OK
    bad = sgn.config_default(1000, 64, 10.0, 5.0)
    assert lib.sgn_apply_operator_noalloc(ctypes.byref(bad), p, q, r, 0, None) == sgn.SGN_ERR_UNSUPPORTED
    assert lib.sgn_apply_operator_noalloc(None, p, q, r, 0, None) == sgn.SGN_ERR_INVALID_ARG


def test_members_workspace_is_per_member():
    one = sgn.sgn_workspace_bytes(sgn.config_default(128, 64, 10.0, 5.0))
    for b in (2, 9, 64):
        assert sgn.sgn_workspace_bytes(sgn.config_default(128, 64, 10.0, 5.0, batch=b)) == b * one
    assert one % 256 == 0
