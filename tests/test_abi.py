"""Host-side checks of the C ABI: the library loads, exports every function that
include/ns.h declares, and validates arguments before any HIP call (so these run
without a GPU)."""

import ctypes
import os
import re

import pytest

from oracle import grid
from paper_2603_08892_amd import ns

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "ns.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(ns(?:1d)?_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert sorted(ns.ABI_FUNCTIONS) == _declared()


def test_pass_names_match_header():
    with open(os.path.join(ROOT, "include", "ns.h")) as f:
        m = re.search(r"#define NS_NUM_PASSES (\d+)", f.read())
    assert int(m.group(1)) == len(ns.PASS_NAMES)


def test_library_exports_every_declared_symbol():
    L = ns.lib()
    for name in _declared():
        assert hasattr(L, name), name


@pytest.mark.parametrize("n", [8, 12, 16, 24, 32, 40, 48, 64, 96, 128, 192, 256, 360, 384, 512])
@pytest.mark.parametrize("ct", [2 / 3, 0.8889, 0.9481, 2 * 2 ** 0.5 / 3, 1.0])
def test_retained_bounds_match_oracle(n, ct):
    assert ns.retained_bound(n, ct, "sphere") == grid.sphere_k2max(n, ct)
    assert ns.retained_bound(n, ct, "cube") == grid.cube_kmax(n, ct)


@pytest.mark.parametrize("n", [8, 12, 16, 32, 128, 192, 360])
@pytest.mark.parametrize("ct", [2 / 3, 0.97, 1.0])
def test_pair_rule_masks_bound_by_their_sphere_or_cube(n, ct):
    assert ns.retained_bound(n, ct, "no_multiple_aliases") == grid.sphere_k2max(n, ct)
    assert ns.retained_bound(n, ct, "rogallo") == grid.cube_kmax(n, ct)


@pytest.mark.parametrize("bad", [-1, 4])
def test_unknown_mask_rejected(bad):
    L = ns.lib()
    cfg = ns.make_config(32, 0.1, 1.0)
    cfg.mask = bad
    assert L.ns_workspace_bytes(ctypes.byref(cfg)) == 0
    assert b"mask" in L.ns_last_error(None)


@pytest.mark.parametrize("n", [8, 16, 32, 128, 192, 360, 512, 1024])
def test_num_shells_matches_oracle(n):
    assert ns.num_shells(n) == grid.n_shells(n)


@pytest.mark.parametrize("n,ct,prec,mask", [(7, 1.0, "fp32", "sphere"), (14, 1.0, "fp32", "sphere"),
                                            (2048, 1.0, "fp32", "sphere"), (6, 1.0, "fp32", "sphere"),
                                            (32, 0.0, "fp32", "sphere"), (32, 1.1, "fp32", "sphere"),
                                            (32, 0.01, "fp32", "sphere"), (33, 1.0, "fp32", "sphere")])
def test_invalid_configs_rejected(n, ct, prec, mask):
    assert ns.workspace_bytes(n, 0.01, ct, mask, prec) == 0
    msg = ns.lib().ns_last_error(None)
    assert msg


def test_invalid_nu_and_precision_rejected():
    L = ns.lib()
    cfg = ns.make_config(32, -1.0, 1.0)
    assert L.ns_workspace_bytes(ctypes.byref(cfg)) == 0
    cfg = ns.make_config(32, float("nan"), 1.0)
    assert L.ns_workspace_bytes(ctypes.byref(cfg)) == 0
    cfg = ns.make_config(32, 0.1, 1.0)
    cfg.precision = 7
    assert L.ns_workspace_bytes(ctypes.byref(cfg)) == 0
    cfg = ns.make_config(32, 0.1, 1.0)
    cfg.flags = 6
    assert L.ns_workspace_bytes(ctypes.byref(cfg)) == 0
    cfg.flags = ns.NS_CFG_GENERIC_PASSES
    assert L.ns_workspace_bytes(ctypes.byref(cfg)) > 0


def test_init_argument_errors_before_any_hip_call():
    L = ns.lib()
    ctx = ctypes.c_void_p()
    cfg = ns.make_config(32, 0.1, 2 / 3)
    assert L.ns_init(ctypes.byref(cfg), None, 1 << 30, ctypes.byref(ctx)) == ns.NS_ERR_ARG
    assert L.ns_init(ctypes.byref(cfg), ctypes.c_void_p(0x1001), 1 << 30, ctypes.byref(ctx)) == ns.NS_ERR_ARG
    need = L.ns_workspace_bytes(ctypes.byref(cfg))
    assert L.ns_init(ctypes.byref(cfg), ctypes.c_void_p(0x100000), need - 1, ctypes.byref(ctx)) == ns.NS_ERR_SIZE
    assert b"too small" in L.ns_last_error(None)
    assert L.ns_init(None, ctypes.c_void_p(0x100000), need, ctypes.byref(ctx)) == ns.NS_ERR_ARG
    assert L.ns_init(ctypes.byref(cfg), ctypes.c_void_p(0x100000), need, None) == ns.NS_ERR_ARG


def test_null_context_rejected():
    L = ns.lib()
    assert L.ns_nonlinear(None, None, None, None, 0) == ns.NS_ERR_ARG
    assert L.ns_step_rk4_trunc(None, None, 0.1, 1, None, 0) == ns.NS_ERR_ARG
    assert L.ns_step_rk2_phaseshift(None, None, 0.1, 1, 0, None, None, 0, None) == ns.NS_ERR_ARG
    assert L.ns_spectra(None, None, None, None) == ns.NS_ERR_ARG
    assert L.ns_vjp_rk2_phaseshift(None, None, None, 0.1, 0, None, None, 0, None) == ns.NS_ERR_ARG
    assert L.ns_budget_start(None, None) == ns.NS_ERR_ARG
    assert L.ns_budget_stop(None) == ns.NS_ERR_ARG
    assert L.ns_budget_read(None, None) == ns.NS_ERR_ARG


def test_workspace_scales_with_grid():
    small = ns.workspace_bytes(64, 0.01, 1.0)
    big = ns.workspace_bytes(128, 0.01, 1.0)
    assert 6 < big / small < 10
    # the pruned scratch is smaller for 2/3 truncation than for C_t = 1
    assert ns.workspace_bytes(192, 0.01, 2 / 3) < ns.workspace_bytes(192, 0.01, 1.0)


@pytest.mark.parametrize("n,ct,batch,ptr", [(7, 1.0, 1, 256), (2, 1.0, 1, 256), (2048, 1.0, 1, 256),
                                            (8, 0.0, 1, 256), (8, 0.2, 1, 256), (16, 1.0, -1, 256),
                                            (16, 1.0, 1, None), (16, 1.0, 1, 264)])
def test_model1d_argument_errors(n, ct, batch, ptr):
    """Host checks of the 1D model's entry points run before any HIP call."""
    L = ns.lib()
    p = None if ptr is None else ctypes.c_void_p(ptr)
    assert L.ns1d_nonlinear(p, p, n, ct, batch, 0.0, None) == ns.NS_ERR_ARG
    assert L.ns1d_step(p, n, ct, batch, 0.1, 1, 0, None) == ns.NS_ERR_ARG
    assert L.ns_last_error(None)


@pytest.mark.parametrize("dt,nsteps,scheme", [(0.0, 1, 0), (float("nan"), 1, 0), (0.1, -1, 0), (0.1, 1, 6),
                                              (0.1, 1, -1)])
def test_model1d_step_argument_errors(dt, nsteps, scheme):
    L = ns.lib()
    p = ctypes.c_void_p(256)
    assert L.ns1d_step(p, 16, 1.0, 1, dt, nsteps, scheme, None) == ns.NS_ERR_ARG
    assert L.ns1d_nonlinear(p, p, 16, 1.0, 1, float("inf"), None) == ns.NS_ERR_ARG


def test_spectra_static_host_checks():
    """ns_spectra_static rejects grids beyond its static scratch and bad arguments on the
    host, before any HIP call."""
    L = ns.lib()
    out = ns.NSSpectraOut()
    p = ctypes.c_void_p(256)
    assert L.ns_spectra_static(768, ns.NS_FP32, 0.01, p, None, None, ctypes.byref(out)) == ns.NS_ERR_SIZE
    assert b"512" in L.ns_last_error(None)
    assert L.ns_spectra_static(7, ns.NS_FP32, 0.01, p, None, None, ctypes.byref(out)) == ns.NS_ERR_ARG
    assert L.ns_spectra_static(64, 5, 0.01, p, None, None, ctypes.byref(out)) == ns.NS_ERR_ARG
    assert L.ns_spectra_static(64, ns.NS_FP32, -1.0, p, None, None, ctypes.byref(out)) == ns.NS_ERR_ARG
    assert L.ns_spectra_static(64, ns.NS_FP32, 0.01, ctypes.c_void_p(0x101), None, None,
                               ctypes.byref(out)) == ns.NS_ERR_ARG
    assert L.ns_spectra_static(64, ns.NS_FP32, 0.01, p, None, None, None) == ns.NS_ERR_ARG
