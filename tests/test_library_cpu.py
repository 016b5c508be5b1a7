"""Host-side checks of the C-ABI library (no device needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1705_09907_amd as H
from oracle import hdg, mg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "hdggmg.h")).read()
    return sorted(set(re.findall(r"^\s*(?:hdg_status_t|const char\*)\s+(hdg_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 18
    for name in names:
        assert hasattr(H.lib, name), name
        assert name in H.SIGNATURES, f"binding lacks {name}"


def _handle_entries():
    out = []
    for name in declared_functions():
        args = H.SIGNATURES[name]
        if args and args[0] is H._P and name not in ("hdg_last_error", "hdg_apply_trace_operator_batch"):
            out.append(name)
    return out


@pytest.mark.parametrize("name", _handle_entries())
def test_null_handle_is_rejected_before_any_device_call(name):
    """Every entry point that takes a handle returns HDG_ERR_INVALID_ARG for a null
    handle (all other arguments zero or null), touching neither host nor device memory."""
    zero = {H._P: None, H._PD: None, H._PI32: None, H._PI64: None, H._I32: 0, H._I64: 0, H._D: 0.0}
    args = [zero[t] for t in H.SIGNATURES[name]]
    assert getattr(H.lib, name)(*args) == -1, name


@pytest.mark.parametrize("n,k,p,kappa,coarse", [
    (4, 0, 0, 1.0, "galerkin"), (16, 1, 1, 3.7, "galerkin"), (256, 4, 4, 0.3, "galerkin"),
    (1024, 3, 3, 57.0, "galerkin"), (8, 3, 1, 2.0, "galerkin"), (8, 4, 0, 0.01, "galerkin"),
    (64, 8, 8, 1.5, "galerkin"), (32, 3, 2, 0.7, "rediscretize"), (32, 3, 0, 5.0, "rediscretize")])
def test_host_setup_blocks_match_oracle(n, k, p, kappa, coarse):
    """Library setup (U-Schur elimination, product-form Lagrange basis) vs the oracle's
    explicit local systems (full solve with Abb, barycentric basis)."""
    Kl = H.element_block_host(n, k, p, kappa, coarse=coarse)
    top = k if coarse == "galerkin" else p
    Ko = hdg.Problem(n, top, np.full(n * n, kappa)).element_block(0)
    for q in range(top, p, -1):
        P4 = mg.element_prolongation(q)
        Ko = P4.T @ Ko @ P4
    assert np.abs(Kl - Ko).max() <= 1e-13 * np.abs(Ko).max()


def test_quadrature_nodes_match_oracle():
    from oracle import quadrature as qd
    for nq in range(1, 12):
        assert np.abs(H.quadrature_nodes(nq) - qd.gauss_legendre(nq)[0]).max() < 1e-15


@pytest.mark.parametrize("field,value,code", [("n", 1, -1), ("k", 9, -1), ("k", -1, -1), ("tau", 0.0, -1),
                                              ("nu1", 0, -1), ("smoother", 7, -1), ("cheb_lo", 2.0, -1),
                                              ("nq", 0, -1), ("precision", 3, -1), ("precision", -1, -1),
                                              ("graph", 2, -1), ("autotune", -1, -1), ("cycle", 3, -1),
                                              ("cycle", -1, -1), ("q1_schedule", 2, -1),
                                              ("q1_schedule", -1, -1), ("chain_shape", 5, -1),
                                              ("chain_shape", -1, -1)])
def test_create_rejects_bad_config_before_any_device_call(field, value, code):
    cfg = H.Config()
    assert H.lib.hdg_config_default(8, 2, ctypes.byref(cfg)) == 0
    setattr(cfg, field, value)
    kap = np.ones(64)
    h = ctypes.c_void_p()
    st = H.lib.hdg_create(ctypes.byref(cfg), kap.ctypes.data_as(H._PD), None, ctypes.byref(h))
    assert st == code and not h.value


@pytest.mark.parametrize("p,m", [(2, 1), (0, -1), (0, 65), (5, 2)])
def test_create_rejects_bad_inner_steps(p, m):
    cfg = H.Config()
    H.lib.hdg_config_default(8, 2, ctypes.byref(cfg))
    cfg.inner_steps[p] = m
    kap = np.ones(64)
    h = ctypes.c_void_p()
    assert H.lib.hdg_create(ctypes.byref(cfg), kap.ctypes.data_as(H._PD), None, ctypes.byref(h)) == -1
    assert not h.value


@pytest.mark.parametrize("prec", [1, 2])
def test_reduced_precision_face_smoother_needs_omega(prec):
    cfg = H.Config()
    H.lib.hdg_config_default(8, 2, ctypes.byref(cfg))
    cfg.smoother, cfg.precision = H.SMOOTHERS["face"], prec
    kap = np.ones(64)
    h = ctypes.c_void_p()
    assert H.lib.hdg_create(ctypes.byref(cfg), kap.ctypes.data_as(H._PD), None, ctypes.byref(h)) == -1
    assert not h.value


def _first_n_past_lds(k, vb, cap=160 * 1024):
    P = k + 1
    n = 2
    while ((n - 1) * P + P * P) * vb <= cap:
        n += 1
    return n


@pytest.mark.parametrize("k,prec", [(7, 0), (3, 0), (8, 1), (8, 0)])
def test_chain_smoother_rejects_chains_beyond_lds(k, prec):
    """One chain's right-hand side plus one factor block must fit the LDS of one
    gfx950 workgroup: ((n-1)(k+1) + (k+1)^2) * (8 or 4 bytes) <= 160 KiB; each
    case is the first n past it, rejected before any device call."""
    P, vb = k + 1, 8 if prec == 0 else 4
    n = _first_n_past_lds(k, vb)
    assert ((n - 1) * P + P * P) * vb > 163840 >= ((n - 2) * P + P * P) * vb
    cfg = H.Config()
    H.lib.hdg_config_default(n, k, ctypes.byref(cfg))
    cfg.precision = prec
    kap = np.ones(n * n)
    h = ctypes.c_void_p()
    assert H.lib.hdg_create(ctypes.byref(cfg), kap.ctypes.data_as(H._PD), None, ctypes.byref(h)) == -1
    assert not h.value


def test_config_layout_matches_header():
    """The Python mirror of hdg_config_t has the C layout (size and field offsets)."""
    import re
    src = open(__import__("os").path.join(__import__("os").path.dirname(__file__), "..", "include",
                                          "hdggmg.h")).read()
    body = src[src.index("typedef struct {"):src.index("} hdg_config_t;")]
    names = re.findall(r"^\s*(?:int32_t|double)\s+([a-z_0-9]+(?:\s*,\s*[a-z_0-9]+)*)", body, re.M)
    fields = [f.strip() for grp in names for f in grp.split(",")]
    assert fields == [f[0] for f in H.Config._fields_]
    assert ctypes.sizeof(H.Config) == 4 + 4 + 8 + 4 + 4 + 4 + 4 + 8 * 9 + 16 + 8 * 24 + 4 + 4 + 4 + 4 * 9 + 4 + 4 + 4 * 6


@pytest.mark.parametrize("bad", [0.0, -1.0, np.nan, np.inf])
def test_create_rejects_bad_kappa(bad):
    cfg = H.Config()
    H.lib.hdg_config_default(8, 1, ctypes.byref(cfg))
    kap = np.ones(64)
    kap[17] = bad
    h = ctypes.c_void_p()
    assert H.lib.hdg_create(ctypes.byref(cfg), kap.ctypes.data_as(H._PD), None, ctypes.byref(h)) == -1


def test_host_block_rejects_bad_arguments():
    out = np.zeros((8, 8))
    pd = out.ctypes.data_as(H._PD)
    assert H.lib.hdg_element_block_host(8, 1, 2, 1.0, 1.0, 0, pd) == -1      # p > k
    assert H.lib.hdg_element_block_host(8, 1, 1, 1.0, -1.0, 0, pd) == -1     # kappa <= 0
    assert H.lib.hdg_element_block_host(1, 1, 1, 1.0, 1.0, 0, pd) == -1      # n < 2
    assert H.lib.hdg_element_block_host(8, 1, 1, 1.0, 1.0, 5, pd) == -1      # bad coarse mode
    assert H.lib.hdg_status_string(-4) == b"not converged"
    assert H.lib.hdg_status_string(-7) == b"stopped at the rounding floor of the residual"
    assert H.STATUS[-7] == H.lib.hdg_status_string(-7).decode()
