"""Host-side checks of the C ABI library (no GPU needed).

The library loads and exports every symbol include/tcng.h declares; argument
validation rejects bad input before any device call; and the tiled planner's
schedule is a legal reordering of the circuit whose every gate fits its pass's
tile (checked by running the CPU oracle in the planned order).
"""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    import paper_2602_14167_amd as pkg
    pkg.lib()
    return pkg


def header_functions():
    txt = open(os.path.join(ROOT, "include", "tcng.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tcng_[a-z_0-9]+)\s*\(", txt)))


def test_exports_every_declared_symbol(P):
    names = header_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(P.lib(), name), name
    assert set(names) == set(P._lib.EXPORTS)
    assert P.lib().tcng_version() == 1


def test_validation_errors_without_device(P):
    L = P.lib()
    h = ctypes.c_void_p()
    bad = np.array([[W.CNOT, 0, 0, -1, -1, -1]], np.int32)           # duplicate qubit
    assert L.tcng_circuit_create(3, bad.ctypes.data_as(ctypes.c_void_p), 1, 0, None, 0, ctypes.byref(h)) == P._lib.TCNG_E_INVALID
    assert b"duplicate" in L.tcng_last_error()
    bad = np.array([[W.RY, 5, -1, 0, -1, -1]], np.int32)             # qubit out of range
    assert L.tcng_circuit_create(3, bad.ctypes.data_as(ctypes.c_void_p), 1, 1, None, 0, ctypes.byref(h)) == P._lib.TCNG_E_INVALID
    bad = np.array([[W.RY, 1, -1, 3, -1, -1]], np.int32)             # parameter index out of range
    assert L.tcng_circuit_create(3, bad.ctypes.data_as(ctypes.c_void_p), 1, 2, None, 0, ctypes.byref(h)) == P._lib.TCNG_E_INVALID
    bad = np.array([[W.U2, 1, 0, -1, -1, 0]], np.int32)              # matrix index out of range
    assert L.tcng_circuit_create(3, bad.ctypes.data_as(ctypes.c_void_p), 1, 0, None, 0, ctypes.byref(h)) == P._lib.TCNG_E_INVALID
    bad = np.array([[17, 1, -1, -1, -1, -1]], np.int32)              # unknown kind
    assert L.tcng_circuit_create(3, bad.ctypes.data_as(ctypes.c_void_p), 1, 0, None, 0, ctypes.byref(h)) == P._lib.TCNG_E_INVALID
    assert L.tcng_circuit_create(40, None, 0, 0, None, 0, ctypes.byref(h)) == P._lib.TCNG_E_UNSUPPORTED
    codes = np.array([[4, 0]], np.uint8)
    coeffs = np.array([1.0])
    assert L.tcng_pauli_sum_create(2, codes.ctypes.data_as(ctypes.c_void_p), coeffs.ctypes.data_as(ctypes.c_void_p), 1,
                                   ctypes.byref(h)) == P._lib.TCNG_E_INVALID
    assert L.tcng_state_init(None, None, 0, None) == P._lib.TCNG_E_INVALID
    s = P.TcngState(0, 4, 0, 1, 16)
    assert L.tcng_state_init(ctypes.byref(s), None, 0, None) == P._lib.TCNG_E_INVALID   # null amplitudes
    s = P.TcngState(256, 4, 0, 1, 8)
    assert L.tcng_state_init(ctypes.byref(s), None, 0, None) == P._lib.TCNG_E_INVALID   # stride < 2^n
    s = P.TcngState(256, 4, 7, 1, 16)
    assert L.tcng_state_init(ctypes.byref(s), None, 0, None) == P._lib.TCNG_E_INVALID   # dtype
    s = P.TcngState(256, 4, 0, 1, 16)
    q = np.array([1, 1], np.int32)
    assert L.tcng_apply_gate(ctypes.byref(s), q.ctypes.data_as(ctypes.c_void_p), 2, ctypes.c_void_p(256), None) == P._lib.TCNG_E_INVALID
    q = np.array([0, 1, 2, 3, 0, 1], np.int32)
    assert L.tcng_apply_gate(ctypes.byref(s), q.ctypes.data_as(ctypes.c_void_p), 6, ctypes.c_void_p(256), None) == P._lib.TCNG_E_INVALID


def _check_schedule(P, oracle_mod, n, gates, n_params, params, mats, dtype):
    import torch
    order, pass_of, masks = P.plan_inspect(n, gates, n_params, dtype=dtype)
    assert order is not None
    G = len(gates)
    assert sorted(order.tolist()) == list(range(G))
    pos = np.empty(G, int)
    pos[order] = np.arange(G)
    qsets = [{int(g[1])} | ({int(g[2])} if g[2] >= 0 else set()) for g in gates]
    # gates sharing a qubit keep their relative order
    last = {}
    for i in range(G):
        for q in qsets[i]:
            if q in last:
                assert pos[last[q]] < pos[i]
            last[q] = i
    # every gate's qubits lie in its pass's tile; passes are non-decreasing in execution order
    assert np.all(np.diff(pass_of) >= 0)
    m_max = 13 if dtype == torch.complex64 else 12
    for k, gi in enumerate(order):
        mask = int(masks[pass_of[k]])
        assert bin(mask).count("1") == min(n, m_max)
        for q in qsets[gi]:
            assert (mask >> q) & 1
    # the reordered circuit computes the same state (CPU oracle)
    if n <= 14:
        a = oracle_mod.run(n, gates, params, mats)
        b = oracle_mod.run(n, gates[order], params, mats)
        np.testing.assert_allclose(a, b, atol=1e-12)
    return len(masks)


@pytest.mark.parametrize("n", [11, 12, 14])
def test_planner_random_circuits(P, oracle_mod, n):
    import torch
    r = np.random.default_rng(40 + n)
    gates, params, mats = W.random_circuit(n, 150, r)
    for dt in (torch.complex64, torch.complex128):
        _check_schedule(P, oracle_mod, n, gates, len(params), params, mats, dt)


def test_planner_workloads(P, oracle_mod):
    import torch
    c = W.cfg2(n=14, layers=3)
    _check_schedule(P, oracle_mod, 14, c["gates"], c["n_params"], c["params"], None, torch.complex64)
    c = W.cfg2()
    npass = _check_schedule(P, oracle_mod, 28, c["gates"], c["n_params"], c["params"], None, torch.complex64)
    assert npass <= 20          # 996 gates in a handful of HBM round trips
    c = W.cfg5()
    _check_schedule(P, oracle_mod, 32, c["gates"], c["n_params"], c["params"], None, torch.complex64)
    c = W.cfg4(count=4)
    for cc in c["circuits"]:
        _check_schedule(P, oracle_mod, cc["n"], cc["gates"], 0, None, cc["mats"], torch.complex64)


def _check_fused_schedule(P, oracle_mod, n, gates, n_params, params, mats, k=4):
    order, pass_of, block_of, npass, nblk, bad = P.fused_plan_inspect(n, gates, n_params, k)
    G = len(gates)
    assert bad == 0                                   # every LDS layout a bank-conflict-free bijection
    assert sorted(order.tolist()) == list(range(G))
    pos = np.empty(G, int)
    pos[order] = np.arange(G)
    qsets = [{int(g[1])} | ({int(g[2])} if g[2] >= 0 else set()) for g in gates]
    last = {}
    for i in range(G):
        for q in qsets[i]:
            if q in last:
                assert pos[last[q]] < pos[i]
            last[q] = i
    assert np.all(np.diff(pass_of) >= 0) and np.all(np.diff(block_of) >= 0)
    # a block touches at most k qubits; a pass holds at most 8 (k = 4) or 4 (k = 5) blocks
    for b in range(nblk):
        qs = set().union(*[qsets[gi] for gi in order[block_of == b]])
        assert 1 <= len(qs) <= k
    for p in range(npass):
        assert len(set(block_of[pass_of == p].tolist())) <= (8 if k == 4 else 4)
    if n <= 14:
        a = oracle_mod.run(n, gates, params, mats)
        b = oracle_mod.run(n, gates[order], params, mats)
        np.testing.assert_allclose(a, b, atol=1e-12)
    return npass, nblk


@pytest.mark.parametrize("n,k", [(9, 4), (12, 4), (14, 4), (12, 5), (14, 5)])
def test_fused_planner_random_circuits(P, oracle_mod, n, k):
    r = np.random.default_rng(60 + n)
    gates, params, mats = W.random_circuit(n, 200, r)
    _check_fused_schedule(P, oracle_mod, n, gates, len(params), params, mats, k)


def test_fused_planner_workloads(P, oracle_mod):
    c = W.cfg2()
    npass, nblk = _check_fused_schedule(P, oracle_mod, 28, c["gates"], c["n_params"], c["params"], None)
    assert nblk < len(c["gates"]) // 5          # blocks hold many gates each
    c = W.cfg5()
    _check_fused_schedule(P, oracle_mod, 32, c["gates"], c["n_params"], c["params"], None)
    c = W.cfg3(batch=2)
    _check_fused_schedule(P, oracle_mod, 16, c["gates"], c["n_params"], c["params"][0], None)
    for cc in W.cfg4(count=4)["circuits"]:
        _check_fused_schedule(P, oracle_mod, cc["n"], cc["gates"], 0, None, cc["mats"])


def test_fused5_planner_workloads(P, oracle_mod):
    # 5-qubit blocks hold more gates than 4-qubit ones
    for w, n in ((W.cfg2(), 28), (W.cfg5(), 32)):
        _, nb4 = _check_fused_schedule(P, oracle_mod, n, w["gates"], w["n_params"], w["params"], None, 4)
        _, nb5 = _check_fused_schedule(P, oracle_mod, n, w["gates"], w["n_params"], w["params"], None, 5)
        assert nb5 < nb4
    for cc in W.cfg4(count=4, n_lo=12)["circuits"]:
        _check_fused_schedule(P, oracle_mod, cc["n"], cc["gates"], 0, None, cc["mats"], 5)


def test_fused_planner_rejects_small_tiles(P):
    gates = np.array([W.gate(W.RY, 0, p0=0)], np.int32)
    with pytest.raises(P.TcngError):
        P.fused_plan_inspect(8, gates, 1)
    with pytest.raises(P.TcngError):
        P.fused_plan_inspect(11, gates, 1, 5)     # 5-qubit blocks need full 12-bit tiles
    with pytest.raises(P.TcngError):
        P.fused_plan_inspect(12, gates, 1, 6)


def _ry_rz_cnot(n, n_gates, rng):
    g, npar = [], 0
    for _ in range(n_gates):
        k = rng.integers(3)
        if k == 2:
            a, b = rng.choice(n, size=2, replace=False)
            g.append(W.gate(W.CNOT, int(a), int(b)))
        else:
            g.append(W.gate(W.RY if k == 0 else W.RZ, int(rng.integers(n)), p0=npar))
            npar += 1
    return W.as_gate_array(g), npar


@pytest.mark.parametrize("tiling", [(13, 5, 4), (13, 5, 5), (13, 4, 4), (12, 4, 3), (12, 4, 4), (11, 5, 4)])
def test_rounds_planner_layouts(P, tiling):
    """The LDS layouts between round phases: bijections of the tile, the tile
    load's layout first, and at every inner phase boundary 8, 16 and 32
    consecutive lanes of the reading phase, and of the writing phase through
    its CNOT permutation, on distinct banks (rotation rounds on the HEA and
    random RY/RZ/CNOT circuits, fSim rounds on the brick wall)."""
    c = W.cfg2()
    rp, nph, bad = P.rounds_plan_inspect(28, c["gates"], c["n_params"], tiling)
    assert rp > 0 and nph > rp and bad == 0
    f = W.cfg5()
    rp, nph, bad = P.rounds_plan_inspect(32, f["gates"], f["n_params"], tiling)
    assert rp > 0 and bad == 0
    r = np.random.default_rng(70 + tiling[0] + tiling[2])
    for n in (11, 14, 20):
        gates, npar = _ry_rz_cnot(n, 300, r)
        rp, nph, bad = P.rounds_plan_inspect(n, gates, npar, tiling)
        assert rp > 0 and bad == 0, (n, rp, bad)


def test_rounds_planner_rejects_bad_tilings(P):
    c = W.cfg2(n=14, layers=2)
    for tiling in ((14, 5, 4), (13, 6, 4), (13, 5, 2), (8, 4, 4)):
        with pytest.raises(P.TcngError):
            P.rounds_plan_inspect(14, c["gates"], c["n_params"], tiling)
