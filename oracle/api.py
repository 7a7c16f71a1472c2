"""ctypes wrapper around the oracle's C++ source (oracle/tcng_oracle.cpp).

Test infrastructure only.  Arrays are numpy; complex vectors are complex128.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tcng_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with g++ -O2 (no fast-math)."""
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i32 = ctypes.c_int
        L.orc_run.argtypes = [i32, P, i32, P, P, i32, P, P]
        L.orc_apply_matrix.argtypes = [i32, P, P, i32, P]
        L.orc_gate_matrix.argtypes = [P, P, P, i32, P]
        L.orc_expect.argtypes = [i32, P, P, P, i32, P]
        L.orc_apply_hamiltonian.argtypes = [i32, P, P, P, i32, P]
        L.orc_norm2.argtypes = [i32, P]
        L.orc_norm2.restype = ctypes.c_double
        L.orc_expect_grad.argtypes = [i32, P, i32, P, i32, P, i32, P, P, i32, P, P, P, P, P, P]
        L.orc_param_shift.argtypes = [i32, P, i32, P, i32, P, i32, P, P, i32, P, P, P]
        L.orc_pauli_coo.argtypes = [i32, P, P, i32, ctypes.c_int64, ctypes.c_int64, P, P, P, P]
        L.orc_shadow.argtypes = [i32, P, i32, P, P, P, P, P]
        L.orc_su4.argtypes = [P, P, P]
        L.orc_qml.argtypes = [i32, P, i32, P, P, i32, P, i32, i32, P, P, P]
        L.orc_mipt.argtypes = [i32, P, i32, i32, P, i32, P, P, ctypes.c_double, P, P, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c128(v):
    return None if v is None else np.ascontiguousarray(v, dtype=np.complex128)


def _gates(g):
    return np.ascontiguousarray(np.asarray(g, dtype=np.int32).reshape(-1, 6))


def _mats(m):
    m = np.zeros((0, 4, 4), np.complex128) if m is None else m
    return np.ascontiguousarray(np.asarray(m, dtype=np.complex128).reshape(-1, 4, 4))


def _params(p):
    p = np.zeros(0) if p is None else p
    return np.ascontiguousarray(np.asarray(p, dtype=np.float64).reshape(-1))


def _ham(codes, coeffs, n):
    codes = np.ascontiguousarray(np.asarray(codes, dtype=np.uint8).reshape(-1, n))
    coeffs = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64).reshape(-1))
    assert codes.shape[0] == coeffs.shape[0]
    return codes, coeffs


def run(n, gates, params=None, mats=None, init=None):
    """Final state psi_D (complex128 [2^n])."""
    g, p, m, x = _gates(gates), _params(params), _mats(mats), _c128(init)
    out = np.empty(2 ** n, np.complex128)
    lib().orc_run(n, _p(g), g.shape[0], _p(p), _p(m), m.shape[0], _p(x), _p(out))
    return out


def apply_matrix(n, state, qubits, U):
    s = np.array(state, dtype=np.complex128, copy=True)
    q = np.ascontiguousarray(np.asarray(qubits, dtype=np.int32))
    u = np.ascontiguousarray(np.asarray(U, dtype=np.complex128))
    assert u.shape == (2 ** len(q), 2 ** len(q))
    rc = lib().orc_apply_matrix(n, _p(s), _p(q), len(q), _p(u))
    assert rc == 0
    return s


def gate_matrix(gate_record, params=None, mats=None):
    g = np.ascontiguousarray(np.asarray(gate_record, dtype=np.int32).reshape(6))
    p, m = _params(params), _mats(mats)
    out = np.empty((4, 4), np.complex128)
    lib().orc_gate_matrix(_p(g), _p(p), _p(m), m.shape[0], _p(out))
    return out


def expect(n, state, codes, coeffs):
    """Complex <psi|H|psi>; the real part is E."""
    s = _c128(state)
    c, w = _ham(codes, coeffs, n)
    out = np.empty(2)
    lib().orc_expect(n, _p(s), _p(c), _p(w), c.shape[0], _p(out))
    return complex(out[0], out[1])


def apply_hamiltonian(n, state, codes, coeffs):
    s = _c128(state)
    c, w = _ham(codes, coeffs, n)
    out = np.empty(2 ** n, np.complex128)
    lib().orc_apply_hamiltonian(n, _p(s), _p(c), _p(w), c.shape[0], _p(out))
    return out


def norm2(n, state):
    s = _c128(state)
    return lib().orc_norm2(n, _p(s))


def expect_grad(n, gates, params, codes, coeffs, mats=None, init=None, want_cot=False,
                want_lie=False, want_state=False):
    """Adjoint-method E and dE/dtheta.  Returns dict(E, E_imag, grad, [cot, lie, state])."""
    g, p, m, x = _gates(gates), _params(params), _mats(mats), _c128(init)
    c, w = _ham(codes, coeffs, n)
    G = g.shape[0]
    e = np.empty(2)
    grad = np.empty(max(p.shape[0], 1))
    cot = np.empty((G, 4, 4), np.complex128) if want_cot else None
    lie = np.empty((G, 15)) if want_lie else None
    st = np.empty(2 ** n, np.complex128) if want_state else None
    lib().orc_expect_grad(n, _p(g), G, _p(p), p.shape[0], _p(m), m.shape[0], _p(c), _p(w), c.shape[0],
                          _p(x), _p(e), _p(grad), _p(cot), _p(lie), _p(st))
    out = dict(E=e[0], E_imag=e[1], grad=grad[: p.shape[0]])
    if want_cot:
        out["cot"] = cot
    if want_lie:
        out["lie"] = lie
    if want_state:
        out["state"] = st
    return out


def param_shift(n, gates, params, codes, coeffs, mats=None, init=None, want_lie=False):
    g, p, m, x = _gates(gates), _params(params), _mats(mats), _c128(init)
    c, w = _ham(codes, coeffs, n)
    G = g.shape[0]
    grad = np.empty(max(p.shape[0], 1))
    lie = np.empty((G, 15)) if want_lie else None
    lib().orc_param_shift(n, _p(g), G, _p(p), p.shape[0], _p(m), m.shape[0], _p(c), _p(w), c.shape[0],
                          _p(x), _p(grad), _p(lie))
    out = dict(grad=grad[: p.shape[0]])
    if want_lie:
        out["lie"] = lie
    return out


__all__ = ["build", "lib", "run", "apply_matrix", "gate_matrix", "expect", "apply_hamiltonian", "norm2",
           "expect_grad", "param_shift", "mipt", "pauli_coo", "shadow", "su4", "qml"]


def mipt(n, gates, mats, u, p, init=None, force=None):
    """One monitored brick-wall trajectory (complex128).

    gates: the gates of one time step (all U2); mats [n_steps, n_step_mats, 4, 4];
    u [n_steps, n] uniforms; force (optional) [n_steps, n] int: -1 free, 0 / 1 forced.
    Returns dict(state, rec [n_steps, 2] uint32 (mask, outcomes), logp, margin [n_steps, n]).
    """
    g = _gates(gates)
    mats = np.ascontiguousarray(np.asarray(mats, dtype=np.complex128))
    assert mats.ndim == 4 and mats.shape[2:] == (4, 4)
    n_steps, n_step_mats = mats.shape[0], mats.shape[1]
    uu = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(n_steps, n))
    f = None if force is None else np.ascontiguousarray(np.asarray(force, dtype=np.int32).reshape(n_steps, n))
    x = _c128(init)
    st = np.empty(2 ** n, np.complex128)
    rec = np.zeros((max(n_steps, 1), 2), np.uint32)
    logp = np.zeros(1)
    margin = np.empty((max(n_steps, 1), n))
    rc = lib().orc_mipt(n, _p(g), g.shape[0], n_steps, _p(mats), n_step_mats, _p(x), _p(uu), float(p), _p(f),
                        _p(st), _p(rec), _p(logp), _p(margin))
    assert rc == 0, rc
    return dict(state=st, rec=rec[:n_steps], logp=float(logp[0]), margin=margin[:n_steps])


def pauli_coo(n, codes, coeffs, row_begin=0, row_count=None):
    """COO entries of H = sum_k c_k P_k for rows [row_begin, row_begin + row_count):
    (rows int64, cols int64, vals complex128, n_groups), group-major (X-mask
    groups in first-appearance order), one entry per (group, row)."""
    c, w = _ham(codes, coeffs, n)
    count = 2 ** n - row_begin if row_count is None else int(row_count)
    # group count first (a single row), then the full range
    ng = ctypes.c_int()
    cap = max(c.shape[0], 1) * max(count, 1)
    rows = np.empty(cap, np.int64)
    cols = np.empty(cap, np.int64)
    vals = np.empty(cap, np.complex128)
    rc = lib().orc_pauli_coo(n, _p(c), _p(w), c.shape[0], int(row_begin), count, _p(rows), _p(cols), _p(vals),
                             ctypes.byref(ng))
    assert rc == 0, rc
    m = ng.value * count
    return rows[:m], cols[:m], vals[:m], ng.value


def shadow(n, psi, bases, u):
    """Classical-shadow snapshots of one state: bases uint8 [S, n] (1=X, 2=Y, 3=Z),
    u [S] uniforms.  Returns (outcomes int64 [S], lo [S], hi [S]) with lo / hi the
    normalised running probability just before and at the outcome."""
    x = _c128(psi)
    b = np.ascontiguousarray(np.asarray(bases, dtype=np.uint8).reshape(-1, n))
    S = b.shape[0]
    uu = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(S))
    out = np.empty(max(S, 1), np.int64)
    lo = np.empty(max(S, 1))
    hi = np.empty(max(S, 1))
    rc = lib().orc_shadow(n, _p(x), S, _p(b), _p(uu), _p(out), _p(lo), _p(hi))
    assert rc == 0, rc
    return out[:S], lo[:S], hi[:S]


def su4(theta):
    """SU(4) gate exp(-i sum_k theta_k P_k / 2) and its 15 derivatives: (U [4, 4], dU [15, 4, 4])."""
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(15))
    U = np.empty((4, 4), np.complex128)
    dU = np.empty((15, 4, 4), np.complex128)
    lib().orc_su4(_p(th), _p(U), _p(dU))
    return U, dU


def qml(n, gates, theta, inputs, labels, k, C, want_probs=False):
    """Softmax cross-entropy loss per sample and the batch-mean gradient
    d(mean L)/dtheta [G, 15] of the SU(4) QML circuit."""
    g = _gates(gates)
    G = g.shape[0]
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).reshape(G, 15))
    x = np.ascontiguousarray(np.asarray(inputs, dtype=np.complex128).reshape(-1, 2 ** n))
    B = x.shape[0]
    y = np.ascontiguousarray(np.asarray(labels, dtype=np.int32).reshape(B))
    loss = np.empty(B)
    grad = np.empty((G, 15))
    probs = np.empty((B, 2 ** k)) if want_probs else None
    rc = lib().orc_qml(n, _p(g), G, _p(th), _p(x), B, _p(y), int(k), int(C), _p(loss), _p(grad), _p(probs))
    assert rc == 0, rc
    out = dict(loss=loss, grad=grad)
    if want_probs:
        out["probs"] = probs
    return out
