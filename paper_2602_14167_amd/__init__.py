"""MI355X statevector hot path: gates, Pauli-sum <H> and adjoint gradients.

Python face of the C ABI (include/tcng.h).  PyTorch supplies device memory
and the stream; the computation runs in the HIP kernels of libtcng.so.
Following the paper's problem statement (Sec. "Foundations Recap"):

    circ = Circuit(n, gates, n_params)            # tc.Circuit + gate calls
    H = PauliSum(n, codes, coeffs)                # expectation_ps terms
    E, g = expect_grad(circ, params, H)           # jit(vmap(value_and_grad(...)))
    E = TcngEnergy.apply(params, circ, H)         # torch autograd op
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import (TCNG_C64, TCNG_C128, TCNG_MODE_AUTO, TCNG_MODE_FUSED, TCNG_MODE_FUSED5,  # noqa: F401
                   TCNG_MODE_PLAIN, TCNG_MODE_TILED, TCNG_U1_KIND,
                   TcngError, TcngGate, TcngState, check, lib)

__all__ = ["expect_grad_multi", "Multi", "expect_grad_noalloc", "autotune", "plan_inspect", "Circuit", "PauliSum", "state_init", "apply_gate", "run_circuit", "expect_pauli", "expect_grad",
           "TcngEnergy", "new_state", "TcngError", "MODES", "fused_plan_inspect", "rounds_plan_inspect", "Graph",
           "mipt_run",
           "apply_pauli", "pauli_coo", "shadow_layer", "shadow_snapshots", "qml_step"]

MODES = {"tiled": TCNG_MODE_TILED, "plain": TCNG_MODE_PLAIN, "fused": TCNG_MODE_FUSED, "fused5": TCNG_MODE_FUSED5,
         "auto": TCNG_MODE_AUTO}
MODE_NAMES = {v: k for k, v in MODES.items()}


def _mode(mode):
    return MODES[mode] if isinstance(mode, str) else int(mode)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype_code(t: torch.Tensor):
    if t.dtype == torch.complex64:
        return TCNG_C64
    if t.dtype == torch.complex128:
        return TCNG_C128
    raise TypeError(f"state must be complex64 or complex128, got {t.dtype}")


def _state(t: torch.Tensor, n: int) -> TcngState:
    if not t.is_cuda:
        raise ValueError("state must be a device tensor")
    if t.dim() == 1:
        t2 = t.view(1, -1)
    else:
        t2 = t
    if t2.dim() != 2 or t2.shape[1] != 2 ** n or t2.stride(1) != 1:
        raise ValueError(f"state must be [batch, 2^{n}] with unit inner stride")
    return TcngState(t2.data_ptr(), n, _dtype_code(t2), t2.shape[0], t2.stride(0))


def _nqubits(t: torch.Tensor) -> int:
    d = t.shape[-1]
    n = int(d).bit_length() - 1
    if d != 2 ** n:
        raise ValueError("last dimension must be a power of two")
    return n


def new_state(n, batch=1, dtype=torch.complex64, device="cuda"):
    """|0...0> for every batch member, shape [batch, 2^n]."""
    psi = torch.empty((batch, 2 ** n), dtype=dtype, device=device)
    state_init(psi)
    return psi


def state_init(psi: torch.Tensor, amps: torch.Tensor | None = None, basis: int = 0):
    n = _nqubits(psi)
    s = _state(psi, n)
    ptr = None
    if amps is not None:
        amps = amps.to(device=psi.device, dtype=psi.dtype).contiguous().view(-1)
        if amps.numel() != 2 ** n:
            raise ValueError("amps must have 2^n entries")
        ptr = amps.data_ptr()
    check(lib().tcng_state_init(ctypes.byref(s), ptr, int(basis), _stream()))
    return psi


def apply_gate(psi: torch.Tensor, qubits, U: torch.Tensor):
    """Apply a k-qubit matrix (qubits[0] = most significant local bit) in place."""
    n = _nqubits(psi)
    s = _state(psi, n)
    q = np.ascontiguousarray(np.asarray(qubits, dtype=np.int32).reshape(-1))
    U = U.to(device=psi.device, dtype=psi.dtype).contiguous()
    if U.numel() != 4 ** len(q):
        raise ValueError("U must be 2^k x 2^k")
    check(lib().tcng_apply_gate(ctypes.byref(s), q.ctypes.data_as(ctypes.c_void_p), len(q),
                                ctypes.c_void_p(U.data_ptr()), _stream()))
    return psi


class Circuit:
    """Immutable circuit handle: gate records int32 [G][6] = (kind, q0, q1, p0, p1, mat)."""

    def __init__(self, n: int, gates, n_params: int, mats=None):
        g = np.ascontiguousarray(np.asarray(gates, dtype=np.int32).reshape(-1, 6))
        m = np.zeros((0, 4, 4), np.complex128) if mats is None else np.asarray(mats, dtype=np.complex128)
        m = np.ascontiguousarray(m.reshape(-1, 4, 4))
        h = ctypes.c_void_p()
        check(lib().tcng_circuit_create(int(n), g.ctypes.data_as(ctypes.c_void_p), g.shape[0], int(n_params),
                                        m.ctypes.data_as(ctypes.c_void_p) if m.shape[0] else None, m.shape[0],
                                        ctypes.byref(h)))
        self.handle = h
        self.n, self.n_params, self.n_gates, self.n_mats = int(n), int(n_params), g.shape[0], m.shape[0]
        self.gates = g

    def num_passes(self, dtype=torch.complex64):
        out = ctypes.c_int32()
        check(lib().tcng_circuit_num_passes(self.handle, TCNG_C64 if dtype == torch.complex64 else TCNG_C128,
                                            ctypes.byref(out)))
        return out.value

    def configure(self, dtype, m_max, rb, rb_rev):
        check(lib().tcng_circuit_configure(self.handle, _dt(dtype), int(m_max), int(rb), int(rb_rev)))

    def config(self, dtype=torch.complex64):
        v = [ctypes.c_int32() for _ in range(3)]
        check(lib().tcng_circuit_get_config(self.handle, _dt(dtype), *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def mode(self, dtype=torch.complex64):
        """Name of the mode "auto" runs for this dtype (the autotuner's choice, or the default)."""
        v = ctypes.c_int32()
        check(lib().tcng_circuit_get_mode(self.handle, _dt(dtype), ctypes.byref(v)))
        return MODE_NAMES[v.value]

    def rounds(self, dtype=torch.complex64):
        """Number of rotation-round phases of the tiled plan (0: not on that path)."""
        v = ctypes.c_int32()
        check(lib().tcng_circuit_rounds(self.handle, _dt(dtype), ctypes.byref(v)))
        return v.value

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib._lib is not None:
            _lib._lib.tcng_circuit_destroy(h)
            self.handle = None


def _dt(dtype):
    return TCNG_C64 if dtype in (torch.complex64, "c64", TCNG_C64) else TCNG_C128


def autotune(circ, params, H, psi, lam=None, repeats=3, cache_path=None):
    """Pick the fastest execution mode (tilings of the tiled passes, matrix-core
    passes with 4- or 5-qubit blocks) for this circuit, dtype and batch (see
    tcng_autotune); circ.mode(dtype) names the choice, which mode="auto" runs.
    Returns (tiling of the tiled passes, the winner's median ms)."""
    s = _state(psi, circ.n)
    if lam is None:
        lam = torch.empty_like(psi)
    sl = _state(lam, circ.n)
    p, pp = _params(circ, params, psi, s.batch)
    best = ctypes.c_double()
    check(lib().tcng_autotune(circ.handle, H.handle, pp, ctypes.byref(s), ctypes.byref(sl), int(repeats),
                              cache_path.encode() if cache_path else None, ctypes.byref(best), _stream()))
    return circ.config(psi.dtype), best.value


class PauliSum:
    """Immutable Hamiltonian handle: codes uint8 [T][n] (0=I,1=X,2=Y,3=Z), coefficients float64 [T]."""

    def __init__(self, n: int, codes, coeffs):
        c = np.ascontiguousarray(np.asarray(codes, dtype=np.uint8).reshape(-1, n))
        w = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64).reshape(-1))
        if c.shape[0] != w.shape[0]:
            raise ValueError("codes and coeffs disagree in length")
        h = ctypes.c_void_p()
        check(lib().tcng_pauli_sum_create(int(n), c.ctypes.data_as(ctypes.c_void_p),
                                          w.ctypes.data_as(ctypes.c_void_p), c.shape[0], ctypes.byref(h)))
        self.handle = h
        self.n, self.n_terms = int(n), c.shape[0]
        self.abs_sum = float(np.abs(w).sum())

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib._lib is not None:
            _lib._lib.tcng_pauli_sum_destroy(h)
            self.handle = None


def _workspace(circ, H, dtype_code, batch, mode, device):
    nbytes = ctypes.c_size_t()
    check(lib().tcng_workspace_size(circ.handle if circ is not None else None, H.handle if H is not None else None,
                                    dtype_code, int(batch), mode, ctypes.byref(nbytes)))
    ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=device)
    return ws


def _params(circ, params, psi, batch):
    if circ.n_params == 0:
        return None, None
    rdt = torch.float32 if psi.dtype == torch.complex64 else torch.float64
    p = params.to(device=psi.device, dtype=rdt).reshape(batch, circ.n_params).contiguous()
    return p, ctypes.c_void_p(p.data_ptr())


def run_circuit(circ: Circuit, params, psi: torch.Tensor, mode="tiled", ws=None):
    """Apply the circuit in place to every batch member (params [batch][n_params])."""
    s = _state(psi, circ.n)
    m = _mode(mode)
    p, pp = _params(circ, params, psi, s.batch)
    if ws is None:
        ws = _workspace(circ, None, s.dtype, s.batch, m, psi.device)
    check(lib().tcng_run_circuit(circ.handle, pp, ctypes.byref(s), m, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                 _stream()))
    return psi


def expect_pauli(psi: torch.Tensor, H: PauliSum, mode="tiled", out=None):
    """float64 [batch] of Re <psi|H|psi>."""
    s = _state(psi, H.n)
    m = _mode(mode)
    ws = _workspace(None, H, s.dtype, s.batch, m, psi.device)
    if out is None:
        out = torch.empty(s.batch, dtype=torch.float64, device=psi.device)
    check(lib().tcng_expect_pauli(ctypes.byref(s), H.handle, ctypes.c_void_p(out.data_ptr()), m,
                                  ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return out


def apply_pauli(psi: torch.Tensor, H: PauliSum, out=None, want_energy=False, mode="tiled"):
    """Matrix-free H psi for every batch member (a new tensor unless `out` is
    given); with want_energy also float64 [batch] of Re <psi|H|psi>."""
    s = _state(psi, H.n)
    if out is None:
        out = torch.empty_like(psi)
    o = _state(out, H.n)
    m = _mode(mode)
    ws = _workspace(None, H, s.dtype, s.batch, m, psi.device)
    e = torch.empty(s.batch, dtype=torch.float64, device=psi.device) if want_energy else None
    check(lib().tcng_apply_pauli(ctypes.byref(s), H.handle, ctypes.byref(o),
                                 ctypes.c_void_p(e.data_ptr()) if e is not None else None, m,
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return (out, e) if want_energy else out


def pauli_coo(H: PauliSum, row_begin=0, row_count=None, device="cuda"):
    """Sparse (COO) form of H for rows [row_begin, row_begin + row_count):
    (rows int64, cols int64, vals complex128), group-major (one entry per
    X-mask group and row)."""
    g = ctypes.c_int32()
    check(lib().tcng_pauli_coo_info(H.handle, ctypes.byref(g)))
    count = (1 << H.n) - row_begin if row_count is None else int(row_count)
    m = g.value * count
    rows = torch.empty(m, dtype=torch.int64, device=device)
    cols = torch.empty(m, dtype=torch.int64, device=device)
    vals = torch.empty(m, dtype=torch.complex128, device=device)
    check(lib().tcng_pauli_coo(H.handle, int(row_begin), count, ctypes.c_void_p(rows.data_ptr()) if m else None,
                               ctypes.c_void_p(cols.data_ptr()) if m else None,
                               ctypes.c_void_p(vals.data_ptr()) if m else None, _stream()))
    return rows, cols, vals


def expect_grad(circ: Circuit, params, H: PauliSum, psi=None, lam=None, batch=None, dtype=torch.complex64,
                want_gate_grad=False, mode="tiled", ws=None):
    """E and dE/dtheta (float64) for every parameter set.

    psi: initial states [batch, 2^n] (default |0...0>); it holds the
    recomputed initial states on return.  lam: scratch state of the same shape.
    """
    if psi is None:
        if batch is None:
            batch = 1 if params is None or circ.n_params == 0 else params.numel() // circ.n_params
        psi = new_state(circ.n, batch, dtype)
    s = _state(psi, circ.n)
    if lam is None:
        lam = torch.empty_like(psi)
    sl = _state(lam, circ.n)
    m = _mode(mode)
    if ws is None:
        ws = _workspace(circ, H, s.dtype, s.batch, m, psi.device)
    p, pp = _params(circ, params, psi, s.batch)
    energy = torch.empty(s.batch, dtype=torch.float64, device=psi.device)
    grad = torch.empty((s.batch, max(circ.n_params, 0)), dtype=torch.float64, device=psi.device)
    gg = torch.empty((s.batch, circ.n_gates, 15), dtype=torch.float64, device=psi.device) if want_gate_grad else None
    check(lib().tcng_expect_grad(circ.handle, pp, H.handle, ctypes.byref(s), ctypes.byref(sl),
                                 ctypes.c_void_p(energy.data_ptr()),
                                 ctypes.c_void_p(grad.data_ptr()) if circ.n_params else None,
                                 ctypes.c_void_p(gg.data_ptr()) if gg is not None else None, m,
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    if want_gate_grad:
        return energy, grad, gg
    return energy, grad


def expect_grad_noalloc(circ: Circuit, params, H: PauliSum, psi=None, lam=None, batch=None, dtype=torch.complex64,
                        want_gate_grad=False, mode="tiled"):
    """expect_grad through the allocation-free entry point: the library's
    fixed per-GPU scratch array replaces the workspace (shapes whose workspace
    exceeds it raise).  Calls that overlap on one GPU race on that array."""
    if psi is None:
        if batch is None:
            batch = 1 if params is None or circ.n_params == 0 else params.numel() // circ.n_params
        psi = new_state(circ.n, batch, dtype)
    s = _state(psi, circ.n)
    if lam is None:
        lam = torch.empty_like(psi)
    sl = _state(lam, circ.n)
    m = _mode(mode)
    p, pp = _params(circ, params, psi, s.batch)
    energy = torch.empty(s.batch, dtype=torch.float64, device=psi.device)
    grad = torch.empty((s.batch, max(circ.n_params, 0)), dtype=torch.float64, device=psi.device)
    gg = torch.empty((s.batch, circ.n_gates, 15), dtype=torch.float64, device=psi.device) if want_gate_grad else None
    check(lib().tcng_expect_grad_noalloc(circ.handle, pp, H.handle, ctypes.byref(s), ctypes.byref(sl),
                                         ctypes.c_void_p(energy.data_ptr()),
                                         ctypes.c_void_p(grad.data_ptr()) if circ.n_params else None,
                                         ctypes.c_void_p(gg.data_ptr()) if gg is not None else None, m, _stream()))
    if want_gate_grad:
        return energy, grad, gg
    return energy, grad


def expect_grad_multi(circs, hams, params_list, dtype=torch.complex64, psis=None, want_gate_grad=False, ws=None):
    """Uneven batch: E and gradients of many different circuits in shared launches.

    params_list[i]: device tensor of circuit i's angles (or None); psis: optional
    list of initial states [1, 2^n_i] (default |0...0>).  Returns (energy [count]
    float64, list of gradients, list of gate gradients or None)."""
    count = len(circs)
    dev = torch.device("cuda")
    rdt = torch.float32 if dtype == torch.complex64 else torch.float64
    if psis is None:
        psis = [new_state(c.n, 1, dtype) for c in circs]
    lams = [torch.empty_like(p) for p in psis]
    st_psi = (TcngState * count)(*[_state(p, c.n) for p, c in zip(psis, circs)])
    st_lam = (TcngState * count)(*[_state(l, c.n) for l, c in zip(lams, circs)])
    ch = (ctypes.c_void_p * count)(*[c.handle.value for c in circs])
    hh = (ctypes.c_void_p * count)(*[h.handle.value for h in hams])
    keep = []
    pp = (ctypes.c_void_p * count)()
    grads, ggs = [], []
    gp = (ctypes.c_void_p * count)()
    ggp = (ctypes.c_void_p * count)()
    for i, c in enumerate(circs):
        if c.n_params:
            t = params_list[i].to(device=dev, dtype=rdt).contiguous()
            keep.append(t)
            pp[i] = t.data_ptr()
        g = torch.empty(max(c.n_params, 1), dtype=torch.float64, device=dev)
        grads.append(g[: c.n_params])
        gp[i] = g.data_ptr()
        if want_gate_grad:
            gg = torch.empty((c.n_gates, 15), dtype=torch.float64, device=dev)
            ggs.append(gg)
            ggp[i] = gg.data_ptr()
    dcode = _dt(dtype)
    if ws is None:
        nbytes = ctypes.c_size_t()
        check(lib().tcng_workspace_size_multi(ch, hh, count, dcode, ctypes.byref(nbytes)))
        ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=dev)
    energy = torch.empty(count, dtype=torch.float64, device=dev)
    check(lib().tcng_expect_grad_multi(ch, hh, count, pp, st_psi, st_lam, ctypes.c_void_p(energy.data_ptr()), gp,
                                       ggp if want_gate_grad else None, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                       _stream()))
    return energy, grads, (ggs if want_gate_grad else None)


class Multi:
    """An uneven batch bound once (tcng_multi_*): circuits, Pauli sums, angle
    tensors (written in place between launches), states, outputs and
    workspace.  launch() enqueues one evaluation (kernels only); graph()
    records one as a replayable graph.  init_basis >= 0 starts every circuit
    from that basis state at each launch; -1 from the states' contents."""

    def __init__(self, circs, hams, params_list, dtype=torch.complex64, psis=None, want_gate_grad=False,
                 init_basis=0, ws=None):
        count = len(circs)
        dev = torch.device("cuda")
        rdt = torch.float32 if dtype == torch.complex64 else torch.float64
        self.psis = psis if psis is not None else [new_state(c.n, 1, dtype) for c in circs]
        self.lams = [torch.empty_like(p) for p in self.psis]
        st_psi = (TcngState * count)(*[_state(p, c.n) for p, c in zip(self.psis, circs)])
        st_lam = (TcngState * count)(*[_state(l, c.n) for l, c in zip(self.lams, circs)])
        ch = (ctypes.c_void_p * count)(*[c.handle.value for c in circs])
        hh = (ctypes.c_void_p * count)(*[h.handle.value for h in hams])
        pp = (ctypes.c_void_p * count)()
        gp = (ctypes.c_void_p * count)()
        ggp = (ctypes.c_void_p * count)()
        self.params, self.grads, self.gate_grads = [], [], []
        for i, c in enumerate(circs):
            if c.n_params:
                t = params_list[i]
                if t.dtype != rdt or not t.is_cuda or not t.is_contiguous():
                    raise ValueError("angle tensors must be contiguous device tensors of the run's real type")
                self.params.append(t)
                pp[i] = t.data_ptr()
            g = torch.empty(max(c.n_params, 1), dtype=torch.float64, device=dev)
            self.grads.append(g[: c.n_params])
            gp[i] = g.data_ptr()
            if want_gate_grad:
                gg = torch.empty((c.n_gates, 15), dtype=torch.float64, device=dev)
                self.gate_grads.append(gg)
                ggp[i] = gg.data_ptr()
        if ws is None:
            nbytes = ctypes.c_size_t()
            check(lib().tcng_workspace_size_multi(ch, hh, count, _dt(dtype), ctypes.byref(nbytes)))
            ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=dev)
        self.ws = ws
        self.energy = torch.empty(count, dtype=torch.float64, device=dev)
        self.keep = (circs, hams)
        h = ctypes.c_void_p()
        check(lib().tcng_multi_create(ch, hh, count, pp, st_psi, st_lam, ctypes.c_void_p(self.energy.data_ptr()), gp,
                                      ggp if want_gate_grad else None, int(init_basis),
                                      ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(h)))
        self.handle = h
        self.graph_handle = None

    def launch(self):
        check(lib().tcng_multi_launch(self.handle, _stream()))
        return self.energy, self.grads, (self.gate_grads or None)

    def graph(self):
        """Capture one launch; returns a callable that replays it."""
        g = ctypes.c_void_p()
        check(lib().tcng_graph_create_multi(self.handle, ctypes.byref(g)))
        self.graph_handle = g

        def replay():
            check(lib().tcng_graph_launch(g, _stream()))
            return self.energy, self.grads, (self.gate_grads or None)
        return replay

    def close(self):
        if _lib._lib is None:
            return
        if getattr(self, "graph_handle", None) is not None:
            lib().tcng_graph_destroy(self.graph_handle)
            self.graph_handle = None
        if getattr(self, "handle", None) is not None:
            lib().tcng_multi_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


class Graph:
    """A captured value-and-gradient evaluation (tcng_graph_*): state init to
    |init_basis> (or none if init_basis < 0), forward sweep, H psi and <H>,
    adjoint sweep, final sums.  `params`, `psi`, `lam`, `energy`, `grad` are
    device tensors that stay captured: write new angles into `params` and
    call launch(); the outputs hold the results once the stream reaches them."""

    def __init__(self, circ, params, H, psi, lam, energy, grad, mode="fused", init_basis=0, want_gate_grad=False):
        self.s = _state(psi, circ.n)
        self.sl = _state(lam, circ.n)
        m = _mode(mode)
        self.ws = _workspace(circ, H, self.s.dtype, self.s.batch, m, psi.device)
        self.gg = (torch.empty((self.s.batch, circ.n_gates, 15), dtype=torch.float64, device=psi.device)
                   if want_gate_grad else None)
        self.keep = (circ, params, H, psi, lam, energy, grad)
        h = ctypes.c_void_p()
        check(lib().tcng_graph_create(circ.handle, ctypes.c_void_p(params.data_ptr()) if circ.n_params else None,
                                      H.handle, ctypes.byref(self.s), ctypes.byref(self.sl),
                                      ctypes.c_void_p(energy.data_ptr()),
                                      ctypes.c_void_p(grad.data_ptr()) if circ.n_params else None,
                                      ctypes.c_void_p(self.gg.data_ptr()) if self.gg is not None else None, m,
                                      ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), int(init_basis),
                                      ctypes.byref(h)))
        self.handle = h

    def launch(self):
        check(lib().tcng_graph_launch(self.handle, _stream()))

    def close(self):
        if getattr(self, "handle", None) is not None and _lib._lib is not None:
            lib().tcng_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()


class TcngEnergy(torch.autograd.Function):
    """E(theta) = <psi(theta)|H|psi(theta)> as a differentiable torch op.

    forward runs the whole adjoint sweep once (value and gradient together,
    like the paper's value_and_grad); backward scales the stored gradient.
    params: [batch, n_params] (or [n_params]) float tensor on the device.
    """

    @staticmethod
    def forward(ctx, params, circ, H, dtype=torch.complex64, mode="tiled"):
        p2 = params.detach().reshape(-1, circ.n_params)
        energy, grad = expect_grad(circ, p2, H, batch=p2.shape[0], dtype=dtype, mode=mode)
        ctx.save_for_backward(grad)
        ctx.shape = params.shape
        ctx.pdtype = params.dtype
        out = energy if params.dim() > 1 else energy[0]
        return out.to(params.dtype) if params.dtype != torch.float64 else out

    @staticmethod
    def backward(ctx, gE):
        (grad,) = ctx.saved_tensors
        g = gE.to(torch.float64).reshape(-1, 1) * grad
        return g.reshape(ctx.shape).to(ctx.pdtype), None, None, None, None


def plan_inspect(n, gates, n_params, dtype=torch.complex64):
    """Host-only view of the tiled schedule: (order, pass_of, tile_masks)."""
    g = np.ascontiguousarray(np.asarray(gates, dtype=np.int32).reshape(-1, 6))
    G = g.shape[0]
    order = np.zeros(max(G, 1), np.int32)
    pass_of = np.zeros(max(G, 1), np.int32)
    masks = np.zeros(max(G, 1), np.uint64)
    npass = ctypes.c_int32()
    check(lib().tcng_plan_inspect(int(n), g.ctypes.data_as(ctypes.c_void_p), G, int(n_params),
                                  TCNG_C64 if dtype == torch.complex64 else TCNG_C128,
                                  order.ctypes.data_as(ctypes.c_void_p), pass_of.ctypes.data_as(ctypes.c_void_p),
                                  masks.ctypes.data_as(ctypes.c_void_p), ctypes.byref(npass)))
    k = npass.value
    return order[:G] if k else None, pass_of[:G] if k else None, masks[:k]


def fused_plan_inspect(n, gates, n_params, block_bits=4):
    """Host-only view of the fused schedule (complex64 matrix-core blocks of
    block_bits = 4 or 5 qubits): (order, pass_of, block_of, n_passes, n_blocks, bad_layouts)."""
    g = np.ascontiguousarray(np.asarray(gates, dtype=np.int32).reshape(-1, 6))
    G = g.shape[0]
    order = np.zeros(max(G, 1), np.int32)
    pass_of = np.zeros(max(G, 1), np.int32)
    block_of = np.zeros(max(G, 1), np.int32)
    npass, nblk, bad = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    check(lib().tcng_fused_plan_inspect(int(n), g.ctypes.data_as(ctypes.c_void_p), G, int(n_params), int(block_bits),
                                        order.ctypes.data_as(ctypes.c_void_p), pass_of.ctypes.data_as(ctypes.c_void_p),
                                        block_of.ctypes.data_as(ctypes.c_void_p), ctypes.byref(npass),
                                        ctypes.byref(nblk), ctypes.byref(bad)))
    return order[:G], pass_of[:G], block_of[:G], npass.value, nblk.value, bad.value


def rounds_plan_inspect(n, gates, n_params, tiling=(13, 5, 4)):
    """Host-only view of the rounds of the tiled plan for tiling (tile bits,
    register bits forward, reverse): (n_round_passes, n_phases, bad_layouts)."""
    g = np.ascontiguousarray(np.asarray(gates, dtype=np.int32).reshape(-1, 6))
    rp, nph, bad = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    m, rb, rbr = (int(x) for x in tiling)
    check(lib().tcng_rounds_plan_inspect(int(n), g.ctypes.data_as(ctypes.c_void_p), g.shape[0], int(n_params), m, rb,
                                         rbr, ctypes.byref(rp), ctypes.byref(nph), ctypes.byref(bad)))
    return rp.value, nph.value, bad.value


def mipt_run(step: Circuit, mats: torch.Tensor, psi: torch.Tensor, u: torch.Tensor, p: float, want_margin=False,
             ws=None):
    """Monitored Haar brick-wall trajectories, one per batch member, in place on psi.

    step: Circuit of one time step (U2 gates, no angles); mats: complex64
    [batch][n_steps][step.n_mats][4][4]; psi: complex64 [batch, 2^n] (initial
    states); u: float64 [batch][n_steps][n] uniforms; p: measurement probability.
    Returns (rec int32 [batch][n_steps][2] holding the uint32 measured mask and
    outcome bits, logp float64 [batch], margin float64 [batch][n_steps][n] or None).
    """
    s = _state(psi, step.n)
    batch, n_steps = s.batch, int(u.shape[1]) if u.dim() == 3 else 0
    if mats.dtype != torch.complex64 or not mats.is_contiguous() or u.dtype != torch.float64 or not u.is_contiguous():
        raise ValueError("mats must be contiguous complex64, u contiguous float64")
    if tuple(u.shape) != (batch, n_steps, step.n) or tuple(mats.shape) != (batch, n_steps, step.n_mats, 4, 4):
        raise ValueError("u must be [batch][n_steps][n] and mats [batch][n_steps][n_mats][4][4]")
    dev = psi.device
    rec = torch.empty((batch, n_steps, 2), dtype=torch.int32, device=dev)
    logp = torch.empty(batch, dtype=torch.float64, device=dev)
    margin = torch.full((batch, n_steps, step.n), float("nan"), dtype=torch.float64, device=dev) if want_margin else None
    if ws is None:
        need = ctypes.c_size_t()
        check(lib().tcng_mipt_workspace_size(step.handle, step.n, batch, ctypes.byref(need)))
        ws = torch.empty(max(need.value, 1), dtype=torch.uint8, device=dev)
    check(lib().tcng_mipt_run(step.handle, n_steps, ctypes.c_void_p(mats.data_ptr()), ctypes.byref(s),
                              ctypes.c_void_p(u.data_ptr()), float(p), ctypes.c_void_p(rec.data_ptr()),
                              ctypes.c_void_p(logp.data_ptr()),
                              ctypes.c_void_p(margin.data_ptr()) if margin is not None else None,
                              ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return rec, logp, margin


def shadow_layer(n: int) -> Circuit:
    """The rotation layer of classical-shadow snapshots: U1 on every qubit q
    taking per-snapshot matrix q."""
    g = np.array([[TCNG_U1_KIND, q, -1, -1, -1, q] for q in range(n)], dtype=np.int32)
    return Circuit(n, g, 0, mats=np.tile(np.eye(4), (n, 1, 1)))


def shadow_snapshots(layer: Circuit, psi: torch.Tensor, bases: torch.Tensor, u: torch.Tensor, work=None, ws=None):
    """Classical-shadow snapshots of one complex64 state psi [2^n]: bases uint8
    [S][n] (1=X, 2=Y, 3=Z), u float64 [S].  Returns int64 [S] outcomes (bit q =
    outcome of qubit q); `work` ([S, 2^n] complex64) receives the rotated copies."""
    n, S = layer.n, int(u.shape[0])
    if psi.dtype != torch.complex64 or psi.numel() != 2 ** n or not psi.is_contiguous():
        raise ValueError("psi must be a contiguous complex64 vector of 2^n amplitudes")
    if bases.dtype != torch.uint8 or tuple(bases.shape) != (S, n) or not bases.is_contiguous():
        raise ValueError("bases must be contiguous uint8 [S][n]")
    if u.dtype != torch.float64 or not u.is_contiguous():
        raise ValueError("u must be contiguous float64 [S]")
    if work is None:
        work = torch.empty((S, 2 ** n), dtype=torch.complex64, device=psi.device)
    w = _state(work, n)
    if ws is None:
        need = ctypes.c_size_t()
        check(lib().tcng_shadow_workspace_size(layer.handle, S, ctypes.byref(need)))
        ws = torch.empty(max(need.value, 1), dtype=torch.uint8, device=psi.device)
    out = torch.empty(S, dtype=torch.int64, device=psi.device)
    check(lib().tcng_shadow_snapshots(layer.handle, ctypes.c_void_p(psi.data_ptr()), ctypes.byref(w),
                                      ctypes.c_void_p(bases.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                      _stream()))
    return out


def qml_step(circ: Circuit, theta: torch.Tensor, inputs: torch.Tensor, labels: torch.Tensor, k: int, n_classes: int,
             psi=None, lam=None, ws=None):
    """One SU(4) QML training evaluation: per-sample softmax cross entropy
    (float64 [batch]) and d(mean loss)/dtheta (float64 [n_mats, 15]).
    theta float64 [n_mats, 15]; inputs complex64 [batch, 2^n]; labels int32 [batch]."""
    n, B = circ.n, int(inputs.shape[0])
    if theta.dtype != torch.float64 or tuple(theta.shape) != (circ.n_mats, 15) or not theta.is_contiguous():
        raise ValueError("theta must be contiguous float64 [n_mats, 15]")
    if labels.dtype != torch.int32 or labels.numel() != B or not labels.is_contiguous():
        raise ValueError("labels must be contiguous int32 [batch]")
    x = _state(inputs, n)
    psi = torch.empty_like(inputs) if psi is None else psi
    lam = torch.empty_like(inputs) if lam is None else lam
    p, l = _state(psi, n), _state(lam, n)
    if ws is None:
        need = ctypes.c_size_t()
        check(lib().tcng_qml_workspace_size(circ.handle, B, ctypes.byref(need)))
        ws = torch.empty(max(need.value, 1), dtype=torch.uint8, device=inputs.device)
    loss = torch.empty(B, dtype=torch.float64, device=inputs.device)
    grad = torch.empty((circ.n_mats, 15), dtype=torch.float64, device=inputs.device)
    check(lib().tcng_qml_step(circ.handle, ctypes.c_void_p(theta.data_ptr()), ctypes.byref(x), ctypes.byref(p),
                              ctypes.byref(l), ctypes.c_void_p(labels.data_ptr()), int(k), int(n_classes),
                              ctypes.c_void_p(loss.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
                              ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return loss, grad
