"""Rounds: the complex64 tiled passes of circuits made of RY, RZ and CNOT
(fixed rounds of rotations on 5 register bits, each phase's CNOTs a
permutation of the tile's local index) or of fSim gates and Hadamards (fixed
rounds on register pairs), and circuits mixing them with passes of other
gates (the generic tiled kernels), through the C ABI, against the CPU oracle.

Bars as in test_gpu_parity: |dE| <= 1e-5 S and |d grad|_inf <= 1e-4 S with
S = sum |c_k|; amplitudes within 8 * (gate applications) * 2^-24 of the
state's largest amplitude (tests/bars.py).  Angles are uniform on [0, 2 pi),
so about half of the rotations have cos(theta / 2) < 0 and take the negated
form (-R(a - pi)).
"""
import numpy as np
import pytest
import torch

import workloads as W
from tests.bars import assert_amps

pytestmark = pytest.mark.gpu

TOL = {"c64": (1e-5, 1e-4), "c128": (1e-12, 1e-12)}
TDT = {"c64": torch.complex64, "c128": torch.complex128}
RDT = {"c64": torch.float32, "c128": torch.float64}


@pytest.fixture(scope="module")
def P():
    import paper_2602_14167_amd as pkg
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    pkg.lib()
    return pkg


def ry_rz_cnot_circuit(n, n_gates, rng, low_bias=False):
    """Random RY / RZ / CNOT circuit: each gate's kind and qubits drawn at random
    (CNOT control and target distinct, in either order)."""
    g, npar = [], 0
    for _ in range(n_gates):
        k = rng.integers(3)
        hi = 4 if (low_bias and rng.random() < 0.4) else n
        if k == 2:
            a, b = rng.choice(n if hi == n else max(hi, 2), size=2, replace=False)
            g.append(W.gate(W.CNOT, int(a), int(b)))
        else:
            q = int(rng.integers(hi))
            g.append(W.gate(W.RY if k == 0 else W.RZ, q, p0=npar))
            npar += 1
    return W.as_gate_array(g), npar


def check(P, oracle_mod, n, gates, n_params, codes, coeffs, pb, init, tiling=None, label="", dt="c64"):
    circ = P.Circuit(n, gates, n_params)
    if tiling:
        circ.configure(TDT[dt], *tiling)
    assert circ.rounds(TDT[dt]) > 0, "the circuit should run as rounds"
    H = P.PauliSum(n, codes, coeffs)
    B = pb.shape[0]
    psi = torch.as_tensor(np.tile(init, (B, 1))).to(device="cuda", dtype=TDT[dt])
    psi0 = psi.clone()
    p = torch.as_tensor(pb).to(device="cuda", dtype=RDT[dt])
    E, g = P.expect_grad(circ, p, H, psi=psi, mode="tiled")[:2]
    E, g = E.cpu().numpy(), g.cpu().numpy()
    S = float(np.abs(coeffs).sum())
    worst_e = worst_g = 0.0
    for b in range(B):
        ref = oracle_mod.expect_grad(n, gates, W.round_params(pb[b], dt), codes, coeffs, None, init=init)
        worst_e = max(worst_e, abs(E[b] - ref["E"]) / S)
        worst_g = max(worst_g, float(np.max(np.abs(g[b] - ref["grad"]))) / S)
    print(f"rounds {label} {dt} n={n} gates={len(gates)} phases={circ.rounds(TDT[dt])}: |dE|/S={worst_e:.2e} "
          f"|dg|/S={worst_g:.2e}", flush=True)
    te, tg = TOL[dt]
    assert worst_e <= te and worst_g <= tg, (worst_e, worst_g)
    # the reverse sweep un-computes the states back to the input
    assert_amps(psi.cpu().numpy(), psi0.cpu().numpy(), dt, 8 * len(gates), f"rounds recomputed psi0 {label}")
    # forward only: the final state
    st = torch.empty((1, 2 ** n), dtype=TDT[dt], device="cuda")
    st.copy_(torch.as_tensor(np.ascontiguousarray(init[None, :])))
    P.run_circuit(circ, p[:1].contiguous(), st, mode="tiled")
    ref = oracle_mod.expect_grad(n, gates, W.round_params(pb[0], dt), codes, coeffs, None, init=init,
                                 want_state=True)
    assert_amps(st.cpu().numpy()[0], ref["state"], dt, len(gates), f"rounds final state {label}")


def test_rounds_taken_only_where_they_apply(P):
    w = W.cfg2(n=16, layers=3)
    c = P.Circuit(16, w["gates"], w["n_params"])
    assert c.rounds() > 0 and c.rounds(torch.complex128) > 0
    r = np.random.default_rng(1)
    gates, params, mats = W.random_circuit(14, 40, r)   # every kind: not rotation rounds
    assert P.Circuit(14, gates, len(params), mats).rounds() == 0
    assert P.Circuit(10, w["gates"][:0], 0).rounds() == 0   # below 11 qubits: no 64-lane thread part
    f = W.cfg5(rows=4, cols=4, depth=8)
    assert P.Circuit(16, f["gates"], f["n_params"]).rounds() > 0


@pytest.mark.parametrize("n,layers,tiling", [(11, 2, None), (13, 4, None), (16, 3, None), (16, 3, (12, 5, 5)),
                                             (18, 4, (13, 5, 4)), (18, 3, (13, 4, 4)), (16, 3, (13, 4, 5)),
                                             (12, 3, (12, 4, 4)), (20, 2, None), (17, 3, (13, 5, 5)),
                                             (15, 3, (12, 5, 4)), (15, 3, (12, 4, 5))])
def test_rounds_hea(P, oracle_mod, n, layers, tiling):
    w = W.cfg2(n=n, layers=layers)
    r = np.random.default_rng(100 + n)
    pb = np.stack([w["params"], r.uniform(0, 2 * np.pi, w["n_params"])])
    init = W.random_state(n, r).astype(np.complex64).astype(np.complex128)
    check(P, oracle_mod, n, w["gates"], w["n_params"], w["codes"], w["coeffs"], pb, init, tiling, f"hea L={layers}")


@pytest.mark.parametrize("tiling", [None, (13, 4, 4)])
@pytest.mark.parametrize("n,n_gates,seed", [(11, 60, 1), (12, 120, 2), (13, 150, 3), (14, 150, 4), (16, 200, 5)])
def test_rounds_random_ry_rz_cnot(P, oracle_mod, n, n_gates, seed, tiling):
    """Register blocks of 5 (the default tiling) and of 4 bits per thread."""
    r = np.random.default_rng(seed)
    gates, npar = ry_rz_cnot_circuit(n, n_gates, r, low_bias=(seed % 2 == 0))
    codes, coeffs = W.random_pauli_sum(n, 12, r, max_weight=4)
    pb = r.uniform(0, 2 * np.pi, (2, npar))
    init = W.random_state(n, r).astype(np.complex64).astype(np.complex128)
    check(P, oracle_mod, n, gates, npar, codes, coeffs, pb, init, tiling, f"random seed={seed} tiling={tiling}")


# ---------------------------------------------------------------------------
# fSim rounds: passes of fSim gates and Hadamards (pair slots (0,1), (2,3),
# then (1,2), (3,4) of a chain of register qubits)
# ---------------------------------------------------------------------------
def fsim_h_circuit(n, n_gates, rng, nearest=False):
    """Random fSim / Hadamard circuit: about a fifth Hadamards; fSim pairs
    random (or nearest neighbours), in either order, angles uniform."""
    g, npar = [], 0
    for _ in range(n_gates):
        if rng.random() < 0.2:
            g.append(W.gate(W.H, int(rng.integers(n))))
            continue
        if nearest:
            a = int(rng.integers(n - 1))
            q0, q1 = (a, a + 1) if rng.random() < 0.5 else (a + 1, a)
        else:
            q0, q1 = (int(v) for v in rng.choice(n, size=2, replace=False))
        g.append(W.gate(W.FSIM, q0, q1, p0=npar, p1=npar + 1))
        npar += 2
    return W.as_gate_array(g), npar


@pytest.mark.parametrize("rows,cols,depth,tiling", [(3, 4, 8, None), (2, 7, 10, None), (4, 4, 12, None),
                                                    (4, 4, 12, (13, 4, 4)), (3, 6, 10, (13, 5, 4)),
                                                    (3, 6, 10, (12, 5, 5)), (4, 5, 6, (12, 4, 4)),
                                                    (4, 4, 12, (13, 5, 5)), (3, 5, 10, (12, 4, 5))])
def test_fsim_rounds_brickwork(P, oracle_mod, rows, cols, depth, tiling):
    """The fSim brick-wall workload (Hadamard layer, depth-d fSim brick wall,
    2D TFIM) on small lattices."""
    w = W.cfg5(rows=rows, cols=cols, depth=depth)
    n = w["n"]
    r = np.random.default_rng(200 + n + depth)
    pb = np.stack([w["params"], r.uniform(0, 2 * np.pi, w["n_params"])])
    init = W.random_state(n, r).astype(np.complex64).astype(np.complex128)
    check(P, oracle_mod, n, w["gates"], w["n_params"], w["codes"], w["coeffs"], pb, init, tiling,
          f"fsim {rows}x{cols} d={depth}")


@pytest.mark.parametrize("tiling", [None, (13, 4, 4)])
@pytest.mark.parametrize("n,n_gates,seed,nearest", [(11, 60, 1, True), (12, 90, 2, False), (13, 120, 3, True),
                                                    (14, 120, 4, False), (16, 160, 5, True)])
def test_fsim_rounds_random(P, oracle_mod, n, n_gates, seed, nearest, tiling):
    r = np.random.default_rng(300 + seed)
    gates, npar = fsim_h_circuit(n, n_gates, r, nearest)
    codes, coeffs = W.random_pauli_sum(n, 12, r, max_weight=4)
    pb = r.uniform(0, 2 * np.pi, (2, npar))
    init = W.random_state(n, r).astype(np.complex64).astype(np.complex128)
    check(P, oracle_mod, n, gates, npar, codes, coeffs, pb, init, tiling, f"fsim random seed={seed}")


@pytest.mark.parametrize("n", [15, 16])
def test_rounds_mixed_with_generic_passes(P, oracle_mod, n):
    """fSim-round, rotation-round and generic passes in one circuit (11-bit
    tiles: the planner's passes of these sizes take all three kinds): a
    12-layer fSim brick wall, 8 HEA layers (RY, RZ on every qubit, a CNOT
    chain), then RX on every qubit (no rounds kind)."""
    r = np.random.default_rng(400 + n)
    g, npar = [], 0
    for L in range(12):
        for i in range(L % 2, n - 1, 2):
            g.append(W.gate(W.FSIM, i, i + 1, p0=npar, p1=npar + 1))
            npar += 2
    for L in range(8):
        for q in range(n):
            g.append(W.gate(W.RY, q, p0=npar))
            g.append(W.gate(W.RZ, q, p0=npar + 1))
            npar += 2
        for q in range(n - 1):
            g.append(W.gate(W.CNOT, q, q + 1))
    for q in range(n):
        g.append(W.gate(W.RX, q, p0=npar))
        npar += 1
    gates = W.as_gate_array(g)
    codes, coeffs = W.random_pauli_sum(n, 12, r, max_weight=4)
    pb = r.uniform(0, 2 * np.pi, (2, npar))
    init = W.random_state(n, r).astype(np.complex64).astype(np.complex128)
    check(P, oracle_mod, n, gates, npar, codes, coeffs, pb, init, (11, 5, 4), "mixed")


# ---------------------------------------------------------------------------
# complex128 rounds (12- or 11-bit tiles, 3 or 4 register bits per sweep)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,layers,tiling", [(11, 2, None), (13, 3, None), (16, 3, None), (16, 3, (12, 4, 4)),
                                             (15, 3, (11, 4, 4)), (14, 3, (12, 3, 3)), (14, 3, (11, 3, 4))])
def test_rounds_hea_c128(P, oracle_mod, n, layers, tiling):
    w = W.cfg2(n=n, layers=layers)
    r = np.random.default_rng(500 + n)
    pb = np.stack([w["params"], r.uniform(0, 2 * np.pi, w["n_params"])])
    init = W.random_state(n, r)
    check(P, oracle_mod, n, w["gates"], w["n_params"], w["codes"], w["coeffs"], pb, init, tiling,
          f"hea L={layers}", "c128")


@pytest.mark.parametrize("n,n_gates,seed", [(11, 60, 1), (14, 150, 4)])
def test_rounds_random_ry_rz_cnot_c128(P, oracle_mod, n, n_gates, seed):
    r = np.random.default_rng(600 + seed)
    gates, npar = ry_rz_cnot_circuit(n, n_gates, r, low_bias=(seed % 2 == 0))
    codes, coeffs = W.random_pauli_sum(n, 12, r, max_weight=4)
    pb = r.uniform(0, 2 * np.pi, (2, npar))
    init = W.random_state(n, r)
    check(P, oracle_mod, n, gates, npar, codes, coeffs, pb, init, None, f"random seed={seed}", "c128")


@pytest.mark.parametrize("rows,cols,depth,tiling", [(3, 4, 8, None), (4, 4, 10, None), (4, 4, 10, (12, 4, 4)),
                                                    (3, 5, 8, (11, 3, 4))])
def test_fsim_rounds_c128(P, oracle_mod, rows, cols, depth, tiling):
    w = W.cfg5(rows=rows, cols=cols, depth=depth)
    n = w["n"]
    r = np.random.default_rng(700 + n)
    pb = np.stack([w["params"], r.uniform(0, 2 * np.pi, w["n_params"])])
    init = W.random_state(n, r)
    check(P, oracle_mod, n, w["gates"], w["n_params"], w["codes"], w["coeffs"], pb, init, tiling,
          f"fsim {rows}x{cols} d={depth}", "c128")
