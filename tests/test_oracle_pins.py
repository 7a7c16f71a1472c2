"""Pins of the CPU oracle against the mathematics (no GPU).

Each check reaches the same quantity by a route that shares nothing with the
oracle's code: matrix exponentials of generators, tensor contraction on a
[2]*n array, dense Kronecker-product Hamiltonians, exact diagonalisation,
closed forms, and the free-fermion solution of the open transverse-field Ising
chain.  A dropped term, a wrong sign, a transposed gate or a swapped qubit
order in the oracle fails at least one of them.
"""
import numpy as np
import pytest

import workloads as W
from tests import bruteforce as B


def rng(seed):
    return np.random.default_rng(seed)


# --------------------------------------------------------------------------
# gate matrices
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind", range(14))
def test_gate_matrix_matches_generator_exponential(oracle_mod, kind):
    r = rng(100 + kind)
    params = r.uniform(0, 2 * np.pi, size=2)
    mats = np.stack([W.haar_u4(r), W.haar_u4(r)])
    two = kind in W.TWO_QUBIT
    rec = W.gate(kind, 0, 1 if two else -1,
                 p0=0 if kind in W.PARAM_COUNT else -1,
                 p1=1 if W.PARAM_COUNT.get(kind) == 2 else -1,
                 mat=1 if kind in (W.U1, W.U2) else -1)
    got = oracle_mod.gate_matrix(rec, params, mats)
    ref = B.gate_unitary(np.array(rec), params, mats)
    k = ref.shape[0]
    np.testing.assert_allclose(got[:k, :k], ref, atol=1e-14)
    if kind not in (W.U1,):
        np.testing.assert_allclose(got[:k, :k].conj().T @ got[:k, :k], np.eye(k), atol=1e-14)


def test_textbook_cnot_layout(oracle_mod):
    """qubits = (control, target), control is the MSB of the local index."""
    cx = oracle_mod.gate_matrix(W.gate(W.CNOT, 0, 1))
    np.testing.assert_array_equal(cx.real, [[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]])


# --------------------------------------------------------------------------
# gate application
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_random_circuits_match_tensor_contraction(oracle_mod, n):
    r = rng(200 + n)
    for trial in range(3):
        gates, params, mats = W.random_circuit(n, 25, r)
        init = W.random_state(n, r)
        got = oracle_mod.run(n, gates, params, mats, init)
        ref = B.run_tn(n, gates, params, mats, init)
        np.testing.assert_allclose(got, ref, atol=1e-13)


@pytest.mark.parametrize("q", [0, 2, 4])
def test_one_qubit_gate_matches_kronecker_product(oracle_mod, q):
    n = 5
    r = rng(300 + q)
    U = W.haar_u4(r)[:2, :2]
    w, _, vh = np.linalg.svd(U)
    U = w @ vh
    psi = W.random_state(n, r)
    got = oracle_mod.apply_matrix(n, psi, [q], U)
    np.testing.assert_allclose(got, B.embed_1q(n, U, q) @ psi, atol=1e-14)


def test_two_qubit_gate_order_adjacent_kronecker(oracle_mod):
    """A gate on (q+1, q) is kron(I, U, I) with U's first factor on q+1."""
    n = 5
    r = rng(310)
    U = W.haar_u4(r)
    psi = W.random_state(n, r)
    q = 1
    full = np.kron(np.kron(np.eye(2 ** (n - q - 2)), U), np.eye(2 ** q))
    got = oracle_mod.apply_matrix(n, psi, [q + 1, q], U)
    np.testing.assert_allclose(got, full @ psi, atol=1e-14)
    # reversed order = the same gate conjugated by SWAP
    SW = np.eye(4)[[0, 2, 1, 3]]
    got2 = oracle_mod.apply_matrix(n, psi, [q, q + 1], U)
    full2 = np.kron(np.kron(np.eye(2 ** (n - q - 2)), SW @ U @ SW), np.eye(2 ** q))
    np.testing.assert_allclose(got2, full2 @ psi, atol=1e-14)


def test_bell_and_ghz(oracle_mod):
    g = [W.gate(W.H, 0), W.gate(W.CNOT, 0, 1)]
    psi = oracle_mod.run(2, g)
    np.testing.assert_allclose(psi, [2 ** -0.5, 0, 0, 2 ** -0.5], atol=1e-15)
    for n in (3, 7, 12):
        g = [W.gate(W.H, 0)] + [W.gate(W.CNOT, i, i + 1) for i in range(n - 1)]
        psi = oracle_mod.run(n, g)
        ref = np.zeros(2 ** n)
        ref[0] = ref[-1] = 2 ** -0.5
        np.testing.assert_allclose(psi, ref, atol=1e-15)


def test_x_and_cnot_ladder_on_basis_states(oracle_mod):
    """CNOT ladder (i -> i+1, increasing i) maps |b> to the prefix-XOR of b."""
    n = 9
    r = rng(320)
    for _ in range(5):
        b = int(r.integers(2 ** n))
        g = [W.gate(W.X, q) for q in range(n) if (b >> q) & 1]
        g += [W.gate(W.CNOT, i, i + 1) for i in range(n - 1)]
        psi = oracle_mod.run(n, g)
        img, acc = 0, 0
        for q in range(n):
            acc ^= (b >> q) & 1
            img |= acc << q
        assert abs(psi[img] - 1) < 1e-15 and np.count_nonzero(np.abs(psi) > 1e-15) == 1


def test_norm_preserved_and_inverse_circuit(oracle_mod):
    n = 8
    r = rng(330)
    gates, params, mats = W.random_circuit(n, 60, r, kinds=[k for k in range(14) if k != W.U1])
    psi = oracle_mod.run(n, gates, params, mats)
    assert abs(oracle_mod.norm2(n, psi) - 1) < 1e-13
    # inverse circuit: reversed order, each gate replaced by its adjoint (as a U2/U1 constant)
    inv, inv_mats = [], []
    for rec in gates[::-1]:
        U = oracle_mod.gate_matrix(rec, params, mats)
        k = 2 if rec[2] >= 0 else 1
        M = np.zeros((4, 4), np.complex128)
        M[: 2 ** k, : 2 ** k] = U[: 2 ** k, : 2 ** k].conj().T
        inv_mats.append(M)
        inv.append(W.gate(W.U2 if k == 2 else W.U1, rec[1], rec[2], mat=len(inv_mats) - 1))
    back = oracle_mod.run(n, inv, None, np.array(inv_mats), psi)
    ref = np.zeros(2 ** n)
    ref[0] = 1
    np.testing.assert_allclose(back, ref, atol=1e-13)


# --------------------------------------------------------------------------
# Pauli expectations
# --------------------------------------------------------------------------

def test_single_qubit_closed_forms(oracle_mod):
    for th in (0.3, 1.7, 4.0):
        p = np.array([th])
        psi = oracle_mod.run(1, [W.gate(W.RY, 0, p0=0)], p)
        assert abs(oracle_mod.expect(1, psi, [[3]], [1.0]) - np.cos(th)) < 1e-15
        assert abs(oracle_mod.expect(1, psi, [[1]], [1.0]) - np.sin(th)) < 1e-15
        psi = oracle_mod.run(1, [W.gate(W.RX, 0, p0=0)], p)
        assert abs(oracle_mod.expect(1, psi, [[2]], [1.0]) + np.sin(th)) < 1e-15
        # RZ on |+>: Bloch vector rotates about z by +theta
        psi = oracle_mod.run(1, [W.gate(W.H, 0), W.gate(W.RZ, 0, p0=0)], p)
        assert abs(oracle_mod.expect(1, psi, [[1]], [1.0]) - np.cos(th)) < 1e-15
        assert abs(oracle_mod.expect(1, psi, [[2]], [1.0]) - np.sin(th)) < 1e-15


def test_ghz_pauli_phases(oracle_mod):
    n = 6
    g = [W.gate(W.H, 0)] + [W.gate(W.CNOT, i, i + 1) for i in range(n - 1)]
    psi = oracle_mod.run(n, g)
    allx = np.ones((1, n), np.uint8)
    assert abs(oracle_mod.expect(n, psi, allx, [1.0]) - 1) < 1e-14
    yyx = np.ones((1, n), np.uint8)
    yyx[0, :2] = 2
    assert abs(oracle_mod.expect(n, psi, yyx, [1.0]) + 1) < 1e-14
    zz = np.zeros((1, n), np.uint8)
    zz[0, [1, 4]] = 3
    assert abs(oracle_mod.expect(n, psi, zz, [1.0]) - 1) < 1e-14
    z1 = np.zeros((1, n), np.uint8)
    z1[0, 2] = 3
    assert abs(oracle_mod.expect(n, psi, z1, [1.0])) < 1e-14


def test_basis_state_expectations(oracle_mod):
    n = 7
    r = rng(400)
    for _ in range(10):
        b = int(r.integers(2 ** n))
        psi = np.zeros(2 ** n, np.complex128)
        psi[b] = 1
        codes, coeffs = W.random_pauli_sum(n, 6, r)
        e = oracle_mod.expect(n, psi, codes, coeffs)
        ref = 0.0
        for row, c in zip(codes, coeffs):
            if np.any((row == 1) | (row == 2)):
                continue
            z = sum(1 << q for q in range(n) if row[q] == 3)
            ref += c * (-1) ** bin(b & z).count("1")
        assert abs(e - ref) < 1e-14


@pytest.mark.parametrize("n", [1, 3, 5, 8])
def test_expectation_and_h_apply_match_dense_kronecker(oracle_mod, n):
    r = rng(500 + n)
    codes, coeffs = W.random_pauli_sum(n, 12, r)
    Hm = B.dense_hamiltonian(codes, coeffs)
    for _ in range(2):
        psi = W.random_state(n, r)
        e = oracle_mod.expect(n, psi, codes, coeffs)
        ref = np.vdot(psi, Hm @ psi)
        assert abs(e - ref) < 1e-13
        assert abs(e.imag) < 1e-13
        np.testing.assert_allclose(oracle_mod.apply_hamiltonian(n, psi, codes, coeffs), Hm @ psi, atol=1e-13)


@pytest.mark.parametrize("n,J,h", [(6, 1.0, 1.0), (8, 1.0, 0.5), (10, 1.0, 3.04)])
def test_tfim_ground_energy_exact_diagonalisation(oracle_mod, n, J, h):
    """ED eigenvector of the dense Kronecker H, evaluated by the oracle, gives
    the free-fermion ground energy; the sign-flipped H (+J, +h) has the same
    spectrum on an open chain."""
    codes, coeffs = W.tfim_1d(n, -J, -h)
    Hm = B.dense_hamiltonian(codes, coeffs)
    w, v = np.linalg.eigh(Hm)
    e0 = B.tfim_open_e0_free_fermion(n, J, h)
    assert abs(w[0] - e0) < 1e-10
    assert abs(oracle_mod.expect(n, v[:, 0], codes, coeffs).real - e0) < 1e-10
    codes2, coeffs2 = W.tfim_1d(n, J, h)
    w2 = np.linalg.eigvalsh(B.dense_hamiltonian(codes2, coeffs2))
    assert abs(w2[0] - e0) < 1e-10


def test_product_state_closed_form_tfim(oracle_mod):
    """HEA with one layer and no CNOTs is a product state with Bloch vector
    (sin t cos f, sin t sin f, cos t) per qubit."""
    n = 7
    r = rng(600)
    gates, npar = W.hea_gates(n, 1, cnot=False)
    params = r.uniform(0, 2 * np.pi, npar)
    t, f = params[:n], params[n:]
    bx, by, bz = np.sin(t) * np.cos(f), np.sin(t) * np.sin(f), np.cos(t)
    codes, coeffs = W.xxz_1d(n, 0.7)
    ref = sum(bx[i] * bx[i + 1] + by[i] * by[i + 1] + 0.7 * bz[i] * bz[i + 1] for i in range(n - 1))
    psi = oracle_mod.run(n, gates, params)
    assert abs(oracle_mod.expect(n, psi, codes, coeffs) - ref) < 1e-13


# --------------------------------------------------------------------------
# gradients
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [2, 4, 6])
def test_adjoint_matches_parameter_shift_all_kinds(oracle_mod, n):
    r = rng(700 + n)
    gates, params, mats = W.random_circuit(n, 30, r)
    codes, coeffs = W.random_pauli_sum(n, 8, r)
    # share one parameter between two gates to pin the summation over uses
    pidx = [i for i, g in enumerate(gates) if g[3] >= 0]
    if len(pidx) >= 2:
        gates[pidx[1], 3] = gates[pidx[0], 3]
    init = W.random_state(n, r)
    a = oracle_mod.expect_grad(n, gates, params, codes, coeffs, mats, init, want_lie=True)
    s = oracle_mod.param_shift(n, gates, params, codes, coeffs, mats, init, want_lie=True)
    S = np.abs(coeffs).sum()
    assert np.max(np.abs(a["grad"] - s["grad"])) < 1e-12 * S
    assert np.max(np.abs(a["lie"] - s["lie"])) < 1e-12 * S
    assert abs(a["E_imag"]) < 1e-13


def test_adjoint_energy_and_gradient_vs_dense_finite_differences(oracle_mod):
    """Central differences of <psi|H|psi> computed with the tensor-contraction
    simulator and the dense Kronecker H (h = 1e-5: agreement ~1e-9)."""
    n = 5
    r = rng(800)
    gates, params, mats = W.random_circuit(n, 20, r)
    codes, coeffs = W.random_pauli_sum(n, 6, r)
    Hm = B.dense_hamiltonian(codes, coeffs)

    def energy(p):
        psi = B.run_tn(n, gates, p, mats)
        return np.vdot(psi, Hm @ psi).real

    a = oracle_mod.expect_grad(n, gates, params, codes, coeffs, mats)
    assert abs(a["E"] - energy(params)) < 1e-13
    h = 1e-5
    fd = np.array([(energy(params + h * e) - energy(params - h * e)) / (2 * h) for e in np.eye(len(params))])
    assert np.max(np.abs(fd - a["grad"])) < 1e-8


def test_matrix_cotangent_vs_finite_differences(oracle_mod):
    """dE = 2 Re tr(G^dag dU): perturb one entry of a constant gate matrix."""
    n = 4
    r = rng(810)
    gates, mats = W.brickwork_haar(n, 3, r)
    codes, coeffs = W.random_2local(n, 6, r)
    a = oracle_mod.expect_grad(n, gates, None, codes, coeffs, mats, want_cot=True)
    h = 1e-6
    for gi, (ai, bi) in [(0, (1, 2)), (3, (0, 3)), (len(gates) - 1, (2, 2))]:
        for dz, part in ((1.0, "re"), (1j, "im")):
            mp, mm = mats.copy(), mats.copy()
            mp[gi, ai, bi] += h * dz
            mm[gi, ai, bi] -= h * dz
            ep = oracle_mod.expect(n, oracle_mod.run(n, gates, None, mp), codes, coeffs).real
            em = oracle_mod.expect(n, oracle_mod.run(n, gates, None, mm), codes, coeffs).real
            fd = (ep - em) / (2 * h)
            G = a["cot"][gi, ai, bi]
            ref = 2 * G.real if part == "re" else 2 * G.imag
            assert abs(fd - ref) < 1e-8


def test_gradient_vanishes_at_eigenstate(oracle_mod):
    """theta = 0 HEA without CNOTs leaves |0..0>, an eigenvector of -sum ZZ."""
    n = 6
    gates, npar = W.hea_gates(n, 2, cnot=False)
    codes, coeffs = W.tfim_1d(n, -1.0, 0.0)
    a = oracle_mod.expect_grad(n, gates, np.zeros(npar), codes, coeffs)
    assert abs(a["E"] + (n - 1)) < 1e-14
    assert np.max(np.abs(a["grad"])) < 1e-14


def test_product_state_gradient_closed_form(oracle_mod):
    """Analytic gradient of the one-layer product-state TFIM energy."""
    n = 6
    r = rng(820)
    gates, npar = W.hea_gates(n, 1, cnot=False)
    params = r.uniform(0, 2 * np.pi, npar)
    J, h = -1.0, -0.5
    codes, coeffs = W.tfim_1d(n, J, h)
    t, f = params[:n], params[n:]
    bz = np.cos(t)
    bx = np.sin(t) * np.cos(f)
    dbz_dt = -np.sin(t)
    dbx_dt = np.cos(t) * np.cos(f)
    dbx_df = -np.sin(t) * np.sin(f)
    gt = np.zeros(n)
    gf = np.zeros(n)
    for i in range(n):
        nb = (bz[i - 1] if i > 0 else 0.0) + (bz[i + 1] if i < n - 1 else 0.0)
        gt[i] = J * dbz_dt[i] * nb + h * dbx_dt[i]
        gf[i] = h * dbx_df[i]
    a = oracle_mod.expect_grad(n, gates, params, codes, coeffs)
    np.testing.assert_allclose(a["grad"], np.concatenate([gt, gf]), atol=1e-13)


@pytest.mark.parametrize("k", [3, 4, 5])
def test_k_qubit_matrix_matches_tensor_contraction(oracle_mod, k):
    n = 7
    r = rng(900 + k)
    qs = [int(v) for v in r.choice(n, size=k, replace=False)]
    A = r.standard_normal((2 ** k, 2 ** k)) + 1j * r.standard_normal((2 ** k, 2 ** k))
    psi = W.random_state(n, r)
    got = oracle_mod.apply_matrix(n, psi, qs, A)
    np.testing.assert_allclose(got, B.apply_tn(psi, n, A, qs), atol=1e-12)
