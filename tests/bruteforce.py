"""Textbook reference constructions used to pin the oracle (tests only).

Everything here is built a different way from the oracle: gate matrices come
from matrix exponentials of their generators (scipy.linalg.expm), states are
evolved by tensor contraction on a [2]*n reshaped array (the paper's "gate
application = local tensor contraction"), and Hamiltonians are dense Kronecker
products of 2x2 Pauli matrices.
"""
from functools import reduce

import numpy as np
from scipy.linalg import expm

import workloads as W

I2 = np.eye(2, dtype=np.complex128)
PX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
PAULI = [I2, PX, PY, PZ]


def gate_unitary(rec, params, mats):
    kind = int(rec[0])
    p0 = params[rec[3]] if rec[3] >= 0 else None
    p1 = params[rec[4]] if rec[4] >= 0 else None
    if kind == W.RX:
        return expm(-0.5j * p0 * PX)
    if kind == W.RY:
        return expm(-0.5j * p0 * PY)
    if kind == W.RZ:
        return expm(-0.5j * p0 * PZ)
    if kind == W.H:
        return (PX + PZ) / np.sqrt(2)
    if kind == W.X:
        return PX
    if kind == W.Y:
        return PY
    if kind == W.Z:
        return PZ
    if kind == W.S:
        return expm(0.25j * np.pi * (I2 - PZ))        # diag(1, i)
    if kind == W.CNOT:
        P1 = (I2 - PZ) / 2
        P0 = (I2 + PZ) / 2
        return np.kron(P0, I2) + np.kron(P1, PX)      # control = first (MSB) factor
    if kind == W.CZ:
        return expm(0.25j * np.pi * (np.kron(I2, I2) - np.kron(PZ, I2) - np.kron(I2, PZ) + np.kron(PZ, PZ))) \
            * 1.0
    if kind == W.RZZ:
        return expm(-0.5j * p0 * np.kron(PZ, PZ))
    if kind == W.FSIM:
        gen = 0.5 * (np.kron(PX, PX) + np.kron(PY, PY))
        p11 = np.diag([0, 0, 0, 1]).astype(np.complex128)
        return expm(-1j * p0 * gen) @ expm(-1j * p1 * p11)
    if kind == W.U1:
        return np.asarray(mats[rec[5]])[:2, :2]
    if kind == W.U2:
        return np.asarray(mats[rec[5]])
    raise ValueError(kind)


def apply_tn(state, n, U, qubits):
    """Contract a k-qubit gate tensor with the state tensor.  Axis a of the
    [2]*n tensor is qubit n-1-a (qubit 0 = least significant index bit);
    the gate's first qubit is its most significant local index."""
    k = len(qubits)
    psi = np.asarray(state, dtype=np.complex128).reshape([2] * n)
    axes = [n - 1 - q for q in qubits]
    Ut = np.asarray(U, dtype=np.complex128).reshape([2] * (2 * k))
    psi = np.tensordot(Ut, psi, axes=(list(range(k, 2 * k)), axes))
    psi = np.moveaxis(psi, list(range(k)), axes)
    return psi.reshape(-1)


def run_tn(n, gates, params=None, mats=None, init=None):
    psi = np.zeros(2 ** n, np.complex128)
    if init is None:
        psi[0] = 1
    else:
        psi[:] = init
    for rec in np.asarray(gates).reshape(-1, 6):
        qs = [int(rec[1])] if rec[2] < 0 else [int(rec[1]), int(rec[2])]
        psi = apply_tn(psi, n, gate_unitary(rec, params, mats), qs)
    return psi


def embed_1q(n, U, q):
    """Full 2^n x 2^n operator of a one-qubit gate by Kronecker products."""
    return reduce(np.kron, [U if i == q else I2 for i in reversed(range(n))])


def pauli_string_matrix(code_row):
    n = len(code_row)
    return reduce(np.kron, [PAULI[int(code_row[q])] for q in reversed(range(n))])


def dense_hamiltonian(codes, coeffs):
    codes = np.asarray(codes)
    n = codes.shape[1]
    Hm = np.zeros((2 ** n, 2 ** n), np.complex128)
    for row, c in zip(codes, coeffs):
        Hm += c * pauli_string_matrix(row)
    return Hm


def tfim_open_e0_free_fermion(n, J, h):
    """Ground energy of -J sum Z_i Z_{i+1} - h sum X_i on an open chain from the
    Jordan-Wigner / Bogoliubov solution (Pfeuty 1970): E0 = -sum_k s_k with
    s_k the singular values of the n x n bidiagonal matrix diag(h) + J on the
    superdiagonal."""
    M = np.diag([h] * n) + np.diag([J] * (n - 1), 1)
    return -np.linalg.svd(M, compute_uv=False).sum()
