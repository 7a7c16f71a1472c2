"""Pins of the oracle's Pauli-sum COO construction (no GPU).

The entries are checked against dense Kronecker-product Hamiltonians
(tests/bruteforce.py), Hermiticity, the oracle's separately pinned H psi, and
the group count; none of these shares the oracle's code path.
"""
import numpy as np
import pytest

import workloads as W
from tests import bruteforce as B


def scatter(n, rows, cols, vals):
    d = np.zeros((2 ** n, 2 ** n), np.complex128)
    np.add.at(d, (rows, cols), vals)
    return d


def cases():
    r = np.random.default_rng(41)
    out = []
    for n in (1, 3, 5, 6):
        codes, coeffs = W.random_pauli_sum(n, 9, r)
        codes = np.vstack([codes, codes[:2], np.zeros((1, n), np.uint8)])   # repeated X-masks, identity
        coeffs = np.concatenate([coeffs, r.normal(size=3)])
        out.append((n, codes, coeffs))
    codes, coeffs = W.tfim_1d(6, 1.0, 0.7)
    out.append((6, codes, coeffs))
    return out


@pytest.mark.parametrize("case", range(5))
def test_coo_equals_the_dense_hamiltonian(oracle_mod, case):
    n, codes, coeffs = cases()[case]
    rows, cols, vals, G = oracle_mod.pauli_coo(n, codes, coeffs)
    xmasks = {int(sum((c in (1, 2)) << q for q, c in enumerate(row))) for row in codes}
    assert G == len(xmasks)
    assert len(rows) == G * 2 ** n
    np.testing.assert_allclose(scatter(n, rows, cols, vals), B.dense_hamiltonian(codes, coeffs), atol=1e-13)
    # each entry sits at col = row xor (its group's X-mask), rows ascending within a group
    for g in range(G):
        seg = slice(g * 2 ** n, (g + 1) * 2 ** n)
        np.testing.assert_array_equal(rows[seg], np.arange(2 ** n))
        assert len(set((rows[seg] ^ cols[seg]).tolist())) == 1


@pytest.mark.parametrize("case", range(5))
def test_coo_is_hermitian_and_applies_h(oracle_mod, case):
    n, codes, coeffs = cases()[case]
    rows, cols, vals, G = oracle_mod.pauli_coo(n, codes, coeffs)
    ent = {(int(r), int(c)): v for r, c, v in zip(rows, cols, vals)}
    for (r, c), v in ent.items():
        assert ent[(c, r)] == pytest.approx(np.conj(v), abs=1e-13)
    psi = W.random_state(n, np.random.default_rng(42 + case))
    hpsi = np.zeros(2 ** n, np.complex128)
    np.add.at(hpsi, rows, vals * psi[cols])
    np.testing.assert_allclose(hpsi, oracle_mod.apply_hamiltonian(n, psi, codes, coeffs), atol=1e-13)


def test_coo_row_ranges_concatenate(oracle_mod):
    n, codes, coeffs = cases()[3]
    full = oracle_mod.pauli_coo(n, codes, coeffs)
    G = full[3]
    parts = [oracle_mod.pauli_coo(n, codes, coeffs, b, c) for b, c in ((0, 7), (7, 40), (47, 17))]
    for g in range(G):
        got = np.concatenate([p[2][g * len(p[0]) // G:(g + 1) * len(p[0]) // G] for p in parts])
        np.testing.assert_array_equal(got, full[2][g * 2 ** n:(g + 1) * 2 ** n])
