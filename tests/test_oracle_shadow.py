"""Pins of the oracle's classical-shadow snapshots (no GPU).

Eigenstates fix the basis rotations (a Y-eigenstate measured in the Y basis
gives outcome 0, which pins the sign of the S^dagger), GHZ parities and
product-state frequencies pin the Born draw, the shadow estimator of a
two-qubit Pauli reproduces the exact expectation, and the drawn outcome's
probability equals that of the Kronecker-product rotation of the state.
"""
import numpy as np
import pytest

import workloads as W

H2 = np.array([[1, 1], [1, -1]]) / np.sqrt(2)
V = {1: H2, 2: H2 @ np.diag([1, -1j]), 3: np.eye(2)}


def kron_rotation(bases_row):
    out = np.array([[1.0 + 0j]])
    for b in reversed(list(bases_row)):   # qubit 0 is the least significant bit
        out = np.kron(out, V[int(b)])
    return out


def product(vecs):
    out = np.array([1.0 + 0j])
    for v in reversed(vecs):
        out = np.kron(out, v)
    return out


def test_eigenstates_give_outcome_zero(oracle_mod):
    n, S = 3, 50
    r = np.random.default_rng(70)
    plus = np.array([1, 1]) / np.sqrt(2)
    plus_i = np.array([1, 1j]) / np.sqrt(2)
    for basis, vec in ((1, plus), (2, plus_i), (3, np.array([1.0, 0.0]))):
        out, lo, hi = oracle_mod.shadow(n, product([vec] * n), np.full((S, n), basis), r.uniform(size=S))
        assert not out.any()
        np.testing.assert_allclose(hi, 1.0, atol=1e-12)
    # the -1 eigenvector of Y measured in Y gives outcome 1 on every qubit
    minus_i = np.array([1, -1j]) / np.sqrt(2)
    out, _, _ = oracle_mod.shadow(n, product([minus_i] * n), np.full((S, n), 2), r.uniform(size=S))
    assert (out == 2 ** n - 1).all()


def test_ghz_parities(oracle_mod):
    n, S = 4, 400
    r = np.random.default_rng(71)
    ghz = np.zeros(2 ** n, complex)
    ghz[0] = ghz[-1] = 1 / np.sqrt(2)
    out, _, _ = oracle_mod.shadow(n, ghz, np.full((S, n), 1), r.uniform(size=S))
    assert all(bin(int(x)).count("1") % 2 == 0 for x in out)          # <X X X X> = +1
    out, _, _ = oracle_mod.shadow(n, ghz, np.full((S, n), 3), r.uniform(size=S))
    assert set(int(x) for x in out) <= {0, 2 ** n - 1}
    bases = np.array([[2, 2, 1, 1]] * S)                                 # <Y Y X X> = -1
    out, _, _ = oracle_mod.shadow(n, ghz, bases, r.uniform(size=S))
    assert all(bin(int(x)).count("1") % 2 == 1 for x in out)


def test_product_state_frequencies(oracle_mod):
    n, S = 3, 3000
    r = np.random.default_rng(72)
    th = np.array([0.4, 1.3, 2.2])
    psi = product([np.array([np.cos(t / 2), np.sin(t / 2)]) for t in th])
    for basis, p0 in ((3, np.cos(th / 2) ** 2), (1, (1 + np.sin(th)) / 2), (2, np.full(n, 0.5))):
        out, _, _ = oracle_mod.shadow(n, psi, np.full((S, n), basis), r.uniform(size=S))
        zeros = np.array([np.sum(((out >> q) & 1) == 0) for q in range(n)])
        sd = np.sqrt(S * p0 * (1 - p0))
        assert np.all(np.abs(zeros - S * p0) < 5 * sd + 1), (basis, zeros, S * p0)


def test_shadow_estimator_is_unbiased(oracle_mod):
    n, S = 3, 6000
    w = W.shadow_workload(n, S, seed=73)
    out, _, _ = oracle_mod.shadow(n, w["psi"], w["bases"], w["u"])
    codes = np.array([[1, 3, 0]], np.uint8)          # X_0 Z_1
    exact = oracle_mod.expect(n, w["psi"], codes, np.array([1.0])).real
    hit = (w["bases"][:, 0] == 1) & (w["bases"][:, 1] == 3)
    sgn = (1 - 2 * ((out >> 0) & 1)) * (1 - 2 * ((out >> 1) & 1))
    est = 9.0 * np.where(hit, sgn, 0)
    assert abs(est.mean() - exact) < 5 * est.std() / np.sqrt(S)


def test_outcome_probability_matches_the_kronecker_rotation(oracle_mod):
    n, S = 5, 40
    w = W.shadow_workload(n, S, seed=74)
    out, lo, hi = oracle_mod.shadow(n, w["psi"], w["bases"], w["u"])
    for s in range(S):
        rot = kron_rotation(w["bases"][s]) @ w["psi"]
        p = np.abs(rot) ** 2
        x = int(out[s])
        assert lo[s] <= w["u"][s] < hi[s]
        assert hi[s] - lo[s] == pytest.approx(p[x] / p.sum(), abs=1e-12)
        assert lo[s] == pytest.approx(p[:x].sum() / p.sum(), abs=1e-12)
