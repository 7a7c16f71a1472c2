"""Pins of the oracle's SU(4) QML step (no GPU).

The gate is checked against scipy's matrix exponential (a separate
implementation) and its derivatives against finite differences of that
exponential; the loss against a closed form at theta = 0 (identity gates:
the readout is the input's own marginal); the gradient against central
finite differences of the oracle's loss.
"""
import numpy as np
import pytest
import scipy.linalg

import workloads as W

S = [np.eye(2), np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.diag([1.0, -1.0])]


def generator_sum(theta):
    A = np.zeros((4, 4), complex)
    for k in range(15):
        a, b = (k + 1) >> 2, (k + 1) & 3
        A += theta[k] * np.kron(S[a], S[b])
    return A


@pytest.mark.parametrize("seed", range(4))
def test_su4_gate_matches_expm_and_is_special_unitary(oracle_mod, seed):
    th = np.random.default_rng(seed).uniform(0, 2 * np.pi, size=15) * (0.1 if seed == 0 else 1.0)
    U, dU = oracle_mod.su4(th)
    ref = scipy.linalg.expm(-0.5j * generator_sum(th))
    np.testing.assert_allclose(U, ref, atol=1e-12)
    np.testing.assert_allclose(U.conj().T @ U, np.eye(4), atol=1e-12)
    assert np.linalg.det(U) == pytest.approx(1.0, abs=1e-12)
    h = 1e-6
    for j in range(15):
        e = np.zeros(15)
        e[j] = h
        fd = (scipy.linalg.expm(-0.5j * generator_sum(th + e)) - scipy.linalg.expm(-0.5j * generator_sum(th - e))) / (2 * h)
        np.testing.assert_allclose(dU[j], fd, atol=1e-8)


def test_su4_single_generator_closed_form(oracle_mod):
    for k in range(15):
        th = np.zeros(15)
        th[k] = 1.1
        U, _ = oracle_mod.su4(th)
        a, b = (k + 1) >> 2, (k + 1) & 3
        np.testing.assert_allclose(U, np.cos(0.55) * np.eye(4) - 1j * np.sin(0.55) * np.kron(S[a], S[b]), atol=1e-13)


def test_qml_loss_at_identity_gates(oracle_mod):
    # theta = 0: every gate is the identity, so p is the input's marginal on the top k bits
    w = W.qml_workload("mnist", seed=3, batch=5, layers=2)
    n, k, C = w["n"], w["k"], w["C"]
    out = oracle_mod.qml(n, w["gates"], np.zeros_like(w["theta"]), w["inputs"], w["labels"], k, C, want_probs=True)
    p = (np.abs(w["inputs"]) ** 2).reshape(5, 2 ** k, -1).sum(axis=2)
    np.testing.assert_allclose(out["probs"], p, atol=1e-14)
    np.testing.assert_allclose(out["probs"].sum(axis=1), 1.0, atol=1e-14)
    z = p[:, :C]
    ref = np.log(np.exp(z).sum(axis=1)) - z[np.arange(5), w["labels"]]
    np.testing.assert_allclose(out["loss"], ref, atol=1e-14)


def test_qml_gradient_matches_finite_differences(oracle_mod):
    n, k, C = 4, 2, 3
    r = np.random.default_rng(5)
    gates = W.qml_gates(n, 2)
    G = gates.shape[0]
    th = r.uniform(0, 2 * np.pi, size=(G, 15))
    x = r.uniform(size=(3, 2 ** n))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    y = np.array([0, 2, 1], np.int32)
    out = oracle_mod.qml(n, gates, th, x, y, k, C)
    h = 1e-5
    for g in range(G):
        for j in (0, 4, 9, 14):
            e = np.zeros_like(th)
            e[g, j] = h
            lp = oracle_mod.qml(n, gates, th + e, x, y, k, C)["loss"].mean()
            lm = oracle_mod.qml(n, gates, th - e, x, y, k, C)["loss"].mean()
            assert out["grad"][g, j] == pytest.approx((lp - lm) / (2 * h), abs=1e-8)
