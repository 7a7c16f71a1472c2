"""Pins of the oracle's monitored Haar trajectories (no GPU).

The oracle measures qubit by qubit with conditional probabilities; these
checks reach the same quantities by routes that share none of its code:
unitary evolution by tensor contraction (tests/bruteforce.py), joint Born
probabilities of whole outcome strings from the dense state, closed forms
for p = 0 and p = 1, and sampling statistics over many uniforms.  A flipped
threshold, an unconditional instead of a conditional probability, a missing
renormalisation or a wrong matrix index fails one of them.
"""
import numpy as np
import pytest

import workloads as W
from tests import bruteforce as B


def evolve_step(n, gates, step_mats, psi):
    return B.run_tn(n, gates, mats=step_mats, init=psi)


def test_mipt_without_measurement_is_the_unitary_circuit(oracle_mod):
    n, steps = 5, 3
    w = W.mipt_workload(n, steps, 1, 0.0, seed=11)
    out = oracle_mod.mipt(n, w["gates"], w["mats"][0], w["u"][0], 0.0)
    psi = np.zeros(2 ** n, np.complex128)
    psi[0] = 1
    for s in range(steps):
        psi = evolve_step(n, w["gates"], w["mats"][0, s], psi)
    np.testing.assert_allclose(out["state"], psi, atol=1e-13)
    assert out["logp"] == 0.0
    assert not out["rec"].any()
    assert np.isnan(out["margin"]).all()


def test_mipt_every_qubit_measured_gives_basis_states_and_joint_born_probability(oracle_mod):
    # p = 1: after each step the state is the basis state of the outcome string,
    # and the record's probability is |<o_s| U_s |o_{s-1}>|^2 per step
    n, steps = 4, 3
    w = W.mipt_workload(n, steps, 1, 1.0, seed=12)
    out = oracle_mod.mipt(n, w["gates"], w["mats"][0], w["u"][0], 1.0)
    rec = out["rec"]
    assert (rec[:, 0] == (1 << n) - 1).all()
    prev = np.zeros(2 ** n, np.complex128)
    prev[0] = 1
    lp = 0.0
    for s in range(steps):
        amp = evolve_step(n, w["gates"], w["mats"][0, s], prev)
        o = int(rec[s, 1])
        lp += np.log(abs(amp[o]) ** 2)
        prev = np.zeros(2 ** n, np.complex128)
        prev[o] = amp[o] / abs(amp[o])
    assert out["logp"] == pytest.approx(lp, abs=1e-11)
    np.testing.assert_allclose(out["state"], prev, atol=1e-12)


def test_mipt_forced_record_has_the_dense_probability(oracle_mod):
    # any forced outcome string: ln P = ln of the joint weight of that string
    # in the dense state (sequential conditionals multiply to the joint)
    n = 5
    w = W.mipt_workload(n, 1, 1, 1.0, seed=13)
    psi = evolve_step(n, w["gates"], w["mats"][0, 0], np.eye(2 ** n, dtype=np.complex128)[0])
    for o in (0, 7, 19, 31):
        force = np.array([[(o >> q) & 1 for q in range(n)]])
        out = oracle_mod.mipt(n, w["gates"], w["mats"][0], w["u"][0], 1.0, force=force)
        assert int(out["rec"][0, 1]) == o
        assert out["logp"] == pytest.approx(np.log(abs(psi[o]) ** 2), abs=1e-11)


def test_mipt_partial_measurement_projects_on_the_measured_bits(oracle_mod):
    # measured set M with outcomes o: final state = P_{M,o} psi / ||P_{M,o} psi||,
    # probability = ||P_{M,o} psi||^2 (joint over the measured bits)
    n = 6
    w = W.mipt_workload(n, 1, 1, 0.5, seed=14)
    u = w["u"][0]
    out = oracle_mod.mipt(n, w["gates"], w["mats"][0], u, 0.5)
    mask, bits = int(out["rec"][0, 0]), int(out["rec"][0, 1])
    assert mask == sum(1 << q for q in range(n) if u[0, q] >= 0.5)
    assert mask != 0
    psi = evolve_step(n, w["gates"], w["mats"][0, 0], np.eye(2 ** n, dtype=np.complex128)[0])
    keep = np.array([(x & mask) == bits for x in range(2 ** n)])
    proj = np.where(keep, psi, 0)
    pr = np.vdot(proj, proj).real
    assert out["logp"] == pytest.approx(np.log(pr), abs=1e-11)
    np.testing.assert_allclose(out["state"], proj / np.sqrt(pr), atol=1e-12)


def test_mipt_outcome_frequencies_follow_the_born_rule(oracle_mod):
    # two qubits, one Haar gate, p = 1: the outcome pair x is drawn with
    # probability |psi_x|^2; p = 0.5: each qubit measured with frequency 1/2
    n, trials = 2, 4000
    r = np.random.default_rng(15)
    U = W.haar_u4(r)
    gates = W.mipt_step_gates(n)
    psi = B.run_tn(n, gates, mats=U[None])
    probs = np.abs(psi) ** 2
    counts = np.zeros(4)
    measured = np.zeros(2)
    for t in range(trials):
        u = r.uniform(size=(1, n))
        out = oracle_mod.mipt(n, gates, U[None, None], u, 1.0)
        counts[int(out["rec"][0, 1])] += 1
        u2 = r.uniform(size=(1, n))
        out2 = oracle_mod.mipt(n, gates, U[None, None], u2, 0.5)
        measured += [(int(out2["rec"][0, 0]) >> q) & 1 for q in range(n)]
    sd = np.sqrt(trials * probs * (1 - probs))
    assert np.all(np.abs(counts - trials * probs) < 5 * sd + 1), (counts, trials * probs)
    assert np.all(np.abs(measured - trials / 2) < 5 * np.sqrt(trials / 4))


def test_mipt_trajectory_invariants(oracle_mod):
    n, steps, p = 7, 6, 0.3
    w = W.mipt_workload(n, steps, 1, p, seed=16)
    out = oracle_mod.mipt(n, w["gates"], w["mats"][0], w["u"][0], p)
    st = out["state"]
    assert np.vdot(st, st).real == pytest.approx(1.0, abs=1e-12)
    assert out["logp"] <= 0.0
    for s in range(steps):
        mask = sum(1 << q for q in range(n) if w["u"][0, s, q] >= 1 - p)
        assert int(out["rec"][s, 0]) == mask
        assert int(out["rec"][s, 1]) & ~mask == 0
        for q in range(n):
            assert np.isnan(out["margin"][s, q]) == (not (mask >> q) & 1)
    # the last step's measured qubits are definite in the final state
    mask, bits = int(out["rec"][-1, 0]), int(out["rec"][-1, 1])
    x = np.arange(2 ** n)
    assert np.abs(st[(x & mask) != bits]).max(initial=0.0) == 0.0
