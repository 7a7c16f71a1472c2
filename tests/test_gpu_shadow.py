"""Classical-shadow snapshots: HIP path (through the C ABI) vs the CPU oracle.

An outcome is an integer chosen by comparing a uniform with running sums of
probabilities: the kernels sum float32 probabilities in float64, the oracle
complex128 ones.  The outcomes must agree, except where the uniform lies
within BOUNDARY of an end of the oracle's probability interval for its
outcome (both neighbours are then correct within rounding).
"""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

BOUNDARY = 1e-5


@pytest.fixture(scope="module")
def P():
    import paper_2602_14167_amd as pkg
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    pkg.lib()
    return pkg


def run_gpu(P, n, psi, bases, u):
    print(f"shadow n={n} snapshots={len(u)}", flush=True)
    layer = P.shadow_layer(n)
    out = P.shadow_snapshots(layer, torch.as_tensor(np.asarray(psi, np.complex64)).cuda(),
                             torch.as_tensor(np.ascontiguousarray(bases, np.uint8)).cuda(),
                             torch.as_tensor(np.ascontiguousarray(u, np.float64)).cuda())
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check(got, want, lo, hi, u):
    for s in range(len(u)):
        if got[s] != want[s]:
            assert min(abs(u[s] - lo[s]), abs(u[s] - hi[s])) < BOUNDARY, (s, got[s], want[s], lo[s], hi[s], u[s])


@pytest.mark.parametrize("n", [9, 12, 14])
def test_shadow_matches_oracle(P, oracle_mod, n):
    w = W.shadow_workload(n, 64, seed=80 + n)
    psi = np.asarray(w["psi"], np.complex64).astype(np.complex128)   # the state the kernels see
    got = run_gpu(P, n, psi, w["bases"], w["u"])
    want, lo, hi = oracle_mod.shadow(n, psi, w["bases"], w["u"])
    check(got, want, lo, hi, w["u"])
    assert len(set(got.tolist())) > 1


def test_shadow_z_bases_sample_the_state(P, oracle_mod):
    n, S = 10, 200
    w = W.shadow_workload(n, S, seed=90)
    psi = np.asarray(w["psi"], np.complex64).astype(np.complex128)
    bases = np.full((S, n), 3, np.uint8)
    got = run_gpu(P, n, psi, bases, w["u"])
    want, lo, hi = oracle_mod.shadow(n, psi, bases, w["u"])
    check(got, want, lo, hi, w["u"])


def test_shadow_eigenstates_and_ghz(P):
    n, S = 10, 64
    r = np.random.default_rng(91)
    plus_i = np.array([1, 1j]) / np.sqrt(2)
    psi = np.array([1.0 + 0j])
    for _ in range(n):
        psi = np.kron(psi, plus_i)
    got = run_gpu(P, n, psi, np.full((S, n), 2, np.uint8), r.uniform(size=S))
    assert not got.any()                      # +1 eigenvector of Y on every qubit
    ghz = np.zeros(2 ** n, complex)
    ghz[0] = ghz[-1] = 1 / np.sqrt(2)
    got = run_gpu(P, n, ghz, np.full((S, n), 1, np.uint8), r.uniform(size=S))
    assert all(bin(int(x)).count("1") % 2 == 0 for x in got)   # <X...X> = +1


def test_shadow_full_size_sampled(P, oracle_mod):
    # the benchmarked launch: 256 snapshots of a 20-qubit state
    n, S = 20, 256
    w = W.shadow_workload(n, S, seed=20)
    psi = np.asarray(w["psi"], np.complex64).astype(np.complex128)
    got = run_gpu(P, n, psi, w["bases"], w["u"])
    assert ((got >= 0) & (got < 2 ** n)).all()
    idx = np.random.default_rng(92).choice(S, size=12, replace=False)
    want, lo, hi = oracle_mod.shadow(n, psi, w["bases"][idx], w["u"][idx])
    check(got[idx], want, lo, hi, w["u"][idx])
