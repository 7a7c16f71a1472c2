"""Classical-shadow snapshots: HIP path (through the C ABI) vs the CPU oracle.

An outcome is an integer chosen by comparing a uniform with running sums of
probabilities: the kernels sum float32 probabilities in float64, the oracle
complex128 ones.  The outcomes must agree, except where the uniform lies
within BOUNDARY of an end of the oracle's probability interval for its
outcome; the GPU's outcome must then be the neighbour on that side in the
oracle's cumulative order (found by rerunning the oracle just outside the
interval), never any other index.
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


def check(oracle_mod, n, psi, bases, got, want, lo, hi, u):
    mism = 0
    for s in range(len(u)):
        if got[s] == want[s]:
            continue
        mism += 1
        b = np.ascontiguousarray(bases[s:s + 1])
        if abs(u[s] - lo[s]) < BOUNDARY:
            # the previous outcome: the first x whose running sum exceeds the largest value below lo
            nb, _, _ = oracle_mod.shadow(n, psi, b, np.array([np.nextafter(lo[s], -np.inf)]))
        else:
            assert abs(u[s] - hi[s]) < BOUNDARY, (s, got[s], want[s], lo[s], hi[s], u[s])
            nb, _, _ = oracle_mod.shadow(n, psi, b, np.array([hi[s]]))   # the next outcome
        assert got[s] == nb[0], (s, got[s], want[s], nb[0], lo[s], hi[s], u[s])
    assert mism <= max(1, len(u) // 8)


@pytest.mark.parametrize("n", [9, 12, 14])
def test_shadow_matches_oracle(P, oracle_mod, n):
    w = W.shadow_workload(n, 64, seed=80 + n)
    psi = np.asarray(w["psi"], np.complex64).astype(np.complex128)   # the state the kernels see
    got = run_gpu(P, n, psi, w["bases"], w["u"])
    want, lo, hi = oracle_mod.shadow(n, psi, w["bases"], w["u"])
    check(oracle_mod, n, psi, w["bases"], got, want, lo, hi, w["u"])
    assert len(set(got.tolist())) > 1


def test_shadow_z_bases_sample_the_state(P, oracle_mod):
    n, S = 10, 200
    w = W.shadow_workload(n, S, seed=90)
    psi = np.asarray(w["psi"], np.complex64).astype(np.complex128)
    bases = np.full((S, n), 3, np.uint8)
    got = run_gpu(P, n, psi, bases, w["u"])
    want, lo, hi = oracle_mod.shadow(n, psi, bases, w["u"])
    check(oracle_mod, n, psi, bases, got, want, lo, hi, w["u"])


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
    check(oracle_mod, n, psi, w["bases"][idx], got[idx], want, lo, hi, w["u"][idx])


def test_shadow_rejects_psi_inside_work(P):
    # every snapshot's first rotation reads psi while other snapshots already write work
    n, S = 9, 4
    layer = P.shadow_layer(n)
    work = torch.zeros((S, 2 ** n), dtype=torch.complex64, device="cuda")
    bases = torch.full((S, n), 3, dtype=torch.uint8, device="cuda")
    u = torch.full((S,), 0.5, dtype=torch.float64, device="cuda")
    for psi in (work[0], work[2], work.view(-1)[2 ** n - 8: 2 * 2 ** n - 8]):
        with pytest.raises(Exception, match="overlap"):
            P.shadow_snapshots(layer, psi.contiguous() if psi.is_contiguous() else psi, bases, u, work=work)
    ok = torch.zeros(2 ** n, dtype=torch.complex64, device="cuda")
    ok[0] = 1
    out = P.shadow_snapshots(layer, ok, bases, u, work=work)
    assert (out.cpu().numpy() == 0).all()
