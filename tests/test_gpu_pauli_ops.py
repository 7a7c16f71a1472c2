"""Pauli sum as an operator: matrix-free H psi and its sparse (COO) matrix,
HIP path (through the C ABI) vs the CPU oracle.

COO rows and columns are integers: bit-exact.  Values are sums of +-c_k (or
+-i c_k) in the same term order on both sides, so they agree exactly as well.
H psi is floating-point work on the state: each output amplitude is a sum of
T terms of size at most |c_k| max|psi|, so its error is held below
4 T eps S max|psi| (eps the unit roundoff, S = sum_k |c_k|; tests/bars.py).
"""
import numpy as np
import pytest
import torch

import workloads as W
from tests.bars import assert_hpsi

pytestmark = pytest.mark.gpu

TDT = {"c64": torch.complex64, "c128": torch.complex128}


@pytest.fixture(scope="module")
def P():
    import paper_2602_14167_amd as pkg
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    pkg.lib()
    return pkg


def hams():
    r = np.random.default_rng(51)
    out = []
    codes, coeffs = W.random_pauli_sum(4, 10, r)
    codes = np.vstack([codes, codes[:3], np.zeros((1, 4), np.uint8)])
    out.append((4, codes, np.concatenate([coeffs, r.normal(size=4)])))
    out.append((9,) + tuple(W.tfim_1d(9, 1.0, 0.8)))
    out.append((12,) + tuple(W.xxz_1d(12, 0.5)))
    out.append((13,) + tuple(W.random_2local(13, 30, r)))
    return out


@pytest.mark.parametrize("case", range(4))
def test_coo_matches_oracle(P, oracle_mod, case):
    n, codes, coeffs = hams()[case]
    H = P.PauliSum(n, codes, coeffs)
    print(f"coo n={n} terms={len(coeffs)}", flush=True)
    rows, cols, vals = P.pauli_coo(H)
    torch.cuda.synchronize()
    orows, ocols, ovals, G = oracle_mod.pauli_coo(n, codes, coeffs)
    assert rows.numel() == G * 2 ** n
    np.testing.assert_array_equal(rows.cpu().numpy(), orows)
    np.testing.assert_array_equal(cols.cpu().numpy(), ocols)
    np.testing.assert_array_equal(vals.cpu().numpy(), ovals)


@pytest.mark.parametrize("begin,count", [(0, 1), (5, 1000), (8191, 1), (3000, 5192)])
def test_coo_row_ranges(P, oracle_mod, begin, count):
    n, codes, coeffs = hams()[3]
    H = P.PauliSum(n, codes, coeffs)
    rows, cols, vals = P.pauli_coo(H, begin, count)
    torch.cuda.synchronize()
    orows, ocols, ovals, G = oracle_mod.pauli_coo(n, codes, coeffs, begin, count)
    np.testing.assert_array_equal(rows.cpu().numpy(), orows)
    np.testing.assert_array_equal(cols.cpu().numpy(), ocols)
    np.testing.assert_array_equal(vals.cpu().numpy(), ovals)


def test_coo_degenerate_sums(P, oracle_mod):
    n = 10
    H0 = P.PauliSum(n, np.zeros((0, n), np.uint8), np.zeros(0))
    rows, cols, vals = P.pauli_coo(H0)
    assert rows.numel() == 0 and cols.numel() == 0 and vals.numel() == 0
    Hi = P.PauliSum(n, np.zeros((2, n), np.uint8), np.array([0.75, -0.25]))   # identity twice
    rows, cols, vals = P.pauli_coo(Hi)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(rows.cpu().numpy(), np.arange(2 ** n))
    np.testing.assert_array_equal(cols.cpu().numpy(), np.arange(2 ** n))
    np.testing.assert_array_equal(vals.cpu().numpy(), np.full(2 ** n, 0.5 + 0j))
    with pytest.raises(P.TcngError):
        P.pauli_coo(Hi, 2 ** n - 3, 4)   # past the last row


def test_coo_full_size_tfim24(P, oracle_mod):
    # the benchmarked build: open TFIM on 24 qubits (23 ZZ + 24 X terms)
    n = 24
    codes, coeffs = W.tfim_1d(n, 1.0, 1.0)
    H = P.PauliSum(n, codes, coeffs)
    print("coo n=24 full", flush=True)
    rows, cols, vals = P.pauli_coo(H)
    torch.cuda.synchronize()
    G = rows.numel() >> n
    assert G == n + 1
    ar = torch.arange(1 << n, device="cuda", dtype=torch.int64)
    for g in range(G):
        seg = slice(g << n, (g + 1) << n)
        assert torch.equal(rows[seg], ar)
        x = int(rows[g << n] ^ cols[g << n])
        assert torch.equal(cols[seg], ar ^ x)
    r = np.random.default_rng(52)
    for row in list(r.integers(0, 1 << n, size=40)) + [0, (1 << n) - 1]:
        orows, ocols, ovals, og = oracle_mod.pauli_coo(n, codes, coeffs, int(row), 1)
        idx = torch.tensor([(g << n) + int(row) for g in range(G)], device="cuda")
        np.testing.assert_array_equal(rows[idx].cpu().numpy(), orows)
        np.testing.assert_array_equal(cols[idx].cpu().numpy(), ocols)
        np.testing.assert_array_equal(vals[idx].cpu().numpy(), ovals)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("mode", ["tiled", "plain"])
@pytest.mark.parametrize("case", [1, 3])
def test_apply_pauli_matches_oracle(P, oracle_mod, dtype, mode, case):
    n, codes, coeffs = hams()[case]
    S = float(np.abs(coeffs).sum())
    H = P.PauliSum(n, codes, coeffs)
    r = np.random.default_rng(60 + case)
    psi0 = W.random_state(n, r, batch=2)
    psi = torch.as_tensor(psi0).to(device="cuda", dtype=TDT[dtype])
    seen = psi.cpu().numpy().astype(np.complex128)
    out, e = P.apply_pauli(psi, H, want_energy=True, mode=mode)
    torch.cuda.synchronize()
    for b in range(2):
        ref = oracle_mod.apply_hamiltonian(n, seen[b], codes, coeffs)
        assert_hpsi(out[b].cpu().numpy(), ref, seen[b], coeffs, dtype, f"n={n} {mode}")
        eref = oracle_mod.expect(n, seen[b], codes, coeffs).real
        assert float(e[b]) == pytest.approx(eref, abs=(1e-5 if dtype == "c64" else 1e-12) * S)


def test_apply_pauli_rejects_an_aliased_output(P):
    n = 9
    codes, coeffs = W.tfim_1d(n, 1.0, 1.0)
    H = P.PauliSum(n, codes, coeffs)
    psi = P.new_state(n)
    with pytest.raises(P.TcngError):
        P.apply_pauli(psi, H, out=psi)
