"""The allocation-free value-and-gradient entry point (tcng_expect_grad_noalloc)
against the workspace entry point (tcng_expect_grad) it shares its kernels
with: two calls in a row, the second on a smaller input, in each execution
mode; plus its size limit.  Same kernels, same launch order, fixed-order
sums: the results are bit-identical."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

TDT = {"c64": torch.complex64, "c128": torch.complex128}
RDT = {"c64": torch.float32, "c128": torch.float64}


@pytest.fixture(scope="module")
def P():
    import paper_2602_14167_amd as pkg
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    pkg.lib()
    return pkg


def case(P, n, layers, batch, dtype, seed):
    w = W.hea_workload(n, layers, -1.0, -0.5, seed=seed, batch=batch)
    circ = P.Circuit(n, w["gates"], w["n_params"])
    H = P.PauliSum(n, w["codes"], w["coeffs"])
    p = torch.as_tensor(w["params"]).to(device="cuda", dtype=RDT[dtype])
    return circ, H, p


@pytest.mark.parametrize("dtype,mode", [("c64", "fused"), ("c64", "tiled"), ("c64", "plain"), ("c128", "tiled")])
def test_noalloc_matches_workspace_entry_point(P, dtype, mode):
    print(f"noalloc {dtype} {mode}", flush=True)
    for n, layers, batch, seed in ((14, 4, 3, 11), (11, 2, 2, 12)):   # the second call is smaller
        circ, H, p = case(P, n, layers, batch, dtype, seed)
        E1, g1 = P.expect_grad_noalloc(circ, p, H, dtype=TDT[dtype], mode=mode)
        E0, g0 = P.expect_grad(circ, p, H, dtype=TDT[dtype], mode=mode)
        torch.cuda.synchronize()
        assert torch.equal(E0, E1), (n, E0, E1)
        assert torch.equal(g0, g1), (n, float((g0 - g1).abs().max()))


def test_noalloc_gate_gradients(P):
    # the uneven-batch generator's Haar brick-walls: U2 Lie gradients through the fixed array
    c = W.cfg4(count=2, n_lo=12, n_hi=13, d_lo=3, d_hi=6, seed=93)["circuits"]
    for cc in c:
        circ = P.Circuit(cc["n"], cc["gates"], 0, W.round_mats(cc["mats"], "c64"))
        H = P.PauliSum(cc["n"], cc["codes"], cc["coeffs"])
        E1, _, gg1 = P.expect_grad_noalloc(circ, None, H, want_gate_grad=True, mode="fused")
        E0, _, gg0 = P.expect_grad(circ, None, H, want_gate_grad=True, mode="fused")
        torch.cuda.synchronize()
        assert torch.equal(E0, E1) and torch.equal(gg0, gg1)


def test_noalloc_rejects_a_workspace_beyond_its_array(P):
    import ctypes
    limit = P.lib().tcng_noalloc_scratch_bytes()
    assert limit == 64 << 20
    # the first of these shapes whose workspace exceeds the array is rejected
    for n, layers, batch, mode in ((16, 8, 2048, "tiled"), (16, 8, 2048, "fused"), (22, 12, 1, "fused"),
                                   (24, 12, 1, "fused")):
        circ, H, p = case(P, n, layers, batch, "c64", 13)
        need = ctypes.c_size_t()
        P.check(P.lib().tcng_workspace_size(circ.handle, H.handle, 0, batch, P.MODES[mode], ctypes.byref(need)))
        print(f"workspace n={n} L={layers} batch={batch} {mode}: {need.value} bytes", flush=True)
        if need.value > limit:
            break
    assert need.value > limit
    with pytest.raises(P.TcngError) as e:
        P.expect_grad_noalloc(circ, p, H, mode=mode)
    assert e.value.status == 3   # TCNG_E_WORKSPACE
