"""The HIP path against stored oracle values at full circuit depth.

tests/golden/*.npz are written by tests/golden/make_golden.py, which calls
only the CPU oracle on the seeded generators (inputs rounded once to the
complex64 path's precision and widened, so one set of values serves both
precisions).  Cases:

* the n=28 HEA/TFIM generator with all 12 layers at n = 20 and 22
  (780 gates at n = 22): the float32 un-compute of the adjoint sweep over the
  whole depth, measured against the oracle;
* the n=32 fSim brick-wall generator at depth 20 on 4x5 and 4x6 lattices;
* every circuit of the 1024-circuit uneven Haar batch with n <= 18 (661
  circuits): E and the 15 SU(4) Lie-algebra gradient components of every gate,
  from the full uneven launch (matrix-core passes) and from per-circuit tiled
  runs in complex64 (matrices rounded to complex64, as the run reads them) and
  complex128 (the complex128 matrices: the adjoint sweep inverts a gate by its
  conjugate transpose, so it needs the exactly unitary matrices to match at
  1e-12).

Bars: |dE| <= 1e-5 S and |d grad|_inf <= 1e-4 S in complex64, 1e-12 S in
complex128, with S = sum |c_k| (the bound on |E| and on every gradient
component).
"""
import os

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = {"c64": (1e-5, 1e-4), "c128": (1e-12, 1e-12)}
TDT = {"c64": torch.complex64, "c128": torch.complex128}
RDT = {"c64": torch.float32, "c128": torch.float64}
MODES = [("c64", "fused"), ("c64", "fused5"), ("c64", "tiled"), ("c128", "tiled")]


@pytest.fixture(scope="module")
def P():
    import paper_2602_14167_amd as pkg
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    pkg.lib()
    return pkg


def load(name):
    with np.load(os.path.join(GOLD, name), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def check_one(P, w, gold, dtype, mode, label):
    n = w["n"]
    circ = P.Circuit(n, w["gates"], w["n_params"])
    H = P.PauliSum(n, w["codes"], w["coeffs"])
    p = torch.as_tensor(gold["params"][None, :]).to(device="cuda", dtype=RDT[dtype])
    E, g = P.expect_grad(circ, p, H, dtype=TDT[dtype], mode=mode)[:2]
    torch.cuda.synchronize()
    S = float(np.abs(w["coeffs"]).sum())
    de = abs(float(E[0]) - float(gold["E"])) / S
    dg = float(np.max(np.abs(g.cpu().numpy()[0] - gold["grad"]))) / S
    print(f"{label} {dtype} {mode}: |dE|/S={de:.2e} |dg|/S={dg:.2e}", flush=True)
    te, tg = TOL[dtype]
    assert de <= te and dg <= tg, (de, dg)


@pytest.mark.parametrize("dtype,mode", MODES)
@pytest.mark.parametrize("n", [20, 22])
def test_hea_tfim_full_depth(P, n, dtype, mode):
    w = W.cfg2(n=n, layers=12)
    gold = load(f"hea_tfim_n{n}_L12.npz")
    np.testing.assert_array_equal(gold["params"], W.round_params(w["params"], "c64"))
    check_one(P, w, gold, dtype, mode, f"hea n={n} L=12")


@pytest.mark.parametrize("dtype,mode", MODES)
@pytest.mark.parametrize("cols", [5, 6])
def test_fsim_tfim2d_depth20(P, cols, dtype, mode):
    w = W.cfg5(rows=4, cols=cols, depth=20)
    gold = load(f"fsim_tfim2d_4x{cols}_d20.npz")
    np.testing.assert_array_equal(gold["params"], W.round_params(w["params"], "c64"))
    check_one(P, w, gold, dtype, mode, f"fsim 4x{cols} d=20")


@pytest.fixture(scope="module")
def haar():
    return W.cfg4()["circuits"], {"c64": load("haar_uneven_n_le_18.npz"), "c128": load("haar_uneven_n_le_18_c128.npz")}


def _haar_check(cs, gold, E, lie, dtype, label):
    te, tg = TOL[dtype]
    worst_e = worst_g = 0.0
    for j, i in enumerate(gold["index"]):
        c = cs[i]
        S = float(np.abs(c["coeffs"]).sum())
        ref_lie = gold["lie"][gold["offsets"][j]:gold["offsets"][j + 1]]
        worst_e = max(worst_e, abs(E[j] - gold["E"][j]) / S)
        worst_g = max(worst_g, float(np.max(np.abs(lie[j] - ref_lie))) / S)
    print(f"{label}: {len(gold['index'])} circuits, max |dE|/S={worst_e:.2e} max |dlie|/S={worst_g:.2e}", flush=True)
    assert worst_e <= te and worst_g <= tg, (worst_e, worst_g)


def test_haar_uneven_batch_golden(P, haar):
    """The full 1024-circuit uneven launch (as benchmarked); its 661 circuits
    with n <= 18 against the stored oracle values."""
    cs, gold = haar
    gold = gold["c64"]
    circs = [P.Circuit(c["n"], c["gates"], 0, W.round_mats(c["mats"], "c64")) for c in cs]
    hams = [P.PauliSum(c["n"], c["codes"], c["coeffs"]) for c in cs]
    E, _, ggs = P.expect_grad_multi(circs, hams, [None] * len(cs), dtype=torch.complex64, want_gate_grad=True)
    torch.cuda.synchronize()
    E = E.cpu().numpy()
    idx = gold["index"]
    _haar_check(cs, gold, E[idx], [ggs[i].cpu().numpy() for i in idx], "c64", "uneven launch c64")


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_haar_per_circuit_tiled_golden(P, haar, dtype):
    cs, gold = haar
    gold = gold[dtype]
    Es, lies = [], []
    for i in gold["index"]:
        c = cs[i]
        circ = P.Circuit(c["n"], c["gates"], 0, W.round_mats(c["mats"], dtype))
        H = P.PauliSum(c["n"], c["codes"], c["coeffs"])
        E, _, gg = P.expect_grad(circ, None, H, dtype=TDT[dtype], want_gate_grad=True, mode="tiled")
        Es.append(float(E[0]))
        lies.append(gg[0].cpu().numpy())
    _haar_check(cs, gold, np.array(Es), lies, dtype, f"per-circuit tiled {dtype}")
