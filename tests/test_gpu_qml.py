"""SU(4) QML training step: HIP path (through the C ABI) vs the CPU oracle.

The kernels form each gate in float64 and round it to complex64, evolve
complex64 states on the matrix cores, and reduce probabilities, losses and
gradients in float64; the oracle works in complex128 throughout.  A gate
rounded to float32 moves a state by about 1e-7 per gate, so after G gates
the probabilities carry about G * 1e-7 relative error (G <= 400 here): the
per-sample losses (about ln C in size) must agree to LOSS_TOL absolute, and
every component of the batch-mean gradient to GRAD_RTOL of itself plus
GRAD_FLOOR of the largest component (the floor is for components near zero,
whose error follows the gradient's overall scale; tests/bars.py).
"""
import numpy as np
import pytest
import torch

import workloads as W
from tests.bars import assert_grad_components

pytestmark = pytest.mark.gpu

LOSS_TOL = 1e-4
GRAD_RTOL = 1e-3
GRAD_FLOOR = 1e-4


@pytest.fixture(scope="module")
def P():
    import paper_2602_14167_amd as pkg
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    pkg.lib()
    return pkg


def circuit(P, n, gates):
    return P.Circuit(n, gates, 0, np.tile(np.eye(4, dtype=np.complex128), (len(gates), 1, 1)))


def run_gpu(P, w, idx=None):
    n = w["n"]
    x, y = w["inputs"], w["labels"]
    if idx is not None:
        x, y = x[idx], y[idx]
    print(f"qml {w['task']} n={n} layers={w['layers']} batch={len(y)}", flush=True)
    c = circuit(P, n, w["gates"])
    xs = torch.as_tensor(np.asarray(x, np.complex64)).cuda()
    loss, grad = P.qml_step(c, torch.as_tensor(w["theta"]).cuda(), xs, torch.as_tensor(y).cuda(), w["k"], w["C"])
    torch.cuda.synchronize()
    return loss.cpu().numpy(), grad.cpu().numpy(), np.asarray(x, np.complex64).astype(np.complex128)


def check_oracle(oracle_mod, w, loss, grad, seen, y):
    ref = oracle_mod.qml(w["n"], w["gates"], w["theta"], seen, y, w["k"], w["C"])
    np.testing.assert_allclose(loss, ref["loss"], atol=LOSS_TOL)
    assert_grad_components(grad, ref["grad"], GRAD_RTOL, GRAD_FLOOR, f"qml n={w['n']}")
    assert np.abs(ref["grad"]).max() > 1e-3   # the comparison is not between two near-zero arrays


# Below 12 qubits a batch divisible by 2^(12 - n) runs 2^(12 - n) samples per
# 12-bit tile (the "wide" plan); other batches run one sample per tile.
@pytest.mark.parametrize("task,n,layers,batch", [
    ("mnist", 9, 3, 5),        # one 9-bit tile per sample
    ("mnist", 9, 3, 16),       # eight samples per tile
    ("mnist", 10, 6, 24),      # the MNIST register, four samples per tile
    ("mnist", 10, 3, 26),      # the MNIST register, one sample per tile
    ("mnist", 11, 4, 6),       # two samples per tile
    ("cifar100", 12, 4, 12),   # the CIFAR-100 register, 7 readout qubits, 100 classes
    ("mnist", 10, 2, 2400),    # more (sample group, tile) items than reverse workgroups
    ("mnist", 10, 2, 702),     # the same with one sample per tile
    ("cifar100", 14, 2, 150),  # several tiles per sample
])
def test_qml_matches_oracle(P, oracle_mod, task, n, layers, batch):
    w = W.qml_workload(task, seed=300 + n + layers, batch=batch, layers=layers)
    if n != w["n"]:
        w = dict(w, n=n, gates=W.qml_gates(n, layers))
        r = np.random.default_rng(400 + n)
        w["theta"] = r.uniform(0, 2 * np.pi, size=(w["gates"].shape[0], 15))
        x = np.zeros((batch, 2 ** n))
        feat = min(2 ** n, W.QML_TASKS[task][4])
        x[:, :feat] = r.uniform(size=(batch, feat))
        w["inputs"] = x / np.linalg.norm(x, axis=1, keepdims=True)
    loss, grad, seen = run_gpu(P, w)
    check_oracle(oracle_mod, w, loss, grad, seen, w["labels"])


@pytest.mark.parametrize("n,k,C,batch", [
    (9, 8, 256, 4),   # the widest readout: 256 bins of two amplitudes each
    (10, 1, 1, 3),    # one class: the loss and its gradient vanish
    (10, 2, 3, 1),    # a single sample
])
def test_qml_readout_edge_cases(P, oracle_mod, n, k, C, batch):
    r = np.random.default_rng(500 + n + k)
    gates = W.qml_gates(n, 2)
    w = dict(task="edge", n=n, layers=2, k=k, C=C, gates=gates,
             theta=r.uniform(0, 2 * np.pi, size=(gates.shape[0], 15)),
             labels=r.integers(0, C, size=batch).astype(np.int32))
    x = r.uniform(size=(batch, 2 ** n))
    w["inputs"] = x / np.linalg.norm(x, axis=1, keepdims=True)
    loss, grad, seen = run_gpu(P, w)
    ref = oracle_mod.qml(n, gates, w["theta"], seen, w["labels"], k, C)
    # 18 gates: about 2e-6 relative error in the probabilities, so tighter bounds than above
    np.testing.assert_allclose(loss, ref["loss"], atol=1e-5)
    if C == 1:
        assert np.all(loss == 0.0) and np.all(grad == 0.0) and np.all(ref["grad"] == 0.0)
    else:
        assert_grad_components(grad, ref["grad"], 1e-4, 1e-5, f"qml edge n={n} k={k} C={C}")
    if C == 1:
        assert np.all(loss == 0.0) and np.all(grad == 0.0)


def test_qml_padded_rows(P, oracle_mod):
    # states spaced wider than 2^n (one sample per tile): same results as the oracle
    w = W.qml_workload("mnist", seed=312, batch=8, layers=3)
    n, B, pad = w["n"], 8, 64
    c = circuit(P, n, w["gates"])
    bufs = [torch.zeros((B, 2 ** n + pad), dtype=torch.complex64, device="cuda") for _ in range(3)]
    x, psi, lam = (b[:, :2 ** n] for b in bufs)
    x.copy_(torch.as_tensor(np.asarray(w["inputs"], np.complex64)))
    print("qml padded rows", flush=True)
    loss, grad = P.qml_step(c, torch.as_tensor(w["theta"]).cuda(), x, torch.as_tensor(w["labels"]).cuda(), w["k"],
                            w["C"], psi=psi, lam=lam)
    torch.cuda.synchronize()
    seen = np.asarray(w["inputs"], np.complex64).astype(np.complex128)
    check_oracle(oracle_mod, w, loss.cpu().numpy(), grad.cpu().numpy(), seen, w["labels"])
    assert not bufs[1][:, 2 ** n:].any() and not bufs[2][:, 2 ** n:].any()   # padding untouched


def test_qml_bad_label_gives_nan_and_no_gradient(P, oracle_mod):
    w = W.qml_workload("mnist", seed=310, batch=6, layers=3)
    good = np.arange(6) != 2
    w["labels"] = w["labels"].copy()
    w["labels"][2] = 10   # outside the 10 classes
    loss, grad, seen = run_gpu(P, w)
    assert np.isnan(loss[2]) and np.isfinite(loss[good]).all()
    ref = oracle_mod.qml(w["n"], w["gates"], w["theta"], seen[good], w["labels"][good], w["k"], w["C"])
    np.testing.assert_allclose(loss[good], ref["loss"], atol=LOSS_TOL)
    # the bad sample contributes nothing; the mean is still over all six
    assert_grad_components(grad, ref["grad"] * 5 / 6, GRAD_RTOL, GRAD_FLOOR, "qml bad label")


def test_qml_in_place_and_aliases(P):
    # psi may be the inputs themselves (evolved in place); lambda may share memory with neither
    w = W.qml_workload("mnist", seed=313, batch=8, layers=2)
    c = circuit(P, w["n"], w["gates"])
    th = torch.as_tensor(w["theta"]).cuda()
    y = torch.as_tensor(w["labels"]).cuda()
    x = torch.as_tensor(np.asarray(w["inputs"], np.complex64)).cuda()
    print("qml in place", flush=True)
    loss0, grad0 = P.qml_step(c, th, x, y, w["k"], w["C"])
    x2 = x.clone()
    loss1, grad1 = P.qml_step(c, th, x2, y, w["k"], w["C"], psi=x2)
    torch.cuda.synchronize()
    assert torch.equal(loss0, loss1) and torch.equal(grad0, grad1)
    with pytest.raises(P.TcngError):
        P.qml_step(c, th, x, y, w["k"], w["C"], lam=x)
    psi = torch.empty_like(x)
    with pytest.raises(P.TcngError):
        P.qml_step(c, th, x, y, w["k"], w["C"], psi=psi, lam=psi)


def test_qml_non_finite_angle_gives_nan(P):
    # an infinite angle: the gate's scaling loop is bounded, the results are NaN
    w = W.qml_workload("mnist", seed=314, batch=4, layers=1)
    c = circuit(P, w["n"], w["gates"])
    th = w["theta"].copy()
    th[3, 7] = np.inf
    x = torch.as_tensor(np.asarray(w["inputs"], np.complex64)).cuda()
    print("qml infinite angle", flush=True)
    loss, grad = P.qml_step(c, torch.as_tensor(th).cuda(), x, torch.as_tensor(w["labels"]).cuda(), w["k"], w["C"])
    torch.cuda.synchronize()
    assert torch.isnan(loss).all() and torch.isnan(grad).any()


def test_qml_rejects_bad_arguments(P):
    w = W.qml_workload("mnist", seed=311, batch=2, layers=1)
    c = circuit(P, w["n"], w["gates"])
    x = torch.as_tensor(np.asarray(w["inputs"], np.complex64)).cuda()
    th = torch.as_tensor(w["theta"]).cuda()
    y = torch.as_tensor(w["labels"]).cuda()
    with pytest.raises(P.TcngError):
        P.qml_step(c, th, x, y, 0, 1)        # no readout qubit
    with pytest.raises(P.TcngError):
        P.qml_step(c, th, x, y, 4, 17)       # more classes than 2^k
    shared = np.asarray(w["gates"]).copy()
    shared[1, 5] = 0                         # two gates on one matrix
    with pytest.raises(P.TcngError):
        P.qml_step(P.Circuit(w["n"], shared, 0, np.tile(np.eye(4), (len(shared), 1, 1))), th, x, y, 4, 10)


@pytest.mark.parametrize("task", ["mnist", "cifar100"])
def test_qml_full_size(P, oracle_mod, task):
    # the benchmarked launch: the paper's register, depth and batch
    w = W.qml_workload(task, seed=1)
    loss, grad, _ = run_gpu(P, w)
    B = w["batch"]
    assert np.isfinite(loss).all() and np.isfinite(grad).all()
    # sampled per-sample losses and a sub-batch gradient at full depth against the oracle
    idx = np.random.default_rng(320).choice(B, size=12, replace=False)
    seen = np.asarray(w["inputs"][idx], np.complex64).astype(np.complex128)
    ref = oracle_mod.qml(w["n"], w["gates"], w["theta"], seen, w["labels"][idx], w["k"], w["C"])
    np.testing.assert_allclose(loss[idx], ref["loss"], atol=LOSS_TOL)
    lsub, gsub, _ = run_gpu(P, w, idx)
    np.testing.assert_allclose(lsub, ref["loss"], atol=LOSS_TOL)
    assert_grad_components(gsub, ref["grad"], GRAD_RTOL, GRAD_FLOOR, f"qml full size {task}")
    # the batch-mean gradient is the size-weighted mean of the two halves' gradients
    h = B // 2
    _, g1, _ = run_gpu(P, w, np.arange(h))
    _, g2, _ = run_gpu(P, w, np.arange(h, B))
    np.testing.assert_allclose(grad, (h * g1 + (B - h) * g2) / B, atol=1e-9 + 1e-6 * np.abs(grad).max())
