"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances (the accuracy targets of the build):
  complex128: 1e-12 on <H> and on every gradient component;
  complex64 : 1e-5 on <H>, 1e-4 on the gradient;
all relative to S = sum_k |c_k|, the a-priori bound on |<H>| and on each
gradient component of a generator with norm <= 1 (a relative error of a value
that concentrates near 0 is undefined).  For complex64 the oracle receives the
float32-rounded angles and complex64-rounded matrices widened exactly, so the
comparison measures the kernels, not input rounding.  Amplitudes: the
largest error over the state's largest amplitude, at most 8 * (gate
applications) * (unit roundoff), see tests/bars.py.
"""
import numpy as np
import pytest
import torch

import workloads as W
from tests.bars import assert_amps

pytestmark = pytest.mark.gpu

TOL = {"c64": dict(E=1e-5, g=1e-4, amp=2e-5), "c128": dict(E=1e-12, g=1e-12, amp=1e-12)}
# (precision, mode) pairs: complex128 has no matrix-core plan (its "fused" runs the tiled passes);
# "fused5" is the 5-qubit-block plan (complex64, n >= 12; smaller states run the 4-qubit plan)
DM = [("c64", "tiled"), ("c64", "plain"), ("c64", "fused"), ("c64", "fused5"), ("c128", "tiled"), ("c128", "plain"),
      ("c128", "fused")]
TDT = {"c64": torch.complex64, "c128": torch.complex128}


@pytest.fixture(scope="module")
def P():
    import paper_2602_14167_amd as pkg
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    pkg.lib()
    return pkg


def dev(x, dtype):
    return torch.as_tensor(np.asarray(x)).to(device="cuda", dtype=dtype)


def rdt(dtype):
    return torch.float32 if dtype == "c64" else torch.float64


def run_gpu(P, n, gates, params, mats, dtype, mode, batch_params=None, init=None):
    circ = P.Circuit(n, gates, 0 if params is None else len(params), W.round_mats(mats, dtype) if mats is not None else None)
    pb = np.atleast_2d(params if batch_params is None else batch_params)
    B = pb.shape[0]
    psi = torch.empty((B, 2 ** n), dtype=TDT[dtype], device="cuda")
    if init is None:
        P.state_init(psi)
    else:
        psi.copy_(dev(init, TDT[dtype]))
    p = dev(pb, rdt(dtype)) if circ.n_params else None
    P.run_circuit(circ, p, psi, mode=mode)
    return psi.cpu().numpy()


# ---------------------------------------------------------------------------
# state initialisation and single gates
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_state_init(P, dtype):
    n = 9
    psi = torch.full((3, 2 ** n), 7.0, dtype=TDT[dtype], device="cuda")
    P.state_init(psi, basis=37)
    ref = np.zeros((3, 2 ** n))
    ref[:, 37] = 1
    np.testing.assert_array_equal(psi.cpu().numpy(), ref)
    amps = W.random_state(n, np.random.default_rng(1))
    src = dev(amps, TDT[dtype])
    P.state_init(psi, amps=src)
    # a copy: bit-exact
    np.testing.assert_array_equal(psi.cpu().numpy(), np.tile(src.cpu().numpy(), (3, 1)))


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_apply_gate_matches_oracle(P, oracle_mod, dtype, k):
    n = 9
    r = np.random.default_rng(10 + k)
    init = W.random_state(n, r)
    psi = dev(init, TDT[dtype]).reshape(1, -1).contiguous()
    for trial in range(3):
        qs = [int(v) for v in r.choice(n, size=k, replace=False)]
        A = r.standard_normal((2 ** k, 2 ** k)) + 1j * r.standard_normal((2 ** k, 2 ** k))
        A /= np.linalg.norm(A, 2)
        A = W.round_mats(A, dtype)
        P.apply_gate(psi, qs, dev(A, TDT[dtype]))
        init = oracle_mod.apply_matrix(n, init, qs, A)
    assert_amps(psi.cpu().numpy()[0], init, dtype, 3 * 2 ** k, f"apply_gate k={k}")


@pytest.mark.parametrize("dtype,n", [("c64", 12), ("c64", 13), ("c128", 11), ("c128", 13)])
def test_chunked_gates_every_target(P, oracle_mod, dtype, n):
    """Streaming gate kernels on states of at least one chunk: every target of
    a one-qubit matrix, and two-qubit matrices on pairs of low (lane-bit),
    high and vector-element qubits in both orders, applied in turn."""
    r = np.random.default_rng(20 + n)
    ref = W.random_state(n, r)
    psi = dev(ref, TDT[dtype]).reshape(1, -1).contiguous()
    ref = psi.cpu().numpy()[0].astype(np.complex128)
    ops = 0
    targets = [[q] for q in range(n)]
    pairs = [(0, 1), (1, 0), (0, n - 1), (n - 1, 0), (1, 2), (3, 1), (2, 9), (9, 2), (7, 8), (n - 1, n - 2), (5, 6),
             (6, 7), (0, 7), (10, 4)]
    for qs in targets + [list(p) for p in pairs]:
        k = len(qs)
        A = r.standard_normal((2 ** k, 2 ** k)) + 1j * r.standard_normal((2 ** k, 2 ** k))
        A = np.linalg.qr(A)[0]
        A = W.round_mats(A, dtype)
        P.apply_gate(psi, qs, dev(A, TDT[dtype]))
        ref = oracle_mod.apply_matrix(n, ref, qs, A)
        ops += 2 ** k
    assert_amps(psi.cpu().numpy()[0], ref, dtype, ops, f"chunked gates n={n}")


# ---------------------------------------------------------------------------
# circuits
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype,mode", DM)
@pytest.mark.parametrize("n", [1, 2, 5, 9, 10, 11, 12, 13, 14, 16])
def test_run_circuit_random_all_kinds(P, oracle_mod, dtype, mode, n):
    r = np.random.default_rng(100 + n)
    gates, params, mats = W.random_circuit(n, 120, r)
    B = 2
    bp = np.stack([params, r.uniform(0, 2 * np.pi, params.shape)])
    init = W.random_state(n, r)
    got = run_gpu(P, n, gates, params, mats, dtype, mode, batch_params=bp, init=np.tile(init, (B, 1)))
    for b in range(B):
        ref = oracle_mod.run(n, gates, W.round_params(bp[b], dtype), W.round_mats(mats, dtype), init=init if dtype == "c128" else init.astype(np.complex64))
        assert_amps(got[b], ref, dtype, 4 * len(gates), f"random circuit n={n} {mode}")


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_tiled_and_plain_agree_on_hea(P, dtype):
    c = W.cfg2(n=15, layers=4)
    a = run_gpu(P, 15, c["gates"], c["params"], None, dtype, "tiled")
    b = run_gpu(P, 15, c["gates"], c["params"], None, dtype, "plain")
    assert_amps(a, b, dtype, 2 * len(c["gates"]), "hea15 tiled vs plain")


# ---------------------------------------------------------------------------
# Pauli expectations
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype,mode", DM)
@pytest.mark.parametrize("n,kind", [(3, "random"), (11, "random"), (12, "tfim"), (15, "xxz"), (16, "2local"),
                                    (16, "random")])
def test_expect_pauli_matches_oracle(P, oracle_mod, dtype, mode, n, kind):
    r = np.random.default_rng(300 + n)
    if kind == "random":
        codes, coeffs = W.random_pauli_sum(n, 20, r, max_weight=4 if n > 12 else None)
    elif kind == "tfim":
        codes, coeffs = W.tfim_1d(n, -1.0, -0.5)
    elif kind == "xxz":
        codes, coeffs = W.xxz_1d(n, 0.5)
    else:
        codes, coeffs = W.random_2local(n, 3 * n, r)
    B = 2
    states = np.stack([W.random_state(n, r) for _ in range(B)])
    if dtype == "c64":
        states = states.astype(np.complex64).astype(np.complex128)
    H = P.PauliSum(n, codes, coeffs)
    psi = dev(states, TDT[dtype])
    e = P.expect_pauli(psi, H, mode=mode).cpu().numpy()
    S = np.abs(coeffs).sum()
    for b in range(B):
        ref = oracle_mod.expect(n, states[b], codes, coeffs).real
        assert abs(e[b] - ref) <= TOL[dtype]["E"] * S, (e[b], ref)


# ---------------------------------------------------------------------------
# value and adjoint gradient
# ---------------------------------------------------------------------------

def check_expect_grad(P, oracle_mod, n, gates, params_b, mats, codes, coeffs, dtype, mode, lie=False, init=None):
    """params_b: [B][P] float64 (rounded per dtype here)."""
    B = params_b.shape[0]
    circ = P.Circuit(n, gates, params_b.shape[1], W.round_mats(mats, dtype) if mats is not None else None)
    H = P.PauliSum(n, codes, coeffs)
    psi = torch.empty((B, 2 ** n), dtype=TDT[dtype], device="cuda")
    if init is None:
        P.state_init(psi)
    else:
        psi.copy_(dev(np.tile(init, (B, 1)), TDT[dtype]))
    psi0 = psi.clone()
    p = dev(params_b, rdt(dtype)) if params_b.shape[1] else None
    out = P.expect_grad(circ, p, H, psi=psi, want_gate_grad=lie, mode=mode)
    E, g = out[0].cpu().numpy(), out[1].cpu().numpy()
    S = np.abs(coeffs).sum()
    tol = TOL[dtype]
    for b in range(B):
        ref = oracle_mod.expect_grad(n, gates, W.round_params(params_b[b], dtype), codes, coeffs,
                                     W.round_mats(mats, dtype) if mats is not None else None,
                                     init=init, want_lie=lie)
        assert abs(E[b] - ref["E"]) <= tol["E"] * S, (b, E[b], ref["E"])
        if params_b.shape[1]:
            err = np.max(np.abs(g[b] - ref["grad"]))
            assert err <= tol["g"] * S, (b, err)
        if lie:
            # gate gradients are defined for the constant two-qubit (U2) gates; other rows are zero
            gl = out[2].cpu().numpy()[b]
            u2 = np.asarray(gates)[:, 0] == W.U2
            err = np.max(np.abs(gl[u2] - ref["lie"][u2])) if u2.any() else 0.0
            assert err <= tol["g"] * S, (b, err)
            assert np.all(gl[~u2] == 0.0)
    # the reverse sweep recomputes the initial states
    assert_amps(psi.cpu().numpy(), psi0.cpu().numpy(), dtype, 8 * len(gates), f"recomputed psi0 n={n} {mode}")
    return E, g


@pytest.mark.parametrize("mode", ["tiled", "plain", "fused"])
def test_cfg1_state_energy_gradient_c128(P, oracle_mod, mode):
    """n=10 complex128 HEA L=4, TFIM +ZZ +X: final state, <H>, gradient at 1e-12."""
    c = W.cfg1()
    st = run_gpu(P, 10, c["gates"], c["params"], None, "c128", mode)[0]
    ref = oracle_mod.expect_grad(10, c["gates"], c["params"], c["codes"], c["coeffs"], want_state=True)
    assert_amps(st, ref["state"], "c128", len(c["gates"]), f"cfg1 final state {mode}")
    check_expect_grad(P, oracle_mod, 10, c["gates"], c["params"][None, :], None, c["codes"], c["coeffs"], "c128", mode)


@pytest.mark.parametrize("dtype,mode", DM)
def test_hea_tfim_batched(P, oracle_mod, dtype, mode):
    """Reduced-size instance of the n=28 HEA/TFIM workload (same generator), batch 3."""
    c = W.cfg2(n=16, layers=3)
    r = np.random.default_rng(5)
    pb = np.stack([c["params"], r.uniform(0, 2 * np.pi, c["n_params"]), r.uniform(0, 2 * np.pi, c["n_params"])])
    check_expect_grad(P, oracle_mod, 16, c["gates"], pb, None, c["codes"], c["coeffs"], dtype, mode)


@pytest.mark.parametrize("dtype,mode", DM)
def test_xxz_batched(P, oracle_mod, dtype, mode):
    """Batched XXZ workload (n=16, L=8) on a subset of parameter sets."""
    c = W.cfg3(batch=4)
    check_expect_grad(P, oracle_mod, 16, c["gates"], c["params"], None, c["codes"], c["coeffs"], dtype, mode)


@pytest.mark.parametrize("dtype,mode", DM)
@pytest.mark.parametrize("n", [5, 11, 12, 14])
def test_random_circuits_all_kinds_with_gate_gradients(P, oracle_mod, dtype, mode, n):
    r = np.random.default_rng(500 + n)
    gates, params, mats = W.random_circuit(n, 80, r)
    codes, coeffs = W.random_pauli_sum(n, 10, r, max_weight=4)
    init = W.random_state(n, r)
    if dtype == "c64":
        init = init.astype(np.complex64).astype(np.complex128)
    pb = np.stack([params, r.uniform(0, 2 * np.pi, params.shape)])
    check_expect_grad(P, oracle_mod, n, gates, pb, mats, codes, coeffs, dtype, mode, lie=True, init=init)


@pytest.mark.parametrize("mode", ["tiled", "plain", "fused", "fused5"])
def test_fsim_brickwork_2d_tfim(P, oracle_mod, mode):
    """Reduced-size instance of the n=32 fSim / 2D TFIM workload: 4x4 lattice, depth 8."""
    c = W.cfg5(rows=4, cols=4, depth=8)
    check_expect_grad(P, oracle_mod, 16, c["gates"], c["params"][None, :], None, c["codes"], c["coeffs"], "c64", mode)


@pytest.mark.parametrize("mode", ["tiled", "plain", "fused", "fused5"])
def test_haar_brickwork_lie_gradients(P, oracle_mod, mode):
    """Haar brick-wall circuits with random 2-local H (the uneven-batch generator, small n)."""
    c = W.cfg4(count=3, n_lo=11, n_hi=14, d_lo=2, d_hi=6, seed=44)
    for cc in c["circuits"]:
        check_expect_grad(P, oracle_mod, cc["n"], cc["gates"], np.zeros((1, 0)), cc["mats"], cc["codes"],
                          cc["coeffs"], "c64", mode, lie=True)


def test_fused5_plan_is_used(P, oracle_mod):
    """The 5-qubit-block plan exists from 12 qubits on and its run differs in
    rounding from the 4-qubit plan's, both within the bar of the oracle."""
    n = 14
    r = np.random.default_rng(700)
    gates, params, mats = W.random_circuit(n, 120, r)
    codes, coeffs = W.random_pauli_sum(n, 12, r, max_weight=3)
    assert P.fused_plan_inspect(n, gates, len(params), 5)[4] < P.fused_plan_inspect(n, gates, len(params), 4)[4]
    circ = P.Circuit(n, gates, len(params), W.round_mats(mats, "c64"))
    H = P.PauliSum(n, codes, coeffs)
    p = dev(params[None], torch.float32)
    E4, g4 = P.expect_grad(circ, p, H, mode="fused")
    E5, g5 = P.expect_grad(circ, p, H, mode="fused5")
    torch.cuda.synchronize()
    assert not torch.equal(g4, g5)
    ref = oracle_mod.expect_grad(n, gates, W.round_params(params, "c64"), codes, coeffs, W.round_mats(mats, "c64"))
    S = np.abs(coeffs).sum()
    for E, g in ((E4, g4), (E5, g5)):
        assert abs(float(E[0]) - ref["E"]) <= 1e-5 * S
        assert np.max(np.abs(g.cpu().numpy()[0] - ref["grad"])) <= 1e-4 * S


@pytest.mark.parametrize("dtype,mode", [("c64", "fused"), ("c64", "fused5"), ("c64", "tiled"), ("c128", "tiled")])
@pytest.mark.parametrize("n", [16, 20])
def test_full_weight_pauli_terms_match_oracle(P, oracle_mod, n, dtype, mode):
    """Terms whose X-mask spans more qubits than a tile (X on every qubit,
    Y0 Y1 X...X, and random weight-n X/Y strings): the Pauli sum has no tiled
    plan, so the circuit passes run with the per-group Pauli kernels."""
    if n == 20 and dtype == "c128":
        pytest.skip("covered at n = 16")
    c = W.cfg2(n=n, layers=2)
    r = np.random.default_rng(600 + n)
    codes = [c["codes"]]
    full = np.ones((2, n), np.uint8)
    full[1, :2] = 2
    codes.append(full)
    codes.append(r.integers(1, 3, size=(3, n)).astype(np.uint8))
    codes = np.concatenate(codes)
    coeffs = np.concatenate([c["coeffs"], r.standard_normal(codes.shape[0] - len(c["coeffs"]))])
    print(f"full-weight Pauli n={n} {dtype} {mode}", flush=True)
    E, g = check_expect_grad(P, oracle_mod, n, c["gates"], c["params"][None, :], None, codes, coeffs, dtype, mode)
    assert np.max(np.abs(g)) > 1e-3


def test_autograd_function(P, oracle_mod):
    c = W.cfg2(n=12, layers=2)
    circ = P.Circuit(12, c["gates"], c["n_params"])
    H = P.PauliSum(12, c["codes"], c["coeffs"])
    theta = torch.tensor(c["params"], dtype=torch.float64, device="cuda", requires_grad=True)
    E = P.TcngEnergy.apply(theta, circ, H, torch.complex128)
    (2.0 * E).backward()
    ref = oracle_mod.expect_grad(12, c["gates"], c["params"], c["codes"], c["coeffs"])
    assert abs(E.item() - ref["E"]) < 1e-12 * 20
    np.testing.assert_allclose(theta.grad.cpu().numpy(), 2.0 * ref["grad"], atol=1e-11)


@pytest.mark.parametrize("mode", ["tiled", "plain"])
def test_autograd_gradcheck_and_shift_rule_c128(P, mode):
    """TcngEnergy against torch.autograd.gradcheck (central differences of its
    own forward) and against the exact two-term parameter-shift rule, both
    evaluated with GPU forward runs, complex128."""
    c = W.cfg2(n=11, layers=2)
    circ = P.Circuit(11, c["gates"], c["n_params"])
    H = P.PauliSum(11, c["codes"], c["coeffs"])
    S = np.abs(c["coeffs"]).sum()
    theta = torch.tensor(c["params"], dtype=torch.float64, device="cuda", requires_grad=True)
    f = lambda t: P.TcngEnergy.apply(t, circ, H, torch.complex128, mode)   # noqa: E731
    assert torch.autograd.gradcheck(f, (theta,), eps=1e-6, atol=1e-7, rtol=1e-5)
    E = f(theta)
    E.backward()
    g = theta.grad.cpu().numpy()
    Pn = c["n_params"]
    shifted = np.repeat(c["params"][None, :], 2 * Pn, axis=0)
    shifted[np.arange(Pn), np.arange(Pn)] += np.pi / 2
    shifted[Pn + np.arange(Pn), np.arange(Pn)] -= np.pi / 2
    Es = f(torch.tensor(shifted, dtype=torch.float64, device="cuda")).detach().cpu().numpy()
    shift = 0.5 * (Es[:Pn] - Es[Pn:])
    assert np.max(np.abs(shift - g)) <= 1e-12 * S
    assert np.max(np.abs(g)) > 1e-2


@pytest.mark.parametrize("mode", ["tiled", "fused", "fused5"])
def test_autograd_shift_rule_and_differences_c64(P, mode):
    """TcngEnergy in complex64 (float32 angles): its gradient against the
    two-term shift rule and a fourth-order central difference (h = 0.05),
    from batched GPU forward runs of the same op."""
    c = W.cfg2(n=12, layers=2)
    circ = P.Circuit(12, c["gates"], c["n_params"])
    H = P.PauliSum(12, c["codes"], c["coeffs"])
    S = np.abs(c["coeffs"]).sum()
    p32 = W.round_params(c["params"], "c64")
    theta = torch.tensor(p32, dtype=torch.float32, device="cuda", requires_grad=True)
    f = lambda t: P.TcngEnergy.apply(t, circ, H, torch.complex64, mode)   # noqa: E731
    E = f(theta)
    E.backward()
    g = theta.grad.double().cpu().numpy()
    Pn = c["n_params"]
    rows = []
    for d in (np.pi / 2, -np.pi / 2, 0.1, 0.05, -0.05, -0.1):
        x = np.repeat(p32[None, :], Pn, axis=0)
        x[np.arange(Pn), np.arange(Pn)] += d
        rows.append(x)
    Es = f(torch.tensor(np.concatenate(rows), dtype=torch.float32, device="cuda")).detach().double().cpu().numpy()
    Es = Es.reshape(6, Pn)
    shift = 0.5 * (Es[0] - Es[1])
    fd = (-Es[2] + 8 * Es[3] - 8 * Es[4] + Es[5]) / (12 * 0.05)
    assert np.max(np.abs(shift - g)) <= 1e-4 * S
    # the difference quotient divides float32 rounding of E (~1e-7 S) by h, and its
    # truncation error is h^4 |d^5E| / 30 <= 2e-7 S
    assert np.max(np.abs(fd - g)) <= 1e-4 * S
    assert np.max(np.abs(g)) > 1e-2


def test_results_are_deterministic(P):
    c = W.cfg3(batch=8)
    circ = P.Circuit(16, c["gates"], c["n_params"])
    H = P.PauliSum(16, c["codes"], c["coeffs"])
    p = dev(c["params"], torch.float32)
    e1, g1 = P.expect_grad(circ, p, H, batch=8)
    e2, g2 = P.expect_grad(circ, p, H, batch=8)
    assert torch.equal(e1, e2) and torch.equal(g1, g2)


def tilings(dtype, n):
    """Every tiling the library offers for this precision and qubit count."""
    mmax = 13 if dtype == "c64" else 12
    rbs = (4, 5) if dtype == "c64" else (3, 4)
    out = []
    for m in (mmax - 1, mmax):
        for rb in rbs:
            for rr in rbs:
                if 6 <= m - rb <= 9 and 6 <= m - rr <= 9 and min(n, m) >= max(rb, rr) + 6:
                    out.append((m, rb, rr))
    return out


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_every_tiling_matches_oracle(P, oracle_mod, dtype):
    n = 14
    r = np.random.default_rng(77)
    gates, params, mats = W.random_circuit(n, 90, r)
    codes, coeffs = W.random_pauli_sum(n, 12, r, max_weight=3)
    circ = P.Circuit(n, gates, len(params), W.round_mats(mats, dtype))
    H = P.PauliSum(n, codes, coeffs)
    ref = oracle_mod.expect_grad(n, gates, W.round_params(params, dtype), codes, coeffs, W.round_mats(mats, dtype),
                                 want_lie=True)
    S = np.abs(coeffs).sum()
    u2 = np.asarray(gates)[:, 0] == W.U2
    cfgs = tilings(dtype, n)
    assert len(cfgs) >= 4
    for cfg in cfgs:
        circ.configure(TDT[dtype], *cfg)
        assert circ.config(TDT[dtype]) == cfg
        E, g, gl = P.expect_grad(circ, dev(params[None, :], rdt(dtype)), H, dtype=TDT[dtype], want_gate_grad=True)
        assert abs(E.item() - ref["E"]) <= TOL[dtype]["E"] * S, cfg
        assert np.max(np.abs(g.cpu().numpy()[0] - ref["grad"])) <= TOL[dtype]["g"] * S, cfg
        assert np.max(np.abs(gl.cpu().numpy()[0][u2] - ref["lie"][u2])) <= TOL[dtype]["g"] * S, cfg


def test_autotune_picks_an_available_tiling_and_keeps_results(P, oracle_mod, tmp_path):
    c = W.cfg2(n=15, layers=2)
    circ = P.Circuit(15, c["gates"], c["n_params"])
    H = P.PauliSum(15, c["codes"], c["coeffs"])
    p = dev(c["params"][None, :], torch.float32)
    psi = P.new_state(15, 1, torch.complex64)
    cache = str(tmp_path / "tune.txt")
    cfg, ms = P.autotune(circ, p, H, psi, repeats=2, cache_path=cache)
    assert cfg in tilings("c64", 15) and ms > 0
    assert abs(psi[0, 0].item() - 1) < 1e-4          # initial state restored
    # a second call is answered from the cache file
    circ2 = P.Circuit(15, c["gates"], c["n_params"])
    cfg2, ms2 = P.autotune(circ2, p, H, psi, repeats=2, cache_path=cache)
    assert cfg2 == cfg and ms2 == pytest.approx(ms)
    # the choice among tiled, fused and fused5 is the circuit's "auto" mode
    assert circ.mode() in ("tiled", "fused", "fused5") and circ2.mode() == circ.mode()
    print(f"autotune n=15: mode {circ.mode()}, tiling {cfg}, {ms:.3f} ms", flush=True)
    ref = oracle_mod.expect_grad(15, c["gates"], W.round_params(c["params"], "c64"), c["codes"], c["coeffs"])
    S = np.abs(c["coeffs"]).sum()
    for mode in ("tiled", "auto"):
        E, g = P.expect_grad(circ, p, H, mode=mode)
        assert abs(E.item() - ref["E"]) <= 1e-5 * S
        assert np.max(np.abs(g.cpu().numpy()[0] - ref["grad"])) <= 1e-4 * S
    # complex128: the tiled tilings only
    circ3 = P.Circuit(15, c["gates"], c["n_params"])
    assert circ3.mode(torch.complex128) == "tiled" and circ3.mode() == "fused"   # defaults before tuning
    P.autotune(circ3, dev(c["params"][None, :], torch.float64), H, P.new_state(15, 1, torch.complex128), repeats=1)
    assert circ3.mode(torch.complex128) == "tiled"


# complex64 batches run on the matrix-core passes (one launch per tile size:
# 12-bit tiles, and 11-bit ones for 11-qubit circuits), complex128 on the tiled passes
@pytest.mark.parametrize("dtype,n_lo", [("c64", 11), ("c64", 12), ("c128", 11)])
def test_uneven_batch_matches_oracle(P, oracle_mod, dtype, n_lo):
    """Different circuits (qubit counts, depths, Hamiltonians; Haar brick-walls
    and parameterised ansatzes) in one uneven-batch evaluation."""
    print(f"uneven batch {dtype} n_lo={n_lo}", flush=True)
    r = np.random.default_rng(90)
    cs, hs, ps, refs = [], [], [], []
    c4 = W.cfg4(count=5, n_lo=n_lo, n_hi=15, d_lo=2, d_hi=9, seed=91)
    # two more at the smallest size (at 11 qubits: the group of smaller tiles)
    c4["circuits"] += W.cfg4(count=2, n_lo=n_lo, n_hi=n_lo, d_lo=2, d_hi=6, seed=92)["circuits"]
    for cc in c4["circuits"]:
        cs.append(P.Circuit(cc["n"], cc["gates"], 0, W.round_mats(cc["mats"], dtype)))
        hs.append(P.PauliSum(cc["n"], cc["codes"], cc["coeffs"]))
        ps.append(None)
        refs.append((cc["n"], cc["gates"], None, cc["codes"], cc["coeffs"], W.round_mats(cc["mats"], dtype)))
    for n, L in ((12, 2), (15, 3)):
        w = W.cfg2(n=n, layers=L)
        cs.append(P.Circuit(n, w["gates"], w["n_params"]))
        hs.append(P.PauliSum(n, w["codes"], w["coeffs"]))
        ps.append(dev(w["params"], rdt(dtype)))
        refs.append((n, w["gates"], W.round_params(w["params"], dtype), w["codes"], w["coeffs"], None))
    E, grads, ggs = P.expect_grad_multi(cs, hs, ps, dtype=TDT[dtype], want_gate_grad=True)
    E = E.cpu().numpy()
    for i, (n, g, pr, codes, coeffs, mats) in enumerate(refs):
        ref = oracle_mod.expect_grad(n, g, pr, codes, coeffs, mats, want_lie=True)
        S = np.abs(coeffs).sum()
        assert abs(E[i] - ref["E"]) <= TOL[dtype]["E"] * S, i
        if pr is not None:
            assert np.max(np.abs(grads[i].cpu().numpy() - ref["grad"])) <= TOL[dtype]["g"] * S, i
        u2 = np.asarray(g)[:, 0] == W.U2
        if u2.any():
            assert np.max(np.abs(ggs[i].cpu().numpy()[u2] - ref["lie"][u2])) <= TOL[dtype]["g"] * S, i


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_uneven_bound_batch_and_graph_replays(P, oracle_mod, dtype):
    """An uneven batch bound once (tables uploaded at creation, every circuit
    started from |0...0> inside the launch): launches and graph replays with
    new angles written into the bound tensors match the per-call uneven
    evaluation bit for bit, and the oracle."""
    print(f"bound uneven batch {dtype}", flush=True)
    c4 = W.cfg4(count=5, n_lo=11, n_hi=15, d_lo=2, d_hi=7, seed=95)["circuits"]
    cs = [P.Circuit(c["n"], c["gates"], 0, W.round_mats(c["mats"], dtype)) for c in c4]
    hs = [P.PauliSum(c["n"], c["codes"], c["coeffs"]) for c in c4]
    refs = [(c["n"], c["gates"], c["codes"], c["coeffs"], W.round_mats(c["mats"], dtype), None) for c in c4]
    ps = [None] * len(c4)
    r = np.random.default_rng(96)
    for n, L in ((12, 2), (14, 2)):
        w = W.cfg2(n=n, layers=L)
        cs.append(P.Circuit(n, w["gates"], w["n_params"]))
        hs.append(P.PauliSum(n, w["codes"], w["coeffs"]))
        ps.append(torch.zeros(w["n_params"], dtype=rdt(dtype), device="cuda"))
        refs.append((n, w["gates"], w["codes"], w["coeffs"], None, w["n_params"]))
    M = P.Multi(cs, hs, ps, dtype=TDT[dtype], want_gate_grad=True, init_basis=0)
    replay = M.graph()
    for rep in range(3):
        newp = [None if p is None else W.round_params(r.uniform(0, 2 * np.pi, p.numel()), dtype) for p in ps]
        for p, v in zip(ps, newp):
            if p is not None:
                p.copy_(dev(v, rdt(dtype)))
        E, gr, gg = (M.launch() if rep == 0 else replay())
        torch.cuda.synchronize()
        E, gr, gg = E.clone(), [g.clone() for g in gr], [g.clone() for g in gg]
        E0, gr0, gg0 = P.expect_grad_multi(cs, hs, [None if p is None else p.clone() for p in ps], dtype=TDT[dtype],
                                           want_gate_grad=True)
        torch.cuda.synchronize()
        assert torch.equal(E, E0)
        assert all(torch.equal(a, b) for a, b in zip(gr, gr0)) and all(torch.equal(a, b) for a, b in zip(gg, gg0))
        if rep < 2:
            for i, (n, g, codes, coeffs, mats, npar) in enumerate(refs):
                ref = oracle_mod.expect_grad(n, g, newp[i] if npar else None, codes, coeffs, mats, want_lie=True)
                S = np.abs(coeffs).sum()
                assert abs(float(E[i]) - ref["E"]) <= TOL[dtype]["E"] * S, (rep, i)
                if npar:
                    assert np.max(np.abs(gr[i].cpu().numpy() - ref["grad"])) <= TOL[dtype]["g"] * S, (rep, i)
                u2 = np.asarray(g)[:, 0] == W.U2
                if u2.any():
                    assert np.max(np.abs(gg[i].cpu().numpy()[u2] - ref["lie"][u2])) <= TOL[dtype]["g"] * S, (rep, i)
    M.close()


# ---------------------------------------------------------------------------
# graph capture: replays with new angles written into the captured buffer
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype,mode", [("c64", "fused"), ("c64", "fused5"), ("c64", "tiled"), ("c64", "plain"),
                                        ("c128", "tiled")])
def test_graph_replays_match_eager_and_oracle(P, oracle_mod, dtype, mode):
    n = 12
    c = W.cfg2(n=n, layers=3)
    circ = P.Circuit(n, c["gates"], c["n_params"])
    H = P.PauliSum(n, c["codes"], c["coeffs"])
    S = np.abs(c["coeffs"]).sum()
    r = np.random.default_rng(77)
    params = torch.zeros((1, c["n_params"]), dtype=rdt(dtype), device="cuda")
    psi = torch.empty((1, 2 ** n), dtype=TDT[dtype], device="cuda")
    lam = torch.empty_like(psi)
    energy = torch.empty(1, dtype=torch.float64, device="cuda")
    grad = torch.empty((1, c["n_params"]), dtype=torch.float64, device="cuda")
    g = P.Graph(circ, params, H, psi, lam, energy, grad, mode=mode)
    for rep in range(3):
        newp = W.round_params(r.uniform(0, 2 * np.pi, c["n_params"]), dtype)
        params.copy_(dev(newp[None], rdt(dtype)))
        g.launch()
        torch.cuda.synchronize()
        E_ref, g_ref = P.expect_grad(circ, dev(newp[None], rdt(dtype)), H, dtype=TDT[dtype], mode=mode)
        torch.cuda.synchronize()
        # same kernels, same order, fixed-order sums: bit-identical to the eager call
        assert energy.item() == E_ref.item()
        assert torch.equal(grad, g_ref)
        if rep == 0:
            ref = oracle_mod.expect_grad(n, c["gates"], newp, c["codes"], c["coeffs"])
            E_o, g_o = ref["E"], ref["grad"]
            tol = TOL[dtype]
            assert abs(energy.item() - E_o) <= tol["E"] * S
            assert np.max(np.abs(grad.cpu().numpy()[0] - g_o)) <= tol["g"] * S
    g.close()
