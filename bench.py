"""Benchmark of the statevector hot path on one MI355X.

A step is one value-and-adjoint-gradient evaluation (forward sweep, H|psi>
and <H>, reverse sweep, final reductions) of the measured workload, with all
inputs resident in HBM.  Default workload: n=28 qubits, complex64, the
hardware-efficient ansatz (RY, RZ on every qubit, CNOT ladder) with 12 layers
(996 gates, 672 angles) and the 1D TFIM -sum ZZ - 0.5 sum X.

value = logical amplitude-updates per second: every gate of the circuit is
counted once for the forward sweep and twice for the reverse sweep (psi and
lambda are both un-computed), each updating 2^n amplitudes per batch member:
3 * G * 2^n * batch per step.  Fused passes count as the gates they apply.

Prints one JSON line (see the keys below).  Only one GPU is supported.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
# FP32 / FP64 vector peak without packed-FP32 instructions (not used by this
# build): 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
ALU_PEAK_TFLOPS = 78.6

# algorithmic flops per amplitude of one gate application (complex
# arithmetic: multiply 6, add 2; real x complex 2) and of one gradient term
KIND = {n: i for i, n in enumerate(["RX", "RY", "RZ", "H", "X", "Y", "Z", "S", "CNOT", "CZ", "RZZ", "FSIM", "U1",
                                    "U2"])}
APPLY_FLOPS = {"RX": 6, "RY": 6, "RZ": 6, "H": 4, "X": 0, "Y": 0, "Z": 0, "S": 0, "CNOT": 0, "CZ": 0, "RZZ": 6,
               "FSIM": 4.5, "U1": 14, "U2": 30}
# Im<l|G|p> per amplitude: RX/RY/RZ/RZZ 4; FSIM theta on half and phi on a
# quarter of the amplitudes; U2: the 16-entry cotangent, 4 complex MACs per amplitude
GRAD_FLOPS = {"RX": 4, "RY": 4, "RZ": 4, "RZZ": 4, "FSIM": 3, "U2": 32}
KIND_NAME = {v: k for k, v in KIND.items()}

# HBM bytes per launch measured with rocprofv3 counters (FETCH_SIZE and
# WRITE_SIZE in separate runs, scaled by what each reads for a 2 GiB device
# copy: x1.99993 and x1.0), keyed by workload and kernel family, valid only
# for the kernel sources they were taken with (hash below).
KERNEL_SOURCES = {
    "tile": ["common.h", "devutil.h", "gates.h", "kernels.h", "kern_tile.hip", "plan.cpp", "plan.h"],
    "fused": ["common.h", "devutil.h", "gates.h", "kernels.h", "kern_fused.hip", "plan.cpp", "plan.h"],
    "pauli": ["common.h", "devutil.h", "kernels.h", "kern_pauli.hip"],
    "plain": ["common.h", "devutil.h", "gates.h", "kernels.h", "kern_plain.hip"],
}
TRAFFIC = {
    ("hea_n28_L12_tfim", "rev_tile"): (8.6047e+09, "34cae1f9856ca791"),
    ("hea_n28_L12_tfim", "fwd_tile"): (4.2952e+09, "34cae1f9856ca791"),
    ("hea_n28_L12_tfim", "fused_rev"): (8.7870e+09, "e6701c5affaf0dc5"),
    ("hea_n28_L12_tfim", "fused_fwd"): (4.2968e+09, "e6701c5affaf0dc5"),
    ("fsim_brickwork_n32_d20_tfim2d", "rev_tile"): (1.3745e+11, "34cae1f9856ca791"),
    ("fsim_brickwork_n32_d20_tfim2d", "fwd_tile"): (6.8719e+10, "34cae1f9856ca791"),
    ("mipt_haar_n20_d40_b1000_p0.2", "fused_fwd"): (1.6976e+10, "e6701c5affaf0dc5"),
    ("qml_mnist_n10_l40_b15000", "fused_rev"): (5.0972e+08, "e6701c5affaf0dc5"),
    ("qml_mnist_n10_l40_b15000", "fused_fwd"): (2.4651e+08, "e6701c5affaf0dc5"),
    ("qml_cifar100_n12_l30_b5000", "fused_rev"): (6.7451e+08, "e6701c5affaf0dc5"),
    ("qml_cifar100_n12_l30_b5000", "fused_fwd"): (3.2845e+08, "e6701c5affaf0dc5"),
    ("haar_brickwork_uneven_1024", "fused_rev"): (1.5136e+10, "e6701c5affaf0dc5"),
    ("tfim_coo_n24", "pauli_coo"): (1.3422e+10, "ba2bf1c0385a9695"),
    ("single_gate_sweep_n30_c64", "plain_gate"): (1.7186e+10, "9295abc6ba4265a5"),
}


def source_hash(kernel):
    import hashlib
    h = hashlib.sha1()
    d = os.path.join(ROOT, "paper_2602_14167_amd", "csrc")
    group = ("fused" if kernel.startswith("fused") else "pauli" if kernel.startswith("pauli")
             else "plain" if kernel.startswith("plain") else "tile")
    for f in KERNEL_SOURCES[group]:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_name, kernel):
    """Counter-measured bytes per launch, or None if not taken for these sources."""
    rec = TRAFFIC.get((workload_name, kernel))
    if rec is None or rec[1] != source_hash(kernel):
        return None
    return rec[0]
FAMILIES = ["fwd_tile", "rev_tile", "pauli_tile", "gate1", "gate2", "gatek", "rev1", "rev2", "pauli_group",
            "finish", "init", "fused_fwd", "fused_rev", "fused_grad", "mipt_hist", "mipt_decide", "mipt_collapse",
            "pauli_coo", "shadow_sum", "shadow_pick", "qml"]
MFMA_F32_PEAK_TFLOPS = 157.3   # dense float32 matrix-core peak


def workload(name):
    import workloads as W
    if name.startswith("gates") or name in ("mipt20", "coo22", "coo24", "shadow20", "qml_mnist", "qml_cifar100"):
        return None
    if name == "hea28":
        w = W.cfg2()
        w["batch"] = 1
        w["params"] = w["params"][None, :]
        return w
    if name == "hea30":
        w = W.cfg2(n=30)
        w["batch"] = 1
        w["params"] = w["params"][None, :]
        return w
    if name == "xxz16_b2048":
        return W.cfg3()
    if name == "xxz16_per_circuit":
        w = W.cfg3()
        w["name"] = "hea_n16_L8_xxz_per_circuit"
        return w
    if name == "hea10":
        w = W.cfg1()
        w["batch"] = 1
        w["params"] = w["params"][None, :]
        return w
    if name == "haar_uneven":
        return W.cfg4()
    if name == "fsim32":
        w = W.cfg5()
        w["batch"] = 1
        w["params"] = w["params"][None, :]
        return w
    raise SystemExit(f"unknown workload {name}")


def algorithmic_bytes(family, n, s, batch, n_pauli_passes):
    """HBM bytes one launch of a family must move (per batch member x batch)."""
    amp = (2 ** n) * s * batch
    if family == "fwd_tile":
        return 2 * amp                      # read + write psi
    if family in ("rev_tile", "fused_rev"):
        return 4 * amp                      # read + write psi and lambda
    if family == "fused_fwd":
        return 2 * amp
    if family == "pauli_tile":
        # first pass: read psi, write lambda; later passes also read lambda
        return None if n_pauli_passes == 0 else (2 * amp + 3 * amp * (n_pauli_passes - 1)) / n_pauli_passes
    return None


def sweep_flops(gates, n, batch, with_u2_grad=False):
    """(forward, reverse) algorithmic flops of one evaluation: every gate
    applied once forward; in reverse applied to psi and lambda plus its
    gradient term."""
    fwd = rev = 0.0
    for g in gates:
        k = KIND_NAME[int(g[0])]
        a = APPLY_FLOPS[k]
        grad = GRAD_FLOPS.get(k, 0) if (k != "U2" or with_u2_grad) else 0
        fwd += a
        rev += 2 * a + grad
    amp = float(2 ** n) * batch
    return fwd * amp, rev * amp


def roofline_entry(kernel, flops_per_launch, bytes_per_launch, avg_ms, compute="alu"):
    """Roofline of one kernel family from its average launch: compute-bound
    (vector ALU) when its arithmetic intensity exceeds the ridge point,
    HBM-bound otherwise."""
    t = avg_ms * 1e-3
    ai = flops_per_launch / bytes_per_launch
    peak = MFMA_F32_PEAK_TFLOPS if compute == "mfma" else ALU_PEAK_TFLOPS
    ridge = peak * 1e12 / (HBM_PEAK_GBS * 1e9)
    gbs = bytes_per_launch / t / 1e9
    tfl = flops_per_launch / t / 1e12
    hbm = {"achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}
    alu = {"achieved": round(tfl, 2), "peak": peak, "unit": "TFLOP/s", "frac": round(tfl / peak, 4)}
    main, other = (alu, hbm) if ai > ridge else (hbm, alu)
    out = {"bound": compute if ai > ridge else "hbm", **main, "traffic": None, "kernel": kernel,
           "flops_per_launch": flops_per_launch, "bytes_per_launch": bytes_per_launch,
           "avg_launch_ms": round(avg_ms, 4), "intensity_flop_per_byte": round(ai, 2),
           "ridge_flop_per_byte": round(ridge, 2), "other_roof": other}
    return out


def fused_roofline(kernel, gate_flops, bytes_per_launch, block_flops, avg_ms):
    """Roofline of a matrix-core pass against the method's own work.  The
    gate-by-gate flops of the gates the pass applies (sweep_flops) over its
    algorithmic bytes give the arithmetic intensity; the roof is
    min(matrix-core peak, intensity x HBM peak), so a pass below the ridge is
    HBM-bound and `frac` is its algorithmic bytes per second over 8 TB/s.  The
    dense 16 x 16 block products do more flops than the gates need; their
    rate against the matrix-core peak is reported beside as `mfma_util`."""
    t = avg_ms * 1e-3
    ai = gate_flops / bytes_per_launch
    ridge = MFMA_F32_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    gbs = bytes_per_launch / t / 1e9
    tfl = gate_flops / t / 1e12
    if ai < ridge:
        main = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4)}
    else:
        main = {"bound": "mfma", "achieved": round(tfl, 2), "peak": MFMA_F32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(tfl / MFMA_F32_PEAK_TFLOPS, 4)}
    return {**main, "traffic": None, "kernel": kernel, "gate_level_flops_per_launch": gate_flops,
            "bytes_per_launch": bytes_per_launch, "avg_launch_ms": round(avg_ms, 4),
            "intensity_flop_per_byte": round(ai, 2), "ridge_flop_per_byte": round(ridge, 2),
            "roof": round(min(MFMA_F32_PEAK_TFLOPS, ai * HBM_PEAK_GBS / 1e3), 2), "roof_unit": "TFLOP/s",
            "achieved_gate_TFLOP_s": round(tfl, 2),
            "block_flops_per_launch": block_flops,
            "mfma_util": round(block_flops / t / 1e12 / MFMA_F32_PEAK_TFLOPS, 4)}


def copy_ceiling(torch, nbytes):
    """Measured device-to-device copy rate (read + write bytes per second) of
    torch's copy kernel on a buffer of the state's size."""
    n = max(nbytes // 4, 1)
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return {"bytes": 2 * n * 4, "avg_ms": round(ms, 4), "GB_s": round(2 * n * 4 / (ms * 1e-3) / 1e9, 1)}


def run_uneven(args, w, P, torch):
    """The uneven batch (1024 Haar brick-wall circuits of 12..22 qubits): one
    step = value and Lie-algebra gate gradients of every circuit."""
    cs = w["circuits"]
    circs = [P.Circuit(c["n"], c["gates"], 0, c["mats"]) for c in cs]
    hams = [P.PauliSum(c["n"], c["codes"], c["coeffs"]) for c in cs]
    cdt = torch.complex64
    count = len(cs)
    # bound once: launch tables in the workspace, every circuit started from
    # |0...0> inside its first forward pass; a step enqueues kernels only
    multi = P.Multi(circs, hams, [None] * count, dtype=cdt, want_gate_grad=True, init_basis=0)
    step = multi.graph() if args.graph else multi.launch

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    prof = not args.no_profile and not args.graph   # replays record no per-launch events
    if prof:
        P.check(P.lib().tcng_profile_begin(200000))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        E, _, _ = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    fam = {}
    if prof:
        for i, name in enumerate(FAMILIES):
            cnt, tot = ctypes.c_int32(), ctypes.c_double()
            P.check(P.lib().tcng_profile_query(i, ctypes.byref(cnt), ctypes.byref(tot)))
            if cnt.value:
                fam[name] = dict(launches=cnt.value, total_ms=tot.value, avg_ms=tot.value / cnt.value)
        P.check(P.lib().tcng_profile_end())
    G = sum(len(c["gates"]) for c in cs)
    amp = sum(3.0 * len(c["gates"]) * 2 ** c["n"] for c in cs)
    fused = True   # complex64 batches run on the matrix-core passes
    roofline = None
    if fused and "fused_rev" in fam:
        # reverse sweep (dominant): psi and lambda read and written per pass; 3 block products per amplitude
        plans = [P.fused_plan_inspect(c["n"], c["gates"], 0) for c in cs]
        rev_bytes = sum(pl[3] * 4 * 8 * 2 ** c["n"] for c, pl in zip(cs, plans))
        blk_flops = sum(3 * 8.0 * 16 * 2 ** c["n"] * pl[4] for c, pl in zip(cs, plans))
        gate_flops = sum(sweep_flops(c["gates"], c["n"], 1, with_u2_grad=True)[1] for c in cs)
        L = fam["fused_rev"]["launches"] / args.steps
        roofline = fused_roofline("fused_rev", gate_flops / L, rev_bytes / L, blk_flops / L,
                                  fam["fused_rev"]["avg_ms"])
        roofline["traffic"] = measured_traffic(w["name"], "fused_rev")
    elif "rev_tile" in fam:
        # algorithmic bytes and flops of the reverse sweep (dominant) over one step
        rev_bytes = sum(c2.num_passes() * 4 * 8 * 2 ** c["n"] for c, c2 in zip(cs, circs))
        rev_flops = sum(sweep_flops(c["gates"], c["n"], 1, with_u2_grad=True)[1] for c in cs)
        L = fam["rev_tile"]["launches"] / args.steps
        roofline = roofline_entry("rev_tile", rev_flops / L, rev_bytes / L, fam["rev_tile"]["avg_ms"])
    return {
        "metric": "amplitude-updates/s", "value": amp / dt, "unit": "amplitude-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64 (f32 state, f64 reductions)", "data": "synthetic",
        "config": {"workload": w["name"], "circuits": count, "gates": G,
                   "mode": ("fused" if fused else "tiled") + ", uneven batch", "graph": bool(args.graph),
                   "parallelism": "single GPU"},
        "evals_per_s": count / dt, "roofline": roofline,
        "kernels": {k: {"launches_per_step": v["launches"] / args.steps, "avg_ms": round(v["avg_ms"], 4)}
                    for k, v in fam.items()},
    }


def run_per_circuit(args, w, P, torch):
    """One evaluation per launch sequence (batch 1), the parameter sets of
    the batched n=16 XXZ workload taken in turn: the per-circuit baseline of
    the batched launch (complex128 and per-gate kernels by default), eager or
    as a replayed graph with the angles written into the captured buffer."""
    n, G = w["n"], len(w["gates"])
    cdt = torch.complex64 if args.dtype == "c64" else torch.complex128
    rdt = torch.float32 if args.dtype == "c64" else torch.float64
    circ = P.Circuit(n, w["gates"], w["n_params"])
    H = P.PauliSum(n, w["codes"], w["coeffs"])
    sets = torch.tensor(np.asarray(w["params"]), dtype=rdt, device="cuda")
    nsets = min(int(args.sets), sets.shape[0])
    params = torch.empty((1, w["n_params"]), dtype=rdt, device="cuda")
    psi = torch.empty((1, 2 ** n), dtype=cdt, device="cuda")
    lam = torch.empty_like(psi)
    energy = torch.empty(1, dtype=torch.float64, device="cuda")
    grad = torch.empty((1, w["n_params"]), dtype=torch.float64, device="cuda")
    run_mode = circ.mode(cdt) if args.mode == "auto" else args.mode
    graph = P.Graph(circ, params, H, psi, lam, energy, grad, mode=run_mode) if args.graph else None
    nbytes = ctypes.c_size_t()
    P.check(P.lib().tcng_workspace_size(circ.handle, H.handle, 0 if args.dtype == "c64" else 1, 1,
                                        P.MODES[run_mode], ctypes.byref(nbytes)))
    ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device="cuda")

    def one(i):
        params.copy_(sets[i:i + 1])
        if graph is not None:
            graph.launch()
        else:
            P.state_init(psi)
            P.expect_grad(circ, params, H, psi=psi, lam=lam, mode=run_mode, ws=ws)

    for i in range(min(args.warmup, nsets)):
        one(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for i in range(nsets):
            one(i)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / (args.steps * nsets)
    if graph is not None:
        graph.close()
    return {
        "metric": "amplitude-updates/s", "value": 3.0 * G * 2 ** n / dt, "unit": "amplitude-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * nsets * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": w["name"], "n_qubits": n, "gates": G, "parameter_sets": nsets, "mode": run_mode,
                   "graph": bool(args.graph), "parallelism": "single GPU"},
        "evals_per_s": 1.0 / dt, "us_per_eval": dt * 1e6,
    }


def run_gate_sweep(args, P, torch, n):
    """Per-gate HBM bandwidth of the streaming gate kernels (the unfused path)
    for low and high target qubits: RY (dense real 2x2), RZ (diagonal), CNOT
    (q, q+1) and a Haar 4x4 on (q, q') with q' low or high; complex64 or
    complex128 (--dtype).  Bytes per launch: the state read and written once."""
    import workloads as W
    rng = np.random.default_rng(7)
    c64 = args.dtype == "c64"
    s = 8 if c64 else 16
    # a device copy of the state's size first: the HBM reference of the sweep
    # (and the counter calibration of its profiles)
    copy = copy_ceiling(torch, (2 ** n) * s)
    psi = torch.empty((1, 2 ** n), dtype=torch.complex64 if c64 else torch.complex128, device="cuda")
    P.state_init(psi)
    cases = []
    targets = [0, 1, 2, 3, 4, 6, 8, 12, 16, 20, 24, n - 2]
    for q in targets:
        cases.append(("RY", [W.gate(W.RY, q, p0=0)], None))
        cases.append(("RZ", [W.gate(W.RZ, q, p0=0)], None))
        cases.append(("CNOT", [W.gate(W.CNOT, q, q + 1)], None))
        mats = W.haar_u4(rng)[None]
        cases.append(("U2low", [W.gate(W.U2, max(q, 1), 0, mat=0)], mats))
        cases.append(("U2high", [W.gate(W.U2, q, n - 1 if q != n - 1 else n - 2, mat=0)], mats))
    theta = torch.tensor([[0.37]], dtype=torch.float32 if c64 else torch.float64, device="cuda")
    res = []
    for name, g, mats in cases:
        circ = P.Circuit(n, g, 1 if name in ("RY", "RZ") else 0, mats)
        prm = theta if circ.n_params else None
        for _ in range(2):
            P.run_circuit(circ, prm, psi, mode="plain")
        torch.cuda.synchronize()
        reps = 10
        P.check(P.lib().tcng_profile_begin(64))
        for _ in range(reps):
            P.run_circuit(circ, prm, psi, mode="plain")
        torch.cuda.synchronize()
        fam = 3 if len(g) and g[0][2] < 0 else 4
        cnt, tot = ctypes.c_int32(), ctypes.c_double()
        P.check(P.lib().tcng_profile_query(fam, ctypes.byref(cnt), ctypes.byref(tot)))
        P.check(P.lib().tcng_profile_end())
        ms = tot.value / max(cnt.value, 1)
        gbs = 2 * s * 2 ** n / (ms * 1e-3) / 1e9
        res.append({"gate": name, "q": [int(g[0][1])] + ([int(g[0][2])] if g[0][2] >= 0 else []),
                    "ms": round(ms, 4), "GB_s": round(gbs, 1)})
    gb = sorted(r["GB_s"] for r in res)
    med = gb[len(gb) // 2]
    ms_med = 2 * s * 2 ** n / (med * 1e9) * 1e3
    return {
        "metric": "amplitude-updates/s", "value": 2 ** n / (ms_med * 1e-3), "unit": "amplitude-updates/s",
        "n_gpus": 1, "steps": 10, "warmup": 2, "ms_per_step": ms_med, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": f"single_gate_sweep_n{n}_{args.dtype}", "n_qubits": n, "cases": len(res),
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": med, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(med / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(f"single_gate_sweep_n{n}_{args.dtype}", "plain_gate"),
                     "kernel": "gate1/gate2 (median case)", "bytes_per_launch": 2 * s * 2 ** n,
                     "min_GB_s": gb[0], "max_GB_s": gb[-1], "cases": len(gb),
                     "cases_at_or_above_70pct": sum(1 for v in gb if v >= 0.7 * HBM_PEAK_GBS)},
        "copy_ceiling": copy,
        "gate_sweep": res,
    }


def run_mipt(args, P, torch):
    """Monitored Haar brick-wall trajectories (n = 20, 40 steps, 1000
    trajectories, p = 0.2, complex64): one step = every trajectory from
    |0...0> through all time steps, the record and Born log-probabilities."""
    import workloads as W
    n, S, B, p = 20, 40, 1000, 0.2
    w = W.mipt_workload(n, S, B, p, seed=7)
    G = w["gates"].shape[0]
    step_c = P.Circuit(n, w["gates"], 0, mats=np.tile(np.eye(4), (G, 1, 1)))
    mats = torch.as_tensor(w["mats"].astype(np.complex64)).cuda().contiguous()
    u = torch.as_tensor(w["u"]).cuda().contiguous()
    psi = torch.empty((B, 2 ** n), dtype=torch.complex64, device="cuda")
    need = ctypes.c_size_t()
    P.check(P.lib().tcng_mipt_workspace_size(step_c.handle, n, B, ctypes.byref(need)))
    ws = torch.empty(int(need.value), dtype=torch.uint8, device="cuda")
    steps = max(1, min(args.steps, 5))

    def one():
        P.state_init(psi)
        return P.mipt_run(step_c, mats, psi, u, p, ws=ws)

    for _ in range(min(args.warmup, 1)):
        one()
    torch.cuda.synchronize()
    prof = not args.no_profile
    if prof:
        P.check(P.lib().tcng_profile_begin(4000 * (steps + 1)))
    t0 = time.perf_counter()
    for _ in range(steps):
        rec, logp, _ = one()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    fam = {}
    if prof:
        for i, name in enumerate(FAMILIES):
            cnt, tot = ctypes.c_int32(), ctypes.c_double()
            P.check(P.lib().tcng_profile_query(i, ctypes.byref(cnt), ctypes.byref(tot)))
            if cnt.value:
                fam[name] = dict(launches=cnt.value, total_ms=tot.value, avg_ms=tot.value / cnt.value)
        P.check(P.lib().tcng_profile_end())
    # algorithmic HBM bytes per step: fused passes read + write every state (the
    # first pass of a time step also applies the previous step's collapse); the
    # final collapse reads + writes the states of members measuring in the last step
    meas = w["u"] >= 1 - p
    amp = 2 ** n * 8
    fwd_passes = P.fused_plan_inspect(n, w["gates"], 0)[3]
    # the histogram of round r (the step's measured qubits of rank 8r .. 8r + 7) reads, for a
    # member with a qubit in that round, the amplitudes consistent with the 8r earlier outcomes
    cnt = meas.sum(axis=2)
    hist_states = sum(float(((cnt > 8 * r)) .sum()) * 0.5 ** (8 * r) for r in range((n + 7) // 8))
    alg = {"fused_fwd": S * fwd_passes * B * 2.0 * amp, "mipt_hist": hist_states * amp,
           "mipt_collapse": float(meas[:, -1, :].any(axis=1).sum()) * 2.0 * amp}
    roofline = None
    if fam:
        dom = max((k for k in alg if k in fam), key=lambda k: fam[k]["total_ms"])
        L = fam[dom]["launches"] / steps
        t = fam[dom]["avg_ms"] * 1e-3
        gbs = alg[dom] / L / t / 1e9
        roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic("mipt_haar_n20_d40_b1000_p0.2", dom), "kernel": dom,
                    "bytes_per_launch": alg[dom] / L, "avg_launch_ms": round(fam[dom]["avg_ms"], 4),
                    "algorithmic_bytes_per_step": {k: v for k, v in alg.items()}}
    out = {
        "metric": "trajectories/s", "value": B / dt, "unit": "trajectories/s", "n_gpus": 1, "steps": steps,
        "warmup": min(args.warmup, 1), "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64 (f32 state, f64 probabilities)", "data": "synthetic",
        "config": {"workload": "mipt_haar_n20_d40_b1000_p0.2", "n_qubits": n, "time_steps": S, "trajectories": B,
                   "p": p, "gates_per_step": G, "parallelism": "single GPU"},
        "ms_per_trajectory": dt / B * 1e3,
        "paper_reference": {"ms_per_trajectory": 84.16, "hardware": "NVIDIA H200 (context, not the target)"},
        "measurements_per_trajectory": float(meas.sum()) / B,
        "logp_mean": float(logp.mean().item()),
        "roofline": roofline,
        "kernels": {k: {"launches_per_step": v["launches"] / steps, "avg_ms": round(v["avg_ms"], 4)}
                    for k, v in fam.items()},
    }
    if not args.no_cpu_baseline:
        import oracle
        k, t = 1, 0.0
        while True:
            t0 = time.perf_counter()
            oracle.mipt(n, w["gates"], w["mats"][0, :k], w["u"][0, :k], p)
            t = time.perf_counter() - t0
            if t * 2 > 15.0 or k >= S:
                break
            k = min(S, max(k + 1, int(k * 15.0 / max(t, 1e-3) * 0.5)))
        out["cpu_baseline"] = {"value": (k / S) / t, "unit": "trajectories/s", "cores": 1, "kind": "oracle", **host_info(),
                               "sample": f"first {k} of {S} steps of one trajectory at n={n} (complex128, single "
                                         f"thread), {t:.1f} s, scaled to whole trajectories"}
    return out


def run_coo(args, P, torch, n):
    """Sparse (COO) matrix of the open TFIM (-sum ZZ - sum X) on n qubits in
    complex128: one step = every entry of the matrix written to HBM."""
    import workloads as W
    codes, coeffs = W.tfim_1d(n, 1.0, 1.0)
    H = P.PauliSum(n, codes, coeffs)
    g = ctypes.c_int32()
    P.check(P.lib().tcng_pauli_coo_info(H.handle, ctypes.byref(g)))
    G, dim = g.value, 1 << n
    nnz = G * dim
    rows = torch.empty(nnz, dtype=torch.int64, device="cuda")
    cols = torch.empty(nnz, dtype=torch.int64, device="cuda")
    vals = torch.empty(nnz, dtype=torch.complex128, device="cuda")
    args_c = (H.handle, 0, dim, ctypes.c_void_p(rows.data_ptr()), ctypes.c_void_p(cols.data_ptr()),
              ctypes.c_void_p(vals.data_ptr()), P._stream())

    def one():
        P.check(P.lib().tcng_pauli_coo(*args_c))

    for _ in range(max(args.warmup, 1)):
        one()
    torch.cuda.synchronize()
    prof = not args.no_profile
    if prof:
        P.check(P.lib().tcng_profile_begin(args.steps + 8))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    fam = {}
    if prof:
        for i, name in enumerate(FAMILIES):
            cnt, tot = ctypes.c_int32(), ctypes.c_double()
            P.check(P.lib().tcng_profile_query(i, ctypes.byref(cnt), ctypes.byref(tot)))
            if cnt.value:
                fam[name] = dict(launches=cnt.value, total_ms=tot.value, avg_ms=tot.value / cnt.value)
        P.check(P.lib().tcng_profile_end())
    nbytes = 32.0 * nnz
    roofline = None
    if "pauli_coo" in fam:
        t = fam["pauli_coo"]["avg_ms"] * 1e-3
        gbs = nbytes / t / 1e9
        roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic(f"tfim_coo_n{n}", "pauli_coo"),
                    "kernel": "pauli_coo", "bytes_per_launch": nbytes, "avg_launch_ms": round(fam["pauli_coo"]["avg_ms"], 4)}
    paper_ms = {22: 19.0, 24: 59.0}.get(n)
    out = {
        "metric": "coo-entries/s", "value": nnz / dt, "unit": "coo-entries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": max(args.warmup, 1), "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c128 values, int64 indices", "data": "synthetic",
        "config": {"workload": f"tfim_coo_n{n}", "n_qubits": n, "terms": len(coeffs), "groups": G, "entries": nnz,
                   "parallelism": "single GPU"},
        "paper_reference": ({"ms_per_build": paper_ms, "hardware": "NVIDIA H200 (context, not the target)"}
                            if paper_ms else None),
        "roofline": roofline,
        "kernels": {k: {"launches_per_step": v["launches"] / args.steps, "avg_ms": round(v["avg_ms"], 4)}
                    for k, v in fam.items()},
    }
    if not args.no_cpu_baseline:
        import oracle
        cnt, t = 1 << 10, 0.0
        while True:
            t0 = time.perf_counter()
            oracle.pauli_coo(n, codes, coeffs, 0, cnt)
            t = time.perf_counter() - t0
            if t * 2 > 15.0 or cnt >= dim:
                break
            cnt = min(dim, max(cnt * 2, int(cnt * 15.0 / max(t, 1e-3) * 0.5)))
        out["cpu_baseline"] = {"value": G * cnt / t, "unit": "coo-entries/s", "cores": 1, "kind": "oracle", **host_info(),
                               "sample": f"rows [0, {cnt}) of the n={n} TFIM matrix ({G} groups, single thread), "
                                         f"{t:.1f} s"}
    return out


def run_shadow(args, P, torch):
    """Classical-shadow snapshots (n = 20, 256 snapshots, complex64): one step
    = copy, rotate and sample every snapshot of one state."""
    import workloads as W
    n, S = 20, 256
    w = W.shadow_workload(n, S, seed=20)
    layer = P.shadow_layer(n)
    psi = torch.as_tensor(np.asarray(w["psi"], np.complex64)).cuda()
    bases = torch.as_tensor(w["bases"]).cuda()
    u = torch.as_tensor(w["u"]).cuda()
    work = torch.empty((S, 2 ** n), dtype=torch.complex64, device="cuda")
    need = ctypes.c_size_t()
    P.check(P.lib().tcng_shadow_workspace_size(layer.handle, S, ctypes.byref(need)))
    ws = torch.empty(int(need.value), dtype=torch.uint8, device="cuda")

    def one():
        return P.shadow_snapshots(layer, psi, bases, u, work=work, ws=ws)

    for _ in range(max(args.warmup, 1)):
        one()
    torch.cuda.synchronize()
    prof = not args.no_profile
    if prof:
        P.check(P.lib().tcng_profile_begin(16 * (args.steps + 1)))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = one()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    fam = {}
    if prof:
        for i, name in enumerate(FAMILIES):
            cnt, tot = ctypes.c_int32(), ctypes.c_double()
            P.check(P.lib().tcng_profile_query(i, ctypes.byref(cnt), ctypes.byref(tot)))
            if cnt.value:
                fam[name] = dict(launches=cnt.value, total_ms=tot.value, avg_ms=tot.value / cnt.value)
        P.check(P.lib().tcng_profile_end())
    amp = 2 ** n * 8 * S
    passes = P.fused_plan_inspect(n, layer.gates, 0)[3]
    # per launch: every pass writes the S rotated states; the first reads the one input state,
    # the later ones the S states
    alg = {"fused_fwd": (amp * (2 * passes - 1) + 2 ** n * 8) / passes, "shadow_sum": float(amp)}
    roofline = None
    if fam:
        dom = max((k for k in alg if k in fam), key=lambda k: fam[k]["total_ms"])
        t = fam[dom]["avg_ms"] * 1e-3
        gbs = alg[dom] / t / 1e9
        roofline = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
                    "bytes_per_launch": alg[dom], "avg_launch_ms": round(fam[dom]["avg_ms"], 4)}
    res = {
        "metric": "snapshots/s", "value": S / dt, "unit": "snapshots/s", "n_gpus": 1, "steps": args.steps,
        "warmup": max(args.warmup, 1), "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64 (f32 state, f64 probabilities)", "data": "synthetic",
        "config": {"workload": "shadow_n20_s256", "n_qubits": n, "snapshots": S, "rotation_passes": passes,
                   "parallelism": "single GPU"},
        "paper_reference": {"ms_per_256_snapshots": 290.0, "hardware": "NVIDIA RTX 5090 (context, not the target)"},
        "roofline": roofline,
        "kernels": {k: {"launches_per_step": v["launches"] / args.steps, "avg_ms": round(v["avg_ms"], 4)}
                    for k, v in fam.items()},
    }
    if not args.no_cpu_baseline:
        import oracle
        k, t = 1, 0.0
        while True:
            t0 = time.perf_counter()
            oracle.shadow(n, w["psi"], w["bases"][:k], w["u"][:k])
            t = time.perf_counter() - t0
            if t * 2 > 15.0 or k >= S:
                break
            k = min(S, max(k + 1, int(k * 15.0 / max(t, 1e-3) * 0.5)))
        res["cpu_baseline"] = {"value": k / t, "unit": "snapshots/s", "cores": 1, "kind": "oracle", **host_info(),
                               "sample": f"{k} of {S} snapshots at n={n} (complex128, single thread), {t:.1f} s"}
    return res


def run_qml(args, P, torch, task):
    """SU(4) brick-wall QML training (MNIST: n = 10, 40 layers, batch 15000;
    CIFAR-100: n = 12, 30 layers, batch 5000; synthetic amplitude-encoded
    inputs): one step = loss and gradient of one batch plus a plain gradient
    step on the angles; an epoch is samples / batch steps."""
    import workloads as W
    w = W.qml_workload(task, seed=1)
    n, B, k, C, samples = w["n"], w["batch"], w["k"], w["C"], w["samples"]
    G = w["gates"].shape[0]
    circ = P.Circuit(n, w["gates"], 0, np.tile(np.eye(4, dtype=np.complex128), (G, 1, 1)))
    theta = torch.as_tensor(w["theta"]).cuda()
    x = torch.as_tensor(np.asarray(w["inputs"], np.complex64)).cuda()
    y = torch.as_tensor(w["labels"]).cuda()
    psi, lam = torch.empty_like(x), torch.empty_like(x)
    need = ctypes.c_size_t()
    P.check(P.lib().tcng_qml_workspace_size(circ.handle, B, ctypes.byref(need)))
    ws = torch.empty(int(need.value), dtype=torch.uint8, device="cuda")
    lr = 1e-3

    def one():
        loss, grad = P.qml_step(circ, theta, x, y, k, C, psi=psi, lam=lam, ws=ws)
        theta.add_(grad, alpha=-lr)
        return loss

    for _ in range(max(args.warmup, 1)):
        one()
    torch.cuda.synchronize()
    prof = not args.no_profile
    if prof:
        P.check(P.lib().tcng_profile_begin(512 * (args.steps + 1)))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        loss = one()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    fam = {}
    if prof:
        for i, name in enumerate(FAMILIES):
            cnt, tot = ctypes.c_int32(), ctypes.c_double()
            P.check(P.lib().tcng_profile_query(i, ctypes.byref(cnt), ctypes.byref(tot)))
            if cnt.value:
                fam[name] = dict(launches=cnt.value, total_ms=tot.value, avg_ms=tot.value / cnt.value)
        P.check(P.lib().tcng_profile_end())
    # below 12 qubits, 2^(12 - n) samples share a 12-bit tile when the batch divides evenly
    wide = n < 12 and B % (1 << (12 - n)) == 0
    _, _, _, passes, nblk, _ = P.fused_plan_inspect(12 if wide else n, w["gates"], 0)
    roofline = None
    if "fused_rev" in fam:
        # matrix-core work of the block formulation: 8 * 16 flops per amplitude and block,
        # three products per block in reverse (psi, lambda, outer product)
        blk_flops = 8.0 * 16 * (2 ** n) * B * nblk
        dom = max(("fused_fwd", "fused_rev"), key=lambda f: fam.get(f, {"total_ms": 0})["total_ms"])
        L = fam[dom]["launches"] / args.steps
        flops = (3 * blk_flops if dom == "fused_rev" else blk_flops) / L
        fwd_g, rev_g = sweep_flops(w["gates"], n, B, with_u2_grad=True)
        roofline = fused_roofline(dom, (rev_g if dom == "fused_rev" else fwd_g) / L,
                                  algorithmic_bytes(dom, n, 8, B, 0), flops, fam[dom]["avg_ms"])
        roofline["traffic"] = measured_traffic(f"qml_{task}_n{n}_l{w['layers']}_b{B}", dom)
    epoch_steps = samples / B
    paper = {"mnist": 1.88, "cifar100": 4.60}[task]
    res = {
        "metric": "QML training samples/s", "value": B / dt, "unit": "samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": max(args.warmup, 1), "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64 (f32 state and MFMA, f64 gates and reductions)",
        "data": "synthetic (uniform features, amplitude-encoded; random labels)",
        "config": {"workload": f"qml_{task}_n{n}_l{w['layers']}_b{B}", "n_qubits": n, "layers": w["layers"],
                   "gates": G, "params": 15 * G, "batch": B, "readout_qubits": k, "classes": C,
                   "epoch_samples": samples, "fused_passes": passes, "fused_blocks": nblk,
                   "samples_per_tile": (1 << (12 - n)) if wide else 1,
                   "update": "theta -= 1e-3 grad (one torch axpy over the angles)", "parallelism": "single GPU"},
        "epoch_s": dt * epoch_steps,
        "paper_reference": {"epoch_s": paper, "hardware": "NVIDIA RTX 5090 (context, not the target)"},
        "roofline": roofline,
        "kernels": {f: {"launches_per_step": v["launches"] / args.steps, "avg_ms": round(v["avg_ms"], 4)}
                    for f, v in fam.items()},
    }
    if not args.no_cpu_baseline:
        import oracle
        m, t = 1, 0.0
        while True:
            t0 = time.perf_counter()
            oracle.qml(n, w["gates"], w["theta"], w["inputs"][:m], w["labels"][:m], k, C)
            t = time.perf_counter() - t0
            if t * 2 > 15.0 or m >= B:
                break
            m = min(B, max(m + 1, int(m * 15.0 / max(t, 1e-3) * 0.5)))
        res["cpu_baseline"] = {"value": m / t, "unit": "samples/s", "cores": 1, "kind": "oracle", **host_info(),
                               "sample": f"loss and gradient of {m} of {B} samples (complex128, single thread), "
                                         f"{t:.1f} s"}
    return res


def host_info():
    """CPU model and core counts of the host the oracle runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"host_cpu": model, "host_cores": os.cpu_count(), "host_cores_usable": usable}


def _oracle_eval(w, budget_s, max_evals=1000):
    """Oracle value and gradient of the batch members of w in turn (whole
    circuit, full H) until `budget_s` is spent; (evals, seconds)."""
    import oracle
    prm = np.asarray(w["params"])
    prm = prm.reshape(-1, prm.shape[-1]) if prm.size else np.zeros((1, 0))
    done, t = 0, 0.0
    while done < max_evals and (done == 0 or t < budget_s):
        t0 = time.perf_counter()
        oracle.expect_grad(w["n"], w["gates"], prm[done % prm.shape[0]], w["codes"], w["coeffs"], w.get("mats"))
        t += time.perf_counter() - t0
        done += 1
    return done, t


def cpu_baseline(w, name, budget_s=15.0):
    """The oracle (single-threaded, complex128) on a bounded sample of the
    workload.  Primary figure: whole value-and-gradient evaluations (forward
    sweep, H psi and <H>, adjoint sweep) counted like the GPU's
    3 * G * 2^n amplitude-updates.  When one evaluation at the workload's own
    size would exceed the budget (the 28- and 32-qubit workloads), the same
    generator runs at the largest smaller size whose evaluation fits, found
    from a timed 14-qubit evaluation; beside it, the forward sweep of the
    first K gates at the workload's own n."""
    import oracle
    import workloads as W
    n, G = w["n"], len(w["gates"])
    out = {"unit": "amplitude-updates/s", "cores": 1, "kind": "oracle", **host_info()}
    ew = w
    if n >= 24:
        def small(k):
            v = W.cfg2(n=k) if name.startswith("hea") else W.cfg5(rows=4, cols=k // 4)
            v["params"] = np.asarray(v["params"])[None, :]
            return v
        sizes = list(range(14, 23)) if name.startswith("hea") else [16, 20]
        _, t0 = _oracle_eval(small(sizes[0]), 0.0, 1)
        g0 = len(small(sizes[0])["gates"])
        pick = sizes[0]
        for k in sizes:
            gk = len(small(k)["gates"])
            if t0 * 2 ** (k - sizes[0]) * gk / g0 <= budget_s:
                pick = k
        ew = small(pick)
    done, t = _oracle_eval(ew, min(budget_s, 2.0) if ew is w else 0.0)
    ne, Ge = ew["n"], len(ew["gates"])
    out["value"] = 3.0 * Ge * 2 ** ne * done / t
    out["evals_per_s"] = done / t
    out["sample"] = (f"{done} whole value-and-gradient evaluation(s) of "
                     f"{'the workload' if ew is w else 'the same generator'} at n={ne} ({Ge} gates, "
                     f"{len(ew['coeffs'])} terms; complex128, single thread), {t:.1f} s, each counted as "
                     f"3*G*2^n amplitude-updates")
    if ew is not w:
        params = w["params"][0] if np.asarray(w["params"]).ndim == 2 else w["params"]
        kf, tf = 1, 0.0
        while True:
            t0 = time.perf_counter()
            oracle.run(n, w["gates"][:kf], params, w.get("mats"))
            tf = time.perf_counter() - t0
            if tf * 2 > budget_s or kf >= G:
                break
            kf = min(G, max(kf + 1, int(kf * budget_s / max(tf, 1e-3) * 0.5)))
        out["forward_at_n"] = {"value": kf * (2 ** n) / tf, "unit": "amplitude-updates/s",
                               "sample": f"forward sweep of the first {kf} gates at n={n}, {tf:.1f} s"}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="hea28")
    ap.add_argument("--dtype", default="c64", choices=["c64", "c128"])
    ap.add_argument("--mode", default="auto", choices=["tiled", "plain", "fused", "fused5", "auto"],
                    help="auto: the autotuner's choice among the tiled tilings and the 4- / 5-qubit matrix-core plans")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--autotune", action="store_true", help="tiled mode: pick the tiling by timed search first")
    ap.add_argument("--tiling", default=None, help="m,rb,rb_rev (skips the autotuner)")
    ap.add_argument("--graph", action="store_true", help="replay a captured graph per evaluation")
    ap.add_argument("--sets", type=int, default=32, help="parameter sets of the per-circuit workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU sharding is not built",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2602_14167_amd as P
    assert torch.cuda.is_available(), "no HIP device"
    torch.cuda.set_device(0)
    w = workload(args.workload)
    if args.workload in ("gates28", "gates30"):
        out = run_gate_sweep(args, P, torch, int(args.workload[-2:]))
        print(json.dumps(out), flush=True)
        return
    if args.workload == "haar_uneven":
        out = run_uneven(args, w, P, torch)
        print(json.dumps(out), flush=True)
        return
    if args.workload == "xxz16_per_circuit":
        out = run_per_circuit(args, w, P, torch)
        print(json.dumps(out), flush=True)
        return
    if args.workload == "mipt20":
        out = run_mipt(args, P, torch)
        print(json.dumps(out), flush=True)
        return
    if args.workload == "shadow20":
        out = run_shadow(args, P, torch)
        print(json.dumps(out), flush=True)
        return
    if args.workload in ("qml_mnist", "qml_cifar100"):
        out = run_qml(args, P, torch, args.workload[4:])
        print(json.dumps(out), flush=True)
        return
    if args.workload in ("coo22", "coo24"):
        out = run_coo(args, P, torch, int(args.workload[-2:]))
        print(json.dumps(out), flush=True)
        return
    n, G, B = w["n"], len(w["gates"]), int(w.get("batch", 1))
    s = 8 if args.dtype == "c64" else 16
    copy = copy_ceiling(torch, (2 ** n) * s * B)
    cdt = torch.complex64 if args.dtype == "c64" else torch.complex128
    rdt = torch.float32 if args.dtype == "c64" else torch.float64
    circ = P.Circuit(n, w["gates"], w["n_params"], w.get("mats"))
    H = P.PauliSum(n, w["codes"], w["coeffs"])
    params = torch.tensor(np.asarray(w["params"]).reshape(B, -1), dtype=rdt, device="cuda")
    psi = torch.empty((B, 2 ** n), dtype=cdt, device="cuda")
    lam = torch.empty_like(psi)
    tuned = None
    if args.mode == "tiled" and args.tiling:
        circ.configure(cdt, *[int(v) for v in args.tiling.split(",")])
    elif args.mode == "auto" or (args.mode == "tiled" and args.autotune):
        # timed search (untimed here): tilings of the tiled passes and, in
        # complex64, the 4- and 5-qubit matrix-core plans; cached per shape
        t0 = time.perf_counter()
        P.state_init(psi)
        cfg, tms = P.autotune(circ, params, H, psi, lam, repeats=3,
                              cache_path=os.path.join(os.environ.get("TMPDIR", "/tmp"), "tcng_autotune.txt"))
        tuned = {"mode": circ.mode(cdt), "tiling": list(cfg), "median_ms": round(tms, 3),
                 "search_s": round(time.perf_counter() - t0, 1)}
    run_mode = circ.mode(cdt) if args.mode == "auto" else args.mode
    if args.mode == "tiled" and args.autotune:
        run_mode = "tiled"
    mode = P.MODES[run_mode]
    # workspace for the chosen tiling
    nbytes = ctypes.c_size_t()
    P.check(P.lib().tcng_workspace_size(circ.handle, H.handle, 0 if args.dtype == "c64" else 1, B, mode,
                                        ctypes.byref(nbytes)))
    ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device="cuda")

    graph = None
    if args.graph:
        energy_g = torch.empty(B, dtype=torch.float64, device="cuda")
        grad_g = torch.empty((B, max(w["n_params"], 1)), dtype=torch.float64, device="cuda")
        graph = P.Graph(circ, params, H, psi, lam, energy_g, grad_g, mode=run_mode)

    def step():
        if graph is not None:
            graph.launch()
            return energy_g, grad_g
        P.state_init(psi)
        return P.expect_grad(circ, params, H, psi=psi, lam=lam, mode=run_mode, ws=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    prof = not args.no_profile and graph is None   # replays record no per-launch events
    if prof:
        P.check(P.lib().tcng_profile_begin(64 * (G + 64) * (args.steps + 1)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        E, g = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps

    fam_stats = {}
    if prof:
        for i, name in enumerate(FAMILIES):
            cnt, tot = ctypes.c_int32(), ctypes.c_double()
            P.check(P.lib().tcng_profile_query(i, ctypes.byref(cnt), ctypes.byref(tot)))
            if cnt.value:
                fam_stats[name] = dict(launches=cnt.value, total_ms=tot.value, avg_ms=tot.value / cnt.value)
        P.check(P.lib().tcng_profile_end())

    amp_updates = 3.0 * G * (2 ** n) * B
    value = amp_updates / dt
    fwd_flops, rev_flops = sweep_flops(w["gates"], n, B)
    roofline = None
    if run_mode in ("fused", "fused5") and "fused_rev" in fam_stats:
        # matrix-core work of the block formulation: 8 * 2^k flops per amplitude
        # and block (2^k x 2^k complex product), three products per block in reverse
        kb = 5 if run_mode == "fused5" else 4
        nblk = P.fused_plan_inspect(n, w["gates"], w["n_params"], kb)[4]
        blk_flops = 8.0 * 2 ** kb * (2 ** n) * B * nblk
        dom = max(("fused_fwd", "fused_rev"), key=lambda k: fam_stats.get(k, {"total_ms": 0})["total_ms"])
        L = fam_stats[dom]["launches"] / args.steps
        flops = (3 * blk_flops if dom == "fused_rev" else blk_flops) / L
        roofline = fused_roofline(dom, (rev_flops if dom == "fused_rev" else fwd_flops) / L,
                                  algorithmic_bytes(dom, n, s, B, 0), flops, fam_stats[dom]["avg_ms"])
        roofline["traffic"] = measured_traffic(w["name"], dom) if run_mode == "fused" else None
    elif run_mode == "tiled" and "rev_tile" in fam_stats:
        dom = max(("fwd_tile", "rev_tile"), key=lambda k: fam_stats.get(k, {"total_ms": 0})["total_ms"])
        L = fam_stats[dom]["launches"] / args.steps
        flops = (rev_flops if dom == "rev_tile" else fwd_flops) / L
        nbytes = algorithmic_bytes(dom, n, s, B, 0)
        roofline = roofline_entry(dom, flops, nbytes, fam_stats[dom]["avg_ms"])
        roofline["traffic"] = measured_traffic(w["name"], dom) if args.dtype == "c64" else None
    elif fam_stats:
        dom = max(fam_stats, key=lambda k: fam_stats[k]["total_ms"])
        roofline = {"bound": "hbm", "kernel": dom, "note": "plain per-gate path"}

    out = {
        "metric": "amplitude-updates/s",
        "value": value,
        "unit": "amplitude-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (f32 state, f64 reductions)" if args.dtype == "c64" else "c128",
        "data": "synthetic",
        "config": {"workload": w["name"], "n_qubits": n, "gates": G, "params": w["n_params"], "batch": B,
                   "pauli_terms": len(w["coeffs"]), "mode": run_mode, "graph": bool(args.graph),
                   "parallelism": "single GPU"},
        "evals_per_s": B / dt,
        "us_per_eval": dt / B * 1e6,
        "tiling": list(circ.config(cdt)) if run_mode == "tiled" else None,
        "autotune": tuned,
        "energy0": float(E[0].item()),
        "roofline": roofline,
        "copy_ceiling": copy,
        "kernels": {k: {"launches_per_step": v["launches"] / args.steps, "avg_ms": round(v["avg_ms"], 4)}
                    for k, v in fam_stats.items()},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
