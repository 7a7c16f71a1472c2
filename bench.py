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
FAMILIES = ["fwd_tile", "rev_tile", "pauli_tile", "gate1", "gate2", "gatek", "rev1", "rev2", "pauli_group",
            "finish", "init"]


def workload(name):
    import workloads as W
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
    if family == "rev_tile":
        return 4 * amp                      # read + write psi and lambda
    if family == "pauli_tile":
        # first pass: read psi, write lambda; later passes also read lambda
        return None if n_pauli_passes == 0 else (2 * amp + 3 * amp * (n_pauli_passes - 1)) / n_pauli_passes
    return None


def cpu_baseline(w, budget_s=15.0):
    """The oracle (single-threaded, complex128) on a bounded sample of the
    workload: forward application of the first K gates at full n, K grown
    until about `budget_s` of CPU time."""
    import oracle
    n = w["n"]
    params = w["params"][0] if w["params"].ndim == 2 else w["params"]
    k, t = 1, 0.0
    while True:
        t0 = time.perf_counter()
        oracle.run(n, w["gates"][:k], params, w.get("mats"))
        t = time.perf_counter() - t0
        if t * 2 > budget_s or k >= len(w["gates"]):
            break
        k = min(len(w["gates"]), max(k + 1, int(k * budget_s / max(t, 1e-3) * 0.5)))
    rate = k * (2 ** n) / t
    return {"value": rate, "unit": "amplitude-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"forward sweep of the first {k} gates at n={n} (complex128, single thread), {t:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="hea28")
    ap.add_argument("--dtype", default="c64", choices=["c64", "c128"])
    ap.add_argument("--mode", default="tiled", choices=["tiled", "plain"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
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
    n, G, B = w["n"], len(w["gates"]), int(w.get("batch", 1))
    cdt = torch.complex64 if args.dtype == "c64" else torch.complex128
    rdt = torch.float32 if args.dtype == "c64" else torch.float64
    s = 8 if args.dtype == "c64" else 16
    circ = P.Circuit(n, w["gates"], w["n_params"], w.get("mats"))
    H = P.PauliSum(n, w["codes"], w["coeffs"])
    params = torch.tensor(np.asarray(w["params"]).reshape(B, -1), dtype=rdt, device="cuda")
    psi = torch.empty((B, 2 ** n), dtype=cdt, device="cuda")
    lam = torch.empty_like(psi)
    mode = P.MODES[args.mode]
    nbytes = ctypes.c_size_t()
    P.check(P.lib().tcng_workspace_size(circ.handle, H.handle, 0 if args.dtype == "c64" else 1, B, mode,
                                        ctypes.byref(nbytes)))
    ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device="cuda")

    def step():
        P.state_init(psi)
        return P.expect_grad(circ, params, H, psi=psi, lam=lam, mode=args.mode, ws=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    prof = not args.no_profile
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
    n_pauli = 0
    if "pauli_tile" in fam_stats:
        n_pauli = fam_stats["pauli_tile"]["launches"] // args.steps
    roofline = None
    if fam_stats:
        dom = max((k for k in fam_stats if algorithmic_bytes(k, n, s, B, n_pauli) is not None),
                  key=lambda k: fam_stats[k]["total_ms"], default=None)
        if dom is not None:
            ab = algorithmic_bytes(dom, n, s, B, n_pauli)
            achieved = ab / (fam_stats[dom]["avg_ms"] * 1e-3) / 1e9
            roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
                        "bytes_per_launch": ab, "avg_launch_ms": round(fam_stats[dom]["avg_ms"], 4)}

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
                   "pauli_terms": len(w["coeffs"]), "mode": args.mode, "parallelism": "single GPU"},
        "evals_per_s": B / dt,
        "energy0": float(E[0].item()),
        "roofline": roofline,
        "kernels": {k: {"launches_per_step": v["launches"] / args.steps, "avg_ms": round(v["avg_ms"], 4)}
                    for k, v in fam_stats.items()},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
