"""Writes the stored expected values under tests/golden/ from the CPU oracle.

Every value here comes from ``oracle.expect_grad`` (single-threaded
complex128 statevector, adjoint gradients; the value-and-gradient of the
paper's Sec. "Foundations Recap") applied to the seeded generators in
``workloads`` (which hold no simulation arithmetic).  Nothing is read from the
HIP library.

Inputs are rounded once to the complex64 path's precision (angles to float32,
matrices to complex64) and widened exactly before the oracle sees them, so the
same stored values serve the complex64 runs (which read those rounded values)
and the complex128 runs (which are given the widened values).

Files (numpy .npz, no pickles):
  hea_tfim_n20_L12.npz, hea_tfim_n22_L12.npz
      the n=28 HEA/TFIM generator (RY, RZ on every qubit, CNOT ladder; 12
      layers; -sum ZZ - 0.5 sum X) at n=20 and n=22: params, E, grad.
  fsim_tfim2d_4x5_d20.npz, fsim_tfim2d_4x6_d20.npz
      the n=32 fSim brick-wall generator (Hadamard layer, fSim depth 20, 2D
      open TFIM -sum ZZ - 3.04 sum X) on 4x5 and 4x6 lattices: params, E, grad.
  haar_uneven_n_le_18.npz
      every circuit of the 1024-circuit uneven Haar brick-wall batch with
      n <= 18 (661 circuits): index into the batch, E, and the 15 SU(4)
      Lie-algebra gradient components of every gate, concatenated in circuit
      order with offsets (matrices rounded to complex64, as above).
  haar_uneven_n_le_18_c128.npz
      the same circuits with their complex128 matrices.  The adjoint sweep
      un-computes with U^dagger, the inverse only of a unitary U: the
      complex64-rounded matrices are unitary to about 1e-8, which moves the
      Lie gradients by that much, far inside the complex64 bar but not the
      complex128 one.

Run:  python tests/golden/make_golden.py   (about 10 minutes on 8 cores)
"""
from __future__ import annotations

import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def _hea(n):
    w = W.cfg2(n=n, layers=12)
    p = W.round_params(w["params"], "c64")
    r = oracle.expect_grad(n, w["gates"], p, w["codes"], w["coeffs"])
    return f"hea_tfim_n{n}_L12.npz", dict(n=n, params=p, E=r["E"], E_imag=r["E_imag"], grad=r["grad"])


def _fsim(cols):
    w = W.cfg5(rows=4, cols=cols, depth=20)
    p = W.round_params(w["params"], "c64")
    r = oracle.expect_grad(w["n"], w["gates"], p, w["codes"], w["coeffs"])
    return f"fsim_tfim2d_4x{cols}_d20.npz", dict(n=w["n"], params=p, E=r["E"], E_imag=r["E_imag"], grad=r["grad"])


_CFG4 = None


def _haar(i, prec="c64"):
    global _CFG4
    if _CFG4 is None:
        _CFG4 = W.cfg4()["circuits"]
    c = _CFG4[i]
    m = W.round_mats(c["mats"], prec)
    r = oracle.expect_grad(c["n"], c["gates"], np.zeros(0), c["codes"], c["coeffs"], m, want_lie=True)
    return i, r["E"], r["lie"]


def main():
    t0 = time.time()
    oracle.build(force=False)
    circuits = W.cfg4()["circuits"]
    sel = [i for i, c in enumerate(circuits) if c["n"] <= 18]
    with mp.Pool(min(8, os.cpu_count() or 1)) as pool:
        big = [pool.apply_async(_hea, (22,)), pool.apply_async(_fsim, (6,)), pool.apply_async(_hea, (20,)),
               pool.apply_async(_fsim, (5,))]
        haar = {p: pool.starmap(_haar, [(i, p) for i in sel], chunksize=4) for p in ("c64", "c128")}
        for a in big:
            name, d = a.get()
            np.savez_compressed(os.path.join(HERE, name), **d)
            print("wrote", name, f"{time.time() - t0:.0f} s", flush=True)
    for prec, name in (("c64", "haar_uneven_n_le_18.npz"), ("c128", "haar_uneven_n_le_18_c128.npz")):
        h = haar[prec]
        idx = np.array([x[0] for x in h], np.int32)
        E = np.array([x[1] for x in h])
        lie = [x[2] for x in h]
        off = np.concatenate([[0], np.cumsum([x.shape[0] for x in lie])]).astype(np.int64)
        np.savez_compressed(os.path.join(HERE, name), index=idx, E=E, lie=np.concatenate(lie), offsets=off)
        print("wrote", name, len(sel), "circuits", f"{time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
