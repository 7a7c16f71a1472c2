"""Seeded synthetic inputs for the statevector hot path.

This module only draws inputs: gate lists, angles, constant gate matrices and
Pauli-sum Hamiltonians.  It contains none of the simulation arithmetic, so the
CPU oracle and the HIP library can both be fed from it without sharing code.

Conventions of the arrays produced here (the data format of both sides):

* Gate record: int32[6] = (kind, q0, q1, p0, p1, mat).  q1 = -1 for one-qubit
  gates, p0/p1 = parameter index or -1, mat = constant-matrix index or -1.
  For two-qubit gates q0 is the most significant bit of the 4x4 matrix index;
  for CNOT q0 is the control.
* Angles: float64 vector; for complex64 runs they are rounded to float32 once
  (``round_params``) and the oracle is given the rounded values widened.
* Constant matrices: complex128 [n_mats][4][4]; a one-qubit constant gate uses
  the top-left 2x2 block.
* Pauli sum: codes uint8 [T][n] with 0=I, 1=X, 2=Y, 3=Z (the paper's shadow
  encoding, Sec. "Efficient ML Pipeline via Classical Shadows") and float64
  coefficients [T].
"""
from .gen import *  # noqa: F401,F403
