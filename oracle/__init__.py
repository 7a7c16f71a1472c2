"""TEST INFRASTRUCTURE — the CPU oracle (complex128, single-threaded).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It is an independent statevector
simulator written from the definitions in the paper (Sec. "Foundations
Recap": gates as local contractions, E = <psi|H|psi> with H a Pauli sum,
reverse-mode gradient / parameter-shift rule); it shares no code with the HIP
library.  Pins that tie it to the mathematics live in tests/test_oracle_pins.py.

It also builds the sparse (COO) matrix of a Pauli sum (Sec. "Lattice and
Hamiltonian"), draws classical-shadow snapshots (Sec. "Efficient ML Pipeline
via Classical Shadows"), takes the loss and gradient of the SU(4) QML circuit
(Sec. "End-to-End Pure QML for Computer Vision"), and runs monitored Haar
brick-wall trajectories (Sec. "Universal Quantum
Dynamics of Haar-Random MIPT"): unitary steps, random Z measurements drawn
from passed-in uniforms, Born log-probability of the record.

Parity status: every function here is pinned (closed forms, brute-force
Kronecker products for n <= 6, exact diagonalisation against the free-fermion
closed form, parameter shift vs adjoint, finite differences; for the
trajectories, tensor-contraction evolution, dense joint Born probabilities,
p = 0 / p = 1 closed forms and Born-rule sampling statistics in
tests/test_oracle_mipt.py; for the COO entries, dense Kronecker-product
Hamiltonians, Hermiticity and H psi in tests/test_oracle_coo.py; for the
shadows, eigenstates, GHZ parities, Born frequencies, the unbiased shadow
estimator and Kronecker-product rotations in tests/test_oracle_shadow.py; for
the QML step, scipy's matrix exponential, finite differences and the
identity-gate closed form in tests/test_oracle_qml.py).
"""
from .api import *  # noqa: F401,F403
