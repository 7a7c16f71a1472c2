"""Seeded generators for circuits, angles and Hamiltonians.

Every workload follows the paper's problem statement: a parameterised circuit
built from rotation / entangling gates (Sec. "Foundations Recap", the batched
TFIM VQE example), expectation of a Pauli-string Hamiltonian H = sum_k c_k P_k
(Sec. "Data Parallelism", measurement parallelism), batched over parameter
sets (the VMAP paradigm), and Haar-random brick-wall circuits (Sec. "Universal
Quantum Dynamics of Haar-Random MIPT").  The draw order of every random number
is fixed and documented per function so that a workload is reproducible from
its seed alone.
"""
from __future__ import annotations

import numpy as np

# gate kinds (shared data format; both sides define their own enum with these values)
RX, RY, RZ, H, X, Y, Z, S, CNOT, CZ, RZZ, FSIM, U1, U2 = range(14)
KIND_NAMES = ["RX", "RY", "RZ", "H", "X", "Y", "Z", "S", "CNOT", "CZ", "RZZ", "FSIM", "U1", "U2"]
TWO_QUBIT = {CNOT, CZ, RZZ, FSIM, U2}
PARAM_COUNT = {RX: 1, RY: 1, RZ: 1, RZZ: 1, FSIM: 2}

PI2 = 2.0 * np.pi


def gate(kind, q0, q1=-1, p0=-1, p1=-1, mat=-1):
    return (int(kind), int(q0), int(q1), int(p0), int(p1), int(mat))


def as_gate_array(gates):
    arr = np.asarray(gates, dtype=np.int32).reshape(-1, 6)
    return np.ascontiguousarray(arr)


# ----------------------------------------------------------------------------
# circuits
# ----------------------------------------------------------------------------

def hea_gates(n: int, layers: int, cnot: bool = True):
    """Hardware-efficient ansatz: per layer RY on every qubit, then RZ on every
    qubit, then a CNOT ladder (i -> i+1) in increasing i.

    Parameter index of RY(q) in layer l is l*2n + q, of RZ(q) is l*2n + n + q,
    i.e. the flat parameter vector is theta[L][2][n].
    """
    g = []
    for l in range(layers):
        for q in range(n):
            g.append(gate(RY, q, p0=l * 2 * n + q))
        for q in range(n):
            g.append(gate(RZ, q, p0=l * 2 * n + n + q))
        if cnot:
            for q in range(n - 1):
                g.append(gate(CNOT, q, q + 1))
    return as_gate_array(g), layers * 2 * n


def brickwork_bonds(n: int, depth: int):
    """1D brick-wall: layer t uses bonds (i, i+1) with i = t mod 2, t mod 2 + 2, ...
    (even bonds first), bonds in ascending order inside a layer."""
    out = []
    for t in range(depth):
        for i in range(t % 2, n - 1, 2):
            out.append((i, i + 1))
    return out


def haar_u4(rng: np.random.Generator) -> np.ndarray:
    """Haar-random 4x4 unitary: QR of a complex Ginibre matrix with the phases
    of R's diagonal moved into Q (Mezzadri's construction).  Draw order: the
    16 real parts, then the 16 imaginary parts, row-major."""
    a = rng.standard_normal((4, 4))
    b = rng.standard_normal((4, 4))
    z = (a + 1j * b) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))[None, :]


def brickwork_haar(n: int, depth: int, rng: np.random.Generator):
    bonds = brickwork_bonds(n, depth)
    mats = np.zeros((len(bonds), 4, 4), dtype=np.complex128)
    g = []
    for idx, (i, j) in enumerate(bonds):
        mats[idx] = haar_u4(rng)
        g.append(gate(U2, i, j, mat=idx))
    return as_gate_array(g), mats


def haar_u4_many(rng: np.random.Generator, count: int) -> np.ndarray:
    """`count` Haar 4x4 unitaries with the same draws, in the same order, as
    `count` calls of haar_u4 (16 real parts then 16 imaginary parts each)."""
    z = rng.standard_normal((count, 2, 4, 4))
    z = (z[:, 0] + 1j * z[:, 1]) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    return q * (d / np.abs(d))[:, None, :]


def mipt_step_gates(n: int):
    """One time step of the monitored brick-wall circuit: two-qubit gates on the
    even bonds (0,1), (2,3), ..., then on the odd bonds (1,2), (3,4), ...;
    gate g takes step matrix g."""
    g = [gate(U2, i, j, mat=k) for k, (i, j) in enumerate(brickwork_bonds(n, 2))]
    return as_gate_array(g)


def mipt_workload(n: int, steps: int, batch: int, p: float, seed: int):
    """Haar-random monitored trajectories (Sec. "Universal Quantum Dynamics of
    Haar-Random MIPT"): per trajectory and step, independent Haar gates on the
    step's bonds, then one uniform per qubit for the measurement layer.
    Draw order: all gate matrices (trajectory-major, then step, then gate),
    then the uniforms u[batch][steps][n]."""
    rng = np.random.default_rng(seed)
    gates = mipt_step_gates(n)
    G = gates.shape[0]
    mats = haar_u4_many(rng, batch * steps * G).reshape(batch, steps, G, 4, 4)
    u = rng.uniform(0.0, 1.0, size=(batch, steps, n))
    return dict(n=n, steps=steps, batch=batch, p=float(p), gates=gates, mats=mats, u=u)


def shadow_workload(n: int, snapshots: int, seed: int):
    """Classical-shadow snapshots of one n-qubit state (Sec. "Efficient ML
    Pipeline via Classical Shadows"): a seeded random state (standing in for
    the paper's ground state), Pauli bases drawn uniformly from {1=X, 2=Y, 3=Z}
    per snapshot and qubit, and one uniform per snapshot for the outcome draw.
    Draw order: state, bases [snapshots][n], uniforms [snapshots]."""
    rng = np.random.default_rng(seed)
    psi = random_state(n, rng)
    bases = rng.integers(1, 4, size=(snapshots, n)).astype(np.uint8)
    u = rng.uniform(0.0, 1.0, size=snapshots)
    return dict(n=n, snapshots=snapshots, psi=psi, bases=bases, u=u)


def qml_gates(n: int, layers: int):
    """SU(4) brick-wall QML ansatz (Sec. "End-to-End Pure QML for Computer
    Vision"): per layer one gate on each even bond (0,1), (2,3), ..., then on
    each odd bond (1,2), (3,4), ...; gate g has its own 15 angles theta[g]."""
    g = []
    for _ in range(layers):
        for i in list(range(0, n - 1, 2)) + list(range(1, n - 1, 2)):
            g.append(gate(U2, i, i + 1, mat=len(g)))
    return as_gate_array(g)


QML_TASKS = {   # qubits, layers, samples, batch, input features, readout qubits, classes
    "mnist": (10, 40, 60000, 15000, 784, 4, 10),
    "cifar100": (12, 30, 50000, 5000, 3072, 7, 100),
}


def qml_workload(task: str, seed: int, batch=None, layers=None):
    """Synthetic stand-in for the paper's MNIST / CIFAR-100 QML runs (the
    datasets are not used): angles theta[G][15] ~ U[0, 2 pi), then per sample
    `features` values ~ U[0, 1) zero-padded to 2^n and normalised (amplitude
    encoding), then labels ~ U{0..C-1}; in that order."""
    n, L, samples, B, feat, k, C = QML_TASKS[task]
    B = B if batch is None else batch
    L = L if layers is None else layers
    rng = np.random.default_rng(seed)
    gates = qml_gates(n, L)
    theta = rng.uniform(0.0, PI2, size=(gates.shape[0], 15))
    x = np.zeros((B, 2 ** n))
    x[:, :feat] = rng.uniform(0.0, 1.0, size=(B, feat))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    labels = rng.integers(0, C, size=B).astype(np.int32)
    return dict(task=task, n=n, layers=L, samples=samples, batch=B, k=k, C=C, gates=gates, theta=theta,
                inputs=x, labels=labels)


def brickwork_fsim(n: int, depth: int, rng: np.random.Generator):
    """fSim brick-wall; per gate theta then phi drawn U[0, 2pi) in gate order."""
    bonds = brickwork_bonds(n, depth)
    g = []
    params = np.empty(2 * len(bonds))
    for idx, (i, j) in enumerate(bonds):
        params[2 * idx] = rng.uniform(0.0, PI2)
        params[2 * idx + 1] = rng.uniform(0.0, PI2)
        g.append(gate(FSIM, i, j, p0=2 * idx, p1=2 * idx + 1))
    return as_gate_array(g), params


def random_circuit(n: int, n_gates: int, rng: np.random.Generator, kinds=None):
    """Random mixture of every gate kind on random (ordered) qubits, for the
    brute-force and parity tests.  Returns (gates, params, mats)."""
    if kinds is None:
        kinds = list(range(14)) if n >= 2 else [k for k in range(14) if k not in TWO_QUBIT]
    g, params, mats = [], [], []
    for _ in range(n_gates):
        k = int(rng.choice(kinds))
        if k in TWO_QUBIT:
            q0, q1 = (int(v) for v in rng.choice(n, size=2, replace=False))
        else:
            q0, q1 = int(rng.integers(n)), -1
        p0 = p1 = m = -1
        if k in PARAM_COUNT:
            p0 = len(params)
            params.append(rng.uniform(0.0, PI2))
            if PARAM_COUNT[k] == 2:
                p1 = len(params)
                params.append(rng.uniform(0.0, PI2))
        if k == U2:
            m = len(mats)
            mats.append(haar_u4(rng))
        elif k == U1:
            m = len(mats)
            u = np.zeros((4, 4), dtype=np.complex128)
            u[:2, :2] = haar_u4(rng)[:2, :2]
            # make the 2x2 block unitary (polar factor) -- any 2x2 works for
            # the simulator, a unitary keeps norms at 1
            w, _, vh = np.linalg.svd(u[:2, :2])
            u[:2, :2] = w @ vh
            mats.append(u)
        g.append(gate(k, q0, q1, p0, p1, m))
    mats_arr = np.array(mats, dtype=np.complex128).reshape(-1, 4, 4)
    return as_gate_array(g), np.asarray(params, dtype=np.float64), mats_arr


# ----------------------------------------------------------------------------
# Hamiltonians (Pauli sums)
# ----------------------------------------------------------------------------

def _term(n, ops):
    c = np.zeros(n, dtype=np.uint8)
    for q, p in ops:
        c[q] = p
    return c


def tfim_1d(n: int, J: float, h: float):
    """H = J sum_i Z_i Z_{i+1} + h sum_i X_i on an open chain (coefficients
    are data: the paper's form has J, h negative).  ZZ terms first, then X."""
    codes, coeffs = [], []
    for i in range(n - 1):
        codes.append(_term(n, [(i, 3), (i + 1, 3)]))
        coeffs.append(J)
    for i in range(n):
        codes.append(_term(n, [(i, 1)]))
        coeffs.append(h)
    return np.array(codes, dtype=np.uint8), np.array(coeffs, dtype=np.float64)


def xxz_1d(n: int, delta: float):
    """H = sum_i (X_i X_{i+1} + Y_i Y_{i+1} + delta Z_i Z_{i+1}), open chain;
    per bond the order is XX, YY, ZZ."""
    codes, coeffs = [], []
    for i in range(n - 1):
        for p, c in ((1, 1.0), (2, 1.0), (3, delta)):
            codes.append(_term(n, [(i, p), (i + 1, p)]))
            coeffs.append(c)
    return np.array(codes, dtype=np.uint8), np.array(coeffs, dtype=np.float64)


def square_lattice_edges(rows: int, cols: int):
    """Open rows x cols lattice, site (r, c) -> qubit cols*r + c.  Horizontal
    edges first (row-major), then vertical edges (row-major)."""
    e = []
    for r in range(rows):
        for c in range(cols - 1):
            e.append((cols * r + c, cols * r + c + 1))
    for r in range(rows - 1):
        for c in range(cols):
            e.append((cols * r + c, cols * (r + 1) + c))
    return e


def tfim_2d(rows: int, cols: int, J: float, h: float):
    n = rows * cols
    codes, coeffs = [], []
    for (a, b) in square_lattice_edges(rows, cols):
        codes.append(_term(n, [(a, 3), (b, 3)]))
        coeffs.append(J)
    for q in range(n):
        codes.append(_term(n, [(q, 1)]))
        coeffs.append(h)
    return np.array(codes, dtype=np.uint8), np.array(coeffs, dtype=np.float64)


def random_2local(n: int, n_terms: int, rng: np.random.Generator):
    """n_terms weight-2 terms; per term, in order: a qubit pair uniform over all
    unordered pairs, two Pauli labels uniform in {X, Y, Z}, coefficient N(0,1).
    Duplicated terms are kept (they add up)."""
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    codes, coeffs = [], []
    for _ in range(n_terms):
        i, j = pairs[int(rng.integers(len(pairs)))]
        pa, pb = (int(v) for v in rng.integers(1, 4, size=2))
        codes.append(_term(n, [(i, pa), (j, pb)]))
        coeffs.append(float(rng.standard_normal()))
    return np.array(codes, dtype=np.uint8), np.array(coeffs, dtype=np.float64)


def random_pauli_sum(n: int, n_terms: int, rng: np.random.Generator, max_weight=None):
    """Arbitrary-weight random Pauli strings (tests only)."""
    codes = rng.integers(0, 4, size=(n_terms, n)).astype(np.uint8)
    if max_weight is not None:
        for t in range(n_terms):
            nz = np.flatnonzero(codes[t])
            if len(nz) > max_weight:
                codes[t, rng.choice(nz, size=len(nz) - max_weight, replace=False)] = 0
    coeffs = rng.standard_normal(n_terms)
    return codes, coeffs


# ----------------------------------------------------------------------------
# precision handling of inputs
# ----------------------------------------------------------------------------

def round_params(params, dtype: str):
    """Angles as the run sees them: float32 for complex64, float64 otherwise.
    Returns float64 values (widened exactly) for the oracle."""
    if dtype == "c64":
        return np.asarray(params, dtype=np.float32).astype(np.float64)
    return np.asarray(params, dtype=np.float64)


def round_mats(mats, dtype: str):
    if dtype == "c64":
        return np.asarray(mats, dtype=np.complex64).astype(np.complex128)
    return np.asarray(mats, dtype=np.complex128)


def random_state(n: int, rng: np.random.Generator, batch=None):
    shape = (2 ** n,) if batch is None else (batch, 2 ** n)
    v = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    v /= np.linalg.norm(v, axis=-1, keepdims=True)
    return v


# ----------------------------------------------------------------------------
# the five measured workloads
# ----------------------------------------------------------------------------

def hea_workload(n, layers, J, h, seed, batch=None):
    rng = np.random.default_rng(seed)
    gates, n_params = hea_gates(n, layers)
    shape = (n_params,) if batch is None else (batch, n_params)
    params = rng.uniform(0.0, PI2, size=shape)
    codes, coeffs = tfim_1d(n, J, h)
    return dict(n=n, gates=gates, n_params=n_params, params=params,
                mats=np.zeros((0, 4, 4), np.complex128), codes=codes, coeffs=coeffs)


def cfg1():
    """n=10 complex128, HEA L=4, H = +sum ZZ + sum X (J = h = 1), seed 1."""
    w = hea_workload(10, 4, 1.0, 1.0, seed=1)
    w.update(name="hea_n10_L4_tfim_c128", dtype="c128")
    return w


def cfg2(n=28, layers=12):
    """n=28 HEA L=12, TFIM -sum ZZ - 0.5 sum X, seed 2 (n and L overridable
    for reduced-size parity runs of the same generator)."""
    w = hea_workload(n, layers, -1.0, -0.5, seed=2)
    w.update(name=f"hea_n{n}_L{layers}_tfim", dtype="c64")
    return w


def cfg3(batch=2048, n=16, layers=8):
    """n=16, B=2048 parameter sets of HEA L=8 (256 angles each), XXZ with
    delta = 0.5, seed 3; angles drawn as one [B][L*2*n] array."""
    rng = np.random.default_rng(3)
    gates, n_params = hea_gates(n, layers)
    params = rng.uniform(0.0, PI2, size=(batch, n_params))
    codes, coeffs = xxz_1d(n, 0.5)
    return dict(name=f"hea_n{n}_L{layers}_xxz_B{batch}", dtype="c64", n=n, gates=gates,
                n_params=n_params, params=params, mats=np.zeros((0, 4, 4), np.complex128),
                codes=codes, coeffs=coeffs, batch=batch)


def cfg4(count=1024, n_lo=12, n_hi=22, d_lo=2, d_hi=16, seed=4):
    """Uneven batch of Haar brick-wall circuits.  Per circuit, in order: n ~
    U{n_lo..n_hi}, depth ~ U{d_lo..d_hi}, the Haar gates (layer-major, bonds
    ascending), then H = 3n random weight-2 terms."""
    rng = np.random.default_rng(seed)
    circuits = []
    for _ in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        d = int(rng.integers(d_lo, d_hi + 1))
        gates, mats = brickwork_haar(n, d, rng)
        codes, coeffs = random_2local(n, 3 * n, rng)
        circuits.append(dict(n=n, depth=d, gates=gates, mats=mats, n_params=0,
                             params=np.zeros(0), codes=codes, coeffs=coeffs))
    return dict(name=f"haar_brickwork_uneven_{count}", dtype="c64", circuits=circuits)


def cfg5(rows=4, cols=8, depth=20, seed=5):
    """n = rows*cols: a Hadamard on every qubit, then the fSim brick-wall
    (depth 20 -> 310 fSim gates at n=32, 620 angles), 2D open TFIM
    -sum ZZ - 3.04 sum X on the rows x cols lattice.  The Hadamard layer is
    part of the reading of this workload: an fSim gate keeps |00> as it is and
    only mixes |01> with |10>, so the brick wall alone would leave |0...0>
    unchanged (E = -sum ZZ for every angle, a zero gradient)."""
    rng = np.random.default_rng(seed)
    n = rows * cols
    gates, params = brickwork_fsim(n, depth, rng)
    gates = np.concatenate([as_gate_array([gate(H, q) for q in range(n)]), gates])
    codes, coeffs = tfim_2d(rows, cols, -1.0, -3.04)
    return dict(name=f"fsim_brickwork_n{n}_d{depth}_tfim2d", dtype="c64", n=n, gates=gates,
                n_params=len(params), params=params, mats=np.zeros((0, 4, 4), np.complex128),
                codes=codes, coeffs=coeffs)
