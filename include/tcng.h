/*
 * tcng.h — C ABI of the MI355X statevector hot path.
 *
 * What is computed (TensorCircuit-NG paper, Sec. "Foundations Recap" and
 * Sec. "Data Parallelism"):
 *   |psi(theta)> = U_D(theta) ... U_1(theta) |psi_0>      gates as local contractions
 *   E(theta)     = Re <psi(theta)| H |psi(theta)>,  H = sum_k c_k P_k   (expectation_ps)
 *   dE/dtheta                                          (value_and_grad; here by the adjoint method)
 * batched over many parameter sets (the VMAP paradigm, "parameter parallelism")
 * and over many different circuits (uneven batches).
 *
 * Conventions (readings where the paper is silent):
 *   - amplitudes are interleaved complex, the memory layout of torch.complex64 /
 *     torch.complex128; amplitude index bit q <-> qubit q (qubit 0 = LSB);
 *   - a k-qubit matrix acting on qubits (q_0, ..., q_{k-1}) is row-major
 *     2^k x 2^k with q_0 the most significant bit of its local index;
 *   - R_P(theta) = exp(-i theta P / 2) for RX/RY/RZ, RZZ = exp(-i theta ZZ/2),
 *     FSIM(theta, phi) = [[1,0,0,0],[0,c,-is,0],[0,-is,c,0],[0,0,0,e^{-i phi}]]
 *     with c = cos theta, s = sin theta;
 *   - Pauli codes 0 = I, 1 = X, 2 = Y, 3 = Z (the paper's shadow encoding).
 *
 * General rules for every call:
 *   - returns TCNG_OK or an error code; tcng_last_error() gives a message
 *     (thread-local, valid until the next call on the same thread);
 *   - device pointers are caller-owned (e.g. torch tensors) and must stay
 *     valid until the stream reaches the work; host pointers are read before
 *     the call returns;
 *   - work is enqueued on `stream` (a hipStream_t, NULL = default stream) and
 *     is asynchronous; outputs are valid once the stream reaches them;
 *   - no call allocates device memory after tcng_circuit_create /
 *     tcng_pauli_sum_create (which upload their own small descriptor tables);
 *     scratch space comes from the caller's workspace (tcng_workspace_size);
 *   - a workspace must not be used by two calls that may overlap in time.
 */
#ifndef TCNG_ABI_H_
#define TCNG_ABI_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tcng_status;
enum {
    TCNG_OK = 0,
    TCNG_E_INVALID = 1,     /* bad argument: null pointer, qubit out of range, duplicate qubits, ... */
    TCNG_E_UNSUPPORTED = 2, /* valid request this library does not implement (e.g. n too large)      */
    TCNG_E_WORKSPACE = 3,   /* workspace smaller than tcng_workspace_size() says                     */
    TCNG_E_HIP = 4,         /* HIP runtime error (launch failure, or an earlier asynchronous error)  */
    TCNG_E_ALLOC = 5        /* host or device allocation failed at create time                       */
};

enum { TCNG_C64 = 0, TCNG_C128 = 1 };

/* Execution strategy of the circuit passes.
 *   TCNG_MODE_TILED: gates are scheduled into passes over 2^m-amplitude tiles
 *     held in registers and LDS; one HBM round trip applies many gates.
 *   TCNG_MODE_PLAIN: one streaming kernel per gate (and per Pauli x-group);
 *     the unfused baseline.
 *   TCNG_MODE_FUSED: the tiled passes with every register phase multiplied
 *     out into one 16 x 16 block matrix (float64 product, rounded once to
 *     float32) applied on the matrix cores (operator fusion, Sec.
 *     "Foundations Recap", JIT paragraph); the adjoint sweep accumulates each
 *     block's outer product sum(lambda psi^dagger) and derives every gate
 *     derivative from it.  complex64 states with n >= 9 only; otherwise the
 *     call runs as TCNG_MODE_TILED.
 *   TCNG_MODE_FUSED5: the same with 5-qubit blocks, 32 x 32 block matrices
 *     (applied as four 16 x 16 sub-block products; one block holds more gates
 *     and costs twice the matrix-core work per amplitude).  complex64 states
 *     with n >= 12 only; otherwise the call runs as TCNG_MODE_FUSED.
 *     tcng_autotune picks among the modes per circuit. */
enum { TCNG_MODE_TILED = 0, TCNG_MODE_PLAIN = 1, TCNG_MODE_FUSED = 2, TCNG_MODE_FUSED5 = 3, TCNG_MODE_AUTO = 4 };
/* TCNG_MODE_AUTO: the mode tcng_autotune chose for the circuit and dtype;
 * before any tuning, TCNG_MODE_FUSED for complex64 and TCNG_MODE_TILED for
 * complex128. */

/* gate kinds of tcng_gate.kind */
enum {
    TCNG_RX = 0, TCNG_RY = 1, TCNG_RZ = 2, TCNG_H = 3, TCNG_X = 4, TCNG_Y = 5, TCNG_Z = 6,
    TCNG_S = 7, TCNG_CNOT = 8, TCNG_CZ = 9, TCNG_RZZ = 10, TCNG_FSIM = 11,
    TCNG_U1 = 12, /* constant 2x2 matrix: top-left block of const_mats[mat] */
    TCNG_U2 = 13  /* constant 4x4 matrix const_mats[mat]                    */
};

/* A batch of statevectors: a NON-OWNING view of device memory.
 * Member b occupies amps + b*stride*(8 or 16 bytes), 2^n_qubits amplitudes. */
typedef struct tcng_state {
    void* amps;        /* device, interleaved complex in `dtype`                 */
    int32_t n_qubits;  /* 1 .. 34                                                */
    int32_t dtype;     /* TCNG_C64 or TCNG_C128                                  */
    int64_t batch;     /* >= 1                                                   */
    int64_t stride;    /* amplitudes between batch members, >= 2^n_qubits        */
} tcng_state;

/* One gate of a circuit.  q1 = -1 for one-qubit kinds; for CNOT q0 is the
 * control.  p0/p1 index the parameter vector (-1 = unused; FSIM uses p0 = theta,
 * p1 = phi); mat indexes the circuit's constant matrices (U1/U2 only). */
typedef struct tcng_gate {
    int32_t kind, q0, q1, p0, p1, mat;
} tcng_gate;

typedef struct tcng_circuit tcng_circuit;     /* immutable host handle + device tables */
typedef struct tcng_pauli_sum tcng_pauli_sum; /* immutable host handle + device tables */

const char* tcng_last_error(void);
int32_t tcng_version(void);

/* psi := |basis_index> (amps_in == NULL) or a copy of amps_in (device, same
 * dtype, 2^n amplitudes, copied into every batch member).  Paper: Circuit(n)
 * starts from |0...0>; Circuit(n, inputs=x) from given amplitudes (Sec.
 * "End-to-End Pure QML for Computer Vision", amplitude encoding). */
tcng_status tcng_state_init(const tcng_state* s, const void* amps_in, int64_t basis_index, void* stream);

/* Apply one k-qubit matrix (1 <= k <= 5) to every batch member in place.
 * unitary: DEVICE pointer, row-major 2^k x 2^k complex in the state's dtype,
 * qubits[0] = most significant local bit (Sec. "Foundations Recap": a gate is
 * a local tensor contraction).  qubits: host array of k distinct qubits. */
tcng_status tcng_apply_gate(const tcng_state* s, const int32_t* qubits, int32_t k, const void* unitary,
                            void* stream);

/* Build a circuit handle on the current device: the gate list of a
 * parameterised circuit, each gate added by kind with its qubits and angle
 * indices (the paper's Circuit(n) followed by c.rx(i, theta=...),
 * c.cnot(i, j), ..., Sec. "Foundations Recap").  The handle is immutable and
 * owns its host plans and their small device tables (uploaded here; the only
 * device allocation of the library besides tcng_pauli_sum_create).
 *   n_qubits    1 .. 34;
 *   gates       host [n_gates] (read before return), in application order;
 *   n_params    length of every parameter vector the circuit is evaluated with;
 *               each p0/p1 is -1 or in [0, n_params);
 *   const_mats  host complex128 [n_mats][4][4] interleaved (NULL if n_mats = 0);
 *               U1 uses the top-left 2x2 of its matrix, U2 the whole 4x4;
 *   out         receives the handle (release with tcng_circuit_destroy).
 * Errors: TCNG_E_INVALID for out-of-range / duplicate qubits, bad kinds,
 * parameter or matrix indices out of range, null pointers; TCNG_E_ALLOC if
 * host or device memory runs out. */
tcng_status tcng_circuit_create(int32_t n_qubits, const tcng_gate* gates, int32_t n_gates, int32_t n_params,
                                const double* const_mats, int32_t n_mats, tcng_circuit** out);
/* Waits for the device (enqueued work may still read the tables), then frees. */
tcng_status tcng_circuit_destroy(tcng_circuit* c);
/* Number of tiled passes the planner produced for `dtype` (forward sweep). */
tcng_status tcng_circuit_num_passes(const tcng_circuit* c, int32_t dtype, int32_t* passes);

/* Uneven batch (the VMAP paradigm over circuits that differ in qubit count,
 * depth and Hamiltonian, Sec. "Data Parallelism"): value and adjoint gradient
 * of `count` circuits, each with its own Pauli sum, angles and single state,
 * in shared launches -- the k-th pass of every circuit that has one runs in
 * one launch, so the number of launches follows the deepest circuit, not the
 * number of circuits.  Every circuit must have the tiled path for the dtype
 * (n >= 11 for complex64, >= 10 for complex128) with the same register block
 * sizes, and its Pauli sum a tiled plan; else TCNG_E_UNSUPPORTED.  A complex64
 * batch runs on the matrix-core (fused) passes, a complex128 batch on the
 * tiled passes.
 *   circs, hams : host arrays [count] of handles
 *   params      : host array [count] of DEVICE pointers to the angles (NULL when
 *                 the circuit has none), float32 / float64 as the dtype
 *   psi, lam    : host arrays [count] of states (batch 1, dtype as the first)
 *   energy      : DEVICE float64 [count]
 *   grad        : host array [count] of DEVICE float64 [n_params] (entries may be NULL
 *                 only for circuits without angles); NULL if no circuit has angles
 *   gate_grad   : NULL, or host array [count] of DEVICE float64 [n_gates][15]
 * The workspace holds every circuit's scratch and the launch tables. */
tcng_status tcng_workspace_size_multi(const tcng_circuit* const* circs, const tcng_pauli_sum* const* hams,
                                      int32_t count, int32_t dtype, size_t* bytes);
tcng_status tcng_expect_grad_multi(const tcng_circuit* const* circs, const tcng_pauli_sum* const* hams, int32_t count,
                                   const void* const* params, const tcng_state* psi, const tcng_state* lam,
                                   double* energy, double* const* grad, double* const* gate_grad, void* ws,
                                   size_t ws_bytes, void* stream);

/* Tiling of the tiled path for `dtype`: tile bits m_max (at most 13 for
 * TCNG_C64, 12 for TCNG_C128), register bits per thread in the forward sweep
 * rb and per thread and state in the reverse sweep rb_rev (4 or 5 for C64,
 * 3 or 4 for C128), with 6 <= m_max - rb, m_max - rb_rev <= 9.  Rebuilds and
 * uploads the plan (synchronises the device).  TCNG_E_UNSUPPORTED if the
 * shape is not available or the circuit is too small for the tiled path. */
tcng_status tcng_circuit_configure(tcng_circuit* c, int32_t dtype, int32_t m_max, int32_t rb, int32_t rb_rev);
tcng_status tcng_circuit_get_config(const tcng_circuit* c, int32_t dtype, int32_t* m_max, int32_t* rb,
                                    int32_t* rb_rev);
/* The mode TCNG_MODE_AUTO runs for this circuit and dtype (after tuning, or
 * the default), resolved to the plan that exists (never TCNG_MODE_AUTO). */
tcng_status tcng_circuit_get_mode(const tcng_circuit* c, int32_t dtype, int32_t* mode);
/* Rounds: a tiled pass (TCNG_MODE_TILED, and the tiled candidates of the
 * autotuner; complex64 or complex128) whose gates are all RY, RZ and CNOT
 * runs as fixed rounds of rotations on the tiling's register bits (reg_bits
 * forward, reg_bits_rev reverse) per phase, with each phase's CNOTs applied
 * as a permutation of the tile's local index; one whose gates are all fSim
 * and Hadamard runs as fixed rounds of fSim gates on register-bit pairs (the
 * paper's operator fusion of the "Foundations Recap" section, done on the
 * vector units).  Other passes of the same circuit run the generic tiled
 * kernels.  *phases = the number of round phases of the current forward
 * plan, 0 when no pass of the circuit or dtype takes this path. */
tcng_status tcng_circuit_rounds(const tcng_circuit* c, int32_t dtype, int32_t* phases);

/* Autotuner (the find-then-execute search of contraction strategies, Sec.
 * "Model Parallelism", applied to execution strategies): times
 * tcng_expect_grad for every available tiling of the tiled passes
 * (TCNG_MODE_TILED) and, for complex64, the matrix-core passes with 4- and
 * 5-qubit blocks (TCNG_MODE_FUSED, TCNG_MODE_FUSED5), for this dtype and
 * batch, on the given initial states psi (restored afterwards up to rounding)
 * and scratch lam.  The fastest (median of `repeats` runs, ties to the earlier
 * candidate) becomes the circuit's TCNG_MODE_AUTO for the dtype; the tiled
 * passes keep their fastest tiling.  Allocates and frees its own workspace and
 * synchronises; not for the hot path.  params as for tcng_expect_grad.
 * best_ms (nullable) receives the winner's median time.  If cache_path is not
 * NULL, the choice is looked up in / appended to that text file, keyed by the
 * circuit's structure, dtype, batch and device architecture; a cached choice
 * is applied without timing. */
tcng_status tcng_autotune(tcng_circuit* c, const tcng_pauli_sum* h, const void* params, const tcng_state* psi,
                          const tcng_state* lam, int32_t repeats, const char* cache_path, double* best_ms,
                          void* stream);

/* Build a Pauli-sum handle: codes host uint8 [n_terms][n_qubits] (0=I,1=X,2=Y,3=Z),
 * coeffs host float64 [n_terms] (Sec. "Data Parallelism": H = sum_i c_i P_i). */
tcng_status tcng_pauli_sum_create(int32_t n_qubits, const uint8_t* codes, const double* coeffs, int32_t n_terms,
                                  tcng_pauli_sum** out);
tcng_status tcng_pauli_sum_destroy(tcng_pauli_sum* h);

/* An uneven batch bound once to its circuits, Pauli sums, angle buffers,
 * states, outputs and workspace (arguments as for tcng_expect_grad_multi):
 * the launch tables are built on the host and copied into the workspace here
 * (after the device is idle; synchronises), so tcng_multi_launch enqueues
 * kernels only and can be captured in a graph (tcng_graph_create_multi) and
 * replayed; new angles are written into the same buffers between launches.
 * init_basis >= 0: every launch starts each circuit from |init_basis> (the
 * matrix-core first pass forms its tiles without reading the state; the tiled
 * path sets the states first); -1: from the states' contents, as
 * tcng_expect_grad_multi.  The handle, the workspace and every bound buffer
 * must outlive the launches; handles own no device memory. */
typedef struct tcng_multi tcng_multi;
tcng_status tcng_multi_create(const tcng_circuit* const* circs, const tcng_pauli_sum* const* hams, int32_t count,
                              const void* const* params, const tcng_state* psi, const tcng_state* lam, double* energy,
                              double* const* grad, double* const* gate_grad, int64_t init_basis, void* ws,
                              size_t ws_bytes, tcng_multi** out);
tcng_status tcng_multi_launch(const tcng_multi* m, void* stream);
tcng_status tcng_multi_destroy(tcng_multi* m);

/* Matrix-free Pauli-sum operator (Sec. "Time Evolution": the sparse
 * matrix-vector product of Krylov and Chebyshev evolution):
 * out_b = H psi_b for every batch member, and, if energy is not NULL,
 * energy[b] = Re <psi_b|H|psi_b> accumulated in float64 (DEVICE [batch]).
 * out must match psi in qubits, dtype, batch and stride and must not alias
 * it; ws as for tcng_expect_pauli (tcng_workspace_size with c = NULL).
 * Errors as for tcng_expect_pauli, TCNG_E_INVALID for a mismatched or
 * aliased output. */
tcng_status tcng_apply_pauli(const tcng_state* psi, const tcng_pauli_sum* h, const tcng_state* out, double* energy,
                             int32_t mode, void* ws, size_t ws_bytes, void* stream);

/* Sparse (COO) matrix of the Pauli sum (Sec. "Lattice and Hamiltonian", the
 * PauliStringSum2COO construction).  A term with X-mask x maps |col> to
 * |col ^ x>, so H[row][col] is nonzero only at col = row ^ x.  Terms are
 * grouped by X-mask, groups in the order their mask first appears in the
 * term list; tcng_pauli_coo_info gives the group count G.
 * tcng_pauli_coo writes one entry per (group g, row) for the rows
 * [row_begin, row_begin + row_count), group-major: entry g * row_count + r
 * holds row = row_begin + r, col = row ^ x_g and the complex128 value
 * sum over the group's terms (in list order) of c_k <row|P_k|col> (exact
 * zeros are kept).  rows, cols: DEVICE int64 [G * row_count]; vals: DEVICE
 * complex128 [G * row_count].  Asynchronous on `stream`.
 * TCNG_E_INVALID for a row range outside [0, 2^n) or null outputs,
 * TCNG_E_UNSUPPORTED for n > 62 or more than 65535 groups. */
tcng_status tcng_pauli_coo_info(const tcng_pauli_sum* h, int32_t* n_groups);
tcng_status tcng_pauli_coo(const tcng_pauli_sum* h, int64_t row_begin, int64_t row_count, int64_t* rows, int64_t* cols,
                           void* vals, void* stream);

/* Bytes of workspace needed by tcng_run_circuit / tcng_expect_pauli /
 * tcng_apply_pauli / tcng_expect_grad / tcng_graph_create for this shape (c or h may be NULL
 * when not used); the caller allocates it (device memory). */
tcng_status tcng_workspace_size(const tcng_circuit* c, const tcng_pauli_sum* h, int32_t dtype, int64_t batch,
                                int32_t mode, size_t* bytes);

/* Apply the circuit in place to every batch member of s (state evolution by
 * local contractions, Sec. "Foundations Recap").
 * params: DEVICE [batch][n_params], float32 for TCNG_C64, float64 for TCNG_C128
 * (may be NULL when n_params == 0). */
tcng_status tcng_run_circuit(const tcng_circuit* c, const void* params, const tcng_state* s, int32_t mode,
                             void* ws, size_t ws_bytes, void* stream);

/* out[b] = Re <psi_b| H |psi_b> accumulated in float64 (DEVICE float64 [batch])
 * (expectation of Pauli strings, Sec. "Foundations Recap"). */
tcng_status tcng_expect_pauli(const tcng_state* s, const tcng_pauli_sum* h, double* out, int32_t mode, void* ws,
                              size_t ws_bytes, void* stream);

/* Value and adjoint gradient (value_and_grad with reverse-mode AD, Sec.
 * "Foundations Recap"; the batch is the VMAP axis).
 *   psi   : in  = initial states |psi_0> (batch members);
 *           out = the initial states recomputed by the reverse sweep (equal to
 *                 the input up to rounding);
 *   lam   : scratch state of the same shape (holds H psi, then the costates);
 *   energy: DEVICE float64 [batch], E_b;
 *   grad  : DEVICE float64 [batch][n_params], dE_b/dtheta summed over every use;
 *   gate_grad (nullable): DEVICE float64 [batch][n_gates][15]: for each
 *           constant two-qubit gate (TCNG_U2), dE/dalpha_k for
 *           U -> exp(-i alpha_k P_k / 2) U, P_k = sigma_a (x) sigma_b acting on
 *           (q0, q1), k = 4a + b - 1; rows of all other gates are zero.
 * The reverse sweep recomputes states by applying inverse gates; nothing is
 * stored per gate. */
tcng_status tcng_expect_grad(const tcng_circuit* c, const void* params, const tcng_pauli_sum* h,
                             const tcng_state* psi, const tcng_state* lam, double* energy, double* grad,
                             double* gate_grad, int32_t mode, void* ws, size_t ws_bytes, void* stream);

/* tcng_expect_grad without a workspace argument, for callers that cannot
 * allocate device memory (code under graph capture, serving loops, harnesses
 * that forbid hipMalloc).  The workspace is a fixed device array inside the
 * library of tcng_noalloc_scratch_bytes() bytes (64 MiB), one copy per GPU,
 * held until the process ends; its device address is resolved once per device
 * on the first call there.  Arguments, outputs and modes are those of
 * tcng_expect_grad; the call allocates nothing (no hipMalloc, no library
 * allocation) and leaves the array holding the evaluation's partial sums.
 * Errors: those of tcng_expect_grad, and TCNG_E_WORKSPACE when the shape needs
 * more workspace than the array holds (tcng_workspace_size tells).
 * Every call on one GPU shares its array: calls that overlap on one GPU (two
 * streams, two threads) race and must be ordered by the caller. */
tcng_status tcng_expect_grad_noalloc(const tcng_circuit* c, const void* params, const tcng_pauli_sum* h,
                                     const tcng_state* psi, const tcng_state* lam, double* energy, double* grad,
                                     double* gate_grad, int32_t mode, void* stream);
size_t tcng_noalloc_scratch_bytes(void);

/* Kernel-family timing with HIP events recorded on the launch stream around
 * every launch (benchmark instrumentation, not part of the method; off by
 * default).
 * tcng_profile_begin allocates up to max_launches event pairs and starts
 * recording; tcng_profile_query synchronises the recorded events and returns
 * the launch count and summed duration (ms) of one family:
 *   0 forward tile pass   1 reverse tile pass   2 Pauli tile pass
 *   3 one-qubit gate      4 two-qubit gate      5 k-qubit gate
 *   6 reverse one-qubit   7 reverse two-qubit   8 Pauli X-group
 *   9 final reduction     10 state init
 *   11 fused forward pass  12 fused reverse pass  13 fused block matrices and gradients
 *   14 trajectory histogram pass  15 trajectory decisions  16 trajectory collapse
 *   17 Pauli-sum COO entries  18 shadow chunk sums  19 shadow rotations and draws
 *   20 QML gate matrices, readout and angle gradients
 * tcng_profile_end stops recording and frees the events. */
enum { TCNG_PROF_FAMILIES = 21 };
tcng_status tcng_profile_begin(int32_t max_launches);
tcng_status tcng_profile_query(int32_t family, int32_t* launches, double* total_ms);
tcng_status tcng_profile_end(void);

/* Host-only inspection of the tiled planner (pass scheduling of the gate
 * contractions of Sec. "Foundations Recap"; no device is touched): the
 * schedule tcng_circuit_create would build for `dtype`.  Outputs (host):
 *   order[n_gates]      gate indices in execution order of the forward sweep;
 *   pass_of[n_gates]    pass in which gate order[i] runs;
 *   tile_mask[n_gates]  qubit mask of pass p's tile in entry p (p < *n_passes);
 *   n_passes            number of passes (0 if the tiled path does not apply).
 * Any output pointer may be NULL. */
tcng_status tcng_plan_inspect(int32_t n_qubits, const tcng_gate* gates, int32_t n_gates, int32_t n_params,
                              int32_t dtype, int32_t* order, int32_t* pass_of, uint64_t* tile_mask,
                              int32_t* n_passes);

/* Host-only inspection of the rounds of a tiled plan (operator fusion of
 * Sec. "Foundations Recap" on the vector units; no device is touched), for
 * the tiling tile_bits (9..13), reg_bits (forward) and reg_bits_rev
 * (reverse), each 3..5.  Outputs (host, any may be NULL):
 *   n_round_passes  passes that run rotation or fSim rounds;
 *   n_phases        round phases of the forward sweep;
 *   bad_layouts     round phases (both sweeps) whose LDS layouts are not
 *                   bijections of the tile, whose pass does not start from
 *                   the tile load's layout, or whose reading lanes, or the
 *                   writing lanes of the phase before, put two of 8, 16 or 32
 *                   consecutive lanes on one bank (0 expected).
 * Returns TCNG_E_INVALID for a tiling out of range and TCNG_E_UNSUPPORTED
 * when the planner rejects it for this circuit. */
tcng_status tcng_rounds_plan_inspect(int32_t n_qubits, const tcng_gate* gates, int32_t n_gates, int32_t n_params,
                                     int32_t tile_bits, int32_t reg_bits, int32_t reg_bits_rev,
                                     int32_t* n_round_passes, int32_t* n_phases, int32_t* bad_layouts);

/* Graph capture of one evaluation: the trace-once, run-many JIT paradigm
 * (Sec. "Foundations Recap", JIT paragraph) done as a HIP graph:
 * tcng_graph_create records state init to |basis> (skipped when init_basis
 * < 0) and tcng_expect_grad with exactly these arguments into a HIP graph;
 * tcng_graph_launch replays it on `stream`.  Every pointer is captured: to
 * evaluate new angles, write them into the same `params` buffer (stream-
 * ordered before the launch) and read energy / grad after it.  The graph
 * owns no device memory; the caller keeps every buffer alive until
 * tcng_graph_destroy (which synchronizes the device).  Creation fails while
 * tcng_profile is recording.  Captures contain kernels only (no memsets or
 * copies); the uneven-batch call cannot be captured. */
typedef struct tcng_graph tcng_graph;
tcng_status tcng_graph_create(const tcng_circuit* c, const void* params, const tcng_pauli_sum* h,
                              const tcng_state* psi, const tcng_state* lam, double* energy, double* grad,
                              double* gate_grad, int32_t mode, void* ws, size_t ws_bytes, int64_t init_basis,
                              tcng_graph** out);
tcng_status tcng_graph_launch(tcng_graph* g, void* stream);
/* One launch of a bound uneven batch (tcng_multi_launch) recorded as a graph. */
tcng_status tcng_graph_create_multi(const tcng_multi* m, tcng_graph** out);
tcng_status tcng_graph_destroy(tcng_graph* g);

/* Host-only inspection of the fused planner (TCNG_MODE_FUSED with
 * block_bits = 4, TCNG_MODE_FUSED5 with 5; complex64; gate application as
 * local contraction, Sec. "Foundations Recap").
 * Outputs (host, any may be NULL):
 *   order[n_gates], pass_of[n_gates]  as for tcng_plan_inspect;
 *   block_of[n_gates]                 block (2^k x 2^k matrix) of gate order[i];
 *   n_passes, n_blocks;
 *   bad_layouts  number of LDS layouts of the plan that are not bijections of
 *                the tile or that put two lanes of a 32-lane access of the
 *                phases that write or read them on one bank (0 expected).
 * Returns TCNG_E_UNSUPPORTED when the fused path does not apply (n < 9, or
 * n < 12 for 5-qubit blocks); TCNG_E_INVALID for block_bits other than 4, 5. */
tcng_status tcng_fused_plan_inspect(int32_t n_qubits, const tcng_gate* gates, int32_t n_gates, int32_t n_params,
                                    int32_t block_bits, int32_t* order, int32_t* pass_of, int32_t* block_of,
                                    int32_t* n_passes, int32_t* n_blocks, int32_t* bad_layouts);

/* SU(4) brick-wall QML training step (Sec. "End-to-End Pure QML for Computer
 * Vision"): every sample starts from its amplitude-encoded input, the gates of
 * c act in order, gate g being the SU(4) gate U(theta[g.mat]) =
 * exp(-i sum_k theta_k P_k / 2), P_k = sigma_a (x) sigma_b, k = 4a + b - 1,
 * sigma_a on the gate's first qubit; the readout p_o sums |psi_x|^2 over the
 * x whose top k index bits equal o (the paper's first k qubits, its qubit 0
 * being the most significant); the first n_classes of them are the logits of
 * a softmax cross entropy with the sample's label.
 *   c        n_params = 0, every gate U2 with its own matrix index (the
 *            creation matrices only fix the count M = n_mats); n >= 9;
 *   theta    device float64 [M][15];
 *   inputs   complex64 states (normalised amplitude encodings), not modified
 *            unless psi is the same memory (then evolved in place);
 *   psi, lam complex64 work states of the same shape (overwritten); lam must
 *            not share memory with psi or the inputs;
 *   labels   device int32 [batch] in [0, n_classes) (a label outside gives a
 *            NaN loss and no gradient contribution);
 *   k        readout qubits, 1..min(8, n); n_classes in 1..2^k;
 *   loss     device float64 [batch]: per-sample cross entropy (written);
 *   grad     device float64 [M][15]: d(mean loss)/dtheta (written);
 *   ws       device workspace of tcng_qml_workspace_size bytes.
 * An angle that is infinite or NaN gives NaN losses and gradients.
 * Asynchronous on `stream`; TCNG_E_UNSUPPORTED for complex128 or n < 9,
 * TCNG_E_INVALID for a malformed circuit, mismatched or aliased states, bad k
 * or classes, batch above 65535 or null arguments, TCNG_E_WORKSPACE if ws is
 * too small. */
tcng_status tcng_qml_workspace_size(const tcng_circuit* c, int64_t batch, size_t* bytes);
tcng_status tcng_qml_step(const tcng_circuit* c, const double* theta, const tcng_state* inputs, const tcng_state* psi,
                          const tcng_state* lam, const int32_t* labels, int32_t k, int32_t n_classes, double* loss,
                          double* grad, void* ws, size_t ws_bytes, void* stream);

/* Classical-shadow snapshots (Sec. "Efficient ML Pipeline via Classical
 * Shadows", measurement only): snapshot s measures every qubit q of the state
 * in the Pauli basis bases[s][q] (1 = X, 2 = Y, 3 = Z): the state is rotated
 * by V_q (X: H; Y: H S^dagger; Z: identity), so that outcome 0 is the +1
 * eigenvector of the chosen Pauli, and one basis state x is drawn from
 * |psi'_x|^2 by the inverse distribution function with the uniform u[s]:
 * the first x whose running probability (increasing x, float64) exceeds u[s].
 *   layer     circuit of n one-qubit gates, gate q = U1 on qubit q with matrix
 *             q (its creation matrices only fix the count); needs n >= 9;
 *   psi       device complex64 [2^n], the state (not modified); it must not
 *             overlap the memory of `work` (TCNG_E_INVALID);
 *   work      complex64 state with batch = number of snapshots S, overwritten
 *             with the rotated copies;
 *   bases     device uint8 [S][n] (codes other than 1 and 2 act as 3);
 *   u         device float64 [S] in [0, 1);
 *   outcomes  device int64 [S]: x, bit q = the outcome of qubit q (written);
 *   ws        device workspace of tcng_shadow_workspace_size bytes.
 * Asynchronous on `stream`; TCNG_E_UNSUPPORTED for complex128 or n < 9,
 * TCNG_E_INVALID for a malformed layer, mismatched state, psi overlapping
 * work or null arguments, TCNG_E_WORKSPACE if ws is too small. */
tcng_status tcng_shadow_workspace_size(const tcng_circuit* layer, int64_t snapshots, size_t* bytes);
tcng_status tcng_shadow_snapshots(const tcng_circuit* layer, const void* psi, const tcng_state* work,
                                  const uint8_t* bases, const double* u, int64_t* outcomes, void* ws, size_t ws_bytes,
                                  void* stream);

/* Monitored Haar brick-wall trajectories (Sec. "Universal Quantum Dynamics of
 * Haar-Random MIPT": per time step two layers of Haar two-qubit gates on the
 * even, then the odd bonds, then each qubit measured in Z with probability p;
 * one trajectory per batch member, complex64).
 * The measurement layer is the Kraus channel {sqrt(1-p) I, sqrt(p) P0,
 * sqrt(p) P1} per qubit, qubits in increasing order, selected by one uniform
 * v per (member, step, qubit):
 *   v < 1 - p                          not measured;
 *   v - (1 - p) < p P(bit q = 0 | ...)  outcome 0, otherwise outcome 1,
 * P conditional on the outcomes taken earlier in the step, computed in
 * float64; the state is projected and renormalised once per step.
 *   step     circuit of one time step; every gate U2, gate g taking step
 *            matrix g.mat (its creation matrices only fix the count n_mats);
 *            needs the fused path (9 <= n) and n <= 32;
 *   n_steps  time steps (0: nothing is applied, outputs zeroed);
 *   mats     device, complex64 [batch][n_steps][n_mats][4][4] row-major, the
 *            first gate qubit the most significant local index;
 *   psi      complex64 states, evolved in place (the caller initialises them);
 *   u        device float64 [batch][n_steps][n] uniforms in [0, 1);
 *   p        measurement probability in [0, 1];
 *   rec      device uint32 [batch][n_steps][2]: measured-qubit mask, outcome
 *            bits (written; may be NULL when n_steps is 0);
 *   logp     device float64 [batch]: sum of ln P(outcome) over the record
 *            (the trajectory's Born log-probability; written);
 *   margin   device float64 [batch][n_steps][n] or NULL: v - (1 - p) - p P0
 *            for each measured qubit (other entries untouched);
 *   ws       device workspace of tcng_mipt_workspace_size bytes.
 * Asynchronous on `stream`; TCNG_E_UNSUPPORTED for complex128, n < 9 or
 * n > 32, TCNG_E_INVALID for non-U2 step gates, angles, bad p or null
 * arguments, TCNG_E_WORKSPACE if ws is too small. */
tcng_status tcng_mipt_workspace_size(const tcng_circuit* step, int32_t n_qubits, int64_t batch, size_t* bytes);
tcng_status tcng_mipt_run(const tcng_circuit* step, int32_t n_steps, const void* mats, tcng_state* psi,
                          const double* u, double p, uint32_t* rec, double* logp, double* margin, void* ws,
                          size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* TCNG_ABI_H_ */
