// Shared definitions of the HIP library: complex arithmetic on interleaved
// (re, im) pairs, the gate-kind enum of the C ABI, and the plan descriptors
// the host planner writes for the tiled kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tcng.h"

namespace tcng {

// ---------------------------------------------------------------------------
// complex numbers in the layout of torch.complex64 / complex128
// ---------------------------------------------------------------------------
template <typename R>
struct alignas(2 * sizeof(R)) cx {
    R re, im;
};

template <typename R>
__host__ __device__ __forceinline__ cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__host__ __device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
__host__ __device__ __forceinline__ float fmaR(float a, float b, float c) { return fmaf(a, b, c); }
__host__ __device__ __forceinline__ double fmaR(double a, double b, double c) { return fma(a, b, c); }
// a*b + c
template <typename R>
__host__ __device__ __forceinline__ cx<R> cfma(cx<R> a, cx<R> b, cx<R> c) {
    return {fmaR(a.re, b.re, fmaR(-a.im, b.im, c.re)), fmaR(a.re, b.im, fmaR(a.im, b.re, c.im))};
}

// gate kinds (values of the C ABI)
enum Kind : int {
    K_RX = TCNG_RX, K_RY = TCNG_RY, K_RZ = TCNG_RZ, K_H = TCNG_H, K_X = TCNG_X, K_Y = TCNG_Y,
    K_Z = TCNG_Z, K_S = TCNG_S, K_CNOT = TCNG_CNOT, K_CZ = TCNG_CZ, K_RZZ = TCNG_RZZ,
    K_FSIM = TCNG_FSIM, K_U1 = TCNG_U1, K_U2 = TCNG_U2, K_COUNT
};

__host__ __device__ inline int kind_arity(int k) {
    return (k == K_CNOT || k == K_CZ || k == K_RZZ || k == K_FSIM || k == K_U2) ? 2 : 1;
}
__host__ __device__ inline int kind_nparams(int k) {
    return (k == K_RX || k == K_RY || k == K_RZ || k == K_RZZ) ? 1 : (k == K_FSIM ? 2 : 0);
}
__host__ __device__ inline bool kind_diagonal(int k) {
    return k == K_RZ || k == K_Z || k == K_S || k == K_CZ || k == K_RZZ;
}
// gradient slots (float64 accumulators) one gate needs in the reverse sweep:
// one per angle, 32 for the 4x4 complex cotangent of a constant U2
__host__ __device__ inline int kind_slots(int k) {
    return k == K_U2 ? 32 : kind_nparams(k);
}

// ---------------------------------------------------------------------------
// tiled-pass plan (written on the host, read by the kernels)
// ---------------------------------------------------------------------------
constexpr int MAX_TILE_BITS = 14;
constexpr int MAX_RB = 5;
constexpr int RED_SLOTS = 256;   // float64 gradient accumulators per wave and reverse pass
constexpr int MAX_THREADS = 512; // threads per tile workgroup (2^(m - rb))

enum OpType : int8_t {
    OP_DENSE1 = 0,  // 2x2 matrix, operand in register bit r0
    OP_DIAG1 = 1,   // diagonal 2x2 on bit (r0 | lb0)
    OP_CX = 2,      // CNOT: target in register bit r1, control bit (r0 | lb0)
    OP_DENSE2 = 3,  // 4x4 matrix, operands in register bits r0 (MSB) and r1
    OP_DIAG2 = 4,   // diagonal 4x4 on bits (r0 | lb0), (r1 | lb1)
    OP_REAL1 = 5,   // real 2x2 matrix (RY, H, X), operand in register bit r0
    OP_RX = 6,      // [[c, -is], [-is, c]], operand in register bit r0
    OP_FSIM = 7,    // fSim: |01>,|10> block [[c, -is], [-is, c]], |11> phase; register bits r0, r1
};

// Descriptor fields are 32-bit: the kernels read them with scalar loads
// (gfx9 has no scalar sub-dword loads; byte fields become per-lane vector
// loads whose waits serialise the amplitude traffic).

// One gate inside a phase.  A qubit operand is either a register bit
// (r >= 0: bit r of the register index j) or a thread bit (r < 0: bit lb of
// the thread's part of the local index).
struct Op {
    int32_t type, kind, r0, r1, lb0, lb1;
    int32_t p0, p1, mat;
    int32_t slot;   // first gradient slot of this gate inside its reverse pass, -1 none
    int32_t gate;   // gate index in the circuit
    int32_t pad;
};

// A run of ops that all act on the same RB local bits held in registers.
struct Phase {
    int32_t op_begin, op_end;
    int32_t R[6];    // local bit position of register bit i (i < RB)
};

// One HBM round trip: tiles of 2^m amplitudes over the qubits in tile_mask.
// Local bits 0..lo-1 are qubits 0..lo-1 (contiguous in memory); local bit
// i >= lo is qubit local_qubit[i].
struct Pass {
    int32_t phase_begin, phase_end;
    int32_t m, lo;
    int32_t n_slots, slot_base;   // reverse sweep: gradient slots [slot_base, slot_base + n_slots)
    uint64_t tile_mask;
    int32_t local_qubit[16];
};

// ---------------------------------------------------------------------------
// Rotation rounds: the tiled passes of a circuit made of RY, RZ and CNOT only
// (complex64, 5 register bits).  The register position of every rotation is
// a compile-time constant of the kernel: a phase holds up to 5 qubits in
// registers and runs rounds (RY on register bits 0..4, then RZ on 0..4; an
// absent gate is the identity rotation).  The phase's CNOTs, all taken after
// its rounds, form a GF(2)-linear permutation of the tile's local index:
// amplitude y of the phase moves to C(y), which the phase applies by writing
// register j at LDS position C(y) (the reverse sweep reads it from there).
// Each boundary between two phases of a pass has its own LDS layout A (a
// linear bijection of the local index): the phase reads y at A_before(y) and
// writes C(y) at A_after(C(y)), so it keeps the images of the local bits in
// both (uimg, cimg); the reverse sweep reads through cimg and writes through
// uimg.  fSim phases have C = I.
//
// fSim rounds: the passes made of fSim gates and Hadamards only.  A phase holds a chain of
// up to 5 qubits in register bits 0..4 and runs steps of two rounds on fixed
// register pairs: (0,1) and (2,3), then (1,2) and (3,4) (an absent gate is
// the identity; fSim is symmetric in its two qubits).  Each step lists the
// gate of pair slot k (k = 0..3 in that order) in ry[k] and its first
// gradient slot (theta; phi is the next) in sy[k].  Hadamards that precede
// every other gate of their qubit in the pass are applied at the start of the
// phase holding the qubit (hmask: register bits).
//
// A pass whose gates are neither kind runs on the generic tiled kernels.
// ---------------------------------------------------------------------------
constexpr int QREG = 5;
constexpr int QK_GENERIC = 0, QK_ROT = 1, QK_FSIM = 2;   // QPass::kind

struct QStep {
    int32_t ry[QREG], rz[QREG];   // gate index of the RY / RZ on register bit i, -1: identity
    int32_t sy[QREG], sz[QREG];   // its gradient slot inside the pass, -1 none
    int32_t kind, pad;            // QK_ROT or QK_FSIM
};

struct QPhase {
    int32_t step_begin, step_end;
    int32_t R[QREG];              // local bit of register bit i
    int32_t has_map;              // 0: C is the identity
    int32_t cimg[16];             // LDS slot of C(e_b) (local bits b < m) in the layout after the phase
    int32_t hmask;                // fSim rounds: register bits taking a Hadamard before the steps
    int32_t rmask;                // local bits held in registers (bits R[i])
    int32_t rimg[QREG];           // cimg[R[i]]: the same for the register bits
    int32_t uimg[16];             // LDS slot of e_b in the layout before the phase
    int32_t ruimg[QREG];          // uimg[R[i]]
};

// The tiles' fixed LDS swizzle, a linear bijection of the local index that
// leaves bit 0 alone (so pairs of amplitudes stay adjacent): bits 5..7 fold
// onto bits 1..3.  The rounds' tile loads and stores use it; the planner
// chooses the layouts between their phases.
__host__ __device__ inline uint32_t tile_swz(uint32_t l) { return l ^ (((l >> 5) & 7u) << 1); }

struct QPass {
    int32_t phase_begin, phase_end;
    int32_t kind, pad;            // QK_*: the pass's kernel
};

// ---------------------------------------------------------------------------
// fused passes: each phase applies one 2^FUSED_K x 2^FUSED_K block matrix on
// matrix cores.  A tile's local index splits, per phase, into the block index
// j (local bits R[0..3], R[t] = bit t of j) and the column index (the other
// local bits in increasing order).  The LDS address of local index l under a
// layout is the XOR of img[b] over the set bits b of l (a linear bijection
// chosen by the planner so that the 32-lane accesses of both the phase that
// writes a layout and the phase that reads it hit distinct banks).
// ---------------------------------------------------------------------------
// A plan uses one block width for all its phases: FUSED_K = 4 (16 x 16 blocks,
// the default), or 5 (32 x 32 blocks, each applied as its four 16 x 16
// sub-blocks: the top block bit selects the half of a column).
constexpr int FUSED_K = 4;
constexpr int FUSED_KMAX = 5;
constexpr int FUSED_MAX_BLOCKS = 8;    // blocks per fused pass (outer-product accumulators in LDS)
constexpr int FUSED5_MAX_BLOCKS = 4;   // the same for 32 x 32 blocks (8 accumulated entries per thread and block)

struct FPhase {
    int32_t op_begin, op_end;      // gates of the block, circuit order (Op.r0/r1 = bit of j)
    int32_t R[FUSED_KMAX];         // local bit of block bit t (t < k)
    int32_t C[9];                  // local bit of column bit k (-1 beyond the tile)
    int32_t rd[MAX_TILE_BITS];     // layout this phase reads
    int32_t wr[MAX_TILE_BITS];     // layout this phase writes
    int32_t block;                 // index of the block (matrix table, outer-product sums)
    int32_t k;                     // block bits (4 or 5)
    // the layouts resolved at the bits the kernels need (no dependent lookups
    // on the device): images of column bit k (0 where C[k] < 0) and of block bit t
    int32_t rdc[9], wrc[9];
    int32_t rdr[FUSED_KMAX], wrr[FUSED_KMAX];
};

struct FPass {
    int32_t phase_begin, phase_end;
    int32_t m, lo;
    int32_t n_slots, slot_base;
    uint64_t tile_mask;
    int32_t local_qubit[16];
    int32_t ld[MAX_TILE_BITS];     // layout the tile load writes
    int32_t st[MAX_TILE_BITS];     // layout the tile store reads
};

// Pauli sum, grouped by X-mask, for the tiled H|psi> / <H> passes.  Inside a
// group the terms are split into classes of equal coefficient c_k i^{#Y_k},
// so the kernels count sign parities with integer adds per class: four
// elements' counts packed as bytes in one 32-bit word, so a class holds at most
// PCLASS_MAX terms.
constexpr int PAULI_RB = 4;          // element-index bits per thread in the Pauli passes (16 elements)
constexpr int PCLASS_MAX = 255;
struct PTerm {
    int32_t z_local;     // Z/Y bits inside the tile, as local bit positions
    int32_t pad;
    uint64_t z_out;      // Z/Y qubits outside the tile
    // element-index part of the sign parity: byte i of word w is
    // parity(((e << (m - PAULI_RB)) ^ x_local) & z_local) for element index e = 4 w + i
    uint32_t epar[4];
};
// A group's coefficient of psi_{l ^ x} is sum over classes of
// c * (n_terms - 2 * #odd parities): the element-independent part
// sum c * n_terms is stored with the group, and terms without Z/Y bits
// (parities all even) are not listed; a group lists at least one class (one
// without terms when none of its terms has Z/Y bits).
struct PClass {
    int32_t term_begin, term_end;
    double cre, cim;     // common coefficient c * i^{#Y}
    float fre, fim;      // the same, rounded to float32 (the complex64 passes)
};
struct PGroup {
    int32_t x_local;     // X/Y bits (all inside the tile), local positions
    int32_t class_begin, class_end;
    int32_t no_z;        // 1: no term has Z/Y bits, so the coefficient is cbr + i cbi for every element
    double cbr, cbi;     // sum over all its classes of c * n_terms
    float fbr, fbi;      // the same, rounded to float32
};
struct PPass {
    int32_t group_begin, group_end;
    int32_t m, lo;
    uint64_t tile_mask;
    int32_t local_qubit[16];
};

// Pauli sum grouped by X-mask over the full index space (plain path).
struct PTermFull {
    uint64_t z;
};
struct PClassFull {
    int32_t term_begin, term_end;
    double cre, cim;
};
struct PGroupFull {
    uint64_t x;
    int32_t class_begin, class_end;
};

}  // namespace tcng
