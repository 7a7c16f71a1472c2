// Tiled circuit passes (forward sweep and adjoint reverse sweep).
//
// One workgroup owns a tile: the 2^m amplitudes whose index bits outside the
// pass's qubit set T are fixed.  The tile is streamed HBM -> LDS with 16-byte
// coalesced accesses (T always contains the low `lo` qubits, so every tile is
// a set of contiguous 2^lo-amplitude runs), then processed in register
// phases: each thread holds 2^RB amplitudes whose local index bits are the
// phase's register bits, applies the phase's gates without any exchange, and
// hands the tile back to LDS for the next phase's bit assignment.  One pass
// thus applies many gates per HBM round trip (the paper's "operator fusion"
// under JIT, Sec. "Foundations Recap", done here in space rather than by
// multiplying matrices).
//
// The reverse sweep holds the state psi and the costate lambda = H psi pushed
// back through the circuit, evaluates each angle's derivative
// 2 Im <lambda|G|psi> in float64 and un-computes both by applying inverse
// gates (adjoint method: nothing is stored per gate).
#include "devutil.h"
#include "gates.h"

namespace tcng {

namespace {

constexpr int NTHREADS = MAX_THREADS;

// largest workgroup of a (precision, register block) instantiation: a full
// 64 KiB tile, 2^(m_max - RB) threads
template <typename R, int RB>
struct MaxThreads {
    static constexpr int value = 1 << ((sizeof(R) == 4 ? 13 : 12) - RB);
};

template <typename R>
struct Tile {
    static constexpr int ELEMS = (sizeof(R) == 4) ? (1 << 13) : (1 << 12);   // 64 KiB of LDS
};

// amplitude index offset of a local index l (disjoint bit sets add);
// lq[] holds the qubit of every local bit (identity below lo)
__device__ __forceinline__ uint64_t loc2glob(uint32_t l, int lo, int m, const int* lq) {
    uint64_t g = l & ((1u << lo) - 1);
#pragma unroll
    for (int i = 0; i < MAX_TILE_BITS; ++i)
        if (i >= lo && i < m) g |= uint64_t((l >> i) & 1) << lq[i];
    return g;
}

// tile base: the tile index's bits deposited into the qubits outside the tile
__device__ __forceinline__ uint64_t tile_base(uint64_t tile, uint64_t tmask, int n) {
    uint64_t base = 0;
    int k = 0;
    for (int q = 0; q < n; ++q) {
        if ((tmask >> q) & 1) continue;
        base |= ((tile >> k) & 1) << q;
        ++k;
    }
    return base;
}

// LDS position of local index l: XOR-swizzle bits 1..3 with bits 5..7 so that
// strided register reads spread over banks; bit 0 is untouched so 16-byte
// pairs of complex64 stay adjacent.
__device__ __forceinline__ uint32_t swz(uint32_t l) { return tile_swz(l); }

// 16-byte vector access of the state
template <typename R>
struct V16;
template <>
struct V16<float> {
    static constexpr int N = 2;
    __device__ static void load(gptr<const cx<float>> p, cx<float>* o) {
        float4 v = *reinterpret_cast<gptr<const float4>>(p);
        o[0] = {v.x, v.y};
        o[1] = {v.z, v.w};
    }
    __device__ static void store(gptr<cx<float>> p, const cx<float>* o) {
        *reinterpret_cast<gptr<float4>>(p) = make_float4(o[0].re, o[0].im, o[1].re, o[1].im);
    }
};
template <>
struct V16<double> {
    static constexpr int N = 1;
    __device__ static void load(gptr<const cx<double>> p, cx<double>* o) {
        double2 v = *reinterpret_cast<gptr<const double2>>(p);
        o[0] = {v.x, v.y};
    }
    __device__ static void store(gptr<cx<double>> p, const cx<double>* o) {
        *reinterpret_cast<gptr<double2>>(p) = make_double2(o[0].re, o[0].im);
    }
};

struct PassInfo {
    int m, lo;
    uint64_t tmask;
    int lq[MAX_TILE_BITS];   // local bit -> qubit (uniform: scalar registers)
};

__device__ __forceinline__ PassInfo read_pass(cptr<Pass> P) {
    PassInfo pi;
    pi.m = P->m;
    pi.lo = P->lo;
    pi.tmask = P->tile_mask;
#pragma unroll
    for (int i = 0; i < MAX_TILE_BITS; ++i) pi.lq[i] = P->local_qubit[i];
    return pi;
}

// HBM -> LDS (coalesced: lane-consecutive 16-byte chunks of local index space)
template <typename R, int RB>
__device__ __forceinline__ void tile_load(cx<R>* lds, gptr<const cx<R>> psi, uint64_t base, const PassInfo& pi, int t,
                                          int nt) {
    constexpr int VN = V16<R>::N;
    const int iters = (1 << RB) / VN;
    const uint64_t off_t = loc2glob(uint32_t(t * VN), pi.lo, pi.m, pi.lq);
    cx<R> v[(1 << RB)];
#pragma unroll
    for (int it = 0; it < iters; ++it) {
        const uint32_t e0 = uint32_t(it * nt * VN);
        const uint64_t g = base + loc2glob(e0, pi.lo, pi.m, pi.lq) + off_t;
        V16<R>::load(psi + g, &v[it * VN]);
    }
#pragma unroll
    for (int it = 0; it < iters; ++it) {
        const uint32_t e = uint32_t((it * nt + t) * VN);
#pragma unroll
        for (int k = 0; k < VN; ++k) lds[swz(e + k)] = v[it * VN + k];
    }
}

// flip: the tile holds -psi (shear rotations taken as -R(a - pi)); stored negated
template <typename R, int RB>
__device__ __forceinline__ void tile_store(const cx<R>* lds, gptr<cx<R>> psi, uint64_t base, const PassInfo& pi, int t,
                                           int nt, bool flip) {
    constexpr int VN = V16<R>::N;
    const int iters = (1 << RB) / VN;
    const uint64_t off_t = loc2glob(uint32_t(t * VN), pi.lo, pi.m, pi.lq);
    const R sg = flip ? R(-1) : R(1);
#pragma unroll
    for (int it = 0; it < iters; ++it) {
        const uint32_t e = uint32_t((it * nt + t) * VN);
        cx<R> v[VN];
#pragma unroll
        for (int k = 0; k < VN; ++k) {
            v[k] = lds[swz(e + k)];
            if (flip) v[k] = {sg * v[k].re, sg * v[k].im};
        }
        const uint64_t g = base + loc2glob(uint32_t(it * nt * VN), pi.lo, pi.m, pi.lq) + off_t;
        V16<R>::store(psi + g, v);
    }
}

// register <-> LDS for a phase.  The swizzle is linear over XOR and the
// thread part and register part of a local index have disjoint bits, so
// swz(tpart | jpart) = swz(tpart) ^ swz(jpart): one per-lane term and one
// uniform term per register.
struct PhaseMap {
    uint32_t tpart;   // thread's bits of the local index (per lane)
    uint32_t tsw;     // swz(tpart)
    uint32_t rbit[MAX_RB];
};

template <int RB>
__device__ __forceinline__ PhaseMap phase_map(cptr<Phase> F, int t, int m) {
    PhaseMap pm;
    uint32_t rmask = 0;
#pragma unroll
    for (int i = 0; i < RB; ++i) {
        pm.rbit[i] = 1u << F->R[i];
        rmask |= pm.rbit[i];
    }
    // deposit the thread index into the non-register local bits
    uint32_t tp = 0;
    int k = 0;
    for (int b = 0; b < m; ++b) {
        if ((rmask >> b) & 1) continue;
        tp |= uint32_t((t >> k) & 1) << b;
        ++k;
    }
    pm.tpart = tp;
    pm.tsw = swz(tp);
    return pm;
}

template <int RB>
__device__ __forceinline__ uint32_t jpart(const PhaseMap& pm, int j) {
    uint32_t p = 0;
#pragma unroll
    for (int i = 0; i < RB; ++i)
        if ((j >> i) & 1) p |= pm.rbit[i];
    return p;
}

template <typename R, int RB>
__device__ __forceinline__ Regs<R, (1 << RB)> regs_from_lds(const cx<R>* lds, const PhaseMap& pm) {
    Regs<R, (1 << RB)> a;
#pragma unroll
    for (int j = 0; j < (1 << RB); ++j) a.v[j] = lds[pm.tsw ^ swz(jpart<RB>(pm, j))];
    return a;
}
template <typename R, int RB>
__device__ __forceinline__ void regs_to_lds(Regs<R, (1 << RB)> a, cx<R>* lds, const PhaseMap& pm) {
#pragma unroll
    for (int j = 0; j < (1 << RB); ++j) lds[pm.tsw ^ swz(jpart<RB>(pm, j))] = a.v[j];
}

// ---------------------------------------------------------------------------
// dispatch on the register bit positions (compile-time register indices)
// ---------------------------------------------------------------------------
#define TCNG_PAIRS(X) X(0, 1) X(0, 2) X(0, 3) X(0, 4) X(1, 0) X(1, 2) X(1, 3) X(1, 4) X(2, 0) X(2, 1) \
    X(2, 3) X(2, 4) X(3, 0) X(3, 1) X(3, 2) X(3, 4) X(4, 0) X(4, 1) X(4, 2) X(4, 3)
#define TCNG_SINGLES(X) X(0) X(1) X(2) X(3) X(4)

template <typename R, int RB>
__device__ __forceinline__ Regs<R, (1 << RB)> dense1_at(Regs<R, (1 << RB)> a, int r, M2<R> u) {
    switch (r) {
#define C1(B) case B: if constexpr (B < RB) a = app_dense1<R, (1 << RB), B>(a, u); break;
        TCNG_SINGLES(C1)
#undef C1
        default: break;
    }
    return a;
}
template <typename R, int RB>
__device__ __forceinline__ Regs<R, (1 << RB)> cx_at(Regs<R, (1 << RB)> a, int rt, int rc, int tb) {
    switch (rt) {
#define C1(B) case B: if constexpr (B < RB) a = app_cx<R, (1 << RB), B>(a, rc, tb); break;
        TCNG_SINGLES(C1)
#undef C1
        default: break;
    }
    return a;
}
template <typename R, int RB>
__device__ __forceinline__ Regs<R, (1 << RB)> dense2_at(Regs<R, (1 << RB)> a, int r0, int r1, M4<R> u) {
    switch (r0 * 8 + r1) {
#define C2(B0, B1) case B0 * 8 + B1: if constexpr (B0 < RB && B1 < RB) a = app_dense2<R, (1 << RB), B0, B1>(a, u); break;
        TCNG_PAIRS(C2)
#undef C2
        default: break;
    }
    return a;
}
template <typename R, int RB>
__device__ __forceinline__ Regs<R, (1 << RB)> real1_at(Regs<R, (1 << RB)> a, int r, R u0, R u1, R u2, R u3) {
    switch (r) {
#define C1(B) case B: if constexpr (B < RB) a = app_real1<R, (1 << RB), B>(a, u0, u1, u2, u3); break;
        TCNG_SINGLES(C1)
#undef C1
        default: break;
    }
    return a;
}
template <typename R, int RB>
__device__ __forceinline__ Regs<R, (1 << RB)> rx_at(Regs<R, (1 << RB)> a, int r, R c, R s) {
    switch (r) {
#define C1(B) case B: if constexpr (B < RB) a = app_rx<R, (1 << RB), B>(a, c, s); break;
        TCNG_SINGLES(C1)
#undef C1
        default: break;
    }
    return a;
}
template <typename R, int RB>
__device__ __forceinline__ Regs<R, (1 << RB)> diag1r_at(Regs<R, (1 << RB)> a, int r, cx<R> d0, cx<R> d1) {
    switch (r) {
#define C1(B) case B: if constexpr (B < RB) a = app_diag1r<R, (1 << RB), B>(a, d0, d1); break;
        TCNG_SINGLES(C1)
#undef C1
        default: break;
    }
    return a;
}
template <typename R, int RB>
__device__ __forceinline__ Regs<R, (1 << RB)> ry_lift_at(Regs<R, (1 << RB)> a, int r, Lift<R> L) {
    switch (r) {
#define C1(B) case B: if constexpr (B < RB) a = app_ry_lift<R, (1 << RB), B>(a, L); break;
        TCNG_SINGLES(C1)
#undef C1
        default: break;
    }
    return a;
}
template <typename R, int RB>
__device__ __forceinline__ Regs<R, (1 << RB)> rx_lift_at(Regs<R, (1 << RB)> a, int r, Lift<R> L) {
    switch (r) {
#define C1(B) case B: if constexpr (B < RB) a = app_rx_lift<R, (1 << RB), B>(a, L); break;
        TCNG_SINGLES(C1)
#undef C1
        default: break;
    }
    return a;
}
template <typename R, int RB>
__device__ __forceinline__ Regs<R, (1 << RB)> rz_lift_at(Regs<R, (1 << RB)> a, int r, Lift<R> L) {
    switch (r) {
#define C1(B) case B: if constexpr (B < RB) a = app_rz_lift<R, (1 << RB), B>(a, L); break;
        TCNG_SINGLES(C1)
#undef C1
        default: break;
    }
    return a;
}
template <typename R, int RB>
__device__ __forceinline__ R grad_rz_at(int r, Regs<R, (1 << RB)> l, Regs<R, (1 << RB)> p) {
    R g = R(0);
    switch (r) {
#define C1(B) case B: if constexpr (B < RB) g = grad_rz<R, (1 << RB), B>(l, p); break;
        TCNG_SINGLES(C1)
#undef C1
        default: break;
    }
    return g;
}
template <typename R, int RB>
__device__ __forceinline__ Regs<R, (1 << RB)> cxr_at(Regs<R, (1 << RB)> a, int rt, int rc) {
    switch (rt * 8 + rc) {
#define C2(B0, B1) case B0 * 8 + B1: if constexpr (B0 < RB && B1 < RB) a = app_cxr<R, (1 << RB), B0, B1>(a); break;
        TCNG_PAIRS(C2)
#undef C2
        default: break;
    }
    return a;
}
template <typename R, int RB>
__device__ __forceinline__ Regs<R, (1 << RB)> fsim_at(Regs<R, (1 << RB)> a, int r0, int r1, R c, R s, cx<R> ph) {
    switch (r0 * 8 + r1) {
#define C2(B0, B1) case B0 * 8 + B1: if constexpr (B0 < RB && B1 < RB) a = app_fsim<R, (1 << RB), B0, B1>(a, c, s, ph); break;
        TCNG_PAIRS(C2)
#undef C2
        default: break;
    }
    return a;
}
template <typename R, int RB>
__device__ __forceinline__ R grad_rot1_at(int kind, int r, Regs<R, (1 << RB)> l, Regs<R, (1 << RB)> p) {
    R g = R(0);
    switch (r) {
#define C1(B) case B: if constexpr (B < RB) g = grad_rot1<R, (1 << RB), B>(kind, l, p); break;
        TCNG_SINGLES(C1)
#undef C1
        default: break;
    }
    return g;
}
template <typename R, int RB>
__device__ __forceinline__ void grad_fsim_at(int r0, int r1, Regs<R, (1 << RB)> l, Regs<R, (1 << RB)> p, R& gt,
                                             R& gp) {
    gt = R(0);
    gp = R(0);
    switch (r0 * 8 + r1) {
#define C2(B0, B1) case B0 * 8 + B1: if constexpr (B0 < RB && B1 < RB) grad_fsim<R, (1 << RB), B0, B1>(l, p, gt, gp); break;
        TCNG_PAIRS(C2)
#undef C2
        default: break;
    }
}
template <typename R, int RB>
__device__ __forceinline__ void cot_u2_at(int r0, int r1, Regs<R, (1 << RB)> l, Regs<R, (1 << RB)> f, int a, int b,
                                          R& re, R& im) {
    re = R(0);
    im = R(0);
    switch (r0 * 8 + r1) {
#define C2(B0, B1) case B0 * 8 + B1: if constexpr (B0 < RB && B1 < RB) cot_u2<R, (1 << RB), B0, B1>(l, f, a, b, re, im); break;
        TCNG_PAIRS(C2)
#undef C2
        default: break;
    }
}

// apply one op (forward, or its inverse when INV) to the register block;
// om: the op's matrix entries for this batch member (k_build_ops)
// RY, RX and RZ go through shear rotations and toggle `flip` (one sign per
// state, see lift_of).
template <typename R, int RB, bool INV>
__device__ __forceinline__ Regs<R, (1 << RB)> apply_op(Regs<R, (1 << RB)> a, const Op& op, uint32_t tpart,
                                                      cptr<cx<R>> om, bool& flip) {
    const int tb0 = op.lb0 >= 0 ? int((tpart >> op.lb0) & 1) : 0;
    const int tb1 = op.lb1 >= 0 ? int((tpart >> op.lb1) & 1) : 0;
    if (op.kind == K_RY) {
        const R c = om[0].re, s = om[2].re;
        return ry_lift_at<R, RB>(a, op.r0, lift_of<R>(c, INV ? -s : s, flip));
    }
    if (op.kind == K_RX) {
        const R c = om[0].re, s = -om[1].im;
        return rx_lift_at<R, RB>(a, op.r0, lift_of<R>(c, INV ? -s : s, flip));
    }
    if (op.kind == K_RZ) {
        // om[1] = c + i s: the phase of |1>
        const R c = om[1].re, s = om[1].im;
        const Lift<R> L = lift_of<R>(c, INV ? -s : s, flip);
        if (op.r0 >= 0) return rz_lift_at<R, RB>(a, op.r0, L);
        const R sg = tb0 ? R(1) : R(-1);
        return app_phase_lift<R, (1 << RB)>(a, Lift<R>{sg * L.t, sg * L.s});
    }
    switch (op.type) {
        case OP_DENSE1: {
            M2<R> u;
#pragma unroll
            for (int i = 0; i < 4; ++i) u.e[i] = om[i];
            if (INV) dagger_inplace<R, 2>(u.e);
            a = dense1_at<R, RB>(a, op.r0, u);
            break;
        }
        case OP_REAL1: {
            // real orthogonal: the inverse is the transpose
            const R u0 = om[0].re, u1 = om[1].re, u2 = om[2].re, u3 = om[3].re;
            a = INV ? real1_at<R, RB>(a, op.r0, u0, u2, u1, u3) : real1_at<R, RB>(a, op.r0, u0, u1, u2, u3);
            break;
        }
        case OP_RX: {
            const R c = om[0].re, s = -om[1].im;
            a = rx_at<R, RB>(a, op.r0, c, INV ? -s : s);
            break;
        }
        case OP_FSIM: {
            const R c = om[5].re, s = -om[6].im;
            const cx<R> w = om[15];
            const cx<R> ph = INV ? conj(w) : w;
            a = fsim_at<R, RB>(a, op.r0, op.r1, c, INV ? -s : s, ph);
            break;
        }
        case OP_DIAG1: {
            const cx<R> w0 = om[0], w1 = om[1];
            const cx<R> d0 = INV ? conj(w0) : w0;
            const cx<R> d1 = INV ? conj(w1) : w1;
            if (op.r0 >= 0) {
                a = diag1r_at<R, RB>(a, op.r0, d0, d1);
            } else {
                D4<R> d;
                d.e[0] = d0;
                d.e[1] = d1;
                d.e[2] = d.e[3] = d0;
                a = app_diag<R, (1 << RB)>(a, -1, tb0, -1, 0, false, d);
            }
            break;
        }
        case OP_CX:
            if (op.r0 >= 0) a = cxr_at<R, RB>(a, op.r1, op.r0);
            else a = cx_at<R, RB>(a, op.r1, -1, tb0);
            break;
        case OP_DENSE2: {
            M4<R> u;
#pragma unroll
            for (int i = 0; i < 16; ++i) u.e[i] = om[i];
            if (INV) dagger_inplace<R, 4>(u.e);
            a = dense2_at<R, RB>(a, op.r0, op.r1, u);
            break;
        }
        default: {   // OP_DIAG2
            D4<R> d;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const cx<R> w = om[i];
                d.e[i] = INV ? conj(w) : w;
            }
            a = app_diag<R, (1 << RB)>(a, op.r0, tb0, op.r1, tb1, true, d);
            break;
        }
    }
    return a;
}

// matrix entries of one op (table indexed by gate)
template <typename R>
__device__ __forceinline__ void build_op(const Op& op, const R* prm, const cx<R>* cm, cx<R>* table) {
    cx<R>* dst = table + size_t(op.gate) * 16;
    cx<R> u[16];
    switch (op.type) {
        case OP_DENSE1: case OP_REAL1: case OP_RX: mat1<R>(op.kind, prm, op.p0, cm, op.mat, u); break;
        case OP_DIAG1: diag1<R>(op.kind, prm, op.p0, u); break;
        case OP_DIAG2: diag2<R>(op.kind, prm, op.p0, u); break;
        case OP_DENSE2: case OP_FSIM: mat2<R>(op.kind, prm, op.p0, op.p1, cm, op.mat, u); break;
        default: break;
    }
    int cnt = (op.type == OP_DENSE2 || op.type == OP_FSIM) ? 16 : (op.type == OP_CX ? 0 : 4);
    if (op.kind == K_RY || op.kind == K_RZ) {
        // shear coefficients for the rotation rounds: entry 4 = (t, s), entry 5 = (-1 if the
        // rotation is taken as -R(a - pi), else 1; 0).  RY: cos, sin of a = theta / 2 in
        // u[0], u[2]; RZ: the phase of |1> is u[1] = cos + i sin.
        const R c = op.kind == K_RY ? u[0].re : u[1].re;
        const R sn = op.kind == K_RY ? u[2].re : u[1].im;
        bool flip = false;
        const Lift<R> L = lift_of<R>(c, sn, flip);
        u[4] = {L.t, L.s};
        u[5] = {flip ? R(-1) : R(1), R(0)};
        cnt = 6;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k)
        if (k < cnt) dst[k] = u[k];
}

// matrix entries of every op of a plan for every batch member, computed once
// per evaluation: dense 2x2 (4 entries), diagonals (2 or 4), dense 4x4 (16)
template <typename R>
__global__ void k_build_ops(const Op* __restrict__ ops, int n_ops, const R* __restrict__ params, int64_t pstride,
                            const cx<R>* __restrict__ cm, int64_t batch, cx<R>* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= int64_t(n_ops) * batch) return;
    const int64_t b = i / n_ops;
    const int o = int(i - b * n_ops);
    build_op<R>(ops[o], params ? params + b * pstride : nullptr, cm, out + size_t(b) * n_ops * 16);
}

// the same for an uneven batch: job j covers threads [prefix[j], prefix[j+1])
template <typename R>
__global__ void k_build_ops_multi(const BuildJob* __restrict__ jobs, const int64_t* __restrict__ prefix, int njobs,
                                  int64_t total) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= total) return;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    const BuildJob& B = jobs[lo];
    const int o = int(i - prefix[lo]);
    build_op<R>(B.ops[o], static_cast<const R*>(B.params), static_cast<const cx<R>*>(B.cmats),
                static_cast<cx<R>*>(B.opm));
}

// ---------------------------------------------------------------------------
// forward pass: one tile per workgroup.  Waves beyond the job's tile size
// (2^(m - RB) threads; jobs of one launch may differ in m) take part in the
// barriers only.
// ---------------------------------------------------------------------------
template <typename R, int RB>
__global__ void __launch_bounds__((MaxThreads<R, RB>::value))
k_tile_fwd(const JobList jl, const Job single) {
    __shared__ cx<R> lds[Tile<R>::ELEMS];
    int64_t local;
    const Job J = load_job(jl, single, blockIdx.x, local);
    cptr<Pass> P = as_const(J.passes) + jl.step;
    const PassInfo pi = read_pass(P);
    const int nt = 1 << (pi.m - RB);
    const int t = threadIdx.x;
    // nt is a multiple of 64: whole waves are active or idle
    const bool active = uniform(t >> 6) < (nt >> 6);
    const int64_t b = local / J.tiles;
    const uint64_t tile = uint64_t(local - b * J.tiles);
    const int n = J.n;
    gptr<cx<R>> psi = as_global(static_cast<cx<R>*>(J.state)) + b * J.stride;
    cptr<cx<R>> om = as_const(static_cast<const cx<R>*>(J.opm)) + size_t(b) * J.n_gates * 16;
    cptr<Phase> phases = as_const(J.phases);
    cptr<Op> ops = as_const(J.ops);
    const uint64_t base = tile_base(tile, pi.tmask, n);
    const int f_end = P->phase_end;

    if (active) tile_load<R, RB>(lds, psi, base, pi, t, nt);
    __syncthreads();
    bool flip = false;
    for (int f = P->phase_begin; f < f_end; ++f) {
        if (active) {
            const PhaseMap pm = phase_map<RB>(phases + f, t, pi.m);
            Regs<R, (1 << RB)> a = regs_from_lds<R, RB>(lds, pm);
            const int o_end = phases[f].op_end;
            for (int o = phases[f].op_begin; o < o_end; ++o) {
                const Op op = ops[o];
                a = apply_op<R, RB, false>(a, op, pm.tpart, om + 16 * op.gate, flip);
            }
            regs_to_lds<R, RB>(a, lds, pm);
        }
        __syncthreads();
    }
    if (active) tile_store<R, RB>(lds, psi, base, pi, t, nt, flip);
}

// accumulate a thread's gradient partial into the wave's slot (float64).  The
// slot is the wave's own, so the add is an LDS atomic without return: the wave
// does not wait for a read of the slot, and the adds of one wave still land in
// program order (the sum's order does not depend on scheduling).
template <typename R>
__device__ __forceinline__ void red_add(double* red, int idx, R v, int lane) {
    // (complex64: the wave's 64 lanes summed in float, each lane holding a
    // float sum of its own amplitudes' products already; waves and tiles in float64)
    const double s = double(wave_sum(v));
    if (lane == 0) (void)__hip_atomic_fetch_add(red + idx, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// ---------------------------------------------------------------------------
// reverse pass (pass n_passes - 1 - step): psi and lambda, gradient slots
// accumulated per wave in LDS; `wgs` workgroups per member loop over the tiles
// ---------------------------------------------------------------------------
template <typename R, int RB>
__global__ void __launch_bounds__((MaxThreads<R, RB>::value))
k_tile_rev(const JobList jl, const Job single) {
    __shared__ cx<R> lds[Tile<R>::ELEMS];
    __shared__ double red[RED_SLOTS * (NTHREADS / 64)];
    using Blk = Regs<R, (1 << RB)>;
    int64_t local;
    const Job J = load_job(jl, single, blockIdx.x, local);
    const int pidx = J.n_passes - 1 - jl.step;
    cptr<Pass> P = as_const(J.rpasses) + pidx;
    const PassInfo pi = read_pass(P);
    const int nt = 1 << (pi.m - RB);
    const int nwaves = nt >> 6;
    const int t = threadIdx.x;
    const int wave = uniform(t >> 6), lane = t & 63;
    const bool active = wave < nwaves;
    const int wgs = J.wgs;
    const int64_t b = local / wgs;
    const int wg = int(local - b * wgs);
    const int n = J.n;
    gptr<cx<R>> psi = as_global(static_cast<cx<R>*>(J.state)) + b * J.stride;
    gptr<cx<R>> lam = as_global(static_cast<cx<R>*>(J.costate)) + b * J.stride;
    cptr<cx<R>> om = as_const(static_cast<const cx<R>*>(J.opm)) + size_t(b) * J.n_gates * 16;
    cptr<Phase> rphases = as_const(J.rphases);
    cptr<Op> rops = as_const(J.rops);
    const int nslots = P->n_slots;
    const int f_begin = P->phase_begin, f_last = P->phase_end - 1;

    for (int i = t; i < nslots * nwaves; i += blockDim.x) red[i] = 0.0;
    // (the first __syncthreads below orders these writes before any accumulation)

    for (int64_t tile = wg; tile < J.tiles; tile += wgs) {
        const uint64_t base = tile_base(uint64_t(tile), pi.tmask, n);
        // phases run backwards; psi and lambda take turns in the one LDS tile
        int f = f_last;
        PhaseMap pm = phase_map<RB>(rphases + f, t, pi.m);
        Blk ps, la;
        bool flip = false, flip_l = false;   // equal: psi and lambda see the same ops
        __syncthreads();
        if (active) tile_load<R, RB>(lds, psi, base, pi, t, nt);
        __syncthreads();
        if (active) ps = regs_from_lds<R, RB>(lds, pm);
        __syncthreads();
        if (active) tile_load<R, RB>(lds, lam, base, pi, t, nt);
        __syncthreads();
        if (active) la = regs_from_lds<R, RB>(lds, pm);
        for (;;) {
            if (active) {
                const int o_begin = rphases[f].op_begin;
                for (int o = rphases[f].op_end - 1; o >= o_begin; --o) {
                    const Op op = rops[o];
                    cptr<cx<R>> m16 = om + 16 * op.gate;
                    const int slot = op.slot * nwaves + wave;
                    if (op.slot >= 0 && op.kind != K_U2) {
                        if (op.kind == K_RX || op.kind == K_RY) {
                            red_add(red, slot, grad_rot1_at<R, RB>(op.kind, op.r0, la, ps), lane);
                        } else if (op.kind == K_FSIM) {
                            R gt, gp;
                            grad_fsim_at<R, RB>(op.r0, op.r1, la, ps, gt, gp);
                            red_add(red, slot, gt, lane);
                            red_add(red, slot + nwaves, gp, lane);
                        } else if (op.kind == K_RZ) {
                            R g;
                            if (op.r0 >= 0) {
                                g = grad_rz_at<R, RB>(op.r0, la, ps);
                            } else {
                                const R v = sum_im_conj<R, (1 << RB)>(la, ps);
                                g = ((pm.tpart >> op.lb0) & 1) ? -v : v;
                            }
                            red_add(red, slot, g, lane);
                        } else {                            // RZZ
                            const int tb0 = op.lb0 >= 0 ? int((pm.tpart >> op.lb0) & 1) : 0;
                            const int tb1 = op.lb1 >= 0 ? int((pm.tpart >> op.lb1) & 1) : 0;
                            red_add(red, slot,
                                    grad_zdiag<R, (1 << RB)>(la, ps, op.r0, tb0, op.type == OP_DIAG2 ? op.r1 : -1,
                                                             op.type == OP_DIAG2 ? tb1 : 0),
                                    lane);
                        }
                    }
                    ps = apply_op<R, RB, true>(ps, op, pm.tpart, m16, flip);
                    if (op.kind == K_U2 && op.slot >= 0) {
#pragma unroll
                        for (int e = 0; e < 16; ++e) {
                            R gr, gi;
                            cot_u2_at<R, RB>(op.r0, op.r1, la, ps, e >> 2, e & 3, gr, gi);
                            red_add(red, slot + 2 * e * nwaves, gr, lane);
                            red_add(red, slot + (2 * e + 1) * nwaves, gi, lane);
                        }
                    }
                    la = apply_op<R, RB, true>(la, op, pm.tpart, m16, flip_l);
                }
            }
            if (f == f_begin) break;
            // hand both blocks to the previous phase's register assignment
            const PhaseMap pn = phase_map<RB>(rphases + (f - 1), t, pi.m);
            __syncthreads();
            if (active) regs_to_lds<R, RB>(ps, lds, pm);
            __syncthreads();
            if (active) ps = regs_from_lds<R, RB>(lds, pn);
            __syncthreads();
            if (active) regs_to_lds<R, RB>(la, lds, pm);
            __syncthreads();
            if (active) la = regs_from_lds<R, RB>(lds, pn);
            pm = pn;
            --f;
        }
        __syncthreads();
        if (active) regs_to_lds<R, RB>(ps, lds, pm);
        __syncthreads();
        if (active) tile_store<R, RB>(lds, psi, base, pi, t, nt, flip);
        __syncthreads();
        if (active) regs_to_lds<R, RB>(la, lds, pm);
        __syncthreads();
        if (active) tile_store<R, RB>(lds, lam, base, pi, t, nt, flip_l);
    }
    __syncthreads();
    double* part = J.part + size_t(b) * J.total_slots * wgs;
    for (int s = t; s < nslots; s += blockDim.x) {
        double v = 0.0;
        for (int w = 0; w < nwaves; ++w) v += red[s * nwaves + w];
        part[size_t(P->slot_base + s) * wgs + wg] = v;
    }
}

// ---------------------------------------------------------------------------
// rounds (complex64: QR = 4 or 5 register bits; complex128: QR = 3 or 4; see QPhase)
// ---------------------------------------------------------------------------
// `pin` passes a value through an empty asm statement: the compiler cannot
// hoist what is computed from it out of the loop it sits in, nor share it
// between two uses (shared or hoisted, the LDS and global addresses of a
// tile's elements stay live across the whole sweep, and the reverse sweep
// needs 370 registers); it costs no instruction.
__device__ __forceinline__ uint64_t pin(uint64_t v) {
    uint32_t lo = uint32_t(v), hi = uint32_t(v >> 32);
    asm volatile("" : "+v"(lo), "+v"(hi));
    return (uint64_t(hi) << 32) | lo;
}
__device__ __forceinline__ uint32_t pin(uint32_t v) {
    asm volatile("" : "+v"(v));
    return v;
}

template <typename R, int QR>
using QBlk = Regs<R, (1 << QR)>;

// register bit B of a block of QR bits, clamped for the branches that only
// blocks of more than B bits take
template <int B, int QR>
constexpr int qb() { return B < QR ? B : 0; }

// tile bits of the rounds kernels (64 KiB of LDS): 13 (complex64), 12 (complex128)
template <typename R>
constexpr int q_tile_bits() { return sizeof(R) == 4 ? 13 : 12; }

// a phase's register map: the LDS positions of the thread's part of the local
// index and of its registers, in the layout before the phase (plain) and
// after it (through the phase's permutation C)
template <int QR>
struct QMap {
    uint32_t tsw, ctsw;              // A_before(tpart), A_after(C(tpart))
    uint32_t rsw[QR], crsw[QR];      // A_before(e_R[i]), A_after(C(e_R[i])) (uniform)
};

template <int QR>
__device__ __forceinline__ QMap<QR> qmap(cptr<QPhase> F, int t, int m) {
    QMap<QR> q;
    const uint32_t rmask = uint32_t(F->rmask);
#pragma unroll
    for (int i = 0; i < QR; ++i) {
        q.rsw[i] = uint32_t(F->ruimg[i]);
        q.crsw[i] = uint32_t(F->rimg[i]);
    }
    // the thread's bits fill the non-register local bits in increasing order:
    // unrolled over the local bits, with uniform control and lane masks, so the
    // images' scalar loads are independent (a loop with a lane-dependent branch
    // around each load serialised them, a scalar load's latency per bit)
    uint32_t tp = 0, ct = 0;
    const uint32_t tt = pin(uint32_t(t));   // (the masks are formed anew per phase, not kept live)
#pragma unroll
    for (int b = 0; b < MAX_TILE_BITS; ++b) {
        if (b >= m || ((rmask >> b) & 1)) continue;
        const int k = __popc(~rmask & ((1u << b) - 1u));   // the thread bit that fills local bit b
        const uint32_t msk = 0u - ((tt >> k) & 1u);
        tp ^= uint32_t(F->uimg[b]) & msk;
        ct ^= uint32_t(F->cimg[b]) & msk;
    }
    q.tsw = tp;
    q.ctsw = ct;
    return q;
}

// LDS position of register j: through C (mapped) or not
template <bool MAPPED, int QR>
__device__ __forceinline__ uint32_t qaddr(const QMap<QR>& q, int j) {
    uint32_t a = MAPPED ? q.ctsw : q.tsw;
#pragma unroll
    for (int i = 0; i < QR; ++i)
        if ((j >> i) & 1) a ^= MAPPED ? q.crsw[i] : q.rsw[i];
    return a;
}

// (each call forms its addresses anew: shared between calls, the compiler
// keeps them all live in registers across the sweep)
template <bool MAPPED, typename R, int QR>
__device__ __forceinline__ QBlk<R, QR> q_read(const cx<R>* lds, QMap<QR> q) {
    q.tsw = pin(q.tsw);
    q.ctsw = pin(q.ctsw);
    QBlk<R, QR> a;
#pragma unroll
    for (int j = 0; j < (1 << QR); ++j) a.v[j] = lds[qaddr<MAPPED>(q, j)];
    return a;
}
template <bool MAPPED, typename R, int QR>
__device__ __forceinline__ void q_write(cx<R>* lds, const QBlk<R, QR>& a, QMap<QR> q) {
    q.tsw = pin(q.tsw);
    q.ctsw = pin(q.ctsw);
#pragma unroll
    for (int j = 0; j < (1 << QR); ++j) lds[qaddr<MAPPED>(q, j)] = a.v[j];
}

// Coefficients of a step, one block per (member, step) written once per
// evaluation by k_rounds_coef, read in place with scalar loads (no round trip
// per gate): c[0..9] = RY shear t x5, s x5 (an absent gate: t = s = 0);
// c[10] = -1 if an odd number of the step's RY are taken as -R(a - pi), else 1;
// c[16 + 2j], c[17 + 2j] = cos, sin of the phase of register amplitude j
// (j < 2^QR) under the step's RZ round, the product over register bits b of
// e^{-i a_b / 2} (bit b of j clear) or e^{+i a_b / 2} (set).
constexpr int QCOEF = 16 + 2 * (1 << QREG);
constexpr int QPH = 16;   // first phase entry

template <bool INV, int QR, typename R, typename CP>
__device__ __forceinline__ QBlk<R, QR> q_ry_round(QBlk<R, QR> a, CP c) {
    constexpr int NB = 1 << QR;
    const R sg = INV ? R(-1) : R(1);
    a = app_ry_lift<R, NB, 0>(a, Lift<R>{sg * c[0], sg * c[5]});
    a = app_ry_lift<R, NB, 1>(a, Lift<R>{sg * c[1], sg * c[6]});
    a = app_ry_lift<R, NB, 2>(a, Lift<R>{sg * c[2], sg * c[7]});
    if constexpr (QR > 3) a = app_ry_lift<R, NB, qb<3, QR>()>(a, Lift<R>{sg * c[3], sg * c[8]});
    if constexpr (QR > 4) a = app_ry_lift<R, NB, qb<4, QR>()>(a, Lift<R>{sg * c[4], sg * c[9]});
    return a;
}
// fSim rounds: pair slot k of a step has [cos t, sin t, Re e^{-ip}, Im e^{-ip}]
// in c[4k .. 4k + 3] (an absent gate: 1, 0, 1, 0, the identity); the inverse
// negates sin t and Im e^{-ip}.  Round A: slots 0, 1 on register bits (0,1),
// (2,3); round B: slots 2, 3 on (1,2), (3,4).
template <bool INV, int QR, typename R>
__device__ __forceinline__ QBlk<R, QR> q_fs_round_a(QBlk<R, QR> a, const R* c) {
    constexpr int NB = 1 << QR;
    const R sg = INV ? R(-1) : R(1);
    a = app_fsim<R, NB, 0, 1>(a, c[0], sg * c[1], cx<R>{c[2], sg * c[3]});
    if constexpr (QR > 3) a = app_fsim<R, NB, 2, qb<3, QR>()>(a, c[4], sg * c[5], cx<R>{c[6], sg * c[7]});
    return a;
}
template <bool INV, int QR, typename R>
__device__ __forceinline__ QBlk<R, QR> q_fs_round_b(QBlk<R, QR> a, const R* c) {
    constexpr int NB = 1 << QR;
    const R sg = INV ? R(-1) : R(1);
    a = app_fsim<R, NB, 1, 2>(a, c[8], sg * c[9], cx<R>{c[10], sg * c[11]});
    if constexpr (QR > 4) a = app_fsim<R, NB, qb<3, QR>(), qb<4, QR>()>(a, c[12], sg * c[13], cx<R>{c[14], sg * c[15]});
    return a;
}

// reverse sweep, one fSim gate on register bits (B0, B1): its (theta, phi)
// derivative partials at the current point, then the inverse on psi and lambda
template <int QR, int B0, int B1, typename R, typename CP>
__device__ __forceinline__ void fs_unapply(QBlk<R, QR>& ps, QBlk<R, QR>& la, CP c, R& gt, R& gp) {
    constexpr int NB = 1 << QR;
    grad_fsim<R, NB, B0, B1>(la, ps, gt, gp);
    ps = app_fsim<R, NB, B0, B1>(ps, c[0], -c[1], cx<R>{c[2], -c[3]});
    la = app_fsim<R, NB, B0, B1>(la, c[0], -c[1], cx<R>{c[2], -c[3]});
}

// Hadamard on the register bits set in mask (uniform), the others unchanged
template <int QR, typename R>
__device__ __forceinline__ QBlk<R, QR> q_h_round(QBlk<R, QR> a, uint32_t mask) {
    constexpr int NB = 1 << QR;
    const R r = R(0.70710678118654752440);
#pragma unroll
    for (int b = 0; b < QR; ++b) {
        const bool on = (mask >> b) & 1;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            if (j & (1 << b)) continue;
            const cx<R> x0 = a.v[j], x1 = a.v[j | (1 << b)];
            const cx<R> y0 = {r * (x0.re + x1.re), r * (x0.im + x1.im)};
            const cx<R> y1 = {r * (x0.re - x1.re), r * (x0.im - x1.im)};
            // (per component: a select of whole complex values goes through scratch for double)
            a.v[j].re = on ? y0.re : x0.re;
            a.v[j].im = on ? y0.im : x0.im;
            a.v[j | (1 << b)].re = on ? y1.re : x1.re;
            a.v[j | (1 << b)].im = on ? y1.im : x1.im;
        }
    }
    return a;
}

template <typename R>
struct QCoef {
    R c[QCOEF];
};

// Tile addressing of the rounds.  A thread's 2^QR amplitudes are VN = 2
// (complex64) or 1 (complex128) amplitudes per 16-byte access: element it of
// thread t is local index it * VN nt + VN t (+ k, k < VN).  The bits of it are
// the top EB = QR - log2(VN) local bits, so its global offset is a
// compile-time sum of their images hb[k] (per pass, uniform), and the
// thread's part off_t is computed once (and pinned per use).
template <typename R, int QR>
struct QTileAddr {
    static constexpr int VN = V16<R>::N;
    static constexpr int EB = QR - (VN == 2 ? 1 : 0);
    uint64_t hb[EB];       // global offsets of the element-index bits (uniform)
    uint64_t off_t;        // the thread's part
    uint32_t lsw_t;        // swz(VN t)
    uint32_t lhb[EB];      // swz of the element-index bits (uniform)
};

template <typename R, int QR>
__device__ __forceinline__ QTileAddr<R, QR> q_tile_addr(const PassInfo& pi, int t) {
    using A_t = QTileAddr<R, QR>;
    A_t A;
    const int b0 = pi.m - A_t::EB;   // first local bit of the element index
#pragma unroll
    for (int k = 0; k < A_t::EB; ++k) {
        int q = b0 + k;
#pragma unroll
        for (int i = 0; i < MAX_TILE_BITS; ++i)
            if (i == b0 + k) q = pi.lq[i];
        A.hb[k] = uint64_t(1) << q;
        A.lhb[k] = swz(1u << (b0 + k));
    }
    A.off_t = loc2glob(uint32_t(t * A_t::VN), pi.lo, pi.m, pi.lq);
    A.lsw_t = swz(uint32_t(t * A_t::VN));
    return A;
}

// (it is a constant once the loops over elements are unrolled: the selects fold)
template <typename R, int QR>
__device__ __forceinline__ uint64_t q_goff(const QTileAddr<R, QR>& A, int it) {
    uint64_t g = 0;
#pragma unroll
    for (int k = 0; k < QTileAddr<R, QR>::EB; ++k)
        if ((it >> k) & 1) g += A.hb[k];
    return g;
}
template <typename R, int QR>
__device__ __forceinline__ uint32_t q_loff(const QTileAddr<R, QR>& A, int it) {
    uint32_t a = 0;
#pragma unroll
    for (int k = 0; k < QTileAddr<R, QR>::EB; ++k)
        if ((it >> k) & 1) a ^= A.lhb[k];
    return a;
}

// HBM -> registers (the loads stay in flight until the registers are used)
// and registers -> LDS, separately, so that a tile can be fetched while
// another one is processed
template <typename R, int QR>
struct QTileRegs {
    cx<R> v[1 << QR];
};

template <typename R, int QR>
__device__ __forceinline__ QTileRegs<R, QR> q_tile_fetch(gptr<const cx<R>> psi, uint64_t base,
                                                         const QTileAddr<R, QR>& A) {
    constexpr int VN = V16<R>::N;
    const gptr<const cx<R>> p = psi + pin(A.off_t);
    QTileRegs<R, QR> r;
#pragma unroll
    for (int it = 0; it < (1 << QR) / VN; ++it) V16<R>::load(p + (base + q_goff<R, QR>(A, it)), &r.v[it * VN]);
    return r;
}

// (swz leaves bit 0 alone: the VN amplitudes of an access stay adjacent)
template <typename R, int QR>
__device__ __forceinline__ void q_tile_put(cx<R>* lds, const QTileRegs<R, QR>& r, const QTileAddr<R, QR>& A) {
    constexpr int VN = V16<R>::N;
    const uint32_t lt = pin(A.lsw_t);
#pragma unroll
    for (int it = 0; it < (1 << QR) / VN; ++it) {
        const uint32_t e = lt ^ q_loff<R, QR>(A, it);
#pragma unroll
        for (int k = 0; k < VN; ++k) lds[e ^ uint32_t(k)] = r.v[it * VN + k];
    }
}

template <typename R, int QR>
__device__ __forceinline__ void q_tile_store(const cx<R>* lds, gptr<cx<R>> psi, uint64_t base,
                                             const QTileAddr<R, QR>& A, bool flip) {
    constexpr int VN = V16<R>::N;
    const gptr<cx<R>> p = psi + pin(A.off_t);
    const uint32_t lt = pin(A.lsw_t);
    const R sg = flip ? R(-1) : R(1);
#pragma unroll
    for (int it = 0; it < (1 << QR) / VN; ++it) {
        const uint32_t e = lt ^ q_loff<R, QR>(A, it);
        cx<R> v[VN];
#pragma unroll
        for (int k = 0; k < VN; ++k) {
            v[k] = lds[e ^ uint32_t(k)];
            if (flip) v[k] = {sg * v[k].re, sg * v[k].im};
        }
        V16<R>::store(p + (base + q_goff<R, QR>(A, it)), v);
    }
}

// a round's derivative partials into their slots (absent gates have none)
template <int QR, typename R>
__device__ __forceinline__ void q_red(double* red, const int32_t* slot, int nwaves, int wave, int lane,
                                      const R* g) {
#pragma unroll
    for (int i = 0; i < QR; ++i)
        if (slot[i] >= 0) red_add(red, slot[i] * nwaves + wave, g[i], lane);
}

// an fSim round's (theta, phi) partials into their slots (slot, slot + 1)
template <int NS, typename R>
__device__ __forceinline__ void q_red_fs(double* red, const int32_t* slot, int nwaves, int wave, int lane,
                                         const R* gt, const R* gp) {
#pragma unroll
    for (int i = 0; i < NS; ++i)
        if (slot[i] >= 0) {
            red_add(red, slot[i] * nwaves + wave, gt[i], lane);
            red_add(red, (slot[i] + 1) * nwaves + wave, gp[i], lane);
        }
}

// forward: `wgs` workgroups per member loop over the tiles; the next tile's
// loads are in flight while the current tile's phases run
template <typename R, int QR, bool FS>
__global__ void __launch_bounds__(1 << (q_tile_bits<R>() - QR)) k_rounds_fwd(const JobList jl, const Job single,
                                                                           int wgs) {
    __shared__ cx<R> lds[Tile<R>::ELEMS];
    int64_t local;
    const Job J = load_job(jl, single, blockIdx.x, local);
    cptr<Pass> P = as_const(J.passes) + jl.step;
    const PassInfo pi = read_pass(P);
    const QPass Q = as_const(J.qpasses)[jl.step];
    // the launch has exactly 2^(m - QR) threads: every wave is active
    const int nt = 1 << (pi.m - QR);
    const int t = threadIdx.x;
    const int64_t b = local / wgs;
    const int wg = int(local - b * wgs);
    gptr<cx<R>> psi = as_global(static_cast<cx<R>*>(J.state)) + b * J.stride;
    cptr<QPhase> phases = as_const(J.qphases);
    cptr<QCoef<R>> coef = as_const(reinterpret_cast<const QCoef<R>*>(J.qcoef)) + size_t(b) * J.qsteps_all;

    const QTileAddr<R, QR> A = q_tile_addr<R, QR>(pi, t);
    QTileRegs<R, QR> nx;
    if (wg < J.tiles) nx = q_tile_fetch<R, QR>(psi, tile_base(uint64_t(wg), pi.tmask, J.n), A);
    for (int64_t tile = wg; tile < J.tiles; tile += wgs) {
        const uint64_t base = tile_base(uint64_t(tile), pi.tmask, J.n);
        __syncthreads();   // the previous tile's stores have read the LDS
        q_tile_put<R, QR>(lds, nx, A);
        if (tile + wgs < J.tiles) nx = q_tile_fetch<R, QR>(psi, tile_base(uint64_t(tile + wgs), pi.tmask, J.n), A);
        __syncthreads();
        bool flip = false;
        for (int f = Q.phase_begin; f < Q.phase_end; ++f) {
            cptr<QPhase> F = phases + f;
            const QMap<QR> q = qmap<QR>(F, t, pi.m);
            QBlk<R, QR> a = q_read<false>(lds, q);
            if constexpr (FS) {
                const uint32_t hm = uint32_t(F->hmask);
                if (hm) a = q_h_round<QR>(a, hm);
            }
            const int s_end = F->step_end;
            for (int s = F->step_begin; s < s_end; ++s) {
                if constexpr (FS) {   // absent gates skipped; coefficients read in place
                    const QStep S = as_const(J.qsteps)[s];
                    cptr<R> c = &coef[s].c[0];
                    if (S.ry[0] >= 0) a = app_fsim<R, (1 << QR), 0, 1>(a, c[0], c[1], cx<R>{c[2], c[3]});
                    if constexpr (QR > 3)
                        if (S.ry[1] >= 0)
                            a = app_fsim<R, (1 << QR), 2, qb<3, QR>()>(a, c[4], c[5], cx<R>{c[6], c[7]});
                    if (S.ry[2] >= 0) a = app_fsim<R, (1 << QR), 1, 2>(a, c[8], c[9], cx<R>{c[10], c[11]});
                    if constexpr (QR > 4)
                        if (S.ry[3] >= 0)
                            a = app_fsim<R, (1 << QR), qb<3, QR>(), qb<4, QR>()>(a, c[12], c[13], cx<R>{c[14], c[15]});
                } else {
                    cptr<R> c = &coef[s].c[0];
                    a = q_ry_round<false, QR>(a, c);
                    a = app_phases<false, R, (1 << QR)>(a, c + QPH);
                    flip = flip != (c[10] < R(0));
                }
            }
            __syncthreads();   // the write permutes positions: every read first
            q_write<true>(lds, a, q);   // (into the next layout)
            __syncthreads();
        }
        q_tile_store<R, QR>(lds, psi, base, A, flip);
    }
}

// reverse: phases and steps backwards; each phase reads through C, un-applies
// its rounds (derivatives first: every rotation of a round at the round's
// end point, where all of them commute) and writes without C
template <typename R, int QR, bool FS>
__global__ void __launch_bounds__(1 << (q_tile_bits<R>() - QR)) k_rounds_rev(const JobList jl, const Job single) {
    constexpr int NB = 1 << QR;
    __shared__ cx<R> lds[Tile<R>::ELEMS];
    __shared__ double red[RED_SLOTS * ((1 << (q_tile_bits<R>() - QR)) / 64)];
    int64_t local;
    const Job J = load_job(jl, single, blockIdx.x, local);
    const int pidx = J.n_passes - 1 - jl.step;
    cptr<Pass> P = as_const(J.passes) + pidx;
    const PassInfo pi = read_pass(P);
    const QPass Q = as_const(J.qrpasses)[pidx];
    const int nt = 1 << (pi.m - QR);   // the launch's thread count: every wave is active
    const int nwaves = nt >> 6;
    const int t = threadIdx.x;
    const int wave = uniform(t >> 6), lane = t & 63;
    const int wgs = J.wgs;
    const int64_t b = local / wgs;
    const int wg = int(local - b * wgs);
    gptr<cx<R>> psi = as_global(static_cast<cx<R>*>(J.state)) + b * J.stride;
    gptr<cx<R>> lam = as_global(static_cast<cx<R>*>(J.costate)) + b * J.stride;
    cptr<QPhase> phases = as_const(J.qrphases);
    cptr<QStep> steps = as_const(J.qrsteps);
    cptr<QCoef<R>> coef = as_const(reinterpret_cast<const QCoef<R>*>(J.qcoef)) + size_t(b) * J.qsteps_all + J.qsteps_fwd;
    const int nslots = P->n_slots;

    for (int i = t; i < nslots * nwaves; i += blockDim.x) red[i] = 0.0;
    // (the first __syncthreads below orders these writes before any accumulation)
    const QTileAddr<R, QR> A = q_tile_addr<R, QR>(pi, t);

    for (int64_t tile = wg; tile < J.tiles; tile += wgs) {
        const uint64_t base = tile_base(uint64_t(tile), pi.tmask, J.n);
        int f = Q.phase_end - 1;
        QMap<QR> q = qmap<QR>(phases + f, t, pi.m);
        QBlk<R, QR> ps, la;
        bool flip = false;   // psi and lambda see the same rotations: one sign for both
        {
            // both states' loads in flight together
            const QTileRegs<R, QR> vp = q_tile_fetch<R, QR>(psi, base, A);
            const QTileRegs<R, QR> vl = q_tile_fetch<R, QR>(lam, base, A);
            __syncthreads();
            q_tile_put<R, QR>(lds, vp, A);
            __syncthreads();
            ps = q_read<true>(lds, q);
            __syncthreads();
            q_tile_put<R, QR>(lds, vl, A);
            __syncthreads();
            la = q_read<true>(lds, q);
        }
        for (;;) {
            cptr<QPhase> F = phases + f;
            const int s_begin = F->step_begin;
            for (int s = F->step_end - 1; s >= s_begin; --s) {
                const QStep S = steps[s];
                if constexpr (FS) {
                    cptr<R> c = &coef[s].c[0];
                    // round B, then round A, gate by gate (the gates of a round
                    // act on disjoint pairs and commute, so each one's derivative
                    // is taken just before it is un-applied); absent gates skipped
                    R gt[4], gp[4];
                    if (S.ry[2] >= 0) fs_unapply<QR, 1, 2>(ps, la, c + 8, gt[2], gp[2]);
                    if constexpr (QR > 4)
                        if (S.ry[3] >= 0) fs_unapply<QR, qb<3, QR>(), qb<4, QR>()>(ps, la, c + 12, gt[3], gp[3]);
                    q_red_fs<(QR > 4 ? 2 : 1)>(red, S.sy + 2, nwaves, wave, lane, gt + 2, gp + 2);
                    if (S.ry[0] >= 0) fs_unapply<QR, 0, 1>(ps, la, c, gt[0], gp[0]);
                    if constexpr (QR > 3)
                        if (S.ry[1] >= 0) fs_unapply<QR, 2, qb<3, QR>()>(ps, la, c + 4, gt[1], gp[1]);
                    q_red_fs<(QR > 3 ? 2 : 1)>(red, S.sy, nwaves, wave, lane, gt, gp);
                    continue;
                }
                cptr<R> c = &coef[s].c[0];
                // the round's derivatives first, then the un-apply, then their
                // reductions (which leave the blocks alone)
                R gz[QR], gy[QR];
                grad_rz_all<R, QR>(la, ps, gz);
                ps = app_phases<true, R, NB>(ps, c + QPH);
                la = app_phases<true, R, NB>(la, c + QPH);
                q_red<QR>(red, S.sz, nwaves, wave, lane, gz);
                gy[0] = grad_rot1<R, NB, 0>(K_RY, la, ps);
                gy[1] = grad_rot1<R, NB, 1>(K_RY, la, ps);
                gy[2] = grad_rot1<R, NB, 2>(K_RY, la, ps);
                if constexpr (QR > 3) gy[qb<3, QR>()] = grad_rot1<R, NB, qb<3, QR>()>(K_RY, la, ps);
                if constexpr (QR > 4) gy[qb<4, QR>()] = grad_rot1<R, NB, qb<4, QR>()>(K_RY, la, ps);
                ps = q_ry_round<true, QR>(ps, c);
                la = q_ry_round<true, QR>(la, c);
                flip = flip != (c[10] < R(0));
                q_red<QR>(red, S.sy, nwaves, wave, lane, gy);
            }
            if constexpr (FS) {   // the phase's Hadamards (their own inverses) last
                const uint32_t hm = uint32_t(F->hmask);
                if (hm) {
                    ps = q_h_round<QR>(ps, hm);
                    la = q_h_round<QR>(la, hm);
                }
            }
            if (f == Q.phase_begin) break;
            // hand both blocks to the previous phase: written in plain order,
            // read back through that phase's permutation
            const QMap<QR> qn = qmap<QR>(phases + (f - 1), t, pi.m);
            __syncthreads();
            q_write<false>(lds, ps, q);
            __syncthreads();
            ps = q_read<true>(lds, qn);
            __syncthreads();
            q_write<false>(lds, la, q);
            __syncthreads();
            la = q_read<true>(lds, qn);
            q = qn;
            --f;
        }
        __syncthreads();
        q_write<false>(lds, ps, q);
        __syncthreads();
        q_tile_store<R, QR>(lds, psi, base, A, flip);
        __syncthreads();
        q_write<false>(lds, la, q);
        __syncthreads();
        q_tile_store<R, QR>(lds, lam, base, A, flip);
    }
    __syncthreads();
    double* part = J.part + size_t(b) * J.total_slots * wgs;
    for (int s = t; s < nslots; s += blockDim.x) {
        double v = 0.0;
        for (int w = 0; w < nwaves; ++w) v += red[s * nwaves + w];
        part[size_t(P->slot_base + s) * wgs + wg] = v;
    }
}

// the shear-coefficient blocks of every (member, step): forward steps, then
// reverse steps, from the ops' matrix tables (entries 4 and 5 of RY / RZ)
template <typename R>
__global__ void k_rounds_coef(const QStep* __restrict__ fsteps, int nf, const QStep* __restrict__ rsteps, int nr,
                              const cx<R>* __restrict__ opm, int n_gates, int64_t batch, QCoef<R>* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int per = nf + nr;
    if (i >= int64_t(per) * batch) return;
    const int64_t b = i / per;
    const int s = int(i - b * per);
    const QStep S = s < nf ? fsteps[s] : rsteps[s - nf];
    const cx<R>* om = opm + size_t(b) * n_gates * 16;
    QCoef<R> C;
    if (S.kind == QK_FSIM) {   // the fSim matrix: entry 5 = cos t, entry 6 = -i sin t, entry 15 = e^{-ip}
        for (int k = 0; k < 4; ++k) {
            const int g = S.ry[k];
            C.c[4 * k] = g >= 0 ? om[size_t(g) * 16 + 5].re : R(1);
            C.c[4 * k + 1] = g >= 0 ? -om[size_t(g) * 16 + 6].im : R(0);
            C.c[4 * k + 2] = g >= 0 ? om[size_t(g) * 16 + 15].re : R(1);
            C.c[4 * k + 3] = g >= 0 ? om[size_t(g) * 16 + 15].im : R(0);
        }
        for (int k = 16; k < QCOEF; ++k) C.c[k] = R(0);
        out[i] = C;
        return;
    }
    bool odd = false;
    for (int k = 0; k < QREG; ++k) {
        const int gy = S.ry[k];
        C.c[k] = gy >= 0 ? om[size_t(gy) * 16 + 4].re : R(0);
        C.c[5 + k] = gy >= 0 ? om[size_t(gy) * 16 + 4].im : R(0);
        if (gy >= 0 && om[size_t(gy) * 16 + 5].re < R(0)) odd = !odd;
    }
    C.c[10] = odd ? R(-1) : R(1);
    for (int k = 11; k < QPH; ++k) C.c[k] = R(0);
    // the RZ round's phases: RZ matrix entries 0 = e^{-ia/2}, 1 = e^{+ia/2}
    for (int j = 0; j < (1 << QREG); ++j) {
        cx<R> ph = {R(1), R(0)};
        for (int k = 0; k < QREG; ++k) {
            const int gz = S.rz[k];
            if (gz >= 0) ph = ph * om[size_t(gz) * 16 + ((j >> k) & 1)];
        }
        C.c[QPH + 2 * j] = ph.re;
        C.c[QPH + 2 * j + 1] = ph.im;
    }
    out[i] = C;
}

}  // namespace

template <typename R>
hipError_t launch_build_ops(const DevPlan& dp, int n_ops, const void* params, int64_t pstride, const void* cmats,
                            int64_t batch, void* opm, hipStream_t st) {
    const int64_t work = int64_t(n_ops) * batch;
    if (work == 0) return hipSuccess;
    hipLaunchKernelGGL((k_build_ops<R>), dim3(unsigned((work + 255) / 256)), dim3(256), 0, st, dp.ops, n_ops,
                       static_cast<const R*>(params), pstride, static_cast<const cx<R>*>(cmats), batch,
                       static_cast<cx<R>*>(opm));
    return hipGetLastError();
}

template <typename R, int RB>
hipError_t launch_tile_fwd(const JobList& jl, const Job& single, int64_t blocks, int nthreads, hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_tile_fwd<R, RB>), dim3(unsigned(blocks)), dim3(nthreads), 0, st, jl, single);
    return hipGetLastError();
}

template <typename R, int RB>
hipError_t launch_tile_rev(const JobList& jl, const Job& single, int64_t blocks, int nthreads, hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_tile_rev<R, RB>), dim3(unsigned(blocks)), dim3(nthreads), 0, st, jl, single);
    return hipGetLastError();
}

// nthreads must be 2^(m - qr) for the launched pass's m (single jobs only)
template <typename R>
hipError_t launch_rounds_coef(const QStep* fsteps, int nf, const QStep* rsteps, int nr, const void* opm, int n_gates,
                              int64_t batch, void* out, hipStream_t st) {
    const int64_t work = int64_t(nf + nr) * batch;
    if (work == 0) return hipSuccess;
    hipLaunchKernelGGL((k_rounds_coef<R>), dim3(unsigned((work + 255) / 256)), dim3(256), 0, st, fsteps, nf, rsteps,
                       nr, static_cast<const cx<R>*>(opm), n_gates, batch, static_cast<QCoef<R>*>(out));
    return hipGetLastError();
}

template <typename R>
size_t rounds_coef_bytes(int steps) { return size_t(steps) * sizeof(QCoef<R>); }

// register bits per precision: 4 or 5 (complex64), 3 or 4 (complex128)
template <typename R>
bool rounds_qr_ok(int qr) { return sizeof(R) == 4 ? (qr == 4 || qr == 5) : (qr == 3 || qr == 4); }

// forward: wgs workgroups per member (each loops over tiles), blocks = wgs * batch
template <typename R>
hipError_t launch_rounds_fwd(const JobList& jl, const Job& single, int qr, bool fsim, int wgs, int64_t blocks,
                             int nthreads, hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    if (jl.jobs || !rounds_qr_ok<R>(qr) || nthreads > (1 << (q_tile_bits<R>() - qr)) || nthreads < 64 || wgs < 1)
        return hipErrorInvalidValue;
    const dim3 g = dim3(unsigned(blocks)), b = dim3(unsigned(nthreads));
    if constexpr (sizeof(R) == 4) {
        if (qr == 5 && fsim) hipLaunchKernelGGL((k_rounds_fwd<R, 5, true>), g, b, 0, st, jl, single, wgs);
        else if (qr == 5) hipLaunchKernelGGL((k_rounds_fwd<R, 5, false>), g, b, 0, st, jl, single, wgs);
        else if (fsim) hipLaunchKernelGGL((k_rounds_fwd<R, 4, true>), g, b, 0, st, jl, single, wgs);
        else hipLaunchKernelGGL((k_rounds_fwd<R, 4, false>), g, b, 0, st, jl, single, wgs);
    } else {
        if (qr == 4 && fsim) hipLaunchKernelGGL((k_rounds_fwd<R, 4, true>), g, b, 0, st, jl, single, wgs);
        else if (qr == 4) hipLaunchKernelGGL((k_rounds_fwd<R, 4, false>), g, b, 0, st, jl, single, wgs);
        else if (fsim) hipLaunchKernelGGL((k_rounds_fwd<R, 3, true>), g, b, 0, st, jl, single, wgs);
        else hipLaunchKernelGGL((k_rounds_fwd<R, 3, false>), g, b, 0, st, jl, single, wgs);
    }
    return hipGetLastError();
}

template <typename R>
hipError_t launch_rounds_rev(const JobList& jl, const Job& single, int qr, bool fsim, int64_t blocks, int nthreads,
                             hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    if (jl.jobs || !rounds_qr_ok<R>(qr) || nthreads > (1 << (q_tile_bits<R>() - qr)) || nthreads < 64)
        return hipErrorInvalidValue;
    const dim3 g = dim3(unsigned(blocks)), b = dim3(unsigned(nthreads));
    if constexpr (sizeof(R) == 4) {
        if (qr == 5 && fsim) hipLaunchKernelGGL((k_rounds_rev<R, 5, true>), g, b, 0, st, jl, single);
        else if (qr == 5) hipLaunchKernelGGL((k_rounds_rev<R, 5, false>), g, b, 0, st, jl, single);
        else if (fsim) hipLaunchKernelGGL((k_rounds_rev<R, 4, true>), g, b, 0, st, jl, single);
        else hipLaunchKernelGGL((k_rounds_rev<R, 4, false>), g, b, 0, st, jl, single);
    } else {
        if (qr == 4 && fsim) hipLaunchKernelGGL((k_rounds_rev<R, 4, true>), g, b, 0, st, jl, single);
        else if (qr == 4) hipLaunchKernelGGL((k_rounds_rev<R, 4, false>), g, b, 0, st, jl, single);
        else if (fsim) hipLaunchKernelGGL((k_rounds_rev<R, 3, true>), g, b, 0, st, jl, single);
        else hipLaunchKernelGGL((k_rounds_rev<R, 3, false>), g, b, 0, st, jl, single);
    }
    return hipGetLastError();
}

#define TCNG_INST_ROUNDS(R)                                                                                       \
    template hipError_t launch_rounds_coef<R>(const QStep*, int, const QStep*, int, const void*, int, int64_t,   \
                                              void*, hipStream_t);                                                \
    template size_t rounds_coef_bytes<R>(int);                                                                    \
    template hipError_t launch_rounds_fwd<R>(const JobList&, const Job&, int, bool, int, int64_t, int, hipStream_t); \
    template hipError_t launch_rounds_rev<R>(const JobList&, const Job&, int, bool, int64_t, int, hipStream_t);
TCNG_INST_ROUNDS(float)
TCNG_INST_ROUNDS(double)

template <typename R>
hipError_t launch_build_ops_multi(const BuildJob* jobs, const int64_t* prefix, int njobs, int64_t total,
                                  hipStream_t st) {
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_build_ops_multi<R>), dim3(unsigned((total + 255) / 256)), dim3(256), 0, st, jobs, prefix,
                       njobs, total);
    return hipGetLastError();
}
template hipError_t launch_build_ops_multi<float>(const BuildJob*, const int64_t*, int, int64_t, hipStream_t);
template hipError_t launch_build_ops_multi<double>(const BuildJob*, const int64_t*, int, int64_t, hipStream_t);

template hipError_t launch_build_ops<float>(const DevPlan&, int, const void*, int64_t, const void*, int64_t, void*,
                                            hipStream_t);
template hipError_t launch_build_ops<double>(const DevPlan&, int, const void*, int64_t, const void*, int64_t, void*,
                                             hipStream_t);
#define TCNG_INST_TILE(R, RB)                                                                                     \
    template hipError_t launch_tile_fwd<R, RB>(const JobList&, const Job&, int64_t, int, hipStream_t);           \
    template hipError_t launch_tile_rev<R, RB>(const JobList&, const Job&, int64_t, int, hipStream_t);
TCNG_INST_TILE(float, 4)
TCNG_INST_TILE(float, 5)
TCNG_INST_TILE(double, 3)
TCNG_INST_TILE(double, 4)

}  // namespace tcng
