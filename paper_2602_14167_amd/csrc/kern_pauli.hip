// Pauli-sum kernels: lambda = H psi and E = <psi|H|psi>.
//
// For a Pauli string P with X-mask x (qubits carrying X or Y) and Z-mask z
// (qubits carrying Z or Y),  (P psi)_j = i^{#Y} (-1)^{popcount((j^x) & z)} psi_{j^x}
// (from X|b> = |b^1>, Z|b> = (-1)^b |b>, Y = i X Z).  Terms sharing an X-mask
// read the same partner amplitude psi_{j^x}, so H is applied group by group:
//   (H psi)_j = psi_{j^x} * sum_{k in group} c_k i^{#Y_k} (-1)^{popcount((j^x) & z_k)}.
// Inside a group, terms of equal coefficient form a class whose signed sum is
// c * (n_terms - 2 * #odd parities): integer counting (four elements' counts
// as bytes of one word), no float adds per term.  The tiled pass forms each
// element's share of (H psi)_l in the state's precision (float32 for
// complex64: lambda is stored in it); E accumulates Re(conj(psi_l) * share)
// in float64, reduced per wave by butterfly shuffles and per workgroup in a
// fixed order (deterministic); the partial sums go to `epart` for a final
// fixed-order sum.
// Measurement parallelism over terms (Sec. "Data Parallelism") is realised on
// one GPU as parallelism over amplitudes with all terms of a group fused.
#include "devutil.h"

namespace tcng {

namespace {

constexpr int NTHREADS = 256;

template <typename R>
struct PTile {
    static constexpr int ELEMS = 1 << 12;   // 12-bit tiles: 32 KiB (complex64) or 64 KiB (complex128)
};

__device__ __forceinline__ uint64_t loc2glob(uint32_t l, int lo, int m, const int* lq) {
    uint64_t g = l & ((1u << lo) - 1);
#pragma unroll
    for (int i = 0; i < MAX_TILE_BITS; ++i)
        if (i >= lo && i < m) g |= uint64_t((l >> i) & 1) << lq[i];
    return g;
}

// the thread's offset passed through an empty asm statement at each use:
// otherwise the compiler keeps every element's 64-bit address live across the
// tile loop (166 registers instead of about 60)
__device__ __forceinline__ uint64_t pinned(uint64_t v) {
    uint32_t lo = uint32_t(v), hi = uint32_t(v >> 32);
    asm volatile("" : "+v"(lo), "+v"(hi));
    return (uint64_t(hi) << 32) | lo;
}

// v ^ u for a per-lane v and a uniform u, as one instruction the compiler
// cannot hoist out of a loop (hoisted, every element's xor would hold a
// register across the group loop)
__device__ __forceinline__ uint32_t lane_xor(uint32_t v, uint32_t u) {
    uint32_t r;
    asm volatile("v_xor_b32 %0, %1, %2" : "=v"(r) : "s"(u), "v"(v));
    return r;
}

// global offset of element it's local index bits it * nt (the top RB local
// bits), from their images: a few selects instead of a loop over every local bit
template <int RB>
__device__ __forceinline__ uint64_t elem_off(const uint64_t* hb, int it) {
    uint64_t g = 0;
#pragma unroll
    for (int k = 0; k < RB; ++k)
        if ((it >> k) & 1) g += hb[k];
    return g;
}

__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v)));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v) >> 32));
    return int64_t((uint64_t(hi) << 32) | lo);
}

// a class's coefficient in the state's precision
template <typename R> __device__ __forceinline__ R coef_re(const PClass& C);
template <typename R> __device__ __forceinline__ R coef_im(const PClass& C);
template <> __device__ __forceinline__ float coef_re<float>(const PClass& C) { return C.fre; }
template <> __device__ __forceinline__ float coef_im<float>(const PClass& C) { return C.fim; }
template <> __device__ __forceinline__ double coef_re<double>(const PClass& C) { return C.cre; }
template <> __device__ __forceinline__ double coef_im<double>(const PClass& C) { return C.cim; }
template <typename R> __device__ __forceinline__ R grp_re(const PGroup& G);
template <typename R> __device__ __forceinline__ R grp_im(const PGroup& G);
template <> __device__ __forceinline__ float grp_re<float>(const PGroup& G) { return G.fbr; }
template <> __device__ __forceinline__ float grp_im<float>(const PGroup& G) { return G.fbi; }
template <> __device__ __forceinline__ double grp_re<double>(const PGroup& G) { return G.cbr; }
template <> __device__ __forceinline__ double grp_im<double>(const PGroup& G) { return G.cbi; }

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

__device__ __forceinline__ double shfl_sum(double v, int width) {
    for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, width);
    return v;
}

// fixed-order workgroup sum of one double per thread (result valid in thread 0)
__device__ double block_sum(double v, double* sh, int nthreads) {
    const int width = nthreads < 64 ? nthreads : 64;
    v = width == 64 ? wave_sum(v) : shfl_sum(v, width);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (nthreads + 63) / 64; ++w) s += sh[w];
    return s;
}

// the tile's element l ^ x for the thread's element l = e + t (e: the element
// index's bits, uniform): the thread's bits and e's are disjoint, so the byte
// offset is the thread's xor a uniform part
template <typename R>
__device__ __forceinline__ cx<R> partner(const cx<R>* lds, uint32_t tb8, uint32_t e, uint32_t x) {
    const uint32_t off = lane_xor(tb8, (e ^ x) * uint32_t(sizeof(cx<R>)));
    return *reinterpret_cast<const cx<R>*>(reinterpret_cast<const char*>(lds) + off);
}

// odd-parity counts of a class's terms for the elements c0 .. c0 + 4 CW - 1 of
// the thread, a byte per element: parity((l ^ x) & z) splits into the
// thread's part, the tile's part and the element index's part (the planner's epar)
template <int CW>
__device__ __forceinline__ void odd_counts(cptr<PTerm> terms, int k0, int k1, uint64_t base, uint32_t t, int c0,
                                           uint32_t (&odd)[CW]) {
#pragma unroll
    for (int w = 0; w < CW; ++w) odd[w] = 0;
    for (int k = k0; k < k1; ++k) {
        const uint32_t zl = uint32_t(terms[k].z_local);
        const uint32_t tb = (__popcll(base & terms[k].z_out) & 1) ? 0x01010101u : 0u;
        const uint32_t pt = (uint32_t(__popc(t & zl)) & 1u) * 0x01010101u;   // per lane
        cptr<uint32_t> ep = terms[k].epar + (c0 >> 2);
#pragma unroll
        for (int w = 0; w < CW; ++w) odd[w] += pt ^ (ep[w] ^ tb);
    }
}

// ---------------------------------------------------------------------------
// tiled: one pass handles every X-group whose mask lies inside its tile
// ---------------------------------------------------------------------------
template <typename R, int RB>
__global__ void __launch_bounds__(NTHREADS)
k_pauli_tile(const JobList jl, const Job single) {
    __shared__ cx<R> lds[PTile<R>::ELEMS];
    __shared__ double sh[NTHREADS / 64];
    constexpr int NB = 1 << RB;
    int64_t local;
    const Job J = load_job(jl, single, blockIdx.x, local);
    const int pass_idx = jl.step;
    cptr<PGroup> groups = as_const(J.pgroups);
    cptr<PClass> classes = as_const(J.pclasses);
    cptr<PTerm> terms = as_const(J.pterms);
    const int accumulate = pass_idx > 0;
    const int wgs = J.e_wgs;
    const int n = J.n;
    // (the 64-bit division runs on the vector unit: its results are moved back
    // to scalar registers, so the tile's base offset and its parities stay scalar)
    const int64_t b = uniform64(local / wgs);
    const int wg = uniform(int(local - b * wgs));
    cptr<PPass> P = as_const(J.ppasses) + pass_idx;
    const int m = P->m, lo = P->lo;
    const uint64_t tmask = P->tile_mask;
    int lq[MAX_TILE_BITS];
#pragma unroll
    for (int i = 0; i < MAX_TILE_BITS; ++i) lq[i] = P->local_qubit[i];
    const int nt = 1 << (m - RB);
    const int64_t tiles_per_state = int64_t(1) << (n - m);
    const int t = threadIdx.x;
    // nt is a multiple of 64: whole waves are active or idle
    const bool active = uniform(t >> 6) < (nt >> 6);
    gptr<const cx<R>> psi = as_global(static_cast<const cx<R>*>(J.state)) + b * J.stride;
    gptr<cx<R>> lam = as_global(J.costate ? static_cast<cx<R>*>(J.costate) : nullptr) + (J.costate ? b * J.stride : 0);
    const bool has_lam = J.costate != nullptr;
    double e_acc = 0.0;
    // element l = it * nt + t: the thread's bits (below m - RB) and the
    // iteration's bits are disjoint, so the global offset and every Z-parity
    // split into a per-thread and a uniform part
    const uint64_t gt = loc2glob(uint32_t(t), lo, m, lq);
    // images of the element-index bits (local bits m - RB .. m - 1)
    uint64_t hb[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) hb[k] = loc2glob(1u << (m - RB + k), lo, m, lq);

    const uint32_t tb8 = uint32_t(t) * uint32_t(sizeof(cx<R>));   // the thread's byte offset in the LDS tile
    const bool read_lam = has_lam && accumulate;
    // elements per chunk: CH lambda values in flight and CH accumulators
    constexpr int CH = (sizeof(R) == 4) ? 8 : 4;
    constexpr int CW = CH / 4;   // packed parity-count words (a byte per element)
    static_assert(NB % CH == 0 && CH % 4 == 0, "chunks of whole count words");
    for (int64_t tile = wg; tile < tiles_per_state; tile += wgs) {
        const uint64_t base = uniform64(int64_t(tile_base(uint64_t(tile), tmask, n)));
        __syncthreads();
        // psi tile -> LDS; element l = it*nt + t (lane-consecutive, coalesced)
        if (active) {
#pragma unroll
            for (int it = 0; it < NB; ++it) {
                const uint32_t l = uint32_t(it * nt + t);
                lds[l] = psi[(base + elem_off<RB>(hb, it)) + pinned(gt)];
            }
        }
        __syncthreads();
        if (!active) continue;
        // elements l = it*nt + t, CH at a time; the term loop is outside the
        // element loop so every scalar load of a term serves CH elements
#pragma unroll 1   // (unrolled, the chunks' accumulators double the registers)
        for (int c0 = 0; c0 < NB; c0 += CH) {
            // the chunk's lambda elements (later passes accumulate into them):
            // in flight while the groups are summed
            cx<R> acc[CH];
#pragma unroll
            for (int i = 0; i < CH; ++i)
                acc[i] = read_lam ? lam[(base + elem_off<RB>(hb, c0 + i)) + pinned(gt)] : cx<R>{R(0), R(0)};
            // this pass's share of (H psi)_l: sum over groups of
            // (cre + i cim) psi_{l ^ x}, in the state's precision; E takes
            // Re(conj(psi_l) * share) in float64 once per element
            R sr[CH], si[CH];
#pragma unroll
            for (int i = 0; i < CH; ++i) { sr[i] = R(0); si[i] = R(0); }
            const int g_end = P->group_end;
            for (int g = P->group_begin; g < g_end; ++g) {
                const PGroup G = groups[g];
                // the group's coefficient of psi_{l ^ x}: the element-independent
                // sum c * n_terms, then -2 c * #odd parities per class
                const R gbr = grp_re<R>(G), gbi = grp_im<R>(G);
                if (G.no_z) {
                    // X-only strings: one coefficient for every element (real
                    // for the field terms of a spin model: two products, not four)
                    if (gbi == R(0)) {
#pragma unroll
                        for (int i = 0; i < CH; ++i) {
                            const cx<R> pp = partner<R>(lds, tb8, uint32_t((c0 + i) * nt), uint32_t(G.x_local));
                            sr[i] = fma(gbr, pp.re, sr[i]);
                            si[i] = fma(gbr, pp.im, si[i]);
                        }
                    } else {
#pragma unroll
                        for (int i = 0; i < CH; ++i) {
                            const cx<R> pp = partner<R>(lds, tb8, uint32_t((c0 + i) * nt), uint32_t(G.x_local));
                            sr[i] = fma(gbr, pp.re, fma(-gbi, pp.im, sr[i]));
                            si[i] = fma(gbr, pp.im, fma(gbi, pp.re, si[i]));
                        }
                    }
                    continue;
                }
                // (every group lists at least one class, possibly without terms)
                int c = G.class_begin;
                const int c_end = G.class_end;
                R cre[CH], cim[CH];
                uint32_t odd[CW];
                odd_counts<CW>(terms, classes[c].term_begin, classes[c].term_end, base, uint32_t(t), c0, odd);
                const R m2r = R(-2) * coef_re<R>(classes[c]), m2i = R(-2) * coef_im<R>(classes[c]);
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const R cnt = R((odd[i >> 2] >> (8 * (i & 3))) & 0xFFu);   // (a byte-to-float convert)
                    cre[i] = fma(m2r, cnt, gbr);
                    cim[i] = fma(m2i, cnt, gbi);
                }
                for (++c; c < c_end; ++c) {
                    odd_counts<CW>(terms, classes[c].term_begin, classes[c].term_end, base, uint32_t(t), c0, odd);
                    const R n2r = R(-2) * coef_re<R>(classes[c]), n2i = R(-2) * coef_im<R>(classes[c]);
#pragma unroll
                    for (int i = 0; i < CH; ++i) {
                        const R cnt = R((odd[i >> 2] >> (8 * (i & 3))) & 0xFFu);
                        cre[i] = fma(n2r, cnt, cre[i]);
                        cim[i] = fma(n2i, cnt, cim[i]);
                    }
                }
#pragma unroll
                for (int i = 0; i < CH; ++i) {
                    const cx<R> pp = partner<R>(lds, tb8, uint32_t((c0 + i) * nt), uint32_t(G.x_local));
                    sr[i] = fma(cre[i], pp.re, fma(-cim[i], pp.im, sr[i]));
                    si[i] = fma(cre[i], pp.im, fma(cim[i], pp.re, si[i]));
                }
            }
#pragma unroll
            for (int i = 0; i < CH; ++i) {
                const cx<R> own = lds[uint32_t((c0 + i) * nt + t)];
                e_acc = fma(double(own.re), double(sr[i]), fma(double(own.im), double(si[i]), e_acc));
                acc[i].re += sr[i];
                acc[i].im += si[i];
            }
            if (has_lam) {
#pragma unroll
                for (int i = 0; i < CH; ++i)
                    lam[(base + elem_off<RB>(hb, c0 + i)) + pinned(gt)] = acc[i];
            }
        }
    }
    const double s = block_sum(e_acc, sh, blockDim.x);
    if (t == 0) J.epart[(size_t(b) * J.e_rows + pass_idx) * wgs + wg] = s;
}

// ---------------------------------------------------------------------------
// plain: one X-group over the whole state
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(NTHREADS)
k_pauli_group(const cx<R>* __restrict__ state, cx<R>* __restrict__ costate, int accumulate, int64_t stride, int n,
              uint64_t x, const PClassFull* __restrict__ classes, int class_begin, int class_end,
              const PTermFull* __restrict__ terms, int wgs, double* __restrict__ epart, int row, int n_rows) {
    __shared__ double sh[NTHREADS / 64];
    const int64_t b = blockIdx.x / wgs;
    const int wg = int(blockIdx.x - b * wgs);
    const cx<R>* psi = state + b * stride;
    cx<R>* lam = costate ? costate + b * stride : nullptr;
    const uint64_t dim = uint64_t(1) << n;
    double e_acc = 0.0;
    for (uint64_t j = uint64_t(wg) * blockDim.x + threadIdx.x; j < dim; j += uint64_t(wgs) * blockDim.x) {
        const uint64_t jp = j ^ x;
        const cx<R> pp = psi[jp], pj = psi[j];
        double cre = 0.0, cim = 0.0;
        for (int c = class_begin; c < class_end; ++c) {
            const PClassFull C = classes[c];
            int odd = 0;
            for (int k = C.term_begin; k < C.term_end; ++k) odd += __popcll(jp & terms[k].z) & 1;
            const double s = double(C.term_end - C.term_begin - 2 * odd);
            cre = fma(C.cre, s, cre);
            cim = fma(C.cim, s, cim);
        }
        const cx<R> cc = {R(cre), R(cim)};
        if (lam) {
            const cx<R> prev = accumulate ? lam[j] : cx<R>{R(0), R(0)};
            lam[j] = cfma(cc, pp, prev);
        }
        const double rr = fma(double(pj.re), double(pp.re), double(pj.im) * double(pp.im));
        const double ri = fma(double(pj.re), double(pp.im), -double(pj.im) * double(pp.re));
        e_acc += cre * rr - cim * ri;
    }
    const double s = block_sum(e_acc, sh, blockDim.x);
    if (threadIdx.x == 0) epart[(size_t(b) * n_rows + row) * wgs + wg] = s;
}

}  // namespace

template <typename R, int RB>
hipError_t launch_pauli_tile(const JobList& jl, const Job& single, int64_t blocks, int nthreads, hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_pauli_tile<R, RB>), dim3(unsigned(blocks)), dim3(nthreads), 0, st, jl, single);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_pauli_group(const void* state, void* costate, bool accumulate, int64_t stride, int n, int64_t batch,
                              uint64_t x, const PClassFull* classes, int class_begin, int class_end,
                              const PTermFull* terms, int wgs, double* epart, int row, int n_rows, hipStream_t st) {
    hipLaunchKernelGGL((k_pauli_group<R>), dim3(unsigned(wgs * batch)), dim3(NTHREADS), 0, st,
                       static_cast<const cx<R>*>(state), static_cast<cx<R>*>(costate), int(accumulate), stride, n, x,
                       classes, class_begin, class_end, terms, wgs, epart, row, n_rows);
    return hipGetLastError();
}

template hipError_t launch_pauli_tile<float, 4>(const JobList&, const Job&, int64_t, int, hipStream_t);
template hipError_t launch_pauli_tile<double, 4>(const JobList&, const Job&, int64_t, int, hipStream_t);
template hipError_t launch_pauli_group<float>(const void*, void*, bool, int64_t, int, int64_t, uint64_t,
                                              const PClassFull*, int, int, const PTermFull*, int, double*, int, int,
                                              hipStream_t);
template hipError_t launch_pauli_group<double>(const void*, void*, bool, int64_t, int, int64_t, uint64_t,
                                               const PClassFull*, int, int, const PTermFull*, int, double*, int, int,
                                               hipStream_t);

// ---------------------------------------------------------------------------
// Sparse (COO) form of a Pauli sum (Sec. "Lattice and Hamiltonian"): a term
// with X-mask x, Z-mask z and ny Y factors maps |col> to i^ny (-1)^popcount(col & z)
// |col ^ x>, so H[row][row ^ x] sums the terms of one X-mask group.  One
// workgroup row (blockIdx.y) per group, so a wave loops over one group's
// terms; entries are group-major and each thread writes consecutive rows
// (coalesced 8 + 8 + 16 bytes).  HBM-bound: 32 bytes written per entry.
// ---------------------------------------------------------------------------
namespace {
__global__ void __launch_bounds__(256) k_pauli_coo(const uint64_t* __restrict__ gx, const int32_t* __restrict__ gstart,
                                                   const uint64_t* __restrict__ tz, const double2* __restrict__ tc,
                                                   int64_t row_begin, int64_t count, int64_t* __restrict__ rows,
                                                   int64_t* __restrict__ cols, double2* __restrict__ vals) {
    const int g = blockIdx.y;
    const uint64_t x = gx[g];
    const int k0 = gstart[g], k1 = gstart[g + 1];
    const size_t off = size_t(g) * size_t(count);
    for (int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x; r < count; r += int64_t(gridDim.x) * 256) {
        const uint64_t row = uint64_t(row_begin + r), col = row ^ x;
        double re = 0.0, im = 0.0;
        for (int k = k0; k < k1; ++k) {
            const double2 c = tc[k];
            const bool neg = __popcll(col & tz[k]) & 1;
            re += neg ? -c.x : c.x;
            im += neg ? -c.y : c.y;
        }
        rows[off + r] = int64_t(row);
        cols[off + r] = int64_t(col);
        vals[off + r] = make_double2(re, im);
    }
}
}  // namespace

hipError_t launch_pauli_coo(const uint64_t* gx, const int32_t* gstart, const uint64_t* tz, const double* tc, int groups,
                            int64_t row_begin, int64_t row_count, int64_t* rows, int64_t* cols, void* vals,
                            hipStream_t st) {
    if (groups == 0 || row_count == 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((row_count + 255) / 256, int64_t(1) << 16);
    hipLaunchKernelGGL(k_pauli_coo, dim3(unsigned(blocks), unsigned(groups)), dim3(256), 0, st, gx, gstart, tz,
                       reinterpret_cast<const double2*>(tc), row_begin, row_count, rows, cols,
                       static_cast<double2*>(vals));
    return hipGetLastError();
}

}  // namespace tcng
