// Fused block passes on matrix cores (complex64 state, float32 MFMA).
//
// A pass streams each tile of 2^m amplitudes through LDS once, as the tiled
// passes do; inside the tile every phase applies ONE block matrix M (the
// product of the phase's gates on its FUSED_K = 4 local bits, formed in
// float64 and rounded once) to all 2^(m-4) columns.  Splitting complex
// numbers into real and imaginary parts turns y = M x into a real 32 x 32
// product, which v_mfma_f32_32x32x2f32 evaluates 32 columns at a time
// (the paper's JIT "operator fusion", done here as explicit block matrices).
//
// Reverse sweep (adjoint): psi and lambda are un-computed block by block
// (psi_in = M^dagger psi_out, lambda_in = M^dagger lambda_out) and the block's
// outer product O = sum over columns of lambda_in psi_in^dagger (16 x 16) is
// accumulated with a third matrix-core product, float32 within a tile and
// float64 across tiles.  Every gate derivative of the block then follows from
// O by 16 x 16 algebra (k_fused_grad): with X_1 = G_1 O and
// X_{g+1} = G_{g+1} X_g G_g^dagger, X_g = sum lambda_after_g phi_before_g^dagger,
// so dE/dtheta = 2 Im sum_ab Gen_ab conj((X_g G_g^dagger)_ab) and the U2
// cotangent is the partial trace of X_g over the block's other bits.
//
// MFMA operand / result layouts (lane l, h = l / 32, v = accumulator index):
//   A[i][k]: lane supplies A[l % 32][2 s + h] in step s
//   B[k][n]: lane supplies B[2 s + h][l % 32]
//   D[i][n]: lane holds D[8 (v / 4) + 4 h + v % 4][l % 32] in register v
#include "devutil.h"
#include "gates.h"

namespace tcng {

namespace {

typedef float f16v __attribute__((ext_vector_type(16)));

constexpr int FTHREADS = 256;            // 4 waves; 32-column tiles dealt round-robin (<= 2 per wave)
constexpr int FMAX_M = 12;               // tile bits of the fused kernels (largest)
// column tiles per wave for tiles of at most 2^MB amplitudes
template <int MB>
constexpr int ct_max() { return MB >= 12 ? 2 : 1; }
constexpr int OSTRIDE = 512;             // doubles per block outer product (16 x 16 complex)

__device__ __forceinline__ uint64_t loc2glob_f(uint32_t l, int lo, int m, cptr<FPass> P) {
    uint64_t g = l & ((1u << lo) - 1);
#pragma unroll
    for (int i = 0; i < MAX_TILE_BITS; ++i)
        if (i >= lo && i < m) g |= uint64_t((l >> i) & 1) << P->local_qubit[i];
    return g;
}

__device__ __forceinline__ uint64_t tile_base_f(uint64_t tile, uint64_t tmask, int n) {
    uint64_t base = 0;
    int k = 0;
    for (int q = 0; q < n; ++q) {
        if ((tmask >> q) & 1) continue;
        base |= ((tile >> k) & 1) << q;
        ++k;
    }
    return base;
}

// address of local index l under a layout (XOR of the images of its bits;
// masks instead of branches: l differs per lane)
__device__ __forceinline__ uint32_t lay_c(uint32_t l, cptr<int32_t> img, int m) {
    uint32_t a = 0;
#pragma unroll
    for (int b = 0; b < MAX_TILE_BITS; ++b)
        if (b < m) a ^= uint32_t(img[b]) & (0u - ((l >> b) & 1u));
    return a;
}

// tile HBM <-> LDS: thread t moves 16-byte chunks c = it * nthr + t (local
// indices 2c, 2c + 1), each amplitude to its address under `img`.  Layouts and
// the local -> global map are linear in the bits, so the thread's part
// (bits 1..log2(2 nthr)) and the iteration's part (higher bits) combine by XOR
// / addition: one per-lane term, uniform terms per iteration.
// Per-kernel addressing of the tile load and store (IT chunks per thread):
// the pass's maps are the same for every tile, so the lane's terms and the
// iterations' uniform terms are formed once.
template <int IT>
struct TileIO {
    uint64_t gt;                 // lane: global offset of local index 2t
    uint32_t at_ld, at_st;       // lane: LDS address of 2t in the load / store layout
    uint64_t gi[IT];             // uniform: global offset of 2 it nthr
    uint32_t ai_ld[IT], ai_st[IT];
    uint32_t a1_ld, a1_st;       // images of local bit 0
};

template <int IT>
__device__ __forceinline__ TileIO<IT> tile_io(cptr<FPass> P, int t, int nthr) {
    TileIO<IT> io;
    const int m = P->m, lo = P->lo;
    const uint32_t lt = 2u * uint32_t(t);
    io.gt = loc2glob_f(lt, lo, m, P);
    io.at_ld = lay_c(lt, as_const(P->ld), m);
    io.at_st = lay_c(lt, as_const(P->st), m);
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const uint32_t li = 2u * uint32_t(it * nthr);
        io.gi[it] = loc2glob_f(li, lo, m, P);
        io.ai_ld[it] = lay_c(li, as_const(P->ld), m);
        io.ai_st[it] = lay_c(li, as_const(P->st), m);
    }
    io.a1_ld = uint32_t(P->ld[0]);
    io.a1_st = uint32_t(P->st[0]);
    return io;
}

// NS states (psi, and lambda in the reverse sweep): every load in flight
// before the first LDS write
template <int IT, int NS>
__device__ __forceinline__ void ftile_load(float2* const* lds, const gptr<cx<float>>* st, uint64_t base,
                                           const TileIO<IT>& io) {
    float4 v[NS][IT];
#pragma unroll
    for (int k = 0; k < NS; ++k)
#pragma unroll
        for (int it = 0; it < IT; ++it)
            v[k][it] = *reinterpret_cast<gptr<const float4>>(st[k] + base + io.gt + io.gi[it]);
#pragma unroll
    for (int k = 0; k < NS; ++k)
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const uint32_t a = io.at_ld ^ io.ai_ld[it];
            lds[k][a] = make_float2(v[k][it].x, v[k][it].y);
            lds[k][a ^ io.a1_ld] = make_float2(v[k][it].z, v[k][it].w);
        }
}
template <int IT, int NS>
__device__ __forceinline__ void ftile_store(float2* const* lds, const gptr<cx<float>>* st, uint64_t base,
                                            const TileIO<IT>& io) {
#pragma unroll
    for (int k = 0; k < NS; ++k)
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const uint32_t a = io.at_st ^ io.ai_st[it];
            const float2 x = lds[k][a], y = lds[k][a ^ io.a1_st];
            *reinterpret_cast<gptr<float4>>(st[k] + base + io.gt + io.gi[it]) = make_float4(x.x, x.y, y.x, y.y);
        }
}

// the same load, each amplitude x first projected: kept (times sc) where
// (x & md) == bd, zero elsewhere (the collapse of a measurement record)
template <int IT>
__device__ __forceinline__ void ftile_load_proj(float2* lds, gptr<cx<float>> st, uint64_t base, const TileIO<IT>& io,
                                                uint32_t md, uint32_t bd, float sc) {
    float4 v[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) v[it] = *reinterpret_cast<gptr<const float4>>(st + base + io.gt + io.gi[it]);
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const uint32_t x = uint32_t(base + io.gt + io.gi[it]);   // global index of local 2c (bit 0 clear)
        const float f0 = ((x & md) == bd) ? sc : 0.f, f1 = (((x | 1u) & md) == bd) ? sc : 0.f;
        const uint32_t a = io.at_ld ^ io.ai_ld[it];
        lds[a] = make_float2(v[it].x * f0, v[it].y * f0);
        lds[a ^ io.a1_ld] = make_float2(v[it].z * f1, v[it].w * f1);
    }
}

// the tile of a basis state |basis> written to LDS under the load layout
// (every chunk zero but the one amplitude equal to 1); nothing is read
template <int IT>
__device__ __forceinline__ void ftile_basis(float2* lds, uint64_t base, const TileIO<IT>& io, uint64_t basis) {
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const uint64_t x = base + io.gt + io.gi[it];   // global index of local 2c (bit 0 clear)
        const uint32_t a = io.at_ld ^ io.ai_ld[it];
        lds[a] = make_float2(x == basis ? 1.f : 0.f, 0.f);
        lds[a ^ io.a1_ld] = make_float2((x | 1u) == basis ? 1.f : 0.f, 0.f);
    }
}

// per-lane view of one phase: addresses of the lane's column (block bits
// zero) and the uniform images of the block bits and of column bits 0..4
struct FView {
    uint32_t rd_col, wr_col;   // column ct * 32 + lane % 32
    uint32_t wr_tile;          // column ct * 32 (write layout)
    uint32_t rdR[FUSED_KMAX], wrR[FUSED_KMAX], wrC[5];   // block bit 4: 32 x 32 blocks only
};

__device__ __forceinline__ FView fview(cptr<FPhase> F, int ct, int lane) {
    FView v;
    uint32_t rl = 0, wl = 0, rw = 0, ww = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const uint32_t ir = uint32_t(F->rdc[k]), iw = uint32_t(F->wrc[k]);   // 0 beyond the tile
        if (k < 5) {
            v.wrC[k] = iw;
            const uint32_t msk = 0u - ((uint32_t(lane) >> k) & 1u);
            rl ^= ir & msk;
            wl ^= iw & msk;
        } else if ((ct >> (k - 5)) & 1) {
            rw ^= ir;
            ww ^= iw;
        }
    }
    v.rd_col = rl ^ rw;
    v.wr_col = wl ^ ww;
    v.wr_tile = ww;
#pragma unroll
    for (int t = 0; t < FUSED_KMAX; ++t) {
        v.rdR[t] = uint32_t(F->rdr[t]);
        v.wrR[t] = uint32_t(F->wrr[t]);
    }
    return v;
}

// the lane's MFMA input: components 2 s + h (s = 0..15) of its column,
// i.e. the 8 amplitudes with block index j = 2 s' + h (re for s < 8, im after);
// `half` is the image of the top block bit of a 32 x 32 block's half (0 otherwise)
__device__ __forceinline__ void read_cols(const float2* lds, const FView& v, int h, float* x, uint32_t half = 0u) {
    const uint32_t base = v.rd_col ^ (v.rdR[0] & (0u - uint32_t(h))) ^ half;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const uint32_t a = base ^ ((s & 1) ? v.rdR[1] : 0u) ^ ((s & 2) ? v.rdR[2] : 0u) ^ ((s & 4) ? v.rdR[3] : 0u);
        const float2 z = lds[a];
        x[s] = z.x;
        x[s + 8] = z.y;
    }
}

// 16 floats of this lane's matrix operand (lane-major table)
__device__ __forceinline__ void read_mat(gptr<const float> tbl, int lane, float* w) {
    gptr<const float4> p = reinterpret_cast<gptr<const float4>>(tbl + lane * 16);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float4 q = p[i];
        w[4 * i] = q.x;
        w[4 * i + 1] = q.y;
        w[4 * i + 2] = q.z;
        w[4 * i + 3] = q.w;
    }
}

// ---------------------------------------------------------------------------
// forward pass: one tile per workgroup
// ---------------------------------------------------------------------------
// waves and column tiles of a tile of 2^m amplitudes: 2^(m - 9) column tiles
// of 32 columns over min(4, 2^(m - 9)) waves
struct FWork {
    int nwv, ctw, nthr;
};
__device__ __forceinline__ FWork fwork(int m, int kb = FUSED_K) {
    FWork k;
    const int ct = 1 << (m - kb - 5);
    k.nwv = ct < 4 ? ct : 4;
    k.ctw = ct / k.nwv;
    k.nthr = 64 * k.nwv;
    return k;
}

// floats of one block's operand tables: the forward order, then the reverse
// one (four sub-blocks each for 32 x 32 blocks)
template <int KB>
constexpr int mats_stride() { return KB == 5 ? 8192 : 2048; }

// XCD-aware block order of a single-job launch: workgroups are dealt to the
// 8 XCDs round-robin, each with its own L2, so consecutive tiles (which share
// the 128-byte lines of 64-byte runs when a tile has 3 low qubits) go to blocks
// 8 apart, on one XCD; the tail past a multiple of 8 keeps its order
__device__ __forceinline__ int64_t xcd_block(int64_t blk, int64_t grid) {
    const int64_t g8 = grid & ~int64_t(7);
    return blk < g8 ? (blk & 7) * (g8 >> 3) + (blk >> 3) : blk;
}

// MB: largest tile bits of the instantiation (LDS size, column tiles per wave);
// KB: block bits of the plan
template <int IT, int MB, int KB>
__global__ void __launch_bounds__(FTHREADS) k_fused_fwd(const JobList jl, const Job single) {
    constexpr int CT_MAX = KB == 5 ? 1 : ct_max<MB>();
    __shared__ float2 lds[1 << MB];
    int64_t local;
    const Job J = load_job(jl, single, jl.jobs ? int64_t(blockIdx.x) : xcd_block(blockIdx.x, gridDim.x), local);
    cptr<FPass> P = as_const(J.fpasses) + jl.step;
    const int m = P->m;
    const FWork K = fwork(m, KB);
    const int t = threadIdx.x;
    const int wave = uniform(t >> 6), lane = t & 63, h = lane >> 5;
    const bool active = wave < K.nwv;
    const int64_t b = local / J.tiles;
    const uint64_t tile = uint64_t(local - b * J.tiles);
    gptr<cx<float>> psi = as_global(static_cast<cx<float>*>(J.state)) + b * J.stride;
    gptr<const float> mats =
        as_global(static_cast<const float*>(J.fmats)) + size_t(J.shared ? 0 : b) * J.n_blocks * mats_stride<KB>();
    cptr<FPhase> phases = as_const(J.fphases);
    const uint64_t base = tile_base_f(tile, P->tile_mask, J.n);
    float2* const bufs[1] = {lds};
    const gptr<cx<float>> sts[1] = {psi};
    // the first pass may load from another state (the tiles are stored into psi)
    const gptr<cx<float>> lsrc[1] = {(J.src && jl.step == 0)
                                         ? as_global(static_cast<cx<float>*>(const_cast<void*>(J.src))) + b * J.src_stride
                                         : psi};
    const TileIO<IT> io = tile_io<IT>(P, t, K.nthr);

    if (active) {
        if (J.init_basis1 && jl.step == 0) {
            ftile_basis<IT>(lds, base, io, uint64_t(J.init_basis1 - 1));
        } else if (J.prec && jl.step == 0 && J.prec[b * J.prec_stride] != 0u) {
            const uint32_t md = J.prec[b * J.prec_stride], bd = J.prec[b * J.prec_stride + 1];
            ftile_load_proj<IT>(lds, lsrc[0], base, io, md, bd, float(1.0 / sqrt(J.pkeep[b])));
        } else {
            ftile_load<IT, 1>(bufs, lsrc, base, io);
        }
    }
    const int f_end = P->phase_end;
    if constexpr (KB == 5) {
        // 32 x 32 blocks: y_i = M_i0 x_0 + M_i1 x_1 over the halves of a column
        // (top block bit 0 / 1), four 16 x 16 sub-block products, one column
        // tile per wave
        __syncthreads();
        for (int f = P->phase_begin; f < f_end; ++f) {
            cptr<FPhase> F = phases + f;
            float x0[16], x1[16], w[4][16];
            FView v;
            if (active) {
                v = fview(F, wave, lane);
                read_cols(lds, v, h, x0);
                read_cols(lds, v, h, x1, v.rdR[4]);
#pragma unroll
                for (int sb = 0; sb < 4; ++sb) read_mat(mats + size_t(F->block) * 8192 + sb * 1024, lane, w[sb]);
            }
            __syncthreads();   // the phase writes another layout: all reads first
            if (active) {
                const f16v z = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                f16v acc[2] = {z, z};
#pragma unroll
                for (int s = 0; s < 16; ++s) {
                    acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(w[0][s], x0[s], acc[0], 0, 0, 0);
                    acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(w[2][s], x0[s], acc[1], 0, 0, 0);
                }
#pragma unroll
                for (int s = 0; s < 16; ++s) {
                    acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(w[1][s], x1[s], acc[0], 0, 0, 0);
                    acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(w[3][s], x1[s], acc[1], 0, 0, 0);
                }
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    const uint32_t wb = v.wr_col ^ (v.wrR[2] & (0u - uint32_t(h))) ^ (i ? v.wrR[4] : 0u);
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        const uint32_t a = wb ^ ((q & 1) ? v.wrR[0] : 0u) ^ ((q & 2) ? v.wrR[1] : 0u) ^
                                           ((q & 4) ? v.wrR[3] : 0u);
                        lds[a] = make_float2(acc[i][q], acc[i][q + 8]);
                    }
                }
            }
            __syncthreads();
        }
        if (active) ftile_store<IT, 1>(bufs, sts, base, io);
        return;
    }
    // block matrices one phase ahead: the next phase's loads are in flight
    // while this phase's matrix products run
    float wn[16];
    if (active) read_mat(mats + size_t(phases[P->phase_begin].block) * 2048, lane, wn);
    __syncthreads();
    for (int f = P->phase_begin; f < f_end; ++f) {
        cptr<FPhase> F = phases + f;
        float x[CT_MAX][16], w[16];
        FView v[CT_MAX];
        if (active) {
#pragma unroll
            for (int k = 0; k < CT_MAX; ++k) {
                if (k >= K.ctw) break;
                v[k] = fview(F, wave + K.nwv * k, lane);
                read_cols(lds, v[k], h, x[k]);
            }
        }
        __syncthreads();   // the phase writes another layout: all reads first
        if (active) {
#pragma unroll
            for (int i = 0; i < 16; ++i) w[i] = wn[i];
            if (f + 1 < f_end) read_mat(mats + size_t(phases[f + 1].block) * 2048, lane, wn);
#pragma unroll
            for (int k = 0; k < CT_MAX; ++k) {
                if (k >= K.ctw) break;
                f16v acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int s = 0; s < 16; ++s) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(w[s], x[k][s], acc, 0, 0, 0);
                // register q (< 8): re of y[j], q + 8: im, j = 8 (q / 4) + 4 h + q % 4
                const uint32_t wb = v[k].wr_col ^ (v[k].wrR[2] & (0u - uint32_t(h)));
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const uint32_t a = wb ^ ((q & 1) ? v[k].wrR[0] : 0u) ^ ((q & 2) ? v[k].wrR[1] : 0u) ^
                                       ((q & 4) ? v[k].wrR[3] : 0u);
                    lds[a] = make_float2(acc[q], acc[q + 8]);
                }
            }
        }
        __syncthreads();
    }
    if (active) ftile_store<IT, 1>(bufs, sts, base, io);
}

// ---------------------------------------------------------------------------
// reverse pass (pass n_passes - 1 - step): psi and lambda tiles in LDS; `wgs`
// workgroups per member loop over the tiles (two workgroups per CU).
//
// Outer product of a block, O[a][b] = sum_col lambda_in[a] conj(psi_in[b]),
// straight from the un-apply results (lane l, register q: component l % 32 of
// column 8 (q / 4) + 4 h + q % 4).  v_permlane16_swap on the registers of a
// pair (q, q + 1) moves the real parts of the four columns (q, q + 1) x
// (h = 0, 1) into one register and the imaginary parts into the other, each
// 16-lane row holding one column; as the A / B operands of
// v_mfma_f32_16x16x4f32 (K index = lane / 16 = that row)
//   O_re += Re(lambda) Re(psi) + Im(lambda) Im(psi),
//   O_im += Im(lambda) Re(psi) - Re(lambda) Im(psi)  (two accumulators).
// Each wave's 512 sums go to a staging area; after the block's barrier every
// thread adds two of the 512 entries over the waves into its registers (no
// atomics), and every FLUSH_TILES tiles into this workgroup's float64
// partials in global memory (its own slice).
// ---------------------------------------------------------------------------
typedef float f4v __attribute__((ext_vector_type(4)));
constexpr int FLUSH_TILES = 16;

// per block width: doubles of one outer product (16 x 16 or 32 x 32 complex),
// entries a thread accumulates, blocks a pass holds
template <int KB>
struct ORev {
    static constexpr int OS = KB == 5 ? 4 * OSTRIDE : OSTRIDE;
    static constexpr int NE = OS / FTHREADS;
    static constexpr int MAXB = KB == 5 ? FUSED5_MAX_BLOCKS : FUSED_MAX_BLOCKS;
};

// staging index e = sb * 512 + r * 128 + part * 64 + lane of MFMA output
// register r of sub-block sb = 2 i + j (O[a = 16 i + 4 (lane / 16) + r]
// [b = 16 j + lane % 16], part 0 = re; sb = 0 for 16 x 16 blocks) -> O entry
template <int KB>
__device__ __forceinline__ int stage_to_o(int e) {
    constexpr int D = 1 << KB;
    const int sb = e >> 9, r = (e >> 7) & 3, part = (e >> 6) & 1, ln = e & 63;
    const int a = 16 * (sb >> 1) + 4 * (ln >> 4) + r, bb = 16 * (sb & 1) + (ln & 15);
    return (a * D + bb) * 2 + part;
}

// add the staged sums of the waves into the thread's entries of block slot kb
template <int KB>
__device__ __forceinline__ void stage_reduce(const float* stage, int nwv, int kb,
                                             float (&acc)[ORev<KB>::MAXB][ORev<KB>::NE]) {
    constexpr int OS = ORev<KB>::OS, NE = ORev<KB>::NE;
    float v[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) v[u] = 0.f;
    for (int w = 0; w < nwv; ++w)
#pragma unroll
        for (int u = 0; u < NE; ++u) v[u] += stage[w * OS + threadIdx.x + FTHREADS * u];
    // every slot takes an add (zero for the others): a uniform runtime slot
    // must not become an indexed register access
#pragma unroll
    for (int k = 0; k < ORev<KB>::MAXB; ++k) {
        const bool hit = k == kb;
#pragma unroll
        for (int u = 0; u < NE; ++u) acc[k][u] += hit ? v[u] : 0.f;
    }
}

template <int KB>
__device__ __forceinline__ void flush_acc(float (&acc)[ORev<KB>::MAXB][ORev<KB>::NE], int nblk, gptr<double> dst,
                                          int wgs, bool first) {
    constexpr int OS = ORev<KB>::OS, NE = ORev<KB>::NE;
    // dst: this workgroup's slice of the pass's first block; block k at + k * wgs * OS.
    // The lane offsets are formed here, at each flush (opaque to loop-invariant
    // code motion): hoisted out of the tile loop, the addresses would hold
    // registers for the whole kernel.
    uint32_t off[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) {
        off[u] = uint32_t(stage_to_o<KB>(int(threadIdx.x) + FTHREADS * u));
        asm volatile("" : "+v"(off[u]));
    }
#pragma unroll
    for (int k = 0; k < ORev<KB>::MAXB; ++k) {
        if (k >= nblk) break;
#pragma unroll
        for (int i = 0; i < NE; ++i) {
            gptr<double> d = dst + size_t(k) * wgs * OS + off[i];
            const double v = double(acc[k][i]);
            *d = first ? v : *d + v;
            acc[k][i] = 0.f;
        }
    }
}

// outer-product contribution of one 16-row half pair: al = the un-applied
// lambda half (rows a), ap = the psi half (rows b), both in the output
// layout of the un-apply (after their write-back); v_permlane16_swap on a
// register pair (q, q + 1) leaves the real parts of the pair's four columns
// in one register and the imaginary parts in the other, one column per
// 16-lane row: the K layout of v_mfma_f32_16x16x4f32
__device__ __forceinline__ void outer_half(const f16v& ap, const f16v& al, f4v& ore, f4v& ore1, f4v& oim, f4v& oim1) {
#pragma unroll
    for (int q = 0; q < 16; q += 2) {
        const auto sp = __builtin_amdgcn_permlane16_swap(__float_as_uint(ap[q]), __float_as_uint(ap[q + 1]), false,
                                                         false);
        const auto sl = __builtin_amdgcn_permlane16_swap(__float_as_uint(al[q]), __float_as_uint(al[q + 1]), false,
                                                         false);
        const float pre = __uint_as_float(sp[0]), pim = __uint_as_float(sp[1]);
        const float lre = __uint_as_float(sl[0]), lim = __uint_as_float(sl[1]);
        ore = __builtin_amdgcn_mfma_f32_16x16x4f32(lre, pre, ore, 0, 0, 0);
        ore1 = __builtin_amdgcn_mfma_f32_16x16x4f32(lim, pim, ore1, 0, 0, 0);
        oim = __builtin_amdgcn_mfma_f32_16x16x4f32(lim, pre, oim, 0, 0, 0);
        oim1 = __builtin_amdgcn_mfma_f32_16x16x4f32(lre, pim, oim1, 0, 0, 0);
    }
}

// write-back of an un-apply result: float component n_c (re if < 16) of block
// index n_c % 16 of the half selected by `half` (the image of block bit 4)
__device__ __forceinline__ void rev_writeback(float* fdst, const FView& v, int n_c, int h, int part, uint32_t half,
                                              const f16v& r) {
    const uint32_t jb = (v.wrR[0] & (0u - uint32_t(n_c & 1))) ^ (v.wrR[1] & (0u - uint32_t((n_c >> 1) & 1))) ^
                        (v.wrR[2] & (0u - uint32_t((n_c >> 2) & 1))) ^ (v.wrR[3] & (0u - uint32_t((n_c >> 3) & 1)));
    const uint32_t wb = v.wr_tile ^ jb ^ (v.wrC[2] & (0u - uint32_t(h))) ^ half;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        // column ct * 32 + 8 (q / 4) + 4 h + q % 4: bits 0, 1 <- q, bit 2 <- h, bits 3, 4 <- q / 4
        const uint32_t a = wb ^ ((q & 1) ? v.wrC[0] : 0u) ^ ((q & 2) ? v.wrC[1] : 0u) ^ ((q & 4) ? v.wrC[3] : 0u) ^
                           ((q & 8) ? v.wrC[4] : 0u);
        fdst[2 * a + part] = r[q];
    }
}

// 16 x 16 blocks: two workgroups per CU (72 KiB of LDS each at MB = 12);
// 32 x 32 blocks: one (96 KiB: both tiles and four staged sub-block products
// per wave)
template <int IT, int MB, int KB>
__global__ void __launch_bounds__(FTHREADS, KB == 5 ? 1 : 2) k_fused_rev(const JobList jl, const Job single) {
    constexpr int CT_MAX = KB == 5 ? 1 : ct_max<MB>();
    constexpr int OS = ORev<KB>::OS, NE = ORev<KB>::NE, MAXB = ORev<KB>::MAXB;
    __shared__ float2 lps[1 << MB];
    __shared__ float2 llm[1 << MB];
    __shared__ float stage[(FTHREADS / 64) * OS];
    int64_t local;
    const Job J = load_job(jl, single, blockIdx.x, local);
    cptr<FPass> P = as_const(J.frpasses) + (J.n_passes - 1 - jl.step);
    const int m = P->m;
    const FWork K = fwork(m, KB);
    const int t = threadIdx.x;
    const int wave = uniform(t >> 6), lane = t & 63, h = lane >> 5;
    const bool active = wave < K.nwv;
    const int wgs = J.wgs;
    // shared block matrices: the workgroups loop over (member, tile) pairs and sum
    // the outer products of all members into member 0's partials
    const int64_t b = J.shared ? 0 : local / wgs;
    const int wg = int(local - b * wgs);
    gptr<cx<float>> psi = as_global(static_cast<cx<float>*>(J.state)) + b * J.stride;
    gptr<cx<float>> lam = as_global(static_cast<cx<float>*>(J.costate)) + b * J.stride;
    gptr<const float> mats = as_global(static_cast<const float*>(J.fmats)) + size_t(b) * J.n_blocks * mats_stride<KB>() +
                             mats_stride<KB>() / 2;
    cptr<FPhase> phases = as_const(J.frphases);
    const int f_begin = P->phase_begin, f_end = P->phase_end;
    const int nblk = f_end - f_begin;
    // blocks of a pass are numbered consecutively (visited in reverse)
    const int blk0 = phases[f_end - 1].block;
    gptr<double> odst = as_global(J.opart) + ((size_t(b) * J.n_blocks + blk0) * wgs + wg) * OS;

    float acc[MAXB][NE];
#pragma unroll
    for (int k = 0; k < MAXB; ++k)
#pragma unroll
        for (int u = 0; u < NE; ++u) acc[k][u] = 0.f;

    const int n_c = lane & 31;
    float* fp = reinterpret_cast<float*>(lps);
    float* fl = reinterpret_cast<float*>(llm);
    float* my_stage = stage + wave * OS + lane;
    const int part = n_c >> 4;
    float2* const bufs[2] = {lps, llm};
    const gptr<cx<float>> sts[2] = {psi, lam};
    const TileIO<IT> io = tile_io<IT>(P, t, K.nthr);
    int pending = 0;
    bool first = true;
    const int64_t items = J.shared ? J.tiles * J.batch : J.tiles;
    for (int64_t item = wg; item < items; item += wgs) {
        const int64_t mb = J.shared ? item / J.tiles : 0;
        const uint64_t base =
            tile_base_f(uint64_t(item - mb * J.tiles), P->tile_mask, J.n) + uint64_t(mb) * uint64_t(J.stride);
        __syncthreads();
        if (active) ftile_load<IT, 2>(bufs, sts, base, io);
        __syncthreads();
        for (int f = f_begin; f < f_end; ++f) {
            cptr<FPhase> F = phases + f;
            // the previous block's staged outer products (after its closing barrier)
            if (f > f_begin) stage_reduce<KB>(stage, K.nwv, phases[f - 1].block - blk0, acc);
            if constexpr (KB == 5) {
                // 32 x 32 blocks: each output half i of psi_in = M^dagger psi_out is
                // sum_j (M_ji)^dagger psi_out_j (sub-block operand 2 i + j); the outer
                // product's four sub-blocks O_ij = sum lambda_in_i psi_in_j^dagger
                float xp[2][16], xl[2][16], w[4][16];
                FView v;
                if (active) {
#pragma unroll
                    for (int sb = 0; sb < 4; ++sb) read_mat(mats + size_t(F->block) * 8192 + sb * 1024, lane, w[sb]);
                    v = fview(F, wave, lane);
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        read_cols(lps, v, h, xp[j], j ? v.rdR[4] : 0u);
                        read_cols(llm, v, h, xl[j], j ? v.rdR[4] : 0u);
                    }
                }
                __syncthreads();
                if (active) {
                    __builtin_amdgcn_s_setprio(1);
                    const f16v z = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                    f16v ap[2] = {z, z}, al[2] = {z, z};
#pragma unroll
                    for (int i = 0; i < 2; ++i)
#pragma unroll
                        for (int j = 0; j < 2; ++j)
#pragma unroll
                            for (int s = 0; s < 16; ++s) {
                                ap[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(xp[j][s], w[2 * i + j][s], ap[i], 0, 0, 0);
                                al[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(xl[j][s], w[2 * i + j][s], al[i], 0, 0, 0);
                            }
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        rev_writeback(fp, v, n_c, h, part, i ? v.wrR[4] : 0u, ap[i]);
                        rev_writeback(fl, v, n_c, h, part, i ? v.wrR[4] : 0u, al[i]);
                    }
                    const f4v z4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int sb = 0; sb < 4; ++sb) {
                        f4v ore = z4, oim = z4, ore1 = z4, oim1 = z4;
                        outer_half(ap[sb & 1], al[sb >> 1], ore, ore1, oim, oim1);
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            my_stage[sb * 512 + r * 128] = ore[r] + ore1[r];
                            my_stage[sb * 512 + r * 128 + 64] = oim[r] - oim1[r];
                        }
                    }
                    __builtin_amdgcn_s_setprio(0);
                }
                __syncthreads();
                continue;
            }
            float xp[CT_MAX][16], xl[CT_MAX][16], w[16];
            FView v[CT_MAX];
            if (active) {
                read_mat(mats + size_t(F->block) * 2048, lane, w);
#pragma unroll
                for (int k = 0; k < CT_MAX; ++k) {
                    if (k >= K.ctw) break;
                    v[k] = fview(F, wave + K.nwv * k, lane);
                    read_cols(lps, v[k], h, xp[k]);
                    read_cols(llm, v[k], h, xl[k]);
                }
            }
            __syncthreads();
            if (active) {
                // issue priority over the co-resident workgroup's memory phase while
                // this wave feeds the matrix cores
                __builtin_amdgcn_s_setprio(1);
                const f16v z = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                const f4v z4 = {0.f, 0.f, 0.f, 0.f};
                f4v ore = z4, oim = z4, ore1 = z4, oim1 = z4;
#pragma unroll
                for (int k = 0; k < CT_MAX; ++k) {
                    if (k >= K.ctw) break;
                    f16v ap = z, al = z;
#pragma unroll
                    for (int s = 0; s < 16; ++s) {
                        ap = __builtin_amdgcn_mfma_f32_32x32x2f32(xp[k][s], w[s], ap, 0, 0, 0);
                        al = __builtin_amdgcn_mfma_f32_32x32x2f32(xl[k][s], w[s], al, 0, 0, 0);
                    }
                    rev_writeback(fp, v[k], n_c, h, part, 0u, ap);
                    rev_writeback(fl, v[k], n_c, h, part, 0u, al);
                    outer_half(ap, al, ore, ore1, oim, oim1);
                    // one column tile at a time (register pressure)
                    __builtin_amdgcn_sched_barrier(0);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    my_stage[r * 128] = ore[r] + ore1[r];
                    my_stage[r * 128 + 64] = oim[r] - oim1[r];
                }
                __builtin_amdgcn_s_setprio(0);
            }
            __syncthreads();
        }
        stage_reduce<KB>(stage, K.nwv, phases[f_end - 1].block - blk0, acc);
        if (active) ftile_store<IT, 2>(bufs, sts, base, io);
        if (++pending == FLUSH_TILES) {
            flush_acc<KB>(acc, nblk, odst, wgs, first);
            first = false;
            pending = 0;
        }
    }
    if (pending || first) flush_acc<KB>(acc, nblk, odst, wgs, first);
}

// ---------------------------------------------------------------------------
// block matrices: M = G_L ... G_1 in float64 on the block's 4 bits, rounded
// to float32 in the two lane-major operand orders (forward: A = M~, reverse:
// B = M~, M~ = [[Re M, -Im M], [Im M, Re M]])
// ---------------------------------------------------------------------------
struct c64d {
    double re, im;
};
__device__ __forceinline__ c64d cmul(c64d a, c64d b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

// gate matrix in float64 (dim 2 or 4), rows = output, q0 = most significant bit
__device__ int gate_u64(const Op& op, const float* prm, const cx<float>* cm, c64d* u) {
    const int k = op.kind;
#pragma unroll
    for (int i = 0; i < 16; ++i) u[i] = {0.0, 0.0};
    double c = 0.0, s = 0.0;
    if (k == K_RX || k == K_RY || k == K_RZ || k == K_RZZ) sincos(0.5 * double(prm[op.p0]), &s, &c);
    const double r = 0.70710678118654752440;
    switch (k) {
        case K_RX: u[0] = {c, 0}; u[1] = {0, -s}; u[2] = {0, -s}; u[3] = {c, 0}; return 2;
        case K_RY: u[0] = {c, 0}; u[1] = {-s, 0}; u[2] = {s, 0}; u[3] = {c, 0}; return 2;
        case K_RZ: u[0] = {c, -s}; u[3] = {c, s}; return 2;
        case K_H: u[0] = {r, 0}; u[1] = {r, 0}; u[2] = {r, 0}; u[3] = {-r, 0}; return 2;
        case K_X: u[1] = {1, 0}; u[2] = {1, 0}; return 2;
        case K_Y: u[1] = {0, -1}; u[2] = {0, 1}; return 2;
        case K_Z: u[0] = {1, 0}; u[3] = {-1, 0}; return 2;
        case K_S: u[0] = {1, 0}; u[3] = {0, 1}; return 2;
        case K_U1: {
            const int ix[4] = {0, 1, 4, 5};
            for (int i = 0; i < 4; ++i) u[i] = {double(cm[16 * op.mat + ix[i]].re), double(cm[16 * op.mat + ix[i]].im)};
            return 2;
        }
        case K_CNOT: u[0] = {1, 0}; u[5] = {1, 0}; u[11] = {1, 0}; u[14] = {1, 0}; return 4;
        case K_CZ: u[0] = {1, 0}; u[5] = {1, 0}; u[10] = {1, 0}; u[15] = {-1, 0}; return 4;
        case K_RZZ: u[0] = {c, -s}; u[5] = {c, s}; u[10] = {c, s}; u[15] = {c, -s}; return 4;
        case K_FSIM: {
            double ct, st, cp, sp;
            sincos(double(prm[op.p0]), &st, &ct);
            sincos(double(prm[op.p1]), &sp, &cp);
            u[0] = {1, 0};
            u[5] = {ct, 0}; u[6] = {0, -st};
            u[9] = {0, -st}; u[10] = {ct, 0};
            u[15] = {cp, -sp};
            return 4;
        }
        default:   // K_U2
            for (int i = 0; i < 16; ++i) u[i] = {double(cm[16 * op.mat + i].re), double(cm[16 * op.mat + i].im)};
            return 4;
    }
}

// gate-local index of block index a, and block index a with the gate bits set to beta
__device__ __forceinline__ int gidx(const Op& op, int a, int dim) {
    return dim == 2 ? ((a >> op.r0) & 1) : ((((a >> op.r0) & 1) << 1) | ((a >> op.r1) & 1));
}
__device__ __forceinline__ int gset(const Op& op, int a, int dim, int beta) {
    if (dim == 2) return (a & ~(1 << op.r0)) | (beta << op.r0);
    return (a & ~((1 << op.r0) | (1 << op.r1))) | ((beta >> 1) << op.r0) | ((beta & 1) << op.r1);
}

// one workgroup of 256 threads per (block f, member b): thread entries
// e = t + 256 i of the 2^KB x 2^KB product (row a = e >> KB, column c)
template <int KB>
__device__ __forceinline__ void fused_mats_body(const FPhase* __restrict__ phases, const Op* __restrict__ ops,
                                                int n_blocks, const float* __restrict__ params, int64_t pstride,
                                                const cx<float>* __restrict__ cm, int64_t cmstride,
                                                float* __restrict__ out, int want_rev, int f, int64_t b) {
    constexpr int D = 1 << KB, EPT = D * D / 256, NSB = KB == 5 ? 4 : 1;
    __shared__ c64d M[D * D];
    __shared__ c64d U[16];
    const int t = threadIdx.x;
    const FPhase F = phases[f];
    const float* prm = params ? params + b * pstride : nullptr;
    cm += b * cmstride * 16;   // per-member matrices (cmstride 0: shared)
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
        const int e = t + 256 * i;
        M[e] = {(e >> KB) == (e & (D - 1)) ? 1.0 : 0.0, 0.0};
    }
    for (int o = F.op_begin; o < F.op_end; ++o) {
        const Op op = ops[o];
        if (t == 0) {   // gate matrix into LDS (indexed by the threads below)
            c64d u[16];
            gate_u64(op, prm, cm, u);
#pragma unroll
            for (int i = 0; i < 16; ++i) U[i] = u[i];
        }
        __syncthreads();
        const int dim = kind_arity(op.kind) == 2 ? 4 : 2;
        c64d nv[EPT];
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = t + 256 * i, a = e >> KB, c = e & (D - 1);
            const int al = gidx(op, a, dim);
            c64d acc = {0.0, 0.0};
            for (int be = 0; be < dim; ++be) {
                const c64d x = M[gset(op, a, dim, be) * D + c];
                const c64d p = cmul(U[al * dim + be], x);
                acc.re += p.re;
                acc.im += p.im;
            }
            nv[i] = acc;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < EPT; ++i) M[t + 256 * i] = nv[i];
    }
    __syncthreads();
    // real embedding entry (i, k), i, k < 32, of the 16 x 16 sub-block (bi, bj)
    auto emb = [&](int bi, int bj, int i, int k) -> float {
        const c64d z = M[(16 * bi + (i & 15)) * D + 16 * bj + (k & 15)];
        if ((i < 16) == (k < 16)) return float(z.re);
        return (i < 16) ? float(-z.im) : float(z.im);
    };
    float* dst = out + (size_t(b) * n_blocks + F.block) * (2048 * NSB);
    for (int sb = 0; sb < NSB; ++sb) {
        const int bi = sb >> 1, bj = sb & 1;
        for (int e = t; e < 1024; e += 256) {
            const int l = e >> 4, s = e & 15;
            const int kk = 2 * s + (l >> 5), ll = l & 31;
            dst[sb * 1024 + e] = emb(bi, bj, ll, kk);                            // forward: A[l % 32][2 s + h] of M_ij
            if (want_rev) dst[NSB * 1024 + sb * 1024 + e] = emb(bj, bi, kk, ll);   // reverse: B[2 s + h][l % 32] of M_ji
        }
    }
}

template <int KB>
__global__ void __launch_bounds__(256)
k_fused_mats(const FPhase* __restrict__ phases, const Op* __restrict__ ops, int n_blocks, const float* __restrict__ params,
             int64_t pstride, const cx<float>* __restrict__ cm, int64_t cmstride, float* __restrict__ out,
             int want_rev) {
    fused_mats_body<KB>(phases, ops, n_blocks, params, pstride, cm, cmstride, out, want_rev, int(blockIdx.x),
                        int64_t(blockIdx.y));
}

// uneven batch: circuit blockIdx.y, its block blockIdx.x (grid x: the most blocks of any circuit)
__global__ void __launch_bounds__(256) k_fused_mats_multi(const FusedCircJob* __restrict__ jobs) {
    const FusedCircJob J = jobs[blockIdx.y];
    if (int(blockIdx.x) >= J.n_blocks) return;   // the whole workgroup leaves together
    fused_mats_body<FUSED_K>(J.phases, J.ops, J.n_blocks, J.params, J.pstride, J.cm, 0, J.fmats, 1, int(blockIdx.x), 0);
}

// ---------------------------------------------------------------------------
// outer products: fixed-order sum over workgroups
// ---------------------------------------------------------------------------
__device__ __forceinline__ void fused_osum_one(const double* __restrict__ opart, int wgs, double* __restrict__ osum,
                                               int64_t i, int os = OSTRIDE) {
    const int64_t r = i / os, e = i - r * os;
    const double* p = opart + size_t(r) * wgs * os + e;
    double s = 0.0;
    for (int w = 0; w < wgs; ++w) s += p[size_t(w) * os];
    osum[i] = s;
}

// os: doubles of one outer product (512 for 16 x 16 blocks, 2048 for 32 x 32)
__global__ void k_fused_osum(const double* __restrict__ opart, int64_t rows, int wgs, double* __restrict__ osum,
                             int os) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= rows * os) return;
    fused_osum_one(opart, wgs, osum, i, os);
}

// uneven batch: circuit blockIdx.y, entries of its n_blocks outer products
__global__ void k_fused_osum_multi(const FusedCircJob* __restrict__ jobs) {
    const FusedCircJob J = jobs[blockIdx.y];
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= int64_t(J.n_blocks) * OSTRIDE) return;
    fused_osum_one(J.opart, J.wgs, J.osum, i);
}

// ---------------------------------------------------------------------------
// gate gradients of a block from its outer product (float64 16 x 16 algebra);
// writes slot values slots[b][slot] (the gradient slots of the tiled plan).
// One wave per (block, member); lane t holds X entries e = t + 64 i.
// ---------------------------------------------------------------------------
// gate matrix into LDS (lane 0 forms it; rows = output)
__device__ __forceinline__ int load_gate(const Op& op, const float* prm, const cx<float>* cm, c64d* U) {
    int dim = kind_arity(op.kind) == 2 ? 4 : 2;
    if (threadIdx.x == 0) {
        c64d u[16];
        gate_u64(op, prm, cm, u);
#pragma unroll
        for (int i = 0; i < 16; ++i) U[i] = u[i];
    }
    __syncthreads();
    return dim;
}

template <int KB>
__device__ __forceinline__ void fused_grad_body(const FPhase* __restrict__ phases, const Op* __restrict__ ops,
                                                int n_blocks, const float* __restrict__ params, int64_t pstride,
                                                const cx<float>* __restrict__ cm, const double* __restrict__ osum,
                                                int total_slots, double* __restrict__ slots, int f, int64_t b) {
    constexpr int D = 1 << KB, EPT = D * D / 64, OS = KB == 5 ? 4 * OSTRIDE : OSTRIDE;
    __shared__ c64d X[D * D];
    __shared__ c64d U[16];
    const int t = threadIdx.x;
    const FPhase F = phases[f];
    if (F.op_end == F.op_begin) return;
    const float* prm = params ? params + b * pstride : nullptr;
    const double* O = osum + (size_t(b) * n_blocks + F.block) * OS;
    double* sl = slots + size_t(b) * total_slots;
    c64d x[EPT];
    // X_1 = G_1 O
    {
        const Op op = ops[F.op_begin];
        const int dim = load_gate(op, prm, cm, U);
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = t + 64 * i, a = e >> KB, c = e & (D - 1);
            const int al = gidx(op, a, dim);
            c64d acc = {0.0, 0.0};
            for (int be = 0; be < dim; ++be) {
                const int r = gset(op, a, dim, be);
                const c64d p = cmul(U[al * dim + be], c64d{O[(r * D + c) * 2], O[(r * D + c) * 2 + 1]});
                acc.re += p.re;
                acc.im += p.im;
            }
            x[i] = acc;
        }
#pragma unroll
        for (int i = 0; i < EPT; ++i) X[t + 64 * i] = x[i];
        __syncthreads();
    }
    for (int o = F.op_begin; o < F.op_end; ++o) {
        const Op op = ops[o];
        const int dim = kind_arity(op.kind) == 2 ? 4 : 2;   // U holds this gate (loaded before)
        // U2 cotangent: partial trace of X over the block's other two bits
        if (op.kind == K_U2 && op.slot >= 0) {
            if (t < 16) {
                const int al = t >> 2, be = t & 3;
                double sr = 0.0, si = 0.0;
                for (int rest = 0; rest < D; ++rest) {
                    if (rest & ((1 << op.r0) | (1 << op.r1))) continue;
                    const c64d v = X[gset(op, rest, 4, al) * D + gset(op, rest, 4, be)];
                    sr += v.re;
                    si += v.im;
                }
                sl[op.slot + 2 * t] = sr;
                sl[op.slot + 2 * t + 1] = si;
            }
        }
        // Y = X G^dagger
        c64d y[EPT];
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            const int e = t + 64 * i, a = e >> KB, c = e & (D - 1);
            const int cl = gidx(op, c, dim);
            c64d acc = {0.0, 0.0};
            for (int de = 0; de < dim; ++de) {
                const c64d xv = X[a * D + gset(op, c, dim, de)];
                const c64d g = U[cl * dim + de];   // (G^dagger)[d][c] = conj(G[c][d])
                acc.re += xv.re * g.re + xv.im * g.im;
                acc.im += xv.im * g.re - xv.re * g.im;
            }
            y[i] = acc;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < EPT; ++i) X[t + 64 * i] = y[i];
        // angle derivatives: 2 Im sum_ab Gen_ab conj(Y_ab)
        if (op.slot >= 0 && op.kind != K_U2) {
            double g0 = 0.0, g1 = 0.0;
            const int mask = dim == 2 ? (1 << op.r0) : ((1 << op.r0) | (1 << op.r1));
#pragma unroll
            for (int i = 0; i < EPT; ++i) {
                const int e = t + 64 * i, a = e >> KB, c = e & (D - 1);
                if ((a & ~mask) != (c & ~mask)) continue;
                const int al = gidx(op, a, dim), clc = gidx(op, c, dim);
                const double yr = y[i].re, yi = -y[i].im;   // conj(Y)
                switch (op.kind) {
                    case K_RX:   // X/2
                        if (al != clc) g0 += yi;
                        break;
                    case K_RY:   // Y/2: 2 Im(-i/2 z) = -Re z, 2 Im(i/2 z) = Re z
                        if (al == 0 && clc == 1) g0 -= yr;
                        if (al == 1 && clc == 0) g0 += yr;
                        break;
                    case K_RZ:   // Z/2
                        if (al == clc) g0 += al == 0 ? yi : -yi;
                        break;
                    case K_RZZ:  // ZZ/2
                        if (al == clc) g0 += (al == 0 || al == 3) ? yi : -yi;
                        break;
                    default:     // FSIM: theta (XX+YY)/2 couples 01 and 10 (weight 1); phi |11><11|
                        if ((al == 1 && clc == 2) || (al == 2 && clc == 1)) g0 += 2.0 * yi;
                        if (al == 3 && clc == 3) g1 += 2.0 * yi;
                        break;
                }
            }
            const double s0 = wave_sum(g0);
            if (t == 0) sl[op.slot] = s0;
            if (op.kind == K_FSIM) {
                const double s1 = wave_sum(g1);
                if (t == 0) sl[op.slot + 1] = s1;
            }
        }
        __syncthreads();
        // X_{next} = G_next Y
        if (o + 1 < F.op_end) {
            const Op nx = ops[o + 1];
            const int nd = load_gate(nx, prm, cm, U);
#pragma unroll
            for (int i = 0; i < EPT; ++i) {
                const int e = t + 64 * i, a = e >> KB, c = e & (D - 1);
                const int al = gidx(nx, a, nd);
                c64d acc = {0.0, 0.0};
                for (int be = 0; be < nd; ++be) {
                    const c64d p = cmul(U[al * nd + be], X[gset(nx, a, nd, be) * D + c]);
                    acc.re += p.re;
                    acc.im += p.im;
                }
                x[i] = acc;
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < EPT; ++i) X[t + 64 * i] = x[i];
            __syncthreads();
        }
    }
}


template <int KB>
__global__ void __launch_bounds__(64)
k_fused_grad(const FPhase* __restrict__ phases, const Op* __restrict__ ops, int n_blocks, const float* __restrict__ params,
             int64_t pstride, const cx<float>* __restrict__ cm, const double* __restrict__ osum, int total_slots,
             double* __restrict__ slots) {
    fused_grad_body<KB>(phases, ops, n_blocks, params, pstride, cm, osum, total_slots, slots, int(blockIdx.x),
                    int64_t(blockIdx.y));
}

// uneven batch: circuit blockIdx.y, its phase blockIdx.x
__global__ void __launch_bounds__(64) k_fused_grad_multi(const FusedCircJob* __restrict__ jobs) {
    const FusedCircJob J = jobs[blockIdx.y];
    if (int(blockIdx.x) >= J.n_blocks || J.total_slots <= 0) return;
    fused_grad_body<FUSED_K>(J.phases, J.ops, J.n_blocks, J.params, J.pstride, J.cm, J.osum, J.total_slots, J.slots,
                    int(blockIdx.x), 0);
}
}  // namespace

hipError_t launch_fused_mats(const FPhase* phases, const Op* ops, int n_blocks, const void* params, int64_t pstride,
                             const void* cmats, int64_t cmstride, int64_t batch, void* out, bool want_rev,
                             hipStream_t st, int kb) {
    if (n_blocks == 0 || batch == 0) return hipSuccess;
    if (kb == 5)
        hipLaunchKernelGGL(k_fused_mats<5>, dim3(unsigned(n_blocks), unsigned(batch)), dim3(256), 0, st, phases, ops,
                           n_blocks, static_cast<const float*>(params), pstride, static_cast<const cx<float>*>(cmats),
                           cmstride, static_cast<float*>(out), int(want_rev));
    else
        hipLaunchKernelGGL(k_fused_mats<4>, dim3(unsigned(n_blocks), unsigned(batch)), dim3(256), 0, st, phases, ops,
                           n_blocks, static_cast<const float*>(params), pstride, static_cast<const cx<float>*>(cmats),
                           cmstride, static_cast<float*>(out), int(want_rev));
    return hipGetLastError();
}

// chunks per thread of the tile load: 8 at m = 12 (256 threads), 4 for m = 9..11;
// 32 x 32 blocks only at m = 12
hipError_t launch_fused_fwd(const JobList& jl, const Job& single, int m, int64_t blocks, hipStream_t st, int kb) {
    if (blocks <= 0) return hipSuccess;
    if (kb == 5) {
        if (m != 12) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_fused_fwd<8, 12, 5>), dim3(unsigned(blocks)), dim3(FTHREADS), 0, st, jl, single);
    } else if (m == 12) {
        hipLaunchKernelGGL((k_fused_fwd<8, 12, 4>), dim3(unsigned(blocks)), dim3(FTHREADS), 0, st, jl, single);
    } else {
        hipLaunchKernelGGL((k_fused_fwd<4, 11, 4>), dim3(unsigned(blocks)), dim3(FTHREADS), 0, st, jl, single);
    }
    return hipGetLastError();
}

hipError_t launch_fused_rev(const JobList& jl, const Job& single, int m, int64_t blocks, hipStream_t st, int kb) {
    if (blocks <= 0) return hipSuccess;
    if (kb == 5) {
        if (m != 12) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_fused_rev<8, 12, 5>), dim3(unsigned(blocks)), dim3(FTHREADS), 0, st, jl, single);
    } else if (m == 12) {
        hipLaunchKernelGGL((k_fused_rev<8, 12, 4>), dim3(unsigned(blocks)), dim3(FTHREADS), 0, st, jl, single);
    } else {
        hipLaunchKernelGGL((k_fused_rev<4, 11, 4>), dim3(unsigned(blocks)), dim3(FTHREADS), 0, st, jl, single);
    }
    return hipGetLastError();
}

hipError_t launch_fused_multi_mats(const FusedCircJob* jobs, int count, int max_blocks, hipStream_t st) {
    if (count == 0 || max_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fused_mats_multi, dim3(unsigned(max_blocks), unsigned(count)), dim3(256), 0, st, jobs);
    return hipGetLastError();
}

hipError_t launch_fused_multi_grad(const FusedCircJob* jobs, int count, int max_blocks, hipStream_t st) {
    if (count == 0 || max_blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fused_osum_multi, dim3(unsigned((int64_t(max_blocks) * OSTRIDE + 255) / 256), unsigned(count)),
                       dim3(256), 0, st, jobs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fused_grad_multi, dim3(unsigned(max_blocks), unsigned(count)), dim3(64), 0, st, jobs);
    return hipGetLastError();
}

hipError_t launch_fused_grad(const FPhase* phases, const Op* ops, int n_blocks, const void* params, int64_t pstride,
                             const void* cmats, int64_t batch, const double* opart, int wgs, double* osum,
                             int total_slots, double* slots, hipStream_t st, int kb) {
    if (n_blocks == 0 || batch == 0) return hipSuccess;
    const int64_t rows = batch * int64_t(n_blocks);
    const int os = kb == 5 ? 4 * OSTRIDE : OSTRIDE;
    hipLaunchKernelGGL(k_fused_osum, dim3(unsigned((rows * os + 255) / 256)), dim3(256), 0, st, opart, rows, wgs,
                       osum, os);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (kb == 5)
        hipLaunchKernelGGL(k_fused_grad<5>, dim3(unsigned(n_blocks), unsigned(batch)), dim3(64), 0, st, phases, ops,
                           n_blocks, static_cast<const float*>(params), pstride, static_cast<const cx<float>*>(cmats),
                           osum, total_slots, slots);
    else
        hipLaunchKernelGGL(k_fused_grad<4>, dim3(unsigned(n_blocks), unsigned(batch)), dim3(64), 0, st, phases, ops,
                           n_blocks, static_cast<const float*>(params), pstride, static_cast<const cx<float>*>(cmats),
                           osum, total_slots, slots);
    return hipGetLastError();
}

}  // namespace tcng
