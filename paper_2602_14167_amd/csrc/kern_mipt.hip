// Measurement layer of monitored Haar brick-wall trajectories (paper,
// Sec. "Universal Quantum Dynamics of Haar-Random MIPT"), complex64 states,
// one batch member per trajectory.
//
// A step's measurements are taken qubit by qubit, in increasing order, as the
// three-outcome Kraus channel {sqrt(1-p) I, sqrt(p) P0, sqrt(p) P1} selected by
// one uniform v per (member, step, qubit): measured iff v >= 1 - p, outcome 0
// iff v - (1 - p) < p P(bit q = 0 | the step's earlier outcomes).  Which
// qubits a member measures follows from its uniforms alone, so one read of
// the state gives the joint distribution of up to HK of them (a histogram of
// |psi_x|^2 over their bit patterns), and every conditional probability of
// their sequential decisions is a ratio of sums of its bins.  A member
// measuring more than HK qubits takes them in rounds of HK, each round's read
// filtered by the outcomes of the rounds before (only consistent amplitudes
// are loaded).  The step's collapse (zero the inconsistent amplitudes, divide
// by the square root of the kept mass) is applied by the next step's first
// forward pass as it loads its tiles, and after the last step by
// k_mipt_collapse.
//
//   k_mipt_hist     per workgroup (2^13 consecutive amplitudes): float64 sums
//                   of the consistent |psi_x|^2 per pattern of the round's
//                   qubits inside the chunk, in a fixed order (HBM-bound read)
//   k_mipt_decide   one wave per member: fixed-order sums of the partials into
//                   the joint histogram, the round's decisions in increasing
//                   qubit order, record, kept mass, ln P(outcome)
//   k_mipt_collapse projection and renormalisation after the last step
//                   (HBM-bound read + write)
// A member with no qubit in a round leaves its workgroups at once.
#include <hip/hip_runtime.h>

#include "common.h"
#include "devutil.h"
#include "kernels.h"

namespace tcng {
namespace {

constexpr int MTHREADS = 256;
constexpr int HK = 8;                 // measured qubits per histogram round
constexpr int HBINS = 1 << HK;
constexpr int HCHUNK = 13;            // amplitudes per histogram workgroup: at most 2^13

__device__ __forceinline__ bool measures(const double* u, int64_t b, int n_steps, int s, int n, int q, double p) {
    return u[(b * n_steps + s) * n + q] >= 1.0 - p;
}

// the qubits member b measures in step s with rank [r HK, (r + 1) HK) among them
__device__ __forceinline__ uint32_t round_mask(const double* u, int64_t b, int n_steps, int s, int n, double p, int r) {
    uint32_t m = 0;
    int c = 0;
    for (int q = 0; q < n; ++q)
        if (u[(b * n_steps + s) * n + q] >= 1.0 - p) {
            if (c >= r * HK && c < (r + 1) * HK) m |= 1u << q;
            ++c;
        }
    return m;
}

// the low bits of v deposited at the set bits of mask (lowest first)
__device__ __forceinline__ uint32_t deposit(uint32_t v, uint32_t mask) {
    uint32_t out = 0;
    for (uint32_t mk = mask; mk; mk &= mk - 1) {
        if (v & 1u) out |= mk & (0u - mk);
        v >>= 1;
    }
    return out;
}

// one member's histogram partial of chunk wg (the whole workgroup returns
// together when the member measures nothing in this round)
__device__ __forceinline__ void hist_member(const float4* __restrict__ psi, int64_t stride4, int n,
                                            const double* __restrict__ u, int n_steps, int s, double p, int r,
                                            const uint32_t* __restrict__ rec, int wgs, double* __restrict__ part,
                                            int64_t b, int wg, float* w2, double* red) {
    const uint32_t M = round_mask(u, b, n_steps, s, n, p, r);
    if (!M) return;
    const uint32_t md = rec[(b * n_steps + s) * 2], bd = rec[(b * n_steps + s) * 2 + 1];
    const uint32_t A = (1u << n) / uint32_t(wgs);   // amplitudes of the chunk (<= 2^HCHUNK)
    const uint32_t c0 = uint32_t(wg) * A;
    const float4* src = psi + b * stride4 + c0 / 2;
    // |psi_x|^2 of the chunk into LDS, zero where x contradicts the round's earlier
    // outcomes; every load of the thread in flight before the first use
    constexpr int LMAX = (1 << HCHUNK) / 2 / MTHREADS;   // 16-byte chunks per thread (at most)
    float4 a[LMAX];
#pragma unroll
    for (int k = 0; k < LMAX; ++k) {
        const uint32_t i = threadIdx.x + uint32_t(k) * MTHREADS;
        const uint32_t x = c0 + 2 * i;
        const bool k0 = (x & md) == bd, k1 = ((x | 1u) & md) == bd;
        a[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (i < A / 2 && (k0 || k1)) a[k] = src[i];   // whole lines of amplitudes ruled out are not read
    }
#pragma unroll
    for (int k = 0; k < LMAX; ++k) {
        const uint32_t i = threadIdx.x + uint32_t(k) * MTHREADS;
        if (i >= A / 2) break;
        const uint32_t x = c0 + 2 * i;
        const bool k0 = (x & md) == bd, k1 = ((x | 1u) & md) == bd;
        w2[2 * i] = k0 ? a[k].x * a[k].x + a[k].y * a[k].y : 0.f;
        w2[2 * i + 1] = k1 ? a[k].z * a[k].z + a[k].w * a[k].w : 0.f;
    }
    __syncthreads();
    // bins of the round's qubits inside the chunk: the T threads of bin t / T (kloc <=
    // HK = 8) take the bin's indices f = part_i + k T (f numbers the chunk's free bits),
    // so lanes read neighbouring LDS words; each thread sums its share in increasing k
    const uint32_t mloc = M & (A - 1), free = (A - 1) & ~mloc;
    const int kloc = __popc(mloc);
    const int T = MTHREADS >> kloc;            // threads per bin
    const uint32_t j = threadIdx.x / T, part_i = threadIdx.x % T;
    const uint32_t per = (A >> kloc) / uint32_t(T);   // indices per thread (>= 1 at A >= 2^HK)
    // free_lo: the lowest log2(T) free bits (chosen by part_i), free_hi: the rest (by k)
    uint32_t free_lo = 0, rest = free;
    for (int i = 1; i < T; i <<= 1) {
        free_lo |= rest & (0u - rest);
        rest &= rest - 1u;
    }
    const uint32_t free_hi = free & ~free_lo;
    const uint32_t base = deposit(j, mloc) | deposit(part_i, free_lo);
    uint32_t v = 0;
    double sum = 0.0;
#pragma unroll 4
    for (uint32_t k = 0; k < per; ++k) {
        sum += double(w2[v | base]);
        v = ((v | ~free_hi) + 1u) & free_hi;   // next index of the high free bits, increasing
    }
    // the T shares of a bin: a butterfly over min(T, 64) lanes (every lane adds the
    // same two operands at each level, so all of them hold the same sum), then the
    // bin's waves in increasing order
    const int L = T < 64 ? T : 64;
    for (int off = 1; off < L; off <<= 1) sum += __shfl_xor(sum, off, 64);
    double* out = part + (size_t(b) * wgs + wg) * HBINS;
    if (T <= 64) {
        if (part_i == 0) out[j] = sum;
    } else {
        const int wave = threadIdx.x >> 6, per_bin = T >> 6;
        if ((threadIdx.x & 63) == 0) red[wave] = sum;
        __syncthreads();
        if (threadIdx.x < (1u << kloc)) {
            double t = 0.0;
            for (int k = 0; k < per_bin; ++k) t += red[threadIdx.x * per_bin + k];
            out[threadIdx.x] = t;
        }
    }
}

// round 0: one member per grid row.  Later rounds: the members listed by the
// previous round's decisions (those with a qubit in this round), looped over by
// the grid rows.
__global__ void __launch_bounds__(MTHREADS) k_mipt_hist(const float4* __restrict__ psi, int64_t stride4, int n,
                                                        const double* __restrict__ u, int n_steps, int s, double p,
                                                        int r, const uint32_t* __restrict__ rec, int wgs,
                                                        double* __restrict__ part, const uint32_t* __restrict__ list,
                                                        const uint32_t* __restrict__ cnt) {
    __shared__ float w2[1 << HCHUNK];
    __shared__ double red[MTHREADS / 64];
    if (!list) {
        hist_member(psi, stride4, n, u, n_steps, s, p, r, rec, wgs, part, blockIdx.y, blockIdx.x, w2, red);
        return;
    }
    const uint32_t C = *cnt;
    for (uint32_t i = blockIdx.y; i < C; i += gridDim.y) {
        __syncthreads();   // LDS of the previous member
        hist_member(psi, stride4, n, u, n_steps, s, p, r, rec, wgs, part, list[i], blockIdx.x, w2, red);
    }
}

// one wave per member: joint histogram of the round's qubits (bins: their bits
// in increasing qubit order), then the decisions
__device__ __forceinline__ void decide_member(const double* __restrict__ u, int n, int n_steps, int s, double p,
                                              int r, int wgs, const double* __restrict__ part,
                                              uint32_t* __restrict__ rec, double* __restrict__ keep,
                                              double* __restrict__ logp, double* __restrict__ margin,
                                              uint32_t* __restrict__ list_next, uint32_t* __restrict__ cnt_next,
                                              int64_t b, double* H) {
    const int lane = threadIdx.x;
    const uint32_t M = round_mask(u, b, n_steps, s, n, p, r);
    if (!M) return;
    const int K = __popc(M);
    const uint32_t A = (1u << n) / uint32_t(wgs);
    const uint32_t mloc = M & (A - 1), mhigh = M & ~(A - 1);
    const int kloc = __popc(mloc);
    // bin g: low kloc bits from inside a chunk, the rest from the chunk's base
    for (int g = lane; g < (1 << K); g += 64) {
        const uint32_t lo = uint32_t(g) & ((1u << kloc) - 1), hi = deposit(uint32_t(g) >> kloc, mhigh);
        double t = 0.0;
        for (int w = 0; w < wgs; ++w)
            if (((uint32_t(w) * A) & mhigh) == hi) t += part[(size_t(b) * wgs + w) * HBINS + lo];
        H[g] = t;
    }
    __syncthreads();
    uint32_t* rc = rec + (b * n_steps + s) * 2;
    uint32_t dm = 0, db = 0;   // decided bits (bin positions) and their values
    double lp = 0.0, kp = 0.0;
    int i = 0;
    for (uint32_t mk = M; mk; mk &= mk - 1, ++i) {
        const int q = __ffs(mk) - 1;
        double s0 = 0.0, s1 = 0.0;
        for (int g = lane; g < (1 << K); g += 64) {
            if ((uint32_t(g) & dm) != db) continue;
            if ((g >> i) & 1) s1 += H[g];
            else s0 += H[g];
        }
        s0 = wave_sum(s0);
        s1 = wave_sum(s1);
        const double v = u[(b * n_steps + s) * n + q];
        const double tot = s0 + s1;
        const double mg = (v - (1.0 - p)) - p * (s0 / tot);
        const int o = mg < 0.0 ? 0 : 1;
        kp = o ? s1 : s0;
        lp += log(kp / tot);
        dm |= 1u << i;
        db |= uint32_t(o) << i;
        if (lane == 0) {
            rc[0] |= 1u << q;
            rc[1] |= uint32_t(o) << q;
            if (margin) margin[(b * n_steps + s) * n + q] = mg;
        }
    }
    if (lane == 0) {
        logp[b] += lp;
        keep[b] = kp;
    }
    // members with a qubit in the next round go on its list
    if (list_next && lane == 0 && round_mask(u, b, n_steps, s, n, p, r + 1) != 0u)
        list_next[atomicAdd(cnt_next, 1u)] = uint32_t(b);
}

// round 0: one member per workgroup; later rounds: the listed members.  The
// order of a list depends on scheduling, its content and every member's
// results do not.
__global__ void __launch_bounds__(64) k_mipt_decide(const double* __restrict__ u, int n, int n_steps, int s, double p,
                                                    int r, int wgs, const double* __restrict__ part,
                                                    uint32_t* __restrict__ rec, double* __restrict__ keep,
                                                    double* __restrict__ logp, double* __restrict__ margin,
                                                    const uint32_t* __restrict__ list, const uint32_t* __restrict__ cnt,
                                                    uint32_t* __restrict__ list_next, uint32_t* __restrict__ cnt_next) {
    __shared__ double H[HBINS];
    if (!list) {
        decide_member(u, n, n_steps, s, p, r, wgs, part, rec, keep, logp, margin, list_next, cnt_next, blockIdx.x, H);
        return;
    }
    const uint32_t C = *cnt;
    for (uint32_t i = blockIdx.x; i < C; i += gridDim.x) {
        __syncthreads();
        decide_member(u, n, n_steps, s, p, r, wgs, part, rec, keep, logp, margin, list_next, cnt_next, list[i], H);
    }
}

__global__ void __launch_bounds__(MTHREADS) k_mipt_collapse(float4* __restrict__ psi, int64_t stride4, int n,
                                                            int n_steps, int s, const uint32_t* __restrict__ rec,
                                                            const double* __restrict__ keep, int wgs) {
    const int64_t b = blockIdx.y;
    const uint32_t md = rec[(b * n_steps + s) * 2], bd = rec[(b * n_steps + s) * 2 + 1];
    if (md == 0) return;
    const float sc = float(1.0 / sqrt(keep[b]));
    const uint64_t per4 = (uint64_t(1) << n) / 2 / uint64_t(wgs);
    const uint64_t c0 = uint64_t(blockIdx.x) * per4;
    float4* dst = psi + b * stride4 + c0;
    for (uint64_t i = threadIdx.x; i < per4; i += MTHREADS) {
        const uint32_t x = uint32_t(2 * (c0 + i));
        const float f0 = ((x & md) == bd) ? sc : 0.f, f1 = (((x | 1u) & md) == bd) ? sc : 0.f;
        float4 a = dst[i];
        a.x *= f0;
        a.y *= f0;
        a.z *= f1;
        a.w *= f1;
        dst[i] = a;
    }
}

__global__ void k_reset_counts(uint32_t* lists, int rounds, size_t stride) {
    if (int(threadIdx.x) < rounds) lists[size_t(threadIdx.x) * stride] = 0u;
}

__global__ void k_zero_u32(uint32_t* p, size_t count) {
    for (size_t i = size_t(blockIdx.x) * 256 + threadIdx.x; i < count; i += size_t(gridDim.x) * 256) p[i] = 0u;
}

}  // namespace

int mipt_wgs(int n) {
    const uint64_t dim = uint64_t(1) << n;
    return int(std::max<uint64_t>(1, std::min<uint64_t>(256, dim >> 13)));
}

int mipt_hist_wgs(int n) { return n > HCHUNK ? 1 << (n - HCHUNK) : 1; }
int mipt_rounds(int n) { return (n + HK - 1) / HK; }
size_t mipt_hist_doubles(int n, int64_t batch) { return size_t(batch) * mipt_hist_wgs(n) * HBINS; }

size_t mipt_list_words(int n, int64_t batch) { return size_t(mipt_rounds(n)) * (size_t(batch) + 1); }

// rows of the grid that loop over a later round's member list
static unsigned list_rows(int64_t batch, unsigned cap) { return unsigned(std::min<int64_t>(batch, cap)); }

hipError_t launch_mipt_hist(const void* psi, int64_t stride, int n, int64_t batch, const double* u, int n_steps, int s,
                            double p, int r, const uint32_t* rec, double* part, const uint32_t* lists,
                            hipStream_t st) {
    if (batch == 0) return hipSuccess;
    if (n < HK) return hipErrorInvalidValue;   // a chunk holds at least one index per thread and bin
    const int wgs = mipt_hist_wgs(n);
    const uint32_t* list = r > 0 ? lists + size_t(r) * (batch + 1) + 1 : nullptr;
    const uint32_t* cnt = r > 0 ? lists + size_t(r) * (batch + 1) : nullptr;
    const unsigned rows = r > 0 ? list_rows(batch, 64) : unsigned(batch);
    hipLaunchKernelGGL(k_mipt_hist, dim3(unsigned(wgs), rows), dim3(MTHREADS), 0, st, static_cast<const float4*>(psi),
                       stride / 2, n, u, n_steps, s, p, r, rec, wgs, part, list, cnt);
    return hipGetLastError();
}

hipError_t launch_mipt_decide(const double* u, int n, int n_steps, int s, double p, int r, const double* part,
                              uint32_t* rec, double* keep, double* logp, double* margin, uint32_t* lists,
                              int64_t batch, hipStream_t st) {
    if (batch == 0) return hipSuccess;
    const size_t L = size_t(batch) + 1;
    const uint32_t* list = r > 0 ? lists + size_t(r) * L + 1 : nullptr;
    const uint32_t* cnt = r > 0 ? lists + size_t(r) * L : nullptr;
    const bool next = r + 1 < mipt_rounds(n);
    uint32_t* list_next = next ? lists + size_t(r + 1) * L + 1 : nullptr;
    uint32_t* cnt_next = next ? lists + size_t(r + 1) * L : nullptr;
    const unsigned rows = r > 0 ? list_rows(batch, 1024) : unsigned(batch);
    hipLaunchKernelGGL(k_mipt_decide, dim3(rows), dim3(64), 0, st, u, n, n_steps, s, p, r, mipt_hist_wgs(n), part,
                       rec, keep, logp, margin, list, cnt, list_next, cnt_next);
    return hipGetLastError();
}

// the list counters of rounds 1.. (before a step's round 0)
hipError_t launch_mipt_lists_reset(uint32_t* lists, int n, int64_t batch, hipStream_t st) {
    if (batch == 0 || mipt_rounds(n) < 2) return hipSuccess;
    hipLaunchKernelGGL(k_reset_counts, dim3(1), dim3(64), 0, st, lists, mipt_rounds(n), size_t(batch) + 1);
    return hipGetLastError();
}

hipError_t launch_mipt_collapse(void* psi, int64_t stride, int n, int64_t batch, int n_steps, int s,
                                const uint32_t* rec, const double* keep, int wgs, hipStream_t st) {
    if (batch == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mipt_collapse, dim3(unsigned(wgs), unsigned(batch)), dim3(MTHREADS), 0, st,
                       static_cast<float4*>(psi), stride / 2, n, n_steps, s, rec, keep, wgs);
    return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t* p, size_t count, hipStream_t st) {
    if (count == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero_u32, dim3(unsigned(blocks)), dim3(256), 0, st, p, count);
    return hipGetLastError();
}

}  // namespace tcng
