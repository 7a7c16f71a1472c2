// Measurement layer of monitored Haar brick-wall trajectories (paper,
// Sec. "Universal Quantum Dynamics of Haar-Random MIPT"), complex64 states,
// one batch member per trajectory.
//
// A step's measurements are taken qubit by qubit, in increasing order, as the
// three-outcome Kraus channel {sqrt(1-p) I, sqrt(p) P0, sqrt(p) P1} selected by
// one uniform v per (member, step, qubit): measured iff v >= 1 - p, outcome 0
// iff v - (1 - p) < p P(bit q = 0 | the step's earlier outcomes).  The
// projections are not applied one by one: the outcomes decided so far in the
// step (mask, bits) filter the amplitudes of the next marginal, which gives
// the conditional probability as a ratio of the two filtered sums.  The
// step's collapse (zero the inconsistent amplitudes, divide by the square
// root of the kept mass) is applied by the next step's first forward pass as
// it loads its tiles, and after the last step by k_mipt_collapse.
//
//   k_mipt_marg     float64 sums of |psi_x|^2 over the consistent x with bit q
//                   = 0 / = 1, one partial pair per workgroup (HBM-bound read)
//   k_mipt_decide   one thread per member: fixed-order sum of the partials,
//                   the Kraus decision, record, kept mass, ln P(outcome)
//   k_mipt_collapse projection and renormalisation after the last step
//                   (HBM-bound read + write)
// A member that does not measure q leaves its workgroups at once.
#include <hip/hip_runtime.h>

#include "common.h"
#include "devutil.h"
#include "kernels.h"

namespace tcng {
namespace {

constexpr int MTHREADS = 256;

__device__ __forceinline__ bool measures(const double* u, int64_t b, int n_steps, int s, int n, int q, double p) {
    return u[(b * n_steps + s) * n + q] >= 1.0 - p;
}

__global__ void __launch_bounds__(MTHREADS) k_mipt_marg(const float4* __restrict__ psi, int64_t stride4, int n,
                                                        const double* __restrict__ u, int n_steps, int s, int q,
                                                        double p, const uint32_t* __restrict__ rec, int wgs,
                                                        double* __restrict__ part) {
    __shared__ double red[2][MTHREADS / 64];
    const int64_t b = blockIdx.y;
    const int wg = blockIdx.x;
    if (!measures(u, b, n_steps, s, n, q, p)) return;   // the whole workgroup leaves together
    const uint32_t md = rec[(b * n_steps + s) * 2], bd = rec[(b * n_steps + s) * 2 + 1];
    const uint64_t per4 = (uint64_t(1) << n) / 2 / uint64_t(wgs);   // 16-byte chunks (amplitude pairs) per workgroup
    const uint64_t c0 = uint64_t(wg) * per4;
    const float4* src = psi + b * stride4 + c0;
    const uint32_t bq = 1u << q;
    double s0 = 0.0, s1 = 0.0;
    for (uint64_t i = threadIdx.x; i < per4; i += MTHREADS) {
        const uint32_t x = uint32_t(2 * (c0 + i));   // n <= 32: the low word holds every qubit
        const bool k0 = (x & md) == bd, k1 = ((x | 1u) & md) == bd;
        // amplitudes ruled out by the step's earlier outcomes are not read: after j outcomes
        // on qubits above the lowest few, whole lines of the state are skipped (2^-j of it read)
        if (!k0 && !k1) continue;
        const float4 a = src[i];
        const float w0 = a.x * a.x + a.y * a.y, w1 = a.z * a.z + a.w * a.w;
        if (k0) {
            if (x & bq) s1 += double(w0);
            else s0 += double(w0);
        }
        if (k1) {
            if ((x | 1u) & bq) s1 += double(w1);
            else s0 += double(w1);
        }
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][wave] = s0;
        red[1][wave] = s1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t0 = 0.0, t1 = 0.0;
        for (int w = 0; w < MTHREADS / 64; ++w) {
            t0 += red[0][w];
            t1 += red[1][w];
        }
        part[(b * wgs + wg) * 2] = t0;
        part[(b * wgs + wg) * 2 + 1] = t1;
    }
}

__global__ void k_mipt_decide(const double* __restrict__ u, int n, int n_steps, int s, int q, double p, int wgs,
                              const double* __restrict__ part, uint32_t* __restrict__ rec, double* __restrict__ keep,
                              double* __restrict__ logp, double* __restrict__ margin, int64_t batch) {
    const int64_t b = int64_t(blockIdx.x) * 64 + threadIdx.x;
    if (b >= batch) return;
    const double v = u[(b * n_steps + s) * n + q];
    if (v < 1.0 - p) return;
    double s0 = 0.0, s1 = 0.0;
    for (int w = 0; w < wgs; ++w) {
        s0 += part[(b * wgs + w) * 2];
        s1 += part[(b * wgs + w) * 2 + 1];
    }
    const double tot = s0 + s1;
    const double mg = (v - (1.0 - p)) - p * (s0 / tot);
    const int o = mg < 0.0 ? 0 : 1;
    const double kp = o ? s1 : s0;
    logp[b] += log(kp / tot);
    keep[b] = kp;
    uint32_t* r = rec + (b * n_steps + s) * 2;
    r[0] |= 1u << q;
    r[1] |= uint32_t(o) << q;
    if (margin) margin[(b * n_steps + s) * n + q] = mg;
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

__global__ void k_zero_u32(uint32_t* p, size_t count) {
    for (size_t i = size_t(blockIdx.x) * 256 + threadIdx.x; i < count; i += size_t(gridDim.x) * 256) p[i] = 0u;
}

}  // namespace

int mipt_wgs(int n) {
    const uint64_t dim = uint64_t(1) << n;
    return int(std::max<uint64_t>(1, std::min<uint64_t>(256, dim >> 13)));
}

hipError_t launch_mipt_marg(const void* psi, int64_t stride, int n, int64_t batch, const double* u, int n_steps, int s,
                            int q, double p, const uint32_t* rec, int wgs, double* part, hipStream_t st) {
    if (batch == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mipt_marg, dim3(unsigned(wgs), unsigned(batch)), dim3(MTHREADS), 0, st,
                       static_cast<const float4*>(psi), stride / 2, n, u, n_steps, s, q, p, rec, wgs, part);
    return hipGetLastError();
}

hipError_t launch_mipt_decide(const double* u, int n, int n_steps, int s, int q, double p, int wgs, const double* part,
                              uint32_t* rec, double* keep, double* logp, double* margin, int64_t batch,
                              hipStream_t st) {
    if (batch == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mipt_decide, dim3(unsigned((batch + 63) / 64)), dim3(64), 0, st, u, n, n_steps, s, q, p, wgs,
                       part, rec, keep, logp, margin, batch);
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
