// Classical-shadow snapshots (paper, Sec. "Efficient ML Pipeline via
// Classical Shadows"), complex64: one batch member per snapshot holds a copy
// of the state, rotated by the fused forward passes of a layer of one-qubit
// gates whose matrices come from the snapshot's Pauli bases, then one basis
// state is drawn from |psi'|^2 by the inverse distribution function.
//
//   k_shadow_mats    basis code -> rotation (X: H, Y: H S^dagger, Z: I), as
//                    the top-left 2 x 2 block of a 4 x 4 table entry
//   k_shadow_chunks  float64 sums of |psi|^2 over chunks of CHUNK amplitudes
//                    (HBM-bound read)
//   k_shadow_pick    one workgroup per snapshot: prefix sums of the chunk sums
//                    (float64 scan in LDS) locate the chunk holding u * total,
//                    prefix sums of the threads' runs inside it locate the
//                    thread, which walks its run to the outcome
#include <hip/hip_runtime.h>

#include "common.h"
#include "devutil.h"
#include "kernels.h"

namespace tcng {
namespace {

constexpr int STHREADS = 256;
constexpr int CHUNK_BITS = 13;   // at least 8192 amplitudes per chunk (32 per thread), at most STHREADS chunks

__global__ void k_shadow_mats(const uint8_t* __restrict__ bases, int n, int64_t S, float2* __restrict__ mats) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;   // (snapshot, qubit)
    if (i >= S * n) return;
    const int b = bases[i];
    const float r = 0.70710678118654752f;
    float2 m[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) m[k] = make_float2(0.f, 0.f);
    if (b == 1) {          // H
        m[0] = make_float2(r, 0.f);
        m[1] = make_float2(r, 0.f);
        m[4] = make_float2(r, 0.f);
        m[5] = make_float2(-r, 0.f);
    } else if (b == 2) {   // H S^dagger = [[r, -i r], [r, i r]]
        m[0] = make_float2(r, 0.f);
        m[1] = make_float2(0.f, -r);
        m[4] = make_float2(r, 0.f);
        m[5] = make_float2(0.f, r);
    } else {               // Z basis (and any code other than 1 and 2)
        m[0] = make_float2(1.f, 0.f);
        m[5] = make_float2(1.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) mats[i * 16 + k] = m[k];
}

__global__ void __launch_bounds__(STHREADS) k_shadow_chunks(const float4* __restrict__ psi, int64_t stride4, int n,
                                                            int nch, double* __restrict__ part) {
    __shared__ double red[STHREADS / 64];
    const int64_t s = blockIdx.y;
    const uint64_t per4 = (uint64_t(1) << n) / 2 / uint64_t(nch);
    const float4* src = psi + s * stride4 + uint64_t(blockIdx.x) * per4;
    double acc = 0.0;
    for (uint64_t i = threadIdx.x; i < per4; i += STHREADS) {
        const float4 a = src[i];
        acc += double(a.x * a.x + a.y * a.y) + double(a.z * a.z + a.w * a.w);
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < STHREADS / 64; ++w) t += red[w];
        part[s * nch + blockIdx.x] = t;
    }
}

// inclusive float64 prefix sum over the workgroup (Hillis-Steele in LDS)
__device__ double wg_scan(double v, double* buf) {
    const int t = threadIdx.x;
    buf[t] = v;
    __syncthreads();
    for (int d = 1; d < STHREADS; d <<= 1) {
        const double add = t >= d ? buf[t - d] : 0.0;
        __syncthreads();
        buf[t] += add;
        __syncthreads();
    }
    return buf[t];
}

__global__ void __launch_bounds__(STHREADS) k_shadow_pick(const float2* __restrict__ psi, int64_t stride, int n,
                                                          int nch, const double* __restrict__ part,
                                                          const double* __restrict__ u, int64_t* __restrict__ out) {
    __shared__ double buf[STHREADS];
    __shared__ int pick;
    __shared__ double below;
    const int64_t s = blockIdx.x;
    const int t = threadIdx.x;
    // one chunk sum per thread (nch <= STHREADS)
    const double cs = t < nch ? part[s * nch + t] : 0.0;
    const double incl = wg_scan(cs, buf);
    const double total = buf[STHREADS - 1];
    const double target = u[s] * total;
    if (t == 0) {
        pick = nch - 1;   // rounding past the last chunk: the last one
        below = total - part[s * nch + nch - 1];
    }
    __syncthreads();
    if (t < nch && incl > target && (t == 0 || incl - cs <= target)) {
        pick = t;
        below = incl - cs;
    }
    __syncthreads();
    const int c = pick;
    const double tc = target - below;   // target inside the chunk
    // the chunk's run of each thread: len = chunk / STHREADS consecutive amplitudes
    const uint64_t clen = (uint64_t(1) << n) / uint64_t(nch);
    const uint64_t len = clen / STHREADS;
    const float2* src = psi + s * stride + uint64_t(c) * clen + uint64_t(t) * len;
    double run = 0.0;
    for (uint64_t i = 0; i < len; ++i) {
        const float2 a = src[i];
        run += double(a.x * a.x + a.y * a.y);
    }
    __syncthreads();
    const double rincl = wg_scan(run, buf);
    if (t == 0) pick = STHREADS - 1;
    __syncthreads();
    if (rincl > tc && (t == 0 || rincl - run <= tc)) pick = t;
    __syncthreads();
    if (t == pick) {
        double acc = rincl - run;
        uint64_t x = len - 1;
        for (uint64_t i = 0; i < len; ++i) {
            const float2 a = src[i];
            acc += double(a.x * a.x + a.y * a.y);
            if (acc > tc) {
                x = i;
                break;
            }
        }
        out[s] = int64_t(uint64_t(c) * clen + uint64_t(t) * len + x);
    }
}

}  // namespace

// chunks of 2^max(13, n - 8) amplitudes: between 1 and STHREADS of them
int shadow_chunks(int n) {
    const int cb = n <= CHUNK_BITS ? n : (n - 8 > CHUNK_BITS ? n - 8 : CHUNK_BITS);
    return 1 << (n - cb);
}

hipError_t launch_shadow_mats(const uint8_t* bases, int n, int64_t S, void* mats, hipStream_t st) {
    if (S == 0) return hipSuccess;
    hipLaunchKernelGGL(k_shadow_mats, dim3(unsigned((S * n + 255) / 256)), dim3(256), 0, st, bases, n, S,
                       static_cast<float2*>(mats));
    return hipGetLastError();
}

hipError_t launch_shadow_chunks(const void* psi, int64_t stride, int n, int64_t S, double* part, hipStream_t st) {
    if (S == 0) return hipSuccess;
    const int nch = shadow_chunks(n);
    hipLaunchKernelGGL(k_shadow_chunks, dim3(unsigned(nch), unsigned(S)), dim3(STHREADS), 0, st,
                       static_cast<const float4*>(psi), stride / 2, n, nch, part);
    return hipGetLastError();
}

hipError_t launch_shadow_pick(const void* psi, int64_t stride, int n, int64_t S, const double* part, const double* u,
                              int64_t* out, hipStream_t st) {
    if (S == 0) return hipSuccess;
    hipLaunchKernelGGL(k_shadow_pick, dim3(unsigned(S)), dim3(STHREADS), 0, st, static_cast<const float2*>(psi),
                       stride, n, shadow_chunks(n), part, u, out);
    return hipGetLastError();
}

}  // namespace tcng
