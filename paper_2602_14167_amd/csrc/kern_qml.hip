// SU(4) brick-wall QML training step (paper, Sec. "End-to-End Pure QML for
// Computer Vision"), complex64 states, float64 gate algebra and reductions.
//
//   k_su4       one workgroup per SU(4) parameter set: U = exp(X),
//               X = -i sum_k theta_k P_k / 2 (P_k = sigma_a (x) sigma_b,
//               k = 4a + b - 1), by its Taylor series after scaling X by 2^-s,
//               and the derivatives dU/dtheta_j by the differentiated series
//               D_m = (D_{m-1} X + T_{m-1} E_j) / m, E_j = -i P_j / 2, carried
//               through the s squarings by the product rule.  Thread
//               16 j + e owns entry e of D_j; threads 240..255 own T and U.
//   k_qml_seed  one workgroup per sample: readout probabilities of the top k
//               index bits (contiguous runs of 2^(n-k) amplitudes), softmax
//               cross entropy of the first C as logits, and the adjoint seed
//               lambda_x = dL/dp_(x >> (n-k)) psi_x of the batch-mean loss
//   k_qml_grad  dL/dtheta_j = 2 Re tr(G^dagger dU/dtheta_j) from the
//               batch-summed cotangent G of every gate
#include <hip/hip_runtime.h>

#include "common.h"
#include "devutil.h"
#include "kernels.h"

namespace tcng {
namespace {

struct cd {
    double re, im;
};
__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }

// entry (r, c) of sigma_a (x) sigma_b, a and b acting on the high and low local bit
__device__ cd pauli2_entry(int a, int b, int r, int c) {
    auto sig = [](int s, int i, int j) -> cd {
        if (s == 0) return {i == j ? 1.0 : 0.0, 0.0};
        if (s == 1) return {i != j ? 1.0 : 0.0, 0.0};
        if (s == 2) return {0.0, i == j ? 0.0 : (i == 0 ? -1.0 : 1.0)};
        return {i == j ? (i == 0 ? 1.0 : -1.0) : 0.0, 0.0};
    };
    return cmul(sig(a, r >> 1, c >> 1), sig(b, r & 1, c & 1));
}

constexpr int TAYLOR = 20;          // terms after scaling to ||X||_inf <= 1/2
constexpr int MAX_SQUARINGS = 64;   // |theta| up to about 2^63

__global__ void __launch_bounds__(256) k_su4(const double* __restrict__ theta, float2* __restrict__ utab,
                                            double* __restrict__ dutab) {
    __shared__ cd X[16], T[16], U[16], E[15][16], D[15][16], L[15][16];
    __shared__ double scale;
    __shared__ int squarings;
    const int g = blockIdx.x, t = threadIdx.x;
    const double* th = theta + size_t(g) * 15;
    const bool dthread = t < 240;
    const int j = t >> 4, e = t & 15, r = e >> 2, c = e & 3;
    // generators and X
    if (dthread) {
        const cd p = pauli2_entry((j + 1) >> 2, (j + 1) & 3, r, c);
        E[j][e] = {0.5 * p.im, -0.5 * p.re};   // -i p / 2
    } else {
        const int ee = t - 240, rr = ee >> 2, cc = ee & 3;
        cd x = {0.0, 0.0};
        for (int k = 0; k < 15; ++k) {
            const cd p = pauli2_entry((k + 1) >> 2, (k + 1) & 3, rr, cc);
            x.re += 0.5 * th[k] * p.im;
            x.im -= 0.5 * th[k] * p.re;
        }
        X[ee] = x;
    }
    __syncthreads();
    if (t == 0) {
        double nrm = 0.0;
        for (int i = 0; i < 4; ++i) {
            double rs = 0.0;
            for (int k = 0; k < 4; ++k) rs += sqrt(X[4 * i + k].re * X[4 * i + k].re + X[4 * i + k].im * X[4 * i + k].im);
            nrm = rs > nrm ? rs : nrm;
        }
        // bounded: an infinite or NaN angle gives a NaN gate, never an endless loop
        int s = 0;
        while (nrm > 0.5 && s < MAX_SQUARINGS) {
            nrm *= 0.5;
            ++s;
        }
        squarings = s;
        scale = ldexp(1.0, -s);
    }
    __syncthreads();
    const double f = scale;
    if (dthread) {
        E[j][e] = {E[j][e].re * f, E[j][e].im * f};
        D[j][e] = {0.0, 0.0};
        L[j][e] = {0.0, 0.0};
    } else {
        const int ee = t - 240;
        X[ee] = {X[ee].re * f, X[ee].im * f};
        T[ee] = {(ee >> 2) == (ee & 3) ? 1.0 : 0.0, 0.0};
        U[ee] = T[ee];
    }
    __syncthreads();
    for (int m = 1; m <= TAYLOR; ++m) {
        cd nv = {0.0, 0.0};
        if (dthread) {
            for (int l = 0; l < 4; ++l) {
                nv = cadd(nv, cmul(D[j][4 * r + l], X[4 * l + c]));
                nv = cadd(nv, cmul(T[4 * r + l], E[j][4 * l + c]));
            }
        } else {
            const int ee = t - 240, rr = ee >> 2, cc = ee & 3;
            for (int l = 0; l < 4; ++l) nv = cadd(nv, cmul(T[4 * rr + l], X[4 * l + cc]));
        }
        const double inv = 1.0 / m;
        nv = {nv.re * inv, nv.im * inv};
        __syncthreads();
        if (dthread) {
            D[j][e] = nv;
            L[j][e] = cadd(L[j][e], nv);
        } else {
            T[t - 240] = nv;
            U[t - 240] = cadd(U[t - 240], nv);
        }
        __syncthreads();
    }
    for (int q = 0; q < squarings; ++q) {
        cd nv = {0.0, 0.0};
        if (dthread) {
            for (int l = 0; l < 4; ++l) {
                nv = cadd(nv, cmul(U[4 * r + l], L[j][4 * l + c]));
                nv = cadd(nv, cmul(L[j][4 * r + l], U[4 * l + c]));
            }
        } else {
            const int ee = t - 240, rr = ee >> 2, cc = ee & 3;
            for (int l = 0; l < 4; ++l) nv = cadd(nv, cmul(U[4 * rr + l], U[4 * l + cc]));
        }
        __syncthreads();
        if (dthread) L[j][e] = nv;
        else U[t - 240] = nv;
        __syncthreads();
    }
    if (dthread) {
        double* d = dutab + (size_t(g) * 15 + j) * 32;
        d[2 * e] = L[j][e].re;
        d[2 * e + 1] = L[j][e].im;
    } else {
        const int ee = t - 240;
        utab[size_t(g) * 16 + ee] = make_float2(float(U[ee].re), float(U[ee].im));
    }
}

__global__ void __launch_bounds__(256) k_qml_seed(const float2* __restrict__ psi, float2* __restrict__ lam,
                                                  int64_t stride, int n, int k, int C, const int32_t* __restrict__ labels,
                                                  double inv_batch, double* __restrict__ loss) {
    __shared__ double red[256];
    __shared__ double dp[256];
    const int64_t b = blockIdx.x;
    const int t = threadIdx.x;
    const int K = 1 << k, tpb = 256 / K;   // threads per readout bin
    const uint64_t R = uint64_t(1) << (n - k);
    const float2* src = psi + b * stride;
    float2* dst = lam + b * stride;
    {
        const int o = t / tpb, part = t % tpb;
        double s = 0.0;
        for (uint64_t i = part; i < R; i += tpb) {
            const float2 a = src[uint64_t(o) * R + i];
            s += double(a.x * a.x + a.y * a.y);
        }
        red[t] = s;
    }
    __syncthreads();
    if (t < K) {
        double p = 0.0;
        for (int i = 0; i < tpb; ++i) p += red[t * tpb + i];
        dp[t] = p;   // probabilities first
    }
    __syncthreads();
    if (t == 0) {
        const int y = labels[b];
        if (y < 0 || y >= C) {
            loss[b] = __longlong_as_double(0x7ff8000000000000LL);   // NaN: label out of range
            for (int o = 0; o < K; ++o) dp[o] = 0.0;
        } else {
            double mx = dp[0];
            for (int o = 1; o < C; ++o) mx = dp[o] > mx ? dp[o] : mx;
            double se = 0.0;
            for (int o = 0; o < C; ++o) se += exp(dp[o] - mx);
            loss[b] = mx + log(se) - dp[y];
            for (int o = 0; o < K; ++o)
                dp[o] = o < C ? (exp(dp[o] - mx) / se - (o == y ? 1.0 : 0.0)) * inv_batch : 0.0;
        }
    }
    __syncthreads();
    const uint64_t dim = uint64_t(1) << n;
    for (uint64_t x = t; x < dim; x += 256) {
        const float w = float(dp[x >> (n - k)]);
        const float2 a = src[x];
        dst[x] = make_float2(w * a.x, w * a.y);
    }
}

__global__ void k_qml_grad(const double* __restrict__ slots, const int32_t* __restrict__ gate_slot,
                           const int32_t* __restrict__ gate_mat, const double* __restrict__ dutab, int n_gates,
                           double* __restrict__ grad) {
    const int gi = blockIdx.x, j = threadIdx.x;
    if (gi >= n_gates || j >= 15) return;
    const int s0 = gate_slot[gi], mi = gate_mat[gi];
    double acc = 0.0;
    if (s0 >= 0) {
        const double* G = slots + s0;
        const double* d = dutab + (size_t(mi) * 15 + j) * 32;
        for (int e = 0; e < 16; ++e) acc += G[2 * e] * d[2 * e] + G[2 * e + 1] * d[2 * e + 1];
    }
    grad[size_t(mi) * 15 + j] = 2.0 * acc;
}

}  // namespace

hipError_t launch_su4(const double* theta, int M, void* utab, double* dutab, hipStream_t st) {
    if (M == 0) return hipSuccess;
    hipLaunchKernelGGL(k_su4, dim3(unsigned(M)), dim3(256), 0, st, theta, static_cast<float2*>(utab), dutab);
    return hipGetLastError();
}

hipError_t launch_qml_seed(const void* psi, void* lam, int64_t stride, int n, int64_t batch, int k, int C,
                           const int32_t* labels, double* loss, hipStream_t st) {
    if (batch == 0) return hipSuccess;
    hipLaunchKernelGGL(k_qml_seed, dim3(unsigned(batch)), dim3(256), 0, st, static_cast<const float2*>(psi),
                       static_cast<float2*>(lam), stride, n, k, C, labels, 1.0 / double(batch), loss);
    return hipGetLastError();
}

hipError_t launch_qml_grad(const double* slots, const int32_t* gate_slot, const int32_t* gate_mat, const double* dutab,
                           int n_gates, double* grad, hipStream_t st) {
    if (n_gates == 0) return hipSuccess;
    hipLaunchKernelGGL(k_qml_grad, dim3(unsigned(n_gates)), dim3(64), 0, st, slots, gate_slot, gate_mat, dutab, n_gates,
                       grad);
    return hipGetLastError();
}

}  // namespace tcng
