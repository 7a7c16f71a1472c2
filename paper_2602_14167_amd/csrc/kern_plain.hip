// Streaming per-gate kernels (the unfused path and tcng_apply_gate), state
// initialisation, and the final fixed-order reductions.
//
// One-qubit gate on qubit q: every amplitude pair (j, j | 2^q) with bit q of
// j clear is multiplied by the 2x2 matrix.  For q >= 1 a thread owns two
// neighbouring pairs, so both halves are read as 16-byte vectors of
// consecutive amplitudes (fully coalesced for every q, including the low
// qubits whose partners sit in the same 64-byte run); for q = 0 the pair is
// itself one 16-byte vector.  Two-qubit gates work on quads the same way.
// Gate matrices are rebuilt per batch member from the device angles, so one
// launch serves every parameter set of a batch (blockIdx.y = member).
#include "gates.h"
#include "kernels.h"

#include <algorithm>

namespace tcng {

namespace {

constexpr int NTHREADS = 256;

__device__ __forceinline__ uint64_t insert0(uint64_t v, int q) {
    const uint64_t lowm = (uint64_t(1) << q) - 1;
    return ((v & ~lowm) << 1) | (v & lowm);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NTHREADS / 64; ++w) s += sh[w];
    return s;
}

// build the (possibly inverted) 2x2 / 4x4 matrix of a gate for batch member b
template <typename R>
__device__ __forceinline__ void gate_mat1(int kind, const R* prm, int p0, const cx<R>* cm, int mat,
                                          const cx<R>* umat, bool inv, cx<R> u[4]) {
    if (umat) {
        u[0] = umat[0]; u[1] = umat[1]; u[2] = umat[2]; u[3] = umat[3];
    } else if (kind_diagonal(kind)) {
        cx<R> d[2];
        diag1<R>(kind, prm, p0, d);
        u[0] = d[0]; u[1] = {R(0), R(0)}; u[2] = {R(0), R(0)}; u[3] = d[1];
    } else {
        mat1<R>(kind, prm, p0, cm, mat, u);
    }
    if (inv) dagger_inplace<R, 2>(u);
}

template <typename R>
__device__ __forceinline__ void gate_mat2(int kind, const R* prm, int p0, int p1, const cx<R>* cm, int mat,
                                          const cx<R>* umat, bool inv, cx<R> u[16]) {
    if (umat) {
#pragma unroll
        for (int i = 0; i < 16; ++i) u[i] = umat[i];
    } else if (kind == K_FSIM || kind == K_U2) {
        mat2<R>(kind, prm, p0, p1, cm, mat, u);
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i) u[i] = {R(0), R(0)};
        if (kind == K_CNOT) {
            u[0] = {R(1), R(0)}; u[5] = {R(1), R(0)}; u[11] = {R(1), R(0)}; u[14] = {R(1), R(0)};
        } else {
            cx<R> d[4];
            diag2<R>(kind, prm, p0, d);
            u[0] = d[0]; u[5] = d[1]; u[10] = d[2]; u[15] = d[3];
        }
    }
    if (inv) dagger_inplace<R, 4>(u);
}

template <typename R>
__device__ __forceinline__ void mv2(const cx<R>* u, cx<R>& a0, cx<R>& a1) {
    const cx<R> x0 = a0, x1 = a1;
    a0 = cfma(u[1], x1, u[0] * x0);
    a1 = cfma(u[3], x1, u[2] * x0);
}

template <typename R>
__device__ __forceinline__ void mv4(const cx<R>* u, cx<R>* x) {
    const cx<R> x0 = x[0], x1 = x[1], x2 = x[2], x3 = x[3];
#pragma unroll
    for (int a = 0; a < 4; ++a) x[a] = cfma(u[4 * a + 3], x3, cfma(u[4 * a + 2], x2, cfma(u[4 * a + 1], x1, u[4 * a] * x0)));
}

// 16-byte streaming access: two complex64 or one complex128 amplitude per
// vector, non-temporal (each amplitude is touched once per gate pass)
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void ld2(const cx<float>* p, cx<float>& a, cx<float>& b) {
    const f4v v = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p));
    a = {v.x, v.y};
    b = {v.z, v.w};
}
__device__ __forceinline__ void st2(cx<float>* p, cx<float> a, cx<float> b) {
    f4v v;
    v.x = a.re; v.y = a.im; v.z = b.re; v.w = b.im;
    __builtin_nontemporal_store(v, reinterpret_cast<f4v*>(p));
}
__device__ __forceinline__ cx<double> ld1(const cx<double>* p) {
    const d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p));
    return {v.x, v.y};
}
__device__ __forceinline__ void st1(cx<double>* p, cx<double> a) {
    d2v v;
    v.x = a.re; v.y = a.im;
    __builtin_nontemporal_store(v, reinterpret_cast<d2v*>(p));
}

// ---------------------------------------------------------------------------
// forward one-qubit gate.  complex64: a thread owns two neighbouring pairs,
// i.e. one 16-byte vector from each half (q >= 1) or two vectors holding two
// pairs (q = 0); complex128: one pair = two 16-byte vectors.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void gate1_unit(cx<float>* psi, uint64_t w, int q, const cx<float>* u) {
    if (q == 0) {
        cx<float> a0, a1, a2, a3;
        ld2(psi + 4 * w, a0, a1);
        ld2(psi + 4 * w + 2, a2, a3);
        mv2(u, a0, a1);
        mv2(u, a2, a3);
        st2(psi + 4 * w, a0, a1);
        st2(psi + 4 * w + 2, a2, a3);
    } else {
        const uint64_t i0 = insert0(2 * w, q);
        cx<float> a0, a1, c0, c1;
        ld2(psi + i0, a0, a1);
        ld2(psi + i0 + (uint64_t(1) << q), c0, c1);
        mv2(u, a0, c0);
        mv2(u, a1, c1);
        st2(psi + i0, a0, a1);
        st2(psi + i0 + (uint64_t(1) << q), c0, c1);
    }
}
__device__ __forceinline__ void gate1_unit(cx<double>* psi, uint64_t w, int q, const cx<double>* u) {
    const uint64_t i0 = insert0(w, q), i1 = i0 | (uint64_t(1) << q);
    cx<double> a0 = ld1(psi + i0), a1 = ld1(psi + i1);
    mv2(u, a0, a1);
    st1(psi + i0, a0);
    st1(psi + i1, a1);
}

template <typename R>
__global__ void __launch_bounds__(NTHREADS)
k_gate1(cx<R>* __restrict__ state, int64_t stride, int n, int q, int kind, int p0, int mat,
        const R* __restrict__ params, int64_t pstride, const cx<R>* __restrict__ cm, const cx<R>* __restrict__ umat,
        int inv) {
    const int64_t b = blockIdx.y;
    cx<R>* psi = state + b * stride;
    cx<R> u[4];
    gate_mat1<R>(kind, params ? params + b * pstride : nullptr, p0, cm, mat, umat, inv != 0, u);
    const uint64_t nunits = (sizeof(R) == 4) ? (uint64_t(1) << (n - 2)) : (uint64_t(1) << (n - 1));
    const uint64_t step = uint64_t(gridDim.x) * blockDim.x;
    uint64_t w = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    // two units in flight per thread
    for (; w + step < nunits; w += 2 * step) {
        gate1_unit(psi, w, q, u);
        gate1_unit(psi, w + step, q, u);
    }
    if (w < nunits) gate1_unit(psi, w, q, u);
}

// one-qubit gates on n = 1 complex64 states (a single pair)
template <typename R>
__global__ void k_gate1_tiny(cx<R>* __restrict__ state, int64_t stride, int q, int kind, int p0, int mat,
                             const R* __restrict__ params, int64_t pstride, const cx<R>* __restrict__ cm,
                             const cx<R>* __restrict__ umat, int inv) {
    const int64_t b = blockIdx.y;
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    cx<R>* psi = state + b * stride;
    cx<R> u[4];
    gate_mat1<R>(kind, params ? params + b * pstride : nullptr, p0, cm, mat, umat, inv != 0, u);
    (void)q;
    cx<R> a0 = psi[0], a1 = psi[1];
    mv2(u, a0, a1);
    psi[0] = a0;
    psi[1] = a1;
}

// ---------------------------------------------------------------------------
// forward two-qubit gate on (q0 = MSB of the local index, q1).  complex64 with
// both qubits >= 1: a thread owns two neighbouring quads (four 16-byte
// vectors); otherwise one quad.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void quad_load(const cx<R>* psi, uint64_t i, uint64_t m0, uint64_t m1, cx<R>* x) {
    x[0] = psi[i]; x[1] = psi[i | m1]; x[2] = psi[i | m0]; x[3] = psi[i | m0 | m1];
}
template <typename R>
__device__ __forceinline__ void quad_store(cx<R>* psi, uint64_t i, uint64_t m0, uint64_t m1, const cx<R>* x) {
    psi[i] = x[0]; psi[i | m1] = x[1]; psi[i | m0] = x[2]; psi[i | m0 | m1] = x[3];
}

template <typename R>
__global__ void __launch_bounds__(NTHREADS)
k_gate2(cx<R>* __restrict__ state, int64_t stride, int n, int q0, int q1, int kind, int p0, int p1, int mat,
        const R* __restrict__ params, int64_t pstride, const cx<R>* __restrict__ cm, const cx<R>* __restrict__ umat,
        int inv) {
    const int64_t b = blockIdx.y;
    cx<R>* psi = state + b * stride;
    cx<R> u[16];
    gate_mat2<R>(kind, params ? params + b * pstride : nullptr, p0, p1, cm, mat, umat, inv != 0, u);
    const int qa = q0 < q1 ? q0 : q1, qb = q0 < q1 ? q1 : q0;
    const uint64_t m0 = uint64_t(1) << q0, m1 = uint64_t(1) << q1;
    const uint64_t nquads = uint64_t(1) << (n - 2);
    const uint64_t step = uint64_t(gridDim.x) * blockDim.x;
    if constexpr (sizeof(R) == 4) {
        if (qa >= 1 && n >= 3) {
            const uint64_t nunits = nquads >> 1;
            for (uint64_t w = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; w < nunits; w += step) {
                const uint64_t i = insert0(insert0(2 * w, qa), qb);   // even: quads i and i + 1
                cx<R> x[4], y[4];
                ld2(psi + i, x[0], y[0]);
                ld2(psi + (i | m1), x[1], y[1]);
                ld2(psi + (i | m0), x[2], y[2]);
                ld2(psi + (i | m0 | m1), x[3], y[3]);
                mv4(u, x);
                mv4(u, y);
                st2(psi + i, x[0], y[0]);
                st2(psi + (i | m1), x[1], y[1]);
                st2(psi + (i | m0), x[2], y[2]);
                st2(psi + (i | m0 | m1), x[3], y[3]);
            }
            return;
        }
    }
    for (uint64_t w = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; w < nquads; w += step) {
        const uint64_t i = insert0(insert0(w, qa), qb);
        cx<R> x[4];
        quad_load(psi, i, m0, m1, x);
        mv4(u, x);
        quad_store(psi, i, m0, m1, x);
    }
}

// generic k-qubit dense matrix (k <= 5), matrix staged in LDS
template <typename R>
__global__ void __launch_bounds__(NTHREADS)
k_gatek(cx<R>* __restrict__ state, int64_t stride, int n, int k, uint64_t qpack, const cx<R>* __restrict__ umat) {
    __shared__ cx<R> U[32 * 32];
    const int kd = 1 << k;
    for (int i = threadIdx.x; i < kd * kd; i += blockDim.x) U[i] = umat[i];
    __syncthreads();
    int q[5], qs[5];
    for (int t = 0; t < k; ++t) q[t] = int((qpack >> (6 * t)) & 63);
    for (int t = 0; t < k; ++t) qs[t] = q[t];
    for (int a = 0; a < k; ++a)          // ascending order for the zero-bit insertion
        for (int c = a + 1; c < k; ++c)
            if (qs[c] < qs[a]) { int tmp = qs[a]; qs[a] = qs[c]; qs[c] = tmp; }
    const int64_t b = blockIdx.y;
    cx<R>* psi = state + b * stride;
    const uint64_t ngroups = uint64_t(1) << (n - k);
    const uint64_t step = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t w = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; w < ngroups; w += step) {
        uint64_t base = w;
        for (int t = 0; t < k; ++t) base = insert0(base, qs[t]);
        cx<R> x[32], y[32];
        for (int a = 0; a < kd; ++a) {
            uint64_t idx = base;
            for (int t = 0; t < k; ++t) idx |= uint64_t((a >> (k - 1 - t)) & 1) << q[t];
            x[a] = psi[idx];
        }
        for (int a = 0; a < kd; ++a) {
            cx<R> s = {R(0), R(0)};
            for (int c = 0; c < kd; ++c) s = cfma(U[a * kd + c], x[c], s);
            y[a] = s;
        }
        for (int a = 0; a < kd; ++a) {
            uint64_t idx = base;
            for (int t = 0; t < k; ++t) idx |= uint64_t((a >> (k - 1 - t)) & 1) << q[t];
            psi[idx] = y[a];
        }
    }
}

// ---------------------------------------------------------------------------
// reverse sweep, one gate: gradient then un-compute psi and lambda
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(NTHREADS)
k_rev1(cx<R>* __restrict__ state, cx<R>* __restrict__ costate, int64_t stride, int n, int q, int kind, int p0,
       int mat, const R* __restrict__ params, int64_t pstride, const cx<R>* __restrict__ cm, int slot, int wgs,
       double* __restrict__ part, int total_slots) {
    __shared__ double sh[NTHREADS / 64];
    const int64_t b = blockIdx.x / wgs;
    const int wg = int(blockIdx.x - b * wgs);
    cx<R>* psi = state + b * stride;
    cx<R>* lam = costate + b * stride;
    cx<R> u[4];
    gate_mat1<R>(kind, params ? params + b * pstride : nullptr, p0, cm, mat, nullptr, true, u);
    const uint64_t npairs = uint64_t(1) << (n - 1);
    double g = 0.0;
    for (uint64_t w = uint64_t(wg) * blockDim.x + threadIdx.x; w < npairs; w += uint64_t(wgs) * blockDim.x) {
        const uint64_t i0 = insert0(w, q), i1 = i0 | (uint64_t(1) << q);
        cx<R> a0 = psi[i0], a1 = psi[i1], l0 = lam[i0], l1 = lam[i1];
        if (slot >= 0) {
            if (kind == K_RX) g += im_conj_mul(l0, a1) + im_conj_mul(l1, a0);
            else if (kind == K_RY) g += re_conj_mul(l1, a0) - re_conj_mul(l0, a1);
            else g += im_conj_mul(l0, a0) - im_conj_mul(l1, a1);   // RZ
        }
        mv2(u, a0, a1);
        mv2(u, l0, l1);
        psi[i0] = a0; psi[i1] = a1; lam[i0] = l0; lam[i1] = l1;
    }
    if (slot >= 0) {
        const double s = block_sum(g, sh);
        if (threadIdx.x == 0) part[(size_t(b) * total_slots + slot) * wgs + wg] = s;
    }
}

template <typename R>
__global__ void __launch_bounds__(NTHREADS)
k_rev2(cx<R>* __restrict__ state, cx<R>* __restrict__ costate, int64_t stride, int n, int q0, int q1, int kind,
       int p0, int p1, int mat, const R* __restrict__ params, int64_t pstride, const cx<R>* __restrict__ cm, int slot,
       int wgs, double* __restrict__ part, int total_slots) {
    __shared__ double sh[NTHREADS / 64];
    const int64_t b = blockIdx.x / wgs;
    const int wg = int(blockIdx.x - b * wgs);
    cx<R>* psi = state + b * stride;
    cx<R>* lam = costate + b * stride;
    cx<R> u[16];
    gate_mat2<R>(kind, params ? params + b * pstride : nullptr, p0, p1, cm, mat, nullptr, true, u);
    const int qa = q0 < q1 ? q0 : q1, qb = q0 < q1 ? q1 : q0;
    const uint64_t m0 = uint64_t(1) << q0, m1 = uint64_t(1) << q1;
    const uint64_t nquads = uint64_t(1) << (n - 2);
    const int nacc = (kind == K_U2) ? 32 : (kind == K_FSIM ? 2 : 1);
    double G[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) G[i] = 0.0;
    for (uint64_t w = uint64_t(wg) * blockDim.x + threadIdx.x; w < nquads; w += uint64_t(wgs) * blockDim.x) {
        const uint64_t i = insert0(insert0(w, qa), qb);
        const uint64_t idx[4] = {i, i | m1, i | m0, i | m0 | m1};
        cx<R> x[4], l[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) { x[a] = psi[idx[a]]; l[a] = lam[idx[a]]; }
        if (slot >= 0) {
            if (kind == K_RZZ) {
                G[0] += im_conj_mul(l[0], x[0]) - im_conj_mul(l[1], x[1]) - im_conj_mul(l[2], x[2]) +
                        im_conj_mul(l[3], x[3]);
            } else if (kind == K_FSIM) {
                G[0] += 2.0 * (im_conj_mul(l[1], x[2]) + im_conj_mul(l[2], x[1]));
                G[1] += 2.0 * im_conj_mul(l[3], x[3]);
            }
        }
        mv4(u, x);
        if (slot >= 0 && kind == K_U2) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    G[2 * (4 * a + c)] += fma(double(l[a].re), double(x[c].re), double(l[a].im) * double(x[c].im));
                    G[2 * (4 * a + c) + 1] += fma(double(l[a].im), double(x[c].re), -double(l[a].re) * double(x[c].im));
                }
        }
        mv4(u, l);
#pragma unroll
        for (int a = 0; a < 4; ++a) { psi[idx[a]] = x[a]; lam[idx[a]] = l[a]; }
    }
    if (slot >= 0) {
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            if (i >= nacc) break;
            const double s = block_sum(G[i], sh);
            if (threadIdx.x == 0) part[(size_t(b) * total_slots + slot + i) * wgs + wg] = s;
        }
    }
}

// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(NTHREADS)
k_init(cx<R>* __restrict__ state, int64_t stride, int n, const cx<R>* __restrict__ amps, int64_t basis) {
    const int64_t b = blockIdx.y;
    cx<R>* psi = state + b * stride;
    const uint64_t dim = uint64_t(1) << n;
    for (uint64_t j = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < dim; j += uint64_t(gridDim.x) * blockDim.x)
        psi[j] = amps ? amps[j] : cx<R>{R(j == uint64_t(basis) ? 1 : 0), R(0)};
}

__global__ void k_zero(double* __restrict__ p, size_t count) {
    for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += size_t(gridDim.x) * blockDim.x)
        p[i] = 0.0;
}

// row sums of the per-workgroup partials: one wave per row, lanes stride the
// row, then a butterfly (fixed order: deterministic)
__global__ void __launch_bounds__(256) k_rowsum(const double* __restrict__ in, int64_t rows, int len,
                                                double* __restrict__ out) {
    const int64_t row = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= rows) return;   // whole wave leaves together
    const double* p = in + size_t(row) * len;
    double v = 0.0;
    for (int i = lane; i < len; i += 64) v += p[i];
    v = wave_sum(v);
    if (lane == 0) out[row] = v;
}

// final sums: one thread per (member, output), fixed order everywhere
// output k of one circuit: k = 0 energy, 1..n_params gradient, then one
// 15-vector of Lie-algebra derivatives per gate (when gate_grad is wanted)
__device__ void finish_one(const FinishJob& F, int64_t k) {
    const double* sl = F.slots;
    if (k == 0) {
        double e = 0.0;
        for (int i = 0; i < F.erows; ++i) e += F.erow[i];
        F.energy[0] = e;
    } else if (k <= F.n_params) {
        const int p = int(k - 1);
        double g = 0.0;
        for (int i = F.slot_ptr[p]; i < F.slot_ptr[p + 1]; ++i) g += sl[F.slot_idx[i]];
        F.grad[p] = g;
    } else {
        // per U2 gate: dE/dalpha_k = Im tr(G^dag P_k U), P_k = sigma_a (x) sigma_b, k = 4a + b - 1
        const int gi = int(k - 1 - F.n_params);
        double* out = F.gate_grad + size_t(gi) * 15;
        const int s0 = F.gate_slot[gi];
        if (s0 < 0) {
            for (int i = 0; i < 15; ++i) out[i] = 0.0;
            return;
        }
        const double* U = F.u2m + size_t(F.gate_mat[gi]) * 32;
        // single-qubit Paulis: entry (r, c) of sigma_a as (re, im)
        auto sig = [](int a, int r, int c, double& re, double& im) {
            re = 0.0; im = 0.0;
            if (a == 0) re = (r == c) ? 1.0 : 0.0;
            else if (a == 1) re = (r != c) ? 1.0 : 0.0;
            else if (a == 2) im = (r == c) ? 0.0 : (r == 0 ? -1.0 : 1.0);
            else re = (r == c) ? (r == 0 ? 1.0 : -1.0) : 0.0;
        };
        for (int kk = 0; kk < 15; ++kk) {
            const int a = (kk + 1) >> 2, c = (kk + 1) & 3;
            double tr_im = 0.0;
            for (int x = 0; x < 4; ++x)
                for (int y = 0; y < 4; ++y) {
                    // (P U)[y][x] = sum_z P[y][z] U[z][x]
                    double pur = 0.0, pui = 0.0;
                    for (int z = 0; z < 4; ++z) {
                        double s1r, s1i, s2r, s2i;
                        sig(a, y >> 1, z >> 1, s1r, s1i);
                        sig(c, y & 1, z & 1, s2r, s2i);
                        const double pr = s1r * s2r - s1i * s2i, pi = s1r * s2i + s1i * s2r;
                        const double ur = U[2 * (4 * z + x)], ui = U[2 * (4 * z + x) + 1];
                        pur += pr * ur - pi * ui;
                        pui += pr * ui + pi * ur;
                    }
                    // conj(G[y][x]) * (PU)[y][x]
                    const double gr = sl[s0 + 2 * (4 * y + x)], gim = sl[s0 + 2 * (4 * y + x) + 1];
                    tr_im += gr * pui - gim * pur;
                }
            out[kk] = tr_im;
        }
    }
}

__global__ void k_finish(const double* __restrict__ slots, int total_slots, const int32_t* __restrict__ slot_ptr,
                         const int32_t* __restrict__ slot_idx, int n_params, const double* __restrict__ erow,
                         int erows, int64_t batch, double* __restrict__ energy, double* __restrict__ grad,
                         double* __restrict__ gate_grad, const int32_t* __restrict__ gate_slot,
                         const double* __restrict__ u2m, const int32_t* __restrict__ gate_mat, int n_gates) {
    const int64_t per = int64_t(1) + n_params + (gate_grad ? int64_t(n_gates) : 0);
    const int64_t tid = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (tid >= per * batch) return;
    const int64_t b = tid / per;
    FinishJob F{};
    F.slots = slots + size_t(b) * total_slots;
    F.erow = erow + size_t(b) * erows;
    F.slot_ptr = slot_ptr;
    F.slot_idx = slot_idx;
    F.gate_slot = gate_slot;
    F.u2m = u2m;
    F.gate_mat = gate_mat;
    F.energy = energy + b;
    F.grad = grad ? grad + size_t(b) * n_params : nullptr;
    F.gate_grad = gate_grad ? gate_grad + size_t(b) * n_gates * 15 : nullptr;
    F.n_params = n_params;
    F.n_gates = n_gates;
    F.erows = erows;
    finish_one(F, tid - b * per);
}

__global__ void k_finish_multi(const FinishJob* __restrict__ jobs, const int64_t* __restrict__ prefix, int njobs,
                               int64_t total) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= total) return;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    finish_one(jobs[lo], i - prefix[lo]);
}

// ---------------------------------------------------------------------------
// chunked one- and two-qubit gates (the state has at least CHUNK_BITS qubits).
// A workgroup owns a chunk of 2^c amplitudes: those whose index bits outside
// a set T of c qubits are fixed, T = the gate's qubits and the lowest other
// qubits.  The chunk moves as 16-byte vectors, thread t taking vectors
// k * 256 + t (k = 0..7), so a wave's 64 vectors are 1 KiB of consecutive
// amplitudes and every access is a full, contiguous wave access; chunks of
// 32 KiB give the grid 2^(n - c) small workgroups, which keep more of HBM
// busy than a persistent grid of large ones.  A gate whose qubits avoid the
// wave's lane bits pairs amplitudes inside a thread's registers (the host
// gives those qubits the local bits of the vector or of k); otherwise the
// chunk goes through LDS once (the low-target case).
// ---------------------------------------------------------------------------
template <typename R>
struct ChunkCfg {
    static constexpr int A = sizeof(R) == 4 ? 2 : 1;          // amplitudes per 16-byte vector
    static constexpr int C = sizeof(R) == 4 ? 12 : 11;        // chunk bits (32 KiB)
    static constexpr int VPT = (1 << C) / A / NTHREADS;       // vectors per thread (8)
    static constexpr int RA = VPT * A;                        // register amplitudes per thread
    static constexpr int TB = sizeof(R) == 4 ? 1 : 0;         // first local bit of the thread index
    static constexpr int KB = TB + 8;                         // first local bit of k
};

struct ChunkMap {
    uint64_t tmask;      // the qubits of T
    int32_t lq[12];      // local bit -> qubit
    int32_t g0, g1;      // local bits of the gate's qubits (q0 = matrix MSB; g1 = -1: one qubit)
};

template <typename R>
__device__ __forceinline__ uint64_t chunk_base(uint64_t chunk, uint64_t tmask, int n) {
    uint64_t base = 0;
    int k = 0;
    for (int q = 0; q < n; ++q) {
        if ((tmask >> q) & 1) continue;
        base |= ((chunk >> k) & 1) << q;
        ++k;
    }
    return base;
}

// global offset of local index l (disjoint bits: OR of the bits' qubits)
template <typename R>
__device__ __forceinline__ uint64_t chunk_off(uint32_t l, const ChunkMap& m) {
    uint64_t g = 0;
#pragma unroll
    for (int i = 0; i < ChunkCfg<R>::C; ++i) g |= uint64_t((l >> i) & 1) << m.lq[i];
    return g;
}

template <typename R>
__device__ __forceinline__ void vload(const cx<R>* p, cx<R>* o);
template <>
__device__ __forceinline__ void vload<float>(const cx<float>* p, cx<float>* o) { ld2(p, o[0], o[1]); }
template <>
__device__ __forceinline__ void vload<double>(const cx<double>* p, cx<double>* o) { o[0] = ld1(p); }
template <typename R>
__device__ __forceinline__ void vstore(cx<R>* p, const cx<R>* o);
template <>
__device__ __forceinline__ void vstore<float>(cx<float>* p, const cx<float>* o) { st2(p, o[0], o[1]); }
template <>
__device__ __forceinline__ void vstore<double>(cx<double>* p, const cx<double>* o) { st1(p, o[0]); }

// register pairing: the gate's qubits sit at register-index bits P0 (matrix
// MSB) and P1 (-1: one qubit) of the thread's RA amplitudes (register index =
// k * A + vector element)
template <typename R, int P0, int P1>
__global__ void __launch_bounds__(NTHREADS)
k_gate_chunk_reg(cx<R>* __restrict__ state, int64_t stride, int n, ChunkMap map, int kind, int p0, int p1, int mat,
                 const R* __restrict__ params, int64_t pstride, const cx<R>* __restrict__ cm,
                 const cx<R>* __restrict__ umat, int inv) {
    using CF = ChunkCfg<R>;
    const int64_t b = blockIdx.y;
    cx<R>* psi = state + b * stride;
    const R* prm = params ? params + b * pstride : nullptr;
    const uint64_t base = chunk_base<R>(blockIdx.x, map.tmask, n);
    const uint64_t lane_off = chunk_off<R>(uint32_t(threadIdx.x) << CF::TB, map);
    cx<R> a[CF::RA];
#pragma unroll
    for (int k = 0; k < CF::VPT; ++k)
        vload<R>(psi + base + lane_off + chunk_off<R>(uint32_t(k) << CF::KB, map), a + k * CF::A);
    if constexpr (P1 < 0) {
        cx<R> u[4];
        gate_mat1<R>(kind, prm, p0, cm, mat, umat, inv != 0, u);
#pragma unroll
        for (int i = 0; i < CF::RA; ++i)
            if (!((i >> P0) & 1)) mv2(u, a[i], a[i | (1 << P0)]);
    } else {
        cx<R> u[16];
        gate_mat2<R>(kind, prm, p0, p1, cm, mat, umat, inv != 0, u);
        constexpr int M0 = 1 << P0, M1 = 1 << P1;
#pragma unroll
        for (int i = 0; i < CF::RA; ++i) {
            if ((i & M0) || (i & M1)) continue;
            cx<R> x[4] = {a[i], a[i | M1], a[i | M0], a[i | M0 | M1]};
            mv4(u, x);
            a[i] = x[0];
            a[i | M1] = x[1];
            a[i | M0] = x[2];
            a[i | M0 | M1] = x[3];
        }
    }
#pragma unroll
    for (int k = 0; k < CF::VPT; ++k)
        vstore<R>(psi + base + lane_off + chunk_off<R>(uint32_t(k) << CF::KB, map), a + k * CF::A);
}

// LDS pairing (a gate qubit among the lane bits): the chunk is staged in LDS
// at its local index; each thread applies the gate to pairs / quads
// j * 256 + t of the local index space, then the chunk is stored back
template <typename R, int NQ>
__global__ void __launch_bounds__(NTHREADS)
k_gate_chunk_lds(cx<R>* __restrict__ state, int64_t stride, int n, ChunkMap map, int kind, int p0, int p1, int mat,
                 const R* __restrict__ params, int64_t pstride, const cx<R>* __restrict__ cm,
                 const cx<R>* __restrict__ umat, int inv) {
    using CF = ChunkCfg<R>;
    __shared__ cx<R> lds[1 << CF::C];
    const int64_t b = blockIdx.y;
    cx<R>* psi = state + b * stride;
    const R* prm = params ? params + b * pstride : nullptr;
    const uint64_t base = chunk_base<R>(blockIdx.x, map.tmask, n);
    const uint32_t t = threadIdx.x;
    const uint64_t lane_off = chunk_off<R>(t << CF::TB, map);
    {
        cx<R> a[CF::RA];
#pragma unroll
        for (int k = 0; k < CF::VPT; ++k)
            vload<R>(psi + base + lane_off + chunk_off<R>(uint32_t(k) << CF::KB, map), a + k * CF::A);
#pragma unroll
        for (int k = 0; k < CF::VPT; ++k)
#pragma unroll
            for (int e = 0; e < CF::A; ++e) lds[((uint32_t(k) << 8 | t) << CF::TB) | uint32_t(e)] = a[k * CF::A + e];
    }
    __syncthreads();
    const int lo = NQ == 2 ? min(map.g0, map.g1) : map.g0, hi = NQ == 2 ? max(map.g0, map.g1) : map.g0;
    const uint32_t m0 = 1u << map.g0, m1 = NQ == 2 ? (1u << map.g1) : 0u;
    if constexpr (NQ == 1) {
        cx<R> u[4];
        gate_mat1<R>(kind, prm, p0, cm, mat, umat, inv != 0, u);
#pragma unroll
        for (int j = 0; j < (1 << CF::C) / 2 / NTHREADS; ++j) {
            const uint32_t i = uint32_t(insert0(uint64_t(j) * NTHREADS + t, lo));
            cx<R> x0 = lds[i], x1 = lds[i | m0];
            mv2(u, x0, x1);
            lds[i] = x0;
            lds[i | m0] = x1;
        }
    } else {
        cx<R> u[16];
        gate_mat2<R>(kind, prm, p0, p1, cm, mat, umat, inv != 0, u);
#pragma unroll
        for (int j = 0; j < (1 << CF::C) / 4 / NTHREADS; ++j) {
            const uint32_t i = uint32_t(insert0(insert0(uint64_t(j) * NTHREADS + t, lo), hi));
            cx<R> x[4] = {lds[i], lds[i | m1], lds[i | m0], lds[i | m0 | m1]};
            mv4(u, x);
            lds[i] = x[0];
            lds[i | m1] = x[1];
            lds[i | m0] = x[2];
            lds[i | m0 | m1] = x[3];
        }
    }
    __syncthreads();
    cx<R> a[CF::RA];
#pragma unroll
    for (int k = 0; k < CF::VPT; ++k)
#pragma unroll
        for (int e = 0; e < CF::A; ++e) a[k * CF::A + e] = lds[((uint32_t(k) << 8 | t) << CF::TB) | uint32_t(e)];
#pragma unroll
    for (int k = 0; k < CF::VPT; ++k)
        vstore<R>(psi + base + lane_off + chunk_off<R>(uint32_t(k) << CF::KB, map), a + k * CF::A);
}

}  // namespace

template <typename R>
static unsigned grid_for(uint64_t work) {
    uint64_t blocks = (work + NTHREADS - 1) / NTHREADS;
    if (blocks > 16384) blocks = 16384;
    if (blocks < 1) blocks = 1;
    return unsigned(blocks);
}

// streaming launches: a persistent-style grid of at most 1024 workgroups per
// batch member (about four per compute unit), each thread looping over units
static unsigned stream_grid(uint64_t units, int64_t batch) {
    uint64_t blocks = (units + NTHREADS - 1) / NTHREADS;
    uint64_t cap = 1024;
    if (batch > 1) cap = std::max<uint64_t>(1, 4096 / uint64_t(batch));
    blocks = std::min(blocks, cap);
    return unsigned(std::max<uint64_t>(blocks, 1));
}

// chunk map and kernel of a one- or two-qubit gate (see k_gate_chunk_reg / _lds)
template <typename R>
static hipError_t launch_gate_chunk(void* state, int64_t stride, int n, int64_t batch, const int* qs, int nq, int kind,
                                    int p0, int p1, int mat, const void* params, int64_t pstride, const void* cmats,
                                    const void* umat, bool inv, hipStream_t st) {
    using CF = ChunkCfg<R>;
    constexpr int LANE_LO = CF::TB, LANE_HI = CF::TB + 5;   // local (= global) bits of a wave's lanes
    bool is_gate[64] = {};
    for (int i = 0; i < nq; ++i) is_gate[qs[i]] = true;
    bool reg = true;
    for (int i = 0; i < nq; ++i)
        if (qs[i] >= LANE_LO && qs[i] <= LANE_HI) reg = false;
    ChunkMap m{};
    int nl = 0;
    auto push = [&](int q) { m.lq[nl++] = q; };
    int next = 0;   // next non-gate qubit candidate
    auto next_other = [&]() {
        while (is_gate[next]) ++next;
        return next++;
    };
    // the k bits not taken by the gate: qubits from c up (a chunk is then 8 runs
    // of 4 KiB spaced 32 KiB apart, the neighbouring chunks filling the gaps,
    // which HBM serves faster than contiguous 32 KiB chunks), then the rest
    int kfill[64], nk = 0;
    for (int q = CF::C; q < n; ++q) kfill[nk++] = q;
    for (int q = 0; q < CF::C && q < n; ++q) kfill[nk++] = q;
    int kf = 0;
    bool used[64] = {};
    auto next_k = [&]() {
        while (is_gate[kfill[kf]] || used[kfill[kf]]) ++kf;
        return kfill[kf++];
    };
    int pos[2] = {-1, -1};
    if (reg) {
        if (CF::TB == 1) {   // complex64: local bit 0 is the vector element, always qubit 0
            if (is_gate[0]) {
                for (int i = 0; i < nq; ++i)
                    if (qs[i] == 0) pos[i] = 0;
                push(0);
            } else {
                push(next_other());
            }
        }
        while (nl < CF::KB) push(next_other());
        for (int i = 0; i < nl; ++i) used[m.lq[i]] = true;
        for (int i = 0; i < nq; ++i)
            if (pos[i] < 0) {
                pos[i] = nl;
                push(qs[i]);
            }
        while (nl < CF::C) push(next_k());
    } else {
        // T = the qubits below the k bits (4 KiB runs), the gate's qubits, the
        // k-bit fill; in increasing order (the lanes keep the lowest qubits)
        bool in_t[64] = {};
        int cnt = 0;
        for (int q = 0; q < CF::KB; ++q) in_t[q] = true, ++cnt;
        for (int i = 0; i < nq; ++i)
            if (!in_t[qs[i]]) in_t[qs[i]] = true, ++cnt;
        for (int q = 0; q < n; ++q) used[q] = in_t[q];
        while (cnt < CF::C) in_t[next_k()] = true, ++cnt;
        for (int q = 0; q < n; ++q)
            if (in_t[q]) {
                for (int i = 0; i < nq; ++i)
                    if (qs[i] == q) pos[i] = nl;
                push(q);
            }
    }
    if (nl != CF::C) return hipErrorInvalidValue;
    for (int i = 0; i < nl; ++i) {
        if (m.lq[i] < 0 || m.lq[i] >= n) return hipErrorInvalidValue;
        m.tmask |= uint64_t(1) << m.lq[i];
    }
    m.g0 = pos[0];
    m.g1 = nq == 2 ? pos[1] : -1;
    const dim3 grid(unsigned(uint64_t(1) << (n - CF::C)), unsigned(batch));
    cx<R>* sp = static_cast<cx<R>*>(state);
    const R* pp = static_cast<const R*>(params);
    const cx<R>* cp = static_cast<const cx<R>*>(cmats);
    const cx<R>* up = static_cast<const cx<R>*>(umat);
    const int iv = int(inv);
    if (!reg) {
        if (nq == 1)
            hipLaunchKernelGGL((k_gate_chunk_lds<R, 1>), grid, dim3(NTHREADS), 0, st, sp, stride, n, m, kind, p0, p1,
                               mat, pp, pstride, cp, up, iv);
        else
            hipLaunchKernelGGL((k_gate_chunk_lds<R, 2>), grid, dim3(NTHREADS), 0, st, sp, stride, n, m, kind, p0, p1,
                               mat, pp, pstride, cp, up, iv);
        return hipGetLastError();
    }
    // register-index bits of the gate's local bits: the vector element (complex64 qubit 0), then k
    constexpr int KSHIFT = CF::TB;   // log2(amplitudes per vector)
    auto rbit = [&](int g) { return g < CF::KB ? g : g - CF::KB + KSHIFT; };
    const int r0 = rbit(m.g0), r1 = nq == 2 ? rbit(m.g1) : -1;
#define TCNG_CHUNK_REG(P0, P1)                                                                                     \
    if (r0 == P0 && r1 == P1) {                                                                                    \
        hipLaunchKernelGGL((k_gate_chunk_reg<R, P0, P1>), grid, dim3(NTHREADS), 0, st, sp, stride, n, m, kind, p0,  \
                           p1, mat, pp, pstride, cp, up, iv);                                                      \
        return hipGetLastError();                                                                                  \
    }
    TCNG_CHUNK_REG(0, -1)
    TCNG_CHUNK_REG(1, -1)
    TCNG_CHUNK_REG(0, 1)
    TCNG_CHUNK_REG(1, 0)
    TCNG_CHUNK_REG(1, 2)
#undef TCNG_CHUNK_REG
    return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_gate1(void* state, int64_t stride, int n, int64_t batch, int q, int kind, int p0, int mat,
                        const void* params, int64_t pstride, const void* cmats, const void* umat, bool inv,
                        hipStream_t st) {
    if (sizeof(R) == 4 && n < 2) {
        hipLaunchKernelGGL((k_gate1_tiny<R>), dim3(1, unsigned(batch)), dim3(64), 0, st, static_cast<cx<R>*>(state),
                           stride, q, kind, p0, mat, static_cast<const R*>(params), pstride,
                           static_cast<const cx<R>*>(cmats), static_cast<const cx<R>*>(umat), int(inv));
        return hipGetLastError();
    }
    if (n >= ChunkCfg<R>::C && batch <= 65535) {
        const int qs[1] = {q};
        return launch_gate_chunk<R>(state, stride, n, batch, qs, 1, kind, p0, -1, mat, params, pstride, cmats, umat,
                                    inv, st);
    }
    const uint64_t units = (sizeof(R) == 4) ? (uint64_t(1) << (n - 2)) : (uint64_t(1) << (n - 1));
    hipLaunchKernelGGL((k_gate1<R>), dim3(stream_grid(units, batch), unsigned(batch)), dim3(NTHREADS), 0, st,
                       static_cast<cx<R>*>(state), stride, n, q, kind, p0, mat, static_cast<const R*>(params), pstride,
                       static_cast<const cx<R>*>(cmats), static_cast<const cx<R>*>(umat), int(inv));
    return hipGetLastError();
}

template <typename R>
hipError_t launch_gate2(void* state, int64_t stride, int n, int64_t batch, int q0, int q1, int kind, int p0, int p1,
                        int mat, const void* params, int64_t pstride, const void* cmats, const void* umat, bool inv,
                        hipStream_t st) {
    if (n >= ChunkCfg<R>::C && batch <= 65535) {
        const int qs[2] = {q0, q1};
        return launch_gate_chunk<R>(state, stride, n, batch, qs, 2, kind, p0, p1, mat, params, pstride, cmats, umat,
                                    inv, st);
    }
    hipLaunchKernelGGL((k_gate2<R>), dim3(stream_grid(uint64_t(1) << (n - 2), batch), unsigned(batch)), dim3(NTHREADS), 0,
                       st, static_cast<cx<R>*>(state), stride, n, q0, q1, kind, p0, p1, mat,
                       static_cast<const R*>(params), pstride, static_cast<const cx<R>*>(cmats),
                       static_cast<const cx<R>*>(umat), int(inv));
    return hipGetLastError();
}

template <typename R>
hipError_t launch_gatek(void* state, int64_t stride, int n, int64_t batch, const int32_t* qubits, int k,
                        const void* umat, hipStream_t st) {
    uint64_t qpack = 0;
    for (int t = 0; t < k; ++t) qpack |= uint64_t(qubits[t]) << (6 * t);
    hipLaunchKernelGGL((k_gatek<R>), dim3(grid_for<R>(uint64_t(1) << (n - k)), unsigned(batch)), dim3(NTHREADS), 0,
                       st, static_cast<cx<R>*>(state), stride, n, k, qpack, static_cast<const cx<R>*>(umat));
    return hipGetLastError();
}

template <typename R>
hipError_t launch_rev1(void* state, void* costate, int64_t stride, int n, int64_t batch, int q, int kind, int p0,
                       int mat, const void* params, int64_t pstride, const void* cmats, int slot, int wgs,
                       double* part, int total_slots, hipStream_t st) {
    hipLaunchKernelGGL((k_rev1<R>), dim3(unsigned(wgs * batch)), dim3(NTHREADS), 0, st, static_cast<cx<R>*>(state),
                       static_cast<cx<R>*>(costate), stride, n, q, kind, p0, mat, static_cast<const R*>(params),
                       pstride, static_cast<const cx<R>*>(cmats), slot, wgs, part, total_slots);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_rev2(void* state, void* costate, int64_t stride, int n, int64_t batch, int q0, int q1, int kind,
                       int p0, int p1, int mat, const void* params, int64_t pstride, const void* cmats, int slot,
                       int wgs, double* part, int total_slots, hipStream_t st) {
    hipLaunchKernelGGL((k_rev2<R>), dim3(unsigned(wgs * batch)), dim3(NTHREADS), 0, st, static_cast<cx<R>*>(state),
                       static_cast<cx<R>*>(costate), stride, n, q0, q1, kind, p0, p1, mat,
                       static_cast<const R*>(params), pstride, static_cast<const cx<R>*>(cmats), slot, wgs, part,
                       total_slots);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_init(void* state, int64_t stride, int n, int64_t batch, const void* amps_in, int64_t basis,
                       hipStream_t st) {
    hipLaunchKernelGGL((k_init<R>), dim3(grid_for<R>(uint64_t(1) << n), unsigned(batch)), dim3(NTHREADS), 0, st,
                       static_cast<cx<R>*>(state), stride, n, static_cast<const cx<R>*>(amps_in), basis);
    return hipGetLastError();
}

hipError_t launch_zero(double* p, size_t count, hipStream_t st) {
    if (count == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero, dim3(unsigned(blocks)), dim3(256), 0, st, p, count);
    return hipGetLastError();
}

hipError_t launch_finish(const double* part, int total_slots, int wgs, const int32_t* slot_ptr,
                         const int32_t* slot_idx, int n_params, const double* epart, int erows, int ewgs,
                         int64_t batch, double* energy, double* grad, double* gate_grad, const int32_t* gate_slot,
                         const double* u2_mats_c128, const int32_t* gate_mat, int n_gates, double* scratch,
                         hipStream_t st) {
    // scratch: [batch][total_slots] slot sums, then [batch][erows] energy row sums
    double* slots = scratch;
    double* erow = scratch + size_t(batch) * total_slots;
    const int64_t srows = batch * int64_t(total_slots), er = batch * int64_t(erows);
    if (srows > 0 && part) {
        hipLaunchKernelGGL(k_rowsum, dim3(unsigned((srows + 3) / 4)), dim3(256), 0, st, part, srows, wgs, slots);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_rowsum, dim3(unsigned((er + 3) / 4)), dim3(256), 0, st, epart, er, ewgs, erow);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t per = 1 + n_params + (gate_grad ? n_gates : 0);
    const int64_t work = per * batch;
    hipLaunchKernelGGL(k_finish, dim3(unsigned((work + 255) / 256)), dim3(256), 0, st, slots, total_slots, slot_ptr,
                       slot_idx, n_params, erow, erows, batch, energy, grad, gate_grad, gate_slot, u2_mats_c128,
                       gate_mat, n_gates);
    return hipGetLastError();
}

hipError_t launch_finish_multi(const double* part, int64_t prows, int wgs, const double* epart, int64_t erows_total,
                               int ewgs, double* slot_sums, double* erow_sums, const FinishJob* jobs,
                               const int64_t* prefix, int njobs, int64_t total, hipStream_t st) {
    if (prows > 0) {
        hipLaunchKernelGGL(k_rowsum, dim3(unsigned((prows + 3) / 4)), dim3(256), 0, st, part, prows, wgs, slot_sums);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (erows_total > 0) {
        hipLaunchKernelGGL(k_rowsum, dim3(unsigned((erows_total + 3) / 4)), dim3(256), 0, st, epart, erows_total, ewgs,
                           erow_sums);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finish_multi, dim3(unsigned((total + 255) / 256)), dim3(256), 0, st, jobs, prefix, njobs,
                       total);
    return hipGetLastError();
}

#define TCNG_INST(R)                                                                                              \
    template hipError_t launch_gate1<R>(void*, int64_t, int, int64_t, int, int, int, int, const void*, int64_t,    \
                                        const void*, const void*, bool, hipStream_t);                             \
    template hipError_t launch_gate2<R>(void*, int64_t, int, int64_t, int, int, int, int, int, int, const void*,   \
                                        int64_t, const void*, const void*, bool, hipStream_t);                    \
    template hipError_t launch_gatek<R>(void*, int64_t, int, int64_t, const int32_t*, int, const void*,            \
                                        hipStream_t);                                                             \
    template hipError_t launch_rev1<R>(void*, void*, int64_t, int, int64_t, int, int, int, int, const void*,       \
                                       int64_t, const void*, int, int, double*, int, hipStream_t);                \
    template hipError_t launch_rev2<R>(void*, void*, int64_t, int, int64_t, int, int, int, int, int, int,          \
                                       const void*, int64_t, const void*, int, int, double*, int, hipStream_t);   \
    template hipError_t launch_init<R>(void*, int64_t, int, int64_t, const void*, int64_t, hipStream_t);
TCNG_INST(float)
TCNG_INST(double)

}  // namespace tcng
