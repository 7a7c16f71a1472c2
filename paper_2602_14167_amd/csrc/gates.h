// Device-side gate matrices, built from the gate kind and its angles, and
// the register-resident gate application / adjoint-gradient primitives used
// by the tiled kernels.
//
// Matrices (rows = output local index, q0 = most significant local bit):
//   RX(t) = [[c, -is], [-is, c]],  RY(t) = [[c, -s], [s, c]],  c = cos t/2, s = sin t/2
//   RZ(t) = diag(e^{-it/2}, e^{it/2}),  RZZ(t) = diag(e^{-it/2}, e^{it/2}, e^{it/2}, e^{-it/2})
//   FSIM(t, p): |01>,|10> block [[cos t, -i sin t], [-i sin t, cos t]], |11> -> e^{-ip}
// Gradient of E with respect to an angle of U = exp(-i t G) V is
//   dE/dt = 2 Im <lambda| G |psi>   (psi, lambda: state and costate after the gate)
// with G = P/2 for the Pauli rotations, (XX+YY)/2 and |11><11| for FSIM.
#pragma once

#include "common.h"

namespace tcng {

__device__ __forceinline__ void sc_half(float t, float& c, float& s) { sincosf(0.5f * t, &s, &c); }
__device__ __forceinline__ void sc_half(double t, double& c, double& s) { sincos(0.5 * t, &s, &c); }
__device__ __forceinline__ void sc_full(float t, float& c, float& s) { sincosf(t, &s, &c); }
__device__ __forceinline__ void sc_full(double t, double& c, double& s) { sincos(t, &s, &c); }

// 2x2 matrix of a one-qubit non-diagonal kind
template <typename R>
__device__ __forceinline__ void mat1(int kind, const R* prm, int p0, const cx<R>* cm, int mat, cx<R>* u) {
    const R z = R(0), o = R(1);
    switch (kind) {
        case K_RX: { R c, s; sc_half(prm[p0], c, s); u[0] = {c, z}; u[1] = {z, -s}; u[2] = {z, -s}; u[3] = {c, z}; break; }
        case K_RY: { R c, s; sc_half(prm[p0], c, s); u[0] = {c, z}; u[1] = {-s, z}; u[2] = {s, z}; u[3] = {c, z}; break; }
        case K_H: { const R r = R(0.70710678118654752440); u[0] = {r, z}; u[1] = {r, z}; u[2] = {r, z}; u[3] = {-r, z}; break; }
        case K_X: u[0] = {z, z}; u[1] = {o, z}; u[2] = {o, z}; u[3] = {z, z}; break;
        case K_Y: u[0] = {z, z}; u[1] = {z, -o}; u[2] = {z, o}; u[3] = {z, z}; break;
        default:  // K_U1
            u[0] = cm[16 * mat + 0]; u[1] = cm[16 * mat + 1]; u[2] = cm[16 * mat + 4]; u[3] = cm[16 * mat + 5];
            break;
    }
}

// diagonal of a one-qubit diagonal kind
template <typename R>
__device__ __forceinline__ void diag1(int kind, const R* prm, int p0, cx<R>* d) {
    const R z = R(0), o = R(1);
    switch (kind) {
        case K_RZ: { R c, s; sc_half(prm[p0], c, s); d[0] = {c, -s}; d[1] = {c, s}; break; }
        case K_Z: d[0] = {o, z}; d[1] = {-o, z}; break;
        default:  // K_S
            d[0] = {o, z}; d[1] = {z, o}; break;
    }
}

// diagonal of a two-qubit diagonal kind
template <typename R>
__device__ __forceinline__ void diag2(int kind, const R* prm, int p0, cx<R>* d) {
    const R z = R(0), o = R(1);
    if (kind == K_RZZ) {
        R c, s; sc_half(prm[p0], c, s);
        d[0] = {c, -s}; d[1] = {c, s}; d[2] = {c, s}; d[3] = {c, -s};
    } else {  // K_CZ
        d[0] = {o, z}; d[1] = {o, z}; d[2] = {o, z}; d[3] = {-o, z};
    }
}

// 4x4 matrix of a dense two-qubit kind (FSIM, U2)
template <typename R>
__device__ __forceinline__ void mat2(int kind, const R* prm, int p0, int p1, const cx<R>* cm, int mat, cx<R>* u) {
    if (kind == K_FSIM) {
        const R z = R(0), o = R(1);
        R c, s, cp, sp;
        sc_full(prm[p0], c, s);
        sc_full(prm[p1], cp, sp);
#pragma unroll
        for (int i = 0; i < 16; ++i) u[i] = {z, z};
        u[0] = {o, z};
        u[5] = {c, z}; u[6] = {z, -s};
        u[9] = {z, -s}; u[10] = {c, z};
        u[15] = {cp, -sp};
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i) u[i] = cm[16 * mat + i];
    }
}

template <typename R, int K>
__device__ __forceinline__ void dagger_inplace(cx<R>* u) {
#pragma unroll
    for (int i = 0; i < K; ++i) {
        u[i * K + i] = conj(u[i * K + i]);
#pragma unroll
        for (int j = i + 1; j < K; ++j) {
            cx<R> a = u[i * K + j], b = u[j * K + i];
            u[i * K + j] = conj(b);
            u[j * K + i] = conj(a);
        }
    }
}

// ---------------------------------------------------------------------------
// register-resident application: a register block holds NB = 2^RB amplitudes
// whose local index bits R[0..RB-1] are the bits of the register index j.
// Blocks and matrices are passed and returned by value: with pointer
// arguments the compiler keeps the block in scratch memory.
// ---------------------------------------------------------------------------
template <typename R, int NB>
struct Regs {
    cx<R> v[NB];
};
template <typename R>
struct M2 {
    cx<R> e[4];
};
template <typename R>
struct M4 {
    cx<R> e[16];
};
template <typename R>
struct D4 {
    cx<R> e[4];
};

// per-element selects on named values (no indexed access to a private array)
template <typename R>
__device__ __forceinline__ cx<R> sel(bool c, cx<R> x, cx<R> y) {
    return {c ? x.re : y.re, c ? x.im : y.im};
}

template <typename R, int NB, int B>
__device__ __forceinline__ Regs<R, NB> app_dense1(Regs<R, NB> a, M2<R> u) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if (j & (1 << B)) continue;
        const cx<R> x0 = a.v[j], x1 = a.v[j | (1 << B)];
        a.v[j] = cfma(u.e[1], x1, u.e[0] * x0);
        a.v[j | (1 << B)] = cfma(u.e[3], x1, u.e[2] * x0);
    }
    return a;
}

template <typename R, int NB, int B0, int B1>
__device__ __forceinline__ Regs<R, NB> app_dense2(Regs<R, NB> a, M4<R> u) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if (j & ((1 << B0) | (1 << B1))) continue;
        const int i1 = j | (1 << B1), i2 = j | (1 << B0), i3 = j | (1 << B0) | (1 << B1);
        const cx<R> x0 = a.v[j], x1 = a.v[i1], x2 = a.v[i2], x3 = a.v[i3];
        a.v[j]  = cfma(u.e[3], x3, cfma(u.e[2], x2, cfma(u.e[1], x1, u.e[0] * x0)));
        a.v[i1] = cfma(u.e[7], x3, cfma(u.e[6], x2, cfma(u.e[5], x1, u.e[4] * x0)));
        a.v[i2] = cfma(u.e[11], x3, cfma(u.e[10], x2, cfma(u.e[9], x1, u.e[8] * x0)));
        a.v[i3] = cfma(u.e[15], x3, cfma(u.e[14], x2, cfma(u.e[13], x1, u.e[12] * x0)));
    }
    return a;
}

// real 2x2 matrix (u0 u1; u2 u3) on register bit B: RY, H, X
template <typename R, int NB, int B>
__device__ __forceinline__ Regs<R, NB> app_real1(Regs<R, NB> a, R u0, R u1, R u2, R u3) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if (j & (1 << B)) continue;
        const cx<R> x0 = a.v[j], x1 = a.v[j | (1 << B)];
        a.v[j] = {fmaR(u1, x1.re, u0 * x0.re), fmaR(u1, x1.im, u0 * x0.im)};
        a.v[j | (1 << B)] = {fmaR(u3, x1.re, u2 * x0.re), fmaR(u3, x1.im, u2 * x0.im)};
    }
    return a;
}

// [[c, -i s], [-i s, c]] on register bit B (RX with c = cos t/2, s = sin t/2)
template <typename R, int NB, int B>
__device__ __forceinline__ Regs<R, NB> app_rx(Regs<R, NB> a, R c, R s) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if (j & (1 << B)) continue;
        const cx<R> x0 = a.v[j], x1 = a.v[j | (1 << B)];
        a.v[j] = {fmaR(s, x1.im, c * x0.re), fmaR(-s, x1.re, c * x0.im)};
        a.v[j | (1 << B)] = {fmaR(s, x0.im, c * x1.re), fmaR(-s, x0.re, c * x1.im)};
    }
    return a;
}

// ---------------------------------------------------------------------------
// Rotations by three shears.  A plane rotation
//   R(a) = [[cos a, -sin a], [sin a, cos a]]
// equals the product of shears [[1, -t], [0, 1]] [[1, 0], [s, 1]] [[1, -t], [0, 1]]
// with t = tan(a/2) = sin a / (1 + cos a) and s = sin a (the three-shear
// factorisation of a rotation, also known as lifting).  Applied to a pair of
// reals it is three in-place FMAs and needs no temporary; a direct 2x2 product
// needs four multiplies plus a copy of one operand.  For cos a < 0 the rotation
// is applied as -R(a - pi), keeping |t| <= 1 (every shear is then as well
// conditioned as the direct product); the factor -1 multiplies every amplitude
// of the state alike, so it is carried as one sign per state and applied when
// the state is stored.
//
// RY(t) rotates (re x0, re x1) and (im x0, im x1) by a = t/2.  RX(t) rotates
// (re x0, im x1) by -a and (im x0, re x1) by a.  A phase c + i sigma s rotates
// (re, im) of an amplitude by sigma a: RZ is sigma = -1 on |0>, +1 on |1>.
// ---------------------------------------------------------------------------
template <typename R>
struct Lift {
    R t, s;
};

// shear coefficients of the rotation with cosine c and sine s; toggles `flip`
// when the rotation is taken as -R(a - pi)
template <typename R>
__device__ __forceinline__ Lift<R> lift_of(R c, R s, bool& flip) {
    if (c < R(0)) {
        c = -c;
        s = -s;
        flip = !flip;
    }
    return {s / (R(1) + c), s};
}

template <typename R>
__device__ __forceinline__ void lift(R& x0, R& x1, R t, R s) {
    x0 = fmaR(-t, x1, x0);
    x1 = fmaR(s, x0, x1);
    x0 = fmaR(-t, x1, x0);
}

template <typename R, int NB, int B>
__device__ __forceinline__ Regs<R, NB> app_ry_lift(Regs<R, NB> a, Lift<R> L) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if (j & (1 << B)) continue;
        lift(a.v[j].re, a.v[j | (1 << B)].re, L.t, L.s);
        lift(a.v[j].im, a.v[j | (1 << B)].im, L.t, L.s);
    }
    return a;
}

template <typename R, int NB, int B>
__device__ __forceinline__ Regs<R, NB> app_rx_lift(Regs<R, NB> a, Lift<R> L) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if (j & (1 << B)) continue;
        lift(a.v[j].re, a.v[j | (1 << B)].im, -L.t, -L.s);
        lift(a.v[j].im, a.v[j | (1 << B)].re, L.t, L.s);
    }
    return a;
}

// RZ on register bit B: phase c - i s on bit 0, c + i s on bit 1
template <typename R, int NB, int B>
__device__ __forceinline__ Regs<R, NB> app_rz_lift(Regs<R, NB> a, Lift<R> L) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if (j & (1 << B)) lift(a.v[j].re, a.v[j].im, L.t, L.s);
        else lift(a.v[j].re, a.v[j].im, -L.t, -L.s);
    }
    return a;
}

// the same phase c + i sigma s on every amplitude (RZ on a thread bit)
template <typename R, int NB>
__device__ __forceinline__ Regs<R, NB> app_phase_lift(Regs<R, NB> a, Lift<R> L) {
#pragma unroll
    for (int j = 0; j < NB; ++j) lift(a.v[j].re, a.v[j].im, L.t, L.s);
    return a;
}

// every amplitude j of a register block times its own phase (ph[2j], ph[2j + 1])
// = (cos, sin), or by the conjugate (INV): a product of RZ rotations on the
// block's bits is one phase per amplitude
template <bool INV, typename R, int NB, typename CP>
__device__ __forceinline__ Regs<R, NB> app_phases(Regs<R, NB> a, CP ph) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const R c = ph[2 * j], s = INV ? -ph[2 * j + 1] : ph[2 * j + 1];
        const cx<R> x = a.v[j];
        a.v[j] = {fmaR(x.re, c, -x.im * s), fmaR(x.re, s, x.im * c)};
    }
    return a;
}

// the RZ gradients of all QR bits of a block at once: with v_j = Im(conj(l_j) p_j),
// g_b = sum_j (-1)^{j_b} v_j = T - 2 P_b, T = sum_j v_j, P_b = sum over j with bit b set
template <typename R, int QR>
__device__ __forceinline__ void grad_rz_all(const Regs<R, (1 << QR)>& l, const Regs<R, (1 << QR)>& p, R* g) {
    constexpr int NB = 1 << QR;
    R v[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) v[j] = fmaR(l.v[j].re, p.v[j].im, -l.v[j].im * p.v[j].re);
    R T = R(0);
#pragma unroll
    for (int j = 0; j < NB; ++j) T += v[j];
#pragma unroll
    for (int b = 0; b < QR; ++b) {
        R P = R(0);
#pragma unroll
        for (int j = 0; j < NB; ++j)
            if (j & (1 << b)) P += v[j];
        g[b] = fmaR(R(-2), P, T);
    }
}

// RZ gradient on register bit B: sum_j (-1)^{j_B} Im(conj(l_j) p_j)
template <typename R, int NB, int B>
__device__ __forceinline__ R grad_rz(Regs<R, NB> l, Regs<R, NB> p) {
    R g = R(0);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if (j & (1 << B)) {
            g = fmaR(-l.v[j].re, p.v[j].im, g);
            g = fmaR(l.v[j].im, p.v[j].re, g);
        } else {
            g = fmaR(l.v[j].re, p.v[j].im, g);
            g = fmaR(-l.v[j].im, p.v[j].re, g);
        }
    }
    return g;
}

// sum_j Im(conj(l_j) p_j) (RZ on a thread bit, before its sign)
template <typename R, int NB>
__device__ __forceinline__ R sum_im_conj(Regs<R, NB> l, Regs<R, NB> p) {
    R g = R(0);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        g = fmaR(l.v[j].re, p.v[j].im, g);
        g = fmaR(-l.v[j].im, p.v[j].re, g);
    }
    return g;
}

// diagonal (d0, d1) on register bit B (compile-time selection)
template <typename R, int NB, int B>
__device__ __forceinline__ Regs<R, NB> app_diag1r(Regs<R, NB> a, cx<R> d0, cx<R> d1) {
#pragma unroll
    for (int j = 0; j < NB; ++j) a.v[j] = a.v[j] * ((j & (1 << B)) ? d1 : d0);
    return a;
}

// CNOT with target register bit BT and control register bit BC: a renaming
template <typename R, int NB, int BT, int BC>
__device__ __forceinline__ Regs<R, NB> app_cxr(Regs<R, NB> a) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if ((j & (1 << BT)) || !(j & (1 << BC))) continue;
        const cx<R> t = a.v[j];
        a.v[j] = a.v[j | (1 << BT)];
        a.v[j | (1 << BT)] = t;
    }
    return a;
}

// fSim on register bits (B0 = q0, B1 = q1): |01>,|10> block [[c, -is], [-is, c]],
// |11> multiplied by ph
template <typename R, int NB, int B0, int B1>
__device__ __forceinline__ Regs<R, NB> app_fsim(Regs<R, NB> a, R c, R s, cx<R> ph) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if (j & ((1 << B0) | (1 << B1))) continue;
        const int i1 = j | (1 << B1), i2 = j | (1 << B0), i3 = j | (1 << B0) | (1 << B1);
        const cx<R> x1 = a.v[i1], x2 = a.v[i2];
        a.v[i1] = {fmaR(s, x2.im, c * x1.re), fmaR(-s, x2.re, c * x1.im)};
        a.v[i2] = {fmaR(s, x1.im, c * x2.re), fmaR(-s, x1.re, c * x2.im)};
        a.v[i3] = a.v[i3] * ph;
    }
    return a;
}

// CNOT with the target in register bit B; control either register bit rc
// (rc >= 0) or the thread-constant bit value tb.
template <typename R, int NB, int B>
__device__ __forceinline__ Regs<R, NB> app_cx(Regs<R, NB> a, int rc, int tb) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if (j & (1 << B)) continue;
        const bool c = (rc >= 0 ? ((j >> rc) & 1) : tb) != 0;
        const cx<R> x0 = a.v[j], x1 = a.v[j | (1 << B)];
        a.v[j] = sel(c, x1, x0);
        a.v[j | (1 << B)] = sel(c, x0, x1);
    }
    return a;
}

// diagonal on one bit (d.e[0], d.e[1]) or two bits (d.e[2 b0 + b1])
template <typename R, int NB>
__device__ __forceinline__ Regs<R, NB> app_diag(Regs<R, NB> a, int r0, int tb0, int r1, int tb1, bool two, D4<R> d) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int b0 = r0 >= 0 ? ((j >> r0) & 1) : tb0;
        const int b1 = r1 >= 0 ? ((j >> r1) & 1) : tb1;
        cx<R> f;
        if (two) {
            const cx<R> lo = sel(b1 != 0, d.e[1], d.e[0]), hi = sel(b1 != 0, d.e[3], d.e[2]);
            f = sel(b0 != 0, hi, lo);
        } else {
            f = sel(b0 != 0, d.e[1], d.e[0]);
        }
        a.v[j] = a.v[j] * f;
    }
    return a;
}

// Im(conj(l) * p) and Re(conj(l) * p) in float64 (exact products for float inputs)
template <typename R>
__device__ __forceinline__ double im_conj_mul(cx<R> l, cx<R> p) {
    return fma(double(l.re), double(p.im), -double(l.im) * double(p.re));
}
template <typename R>
__device__ __forceinline__ double re_conj_mul(cx<R> l, cx<R> p) {
    return fma(double(l.re), double(p.re), double(l.im) * double(p.im));
}

// Gradient partial sums of one thread (2^RB products) are accumulated in the
// state's precision R and widened to float64 for the wave / workgroup / tile
// sums.  For complex64 the relative rounding of a thread's partial is at most
// about 2^RB * 2^-24 of the sum of its terms' magnitudes (< 2e-6), far below
// the float32 state's own error.

// dE/dt contribution of RX / RY on register bit B:  Im <l| P |p>
template <typename R, int NB, int B>
__device__ __forceinline__ R grad_rot1(int kind, Regs<R, NB> l, Regs<R, NB> p) {
    R g = R(0);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if (j & (1 << B)) continue;
        const int j1 = j | (1 << B);
        const cx<R> l0 = l.v[j], l1 = l.v[j1], p0 = p.v[j], p1 = p.v[j1];
        if (kind == K_RX) {   // X: (Xp)_0 = p_1, (Xp)_1 = p_0:  Im(conj(l0) p1) + Im(conj(l1) p0)
            g = fmaR(l0.re, p1.im, g);
            g = fmaR(-l0.im, p1.re, g);
            g = fmaR(l1.re, p0.im, g);
            g = fmaR(-l1.im, p0.re, g);
        } else {              // Y: (Yp)_0 = -i p_1, (Yp)_1 = i p_0:  Re(conj(l1) p0) - Re(conj(l0) p1)
            g = fmaR(l1.re, p0.re, g);
            g = fmaR(l1.im, p0.im, g);
            g = fmaR(-l0.re, p1.re, g);
            g = fmaR(-l0.im, p1.im, g);
        }
    }
    return g;
}

// RZ / RZZ: sum_j sign_j Im(conj(l_j) p_j), sign = (-1)^{bit} resp. (-1)^{b0 ^ b1}
template <typename R, int NB>
__device__ __forceinline__ R grad_zdiag(Regs<R, NB> l, Regs<R, NB> p, int r0, int tb0, int r1, int tb1) {
    R gp = R(0), gm = R(0);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int b0 = r0 >= 0 ? ((j >> r0) & 1) : tb0;
        const int b1 = r1 >= 0 ? ((j >> r1) & 1) : tb1;
        const R v = fmaR(l.v[j].re, p.v[j].im, -l.v[j].im * p.v[j].re);
        if (b0 ^ b1) gm += v;
        else gp += v;
    }
    return gp - gm;
}

// FSIM: theta -> 2 Im(conj(l01) p10 + conj(l10) p01), phi -> 2 Im(conj(l11) p11)
template <typename R, int NB, int B0, int B1>
__device__ __forceinline__ void grad_fsim(Regs<R, NB> l, Regs<R, NB> p, R& gt, R& gp) {
    gt = R(0);
    gp = R(0);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if (j & ((1 << B0) | (1 << B1))) continue;
        const int i1 = j | (1 << B1), i2 = j | (1 << B0), i3 = j | (1 << B0) | (1 << B1);
        gt = fmaR(l.v[i1].re, p.v[i2].im, gt);
        gt = fmaR(-l.v[i1].im, p.v[i2].re, gt);
        gt = fmaR(l.v[i2].re, p.v[i1].im, gt);
        gt = fmaR(-l.v[i2].im, p.v[i1].re, gt);
        gp = fmaR(l.v[i3].re, p.v[i3].im, gp);
        gp = fmaR(-l.v[i3].im, p.v[i3].re, gp);
    }
    gt *= R(2);
    gp *= R(2);
}

// U2 cotangent entry (a, b): sum over quads of lambda_a conj(phi_b)
// (phi = state before the gate), real and imaginary part
template <typename R, int NB, int B0, int B1>
__device__ __forceinline__ void cot_u2(Regs<R, NB> l, Regs<R, NB> f, int a, int b, R& re, R& im) {
    re = R(0);
    im = R(0);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        if (j & ((1 << B0) | (1 << B1))) continue;
        const int i1 = j | (1 << B1), i2 = j | (1 << B0), i3 = j | (1 << B0) | (1 << B1);
        const cx<R> la = sel(a == 0, l.v[j], sel(a == 1, l.v[i1], sel(a == 2, l.v[i2], l.v[i3])));
        const cx<R> fb = sel(b == 0, f.v[j], sel(b == 1, f.v[i1], sel(b == 2, f.v[i2], f.v[i3])));
        re = fmaR(la.re, fb.re, re);
        re = fmaR(la.im, fb.im, re);
        im = fmaR(la.im, fb.re, im);
        im = fmaR(-la.re, fb.im, im);
    }
}

}  // namespace tcng
