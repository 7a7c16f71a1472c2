// TEST INFRASTRUCTURE — the CPU oracle.  Only the test-suite, the smoke check
// and the benchmark's CPU-baseline leg may call this code; the product path
// never does.  It shares no code, header or table with the HIP library.
//
// A plain, single-threaded complex128 statevector simulator written from the
// definitions (TensorCircuit-NG paper, Sec. "Foundations Recap"):
//   * a circuit prepares |psi(theta)> = U_D ... U_1 |psi_0>, every gate being a
//     local contraction of a 2^k x 2^k matrix with k legs of the state;
//   * the VQE objective is E(theta) = <psi(theta)| H |psi(theta)> with
//     H = sum_k c_k P_k a sum of Pauli strings (expectation_ps, real part);
//   * the gradient is the reverse-mode derivative of E (the paper's AD), here
//     written out as the textbook adjoint recursion, and independently as the
//     parameter-shift rule that the paper quotes as the 2k-evaluation
//     alternative.
// Every 2^n-term sum is pairwise (recursive halving), never a running sum.
// Compiled with -O2 and no fast-math: IEEE round-to-nearest throughout.
//
// Conventions (readings where the paper is silent):
//   * amplitude index bit q <-> qubit q (qubit 0 is the least significant bit);
//   * for a k-qubit gate on qubits (q_0 .. q_{k-1}) the local matrix index is
//     a = sum_t bit_{q_t} * 2^(k-1-t), i.e. q_0 is the most significant bit;
//   * R_P(theta) = exp(-i theta P / 2); RZZ = exp(-i theta Z(x)Z / 2);
//   * fSim(theta, phi) = [[1,0,0,0],[0,cos,-i sin,0],[0,-i sin,cos,0],[0,0,0,e^{-i phi}]];
//   * Pauli codes 0=I, 1=X, 2=Y, 3=Z.
#include <complex>
#include <vector>
#include <cstdint>
#include <cmath>
#include <cstring>

namespace {

using cplx = std::complex<double>;
const cplx I1(0.0, 1.0);

enum Kind { RX = 0, RY, RZ, H, X, Y, Z, S, CNOT, CZ, RZZ, FSIM, U1, U2, N_KINDS };

struct Gate { int kind, q0, q1, p0, p1, mat; };

int arity(int kind) {
    switch (kind) {
        case CNOT: case CZ: case RZZ: case FSIM: case U2: return 2;
        default: return 1;
    }
}

// ---------------------------------------------------------------------------
// pairwise summation over an index range [lo, hi)
// ---------------------------------------------------------------------------
template <class F>
cplx pairwise_sum(const F& f, uint64_t lo, uint64_t hi) {
    if (hi - lo <= 16) {
        cplx s = 0.0;
        for (uint64_t i = lo; i < hi; ++i) s += f(i);
        return s;
    }
    uint64_t mid = lo + (hi - lo) / 2;
    return pairwise_sum(f, lo, mid) + pairwise_sum(f, mid, hi);
}

// ---------------------------------------------------------------------------
// gate matrices, written from their definitions
// ---------------------------------------------------------------------------
struct Mat4 { cplx m[4][4]; };   // k = 1 uses the top-left 2x2 block

Mat4 zero4() { Mat4 a; for (auto& r : a.m) for (auto& v : r) v = 0.0; return a; }

// exp(-i t P/2) for P in {X, Y, Z}
Mat4 rot1(int pauli, double t) {
    Mat4 a = zero4();
    double c = std::cos(t / 2), s = std::sin(t / 2);
    if (pauli == 1) { a.m[0][0] = c; a.m[0][1] = -I1 * s; a.m[1][0] = -I1 * s; a.m[1][1] = c; }
    if (pauli == 2) { a.m[0][0] = c; a.m[0][1] = -s;      a.m[1][0] = s;       a.m[1][1] = c; }
    if (pauli == 3) { a.m[0][0] = std::exp(-I1 * (t / 2)); a.m[1][1] = std::exp(I1 * (t / 2)); }
    return a;
}

Mat4 gate_matrix(const Gate& g, const double* params, const cplx* mats) {
    Mat4 a = zero4();
    const double r2 = 1.0 / std::sqrt(2.0);
    switch (g.kind) {
        case RX: return rot1(1, params[g.p0]);
        case RY: return rot1(2, params[g.p0]);
        case RZ: return rot1(3, params[g.p0]);
        case H:  a.m[0][0] = r2; a.m[0][1] = r2; a.m[1][0] = r2; a.m[1][1] = -r2; return a;
        case X:  a.m[0][1] = 1.0; a.m[1][0] = 1.0; return a;
        case Y:  a.m[0][1] = -I1; a.m[1][0] = I1; return a;
        case Z:  a.m[0][0] = 1.0; a.m[1][1] = -1.0; return a;
        case S:  a.m[0][0] = 1.0; a.m[1][1] = I1; return a;
        case CNOT:  // control = q0 (MSB), target = q1
            a.m[0][0] = 1.0; a.m[1][1] = 1.0; a.m[2][3] = 1.0; a.m[3][2] = 1.0; return a;
        case CZ: a.m[0][0] = 1.0; a.m[1][1] = 1.0; a.m[2][2] = 1.0; a.m[3][3] = -1.0; return a;
        case RZZ: {
            double t = params[g.p0];
            cplx em = std::exp(-I1 * (t / 2)), ep = std::exp(I1 * (t / 2));
            a.m[0][0] = em; a.m[1][1] = ep; a.m[2][2] = ep; a.m[3][3] = em; return a;
        }
        case FSIM: {
            double t = params[g.p0], p = params[g.p1];
            a.m[0][0] = 1.0;
            a.m[1][1] = std::cos(t); a.m[1][2] = -I1 * std::sin(t);
            a.m[2][1] = -I1 * std::sin(t); a.m[2][2] = std::cos(t);
            a.m[3][3] = std::exp(-I1 * p);
            return a;
        }
        case U1: case U2:
            for (int i = 0; i < 4; ++i)
                for (int j = 0; j < 4; ++j) a.m[i][j] = mats[16 * g.mat + 4 * i + j];
            return a;
    }
    return a;
}

// d U / d(param role r) for the parameterised kinds, differentiated by hand
// from the closed forms above (r = 0: params[p0], r = 1: params[p1]).
Mat4 gate_matrix_derivative(const Gate& g, int r, const double* params) {
    Mat4 a = zero4();
    switch (g.kind) {
        case RX: { double t = params[g.p0], c = std::cos(t / 2), s = std::sin(t / 2);
            a.m[0][0] = -s / 2; a.m[0][1] = -I1 * (c / 2); a.m[1][0] = -I1 * (c / 2); a.m[1][1] = -s / 2;
            return a; }
        case RY: { double t = params[g.p0], c = std::cos(t / 2), s = std::sin(t / 2);
            a.m[0][0] = -s / 2; a.m[0][1] = -c / 2; a.m[1][0] = c / 2; a.m[1][1] = -s / 2;
            return a; }
        case RZ: { double t = params[g.p0];
            a.m[0][0] = (-I1 / 2.0) * std::exp(-I1 * (t / 2));
            a.m[1][1] = (I1 / 2.0) * std::exp(I1 * (t / 2));
            return a; }
        case RZZ: { double t = params[g.p0];
            cplx dm = (-I1 / 2.0) * std::exp(-I1 * (t / 2)), dp = (I1 / 2.0) * std::exp(I1 * (t / 2));
            a.m[0][0] = dm; a.m[1][1] = dp; a.m[2][2] = dp; a.m[3][3] = dm;
            return a; }
        case FSIM: {
            double t = params[g.p0], p = params[g.p1];
            if (r == 0) {
                a.m[1][1] = -std::sin(t); a.m[1][2] = -I1 * std::cos(t);
                a.m[2][1] = -I1 * std::cos(t); a.m[2][2] = -std::sin(t);
            } else {
                a.m[3][3] = -I1 * std::exp(-I1 * p);
            }
            return a;
        }
    }
    return a;
}

// ---------------------------------------------------------------------------
// gate application: psi'_j = sum_b U[a(j)][b] psi_{j with gate bits := b}
// ---------------------------------------------------------------------------
void apply_matrix(int n, std::vector<cplx>& psi, const int* q, int k, const Mat4& U) {
    const uint64_t dim = uint64_t(1) << n;
    const int kdim = 1 << k;
    std::vector<cplx> out(dim);
    for (uint64_t j = 0; j < dim; ++j) {
        int a = 0;
        for (int t = 0; t < k; ++t) a |= int((j >> q[t]) & 1) << (k - 1 - t);
        uint64_t rest = j;
        for (int t = 0; t < k; ++t) rest &= ~(uint64_t(1) << q[t]);
        cplx s = 0.0;
        for (int b = 0; b < kdim; ++b) {
            uint64_t src = rest;
            for (int t = 0; t < k; ++t) src |= uint64_t((b >> (k - 1 - t)) & 1) << q[t];
            s += U.m[a][b] * psi[src];
        }
        out[j] = s;
    }
    psi.swap(out);
}

// the same definition for a general k-qubit matrix (row-major 2^k x 2^k)
void apply_dense(int n, std::vector<cplx>& psi, const int* q, int k, const std::vector<cplx>& U) {
    const uint64_t dim = uint64_t(1) << n;
    const int kdim = 1 << k;
    std::vector<cplx> out(dim);
    for (uint64_t j = 0; j < dim; ++j) {
        int a = 0;
        for (int t = 0; t < k; ++t) a |= int((j >> q[t]) & 1) << (k - 1 - t);
        uint64_t rest = j;
        for (int t = 0; t < k; ++t) rest &= ~(uint64_t(1) << q[t]);
        cplx s = 0.0;
        for (int b = 0; b < kdim; ++b) {
            uint64_t src = rest;
            for (int t = 0; t < k; ++t) src |= uint64_t((b >> (k - 1 - t)) & 1) << q[t];
            s += U[size_t(a) * kdim + b] * psi[src];
        }
        out[j] = s;
    }
    psi.swap(out);
}

Mat4 dagger(const Mat4& U) {
    Mat4 a;
    for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) a.m[i][j] = std::conj(U.m[j][i]);
    return a;
}

Mat4 matmul(const Mat4& A, const Mat4& B, int kdim) {
    Mat4 c = zero4();
    for (int i = 0; i < kdim; ++i)
        for (int j = 0; j < kdim; ++j)
            for (int l = 0; l < kdim; ++l) c.m[i][j] += A.m[i][l] * B.m[l][j];
    return c;
}

void apply_gate(int n, std::vector<cplx>& psi, const Gate& g, const Mat4& U) {
    int q[2] = {g.q0, g.q1};
    apply_matrix(n, psi, q, arity(g.kind), U);
}

// ---------------------------------------------------------------------------
// Pauli strings, applied qubit by qubit from the single-qubit actions
//   X|b> = |1-b>,  Y|b> = i (-1)^b |1-b>,  Z|b> = (-1)^b |b>.
// P|k> = phase(k) |image(k)>.
// ---------------------------------------------------------------------------
struct PauliTerm { std::vector<std::pair<int, int>> ops; double coeff; };  // (qubit, code)

void pauli_on_basis(const PauliTerm& t, uint64_t k, uint64_t& image, cplx& phase) {
    image = k;
    phase = 1.0;
    for (auto& op : t.ops) {
        int b = int((k >> op.first) & 1);
        if (op.second == 1) { image ^= uint64_t(1) << op.first; }
        else if (op.second == 2) { image ^= uint64_t(1) << op.first; phase *= (b ? -I1 : I1); }
        else if (op.second == 3) { if (b) phase = -phase; }
    }
}

std::vector<PauliTerm> read_terms(int n, const uint8_t* codes, const double* coeffs, int T) {
    std::vector<PauliTerm> terms(T);
    for (int t = 0; t < T; ++t) {
        terms[t].coeff = coeffs[t];
        for (int q = 0; q < n; ++q)
            if (codes[size_t(t) * n + q]) terms[t].ops.push_back({q, int(codes[size_t(t) * n + q])});
    }
    return terms;
}

// <psi|H|psi> (complex; its imaginary part is a check that should vanish)
cplx expectation(int n, const std::vector<cplx>& psi, const std::vector<PauliTerm>& terms) {
    const uint64_t dim = uint64_t(1) << n;
    cplx e = 0.0;
    for (auto& t : terms) {
        auto f = [&](uint64_t k) {
            uint64_t img; cplx ph;
            pauli_on_basis(t, k, img, ph);
            return std::conj(psi[img]) * ph * psi[k];
        };
        e += t.coeff * pairwise_sum(f, 0, dim);
    }
    return e;
}

// lambda = H psi
std::vector<cplx> apply_hamiltonian(int n, const std::vector<cplx>& psi, const std::vector<PauliTerm>& terms) {
    const uint64_t dim = uint64_t(1) << n;
    std::vector<cplx> lam(dim, 0.0);
    for (auto& t : terms)
        for (uint64_t k = 0; k < dim; ++k) {
            uint64_t img; cplx ph;
            pauli_on_basis(t, k, img, ph);
            lam[img] += t.coeff * ph * psi[k];
        }
    return lam;
}

cplx inner(const std::vector<cplx>& a, const std::vector<cplx>& b) {   // <a|b>
    auto f = [&](uint64_t k) { return std::conj(a[k]) * b[k]; };
    return pairwise_sum(f, 0, a.size());
}

std::vector<Gate> read_gates(const int32_t* g, int G) {
    std::vector<Gate> out(G);
    for (int i = 0; i < G; ++i)
        out[i] = Gate{g[6 * i], g[6 * i + 1], g[6 * i + 2], g[6 * i + 3], g[6 * i + 4], g[6 * i + 5]};
    return out;
}

std::vector<cplx> read_mats(const double* mats, int n_mats) {
    std::vector<cplx> m(size_t(n_mats) * 16);
    for (size_t i = 0; i < m.size(); ++i) m[i] = cplx(mats[2 * i], mats[2 * i + 1]);
    return m;
}

std::vector<cplx> initial_state(int n, const double* init) {
    const uint64_t dim = uint64_t(1) << n;
    std::vector<cplx> psi(dim, 0.0);
    if (init) for (uint64_t k = 0; k < dim; ++k) psi[k] = cplx(init[2 * k], init[2 * k + 1]);
    else psi[0] = 1.0;
    return psi;
}

void write_state(const std::vector<cplx>& psi, double* out) {
    for (size_t k = 0; k < psi.size(); ++k) { out[2 * k] = psi[k].real(); out[2 * k + 1] = psi[k].imag(); }
}

std::vector<cplx> forward(int n, const std::vector<Gate>& gates, const double* params,
                          const std::vector<cplx>& mats, const double* init) {
    std::vector<cplx> psi = initial_state(n, init);
    for (auto& g : gates) apply_gate(n, psi, g, gate_matrix(g, params, mats.data()));
    return psi;
}

// two-qubit Pauli sigma_a (x) sigma_b in the local basis (a on the MSB)
Mat4 pauli2(int a, int b) {
    Mat4 s[4];
    for (auto& m : s) m = zero4();
    s[0].m[0][0] = 1.0; s[0].m[1][1] = 1.0;
    s[1].m[0][1] = 1.0; s[1].m[1][0] = 1.0;
    s[2].m[0][1] = -I1; s[2].m[1][0] = I1;
    s[3].m[0][0] = 1.0; s[3].m[1][1] = -1.0;
    Mat4 r = zero4();
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) r.m[i][j] = s[a].m[i >> 1][j >> 1] * s[b].m[i & 1][j & 1];
    return r;
}

// exp(-i t P/2) for a two-qubit Pauli P (P^2 = I): cos(t/2) I - i sin(t/2) P
Mat4 pauli2_rotation(int a, int b, double t) {
    Mat4 P = pauli2(a, b), r = zero4();
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) r.m[i][j] = (i == j ? std::cos(t / 2) : 0.0) - I1 * std::sin(t / 2) * P.m[i][j];
    return r;
}

// E for the circuit with gate `which` replaced by L * U_which (L a 4x4 / 2x2 matrix)
double energy_with_left_factor(int n, const std::vector<Gate>& gates, const double* params,
                               const std::vector<cplx>& mats, const double* init,
                               const std::vector<PauliTerm>& terms, int which, const Mat4& L) {
    std::vector<cplx> psi = initial_state(n, init);
    for (int i = 0; i < int(gates.size()); ++i) {
        Mat4 U = gate_matrix(gates[i], params, mats.data());
        if (i == which) U = matmul(L, U, 1 << arity(gates[i].kind));
        apply_gate(n, psi, gates[i], U);
    }
    return expectation(n, psi, terms).real();
}

double energy_with_param(int n, const std::vector<Gate>& gates, std::vector<double> params_shifted,
                         const std::vector<cplx>& mats, const double* init,
                         const std::vector<PauliTerm>& terms, int which, int role, double shift) {
    // shift only the angle of gate `which` (role 0: p0, role 1: p1), even if
    // other gates share the same parameter: copy it into a private slot
    std::vector<Gate> g2 = gates;
    int p = role == 0 ? gates[which].p0 : gates[which].p1;
    params_shifted.push_back(params_shifted[p] + shift);
    if (role == 0) g2[which].p0 = int(params_shifted.size()) - 1;
    else g2[which].p1 = int(params_shifted.size()) - 1;
    std::vector<cplx> psi = forward(n, g2, params_shifted.data(), mats, init);
    return expectation(n, psi, terms).real();
}

}  // namespace

// ---------------------------------------------------------------------------
// SU(4) gate of the QML ansatz (Sec. "End-to-End Pure QML for Computer
// Vision", the su4 gate): U(theta) = exp(X), X = -i sum_k theta_k P_k / 2,
// P_k = sigma_a (x) sigma_b, k = 4a + b - 1 (sigma_a on the gate's first
// qubit).  The exponential is its Taylor series after scaling X by 2^-s
// (||X|| <= 1/2), then s squarings; the derivative in direction
// E_j = -i P_j / 2 follows the differentiated recurrence
// D_m = (D_{m-1} X + T_{m-1} E) / m beside T_m = T_{m-1} X / m, and the
// product rule through the squarings.
// ---------------------------------------------------------------------------
struct SU4 { Mat4 U; Mat4 dU[15]; };

Mat4 madd(const Mat4& a, const Mat4& b) {
    Mat4 c;
    for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) c.m[i][j] = a.m[i][j] + b.m[i][j];
    return c;
}
Mat4 mscale(const Mat4& a, cplx f) {
    Mat4 c;
    for (int i = 0; i < 4; ++i) for (int j = 0; j < 4; ++j) c.m[i][j] = a.m[i][j] * f;
    return c;
}

SU4 su4_gate(const double* th) {
    Mat4 X = zero4();
    Mat4 E[15];
    for (int k = 0; k < 15; ++k) {
        const int a = (k + 1) >> 2, b = (k + 1) & 3;
        E[k] = mscale(pauli2(a, b), cplx(0.0, -0.5));
        X = madd(X, mscale(E[k], th[k]));
    }
    double nrm = 0.0;
    for (int i = 0; i < 4; ++i) {
        double r = 0.0;
        for (int j = 0; j < 4; ++j) r += std::abs(X.m[i][j]);
        nrm = std::max(nrm, r);
    }
    int sq = 0;
    while (nrm > 0.5) { nrm *= 0.5; ++sq; }
    const double f = std::ldexp(1.0, -sq);
    X = mscale(X, f);
    for (auto& e : E) e = mscale(e, f);
    Mat4 I = zero4();
    for (int i = 0; i < 4; ++i) I.m[i][i] = 1.0;
    SU4 r;
    Mat4 T = I;
    r.U = I;
    Mat4 D[15];
    for (int k = 0; k < 15; ++k) { D[k] = zero4(); r.dU[k] = zero4(); }
    for (int m = 1; m <= 24; ++m) {
        for (int k = 0; k < 15; ++k) {
            D[k] = mscale(madd(matmul(D[k], X, 4), matmul(T, E[k], 4)), 1.0 / m);
            r.dU[k] = madd(r.dU[k], D[k]);
        }
        T = mscale(matmul(T, X, 4), 1.0 / m);
        r.U = madd(r.U, T);
    }
    for (int t = 0; t < sq; ++t) {
        for (int k = 0; k < 15; ++k) r.dU[k] = madd(matmul(r.U, r.dU[k], 4), matmul(r.dU[k], r.U, 4));
        r.U = matmul(r.U, r.U, 4);
    }
    return r;
}

extern "C" {

int orc_version() { return 1; }

// State after the circuit.  init: nullable interleaved complex [2^n] (else |0..0>).
int orc_run(int n, const int32_t* gates, int G, const double* params, const double* mats, int n_mats,
            const double* init, double* out) {
    auto g = read_gates(gates, G);
    auto m = read_mats(mats, n_mats);
    write_state(forward(n, g, params, m, init), out);
    return 0;
}

// Apply one k-qubit matrix (1 <= k <= 6, row-major 2^k x 2^k, interleaved complex) in place.
int orc_apply_matrix(int n, double* state, const int32_t* qubits, int k, const double* U) {
    if (k < 1 || k > 6 || k > n) return 1;
    std::vector<cplx> psi = initial_state(n, state);
    const int kd = 1 << k;
    std::vector<cplx> M(size_t(kd) * kd);
    for (size_t i = 0; i < M.size(); ++i) M[i] = cplx(U[2 * i], U[2 * i + 1]);
    apply_dense(n, psi, qubits, k, M);
    write_state(psi, state);
    return 0;
}

// Matrix of one gate record (4x4 interleaved; one-qubit gates fill the top-left 2x2).
int orc_gate_matrix(const int32_t* gate, const double* params, const double* mats, int n_mats, double* out) {
    Gate g{gate[0], gate[1], gate[2], gate[3], gate[4], gate[5]};
    auto m = read_mats(mats, n_mats);
    Mat4 U = gate_matrix(g, params, m.data());
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) { out[2 * (4 * i + j)] = U.m[i][j].real(); out[2 * (4 * i + j) + 1] = U.m[i][j].imag(); }
    return 0;
}

// E = <psi|H|psi>; out[0] = Re, out[1] = Im (should be ~0).
int orc_expect(int n, const double* state, const uint8_t* codes, const double* coeffs, int T, double* out) {
    std::vector<cplx> psi = initial_state(n, state);
    cplx e = expectation(n, psi, read_terms(n, codes, coeffs, T));
    out[0] = e.real(); out[1] = e.imag();
    return 0;
}

// lambda = H psi
int orc_apply_hamiltonian(int n, const double* state, const uint8_t* codes, const double* coeffs, int T, double* out) {
    std::vector<cplx> psi = initial_state(n, state);
    write_state(apply_hamiltonian(n, psi, read_terms(n, codes, coeffs, T)), out);
    return 0;
}

double orc_norm2(int n, const double* state) {
    std::vector<cplx> psi = initial_state(n, state);
    return inner(psi, psi).real();
}

// Adjoint-method value and gradient.
//   energy[0] = Re E, energy[1] = Im E
//   grad[n_params]       : dE/dtheta_p summed over every gate using theta_p
//   gate_cot (nullable)  : per gate the 4x4 cotangent G_g = sum_rest lambda_g phi_{g-1}^dagger
//                          (lambda_g = U_{g+1}^dag..U_D^dag H psi_D, phi_{g-1} the state before
//                          gate g), so that dE = 2 Re tr(G_g^dag dU_g); one-qubit gates fill 2x2
//   lie (nullable)       : per gate 15 values dE/dalpha_k for U_g -> exp(-i alpha_k P_k/2) U_g,
//                          P_k = sigma_a (x) sigma_b, k = 4a + b - 1 (two-qubit gates only)
//   final_state (nullable): psi_D
int orc_expect_grad(int n, const int32_t* gates, int G, const double* params, int n_params,
                    const double* mats, int n_mats, const uint8_t* codes, const double* coeffs, int T,
                    const double* init, double* energy, double* grad, double* gate_cot, double* lie,
                    double* final_state) {
    auto g = read_gates(gates, G);
    auto m = read_mats(mats, n_mats);
    auto terms = read_terms(n, codes, coeffs, T);
    std::vector<cplx> psi = forward(n, g, params, m, init);
    if (final_state) write_state(psi, final_state);
    std::vector<cplx> lam = apply_hamiltonian(n, psi, terms);
    cplx e = inner(psi, lam);
    energy[0] = e.real(); energy[1] = e.imag();
    for (int p = 0; p < n_params; ++p) grad[p] = 0.0;
    const uint64_t dim = uint64_t(1) << n;
    for (int i = G - 1; i >= 0; --i) {
        const Gate& gi = g[i];
        const int k = arity(gi.kind), kd = 1 << k;
        Mat4 U = gate_matrix(gi, params, m.data());
        Mat4 Ud = dagger(U);
        std::vector<cplx> phi = psi;          // state before gate i
        apply_gate(n, phi, gi, Ud);
        const int roles = (gi.kind == FSIM) ? 2 : ((gi.kind == RX || gi.kind == RY || gi.kind == RZ || gi.kind == RZZ) ? 1 : 0);
        for (int r = 0; r < roles; ++r) {
            std::vector<cplx> t = phi;
            apply_gate(n, t, gi, gate_matrix_derivative(gi, r, params));
            grad[r == 0 ? gi.p0 : gi.p1] += 2.0 * inner(lam, t).real();
        }
        if (gate_cot || lie) {
            Mat4 Gc = zero4();
            int q[2] = {gi.q0, gi.q1};
            for (int a = 0; a < kd; ++a)
                for (int b = 0; b < kd; ++b) {
                    auto f = [&](uint64_t j) {
                        // j runs over the 2^(n-k) indices with the gate bits cleared,
                        // enumerated by inserting zero bits at the gate positions
                        uint64_t base = 0, jj = j;
                        for (int bit = 0, used = 0; bit < n; ++bit) {
                            bool isg = false;
                            for (int t = 0; t < k; ++t) isg |= (q[t] == bit);
                            if (isg) continue;
                            base |= ((jj >> used) & 1) << bit;
                            ++used;
                        }
                        uint64_t ia = base, ib = base;
                        for (int t = 0; t < k; ++t) {
                            ia |= uint64_t((a >> (k - 1 - t)) & 1) << q[t];
                            ib |= uint64_t((b >> (k - 1 - t)) & 1) << q[t];
                        }
                        return lam[ia] * std::conj(phi[ib]);
                    };
                    Gc.m[a][b] = pairwise_sum(f, 0, dim >> k);
                }
            if (gate_cot)
                for (int a = 0; a < 4; ++a)
                    for (int b = 0; b < 4; ++b) {
                        gate_cot[32 * i + 2 * (4 * a + b)] = Gc.m[a][b].real();
                        gate_cot[32 * i + 2 * (4 * a + b) + 1] = Gc.m[a][b].imag();
                    }
            if (lie) {
                for (int kk = 0; kk < 15; ++kk) lie[15 * i + kk] = 0.0;
                if (k == 2) {
                    // dE/dalpha = 2 Re tr(G^dag dU), dU = -i (P/2) U  =>  Im tr(G^dag P U)
                    for (int kk = 0; kk < 15; ++kk) {
                        int a = (kk + 1) >> 2, b = (kk + 1) & 3;
                        Mat4 PU = matmul(pauli2(a, b), U, 4);
                        cplx tr = 0.0;
                        for (int x = 0; x < 4; ++x)
                            for (int y = 0; y < 4; ++y) tr += std::conj(Gc.m[y][x]) * PU.m[y][x];
                        lie[15 * i + kk] = tr.imag();
                    }
                }
            }
        }
        apply_gate(n, lam, gi, Ud);
        psi.swap(phi);
    }
    return 0;
}

// Parameter-shift gradient (exact for these gates): for a gate generated by
// P/2 with P^2 = I, dE/dtheta = (E(theta + pi/2) - E(theta - pi/2)) / 2.
// fSim's phi generator |11><11| has eigenvalues {0, 1}: same two-term rule.
// fSim's theta generator (XX + YY)/2 has three eigenvalues; because XX and YY
// commute, exp(-i theta (XX+YY)/2) = exp(-i theta XX/2) exp(-i theta YY/2) and
// the rule is applied to each factor; a shift of one factor equals a left
// factor exp(-i s XX/2) (resp. YY) on the whole gate.
// lie (nullable): per two-qubit gate the 15 shifted-generator derivatives.
int orc_param_shift(int n, const int32_t* gates, int G, const double* params, int n_params,
                    const double* mats, int n_mats, const uint8_t* codes, const double* coeffs, int T,
                    const double* init, double* grad, double* lie) {
    auto g = read_gates(gates, G);
    auto m = read_mats(mats, n_mats);
    auto terms = read_terms(n, codes, coeffs, T);
    std::vector<double> pv(params, params + n_params);
    const double h = M_PI / 2;
    for (int p = 0; p < n_params; ++p) grad[p] = 0.0;
    for (int i = 0; i < G; ++i) {
        const Gate& gi = g[i];
        switch (gi.kind) {
            case RX: case RY: case RZ: case RZZ:
                grad[gi.p0] += 0.5 * (energy_with_param(n, g, pv, m, init, terms, i, 0, h) -
                                      energy_with_param(n, g, pv, m, init, terms, i, 0, -h));
                break;
            case FSIM:
                grad[gi.p0] += 0.5 * (energy_with_left_factor(n, g, params, m, init, terms, i, pauli2_rotation(1, 1, h)) -
                                      energy_with_left_factor(n, g, params, m, init, terms, i, pauli2_rotation(1, 1, -h)));
                grad[gi.p0] += 0.5 * (energy_with_left_factor(n, g, params, m, init, terms, i, pauli2_rotation(2, 2, h)) -
                                      energy_with_left_factor(n, g, params, m, init, terms, i, pauli2_rotation(2, 2, -h)));
                grad[gi.p1] += 0.5 * (energy_with_param(n, g, pv, m, init, terms, i, 1, h) -
                                      energy_with_param(n, g, pv, m, init, terms, i, 1, -h));
                break;
            default: break;
        }
        if (lie) {
            for (int kk = 0; kk < 15; ++kk) lie[15 * i + kk] = 0.0;
            if (arity(gi.kind) == 2)
                for (int kk = 0; kk < 15; ++kk) {
                    int a = (kk + 1) >> 2, b = (kk + 1) & 3;
                    lie[15 * i + kk] = 0.5 * (energy_with_left_factor(n, g, params, m, init, terms, i, pauli2_rotation(a, b, h)) -
                                              energy_with_left_factor(n, g, params, m, init, terms, i, pauli2_rotation(a, b, -h)));
                }
        }
    }
    return 0;
}

// Monitored Haar circuit, one trajectory (Sec. "Universal Quantum Dynamics of
// Haar-Random MIPT"): every time step applies its two-qubit gates in order,
// then a layer of single-qubit Z measurements, each qubit measured with
// probability p.  The measurement is the three-outcome Kraus channel
// {sqrt(1-p) I, sqrt(p) P0, sqrt(p) P1} picked with one uniform v per
// (step, qubit), qubits in increasing order:
//   v < 1 - p                        -> not measured;
//   v - (1 - p) <  p * P(bit q = 0)  -> outcome 0;  otherwise outcome 1,
// P taken on the current (already collapsed, normalised) state; the state is
// projected on the outcome and renormalised, and ln P(outcome) is added to
// the trajectory's Born log-probability.
//   gates [G_step]: the step's gates; gate g of step s uses matrix
//                   mats[s * n_step_mats + g.mat] (complex128 4x4, row-major);
//   u [n_steps][n]; force (nullable) [n_steps][n]: -1 free, 0 / 1 = take
//   this outcome (the margin is still reported);
//   rec [n_steps][2]: measured-qubit mask, outcome bits;
//   margin (nullable) [n_steps][n]: v - (1 - p) - p P(0) for measured
//   qubits, NaN otherwise.
int orc_mipt(int n, const int32_t* gates, int G, int n_steps, const double* mats, int n_step_mats,
             const double* init, const double* u, double p, const int32_t* force, double* out_state,
             uint32_t* rec, double* logp, double* margin) {
    if (n < 1 || n > 30) return 1;
    auto g = read_gates(gates, G);
    for (auto& gi : g)
        if (gi.kind != U2 || gi.mat < 0 || gi.mat >= n_step_mats) return 2;
    auto m = read_mats(mats, n_steps * n_step_mats);
    std::vector<cplx> psi = initial_state(n, init);
    const uint64_t dim = uint64_t(1) << n;
    double lp = 0.0;
    for (int s = 0; s < n_steps; ++s) {
        for (auto& gi : g) {
            Mat4 U = zero4();
            const cplx* src = m.data() + (size_t(s) * n_step_mats + gi.mat) * 16;
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) U.m[a][b] = src[4 * a + b];
            apply_gate(n, psi, gi, U);
        }
        uint32_t mask = 0, bits = 0;
        for (int q = 0; q < n; ++q) {
            const double v = u[size_t(s) * n + q];
            if (margin) margin[size_t(s) * n + q] = std::nan("");
            if (v < 1.0 - p) continue;
            const uint64_t bq = uint64_t(1) << q;
            auto w0 = [&](uint64_t k) { return cplx((k & bq) ? 0.0 : std::norm(psi[k]), 0.0); };
            auto w1 = [&](uint64_t k) { return cplx((k & bq) ? std::norm(psi[k]) : 0.0, 0.0); };
            const double s0 = pairwise_sum(w0, 0, dim).real(), s1 = pairwise_sum(w1, 0, dim).real();
            const double p0 = s0 / (s0 + s1);
            const double mg = (v - (1.0 - p)) - p * p0;
            if (margin) margin[size_t(s) * n + q] = mg;
            int o = mg < 0.0 ? 0 : 1;
            if (force && force[size_t(s) * n + q] >= 0) o = force[size_t(s) * n + q];
            const double keep = o ? s1 : s0;
            lp += std::log(keep / (s0 + s1));
            const double sc = 1.0 / std::sqrt(keep);
            for (uint64_t k = 0; k < dim; ++k) psi[k] = (((k & bq) != 0) == (o != 0)) ? psi[k] * sc : cplx(0.0, 0.0);
            mask |= uint32_t(1) << q;
            bits |= uint32_t(o) << q;
        }
        rec[2 * s] = mask;
        rec[2 * s + 1] = bits;
    }
    write_state(psi, out_state);
    *logp = lp;
    return 0;
}

// Sparse (COO) matrix of a Pauli sum (Sec. "Lattice and Hamiltonian", the
// PauliStringSum2COO construction): every term P_k maps a basis state |col>
// to phase |col xor x_k>, so H[row][col] = sum_k c_k <row|P_k|col> is nonzero
// only at col = row xor x_k.  Terms are grouped by X-mask, groups in the order
// their mask first appears in the term list; one entry per (group, row) for
// rows [row_begin, row_begin + row_count), group-major, the value the sum over
// the group's terms (taken from the qubit-by-qubit action, in term order; an
// exact zero is kept).  n_groups receives the group count.
int orc_pauli_coo(int n, const uint8_t* codes, const double* coeffs, int T, int64_t row_begin, int64_t row_count,
                  int64_t* rows, int64_t* cols, double* vals, int* n_groups) {
    auto terms = read_terms(n, codes, coeffs, T);
    std::vector<uint64_t> xs;
    std::vector<int> group_of(T);
    for (int k = 0; k < T; ++k) {
        uint64_t img;
        cplx ph;
        pauli_on_basis(terms[k], 0, img, ph);   // the X-mask is the image of |0>
        int g = 0;
        while (g < int(xs.size()) && xs[g] != img) ++g;
        if (g == int(xs.size())) xs.push_back(img);
        group_of[k] = g;
    }
    *n_groups = int(xs.size());
    for (int g = 0; g < int(xs.size()); ++g)
        for (int64_t r = 0; r < row_count; ++r) {
            const uint64_t row = uint64_t(row_begin + r), col = row ^ xs[g];
            cplx v = 0.0;
            for (int k = 0; k < T; ++k) {
                if (group_of[k] != g) continue;
                uint64_t img;
                cplx ph;
                pauli_on_basis(terms[k], col, img, ph);
                if (img != row) return 1;
                v += terms[k].coeff * ph;
            }
            const size_t e = size_t(g) * size_t(row_count) + size_t(r);
            rows[e] = int64_t(row);
            cols[e] = int64_t(col);
            vals[2 * e] = v.real();
            vals[2 * e + 1] = v.imag();
        }
    return 0;
}

// Classical-shadow snapshots (Sec. "Efficient ML Pipeline via Classical
// Shadows", shadow_snapshots with measurement only): snapshot s measures
// every qubit q in the Pauli basis bases[s][q] (1 = X, 2 = Y, 3 = Z): the
// state is rotated by V_q (X: H; Y: H S^dagger; Z: identity), so that Z
// outcome 0 is the +1 eigenvector of the chosen Pauli, and one basis state x
// is drawn from |psi'_x|^2 by the inverse distribution function with the
// uniform u[s]: the first x whose running sum of probabilities (in increasing
// x, normalised by the total) exceeds u[s].
//   out[s]: the outcome x (bit q = outcome of qubit q);
//   lo / hi (nullable) [s]: the running sums just before and at x.
int orc_shadow(int n, const double* psi_in, int S, const uint8_t* bases, const double* u, int64_t* out, double* lo,
               double* hi) {
    if (n < 1 || n > 30) return 1;
    const uint64_t dim = uint64_t(1) << n;
    const double r = 1.0 / std::sqrt(2.0);
    Mat4 VX = zero4(), VY = zero4();
    VX.m[0][0] = r; VX.m[0][1] = r; VX.m[1][0] = r; VX.m[1][1] = -r;
    VY.m[0][0] = r; VY.m[0][1] = cplx(0.0, -r); VY.m[1][0] = r; VY.m[1][1] = cplx(0.0, r);   // H S^dagger
    const std::vector<cplx> psi0 = initial_state(n, psi_in);
    for (int s = 0; s < S; ++s) {
        std::vector<cplx> psi = psi0;
        for (int q = 0; q < n; ++q) {
            const uint8_t b = bases[size_t(s) * n + q];
            if (b < 1 || b > 3) return 2;
            if (b == 3) continue;
            int qq[1] = {q};
            apply_matrix(n, psi, qq, 1, b == 1 ? VX : VY);
        }
        auto w = [&](uint64_t k) { return cplx(std::norm(psi[k]), 0.0); };
        const double total = pairwise_sum(w, 0, dim).real();
        const double target = u[s] * total;
        double run = 0.0, prev = 0.0;
        uint64_t x = dim - 1;
        for (uint64_t k = 0; k < dim; ++k) {
            prev = run;
            run += std::norm(psi[k]);
            if (run > target) { x = k; break; }
        }
        out[s] = int64_t(x);
        if (lo) lo[s] = prev / total;
        if (hi) hi[s] = run / total;
    }
    return 0;
}

// U(theta) and dU/dtheta_j (row-major complex 4 x 4, dU [15][4][4]) of the SU(4) gate
int orc_su4(const double* theta, double* U, double* dU) {
    const SU4 g = su4_gate(theta);
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            U[2 * (4 * a + b)] = g.U.m[a][b].real();
            U[2 * (4 * a + b) + 1] = g.U.m[a][b].imag();
            for (int k = 0; k < 15; ++k) {
                dU[2 * (16 * k + 4 * a + b)] = g.dU[k].m[a][b].real();
                dU[2 * (16 * k + 4 * a + b) + 1] = g.dU[k].m[a][b].imag();
            }
        }
    return 0;
}

// QML training step (Sec. "End-to-End Pure QML for Computer Vision"): every
// sample starts from its amplitude-encoded input (given normalised), the
// gates (all two-qubit, gate g = SU(4) with theta[g][15]) act in order, the
// readout probabilities are p_o = sum of |psi_x|^2 over the x whose top k
// index bits equal o (the paper's first k qubits, its qubit 0 being the most
// significant), the first C of them are the logits, and the loss is the
// softmax cross entropy with the label: L_b = logsumexp(p_0..p_{C-1}) - p_{y_b}.
// grad = d(mean_b L_b)/dtheta by the adjoint recursion: lambda = sum_o
// dL/dp_o Pi_o psi at the end, then per gate (last to first)
// dL/dtheta_j += 2 Re <lambda_g| dU_g/dtheta_j |psi_{g-1}>.
int orc_qml(int n, const int32_t* gates, int G, const double* theta, const double* inputs, int B,
            const int32_t* labels, int k, int C, double* loss, double* grad, double* probs) {
    if (k < 1 || k > n || C < 1 || C > (1 << k)) return 1;
    auto g = read_gates(gates, G);
    for (auto& gi : g)
        if (arity(gi.kind) != 2) return 2;
    std::vector<SU4> su(G);
    for (int i = 0; i < G; ++i) su[i] = su4_gate(theta + 15 * size_t(i));
    const uint64_t dim = uint64_t(1) << n;
    const int K = 1 << k;
    for (int i = 0; i < 15 * G; ++i) grad[i] = 0.0;
    for (int b = 0; b < B; ++b) {
        std::vector<cplx> psi = initial_state(n, inputs + 2 * dim * size_t(b));
        for (int i = 0; i < G; ++i) apply_gate(n, psi, g[i], su[i].U);
        std::vector<double> p(K, 0.0);
        for (int o = 0; o < K; ++o) {
            auto w = [&](uint64_t r) { return cplx(std::norm(psi[(uint64_t(o) << (n - k)) | r]), 0.0); };
            p[o] = pairwise_sum(w, 0, dim >> k).real();
        }
        if (probs) for (int o = 0; o < K; ++o) probs[size_t(b) * K + o] = p[o];
        double mx = p[0];
        for (int o = 1; o < C; ++o) mx = std::max(mx, p[o]);
        double se = 0.0;
        for (int o = 0; o < C; ++o) se += std::exp(p[o] - mx);
        const int y = labels[b];
        if (y < 0 || y >= C) return 3;
        loss[b] = mx + std::log(se) - p[y];
        // dL/dp_o of the batch mean
        std::vector<double> dp(K, 0.0);
        for (int o = 0; o < C; ++o) dp[o] = (std::exp(p[o] - mx) / se - (o == y ? 1.0 : 0.0)) / B;
        std::vector<cplx> lam(dim);
        for (uint64_t x = 0; x < dim; ++x) lam[x] = dp[x >> (n - k)] * psi[x];
        for (int i = G - 1; i >= 0; --i) {
            std::vector<cplx> prev = psi;
            apply_gate(n, prev, g[i], dagger(su[i].U));
            for (int j = 0; j < 15; ++j) {
                std::vector<cplx> t = prev;
                apply_gate(n, t, g[i], su[i].dU[j]);
                grad[15 * i + j] += 2.0 * inner(lam, t).real();
            }
            apply_gate(n, lam, g[i], dagger(su[i].U));
            psi.swap(prev);
        }
    }
    return 0;
}

}  // extern "C"
