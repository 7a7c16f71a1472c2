// C ABI of the statevector hot path: argument validation, handle management,
// device tables, workspace layout and kernel dispatch.  Every step of the
// computation runs in the HIP kernels; this file only orders launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tcng.h"
#include "kernels.h"
#include "plan.h"

using namespace tcng;

namespace {

thread_local std::string g_err;

tcng_status fail(tcng_status s, const std::string& msg) {
    g_err = msg;
    return s;
}
tcng_status ok() {
    g_err.clear();
    return TCNG_OK;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(TCNG_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define PROF_TRY(fam, expr)              \
    do {                                 \
        ProfScope ps_(fam, st);          \
        HIP_TRY(expr);                   \
    } while (0)

constexpr int MAX_QUBITS = 34;

// ---------------------------------------------------------------------------
// optional per-launch timing (events on the launch stream)
// ---------------------------------------------------------------------------
enum Family { F_FWD_TILE, F_REV_TILE, F_PAULI_TILE, F_GATE1, F_GATE2, F_GATEK, F_REV1, F_REV2, F_PAULI_GROUP,
              F_FINISH, F_INIT, F_COUNT };

struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> ev;   // pairs
    std::vector<int> fam;
    size_t used = 0;
};
Profiler g_prof;

struct ProfScope {
    int slot = -1;
    hipStream_t st;
    ProfScope(int family, hipStream_t s) : st(s) {
        if (!g_prof.on || g_prof.used >= g_prof.fam.size()) return;
        slot = int(g_prof.used++);
        g_prof.fam[slot] = family;
        (void)hipEventRecord(g_prof.ev[2 * slot], st);
    }
    ~ProfScope() {
        if (slot >= 0) (void)hipEventRecord(g_prof.ev[2 * slot + 1], st);
    }
};

TileConfig tile_config(int dtype) {
    return dtype == TCNG_C64 ? TileConfig{13, 5, 4} : TileConfig{12, 4, 4};
}
// the tiled kernels need at least one full wave per tile
bool tiled_ok(int n, int dtype) {
    const TileConfig c = tile_config(dtype);
    return n >= c.rb + 6;
}

template <typename T>
hipError_t upload(const std::vector<T>& v, T** dst) {
    *dst = nullptr;
    if (v.empty()) return hipSuccess;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), v.size() * sizeof(T));
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

struct SlotTables {
    int total = 0;
    int32_t* ptr = nullptr;        // [n_params + 1]
    int32_t* idx = nullptr;
    int32_t* gate_slot = nullptr;  // [n_gates]
};

struct DevCircuitPlan {
    bool valid = false;
    CircuitPlan host;
    Pass* passes = nullptr;
    Phase* phases = nullptr;
    Op* ops = nullptr;
    SlotTables slots;
};

}  // namespace

struct tcng_circuit {
    int n = 0, n_params = 0, n_mats = 0;
    std::vector<tcng_gate> gates;
    std::vector<double> mats;         // c128 [n_mats][16][2]
    int device = 0;
    void* cm[2] = {nullptr, nullptr};          // constant matrices in c64 / c128
    double* u2m[2] = {nullptr, nullptr};       // constant matrices as the run sees them, widened to c128
    int32_t* gate_mat = nullptr;               // [n_gates] matrix index (for gate gradients)
    std::vector<int> plain_slot;               // first slot per gate (plain path), -1 none
    SlotTables plain;
    DevCircuitPlan tiled[2];
};

struct tcng_pauli_sum {
    int n = 0, n_terms = 0;
    std::vector<PauliTermHost> terms;
    // plain grouping
    std::vector<PGroupFull> groups_full;
    PClassFull* classes_full = nullptr;
    PTermFull* terms_full = nullptr;
    // tiled plans per dtype
    bool tiled_valid[2] = {false, false};
    PauliPlan tplan[2];
    DevPauliPlan dplan[2];
};

namespace {

tcng_status build_slot_tables(const std::vector<tcng_gate>& gates, int n_params,
                              const std::vector<int32_t>& ptr, const std::vector<int32_t>& idx,
                              const std::vector<int32_t>& gate_slot, int total, SlotTables& out) {
    out.total = total;
    std::vector<int32_t> p = ptr, i = idx, g = gate_slot;
    if (i.empty()) i.push_back(0);
    if (g.empty()) g.push_back(-1);
    HIP_TRY(upload(p, &out.ptr));
    HIP_TRY(upload(i, &out.idx));
    HIP_TRY(upload(g, &out.gate_slot));
    return TCNG_OK;
}

tcng_status check_state(const tcng_state* s, const char* what) {
    if (!s) return fail(TCNG_E_INVALID, std::string(what) + ": null state");
    if (!s->amps) return fail(TCNG_E_INVALID, std::string(what) + ": null amplitude pointer");
    if (s->n_qubits < 1 || s->n_qubits > MAX_QUBITS)
        return fail(TCNG_E_UNSUPPORTED, std::string(what) + ": n_qubits out of range 1..34");
    if (s->dtype != TCNG_C64 && s->dtype != TCNG_C128) return fail(TCNG_E_INVALID, std::string(what) + ": bad dtype");
    if (s->batch < 1 || s->batch > 65535) return fail(TCNG_E_INVALID, std::string(what) + ": batch must be 1..65535");
    if (s->stride < (int64_t(1) << s->n_qubits))
        return fail(TCNG_E_INVALID, std::string(what) + ": stride smaller than 2^n");
    if (s->stride % 2) return fail(TCNG_E_INVALID, std::string(what) + ": stride must be even");
    if (reinterpret_cast<uintptr_t>(s->amps) % 16)
        return fail(TCNG_E_INVALID, std::string(what) + ": amplitudes must be 16-byte aligned");
    return TCNG_OK;
}

int ceil_div(int64_t a, int64_t b) { return int((a + b - 1) / b); }

// workgroups per batch member of the reduction-carrying launches
int rev_wgs_tiled(int n, int dtype, int64_t batch) {
    const int m = std::min(n, tile_config(dtype).m_max);
    const int64_t tiles = int64_t(1) << (n - m);
    const int64_t cap = std::max<int64_t>(1, ceil_div(8192, batch));
    return int(std::min(tiles, cap));
}
int rev_wgs_plain(int n, int64_t batch) {
    const int64_t need = std::max<int64_t>(1, ceil_div(int64_t(1) << std::max(n - 1, 0), 256));
    const int64_t cap = std::max<int64_t>(1, ceil_div(4096, batch));
    return int(std::min(need, cap));
}
int pauli_wgs_plain(int n, int64_t batch) {
    const int64_t need = std::max<int64_t>(1, ceil_div(int64_t(1) << n, 256));
    const int64_t cap = std::max<int64_t>(1, ceil_div(4096, batch));
    return int(std::min(need, cap));
}

struct WsLayout {
    size_t part_off = 0, part_bytes = 0;
    size_t epart_off = 0, epart_bytes = 0;
    size_t red_off = 0, red_bytes = 0;     // row sums of the partials
    size_t opm_off = 0, opm_bytes = 0;     // matrix entries of the plan's ops per batch member
    size_t total = 0;
    int rev_wgs = 0, e_wgs = 0, e_rows = 0, total_slots = 0;
};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

void finish_layout(WsLayout& L, int64_t batch) {
    L.part_off = 0;
    L.epart_off = align256(L.part_bytes);
    L.red_off = L.epart_off + align256(L.epart_bytes);
    L.red_bytes = size_t(batch) * size_t(std::max(L.total_slots, 1) + std::max(L.e_rows, 1)) * sizeof(double);
    L.opm_off = L.red_off + align256(L.red_bytes);
    L.total = L.opm_off + align256(L.opm_bytes);
}

bool use_tiled(int mode, int n, int dtype) { return mode == TCNG_MODE_TILED && tiled_ok(n, dtype); }

WsLayout layout(const tcng_circuit* c, const tcng_pauli_sum* h, int n, int dtype, int64_t batch, int mode) {
    WsLayout L;
    const bool tiled = use_tiled(mode, n, dtype);
    if (c) {
        if (tiled)
            L.opm_bytes = size_t(batch) * c->tiled[dtype].host.ops.size() * 16 * (dtype == TCNG_C64 ? 8 : 16);
        L.total_slots = tiled ? c->tiled[dtype].host.total_slots : c->plain.total;
        L.rev_wgs = tiled ? rev_wgs_tiled(n, dtype, batch) : rev_wgs_plain(n, batch);
        L.part_bytes = size_t(batch) * size_t(std::max(L.total_slots, 1)) * size_t(L.rev_wgs) * sizeof(double);
    }
    if (h) {
        if (tiled) {
            L.e_rows = int(h->tplan[dtype].passes.size());
            L.e_wgs = rev_wgs_tiled(n, dtype, batch);
        } else {
            L.e_rows = int(h->groups_full.size());
            L.e_wgs = pauli_wgs_plain(n, batch);
        }
        L.e_rows = std::max(L.e_rows, 1);
        L.epart_bytes = size_t(batch) * size_t(L.e_rows) * size_t(L.e_wgs) * sizeof(double);
    }
    finish_layout(L, batch);
    return L;
}

// op matrix entries for the tiled passes (once per evaluation)
template <typename R>
tcng_status build_ops(const tcng_circuit* c, const void* params, int64_t batch, int dt, void* opm, hipStream_t st) {
    const DevCircuitPlan& P = c->tiled[dt];
    DevPlan dp{P.passes, P.phases, P.ops};
    PROF_TRY(F_FINISH, launch_build_ops<R>(dp, int(P.host.ops.size()), params, c->n_params, c->cm[dt], batch, opm, st));
    return TCNG_OK;
}

template <typename R, int RB>
tcng_status run_forward(const tcng_circuit* c, const void* params, const tcng_state* s, int mode, const void* opm,
                        hipStream_t st) {
    const int dt = s->dtype;
    const int n = s->n_qubits;
    if (use_tiled(mode, n, dt)) {
        const DevCircuitPlan& P = c->tiled[dt];
        DevPlan dp{P.passes, P.phases, P.ops};
        for (size_t p = 0; p < P.host.passes.size(); ++p)
            PROF_TRY(F_FWD_TILE, (launch_tile_fwd<R, RB>(dp, int(p), P.host.passes[p].m, s->amps, s->stride, n, s->batch,
                                                          opm, int(P.host.ops.size()), st)));
    } else {
        for (const tcng_gate& g : c->gates) {
            if (kind_arity(g.kind) == 1)
                PROF_TRY(F_GATE1, launch_gate1<R>(s->amps, s->stride, n, s->batch, g.q0, g.kind, g.p0, g.mat, params,
                                        c->n_params, c->cm[dt], nullptr, false, st));
            else
                PROF_TRY(F_GATE2, launch_gate2<R>(s->amps, s->stride, n, s->batch, g.q0, g.q1, g.kind, g.p0, g.p1, g.mat,
                                        params, c->n_params, c->cm[dt], nullptr, false, st));
        }
    }
    return TCNG_OK;
}

// H psi into lam (if lam) and energy partial sums into epart
template <typename R, int RB>
tcng_status run_pauli(const tcng_pauli_sum* h, const tcng_state* s, void* lam, const WsLayout& L, double* epart,
                      int mode, hipStream_t st) {
    const int dt = s->dtype;
    const int n = s->n_qubits;
    if (use_tiled(mode, n, dt)) {
        const PauliPlan& P = h->tplan[dt];
        for (size_t p = 0; p < P.passes.size(); ++p)
            PROF_TRY(F_PAULI_TILE, (launch_pauli_tile<R, RB>(h->dplan[dt], int(p), L.e_rows, P.passes[p].m, s->amps, lam, p > 0,
                                               s->stride, n, s->batch, L.e_wgs, epart, st)));
        if (P.passes.empty()) HIP_TRY(launch_zero(epart, L.epart_bytes / sizeof(double), st));
    } else {
        for (size_t g = 0; g < h->groups_full.size(); ++g) {
            const PGroupFull& G = h->groups_full[g];
            PROF_TRY(F_PAULI_GROUP, launch_pauli_group<R>(s->amps, lam, g > 0, s->stride, n, s->batch, G.x, h->classes_full,
                                          G.class_begin, G.class_end, h->terms_full, L.e_wgs, epart, int(g), L.e_rows,
                                          st));
        }
        if (h->groups_full.empty()) HIP_TRY(launch_zero(epart, L.epart_bytes / sizeof(double), st));
    }
    if (lam && h->n_terms == 0) {
        // H = 0: lambda = 0 (a fill kernel with no basis index in range)
        HIP_TRY(launch_init<R>(lam, s->stride, n, s->batch, nullptr, -1, st));
    }
    return TCNG_OK;
}

template <typename R, int RB>
tcng_status run_reverse(const tcng_circuit* c, const void* params, const tcng_state* psi, void* lam,
                        const WsLayout& L, double* part, int mode, const void* opm, hipStream_t st) {
    const int dt = psi->dtype;
    const int n = psi->n_qubits;
    if (use_tiled(mode, n, dt)) {
        const DevCircuitPlan& P = c->tiled[dt];
        DevPlan dp{P.passes, P.phases, P.ops};
        for (int p = int(P.host.passes.size()) - 1; p >= 0; --p)
            PROF_TRY(F_REV_TILE, (launch_tile_rev<R, RB>(dp, p, P.host.passes[p].m, psi->amps, lam, psi->stride, n, psi->batch,
                                                          opm, int(P.host.ops.size()), L.rev_wgs, part, L.total_slots,
                                                          st)));
    } else {
        for (int gi = int(c->gates.size()) - 1; gi >= 0; --gi) {
            const tcng_gate& g = c->gates[gi];
            const int slot = c->plain_slot[gi];
            if (kind_arity(g.kind) == 1)
                PROF_TRY(F_REV1, launch_rev1<R>(psi->amps, lam, psi->stride, n, psi->batch, g.q0, g.kind, g.p0, g.mat, params,
                                       c->n_params, c->cm[dt], slot, L.rev_wgs, part, L.total_slots, st));
            else
                PROF_TRY(F_REV2, launch_rev2<R>(psi->amps, lam, psi->stride, n, psi->batch, g.q0, g.q1, g.kind, g.p0, g.p1,
                                       g.mat, params, c->n_params, c->cm[dt], slot, L.rev_wgs, part, L.total_slots,
                                       st));
        }
    }
    return TCNG_OK;
}

tcng_status check_circuit_state(const tcng_circuit* c, const tcng_state* s, const void* params) {
    if (!c) return fail(TCNG_E_INVALID, "null circuit");
    if (c->n != s->n_qubits) return fail(TCNG_E_INVALID, "circuit and state have different qubit counts");
    if (c->n_params > 0 && !params) return fail(TCNG_E_INVALID, "null params for a parameterised circuit");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != c->device) return fail(TCNG_E_INVALID, "circuit was created on another device");
    if (use_tiled(TCNG_MODE_TILED, c->n, s->dtype) && !c->tiled[s->dtype].valid)
        return fail(TCNG_E_UNSUPPORTED, "no tiled plan for this circuit");
    return TCNG_OK;
}

}  // namespace

extern "C" {

const char* tcng_last_error(void) { return g_err.c_str(); }
int32_t tcng_version(void) { return 1; }

tcng_status tcng_state_init(const tcng_state* s, const void* amps_in, int64_t basis_index, void* stream) {
    if (tcng_status e = check_state(s, "tcng_state_init")) return e;
    if (!amps_in && (basis_index < 0 || basis_index >= (int64_t(1) << s->n_qubits)))
        return fail(TCNG_E_INVALID, "basis index out of range");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (s->dtype == TCNG_C64) PROF_TRY(F_INIT, launch_init<float>(s->amps, s->stride, s->n_qubits, s->batch, amps_in, basis_index, st));
    else PROF_TRY(F_INIT, launch_init<double>(s->amps, s->stride, s->n_qubits, s->batch, amps_in, basis_index, st));
    return ok();
}

tcng_status tcng_apply_gate(const tcng_state* s, const int32_t* qubits, int32_t k, const void* unitary, void* stream) {
    if (tcng_status e = check_state(s, "tcng_apply_gate")) return e;
    if (!qubits || !unitary) return fail(TCNG_E_INVALID, "null qubits or unitary");
    if (k < 1 || k > 5) return fail(TCNG_E_INVALID, "k must be 1..5");
    if (k > s->n_qubits) return fail(TCNG_E_INVALID, "k larger than the qubit count");
    for (int i = 0; i < k; ++i) {
        if (qubits[i] < 0 || qubits[i] >= s->n_qubits) return fail(TCNG_E_INVALID, "qubit out of range");
        for (int j = 0; j < i; ++j)
            if (qubits[i] == qubits[j]) return fail(TCNG_E_INVALID, "duplicate qubit");
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool f = s->dtype == TCNG_C64;
    if (k == 1) {
        if (f) PROF_TRY(F_GATE1, launch_gate1<float>(s->amps, s->stride, s->n_qubits, s->batch, qubits[0], TCNG_U1, -1, -1, nullptr, 0, nullptr, unitary, false, st));
        else PROF_TRY(F_GATE1, launch_gate1<double>(s->amps, s->stride, s->n_qubits, s->batch, qubits[0], TCNG_U1, -1, -1, nullptr, 0, nullptr, unitary, false, st));
    } else if (k == 2) {
        if (f) PROF_TRY(F_GATE2, launch_gate2<float>(s->amps, s->stride, s->n_qubits, s->batch, qubits[0], qubits[1], TCNG_U2, -1, -1, -1, nullptr, 0, nullptr, unitary, false, st));
        else PROF_TRY(F_GATE2, launch_gate2<double>(s->amps, s->stride, s->n_qubits, s->batch, qubits[0], qubits[1], TCNG_U2, -1, -1, -1, nullptr, 0, nullptr, unitary, false, st));
    } else {
        if (f) PROF_TRY(F_GATEK, launch_gatek<float>(s->amps, s->stride, s->n_qubits, s->batch, qubits, k, unitary, st));
        else PROF_TRY(F_GATEK, launch_gatek<double>(s->amps, s->stride, s->n_qubits, s->batch, qubits, k, unitary, st));
    }
    return ok();
}

tcng_status tcng_circuit_create(int32_t n_qubits, const tcng_gate* gates, int32_t n_gates, int32_t n_params,
                                const double* const_mats, int32_t n_mats, tcng_circuit** out) {
    if (!out) return fail(TCNG_E_INVALID, "null output handle");
    *out = nullptr;
    if (n_qubits < 1 || n_qubits > MAX_QUBITS) return fail(TCNG_E_UNSUPPORTED, "n_qubits out of range 1..34");
    if (n_gates < 0 || n_params < 0 || n_mats < 0) return fail(TCNG_E_INVALID, "negative count");
    if (n_gates > 0 && !gates) return fail(TCNG_E_INVALID, "null gate list");
    if (n_mats > 0 && !const_mats) return fail(TCNG_E_INVALID, "null constant matrices");
    for (int i = 0; i < n_gates; ++i) {
        const tcng_gate& g = gates[i];
        if (g.kind < 0 || g.kind >= K_COUNT) return fail(TCNG_E_INVALID, "gate " + std::to_string(i) + ": bad kind");
        if (g.q0 < 0 || g.q0 >= n_qubits) return fail(TCNG_E_INVALID, "gate " + std::to_string(i) + ": qubit out of range");
        if (kind_arity(g.kind) == 2) {
            if (g.q1 < 0 || g.q1 >= n_qubits) return fail(TCNG_E_INVALID, "gate " + std::to_string(i) + ": qubit out of range");
            if (g.q1 == g.q0) return fail(TCNG_E_INVALID, "gate " + std::to_string(i) + ": duplicate qubit");
        }
        const int np = kind_nparams(g.kind);
        if (np >= 1 && (g.p0 < 0 || g.p0 >= n_params)) return fail(TCNG_E_INVALID, "gate " + std::to_string(i) + ": parameter index out of range");
        if (np >= 2 && (g.p1 < 0 || g.p1 >= n_params)) return fail(TCNG_E_INVALID, "gate " + std::to_string(i) + ": parameter index out of range");
        if ((g.kind == K_U1 || g.kind == K_U2) && (g.mat < 0 || g.mat >= n_mats))
            return fail(TCNG_E_INVALID, "gate " + std::to_string(i) + ": matrix index out of range");
    }
    auto* c = new (std::nothrow) tcng_circuit();
    if (!c) return fail(TCNG_E_ALLOC, "host allocation failed");
    c->n = n_qubits;
    c->n_params = n_params;
    c->n_mats = n_mats;
    c->gates.assign(gates, gates + n_gates);
    c->mats.assign(const_mats ? const_mats : nullptr, const_mats ? const_mats + size_t(n_mats) * 32 : nullptr);
    auto cleanup = [&](tcng_status s) { tcng_circuit_destroy(c); return s; };
    if (hipGetDevice(&c->device) != hipSuccess) return cleanup(fail(TCNG_E_HIP, "no HIP device"));

    // constant matrices: c64 copy, c128 copy, and both widened to c128 for gate gradients
    {
        std::vector<float> mf(std::max<size_t>(c->mats.size(), 2));
        std::vector<double> md(std::max<size_t>(c->mats.size(), 2)), mfw(std::max<size_t>(c->mats.size(), 2));
        for (size_t i = 0; i < c->mats.size(); ++i) {
            mf[i] = float(c->mats[i]);
            md[i] = c->mats[i];
            mfw[i] = double(mf[i]);
        }
        float* pf = nullptr;
        double* pd = nullptr;
        if (upload(mf, &pf) != hipSuccess || upload(md, &pd) != hipSuccess) return cleanup(fail(TCNG_E_ALLOC, "device allocation failed"));
        c->cm[0] = pf;
        c->cm[1] = pd;
        if (upload(mfw, &c->u2m[0]) != hipSuccess || upload(md, &c->u2m[1]) != hipSuccess)
            return cleanup(fail(TCNG_E_ALLOC, "device allocation failed"));
        std::vector<int32_t> gm(std::max(n_gates, 1), 0);
        for (int i = 0; i < n_gates; ++i) gm[i] = std::max(gates[i].mat, 0);
        if (upload(gm, &c->gate_mat) != hipSuccess) return cleanup(fail(TCNG_E_ALLOC, "device allocation failed"));
    }
    // plain path slots: in gate order
    {
        c->plain_slot.assign(n_gates, -1);
        int total = 0;
        std::vector<std::vector<int32_t>> per_param(n_params);
        std::vector<int32_t> gate_slot(n_gates, -1);
        for (int i = 0; i < n_gates; ++i) {
            const int s = kind_slots(gates[i].kind);
            if (!s) continue;
            c->plain_slot[i] = total;
            if (gates[i].kind == K_U2) gate_slot[i] = total;
            else {
                per_param[gates[i].p0].push_back(total);
                if (kind_nparams(gates[i].kind) == 2) per_param[gates[i].p1].push_back(total + 1);
            }
            total += s;
        }
        std::vector<int32_t> ptr(1, 0), idx;
        for (auto& v : per_param) { idx.insert(idx.end(), v.begin(), v.end()); ptr.push_back(int32_t(idx.size())); }
        if (tcng_status e = build_slot_tables(c->gates, n_params, ptr, idx, gate_slot, total, c->plain))
            return cleanup(e);
    }
    // tiled plans
    for (int dt = 0; dt < 2; ++dt) {
        if (!tiled_ok(n_qubits, dt)) continue;
        DevCircuitPlan& P = c->tiled[dt];
        std::string why = plan_circuit(n_qubits, c->gates, n_params, tile_config(dt), P.host);
        if (!why.empty()) return cleanup(fail(TCNG_E_UNSUPPORTED, "planner: " + why));
        if (upload(P.host.passes, &P.passes) != hipSuccess || upload(P.host.phases, &P.phases) != hipSuccess ||
            upload(P.host.ops, &P.ops) != hipSuccess)
            return cleanup(fail(TCNG_E_ALLOC, "device allocation failed"));
        if (tcng_status e = build_slot_tables(c->gates, n_params, P.host.slot_ptr, P.host.slot_idx, P.host.gate_slot,
                                              P.host.total_slots, P.slots))
            return cleanup(e);
        P.valid = true;
    }
    *out = c;
    return ok();
}

tcng_status tcng_circuit_destroy(tcng_circuit* c) {
    if (!c) return ok();
    // work already enqueued may still read the tables
    (void)hipDeviceSynchronize();
    (void)hipFree(c->cm[0]);
    (void)hipFree(c->cm[1]);
    (void)hipFree(c->u2m[0]);
    (void)hipFree(c->u2m[1]);
    (void)hipFree(c->gate_mat);
    (void)hipFree(c->plain.ptr);
    (void)hipFree(c->plain.idx);
    (void)hipFree(c->plain.gate_slot);
    for (auto& P : c->tiled) {
        (void)hipFree(P.passes);
        (void)hipFree(P.phases);
        (void)hipFree(P.ops);
        (void)hipFree(P.slots.ptr);
        (void)hipFree(P.slots.idx);
        (void)hipFree(P.slots.gate_slot);
    }
    delete c;
    return ok();
}

tcng_status tcng_circuit_num_passes(const tcng_circuit* c, int32_t dtype, int32_t* passes) {
    if (!c || !passes) return fail(TCNG_E_INVALID, "null argument");
    if (dtype != TCNG_C64 && dtype != TCNG_C128) return fail(TCNG_E_INVALID, "bad dtype");
    *passes = c->tiled[dtype].valid ? int32_t(c->tiled[dtype].host.passes.size()) : 0;
    return ok();
}

tcng_status tcng_pauli_sum_create(int32_t n_qubits, const uint8_t* codes, const double* coeffs, int32_t n_terms,
                                  tcng_pauli_sum** out) {
    if (!out) return fail(TCNG_E_INVALID, "null output handle");
    *out = nullptr;
    if (n_qubits < 1 || n_qubits > MAX_QUBITS) return fail(TCNG_E_UNSUPPORTED, "n_qubits out of range 1..34");
    if (n_terms < 0) return fail(TCNG_E_INVALID, "negative term count");
    if (n_terms > 0 && (!codes || !coeffs)) return fail(TCNG_E_INVALID, "null codes or coefficients");
    auto* h = new (std::nothrow) tcng_pauli_sum();
    if (!h) return fail(TCNG_E_ALLOC, "host allocation failed");
    auto cleanup = [&](tcng_status s) { tcng_pauli_sum_destroy(h); return s; };
    h->n = n_qubits;
    h->n_terms = n_terms;
    for (int t = 0; t < n_terms; ++t) {
        PauliTermHost th{0, 0, 0, coeffs[t]};
        if (!std::isfinite(coeffs[t])) return cleanup(fail(TCNG_E_INVALID, "non-finite coefficient"));
        for (int q = 0; q < n_qubits; ++q) {
            const uint8_t c = codes[size_t(t) * n_qubits + q];
            if (c > 3) return cleanup(fail(TCNG_E_INVALID, "Pauli code > 3"));
            if (c == 1 || c == 2) th.x |= uint64_t(1) << q;
            if (c == 2 || c == 3) th.z |= uint64_t(1) << q;
            if (c == 2) th.ny++;
        }
        h->terms.push_back(th);
    }
    std::vector<PClassFull> cls;
    std::vector<PTermFull> tf;
    group_pauli_full(h->terms, h->groups_full, cls, tf);
    if (cls.empty()) cls.push_back(PClassFull{});
    if (tf.empty()) tf.push_back(PTermFull{});
    if (upload(cls, &h->classes_full) != hipSuccess || upload(tf, &h->terms_full) != hipSuccess)
        return cleanup(fail(TCNG_E_ALLOC, "device allocation failed"));
    for (int dt = 0; dt < 2; ++dt) {
        if (!tiled_ok(n_qubits, dt)) continue;
        std::string why = plan_pauli(n_qubits, h->terms, tile_config(dt), h->tplan[dt]);
        if (!why.empty()) continue;   // the plain path still serves this Hamiltonian
        PauliPlan& P = h->tplan[dt];
        PPass* pp = nullptr; PGroup* pg = nullptr; PClass* pc = nullptr; PTerm* pt = nullptr;
        std::vector<PClass> cl = P.classes; if (cl.empty()) cl.push_back(PClass{});
        std::vector<PTerm> te = P.terms; if (te.empty()) te.push_back(PTerm{});
        std::vector<PGroup> gr = P.groups; if (gr.empty()) gr.push_back(PGroup{});
        std::vector<PPass> ps = P.passes; if (ps.empty()) ps.push_back(PPass{});
        if (upload(ps, &pp) != hipSuccess || upload(gr, &pg) != hipSuccess || upload(cl, &pc) != hipSuccess ||
            upload(te, &pt) != hipSuccess)
            return cleanup(fail(TCNG_E_ALLOC, "device allocation failed"));
        h->dplan[dt] = DevPauliPlan{pp, pg, pc, pt};
        h->tiled_valid[dt] = true;
    }
    *out = h;
    return ok();
}

tcng_status tcng_pauli_sum_destroy(tcng_pauli_sum* h) {
    if (!h) return ok();
    (void)hipDeviceSynchronize();
    (void)hipFree(h->classes_full);
    (void)hipFree(h->terms_full);
    for (auto& d : h->dplan) {
        (void)hipFree(const_cast<PPass*>(d.passes));
        (void)hipFree(const_cast<PGroup*>(d.groups));
        (void)hipFree(const_cast<PClass*>(d.classes));
        (void)hipFree(const_cast<PTerm*>(d.terms));
    }
    delete h;
    return ok();
}

tcng_status tcng_workspace_size(const tcng_circuit* c, const tcng_pauli_sum* h, int32_t dtype, int64_t batch,
                                int32_t mode, size_t* bytes) {
    if (!bytes) return fail(TCNG_E_INVALID, "null output");
    if (dtype != TCNG_C64 && dtype != TCNG_C128) return fail(TCNG_E_INVALID, "bad dtype");
    if (batch < 1) return fail(TCNG_E_INVALID, "batch < 1");
    if (mode != TCNG_MODE_TILED && mode != TCNG_MODE_PLAIN) return fail(TCNG_E_INVALID, "bad mode");
    const int n = c ? c->n : (h ? h->n : 0);
    if (!n) return fail(TCNG_E_INVALID, "need a circuit or a Pauli sum");
    if (c && h && c->n != h->n) return fail(TCNG_E_INVALID, "circuit and Pauli sum differ in qubit count");
    if (h && use_tiled(mode, n, dtype) && !h->tiled_valid[dtype]) mode = TCNG_MODE_PLAIN;
    *bytes = layout(c, h, n, dtype, batch, mode).total;
    return ok();
}

tcng_status tcng_run_circuit(const tcng_circuit* c, const void* params, const tcng_state* s, int32_t mode, void* ws,
                             size_t ws_bytes, void* stream) {
    if (tcng_status e = check_state(s, "tcng_run_circuit")) return e;
    if (tcng_status e = check_circuit_state(c, s, params)) return e;
    if (mode != TCNG_MODE_TILED && mode != TCNG_MODE_PLAIN) return fail(TCNG_E_INVALID, "bad mode");
    const WsLayout L = layout(c, nullptr, s->n_qubits, s->dtype, s->batch, mode);
    const bool tiled = use_tiled(mode, s->n_qubits, s->dtype);
    if (tiled && (!ws || ws_bytes < L.total))
        return fail(TCNG_E_WORKSPACE, "workspace too small: need " + std::to_string(L.total));
    hipStream_t st = static_cast<hipStream_t>(stream);
    void* opm = tiled ? static_cast<char*>(ws) + L.opm_off : nullptr;
    tcng_status e;
    if (s->dtype == TCNG_C64) {
        e = tiled ? build_ops<float>(c, params, s->batch, s->dtype, opm, st) : TCNG_OK;
        if (!e) e = run_forward<float, 5>(c, params, s, mode, opm, st);
    } else {
        e = tiled ? build_ops<double>(c, params, s->batch, s->dtype, opm, st) : TCNG_OK;
        if (!e) e = run_forward<double, 4>(c, params, s, mode, opm, st);
    }
    return e ? e : ok();
}

tcng_status tcng_expect_pauli(const tcng_state* s, const tcng_pauli_sum* h, double* out, int32_t mode, void* ws,
                              size_t ws_bytes, void* stream) {
    if (tcng_status e = check_state(s, "tcng_expect_pauli")) return e;
    if (!h || !out) return fail(TCNG_E_INVALID, "null Pauli sum or output");
    if (h->n != s->n_qubits) return fail(TCNG_E_INVALID, "Pauli sum and state differ in qubit count");
    if (mode != TCNG_MODE_TILED && mode != TCNG_MODE_PLAIN) return fail(TCNG_E_INVALID, "bad mode");
    if (use_tiled(mode, h->n, s->dtype) && !h->tiled_valid[s->dtype]) mode = TCNG_MODE_PLAIN;
    const WsLayout L = layout(nullptr, h, s->n_qubits, s->dtype, s->batch, mode);
    if (!ws || ws_bytes < L.total) return fail(TCNG_E_WORKSPACE, "workspace too small: need " + std::to_string(L.total));
    hipStream_t st = static_cast<hipStream_t>(stream);
    double* epart = reinterpret_cast<double*>(static_cast<char*>(ws) + L.epart_off);
    tcng_status e = s->dtype == TCNG_C64 ? run_pauli<float, 5>(h, s, nullptr, L, epart, mode, st)
                                         : run_pauli<double, 4>(h, s, nullptr, L, epart, mode, st);
    if (e) return e;
    double* red = reinterpret_cast<double*>(static_cast<char*>(ws) + L.red_off);
    PROF_TRY(F_FINISH, launch_finish(nullptr, 0, 1, nullptr, nullptr, 0, epart, L.e_rows, L.e_wgs, s->batch, out, nullptr,
                          nullptr, nullptr, nullptr, nullptr, 0, red, st));
    return ok();
}

tcng_status tcng_expect_grad(const tcng_circuit* c, const void* params, const tcng_pauli_sum* h,
                             const tcng_state* psi, const tcng_state* lam, double* energy, double* grad,
                             double* gate_grad, int32_t mode, void* ws, size_t ws_bytes, void* stream) {
    if (tcng_status e = check_state(psi, "tcng_expect_grad(psi)")) return e;
    if (tcng_status e = check_state(lam, "tcng_expect_grad(lam)")) return e;
    if (tcng_status e = check_circuit_state(c, psi, params)) return e;
    if (!h) return fail(TCNG_E_INVALID, "null Pauli sum");
    if (h->n != psi->n_qubits) return fail(TCNG_E_INVALID, "Pauli sum and state differ in qubit count");
    if (lam->n_qubits != psi->n_qubits || lam->dtype != psi->dtype || lam->batch != psi->batch ||
        lam->stride != psi->stride)
        return fail(TCNG_E_INVALID, "psi and lam must have the same shape");
    if (lam->amps == psi->amps) return fail(TCNG_E_INVALID, "psi and lam must not alias");
    if (!energy) return fail(TCNG_E_INVALID, "null energy output");
    if (c->n_params > 0 && !grad) return fail(TCNG_E_INVALID, "null gradient output");
    if (mode != TCNG_MODE_TILED && mode != TCNG_MODE_PLAIN) return fail(TCNG_E_INVALID, "bad mode");
    const int dt = psi->dtype;
    // the Pauli passes follow the circuit's mode unless the tiled Pauli plan is impossible
    const int pmode = (use_tiled(mode, h->n, dt) && !h->tiled_valid[dt]) ? TCNG_MODE_PLAIN : mode;
    WsLayout Lc = layout(c, nullptr, psi->n_qubits, dt, psi->batch, mode);
    WsLayout Lh = layout(nullptr, h, psi->n_qubits, dt, psi->batch, pmode);
    WsLayout L = Lc;
    L.e_rows = Lh.e_rows;
    L.e_wgs = Lh.e_wgs;
    L.epart_bytes = Lh.epart_bytes;
    finish_layout(L, psi->batch);
    if (!ws || ws_bytes < L.total) return fail(TCNG_E_WORKSPACE, "workspace too small: need " + std::to_string(L.total));
    hipStream_t st = static_cast<hipStream_t>(stream);
    double* part = reinterpret_cast<double*>(static_cast<char*>(ws) + L.part_off);
    double* epart = reinterpret_cast<double*>(static_cast<char*>(ws) + L.epart_off);
    const bool ctiled = use_tiled(mode, psi->n_qubits, dt);
    void* opm = ctiled ? static_cast<char*>(ws) + L.opm_off : nullptr;
    tcng_status e;
    if (dt == TCNG_C64) {
        e = ctiled ? build_ops<float>(c, params, psi->batch, dt, opm, st) : TCNG_OK;
        if (!e) e = run_forward<float, 5>(c, params, psi, mode, opm, st);
        if (!e) e = run_pauli<float, 5>(h, psi, lam->amps, L, epart, pmode, st);
        if (!e) e = run_reverse<float, 5>(c, params, psi, lam->amps, L, part, mode, opm, st);
    } else {
        e = ctiled ? build_ops<double>(c, params, psi->batch, dt, opm, st) : TCNG_OK;
        if (!e) e = run_forward<double, 4>(c, params, psi, mode, opm, st);
        if (!e) e = run_pauli<double, 4>(h, psi, lam->amps, L, epart, pmode, st);
        if (!e) e = run_reverse<double, 4>(c, params, psi, lam->amps, L, part, mode, opm, st);
    }
    if (e) return e;
    const bool tiled = use_tiled(mode, psi->n_qubits, dt);
    const SlotTables& S = tiled ? c->tiled[dt].slots : c->plain;
    PROF_TRY(F_FINISH, launch_finish(part, std::max(L.total_slots, 1), L.rev_wgs, S.ptr, S.idx, c->n_params, epart, L.e_rows,
                          L.e_wgs, psi->batch, energy, grad, gate_grad, S.gate_slot, c->u2m[dt], c->gate_mat,
                          int(c->gates.size()), reinterpret_cast<double*>(static_cast<char*>(ws) + L.red_off), st));
    return ok();
}

tcng_status tcng_profile_begin(int32_t max_launches) {
    if (max_launches < 1) return fail(TCNG_E_INVALID, "max_launches < 1");
    tcng_profile_end();
    g_prof.ev.assign(2 * size_t(max_launches), nullptr);
    g_prof.fam.assign(size_t(max_launches), -1);
    for (auto& e : g_prof.ev) HIP_TRY(hipEventCreate(&e));
    g_prof.used = 0;
    g_prof.on = true;
    return ok();
}

tcng_status tcng_profile_query(int32_t family, int32_t* launches, double* total_ms) {
    if (family < 0 || family >= F_COUNT || !launches || !total_ms) return fail(TCNG_E_INVALID, "bad argument");
    int cnt = 0;
    double tot = 0.0;
    for (size_t i = 0; i < g_prof.used; ++i) {
        if (g_prof.fam[i] != family) continue;
        HIP_TRY(hipEventSynchronize(g_prof.ev[2 * i + 1]));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, g_prof.ev[2 * i], g_prof.ev[2 * i + 1]));
        tot += ms;
        ++cnt;
    }
    *launches = cnt;
    *total_ms = tot;
    return ok();
}

tcng_status tcng_profile_end(void) {
    g_prof.on = false;
    for (auto& e : g_prof.ev)
        if (e) (void)hipEventDestroy(e);
    g_prof.ev.clear();
    g_prof.fam.clear();
    g_prof.used = 0;
    return ok();
}

tcng_status tcng_plan_inspect(int32_t n_qubits, const tcng_gate* gates, int32_t n_gates, int32_t n_params,
                              int32_t dtype, int32_t* order, int32_t* pass_of, uint64_t* tile_mask,
                              int32_t* n_passes) {
    if (dtype != TCNG_C64 && dtype != TCNG_C128) return fail(TCNG_E_INVALID, "bad dtype");
    if (n_qubits < 1 || n_qubits > MAX_QUBITS) return fail(TCNG_E_UNSUPPORTED, "n_qubits out of range 1..34");
    if (n_gates < 0 || (n_gates > 0 && !gates)) return fail(TCNG_E_INVALID, "bad gate list");
    for (int i = 0; i < n_gates; ++i) {
        const tcng_gate& g = gates[i];
        if (g.kind < 0 || g.kind >= K_COUNT || g.q0 < 0 || g.q0 >= n_qubits ||
            (kind_arity(g.kind) == 2 && (g.q1 < 0 || g.q1 >= n_qubits || g.q1 == g.q0)))
            return fail(TCNG_E_INVALID, "gate " + std::to_string(i) + ": bad kind or qubits");
        const int np = kind_nparams(g.kind);
        if ((np >= 1 && (g.p0 < 0 || g.p0 >= n_params)) || (np >= 2 && (g.p1 < 0 || g.p1 >= n_params)))
            return fail(TCNG_E_INVALID, "gate " + std::to_string(i) + ": parameter index out of range");
    }
    if (n_passes) *n_passes = 0;
    if (!tiled_ok(n_qubits, dtype)) return ok();
    CircuitPlan P;
    std::vector<tcng_gate> g(gates, gates + n_gates);
    std::string why = plan_circuit(n_qubits, g, n_params, tile_config(dtype), P);
    if (!why.empty()) return fail(TCNG_E_UNSUPPORTED, "planner: " + why);
    int k = 0;
    for (size_t p = 0; p < P.passes.size(); ++p) {
        if (tile_mask) tile_mask[p] = P.passes[p].tile_mask;
        for (int f = P.passes[p].phase_begin; f < P.passes[p].phase_end; ++f)
            for (int o = P.phases[f].op_begin; o < P.phases[f].op_end; ++o) {
                if (order) order[k] = P.ops[o].gate;
                if (pass_of) pass_of[k] = int32_t(p);
                ++k;
            }
    }
    if (n_passes) *n_passes = int32_t(P.passes.size());
    return ok();
}

}  // extern "C"
