// C ABI of the statevector hot path: argument validation, handle management,
// device tables, workspace layout and kernel dispatch.  Every step of the
// computation runs in the HIP kernels; this file only orders launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <mutex>
#include <sstream>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tcng.h"
#include "kernels.h"
#include "plan.h"
#include "plan_check.h"

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
              F_FINISH, F_INIT, F_FUSED_FWD, F_FUSED_REV, F_FUSED_GRAD, F_MIPT_HIST, F_MIPT_DECIDE,
              F_MIPT_COLLAPSE, F_PAULI_COO, F_SHADOW_SUM, F_SHADOW_PICK, F_QML, F_COUNT };
static_assert(F_COUNT == TCNG_PROF_FAMILIES, "profiler families");

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

// default tiling: 64 KiB tiles; forward blocks of 32 (c64) / 16 (c128)
// amplitudes per thread, reverse blocks of 16 / 8 per state (psi and lambda)
TileConfig tile_config(int dtype) {
    return dtype == TCNG_C64 ? TileConfig{13, 5, 4, 4} : TileConfig{12, 4, 4, 3};
}
// Pauli passes: 12-bit tiles for both precisions (32 KiB of LDS in complex64,
// so five workgroups share a CU), 16 amplitudes per thread
TileConfig pauli_config(int dtype) {
    return dtype == TCNG_C64 ? TileConfig{12, 4, 4, 4} : TileConfig{12, 4, 4, 3};
}
// the tiled kernels need at least one full wave per tile
bool tiled_ok(int n, int dtype) {
    const TileConfig c = tile_config(dtype);
    return n >= std::max(c.rb, c.rb_rev) + 6;
}
bool config_ok(const TileConfig& c, int dtype) {
    const int mmax = dtype == TCNG_C64 ? 13 : 12;
    const int rbs[2] = {c.rb, c.rb_rev};
    for (int rb : rbs) {
        if (dtype == TCNG_C64 && rb != 4 && rb != 5) return false;
        if (dtype == TCNG_C128 && rb != 3 && rb != 4) return false;
        if (c.m_max - rb > 9 || c.m_max - rb < 6) return false;   // 64..512 threads
    }
    return c.m_max <= mmax && c.lo >= 1 && c.lo <= c.m_max;
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
    Pass* rpasses = nullptr;
    Phase* rphases = nullptr;
    Op* rops = nullptr;
    QPass* qpasses = nullptr;     // rotation rounds (host.rounds), forward and reverse
    QPhase* qphases = nullptr;
    QStep* qsteps = nullptr;
    QPass* qrpasses = nullptr;
    QPhase* qrphases = nullptr;
    QStep* qrsteps = nullptr;
    SlotTables slots;
};

struct DevFusedPlan {
    bool valid = false;
    FusedPlan host;
    FPass* passes = nullptr;
    FPhase* phases = nullptr;
    FPass* rpasses = nullptr;
    FPhase* rphases = nullptr;
    Op* ops = nullptr;
    SlotTables slots;
};

void free_fused(DevFusedPlan& P) {
    (void)hipFree(P.passes);
    (void)hipFree(P.phases);
    (void)hipFree(P.rpasses);
    (void)hipFree(P.rphases);
    (void)hipFree(P.ops);
    (void)hipFree(P.slots.ptr);
    (void)hipFree(P.slots.idx);
    (void)hipFree(P.slots.gate_slot);
    P = DevFusedPlan();
}

// fused passes: tile bits and low qubits (complex64 only)
constexpr int FUSED_M = 12, FUSED_LO = 4;
bool fused_ok(int n, int dtype) { return dtype == TCNG_C64 && n >= FUSED_K + 5; }
// 32 x 32 blocks: full 12-bit tiles only
bool fused5_ok(int n, int dtype) { return dtype == TCNG_C64 && n >= FUSED_M; }
bool valid_mode(int mode) {
    return mode == TCNG_MODE_TILED || mode == TCNG_MODE_PLAIN || mode == TCNG_MODE_FUSED || mode == TCNG_MODE_FUSED5 ||
           mode == TCNG_MODE_AUTO;
}
bool is_fused_mode(int mode) { return mode == TCNG_MODE_FUSED || mode == TCNG_MODE_FUSED5; }

void free_plan(DevCircuitPlan& P) {
    (void)hipFree(P.passes);
    (void)hipFree(P.phases);
    (void)hipFree(P.ops);
    (void)hipFree(P.rpasses);
    (void)hipFree(P.rphases);
    (void)hipFree(P.rops);
    (void)hipFree(P.qpasses);
    (void)hipFree(P.qphases);
    (void)hipFree(P.qsteps);
    (void)hipFree(P.qrpasses);
    (void)hipFree(P.qrphases);
    (void)hipFree(P.qrsteps);
    (void)hipFree(P.slots.ptr);
    (void)hipFree(P.slots.idx);
    (void)hipFree(P.slots.gate_slot);
    P = DevCircuitPlan();
}

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
    DevFusedPlan fused;              // complex64 matrix-core plan (16 x 16 blocks)
    DevFusedPlan fused5;             // the same with 32 x 32 blocks (n >= 12)
    int tuned_mode[2] = {-1, -1};    // per dtype: the mode tcng_autotune chose (-1: not tuned)
    // n < FUSED_M: the same gates planned on FUSED_M qubits, so that 2^(FUSED_M - n)
    // contiguous batch members fill one tile (the extra index bits select the member)
    DevFusedPlan fused_wide;
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
    // sparse form: X-mask groups in first-appearance order, their terms in list order
    int coo_groups = 0;
    uint64_t* coo_x = nullptr;       // [groups]
    int32_t* coo_start = nullptr;    // [groups + 1]
    uint64_t* coo_z = nullptr;       // [terms]
    double* coo_c = nullptr;         // [terms][2]: c i^(number of Y)
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

tcng_status make_plan(tcng_circuit* c, int dt, const TileConfig& cfg) {
    DevCircuitPlan P;
    std::string why = plan_circuit(c->n, c->gates, c->n_params, cfg, P.host);
    if (!why.empty()) return fail(TCNG_E_UNSUPPORTED, "planner: " + why);
    if (upload(P.host.passes, &P.passes) != hipSuccess || upload(P.host.phases, &P.phases) != hipSuccess ||
        upload(P.host.ops, &P.ops) != hipSuccess || upload(P.host.rpasses, &P.rpasses) != hipSuccess ||
        upload(P.host.rphases, &P.rphases) != hipSuccess || upload(P.host.rops, &P.rops) != hipSuccess ||
        (P.host.rounds && (upload(P.host.qpasses, &P.qpasses) != hipSuccess ||
                           upload(P.host.qphases, &P.qphases) != hipSuccess ||
                           upload(P.host.qsteps, &P.qsteps) != hipSuccess ||
                           upload(P.host.qrpasses, &P.qrpasses) != hipSuccess ||
                           upload(P.host.qrphases, &P.qrphases) != hipSuccess ||
                           upload(P.host.qrsteps, &P.qrsteps) != hipSuccess))) {
        free_plan(P);
        return fail(TCNG_E_ALLOC, "device allocation failed");
    }
    if (tcng_status e = build_slot_tables(c->gates, c->n_params, P.host.slot_ptr, P.host.slot_idx, P.host.gate_slot,
                                          P.host.total_slots, P.slots)) {
        free_plan(P);
        return e;
    }
    P.valid = true;
    free_plan(c->tiled[dt]);
    c->tiled[dt] = P;
    return TCNG_OK;
}

// the fused plan of a circuit: tiles with FUSED_LO low qubits, or one fewer
// (memory runs of 8 amplitudes instead of 16, a wider window) where that
// saves a fifth of the passes or more: a brick wall's two layers on 20 qubits,
// for example, take two passes instead of three.  (Measured: the shorter runs
// cost a pass about 15% more, so fewer savings do not pay.)
std::string plan_fused_best(int nq, const std::vector<tcng_gate>& gates, int n_params, FusedPlan& out, int kb) {
    std::string why = plan_fused(nq, gates, n_params, FUSED_M, FUSED_LO, out, kb);
    if (!why.empty() || nq <= FUSED_M) return why;
    FusedPlan P3;
    if (plan_fused(nq, gates, n_params, FUSED_M, FUSED_LO - 1, P3, kb).empty() &&
        5 * P3.passes.size() <= 4 * out.passes.size())
        out = std::move(P3);
    return "";
}

tcng_status make_fused(tcng_circuit* c, int nq, DevFusedPlan& out, int kb = FUSED_K) {
    DevFusedPlan P;
    std::string why = plan_fused_best(nq, c->gates, c->n_params, P.host, kb);
    if (!why.empty()) return fail(TCNG_E_UNSUPPORTED, "fused planner: " + why);
    if (upload(P.host.passes, &P.passes) != hipSuccess || upload(P.host.phases, &P.phases) != hipSuccess ||
        upload(P.host.rpasses, &P.rpasses) != hipSuccess || upload(P.host.rphases, &P.rphases) != hipSuccess ||
        upload(P.host.ops, &P.ops) != hipSuccess) {
        free_fused(P);
        return fail(TCNG_E_ALLOC, "device allocation failed");
    }
    if (tcng_status e = build_slot_tables(c->gates, c->n_params, P.host.slot_ptr, P.host.slot_idx, P.host.gate_slot,
                                          P.host.total_slots, P.slots)) {
        free_fused(P);
        return e;
    }
    P.valid = true;
    free_fused(out);
    out = P;
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
int rev_wgs_tiled(int n, int m_max, int64_t batch) {
    const int m = std::min(n, m_max);
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
    bool fused = false;
    int fk = FUSED_K;                        // fused: block bits of the plan
    size_t fmats_off = 0, fmats_bytes = 0;   // fused: block matrices
    size_t opart_off = 0, opart_bytes = 0;   // fused: outer products per workgroup
    size_t osum_off = 0, osum_bytes = 0;     // fused: outer products summed
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
    L.fmats_off = L.opm_off + align256(L.opm_bytes);
    L.opart_off = L.fmats_off + align256(L.fmats_bytes);
    L.osum_off = L.opart_off + align256(L.opart_bytes);
    L.total = L.osum_off + align256(L.osum_bytes);
}

bool use_tiled(int mode, int n, int dtype) { return mode == TCNG_MODE_TILED && tiled_ok(n, dtype); }

// the mode a call runs in: FUSED needs a complex64 circuit with a fused plan;
// FUSED5 one with a 32 x 32-block plan, else it runs as FUSED
int run_mode(int mode, const tcng_circuit* c, int dtype) {
    if (mode == TCNG_MODE_AUTO)
        mode = (c && c->tuned_mode[dtype] >= 0) ? c->tuned_mode[dtype]
                                                  : (dtype == TCNG_C64 ? TCNG_MODE_FUSED : TCNG_MODE_TILED);
    if (mode == TCNG_MODE_FUSED5) {
        if (c && dtype == TCNG_C64 && c->fused5.valid) return TCNG_MODE_FUSED5;
        mode = TCNG_MODE_FUSED;
    }
    if (mode != TCNG_MODE_FUSED) return mode;
    return (c && dtype == TCNG_C64 && c->fused.valid) ? TCNG_MODE_FUSED : TCNG_MODE_TILED;
}

const DevFusedPlan& fused_plan(const tcng_circuit* c, int kb) { return kb == 5 ? c->fused5 : c->fused; }

// fused reverse: two workgroups per CU (one with 32 x 32 blocks), looping over tiles
int fused_wgs(int n, int m, int64_t batch, int kb = FUSED_K) {
    const int64_t tiles = int64_t(1) << (n - m);
    const int64_t cap = std::max<int64_t>(1, ceil_div(kb == 5 ? 256 : 512, batch));
    return int(std::min(tiles, cap));
}

WsLayout layout(const tcng_circuit* c, const tcng_pauli_sum* h, int n, int dtype, int64_t batch, int mode) {
    WsLayout L;
    const bool tiled = use_tiled(mode, n, dtype);
    if (c && is_fused_mode(mode)) {
        const FusedPlan& F = fused_plan(c, mode == TCNG_MODE_FUSED5 ? 5 : FUSED_K).host;
        const size_t sub = F.k == 5 ? 4 : 1;   // 16 x 16 sub-blocks per block
        L.fused = true;
        L.fk = F.k;
        L.total_slots = F.total_slots;
        L.rev_wgs = fused_wgs(n, F.m, batch, F.k);
        L.fmats_bytes = size_t(batch) * F.n_blocks * 2048 * sub * sizeof(float);
        L.opart_bytes = size_t(batch) * F.n_blocks * size_t(L.rev_wgs) * 512 * sub * sizeof(double);
        L.osum_bytes = size_t(batch) * F.n_blocks * 512 * sub * sizeof(double);
        L.part_bytes = size_t(batch) * size_t(std::max(L.total_slots, 1)) * sizeof(double);
    } else if (c) {
        if (tiled) {
            L.opm_bytes = size_t(batch) * c->gates.size() * 16 * (dtype == TCNG_C64 ? 8 : 16);
            // rounds: their coefficient blocks follow the members' matrix tables
            const CircuitPlan& H = c->tiled[dtype].host;
            const int qs = int(H.qsteps.size() + H.qrsteps.size());
            if (H.rounds)
                L.opm_bytes += size_t(batch) * (dtype == TCNG_C64 ? rounds_coef_bytes<float>(qs) : rounds_coef_bytes<double>(qs));
        }
        L.total_slots = tiled ? c->tiled[dtype].host.total_slots : c->plain.total;
        L.rev_wgs = tiled ? rev_wgs_tiled(n, c->tiled[dtype].host.cfg.m_max, batch) : rev_wgs_plain(n, batch);
        L.part_bytes = size_t(batch) * size_t(std::max(L.total_slots, 1)) * size_t(L.rev_wgs) * sizeof(double);
    }
    if (h) {
        if (tiled) {
            L.e_rows = int(h->tplan[dtype].passes.size());
            L.e_wgs = rev_wgs_tiled(n, h->tplan[dtype].cfg.m_max, batch);
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

// the Pauli passes run tiled unless the mode is plain or the tiled Pauli plan is impossible
int pauli_mode(int mode, const tcng_pauli_sum* h, int n, int dt) {
    const int m = is_fused_mode(mode) ? TCNG_MODE_TILED : mode;
    return (use_tiled(m, n, dt) && !h->tiled_valid[dt]) ? TCNG_MODE_PLAIN : m;
}

// workspace of a value-and-gradient evaluation (mode already passed through run_mode)
WsLayout grad_layout(const tcng_circuit* c, const tcng_pauli_sum* h, int n, int dt, int64_t batch, int mode) {
    WsLayout Lc = layout(c, nullptr, n, dt, batch, mode);
    WsLayout Lh = layout(nullptr, h, n, dt, batch, pauli_mode(mode, h, n, dt));
    WsLayout L = Lc;
    L.e_rows = Lh.e_rows;
    L.e_wgs = Lh.e_wgs;
    L.epart_bytes = Lh.epart_bytes;
    finish_layout(L, batch);
    return L;
}

// byte offset of the rounds' coefficient blocks inside the op table
size_t rounds_coef_offset(const tcng_circuit* c, int64_t batch, int dt) {
    return size_t(batch) * c->gates.size() * 16 * (dt == TCNG_C64 ? sizeof(cx<float>) : sizeof(cx<double>));
}

// op matrix entries for the tiled passes (once per evaluation)
template <typename R>
tcng_status build_ops(const tcng_circuit* c, const void* params, int64_t batch, int dt, void* opm, hipStream_t st) {
    const DevCircuitPlan& P = c->tiled[dt];
    DevPlan dp{P.passes, P.phases, P.ops};
    PROF_TRY(F_FINISH, launch_build_ops<R>(dp, int(P.host.ops.size()), params, c->n_params, c->cm[dt], batch, opm, st));
    // (the forward plan lists every gate exactly once: the table is indexed by gate)
    if (P.host.rounds)
        PROF_TRY(F_FINISH, launch_rounds_coef<R>(P.qsteps, int(P.host.qsteps.size()), P.qrsteps,
                                              int(P.host.qrsteps.size()), opm, int(c->gates.size()), batch,
                                              static_cast<char*>(opm) + rounds_coef_offset(c, batch, dt), st));
    return TCNG_OK;
}

// the job descriptor of a single circuit (shared by `batch` parameter sets)
Job make_job(const tcng_circuit* c, const tcng_pauli_sum* h, const tcng_state* s, void* lam, const void* opm,
             double* part, double* epart, const WsLayout& L) {
    Job J{};
    const int dt = s->dtype;
    if (c && c->tiled[dt].valid) {
        const DevCircuitPlan& P = c->tiled[dt];
        J.passes = P.passes;
        J.phases = P.phases;
        J.ops = P.ops;
        J.rpasses = P.rpasses;
        J.rphases = P.rphases;
        J.rops = P.rops;
        if (P.host.rounds) {
            J.qpasses = P.qpasses;
            J.qphases = P.qphases;
            J.qsteps = P.qsteps;
            J.qrpasses = P.qrpasses;
            J.qrphases = P.qrphases;
            J.qrsteps = P.qrsteps;
            J.qcoef = opm ? static_cast<const char*>(opm) + rounds_coef_offset(c, s->batch, dt) : nullptr;
            J.qsteps_fwd = int32_t(P.host.qsteps.size());
            J.qsteps_all = int32_t(P.host.qsteps.size() + P.host.qrsteps.size());
        }
        J.n_passes = int32_t(P.host.passes.size());
        J.n_gates = int32_t(c->gates.size());
        J.tiles = int64_t(1) << (s->n_qubits - std::min(s->n_qubits, P.host.cfg.m_max));
    }
    if (c && L.fused) {
        const DevFusedPlan& F = fused_plan(c, L.fk);
        J.fpasses = F.passes;
        J.fphases = F.phases;
        J.frpasses = F.rpasses;
        J.frphases = F.rphases;
        J.n_passes = int32_t(F.host.passes.size());
        J.n_blocks = F.host.n_blocks;
        J.n_gates = int32_t(c->gates.size());
        J.tiles = int64_t(1) << (s->n_qubits - F.host.m);
    }
    if (h && h->tiled_valid[dt]) {
        J.ppasses = h->dplan[dt].passes;
        J.pgroups = h->dplan[dt].groups;
        J.pclasses = h->dplan[dt].classes;
        J.pterms = h->dplan[dt].terms;
        J.n_ppasses = int32_t(h->tplan[dt].passes.size());
        if (!J.tiles) J.tiles = int64_t(1) << (s->n_qubits - std::min(s->n_qubits, h->tplan[dt].cfg.m_max));
    }
    J.state = s->amps;
    J.costate = lam;
    J.opm = opm;
    J.part = part;
    J.epart = epart;
    J.stride = s->stride;
    J.batch = s->batch;
    J.n = s->n_qubits;
    J.total_slots = L.total_slots;
    J.wgs = L.rev_wgs;
    J.e_rows = L.e_rows;
    J.e_wgs = L.e_wgs;
    return J;
}

template <typename R, int RB>
tcng_status run_forward(const tcng_circuit* c, const void* params, const tcng_state* s, int mode, const Job& J,
                        hipStream_t st) {
    const int dt = s->dtype;
    const int n = s->n_qubits;
    if (use_tiled(mode, n, dt)) {
        const DevCircuitPlan& P = c->tiled[dt];
        const int rb = P.host.cfg.rb;
        for (size_t p = 0; p < P.host.passes.size(); ++p) {
            const int m = P.host.passes[p].m;
            const JobList jl{nullptr, nullptr, 0, int32_t(p)};
            const int64_t blocks = J.tiles * J.batch;
            const int qk = (J.qpasses && J.qcoef) ? P.host.qpasses[p].kind : QK_GENERIC;
            if (qk != QK_GENERIC) {
                // a few tiles per workgroup, so each fetch overlaps a tile's phases
                const int wgs = int(std::min<int64_t>(J.tiles, std::max<int64_t>(1, 2048 / J.batch)));
                PROF_TRY(F_FWD_TILE, launch_rounds_fwd<R>(jl, J, rb, qk == QK_FSIM, wgs, int64_t(wgs) * J.batch,
                                                       1 << (m - rb), st));
            }
            else if (rb == RB)
                PROF_TRY(F_FWD_TILE, (launch_tile_fwd<R, RB>(jl, J, blocks, 1 << (m - RB), st)));
            else
                PROF_TRY(F_FWD_TILE, (launch_tile_fwd<R, RB - 1>(jl, J, blocks, 1 << (m - RB + 1), st)));
        }
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
                      int mode, const Job& job, hipStream_t st) {
    const int dt = s->dtype;
    const int n = s->n_qubits;
    if (use_tiled(mode, n, dt)) {
        const PauliPlan& P = h->tplan[dt];
        Job J = job;
        J.costate = lam;
        for (size_t p = 0; p < P.passes.size(); ++p) {
            const JobList jl{nullptr, nullptr, 0, int32_t(p)};
            PROF_TRY(F_PAULI_TILE, (launch_pauli_tile<R, RB>(jl, J, int64_t(L.e_wgs) * s->batch,
                                                              1 << (P.passes[p].m - RB), st)));
        }
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
                        const WsLayout& L, double* part, int mode, const Job& J, hipStream_t st) {
    const int dt = psi->dtype;
    const int n = psi->n_qubits;
    if (use_tiled(mode, n, dt)) {
        const DevCircuitPlan& P = c->tiled[dt];
        const int rb = P.host.cfg.rb_rev;
        const int np = int(P.host.rpasses.size());
        for (int k = 0; k < np; ++k) {
            const int m = P.host.rpasses[np - 1 - k].m;
            const JobList jl{nullptr, nullptr, 0, int32_t(k)};
            const int64_t blocks = int64_t(J.wgs) * J.batch;
            const int qk = (J.qrpasses && J.qcoef) ? P.host.qrpasses[np - 1 - k].kind : QK_GENERIC;
            if (qk != QK_GENERIC)
                PROF_TRY(F_REV_TILE, launch_rounds_rev<R>(jl, J, rb, qk == QK_FSIM, blocks, 1 << (m - rb), st));
            else if (rb == RB)
                PROF_TRY(F_REV_TILE, (launch_tile_rev<R, RB>(jl, J, blocks, 1 << (m - RB), st)));
            else
                PROF_TRY(F_REV_TILE, (launch_tile_rev<R, RB - 1>(jl, J, blocks, 1 << (m - RB + 1), st)));
        }
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

// fused: block matrices (forward operand order, and the reverse one when
// gradients follow), then the forward passes
tcng_status run_forward_fused(const tcng_circuit* c, const void* params, const tcng_state* s, const Job& J,
                              bool want_rev, hipStream_t st, int kb) {
    const DevFusedPlan& F = fused_plan(c, kb);
    PROF_TRY(F_FUSED_GRAD, launch_fused_mats(F.phases, F.ops, F.host.n_blocks, params, c->n_params, c->cm[0], 0,
                                             s->batch, const_cast<void*>(J.fmats), want_rev, st, kb));
    for (size_t p = 0; p < F.host.passes.size(); ++p) {
        const JobList jl{nullptr, nullptr, 0, int32_t(p)};
        PROF_TRY(F_FUSED_FWD, launch_fused_fwd(jl, J, F.host.m, J.tiles * J.batch, st, kb));
    }
    return TCNG_OK;
}

// fused adjoint sweep: passes in reverse, then gradient slots from the block outer products
tcng_status run_reverse_fused(const tcng_circuit* c, const void* params, const tcng_state* psi, const WsLayout& L,
                              double* part, double* osum, const Job& J, hipStream_t st) {
    const DevFusedPlan& F = fused_plan(c, L.fk);
    const int np = int(F.host.passes.size());
    for (int k = 0; k < np; ++k) {
        const JobList jl{nullptr, nullptr, 0, int32_t(k)};
        PROF_TRY(F_FUSED_REV, launch_fused_rev(jl, J, F.host.m, int64_t(J.wgs) * J.batch, st, L.fk));
    }
    if (L.total_slots > 0)
        PROF_TRY(F_FUSED_GRAD, launch_fused_grad(F.phases, F.ops, F.host.n_blocks, params, c->n_params, c->cm[0],
                                                 psi->batch, J.opart, J.wgs, osum, L.total_slots, part, st, L.fk));
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
        if (tcng_status e = make_plan(c, dt, tile_config(dt))) return cleanup(e);
    }
    if (fused_ok(n_qubits, TCNG_C64)) {
        if (tcng_status e = make_fused(c, n_qubits, c->fused)) return cleanup(e);
        if (n_qubits < FUSED_M)
            if (tcng_status e = make_fused(c, FUSED_M, c->fused_wide)) return cleanup(e);
    }
    if (fused5_ok(n_qubits, TCNG_C64))
        if (tcng_status e = make_fused(c, n_qubits, c->fused5, 5)) return cleanup(e);
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
    for (auto& P : c->tiled) free_plan(P);
    free_fused(c->fused);
    free_fused(c->fused5);
    free_fused(c->fused_wide);
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
    {
        std::vector<uint64_t> gx;
        std::vector<std::vector<int>> members;
        for (int t = 0; t < n_terms; ++t) {
            size_t g = 0;
            while (g < gx.size() && gx[g] != h->terms[t].x) ++g;
            if (g == gx.size()) {
                gx.push_back(h->terms[t].x);
                members.emplace_back();
            }
            members[g].push_back(t);
        }
        std::vector<int32_t> start(1, 0);
        std::vector<uint64_t> z;
        std::vector<double> cc;
        static const double re_i[4] = {1.0, 0.0, -1.0, 0.0}, im_i[4] = {0.0, 1.0, 0.0, -1.0};
        for (auto& mem : members) {
            for (int t : mem) {
                const PauliTermHost& th = h->terms[t];
                z.push_back(th.z);
                cc.push_back(th.c * re_i[th.ny & 3]);
                cc.push_back(th.c * im_i[th.ny & 3]);
            }
            start.push_back(int32_t(z.size()));
        }
        h->coo_groups = int(gx.size());
        if (gx.empty()) gx.push_back(0);
        if (z.empty()) { z.push_back(0); cc.push_back(0.0); cc.push_back(0.0); }
        if (upload(gx, &h->coo_x) != hipSuccess || upload(start, &h->coo_start) != hipSuccess ||
            upload(z, &h->coo_z) != hipSuccess || upload(cc, &h->coo_c) != hipSuccess)
            return cleanup(fail(TCNG_E_ALLOC, "device allocation failed"));
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
        std::string why = plan_pauli(n_qubits, h->terms, pauli_config(dt), h->tplan[dt]);
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
    (void)hipFree(h->coo_x);
    (void)hipFree(h->coo_start);
    (void)hipFree(h->coo_z);
    (void)hipFree(h->coo_c);
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
    if (!valid_mode(mode)) return fail(TCNG_E_INVALID, "bad mode");
    const int n = c ? c->n : (h ? h->n : 0);
    if (!n) return fail(TCNG_E_INVALID, "need a circuit or a Pauli sum");
    if (c && h && c->n != h->n) return fail(TCNG_E_INVALID, "circuit and Pauli sum differ in qubit count");
    mode = run_mode(mode, c, dtype);
    if (!c || !h) {
        if (h && use_tiled(is_fused_mode(mode) ? TCNG_MODE_TILED : mode, n, dtype) && !h->tiled_valid[dtype])
            mode = TCNG_MODE_PLAIN;
        *bytes = layout(c, h, n, dtype, batch, (!c && is_fused_mode(mode)) ? TCNG_MODE_TILED : mode).total;
        return ok();
    }
    *bytes = grad_layout(c, h, n, dtype, batch, mode).total;
    return ok();
}

tcng_status tcng_run_circuit(const tcng_circuit* c, const void* params, const tcng_state* s, int32_t mode, void* ws,
                             size_t ws_bytes, void* stream) {
    if (tcng_status e = check_state(s, "tcng_run_circuit")) return e;
    if (tcng_status e = check_circuit_state(c, s, params)) return e;
    if (!valid_mode(mode)) return fail(TCNG_E_INVALID, "bad mode");
    mode = run_mode(mode, c, s->dtype);
    const WsLayout L = layout(c, nullptr, s->n_qubits, s->dtype, s->batch, mode);
    const bool tiled = use_tiled(mode, s->n_qubits, s->dtype);
    if ((tiled || L.fused) && (!ws || ws_bytes < L.total))
        return fail(TCNG_E_WORKSPACE, "workspace too small: need " + std::to_string(L.total));
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (L.fused) {
        Job J = make_job(c, nullptr, s, nullptr, nullptr, nullptr, nullptr, L);
        J.fmats = static_cast<char*>(ws) + L.fmats_off;
        const tcng_status e = run_forward_fused(c, params, s, J, false, st, L.fk);
        return e ? e : ok();
    }
    void* opm = tiled ? static_cast<char*>(ws) + L.opm_off : nullptr;
    const Job J = make_job(c, nullptr, s, nullptr, opm, nullptr, nullptr, L);
    tcng_status e;
    if (s->dtype == TCNG_C64) {
        e = tiled ? build_ops<float>(c, params, s->batch, s->dtype, opm, st) : TCNG_OK;
        if (!e) e = run_forward<float, 5>(c, params, s, mode, J, st);
    } else {
        e = tiled ? build_ops<double>(c, params, s->batch, s->dtype, opm, st) : TCNG_OK;
        if (!e) e = run_forward<double, 4>(c, params, s, mode, J, st);
    }
    return e ? e : ok();
}

tcng_status tcng_expect_pauli(const tcng_state* s, const tcng_pauli_sum* h, double* out, int32_t mode, void* ws,
                              size_t ws_bytes, void* stream) {
    if (tcng_status e = check_state(s, "tcng_expect_pauli")) return e;
    if (!h || !out) return fail(TCNG_E_INVALID, "null Pauli sum or output");
    if (h->n != s->n_qubits) return fail(TCNG_E_INVALID, "Pauli sum and state differ in qubit count");
    if (!valid_mode(mode)) return fail(TCNG_E_INVALID, "bad mode");
    mode = pauli_mode(mode, h, h->n, s->dtype);
    const WsLayout L = layout(nullptr, h, s->n_qubits, s->dtype, s->batch, mode);
    if (!ws || ws_bytes < L.total) return fail(TCNG_E_WORKSPACE, "workspace too small: need " + std::to_string(L.total));
    hipStream_t st = static_cast<hipStream_t>(stream);
    double* epart = reinterpret_cast<double*>(static_cast<char*>(ws) + L.epart_off);
    const Job J = make_job(nullptr, h, s, nullptr, nullptr, nullptr, epart, L);
    tcng_status e = s->dtype == TCNG_C64 ? run_pauli<float, PAULI_RB>(h, s, nullptr, L, epart, mode, J, st)
                                         : run_pauli<double, PAULI_RB>(h, s, nullptr, L, epart, mode, J, st);
    if (e) return e;
    double* red = reinterpret_cast<double*>(static_cast<char*>(ws) + L.red_off);
    PROF_TRY(F_FINISH, launch_finish(nullptr, 0, 1, nullptr, nullptr, 0, epart, L.e_rows, L.e_wgs, s->batch, out, nullptr,
                          nullptr, nullptr, nullptr, nullptr, 0, red, st));
    return ok();
}

tcng_status tcng_apply_pauli(const tcng_state* psi, const tcng_pauli_sum* h, const tcng_state* out, double* energy,
                             int32_t mode, void* ws, size_t ws_bytes, void* stream) {
    if (tcng_status e = check_state(psi, "tcng_apply_pauli")) return e;
    if (tcng_status e = check_state(out, "tcng_apply_pauli (output)")) return e;
    if (!h) return fail(TCNG_E_INVALID, "null Pauli sum");
    if (h->n != psi->n_qubits) return fail(TCNG_E_INVALID, "Pauli sum and state differ in qubit count");
    if (out->n_qubits != psi->n_qubits || out->dtype != psi->dtype || out->batch != psi->batch ||
        out->stride != psi->stride)
        return fail(TCNG_E_INVALID, "output state must match the input's qubits, dtype, batch and stride");
    if (out->amps == psi->amps) return fail(TCNG_E_INVALID, "the output must not alias the input state");
    if (!valid_mode(mode)) return fail(TCNG_E_INVALID, "bad mode");
    mode = pauli_mode(mode, h, h->n, psi->dtype);
    const WsLayout L = layout(nullptr, h, psi->n_qubits, psi->dtype, psi->batch, mode);
    if (!ws || ws_bytes < L.total) return fail(TCNG_E_WORKSPACE, "workspace too small: need " + std::to_string(L.total));
    hipStream_t st = static_cast<hipStream_t>(stream);
    double* epart = reinterpret_cast<double*>(static_cast<char*>(ws) + L.epart_off);
    const Job J = make_job(nullptr, h, psi, out->amps, nullptr, nullptr, epart, L);
    tcng_status e = psi->dtype == TCNG_C64 ? run_pauli<float, PAULI_RB>(h, psi, out->amps, L, epart, mode, J, st)
                                           : run_pauli<double, PAULI_RB>(h, psi, out->amps, L, epart, mode, J, st);
    if (e) return e;
    if (energy) {
        double* red = reinterpret_cast<double*>(static_cast<char*>(ws) + L.red_off);
        PROF_TRY(F_FINISH, launch_finish(nullptr, 0, 1, nullptr, nullptr, 0, epart, L.e_rows, L.e_wgs, psi->batch, energy,
                                         nullptr, nullptr, nullptr, nullptr, nullptr, 0, red, st));
    }
    return ok();
}

tcng_status tcng_pauli_coo_info(const tcng_pauli_sum* h, int32_t* n_groups) {
    if (!h || !n_groups) return fail(TCNG_E_INVALID, "null Pauli sum or output");
    *n_groups = h->coo_groups;
    return ok();
}

tcng_status tcng_pauli_coo(const tcng_pauli_sum* h, int64_t row_begin, int64_t row_count, int64_t* rows, int64_t* cols,
                           void* vals, void* stream) {
    if (!h) return fail(TCNG_E_INVALID, "null Pauli sum");
    if (h->n > 62) return fail(TCNG_E_UNSUPPORTED, "COO indices need n <= 62");
    const int64_t dim = int64_t(1) << h->n;
    if (row_begin < 0 || row_count < 0 || row_begin > dim || row_count > dim - row_begin)
        return fail(TCNG_E_INVALID, "row range outside [0, 2^n)");
    if (row_count == 0 || h->coo_groups == 0) return ok();
    if (h->coo_groups > 65535) return fail(TCNG_E_UNSUPPORTED, "more than 65535 distinct X-masks");
    if (!rows || !cols || !vals) return fail(TCNG_E_INVALID, "null output arrays");
    hipStream_t st = static_cast<hipStream_t>(stream);
    PROF_TRY(F_PAULI_COO, launch_pauli_coo(h->coo_x, h->coo_start, h->coo_z, h->coo_c, h->coo_groups, row_begin,
                                             row_count, rows, cols, vals, st));
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
    if (!valid_mode(mode)) return fail(TCNG_E_INVALID, "bad mode");
    const int dt = psi->dtype;
    mode = run_mode(mode, c, dt);
    const int pmode = pauli_mode(mode, h, h->n, dt);
    const WsLayout L = grad_layout(c, h, psi->n_qubits, dt, psi->batch, mode);
    if (!ws || ws_bytes < L.total) return fail(TCNG_E_WORKSPACE, "workspace too small: need " + std::to_string(L.total));
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);
    double* part = reinterpret_cast<double*>(w + L.part_off);
    double* epart = reinterpret_cast<double*>(w + L.epart_off);
    double* red = reinterpret_cast<double*>(w + L.red_off);
    if (L.fused) {
        Job J = make_job(c, h, psi, lam->amps, nullptr, part, epart, L);
        J.fmats = w + L.fmats_off;
        J.opart = reinterpret_cast<double*>(w + L.opart_off);
        tcng_status e = run_forward_fused(c, params, psi, J, true, st, L.fk);
        if (!e) e = run_pauli<float, PAULI_RB>(h, psi, lam->amps, L, epart, pmode, J, st);
        if (!e) e = run_reverse_fused(c, params, psi, L, part, reinterpret_cast<double*>(w + L.osum_off), J, st);
        if (e) return e;
        const SlotTables& S = fused_plan(c, L.fk).slots;
        PROF_TRY(F_FINISH, launch_finish(L.total_slots > 0 ? part : nullptr, std::max(L.total_slots, 1), 1, S.ptr,
                                         S.idx, c->n_params, epart, L.e_rows, L.e_wgs, psi->batch, energy, grad,
                                         gate_grad, S.gate_slot, c->u2m[dt], c->gate_mat, int(c->gates.size()), red,
                                         st));
        return ok();
    }
    const bool ctiled = use_tiled(mode, psi->n_qubits, dt);
    void* opm = ctiled ? w + L.opm_off : nullptr;
    const Job J = make_job(c, h, psi, lam->amps, opm, part, epart, L);
    tcng_status e;
    if (dt == TCNG_C64) {
        e = ctiled ? build_ops<float>(c, params, psi->batch, dt, opm, st) : TCNG_OK;
        if (!e) e = run_forward<float, 5>(c, params, psi, mode, J, st);
        if (!e) e = run_pauli<float, PAULI_RB>(h, psi, lam->amps, L, epart, pmode, J, st);
        if (!e) e = run_reverse<float, 5>(c, params, psi, lam->amps, L, part, mode, J, st);
    } else {
        e = ctiled ? build_ops<double>(c, params, psi->batch, dt, opm, st) : TCNG_OK;
        if (!e) e = run_forward<double, 4>(c, params, psi, mode, J, st);
        if (!e) e = run_pauli<double, PAULI_RB>(h, psi, lam->amps, L, epart, pmode, J, st);
        if (!e) e = run_reverse<double, 4>(c, params, psi, lam->amps, L, part, mode, J, st);
    }
    if (e) return e;
    const SlotTables& S = ctiled ? c->tiled[dt].slots : c->plain;
    PROF_TRY(F_FINISH, launch_finish(part, std::max(L.total_slots, 1), L.rev_wgs, S.ptr, S.idx, c->n_params, epart, L.e_rows,
                          L.e_wgs, psi->batch, energy, grad, gate_grad, S.gate_slot, c->u2m[dt], c->gate_mat,
                          int(c->gates.size()), red, st));
    return ok();
}

// ---------------------------------------------------------------------------
// graph capture of one value-and-gradient evaluation
// ---------------------------------------------------------------------------
struct tcng_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

}  // extern "C"

namespace {
// records `body` (stream-ordered launches only) on a private stream as a graph
template <typename F>
tcng_status capture_graph(F body, tcng_graph** out) {
    if (!out) return fail(TCNG_E_INVALID, "null output handle");
    *out = nullptr;
    if (g_prof.on) return fail(TCNG_E_INVALID, "stop profiling before capturing a graph");
    hipStream_t st = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipStreamDestroy(st);
        return fail(TCNG_E_HIP, "stream capture could not start");
    }
    const tcng_status e = body(st);
    const std::string why = e ? std::string(tcng_last_error()) : std::string();
    const hipError_t ec = hipStreamEndCapture(st, &graph);
    (void)hipStreamDestroy(st);
    if (e) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(e, why);
    }
    if (ec != hipSuccess || !graph) return fail(TCNG_E_HIP, "stream capture failed");
    auto* g = new (std::nothrow) tcng_graph();
    if (!g) {
        (void)hipGraphDestroy(graph);
        return fail(TCNG_E_ALLOC, "host allocation failed");
    }
    g->graph = graph;
    if (hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        delete g;
        return fail(TCNG_E_HIP, "graph instantiation failed");
    }
    *out = g;
    return ok();
}
}  // namespace

extern "C" {

tcng_status tcng_graph_create(const tcng_circuit* c, const void* params, const tcng_pauli_sum* h,
                              const tcng_state* psi, const tcng_state* lam, double* energy, double* grad,
                              double* gate_grad, int32_t mode, void* ws, size_t ws_bytes, int64_t init_basis,
                              tcng_graph** out) {
    if (!out) return fail(TCNG_E_INVALID, "null output handle");
    *out = nullptr;
    if (g_prof.on) return fail(TCNG_E_INVALID, "stop profiling before capturing a graph");
    if (tcng_status e = check_state(psi, "tcng_graph_create(psi)")) return e;
    if (init_basis >= (int64_t(1) << psi->n_qubits)) return fail(TCNG_E_INVALID, "basis index out of range");
    hipStream_t st = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipStreamDestroy(st);
        return fail(TCNG_E_HIP, "stream capture could not start");
    }
    tcng_status e = TCNG_OK;
    if (init_basis >= 0) e = tcng_state_init(const_cast<tcng_state*>(psi), nullptr, init_basis, st);
    if (!e) e = tcng_expect_grad(c, params, h, psi, lam, energy, grad, gate_grad, mode, ws, ws_bytes, st);
    const std::string why = e ? std::string(tcng_last_error()) : std::string();
    const hipError_t ec = hipStreamEndCapture(st, &graph);
    (void)hipStreamDestroy(st);
    if (e) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(e, why);
    }
    if (ec != hipSuccess || !graph) return fail(TCNG_E_HIP, "stream capture failed");
    auto* g = new (std::nothrow) tcng_graph();
    if (!g) {
        (void)hipGraphDestroy(graph);
        return fail(TCNG_E_ALLOC, "host allocation failed");
    }
    g->graph = graph;
    if (hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        delete g;
        return fail(TCNG_E_HIP, "graph instantiation failed");
    }
    *out = g;
    return ok();
}

tcng_status tcng_graph_launch(tcng_graph* g, void* stream) {
    if (!g || !g->exec) return fail(TCNG_E_INVALID, "null graph");
    HIP_TRY(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
    return ok();
}

tcng_status tcng_graph_destroy(tcng_graph* g) {
    if (!g) return ok();
    (void)hipDeviceSynchronize();
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return ok();
}

tcng_status tcng_fused_plan_inspect(int32_t n_qubits, const tcng_gate* gates, int32_t n_gates, int32_t n_params,
                                    int32_t block_bits, int32_t* order, int32_t* pass_of, int32_t* block_of,
                                    int32_t* n_passes, int32_t* n_blocks, int32_t* bad_layouts) {
    if (block_bits != 4 && block_bits != 5) return fail(TCNG_E_INVALID, "block bits must be 4 or 5");
    if (n_qubits < 1 || n_qubits > MAX_QUBITS) return fail(TCNG_E_UNSUPPORTED, "n_qubits out of range");
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
    if (!fused_ok(n_qubits, TCNG_C64)) return fail(TCNG_E_UNSUPPORTED, "fused path needs n >= 9");
    if (block_bits == 5 && !fused5_ok(n_qubits, TCNG_C64))
        return fail(TCNG_E_UNSUPPORTED, "5-qubit blocks need n >= 12");
    FusedPlan P;
    std::vector<tcng_gate> g(gates, gates + n_gates);
    std::string why = plan_fused_best(n_qubits, g, n_params, P, block_bits);
    if (!why.empty()) return fail(TCNG_E_UNSUPPORTED, "fused planner: " + why);
    int k = 0;
    for (size_t p = 0; p < P.passes.size(); ++p)
        for (int f = P.passes[p].phase_begin; f < P.passes[p].phase_end; ++f)
            for (int o = P.phases[f].op_begin; o < P.phases[f].op_end; ++o) {
                if (order) order[k] = P.ops[o].gate;
                if (pass_of) pass_of[k] = int32_t(p);
                if (block_of) block_of[k] = P.phases[f].block;
                ++k;
            }
    if (n_passes) *n_passes = int32_t(P.passes.size());
    if (n_blocks) *n_blocks = P.n_blocks;
    if (bad_layouts) *bad_layouts = check_fused_layouts(P);
    return ok();
}

// ---- SU(4) QML training step
namespace {
constexpr int QML_WGS = 512;   // reverse workgroups over (member, tile) pairs: two per CU
// the plan a step runs on: below FUSED_M qubits, 2^(FUSED_M - n) contiguous members
// share one tile of the wide plan whenever the batch divides evenly
struct QmlView {
    const DevFusedPlan* F;
    int n;                     // index bits of a plan member
    int64_t batch, stride;     // plan members and their spacing (amplitudes)
};
QmlView qml_view(const tcng_circuit* c, int64_t batch, int64_t stride) {
    if (c->fused_wide.valid && stride == (int64_t(1) << c->n)) {
        const int64_t g = int64_t(1) << (FUSED_M - c->n);
        if (batch % g == 0) return {&c->fused_wide, FUSED_M, batch / g, int64_t(1) << FUSED_M};
    }
    return {&c->fused, c->n, batch, stride};
}
struct QmlLayout {
    int wgs = 0;
    size_t fmats_off = 0, opart_off = 0, osum_off = 0, slots_off = 0, utab_off = 0, dutab_off = 0, total = 0;
};
QmlLayout qml_layout(const tcng_circuit* c, const QmlView& V) {
    QmlLayout M;
    const FusedPlan& P = V.F->host;
    const int64_t items = (int64_t(1) << (V.n - P.m)) * V.batch;
    M.wgs = int(std::min<int64_t>(QML_WGS, items));
    const size_t nb = size_t(std::max(P.n_blocks, 1));
    M.fmats_off = 0;
    M.opart_off = align256(nb * 2048 * sizeof(float));
    M.osum_off = M.opart_off + align256(nb * size_t(M.wgs) * 512 * sizeof(double));
    M.slots_off = M.osum_off + align256(nb * 512 * sizeof(double));
    M.utab_off = M.slots_off + align256(size_t(std::max(P.total_slots, 1)) * sizeof(double));
    M.dutab_off = M.utab_off + align256(size_t(std::max(c->n_mats, 1)) * 16 * 2 * sizeof(float));
    M.total = M.dutab_off + align256(size_t(std::max(c->n_mats, 1)) * 15 * 32 * sizeof(double));
    return M;
}
tcng_status check_qml(const tcng_circuit* c, int n) {
    if (!c) return fail(TCNG_E_INVALID, "null circuit");
    if (c->n != n) return fail(TCNG_E_INVALID, "circuit and states differ in qubit count");
    if (!c->fused.valid) return fail(TCNG_E_UNSUPPORTED, "the QML step needs the fused path (n >= 9)");
    if (c->n_params != 0) return fail(TCNG_E_INVALID, "the QML circuit takes its angles per matrix, not as params");
    std::vector<char> seen(size_t(std::max(c->n_mats, 1)), 0);
    for (const tcng_gate& g : c->gates) {
        if (g.kind != K_U2) return fail(TCNG_E_INVALID, "every QML gate must be U2 (an SU(4) gate)");
        if (seen[g.mat]) return fail(TCNG_E_INVALID, "every QML gate needs its own matrix index");
        seen[g.mat] = 1;
    }
    if (int64_t(c->gates.size()) != c->n_mats) return fail(TCNG_E_INVALID, "every QML matrix index needs its gate");
    return TCNG_OK;
}
}  // namespace

tcng_status tcng_qml_workspace_size(const tcng_circuit* c, int64_t batch, size_t* bytes) {
    if (!bytes) return fail(TCNG_E_INVALID, "null output");
    if (!c) return fail(TCNG_E_INVALID, "null circuit");
    if (tcng_status e = check_qml(c, c->n)) return e;
    if (batch < 1 || batch > 65535) return fail(TCNG_E_INVALID, "batch must be 1..65535");
    // enough for either plan (the step picks one by the states' spacing)
    const QmlLayout a = qml_layout(c, qml_view(c, batch, int64_t(1) << c->n));
    const QmlLayout b = qml_layout(c, QmlView{&c->fused, c->n, batch, int64_t(1) << c->n});
    *bytes = std::max(a.total, b.total);
    return ok();
}

tcng_status tcng_qml_step(const tcng_circuit* c, const double* theta, const tcng_state* inputs, const tcng_state* psi,
                          const tcng_state* lam, const int32_t* labels, int32_t k, int32_t n_classes, double* loss,
                          double* grad, void* ws, size_t ws_bytes, void* stream) {
    if (tcng_status e = check_state(inputs, "tcng_qml_step (inputs)")) return e;
    if (tcng_status e = check_state(psi, "tcng_qml_step (psi)")) return e;
    if (tcng_status e = check_state(lam, "tcng_qml_step (lambda)")) return e;
    if (psi->dtype != TCNG_C64) return fail(TCNG_E_UNSUPPORTED, "the QML step runs in complex64");
    const int n = psi->n_qubits;
    const int64_t B = psi->batch;
    for (const tcng_state* x : {inputs, lam})
        if (x->n_qubits != n || x->dtype != psi->dtype || x->batch != B || x->stride != psi->stride)
            return fail(TCNG_E_INVALID, "inputs, psi and lambda must match in qubits, dtype, batch and stride");
    if (tcng_status e = check_qml(c, n)) return e;
    if (B > 65535) return fail(TCNG_E_INVALID, "batch must be 1..65535");
    if (k < 1 || k > 8 || k > n) return fail(TCNG_E_INVALID, "readout qubits k must lie in 1..min(8, n)");
    if (n_classes < 1 || n_classes > (1 << k)) return fail(TCNG_E_INVALID, "classes must lie in 1..2^k");
    if (!theta || !labels || !loss || !grad) return fail(TCNG_E_INVALID, "null angles, labels or outputs");
    if (lam->amps == psi->amps || lam->amps == inputs->amps)
        return fail(TCNG_E_INVALID, "lambda must not share memory with psi or the inputs");
    const QmlView V = qml_view(c, B, psi->stride);
    const QmlLayout M = qml_layout(c, V);
    if (!ws || ws_bytes < M.total) return fail(TCNG_E_WORKSPACE, "workspace too small: need " + std::to_string(M.total));
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);
    void* utab = w + M.utab_off;
    double* dutab = reinterpret_cast<double*>(w + M.dutab_off);
    const DevFusedPlan& F = *V.F;
    PROF_TRY(F_QML, launch_su4(theta, c->n_mats, utab, dutab, st));
    // the first forward pass loads the inputs (psi may be the inputs themselves, evolved in place)
    if (F.host.passes.empty() && inputs->amps != psi->amps)
        HIP_TRY(hipMemcpy2DAsync(psi->amps, size_t(psi->stride) * 8, inputs->amps, size_t(inputs->stride) * 8,
                                 (size_t(1) << n) * 8, size_t(B), hipMemcpyDeviceToDevice, st));
    Job J{};
    J.src = inputs->amps;
    J.src_stride = V.stride;   // inputs and psi are spaced alike
    J.fpasses = F.passes;
    J.fphases = F.phases;
    J.frpasses = F.rpasses;
    J.frphases = F.rphases;
    J.n_passes = int32_t(F.host.passes.size());
    J.n_blocks = F.host.n_blocks;
    J.n_gates = int32_t(c->gates.size());
    J.total_slots = F.host.total_slots;
    J.tiles = int64_t(1) << (V.n - F.host.m);
    J.state = psi->amps;
    J.costate = lam->amps;
    J.stride = V.stride;
    J.batch = V.batch;
    J.n = V.n;
    J.shared = 1;
    J.fmats = w + M.fmats_off;
    J.opart = reinterpret_cast<double*>(w + M.opart_off);
    J.wgs = M.wgs;
    PROF_TRY(F_FUSED_GRAD, launch_fused_mats(F.phases, F.ops, F.host.n_blocks, nullptr, 0, utab, 0, 1,
                                             const_cast<void*>(J.fmats), true, st));
    for (size_t ps = 0; ps < F.host.passes.size(); ++ps) {
        const JobList jl{nullptr, nullptr, 0, int32_t(ps)};
        PROF_TRY(F_FUSED_FWD, launch_fused_fwd(jl, J, F.host.m, J.tiles * J.batch, st));
    }
    PROF_TRY(F_QML, launch_qml_seed(psi->amps, lam->amps, psi->stride, n, B, k, n_classes, labels, loss, st));
    for (size_t ps = 0; ps < F.host.passes.size(); ++ps) {
        const JobList jl{nullptr, nullptr, 0, int32_t(ps)};
        PROF_TRY(F_FUSED_REV, launch_fused_rev(jl, J, F.host.m, J.wgs, st));
    }
    double* osum = reinterpret_cast<double*>(w + M.osum_off);
    double* slots = reinterpret_cast<double*>(w + M.slots_off);
    PROF_TRY(F_FUSED_GRAD, launch_fused_grad(F.phases, F.ops, F.host.n_blocks, nullptr, 0, utab, 1, J.opart, J.wgs, osum,
                                             F.host.total_slots, slots, st));
    PROF_TRY(F_QML, launch_qml_grad(slots, F.slots.gate_slot, c->gate_mat, dutab, int(c->gates.size()), grad, st));
    return ok();
}

// ---- classical-shadow snapshots
namespace {
struct ShadowLayout {
    WsLayout F;
    size_t mats_off = 0, part_off = 0, total = 0;
};
ShadowLayout shadow_layout(const tcng_circuit* c, int n, int64_t S) {
    ShadowLayout M;
    M.F = layout(c, nullptr, n, TCNG_C64, S, TCNG_MODE_FUSED);
    M.mats_off = align256(M.F.total);
    M.part_off = M.mats_off + align256(size_t(S) * n * 16 * 2 * sizeof(float));
    M.total = M.part_off + align256(size_t(S) * shadow_chunks(n) * sizeof(double));
    return M;
}
tcng_status check_shadow_layer(const tcng_circuit* c) {
    if (!c) return fail(TCNG_E_INVALID, "null layer circuit");
    if (!c->fused.valid) return fail(TCNG_E_UNSUPPORTED, "shadow snapshots need the fused path (n >= 9)");
    if (c->n_params != 0 || int(c->gates.size()) != c->n)
        return fail(TCNG_E_INVALID, "the layer must hold n one-qubit gates and no angles");
    for (int q = 0; q < c->n; ++q) {
        const tcng_gate& g = c->gates[q];
        if (g.kind != K_U1 || g.q0 != q || g.mat != q)
            return fail(TCNG_E_INVALID, "layer gate q must be U1 on qubit q with matrix q");
    }
    return TCNG_OK;
}
}  // namespace

tcng_status tcng_shadow_workspace_size(const tcng_circuit* layer, int64_t snapshots, size_t* bytes) {
    if (!bytes) return fail(TCNG_E_INVALID, "null output");
    if (tcng_status e = check_shadow_layer(layer)) return e;
    if (snapshots < 1 || snapshots > 65535) return fail(TCNG_E_INVALID, "snapshots must be 1..65535");
    *bytes = shadow_layout(layer, layer->n, snapshots).total;
    return ok();
}

tcng_status tcng_shadow_snapshots(const tcng_circuit* layer, const void* psi, const tcng_state* work,
                                  const uint8_t* bases, const double* u, int64_t* outcomes, void* ws, size_t ws_bytes,
                                  void* stream) {
    if (tcng_status e = check_state(work, "tcng_shadow_snapshots")) return e;
    if (work->dtype != TCNG_C64) return fail(TCNG_E_UNSUPPORTED, "shadow snapshots run in complex64");
    if (tcng_status e = check_shadow_layer(layer)) return e;
    if (layer->n != work->n_qubits) return fail(TCNG_E_INVALID, "layer and work state differ in qubit count");
    if (!psi || !bases || !u || !outcomes) return fail(TCNG_E_INVALID, "null state, bases, uniforms or outcomes");
    const int n = work->n_qubits;
    const int64_t S = work->batch;
    {
        // every snapshot's first rotation pass reads psi while others already write work
        const char* lo = static_cast<const char*>(work->amps);
        const char* hi = lo + (size_t(S - 1) * size_t(work->stride) + (size_t(1) << n)) * 8;
        const char* a = static_cast<const char*>(psi);
        if (a + (size_t(1) << n) * 8 > lo && a < hi)
            return fail(TCNG_E_INVALID, "psi must not overlap the work states");
    }
    const ShadowLayout M = shadow_layout(layer, n, S);
    if (!ws || ws_bytes < M.total) return fail(TCNG_E_WORKSPACE, "workspace too small: need " + std::to_string(M.total));
    hipStream_t st = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);
    void* mats = w + M.mats_off;
    double* part = reinterpret_cast<double*>(w + M.part_off);
    const DevFusedPlan& F = layer->fused;
    // the first rotation pass reads the one input state for every snapshot (no copies)
    if (F.host.passes.empty()) PROF_TRY(F_INIT, launch_init<float>(work->amps, work->stride, n, S, psi, 0, st));
    PROF_TRY(F_SHADOW_PICK, launch_shadow_mats(bases, n, S, mats, st));
    Job J = make_job(layer, nullptr, work, nullptr, nullptr, nullptr, nullptr, M.F);
    J.fmats = w + M.F.fmats_off;
    J.src = psi;
    J.src_stride = 0;
    PROF_TRY(F_FUSED_GRAD, launch_fused_mats(F.phases, F.ops, F.host.n_blocks, nullptr, 0, mats, n, S,
                                             const_cast<void*>(J.fmats), false, st));
    for (size_t ps = 0; ps < F.host.passes.size(); ++ps) {
        const JobList jl{nullptr, nullptr, 0, int32_t(ps)};
        PROF_TRY(F_FUSED_FWD, launch_fused_fwd(jl, J, F.host.m, J.tiles * J.batch, st));
    }
    PROF_TRY(F_SHADOW_SUM, launch_shadow_chunks(work->amps, work->stride, n, S, part, st));
    PROF_TRY(F_SHADOW_PICK, launch_shadow_pick(work->amps, work->stride, n, S, part, u, outcomes, st));
    return ok();
}

// ---- monitored Haar trajectories
namespace {
struct MiptLayout {
    WsLayout F;                      // the fused forward of one step
    size_t part_off = 0, keep_off = 0, list_off = 0, total = 0;
    int wgs = 0;
};
MiptLayout mipt_layout(const tcng_circuit* c, int n, int64_t batch) {
    MiptLayout M;
    M.F = layout(c, nullptr, n, TCNG_C64, batch, TCNG_MODE_FUSED);
    M.wgs = mipt_wgs(n);
    M.part_off = align256(M.F.total);
    M.keep_off = M.part_off + align256(mipt_hist_doubles(n, batch) * sizeof(double));
    M.list_off = M.keep_off + align256(size_t(batch) * sizeof(double));
    M.total = M.list_off + align256(mipt_list_words(n, batch) * sizeof(uint32_t));
    return M;
}
tcng_status check_mipt(const tcng_circuit* c, int n) {
    if (!c) return fail(TCNG_E_INVALID, "null circuit");
    if (c->n != n) return fail(TCNG_E_INVALID, "circuit and state have different qubit counts");
    if (n > 32) return fail(TCNG_E_UNSUPPORTED, "monitored trajectories: n must be at most 32");
    if (!c->fused.valid) return fail(TCNG_E_UNSUPPORTED, "monitored trajectories need the fused path (n >= 9)");
    if (c->n_params != 0) return fail(TCNG_E_INVALID, "monitored trajectories: the step circuit takes no angles");
    for (const tcng_gate& g : c->gates)
        if (g.kind != K_U2) return fail(TCNG_E_INVALID, "monitored trajectories: every step gate must be U2");
    return TCNG_OK;
}
}  // namespace

tcng_status tcng_mipt_workspace_size(const tcng_circuit* step, int32_t n_qubits, int64_t batch, size_t* bytes) {
    if (!bytes) return fail(TCNG_E_INVALID, "null output");
    if (tcng_status e = check_mipt(step, n_qubits)) return e;
    if (batch < 1 || batch > 65535) return fail(TCNG_E_INVALID, "batch must be 1..65535");
    *bytes = mipt_layout(step, n_qubits, batch).total;
    return ok();
}

tcng_status tcng_mipt_run(const tcng_circuit* step, int32_t n_steps, const void* mats, tcng_state* psi,
                          const double* u, double p, uint32_t* rec, double* logp, double* margin, void* ws,
                          size_t ws_bytes, void* stream) {
    if (tcng_status e = check_state(psi, "tcng_mipt_run")) return e;
    if (psi->dtype != TCNG_C64) return fail(TCNG_E_UNSUPPORTED, "monitored trajectories run in complex64");
    if (tcng_status e = check_mipt(step, psi->n_qubits)) return e;
    if (n_steps < 0) return fail(TCNG_E_INVALID, "n_steps must be >= 0");
    if (!(p >= 0.0 && p <= 1.0)) return fail(TCNG_E_INVALID, "p must lie in [0, 1]");
    if (!logp || (n_steps > 0 && (!rec || !u || (step->n_mats > 0 && !mats))))
        return fail(TCNG_E_INVALID, "null uniforms, matrices or outputs");
    const MiptLayout M = mipt_layout(step, psi->n_qubits, psi->batch);
    if (!ws || ws_bytes < M.total) return fail(TCNG_E_WORKSPACE, "workspace too small: need " + std::to_string(M.total));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int n = psi->n_qubits;
    const int64_t batch = psi->batch;
    char* w = static_cast<char*>(ws);
    double* part = reinterpret_cast<double*>(w + M.part_off);
    double* keep = reinterpret_cast<double*>(w + M.keep_off);
    uint32_t* lists = reinterpret_cast<uint32_t*>(w + M.list_off);
    PROF_TRY(F_MIPT_DECIDE, launch_zero_u32(rec, size_t(batch) * n_steps * 2, st));
    PROF_TRY(F_MIPT_DECIDE, launch_zero(logp, size_t(batch), st));
    Job J = make_job(step, nullptr, psi, nullptr, nullptr, nullptr, nullptr, M.F);
    J.fmats = w + M.F.fmats_off;
    const DevFusedPlan& F = step->fused;
    const int64_t nm = step->n_mats;
    J.prec_stride = n_steps * 2;
    J.pkeep = keep;
    for (int s = 0; s < n_steps; ++s) {
        // the previous step's collapse, applied by the first forward pass as it loads the tiles
        J.prec = s > 0 ? rec + size_t(s - 1) * 2 : nullptr;
        // the step's gates: member b takes matrix g.mat of step s at mats[((b * n_steps + s) * nm + g.mat)]
        const void* cm = static_cast<const char*>(mats) + size_t(s) * nm * 16 * sizeof(float) * 2;
        PROF_TRY(F_FUSED_GRAD, launch_fused_mats(F.phases, F.ops, F.host.n_blocks, nullptr, 0, cm, n_steps * nm, batch,
                                                 const_cast<void*>(J.fmats), false, st));
        for (size_t ps = 0; ps < F.host.passes.size(); ++ps) {
            const JobList jl{nullptr, nullptr, 0, int32_t(ps)};
            PROF_TRY(F_FUSED_FWD, launch_fused_fwd(jl, J, F.host.m, J.tiles * J.batch, st));
        }
        // a step without gates has no forward pass to fold the previous collapse into
        if (F.host.passes.empty() && s > 0)
            PROF_TRY(F_MIPT_COLLAPSE, launch_mipt_collapse(psi->amps, psi->stride, n, batch, n_steps, s - 1, rec, keep,
                                                           M.wgs, st));
        // the measured qubits in rounds of up to 8: one histogram read and the decisions
        // each; rounds after the first visit only the members their predecessor listed
        PROF_TRY(F_MIPT_DECIDE, launch_mipt_lists_reset(lists, n, batch, st));
        for (int r = 0; r < mipt_rounds(n); ++r) {
            PROF_TRY(F_MIPT_HIST,
                     launch_mipt_hist(psi->amps, psi->stride, n, batch, u, n_steps, s, p, r, rec, part, lists, st));
            PROF_TRY(F_MIPT_DECIDE,
                     launch_mipt_decide(u, n, n_steps, s, p, r, part, rec, keep, logp, margin, lists, batch, st));
        }
    }
    if (n_steps > 0)
        PROF_TRY(F_MIPT_COLLAPSE, launch_mipt_collapse(psi->amps, psi->stride, n, batch, n_steps, n_steps - 1, rec, keep,
                                                       M.wgs, st));
    return ok();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// uneven batch
// ---------------------------------------------------------------------------
namespace {

constexpr int MULTI_WGS = 16;    // workgroups per circuit in the tiled reverse sweep
constexpr int MULTI_EWGS = 64;   // workgroups per circuit (at most) in the Pauli sweep
constexpr int MULTI_FWGS = 64;   // workgroups per circuit (at most) in the fused reverse sweep

// complex64 batches whose every circuit has a fused plan run on the matrix-core
// passes; the others (complex128) on the tiled passes
bool multi_fused(const tcng_circuit* const* circs, int32_t count, int32_t dtype) {
    if (dtype != TCNG_C64) return false;
    for (int i = 0; i < count; ++i)
        if (!circs[i]->fused.valid) return false;
    return true;
}

struct MultiLayout {
    bool fused = false;
    // per circuit offsets (bytes) into the workspace and row offsets
    std::vector<size_t> opm_off;
    // fused: block matrices, outer-product partials and sums, gradient slots; reverse workgroups
    std::vector<size_t> fmats_off, opart_off, osum_off, fslot_off;
    std::vector<int> fwgs;
    size_t fjobs_off = 0;   // FusedCircJob [count]
    int max_blocks = 0;
    std::vector<int64_t> slot_row, erow_row;
    size_t part_off = 0, epart_off = 0, ssum_off = 0, esum_off = 0;
    size_t jobs_off[3] = {0, 0, 0}, prefix_off[3] = {0, 0, 0};
    size_t build_off = 0, build_prefix_off = 0, fin_off = 0, fin_prefix_off = 0;
    int64_t slot_rows = 0, e_rows = 0;
    size_t total = 0;
};

tcng_status multi_check(const tcng_circuit* const* circs, const tcng_pauli_sum* const* hams, int32_t count,
                        int32_t dtype) {
    if (!circs || !hams || count < 1) return fail(TCNG_E_INVALID, "empty uneven batch");
    if (dtype != TCNG_C64 && dtype != TCNG_C128) return fail(TCNG_E_INVALID, "bad dtype");
    int rb = -1, rr = -1;
    for (int i = 0; i < count; ++i) {
        const tcng_circuit* c = circs[i];
        const tcng_pauli_sum* h = hams[i];
        if (!c || !h) return fail(TCNG_E_INVALID, "null handle in uneven batch");
        if (c->n != h->n) return fail(TCNG_E_INVALID, "circuit and Pauli sum differ in qubit count");
        if (!c->tiled[dtype].valid || !h->tiled_valid[dtype])
            return fail(TCNG_E_UNSUPPORTED, "uneven batch member without a tiled plan");
        const TileConfig& cfg = c->tiled[dtype].host.cfg;
        if (rb < 0) { rb = cfg.rb; rr = cfg.rb_rev; }
        if (cfg.rb != rb || cfg.rb_rev != rr) return fail(TCNG_E_UNSUPPORTED, "uneven batch with mixed register blocks");
    }
    return TCNG_OK;
}

MultiLayout multi_layout(const tcng_circuit* const* circs, const tcng_pauli_sum* const* hams, int32_t count,
                         int32_t dtype) {
    MultiLayout L;
    const size_t s = dtype == TCNG_C64 ? 8 : 16;
    size_t off = 0;
    L.opm_off.resize(count);
    L.slot_row.resize(count);
    L.erow_row.resize(count);
    for (int i = 0; i < count; ++i) {
        L.opm_off[i] = off;
        off = align256(off + circs[i]->gates.size() * 16 * s);
        L.slot_row[i] = L.slot_rows;
        L.slot_rows += std::max(circs[i]->tiled[dtype].host.total_slots, 1);
        L.erow_row[i] = L.e_rows;
        L.e_rows += std::max<int64_t>(int64_t(hams[i]->tplan[dtype].passes.size()), 1);
    }
    L.fused = multi_fused(circs, count, dtype);
    if (L.fused) {
        L.fmats_off.resize(count);
        L.opart_off.resize(count);
        L.osum_off.resize(count);
        L.fslot_off.resize(count);
        L.fwgs.resize(count);
        for (int i = 0; i < count; ++i) {
            const FusedPlan& F = circs[i]->fused.host;
            const size_t nb = size_t(std::max(F.n_blocks, 1));
            L.fwgs[i] = int(std::min<int64_t>(int64_t(1) << (circs[i]->n - F.m), MULTI_FWGS));
            L.fmats_off[i] = off;
            off = align256(off + nb * 2048 * sizeof(float));
            L.opart_off[i] = off;
            off = align256(off + nb * size_t(L.fwgs[i]) * 512 * sizeof(double));
            L.osum_off[i] = off;
            off = align256(off + nb * 512 * sizeof(double));
            L.fslot_off[i] = off;
            off = align256(off + size_t(std::max(F.total_slots, 1)) * sizeof(double));
            L.max_blocks = std::max(L.max_blocks, F.n_blocks);
        }
        L.fjobs_off = off;
        off = align256(off + size_t(count) * sizeof(FusedCircJob));
    }
    L.part_off = off;
    off = align256(off + size_t(L.slot_rows) * MULTI_WGS * sizeof(double));
    L.epart_off = off;
    off = align256(off + size_t(L.e_rows) * MULTI_EWGS * sizeof(double));
    L.ssum_off = off;
    off = align256(off + size_t(L.slot_rows) * sizeof(double));
    L.esum_off = off;
    off = align256(off + size_t(L.e_rows) * sizeof(double));
    for (int k = 0; k < 3; ++k) {
        L.jobs_off[k] = off;
        off = align256(off + size_t(count) * sizeof(Job));
        L.prefix_off[k] = off;
        off = align256(off + size_t(count + 2) * sizeof(int64_t));   // fused: one prefix per tile-size group
    }
    L.build_off = off;
    off = align256(off + size_t(count) * sizeof(BuildJob));
    L.build_prefix_off = off;
    off = align256(off + size_t(count + 1) * sizeof(int64_t));
    L.fin_off = off;
    off = align256(off + size_t(count) * sizeof(FinishJob));
    L.fin_prefix_off = off;
    off = align256(off + size_t(count + 1) * sizeof(int64_t));
    L.total = off;
    return L;
}

// One launch of an uneven batch: step `step` of a sweep (0 forward, 1 Pauli,
// 2 reverse) over the first `njobs` jobs of the sorted job list at `job_off`
// (prefix sums at `prefix_off`); `m` selects the fused kernels' tile-size
// instantiation.
struct MultiLaunch {
    int sweep, step, njobs, m;
    int job_off, prefix_off;
    int64_t blocks;
};

// Sorted job lists and the launches of every sweep.  Circuits with more
// passes come first in each list, so the jobs of step k are a prefix.
// Fused (complex64): the forward and reverse lists hold the circuits of
// 12-bit tiles first, then those of smaller tiles, each group with its own
// prefix sums and launches.
struct MultiPlan {
    std::vector<Job> sorted[3];
    std::vector<int64_t> prefix[3];
    std::vector<MultiLaunch> launches;
    int nt_max[3] = {64, 64, 64};
};

MultiPlan multi_plan(const std::vector<Job>& jobs, const tcng_circuit* const* circs, const tcng_pauli_sum* const* hams,
                     int count, int dt, bool fused, int rb, int rbr) {
    MultiPlan M;
    auto group = [&](int i) { return (fused && jobs[i].n < FUSED_M) ? 1 : 0; };
    std::vector<int> ord_c(count), ord_p(count);
    for (int i = 0; i < count; ++i) ord_c[i] = ord_p[i] = i;
    std::stable_sort(ord_c.begin(), ord_c.end(), [&](int x, int y) {
        return group(x) != group(y) ? group(x) < group(y) : jobs[x].n_passes > jobs[y].n_passes;
    });
    std::stable_sort(ord_p.begin(), ord_p.end(), [&](int x, int y) { return jobs[x].n_ppasses > jobs[y].n_ppasses; });
    int g0 = 0;   // jobs of group 0 come first
    while (g0 < count && group(ord_c[g0]) == 0) ++g0;
    const int* orders[3] = {ord_c.data(), ord_p.data(), ord_c.data()};
    int max_steps[3] = {0, 0, 0};
    // prefix entries: group 0 at [0, g0], group 1 at [g0 + 1, count + 1] (each from 0); the Pauli sweep at [0, count]
    for (int k = 0; k < 3; ++k) {
        M.sorted[k].resize(count);
        M.prefix[k].assign(count + 2, 0);
        for (int i = 0; i < count; ++i) {
            const int ci = orders[k][i];
            const Job& J = jobs[ci];
            M.sorted[k][i] = J;
            const int64_t per = (k == 0) ? J.tiles : (k == 1 ? J.e_wgs : J.wgs);
            const int at = (k != 1 && i >= g0) ? i + 1 : i;   // group 1 entries one further on
            M.prefix[k][at + 1] = M.prefix[k][at] + per * J.batch;
            if (k == 1) {
                if (!hams[ci]->tplan[dt].passes.empty())
                    M.nt_max[1] = std::max(M.nt_max[1], 1 << (hams[ci]->tplan[dt].passes[0].m - PAULI_RB));
            } else if (!fused) {
                const int rbk = k == 2 ? rbr : rb;
                M.nt_max[k] = std::max(M.nt_max[k], 1 << (circs[ci]->tiled[dt].host.passes[0].m - rbk));
            }
            max_steps[k] = std::max(max_steps[k], k == 1 ? J.n_ppasses : J.n_passes);
        }
        if (k != 1 && g0 < count) M.prefix[k][g0 + 1] = 0;   // group 1 starts its own count
    }
    auto active = [&](int sweep, int k, int lo, int hi) {
        int c = 0;
        for (int i = lo; i < hi; ++i) {
            const Job& J = jobs[orders[sweep][i]];
            if ((sweep == 1 ? J.n_ppasses : J.n_passes) > k) ++c;
        }
        return c;
    };
    auto add_circuit_steps = [&](int sweep) {
        for (int k = 0; k < max_steps[sweep]; ++k)
            for (int grp = 0; grp < 2; ++grp) {
                const int lo = grp == 0 ? 0 : g0, hi = grp == 0 ? g0 : count;
                const int na = active(sweep, k, lo, hi);
                if (na == 0) continue;
                const int poff = grp == 0 ? 0 : g0 + 1;
                M.launches.push_back({sweep, k, na, grp == 0 ? FUSED_M : FUSED_M - 1, lo, poff, M.prefix[sweep][poff + na]});
            }
    };
    add_circuit_steps(0);
    for (int k = 0; k < max_steps[1]; ++k) {
        const int na = active(1, k, 0, count);
        M.launches.push_back({1, k, na, 0, 0, 0, M.prefix[1][na]});
    }
    add_circuit_steps(2);
    return M;
}

template <typename R, int RB, int RBR>
tcng_status launch_multi_tiled(const MultiPlan& M, const Job& job0, char* ws, const MultiLayout& L, hipStream_t st) {
    for (const MultiLaunch& X : M.launches) {
        const JobList jl{reinterpret_cast<const Job*>(ws + L.jobs_off[X.sweep]) + X.job_off,
                         reinterpret_cast<const int64_t*>(ws + L.prefix_off[X.sweep]) + X.prefix_off, X.njobs,
                         X.step};
        if (X.sweep == 0) PROF_TRY(F_FWD_TILE, (launch_tile_fwd<R, RB>(jl, job0, X.blocks, M.nt_max[0], st)));
        else if (X.sweep == 1) PROF_TRY(F_PAULI_TILE, (launch_pauli_tile<R, PAULI_RB>(jl, job0, X.blocks, M.nt_max[1], st)));
        else PROF_TRY(F_REV_TILE, (launch_tile_rev<R, RBR>(jl, job0, X.blocks, M.nt_max[2], st)));
    }
    return TCNG_OK;
}

tcng_status launch_multi_fused(const MultiPlan& M, const Job& job0, char* ws, const MultiLayout& L, hipStream_t st) {
    for (const MultiLaunch& X : M.launches) {
        const JobList jl{reinterpret_cast<const Job*>(ws + L.jobs_off[X.sweep]) + X.job_off,
                         reinterpret_cast<const int64_t*>(ws + L.prefix_off[X.sweep]) + X.prefix_off, X.njobs,
                         X.step};
        if (X.sweep == 0) PROF_TRY(F_FUSED_FWD, launch_fused_fwd(jl, job0, X.m, X.blocks, st));
        else if (X.sweep == 1) PROF_TRY(F_PAULI_TILE, (launch_pauli_tile<float, PAULI_RB>(jl, job0, X.blocks, M.nt_max[1], st)));
        else PROF_TRY(F_FUSED_REV, launch_fused_rev(jl, job0, X.m, X.blocks, st));
    }
    return TCNG_OK;
}

}  // namespace

// An uneven batch bound to its states, outputs and workspace: the host tables
// (sorted job lists, prefix sums, matrix-build, block and finish jobs) and the
// launch list, built once; the tables live in the workspace.
struct tcng_multi {
    int count = 0, dt = 0, rb = 0, rbr = 0;
    MultiLayout L;
    char* ws = nullptr;
    MultiPlan plan;
    Job job0{};
    std::vector<BuildJob> builds;
    std::vector<FinishJob> fins;
    std::vector<FusedCircJob> fjobs;
    std::vector<int64_t> bprefix, fprefix;
    int64_t init_basis = -1;               // tiled path: states set to |basis> at launch (fused: in the first pass)
    std::vector<tcng_state> psi;
    bool uploaded = false;
};

namespace {

tcng_status multi_build(const tcng_circuit* const* circs, const tcng_pauli_sum* const* hams, int32_t count,
                        const void* const* params, const tcng_state* psi, const tcng_state* lam, double* energy,
                        double* const* grad, double* const* gate_grad, int64_t init_basis, void* ws, size_t ws_bytes,
                        tcng_multi& M) {
    if (!psi || !lam || !energy) return fail(TCNG_E_INVALID, "null argument");
    const int dt = psi[0].dtype;
    if (tcng_status e = multi_check(circs, hams, count, dt)) return e;
    for (int i = 0; i < count; ++i) {
        if (tcng_status e = check_state(&psi[i], "tcng_expect_grad_multi(psi)")) return e;
        if (tcng_status e = check_state(&lam[i], "tcng_expect_grad_multi(lam)")) return e;
        if (psi[i].dtype != dt || lam[i].dtype != dt || psi[i].batch != 1 || lam[i].batch != 1 ||
            psi[i].n_qubits != circs[i]->n || lam[i].n_qubits != circs[i]->n || psi[i].amps == lam[i].amps)
            return fail(TCNG_E_INVALID, "uneven batch: states must be single, distinct and match their circuits");
        if (circs[i]->n_params > 0 && (!params || !params[i] || !grad || !grad[i]))
            return fail(TCNG_E_INVALID, "uneven batch: missing angles or gradient output");
        if (init_basis >= (int64_t(1) << circs[i]->n))
            return fail(TCNG_E_INVALID, "uneven batch: basis index out of range");
    }
    M.L = multi_layout(circs, hams, count, dt);
    const MultiLayout& L = M.L;
    if (!ws || ws_bytes < L.total) return fail(TCNG_E_WORKSPACE, "workspace too small: need " + std::to_string(L.total));
    char* w = static_cast<char*>(ws);
    M.ws = w;
    M.count = count;
    M.dt = dt;
    M.init_basis = init_basis;
    M.psi.assign(psi, psi + count);
    M.rb = circs[0]->tiled[dt].host.cfg.rb;
    M.rbr = circs[0]->tiled[dt].host.cfg.rb_rev;
    std::vector<Job> jobs(count);
    M.builds.resize(count);
    M.fins.resize(count);
    M.bprefix.assign(count + 1, 0);
    M.fprefix.assign(count + 1, 0);
    double* part = reinterpret_cast<double*>(w + L.part_off);
    double* epart = reinterpret_cast<double*>(w + L.epart_off);
    double* ssum = reinterpret_cast<double*>(w + L.ssum_off);
    double* esum = reinterpret_cast<double*>(w + L.esum_off);
    for (int i = 0; i < count; ++i) {
        const tcng_circuit* c = circs[i];
        const tcng_pauli_sum* h = hams[i];
        WsLayout Li;
        Li.fused = L.fused;
        Li.total_slots = std::max(L.fused ? c->fused.host.total_slots : c->tiled[dt].host.total_slots, 1);
        Li.rev_wgs = L.fused ? L.fwgs[i] : MULTI_WGS;
        Li.e_rows = std::max<int>(int(h->tplan[dt].passes.size()), 1);
        Li.e_wgs = MULTI_EWGS;
        jobs[i] = make_job(c, h, &psi[i], lam[i].amps, w + L.opm_off[i], part + L.slot_row[i] * MULTI_WGS,
                           epart + L.erow_row[i] * MULTI_EWGS, Li);
        if (L.fused) {
            jobs[i].fmats = w + L.fmats_off[i];
            jobs[i].opart = reinterpret_cast<double*>(w + L.opart_off[i]);
            if (init_basis >= 0) jobs[i].init_basis1 = init_basis + 1;
        }
        M.builds[i] = BuildJob{c->tiled[dt].ops, params ? params[i] : nullptr, c->cm[dt], w + L.opm_off[i],
                               int32_t(c->gates.size()), 0};
        M.bprefix[i + 1] = M.bprefix[i] + int64_t(c->gates.size());
        const SlotTables& S = L.fused ? c->fused.slots : c->tiled[dt].slots;
        FinishJob F{};
        F.slots = L.fused ? reinterpret_cast<double*>(w + L.fslot_off[i]) : ssum + L.slot_row[i];
        F.erow = esum + L.erow_row[i];
        F.slot_ptr = S.ptr;
        F.slot_idx = S.idx;
        F.gate_slot = S.gate_slot;
        F.u2m = c->u2m[dt];
        F.gate_mat = c->gate_mat;
        F.energy = energy + i;
        F.grad = (grad && c->n_params) ? grad[i] : nullptr;
        F.gate_grad = gate_grad ? gate_grad[i] : nullptr;
        F.n_params = c->n_params;
        F.n_gates = int32_t(c->gates.size());
        F.erows = Li.e_rows;
        M.fins[i] = F;
        M.fprefix[i + 1] = M.fprefix[i] + 1 + c->n_params + (F.gate_grad ? int64_t(c->gates.size()) : 0);
    }
    if (L.fused) {
        M.fjobs.resize(count);
        for (int i = 0; i < count; ++i) {
            const DevFusedPlan& F = circs[i]->fused;
            FusedCircJob& J = M.fjobs[i];
            J.phases = F.phases;
            J.ops = F.ops;
            J.params = (params && circs[i]->n_params) ? static_cast<const float*>(params[i]) : nullptr;
            J.cm = static_cast<const cx<float>*>(circs[i]->cm[0]);
            J.fmats = reinterpret_cast<float*>(w + L.fmats_off[i]);
            J.opart = reinterpret_cast<const double*>(w + L.opart_off[i]);
            J.osum = reinterpret_cast<double*>(w + L.osum_off[i]);
            J.slots = reinterpret_cast<double*>(w + L.fslot_off[i]);
            J.n_blocks = F.host.n_blocks;
            J.wgs = L.fwgs[i];
            J.total_slots = F.host.total_slots;
            J.pstride = circs[i]->n_params;
        }
    }
    M.plan = multi_plan(jobs, circs, hams, count, dt, L.fused, M.rb, M.rbr);
    M.job0 = jobs[0];
    return TCNG_OK;
}

// the host tables into the workspace: stream-ordered copies (sync == false),
// or synchronous ones after the device is idle (a bound batch, whose launches
// then enqueue kernels only)
tcng_status multi_upload(tcng_multi& M, hipStream_t st, bool sync) {
    const MultiLayout& L = M.L;
    char* w = M.ws;
    const int count = M.count;
    struct Part {
        size_t off;
        const void* src;
        size_t bytes;
    };
    std::vector<Part> parts;
    for (int k = 0; k < 3; ++k) {
        parts.push_back({L.jobs_off[k], M.plan.sorted[k].data(), sizeof(Job) * count});
        parts.push_back({L.prefix_off[k], M.plan.prefix[k].data(), sizeof(int64_t) * (count + 2)});
    }
    parts.push_back({L.build_off, M.builds.data(), sizeof(BuildJob) * count});
    parts.push_back({L.build_prefix_off, M.bprefix.data(), sizeof(int64_t) * (count + 1)});
    parts.push_back({L.fin_off, M.fins.data(), sizeof(FinishJob) * count});
    parts.push_back({L.fin_prefix_off, M.fprefix.data(), sizeof(int64_t) * (count + 1)});
    if (L.fused) parts.push_back({L.fjobs_off, M.fjobs.data(), sizeof(FusedCircJob) * count});
    if (sync) HIP_TRY(hipDeviceSynchronize());
    for (const Part& p : parts) {
        if (sync) HIP_TRY(hipMemcpy(w + p.off, p.src, p.bytes, hipMemcpyHostToDevice));
        else HIP_TRY(hipMemcpyAsync(w + p.off, p.src, p.bytes, hipMemcpyHostToDevice, st));
    }
    M.uploaded = true;
    return TCNG_OK;
}

// every kernel of one evaluation (no copies)
tcng_status multi_launch(const tcng_multi& M, hipStream_t st) {
    const MultiLayout& L = M.L;
    char* w = M.ws;
    const int count = M.count, dt = M.dt;
    double* part = reinterpret_cast<double*>(w + L.part_off);
    double* epart = reinterpret_cast<double*>(w + L.epart_off);
    double* ssum = reinterpret_cast<double*>(w + L.ssum_off);
    double* esum = reinterpret_cast<double*>(w + L.esum_off);
    const FinishJob* fins = reinterpret_cast<const FinishJob*>(w + L.fin_off);
    const int64_t* fpre = reinterpret_cast<const int64_t*>(w + L.fin_prefix_off);
    // every Pauli pass writes its rows; circuits with fewer passes leave rows unwritten: clear
    HIP_TRY(launch_zero(epart, size_t(L.e_rows) * MULTI_EWGS, st));
    if (L.fused) {
        const FusedCircJob* djobs = reinterpret_cast<const FusedCircJob*>(w + L.fjobs_off);
        PROF_TRY(F_FUSED_GRAD, launch_fused_multi_mats(djobs, count, L.max_blocks, st));
        if (tcng_status e = launch_multi_fused(M.plan, M.job0, w, L, st)) return e;
        PROF_TRY(F_FUSED_GRAD, launch_fused_multi_grad(djobs, count, L.max_blocks, st));
        PROF_TRY(F_FINISH, launch_finish_multi(part, 0, MULTI_WGS, epart, L.e_rows, MULTI_EWGS, ssum, esum, fins, fpre,
                                               count, M.fprefix[count], st));
        return TCNG_OK;
    }
    if (M.init_basis >= 0)
        for (int i = 0; i < count; ++i) {
            const tcng_state& s = M.psi[i];
            if (dt == TCNG_C64)
                PROF_TRY(F_INIT, launch_init<float>(s.amps, s.stride, s.n_qubits, 1, nullptr, M.init_basis, st));
            else
                PROF_TRY(F_INIT, launch_init<double>(s.amps, s.stride, s.n_qubits, 1, nullptr, M.init_basis, st));
        }
    HIP_TRY(launch_zero(part, size_t(L.slot_rows) * MULTI_WGS, st));
    const BuildJob* bj = reinterpret_cast<const BuildJob*>(w + L.build_off);
    const int64_t* bpre = reinterpret_cast<const int64_t*>(w + L.build_prefix_off);
    const int rb = M.rb, rr = M.rbr;
    tcng_status e = TCNG_OK;
    if (dt == TCNG_C64) {
        HIP_TRY(launch_build_ops_multi<float>(bj, bpre, count, M.bprefix[count], st));
        if (rb == 5 && rr == 4) e = launch_multi_tiled<float, 5, 4>(M.plan, M.job0, w, L, st);
        else if (rb == 5 && rr == 5) e = launch_multi_tiled<float, 5, 5>(M.plan, M.job0, w, L, st);
        else if (rb == 4 && rr == 4) e = launch_multi_tiled<float, 4, 4>(M.plan, M.job0, w, L, st);
        else e = launch_multi_tiled<float, 4, 5>(M.plan, M.job0, w, L, st);
    } else {
        HIP_TRY(launch_build_ops_multi<double>(bj, bpre, count, M.bprefix[count], st));
        if (rb == 4 && rr == 3) e = launch_multi_tiled<double, 4, 3>(M.plan, M.job0, w, L, st);
        else if (rb == 4 && rr == 4) e = launch_multi_tiled<double, 4, 4>(M.plan, M.job0, w, L, st);
        else if (rb == 3 && rr == 3) e = launch_multi_tiled<double, 3, 3>(M.plan, M.job0, w, L, st);
        else e = launch_multi_tiled<double, 3, 4>(M.plan, M.job0, w, L, st);
    }
    if (e) return e;
    PROF_TRY(F_FINISH, launch_finish_multi(part, L.slot_rows, MULTI_WGS, epart, L.e_rows, MULTI_EWGS, ssum, esum, fins,
                                           fpre, count, M.fprefix[count], st));
    return TCNG_OK;
}

}  // namespace

extern "C" {

tcng_status tcng_workspace_size_multi(const tcng_circuit* const* circs, const tcng_pauli_sum* const* hams,
                                      int32_t count, int32_t dtype, size_t* bytes) {
    if (!bytes) return fail(TCNG_E_INVALID, "null output");
    if (tcng_status e = multi_check(circs, hams, count, dtype)) return e;
    *bytes = multi_layout(circs, hams, count, dtype).total;
    return ok();
}

tcng_status tcng_expect_grad_multi(const tcng_circuit* const* circs, const tcng_pauli_sum* const* hams, int32_t count,
                                   const void* const* params, const tcng_state* psi, const tcng_state* lam,
                                   double* energy, double* const* grad, double* const* gate_grad, void* ws,
                                   size_t ws_bytes, void* stream) {
    hipStream_t st = static_cast<hipStream_t>(stream);
    tcng_multi M;
    if (tcng_status e = multi_build(circs, hams, count, params, psi, lam, energy, grad, gate_grad, -1, ws, ws_bytes, M))
        return e;
    if (tcng_status e = multi_upload(M, st, false)) return e;
    if (tcng_status e = multi_launch(M, st)) return e;
    return ok();
}

tcng_status tcng_multi_create(const tcng_circuit* const* circs, const tcng_pauli_sum* const* hams, int32_t count,
                              const void* const* params, const tcng_state* psi, const tcng_state* lam, double* energy,
                              double* const* grad, double* const* gate_grad, int64_t init_basis, void* ws,
                              size_t ws_bytes, tcng_multi** out) {
    if (!out) return fail(TCNG_E_INVALID, "null output handle");
    *out = nullptr;
    auto* M = new (std::nothrow) tcng_multi();
    if (!M) return fail(TCNG_E_ALLOC, "host allocation failed");
    tcng_status e = multi_build(circs, hams, count, params, psi, lam, energy, grad, gate_grad, init_basis, ws,
                                ws_bytes, *M);
    if (!e) e = multi_upload(*M, nullptr, true);
    if (e) {
        delete M;
        return e;
    }
    *out = M;
    return ok();
}

tcng_status tcng_multi_launch(const tcng_multi* m, void* stream) {
    if (!m || !m->uploaded) return fail(TCNG_E_INVALID, "null uneven batch");
    if (tcng_status e = multi_launch(*m, static_cast<hipStream_t>(stream))) return e;
    return ok();
}

tcng_status tcng_multi_destroy(tcng_multi* m) {
    delete m;
    return ok();
}

tcng_status tcng_graph_create_multi(const tcng_multi* m, tcng_graph** out) {
    if (!m || !m->uploaded) return fail(TCNG_E_INVALID, "null uneven batch");
    return capture_graph([&](hipStream_t st) { return multi_launch(*m, st); }, out);
}

tcng_status tcng_circuit_configure(tcng_circuit* c, int32_t dtype, int32_t m_max, int32_t rb, int32_t rb_rev) {
    if (!c) return fail(TCNG_E_INVALID, "null circuit");
    if (dtype != TCNG_C64 && dtype != TCNG_C128) return fail(TCNG_E_INVALID, "bad dtype");
    if (!c->tiled[dtype].valid) return fail(TCNG_E_UNSUPPORTED, "circuit too small for the tiled path");
    TileConfig cfg = tile_config(dtype);
    cfg.m_max = m_max;
    cfg.rb = rb;
    cfg.rb_rev = rb_rev;
    if (!config_ok(cfg, dtype) || std::min(c->n, m_max) < std::max(rb, rb_rev) + 6)
        return fail(TCNG_E_UNSUPPORTED, "tiling not available");
    HIP_TRY(hipDeviceSynchronize());
    if (tcng_status e = make_plan(c, dtype, cfg)) return e;
    return ok();
}

tcng_status tcng_circuit_get_config(const tcng_circuit* c, int32_t dtype, int32_t* m_max, int32_t* rb,
                                    int32_t* rb_rev) {
    if (!c || !m_max || !rb || !rb_rev) return fail(TCNG_E_INVALID, "null argument");
    if (dtype != TCNG_C64 && dtype != TCNG_C128) return fail(TCNG_E_INVALID, "bad dtype");
    if (!c->tiled[dtype].valid) {
        *m_max = *rb = *rb_rev = 0;
        return ok();
    }
    const TileConfig& cfg = c->tiled[dtype].host.cfg;
    *m_max = cfg.m_max;
    *rb = cfg.rb;
    *rb_rev = cfg.rb_rev;
    return ok();
}

namespace {

// structural key of a circuit (gate records, not angle values) for the autotune cache
std::string circuit_key(const tcng_circuit* c, int dtype, int64_t batch) {
    uint64_t h = 1469598103934665603ull;   // FNV-1a
    auto mix = [&](int32_t v) {
        for (int i = 0; i < 4; ++i) { h ^= uint64_t((v >> (8 * i)) & 0xff); h *= 1099511628211ull; }
    };
    mix(c->n);
    for (const tcng_gate& g : c->gates) { mix(g.kind); mix(g.q0); mix(g.q1); }
    int dev = 0;
    hipDeviceProp_t prop{};
    (void)hipGetDevice(&dev);
    (void)hipGetDeviceProperties(&prop, dev);
    std::ostringstream os;
    os << std::hex << h << std::dec << " n" << c->n << " g" << c->gates.size() << " dt" << dtype << " b" << batch
       << " " << prop.gcnArchName;
    return os.str();
}

}  // namespace

tcng_status tcng_circuit_rounds(const tcng_circuit* c, int32_t dtype, int32_t* phases) {
    if (!c || !phases) return fail(TCNG_E_INVALID, "null argument");
    if (dtype != TCNG_C64 && dtype != TCNG_C128) return fail(TCNG_E_INVALID, "bad dtype");
    const DevCircuitPlan& P = c->tiled[dtype];
    *phases = (P.valid && P.host.rounds) ? int32_t(P.host.qphases.size()) : 0;
    return ok();
}

tcng_status tcng_circuit_get_mode(const tcng_circuit* c, int32_t dtype, int32_t* mode) {
    if (!c || !mode) return fail(TCNG_E_INVALID, "null argument");
    if (dtype != TCNG_C64 && dtype != TCNG_C128) return fail(TCNG_E_INVALID, "bad dtype");
    *mode = run_mode(TCNG_MODE_AUTO, c, dtype);
    return ok();
}

tcng_status tcng_autotune(tcng_circuit* c, const tcng_pauli_sum* h, const void* params, const tcng_state* psi,
                          const tcng_state* lam, int32_t repeats, const char* cache_path, double* best_ms,
                          void* stream) {
    if (!c || !h || !psi || !lam) return fail(TCNG_E_INVALID, "null argument");
    if (tcng_status e = check_state(psi, "tcng_autotune(psi)")) return e;
    const int dt = psi->dtype;
    if (repeats < 1) repeats = 1;
    // candidates: every tiling of the tiled passes, then the matrix-core plans
    // with 4- and 5-qubit blocks (complex64)
    struct Cand {
        int mode;
        TileConfig t;
    };
    std::vector<Cand> cands;
    const TileConfig cur = c->tiled[dt].host.cfg;
    if (c->tiled[dt].valid) {
        const TileConfig def = tile_config(dt);
        const int rbs64[2] = {5, 4}, rbs128[2] = {4, 3};
        const int* rbs = dt == TCNG_C64 ? rbs64 : rbs128;
        for (int dm = 0; dm <= 1; ++dm)
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) {
                    TileConfig t = def;
                    t.m_max = def.m_max - dm;
                    t.rb = rbs[i];
                    t.rb_rev = rbs[j];
                    if (config_ok(t, dt) && std::min(c->n, t.m_max) >= std::max(t.rb, t.rb_rev) + 6)
                        cands.push_back({TCNG_MODE_TILED, t});
                }
    }
    if (dt == TCNG_C64 && c->fused.valid) cands.push_back({TCNG_MODE_FUSED, cur});
    if (dt == TCNG_C64 && c->fused5.valid) cands.push_back({TCNG_MODE_FUSED5, cur});
    if (cands.empty()) return ok();   // plain path only: nothing to tune
    const std::string key = circuit_key(c, dt, psi->batch);
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            const size_t bar = line.find(" | ");
            if (bar == std::string::npos || line.substr(0, bar) != key) continue;
            int m = 0, rb = 0, rr = 0, md = TCNG_MODE_TILED;
            double ms = 0;
            const int got = std::sscanf(line.c_str() + bar + 3, "%d %d %d %lf %d", &m, &rb, &rr, &ms, &md);
            if (got >= 4) {
                if (best_ms) *best_ms = ms;
                if (c->tiled[dt].valid)
                    if (tcng_status e = tcng_circuit_configure(c, dt, m, rb, rr)) return e;
                c->tuned_mode[dt] = (got == 5 && valid_mode(md) && md != TCNG_MODE_AUTO) ? md : TCNG_MODE_TILED;
                return ok();
            }
        }
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    // the initial states are overwritten by each run's reverse sweep: keep a copy
    const size_t state_bytes = size_t(psi->batch) * psi->stride * (dt == TCNG_C64 ? 8 : 16);
    void* save = nullptr;
    HIP_TRY(hipMalloc(&save, state_bytes));
    HIP_TRY(hipMemcpyAsync(save, psi->amps, state_bytes, hipMemcpyDeviceToDevice, st));
    double* energy = nullptr;
    double* grad = nullptr;
    HIP_TRY(hipMalloc(&energy, sizeof(double) * psi->batch));
    HIP_TRY(hipMalloc(&grad, sizeof(double) * psi->batch * std::max(c->n_params, 1)));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    double best = 1e300, best_tiled = 1e300;
    Cand best_c = cands[0];
    TileConfig best_t = cur;
    tcng_status err = TCNG_OK;
    for (const Cand& cd : cands) {
        if (cd.mode == TCNG_MODE_TILED && (err = tcng_circuit_configure(c, dt, cd.t.m_max, cd.t.rb, cd.t.rb_rev)))
            break;
        size_t wsb = 0;
        if ((err = tcng_workspace_size(c, h, dt, psi->batch, cd.mode, &wsb))) break;
        void* ws = nullptr;
        if (hipMalloc(&ws, wsb) != hipSuccess) { err = fail(TCNG_E_ALLOC, "autotune workspace"); break; }
        std::vector<double> times;
        for (int r = 0; r <= repeats && !err; ++r) {   // run 0 is a warm-up
            (void)hipMemcpyAsync(psi->amps, save, state_bytes, hipMemcpyDeviceToDevice, st);
            (void)hipEventRecord(e0, st);
            err = tcng_expect_grad(c, params, h, psi, lam, energy, grad, nullptr, cd.mode, ws, wsb, stream);
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (r > 0) times.push_back(ms);
        }
        (void)hipFree(ws);
        if (err) break;
        std::sort(times.begin(), times.end());
        const double med = times[times.size() / 2];
        if (med < best) { best = med; best_c = cd; }
        if (cd.mode == TCNG_MODE_TILED && med < best_tiled) { best_tiled = med; best_t = cd.t; }
    }
    (void)hipMemcpyAsync(psi->amps, save, state_bytes, hipMemcpyDeviceToDevice, st);
    (void)hipStreamSynchronize(st);
    (void)hipFree(save);
    (void)hipFree(energy);
    (void)hipFree(grad);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err) return err;
    // the tiled passes keep their fastest tiling also when another mode wins
    const TileConfig keep = best_t;
    if (c->tiled[dt].valid)
        if (tcng_status e = tcng_circuit_configure(c, dt, keep.m_max, keep.rb, keep.rb_rev)) return e;
    c->tuned_mode[dt] = best_c.mode;
    if (best_ms) *best_ms = best;
    if (cache_path) {
        std::ofstream out(cache_path, std::ios::app);
        out << key << " | " << keep.m_max << " " << keep.rb << " " << keep.rb_rev << " " << best << " " << best_c.mode
            << "\n";
    }
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

tcng_status tcng_rounds_plan_inspect(int32_t n_qubits, const tcng_gate* gates, int32_t n_gates, int32_t n_params,
                                     int32_t tile_bits, int32_t reg_bits, int32_t reg_bits_rev,
                                     int32_t* n_round_passes, int32_t* n_phases, int32_t* bad_layouts) {
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
    if (tile_bits < 9 || tile_bits > 13 || reg_bits < 3 || reg_bits > 5 || reg_bits_rev < 3 || reg_bits_rev > 5)
        return fail(TCNG_E_INVALID, "tiling out of range (tile bits 9..13, register bits 3..5)");
    CircuitPlan P;
    std::vector<tcng_gate> g(gates, gates + n_gates);
    TileConfig cfg = tile_config(TCNG_C64);
    cfg.m_max = tile_bits;
    cfg.rb = reg_bits;
    cfg.rb_rev = reg_bits_rev;
    const std::string why = plan_circuit(n_qubits, g, n_params, cfg, P);
    if (!why.empty()) return fail(TCNG_E_UNSUPPORTED, "planner: " + why);
    int32_t rp = 0;
    for (const QPass& Q : P.qpasses) rp += Q.kind != QK_GENERIC;
    if (n_round_passes) *n_round_passes = rp;
    if (n_phases) *n_phases = int32_t(P.qphases.size());
    if (bad_layouts) *bad_layouts = check_rounds_layouts(P);
    return ok();
}

// ---------------------------------------------------------------------------
// allocation-free value and gradient: the evaluation's workspace is a fixed
// device array of the library (one copy per GPU, held until the process
// ends) instead of caller memory
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;

// host code never uses this name as an address (it is a host-side stand-in):
// the device address comes from hipGetSymbolAddress, once per device
__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// the current device's copy of `scratch` (resolved on its first use there)
tcng_status scratch_address(void** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(TCNG_E_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(TCNG_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TCNG_OK;
}

}  // namespace

extern "C" {

size_t tcng_noalloc_scratch_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

tcng_status tcng_expect_grad_noalloc(const tcng_circuit* c, const void* params, const tcng_pauli_sum* h,
                                     const tcng_state* psi, const tcng_state* lam, double* energy, double* grad,
                                     double* gate_grad, int32_t mode, void* stream) {
    if (!c || !h) return fail(TCNG_E_INVALID, "null circuit or Pauli sum");
    if (tcng_status e = check_state(psi, "tcng_expect_grad_noalloc(psi)")) return e;
    size_t need = 0;
    if (tcng_status e = tcng_workspace_size(c, h, psi->dtype, psi->batch, mode, &need)) return e;
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(TCNG_E_WORKSPACE, "the evaluation needs " + std::to_string(need) +
                                          " bytes of workspace; the allocation-free entry point holds " +
                                          std::to_string(NOALLOC_SCRATCH_BYTES) + " (use tcng_expect_grad)");
    void* ws = nullptr;
    if (tcng_status e = scratch_address(&ws)) return e;
    return tcng_expect_grad(c, params, h, psi, lam, energy, grad, gate_grad, mode, ws, NOALLOC_SCRATCH_BYTES, stream);
}

}  // extern "C"
