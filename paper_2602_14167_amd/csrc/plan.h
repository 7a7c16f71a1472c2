// Host-side planner: schedules a circuit's gates into tiled passes and
// register phases, and groups a Pauli sum by X-mask into tiled passes.
#pragma once

#include <string>
#include <vector>

#include "common.h"

namespace tcng {

struct TileConfig {
    int m_max;   // tile bits (2^m amplitudes per tile)
    int rb;      // register bits per thread in the forward sweep (2^rb amplitudes per thread)
    int lo;      // low qubits always in the tile (memory-contiguous runs of 2^lo amplitudes)
    int rb_rev;  // register bits per thread and state in the reverse sweep
};

struct CircuitPlan {
    TileConfig cfg{};
    // forward sweep (register blocks of 2^rb) and reverse sweep (2^rb_rev):
    // the same passes (tiles, gates, gradient slots), phased separately
    std::vector<Pass> passes, rpasses;
    std::vector<Phase> phases, rphases;
    std::vector<Op> ops, rops;
    int total_slots = 0;
    // gradient assembly: slots of parameter p are slot_idx[slot_ptr[p] .. slot_ptr[p+1])
    std::vector<int32_t> slot_ptr, slot_idx;
    // U2 gates: gate index -> first of its 32 cotangent slots (-1 otherwise)
    std::vector<int32_t> gate_slot;
    // rounds of the same passes, one QPass per pass (kind QK_GENERIC where the
    // pass's gates are not all RY / RZ / CNOT, or all fSim, or a wave's 64
    // lanes do not fit the thread bits): the forward sweep with cfg.rb register
    // bits, the reverse sweep with cfg.rb_rev; `rounds`: some pass has them
    bool rounds = false;
    std::vector<QPass> qpasses, qrpasses;
    std::vector<QPhase> qphases, qrphases;
    std::vector<QStep> qsteps, qrsteps;
};

// Fused passes: the same tiles as the tiled plan, phases of FUSED_K bits that
// hold every qubit of their gates, one block matrix per phase.
struct FusedPlan {
    int m = 0;
    int k = FUSED_K;                        // block bits of every phase (4 or 5)
    std::vector<FPass> passes, rpasses;     // reverse: phases listed in the order the reverse sweep visits them
    std::vector<FPhase> phases, rphases;
    std::vector<Op> ops;                    // gates of the forward phases (r0/r1 = bit of the block index)
    int n_blocks = 0, total_slots = 0;
    std::vector<int32_t> slot_ptr, slot_idx, gate_slot;
};

struct PauliPlan {
    TileConfig cfg{};
    std::vector<PPass> passes;
    std::vector<PGroup> groups;
    std::vector<PClass> classes;
    std::vector<PTerm> terms;
};

struct PauliTermHost {
    uint64_t x, z;
    int ny;
    double c;
};

// Returns an empty string on success, else the reason the plan is impossible.
std::string plan_circuit(int n, const std::vector<tcng_gate>& gates, int n_params, const TileConfig& cfg,
                         CircuitPlan& out);
std::string plan_fused(int n, const std::vector<tcng_gate>& gates, int n_params, int m_max, int lo,
                       FusedPlan& out, int k = FUSED_K);
// LDS layout of a tile of 2^m amplitudes: img[b] = address of local bit b
// alone; 32-lane accesses varying the local bits of v_read (5 bits), or of
// v_write, map to 32 distinct 8-byte bank pairs.
void lds_layout(int m, uint32_t v_read, uint32_t v_write, int32_t* img);
// number of layouts of a fused plan that are not bank-conflict-free bijections
int check_fused_layouts(const FusedPlan& P);
std::string plan_pauli(int n, const std::vector<PauliTermHost>& terms, const TileConfig& cfg, PauliPlan& out);

// Plain path: terms grouped by full X-mask.
void group_pauli_full(const std::vector<PauliTermHost>& terms, std::vector<PGroupFull>& groups,
                      std::vector<PClassFull>& classes, std::vector<PTermFull>& out_terms);

}  // namespace tcng
