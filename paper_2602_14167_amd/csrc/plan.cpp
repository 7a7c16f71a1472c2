// Host-side planner for the tiled passes.
//
// A pass streams the state through the GPU once: every tile of 2^m
// amplitudes whose index bits outside the tile's qubit set T are fixed is
// loaded, has a run of gates applied in registers/LDS, and is written back.
// Gates are scheduled greedily in circuit order: a gate joins the pass when
// all its qubits lie in T and no earlier, not yet applied gate shares a qubit
// with it (gates on disjoint qubits commute, so the result is that of the
// original order).  Inside a pass, register phases are formed the same way:
// a phase holds rb local bits in registers, and a gate joins it when the bits
// it needs in registers fit.
#include "plan.h"

#include <algorithm>
#include <array>
#include <map>

namespace tcng {

namespace {

int popc(uint64_t v) { return __builtin_popcountll(v); }

uint64_t gate_qmask(const tcng_gate& g) {
    uint64_t m = uint64_t(1) << g.q0;
    if (kind_arity(g.kind) == 2) m |= uint64_t(1) << g.q1;
    return m;
}

// Greedy schedule of `rem` (gate indices in order) into tile T.
// Fills `taken` (flags per position in rem) and returns the number taken.
int schedule_into_tile(const std::vector<tcng_gate>& gates, const std::vector<int>& rem, uint64_t T,
                       int slot_budget, std::vector<char>* taken) {
    uint64_t blocked = 0;
    int count = 0, slots = 0;
    for (size_t i = 0; i < rem.size(); ++i) {
        const tcng_gate& g = gates[rem[i]];
        uint64_t qm = gate_qmask(g);
        int s = kind_slots(g.kind);
        bool ok = !(qm & blocked) && ((qm & ~T) == 0) && (slots + s <= slot_budget);
        if (ok) {
            ++count;
            slots += s;
            if (taken) (*taken)[i] = 1;
        } else {
            blocked |= qm;
        }
        if (taken == nullptr && blocked == ~uint64_t(0)) break;
    }
    return count;
}

// terms of one X-group split by their coefficient c * i^{#Y} (order of first appearance)
std::vector<std::pair<std::pair<double, double>, std::vector<int>>> coefficient_classes(
    const std::vector<PauliTermHost>& terms, const std::vector<int>& idx) {
    std::vector<std::pair<std::pair<double, double>, std::vector<int>>> out;
    for (int t : idx) {
        const PauliTermHost& h = terms[t];
        const int r = h.ny & 3;
        const double re = (r == 0) ? h.c : (r == 2 ? -h.c : 0.0);
        const double im = (r == 1) ? h.c : (r == 3 ? -h.c : 0.0);
        bool found = false;
        for (auto& cls : out)
            if (cls.first.first == re && cls.first.second == im) { cls.second.push_back(t); found = true; break; }
        if (!found) out.push_back({{re, im}, {t}});
    }
    return out;
}

uint64_t fill_tile(uint64_t T, int n, int m) {
    for (int q = 0; q < n && popc(T) < m; ++q) T |= uint64_t(1) << q;
    return T;
}

// Register phases of one pass: a phase holds rb local bits in registers; a
// gate joins it when no earlier unapplied gate of the pass shares a qubit and
// the bits it needs in registers fit.
std::string plan_phases(const std::vector<tcng_gate>& gates, const std::vector<int>& sel, const int* qubit_to_local,
                        int m, int rb, const std::vector<int32_t>& gate_slot_first, Pass& P,
                        std::vector<Phase>& phases, std::vector<Op>& ops) {
    P.phase_begin = int(phases.size());
    std::vector<int> prem = sel;
    while (!prem.empty()) {
        uint32_t R = 0;   // local bits in registers
        uint64_t blocked = 0;
        std::vector<int> ph, rest2;
        for (int gi : prem) {
            const tcng_gate& g = gates[gi];
            uint64_t qm = gate_qmask(g);
            uint32_t need = 0;
            const int l0 = qubit_to_local[g.q0];
            const int l1 = kind_arity(g.kind) == 2 ? qubit_to_local[g.q1] : -1;
            if (g.kind == K_CNOT) need = 1u << l1;
            else if (g.kind == K_CZ || g.kind == K_RZZ || kind_diagonal(g.kind)) need = 0;
            else need = (1u << l0) | (l1 >= 0 ? (1u << l1) : 0u);
            if (!(qm & blocked) && popc(R | need) <= rb) {
                R |= need;
                ph.push_back(gi);
            } else {
                blocked |= qm;
                rest2.push_back(gi);
            }
        }
        prem.swap(rest2);
        // fill the register set to exactly rb bits, preferring high local bits
        // (keeps consecutive lanes on consecutive LDS addresses)
        for (int b = m - 1; b >= 0 && popc(R) < rb; --b) R |= 1u << b;
        Phase F{};
        for (int i = 0; i < 6; ++i) F.R[i] = -1;
        int ri = 0, reg_of_local[MAX_TILE_BITS];
        for (int b = 0; b < MAX_TILE_BITS; ++b) reg_of_local[b] = -1;
        for (int b = 0; b < m; ++b)
            if ((R >> b) & 1) { F.R[ri] = b; reg_of_local[b] = ri; ++ri; }
        F.op_begin = int(ops.size());
        for (int gi : ph) {
            const tcng_gate& g = gates[gi];
            Op o{};
            o.kind = g.kind;
            o.p0 = g.p0;
            o.p1 = g.p1;
            o.mat = g.mat;
            o.gate = gi;
            o.slot = gate_slot_first[gi];
            const int l0 = qubit_to_local[g.q0];
            const int l1 = kind_arity(g.kind) == 2 ? qubit_to_local[g.q1] : -1;
            o.lb0 = l0;
            o.lb1 = l1;
            o.r0 = reg_of_local[l0];
            o.r1 = l1 >= 0 ? reg_of_local[l1] : -1;
            switch (g.kind) {
                case K_RZ: case K_Z: case K_S: o.type = OP_DIAG1; break;
                case K_CZ: case K_RZZ: o.type = OP_DIAG2; break;
                case K_CNOT: o.type = OP_CX; break;
                case K_FSIM: o.type = OP_FSIM; break;
                case K_U2: o.type = OP_DENSE2; break;
                case K_RY: case K_H: case K_X: o.type = OP_REAL1; break;
                case K_RX: o.type = OP_RX; break;
                default: o.type = OP_DENSE1; break;   // Y, U1
            }
            const bool one = o.type == OP_DENSE1 || o.type == OP_REAL1 || o.type == OP_RX;
            const bool two = o.type == OP_DENSE2 || o.type == OP_FSIM;
            if ((one && o.r0 < 0) || (o.type == OP_CX && o.r1 < 0) || (two && (o.r0 < 0 || o.r1 < 0)))
                return "internal: register operand missing";
            ops.push_back(o);
        }
        F.op_end = int(ops.size());
        phases.push_back(F);
    }
    P.phase_end = int(phases.size());
    return "";
}

// the LDS layouts between the count phases of one rounds pass (QPhase::uimg,
// cimg, rimg, ruimg; cimg holds C(e_b) on entry), below
void rounds_lds_layouts(int m, QPhase* ph, int count, int qreg);

// Rotation rounds of one pass (see QPhase).  A phase takes up to qreg qubits
// whose first remaining gate is a rotation, then steps: each step applies, per
// register qubit, its first remaining gate if that is an RY, then its next if
// that is an RZ.  Then every CNOT whose qubits no earlier remaining gate
// touches joins the phase's permutation, in circuit order.
std::string plan_rounds(const std::vector<tcng_gate>& gates, const std::vector<int>& sel, const int* qubit_to_local,
                        int m, int qreg, const std::vector<int32_t>& gate_slot_first, std::vector<QPhase>& phases,
                        std::vector<QStep>& steps, QPass& qp) {
    qp.phase_begin = int(phases.size());
    const size_t first_step = steps.size();
    size_t cnots = 0;
    std::vector<int> rem = sel;
    auto first_gate = [&](int q) -> int {   // position in rem of the first remaining gate on q
        for (size_t i = 0; i < rem.size(); ++i)
            if ((gate_qmask(gates[rem[i]]) >> q) & 1) return int(i);
        return -1;
    };
    auto drop = [&](std::vector<char>& mark) {
        std::vector<int> keep;
        for (size_t i = 0; i < rem.size(); ++i)
            if (!mark[i]) keep.push_back(rem[i]);
        rem.swap(keep);
    };
    while (!rem.empty()) {
        // register qubits: the first qreg whose first remaining gate is a rotation
        std::vector<int> R;
        for (size_t i = 0; i < rem.size() && int(R.size()) < qreg; ++i) {
            const tcng_gate& g = gates[rem[i]];
            if (g.kind == K_CNOT) continue;
            if (std::find(R.begin(), R.end(), g.q0) != R.end()) continue;
            if (first_gate(g.q0) == int(i)) R.push_back(g.q0);
        }
        QPhase F{};
        F.step_begin = int(steps.size());
        for (;;) {
            QStep S{};
            for (int b = 0; b < QREG; ++b) S.ry[b] = S.rz[b] = S.sy[b] = S.sz[b] = -1;
            S.kind = QK_ROT;
            bool took = false;
            for (int round = 0; round < 2; ++round) {
                const int kind = round == 0 ? K_RY : K_RZ;
                std::vector<char> mark(rem.size(), 0);
                for (size_t b = 0; b < R.size(); ++b) {
                    const int i = first_gate(R[b]);
                    if (i < 0 || gates[rem[i]].kind != kind) continue;
                    const int gi = rem[i];
                    (round == 0 ? S.ry : S.rz)[b] = gi;
                    (round == 0 ? S.sy : S.sz)[b] = gate_slot_first[gi];
                    mark[i] = 1;
                    took = true;
                }
                drop(mark);
            }
            if (!took) break;
            steps.push_back(S);
        }
        F.step_end = int(steps.size());
        // the phase's CNOTs: images of the local basis bits under their product
        for (int b = 0; b < 16; ++b) F.cimg[b] = b < m ? (1 << b) : 0;
        {
            std::vector<char> mark(rem.size(), 0);
            uint64_t blocked = 0;
            for (size_t i = 0; i < rem.size(); ++i) {
                const tcng_gate& g = gates[rem[i]];
                const uint64_t qm = gate_qmask(g);
                if (g.kind == K_CNOT && !(qm & blocked)) {
                    const int lc = qubit_to_local[g.q0], lt = qubit_to_local[g.q1];
                    for (int b = 0; b < m; ++b)
                        if ((F.cimg[b] >> lc) & 1) F.cimg[b] ^= 1 << lt;
                    F.has_map = 1;
                    mark[i] = 1;
                    ++cnots;
                } else {
                    blocked |= qm;
                }
            }
            drop(mark);
        }
        if (F.step_end == F.step_begin && !F.has_map) return "internal: rotation rounds made no progress";
        // register bits: the phase's qubits, then the highest unused local bits
        uint32_t used = 0;
        for (size_t b = 0; b < R.size(); ++b) {
            F.R[b] = qubit_to_local[R[b]];
            used |= 1u << F.R[b];
        }
        for (int b = int(R.size()), l = m - 1; b < qreg; ++b) {
            while ((used >> l) & 1) --l;
            F.R[b] = l;
            used |= 1u << l;
        }
        for (int b = qreg; b < QREG; ++b) F.R[b] = -1;
        for (int b = 0; b < qreg; ++b) {
            F.rmask |= 1 << F.R[b];
            F.rimg[b] = F.cimg[F.R[b]];
        }
        phases.push_back(F);
    }
    qp.phase_end = int(phases.size());
    qp.kind = QK_ROT;
    rounds_lds_layouts(m, phases.data() + qp.phase_begin, qp.phase_end - qp.phase_begin, qreg);
    size_t rots = 0;
    for (size_t k = first_step; k < steps.size(); ++k)
        for (int b = 0; b < QREG; ++b) rots += (steps[k].ry[b] >= 0) + (steps[k].rz[b] >= 0);
    if (rots + cnots != sel.size()) return "internal: rotation rounds lost a gate";
    return "";
}

// LDS layouts of the rounds (see QPhase).  The boundary between phases k - 1
// and k of a pass is seen by the lanes of both: through C_{k-1} from phase
// k - 1 (its lanes vary its 5 lowest non-register local bits) and plainly from
// phase k, in the forward and in the reverse sweep alike.  Its layout A is
// chosen so that, on both sides, the lanes' local-index vectors for lane bits
// 0..s-1 map onto independent low s bits of the LDS slot, for s = 3, 4 and 5:
// 8, 16 and 32 consecutive lanes then address distinct banks (amplitudes of
// 16 and 8 bytes, 32 or 64 banks of 4 bytes).  The first and last boundaries
// keep the tile load / store swizzle.  Deterministic (a fixed-seed search).
namespace {

int rank_of(std::vector<uint32_t> v) {
    int r = 0;
    for (int b = 0; b < 32; ++b) {
        size_t p = size_t(r);
        while (p < v.size() && !((v[p] >> b) & 1)) ++p;
        if (p >= v.size()) continue;
        std::swap(v[p], v[size_t(r)]);
        for (size_t i = 0; i < v.size(); ++i)
            if (int(i) != r && ((v[i] >> b) & 1)) v[i] ^= v[size_t(r)];
        ++r;
    }
    return r;
}

// rows[i]: bit i of the slot as a mask over the local index
bool lanes_spread(const uint32_t* rows, const uint32_t* vec) {
    for (int s = 3; s <= 5; ++s) {
        std::vector<uint32_t> x(size_t(s), 0u);
        for (int j = 0; j < s; ++j)
            for (int i = 0; i < s; ++i) x[size_t(j)] |= uint32_t(popc(uint64_t(rows[i] & vec[j])) & 1) << i;
        if (rank_of(x) != s) return false;
    }
    return true;
}

// images of the local bits under the layout whose low 5 slot bits are rows[0..4]
// (the other slot bits: local bits, taken in increasing order while independent)
void layout_images(int m, const uint32_t* low_rows, int32_t* img) {
    std::vector<uint32_t> rows(low_rows, low_rows + 5);
    for (int j = 0; j < m && int(rows.size()) < m; ++j) {
        std::vector<uint32_t> t = rows;
        t.push_back(1u << j);
        if (rank_of(t) == int(t.size())) rows.push_back(1u << j);
    }
    for (int b = 0; b < 16; ++b) {
        uint32_t v = 0;
        if (b < m)
            for (size_t i = 0; i < rows.size(); ++i) v |= ((rows[i] >> b) & 1u) << i;
        img[b] = int32_t(v);
    }
}

uint32_t apply_images(const int32_t* img, uint32_t v) {
    uint32_t r = 0;
    for (int b = 0; b < 16; ++b)
        if ((v >> b) & 1) r ^= uint32_t(img[b]);
    return r;
}

}  // namespace

void rounds_lds_layouts(int m, QPhase* ph, int count, int qreg) {
    if (count <= 0) return;
    const uint32_t full = (1u << m) - 1u;
    std::vector<std::array<int32_t, 16>> A(size_t(count) + 1);
    for (int b = 0; b < 16; ++b) A[0][size_t(b)] = b < m ? int32_t(tile_swz(1u << b)) : 0;
    A[size_t(count)] = A[0];
    auto lanes = [&](const QPhase& F, bool mapped, uint32_t* vec) {
        int k = 0;
        for (int b = 0; b < m && k < 5; ++b)
            if (!((F.rmask >> b) & 1)) vec[k++] = mapped ? uint32_t(F.cimg[b]) : (1u << b);
    };
    uint32_t swz_rows[5], id_rows[5];
    for (int i = 0; i < 5; ++i) {
        swz_rows[i] = 1u << i;
        if (i >= 1 && i <= 3) swz_rows[i] |= 1u << (i + 4);
        id_rows[i] = 1u << i;
    }
    uint64_t seed = 0x9E3779B97F4A7C15ull;
    for (int k = 1; k < count; ++k) {
        uint32_t w[5], r[5];
        lanes(ph[k - 1], true, w);
        lanes(ph[k], false, r);
        const uint32_t* pick = nullptr;
        uint32_t rows[5];
        if (lanes_spread(swz_rows, w) && lanes_spread(swz_rows, r)) pick = swz_rows;
        else if (lanes_spread(id_rows, w) && lanes_spread(id_rows, r)) pick = id_rows;
        for (int tries = 0; !pick && tries < 200000; ++tries) {
            for (int i = 0; i < 5; ++i) {
                seed ^= seed << 13; seed ^= seed >> 7; seed ^= seed << 17;
                rows[i] = uint32_t(seed) & full;
            }
            if (lanes_spread(rows, w) && lanes_spread(rows, r)) pick = rows;
        }
        if (pick) layout_images(m, pick, A[size_t(k)].data());
        else A[size_t(k)] = A[0];   // (not expected: the swizzle, with its conflicts)
    }
    for (int k = 0; k < count; ++k) {
        QPhase& F = ph[k];
        int32_t c[16];
        for (int b = 0; b < 16; ++b) {
            c[b] = b < m ? int32_t(apply_images(A[size_t(k) + 1].data(), uint32_t(F.cimg[b]))) : 0;
            F.uimg[b] = A[size_t(k)][size_t(b)];
        }
        for (int b = 0; b < 16; ++b) F.cimg[b] = c[b];
        for (int i = 0; i < QREG; ++i) {
            F.rimg[i] = i < qreg ? F.cimg[F.R[i]] : 0;
            F.ruimg[i] = i < qreg ? F.uimg[F.R[i]] : 0;
        }
    }
}

// fSim rounds of one pass (see QPhase).  A phase's register qubits form a
// chain grown from the first remaining gate: later fSim gates (in circuit order)
// that join one end of the chain with a new qubit extend it, up to qreg
// qubits, so that chain neighbours sit on adjacent register bits.  Steps then
// take, per pair slot, the gate that is the first remaining gate of both of
// the pair's qubits: pairs (0,1), (2,3), then (1,2), (3,4).
std::string plan_rounds_fsim(const std::vector<tcng_gate>& gates, const std::vector<int>& sel,
                             const int* qubit_to_local, int m, int qreg, const std::vector<int32_t>& gate_slot_first,
                             std::vector<QPhase>& phases, std::vector<QStep>& steps, QPass& qp) {
    static const int pair_lo[4] = {0, 2, 1, 3};   // pair slot k: register bits (pair_lo[k], pair_lo[k] + 1)
    qp.phase_begin = int(phases.size());
    qp.kind = QK_FSIM;
    size_t taken_total = 0;
    std::vector<int> rem = sel;
    auto first_gate = [&](int q) -> int {
        for (size_t i = 0; i < rem.size(); ++i)
            if ((gate_qmask(gates[rem[i]]) >> q) & 1) return int(i);
        return -1;
    };
    while (!rem.empty()) {
        std::vector<int> chain = {gates[rem[0]].q0};
        if (gates[rem[0]].kind == K_FSIM) chain.push_back(gates[rem[0]].q1);
        for (size_t i = 1; i < rem.size() && int(chain.size()) < qreg; ++i) {
            const tcng_gate& g = gates[rem[i]];
            if (g.kind != K_FSIM) continue;
            const bool in0 = std::find(chain.begin(), chain.end(), g.q0) != chain.end();
            const bool in1 = std::find(chain.begin(), chain.end(), g.q1) != chain.end();
            if (in0 == in1) continue;
            const int inner = in0 ? g.q0 : g.q1, outer = in0 ? g.q1 : g.q0;
            if (inner == chain.back()) chain.push_back(outer);
            else if (inner == chain.front()) chain.insert(chain.begin(), outer);
        }
        const int len = int(chain.size());
        QPhase F{};
        for (int b = 0; b < len; ++b) {   // Hadamards first
            const int i = first_gate(chain[b]);
            if (i >= 0 && gates[rem[i]].kind == K_H) {
                F.hmask |= 1 << b;
                rem.erase(rem.begin() + i);
                ++taken_total;
            }
        }
        F.step_begin = int(steps.size());
        for (;;) {
            QStep S{};
            for (int b = 0; b < QREG; ++b) S.ry[b] = S.rz[b] = S.sy[b] = S.sz[b] = -1;
            S.kind = QK_FSIM;
            bool took = false;
            for (int k = 0; k < 4; ++k) {
                const int p = pair_lo[k];
                if (p + 1 >= len || p + 1 >= qreg) continue;
                const int a = first_gate(chain[p]), b = first_gate(chain[p + 1]);
                if (a < 0 || a != b || gates[rem[a]].kind != K_FSIM) continue;
                const int gi = rem[a];
                S.ry[k] = gi;
                S.sy[k] = gate_slot_first[gi];
                rem.erase(rem.begin() + a);
                took = true;
                ++taken_total;
            }
            if (!took) break;
            steps.push_back(S);
        }
        F.step_end = int(steps.size());
        if (F.step_end == F.step_begin && !F.hmask) return "internal: fSim rounds made no progress";
        for (int b = 0; b < 16; ++b) F.cimg[b] = b < m ? (1 << b) : 0;
        uint32_t used = 0;
        for (int b = 0; b < len; ++b) {
            F.R[b] = qubit_to_local[chain[b]];
            used |= 1u << F.R[b];
        }
        for (int b = len, l = m - 1; b < qreg; ++b) {
            while ((used >> l) & 1) --l;
            F.R[b] = l;
            used |= 1u << l;
        }
        for (int b = qreg; b < QREG; ++b) F.R[b] = -1;
        for (int b = 0; b < qreg; ++b) {
            F.rmask |= 1 << F.R[b];
            F.rimg[b] = F.cimg[F.R[b]];
        }
        phases.push_back(F);
    }
    qp.phase_end = int(phases.size());
    rounds_lds_layouts(m, phases.data() + qp.phase_begin, qp.phase_end - qp.phase_begin, qreg);
    if (taken_total != sel.size()) return "internal: fSim rounds lost a gate";
    return "";
}

}  // namespace

std::string plan_circuit(int n, const std::vector<tcng_gate>& gates, int n_params, const TileConfig& cfg,
                         CircuitPlan& out) {
    out = CircuitPlan();
    out.cfg = cfg;
    const int m = std::min(n, cfg.m_max);
    const int lo = std::min(cfg.lo, m);
    if (m < cfg.rb || m < cfg.rb_rev) return "tile smaller than the register block";
    if (cfg.rb < 1 || cfg.rb > MAX_RB || cfg.rb_rev < 1 || cfg.rb_rev > MAX_RB) return "register block out of range";
    const uint64_t lo_mask = (lo >= 64) ? ~uint64_t(0) : ((uint64_t(1) << lo) - 1);
    const uint64_t all_mask = (n >= 64) ? ~uint64_t(0) : ((uint64_t(1) << n) - 1);

    std::vector<int> rem(gates.size());
    for (size_t i = 0; i < gates.size(); ++i) rem[i] = int(i);
    // rounds: a wave's 64 lanes hold thread bits in both sweeps
    const bool rounds_ok = m >= std::max(cfg.rb, cfg.rb_rev) + 6 && cfg.rb >= 3 && cfg.rb_rev >= 3;
    out.rounds = false;

    // per-gate slot assignment (global, in reverse-sweep order is not needed:
    // slots are contiguous per pass, assigned as passes are formed)
    std::vector<int32_t> gate_slot_first(gates.size(), -1);
    out.gate_slot.assign(gates.size(), -1);

    while (!rem.empty()) {
        // ---- choose the tile
        std::vector<uint64_t> cands;
        if (n <= m) {
            cands.push_back(all_mask);
        } else {
            const int h = m - lo;
            for (int a = lo; a + h <= n; ++a) {
                uint64_t w = lo_mask;
                for (int q = a; q < a + h; ++q) w |= uint64_t(1) << q;
                cands.push_back(w);
            }
            // frontier candidate: qubits of the earliest unblocked gates
            uint64_t T = lo_mask, blocked = 0;
            for (int gi : rem) {
                uint64_t qm = gate_qmask(gates[gi]);
                if (!(qm & blocked) && popc(T | qm) <= m) T |= qm;
                else blocked |= qm;
            }
            cands.push_back(fill_tile(T, n, m));
        }
        int best = -1, best_count = -1;
        for (size_t c = 0; c < cands.size(); ++c) {
            int cnt = schedule_into_tile(gates, rem, cands[c], RED_SLOTS, nullptr);
            if (cnt > best_count) { best_count = cnt; best = int(c); }
        }
        if (best_count <= 0) return "planner made no progress (gate needs more than the tile's qubits)";
        const uint64_t T = cands[best];
        std::vector<char> taken(rem.size(), 0);
        schedule_into_tile(gates, rem, T, RED_SLOTS, &taken);
        std::vector<int> sel, rest;
        for (size_t i = 0; i < rem.size(); ++i) (taken[i] ? sel : rest).push_back(rem[i]);
        rem.swap(rest);

        // ---- local bit map
        Pass P{};
        P.m = m;
        P.lo = lo;
        P.tile_mask = T;
        int qubit_to_local[64];
        for (int q = 0; q < 64; ++q) qubit_to_local[q] = -1;
        for (int i = 0; i < 16; ++i) P.local_qubit[i] = -1;
        int li = 0;
        for (int q = 0; q < n; ++q)
            if ((T >> q) & 1) { qubit_to_local[q] = li; P.local_qubit[li] = q; ++li; }
        if (li != m) return "internal: tile size mismatch";
        for (int q = 0; q < lo; ++q)
            if (qubit_to_local[q] != q) return "internal: low qubits not contiguous";

        // ---- slots of this pass
        P.slot_base = out.total_slots;
        int pass_slots = 0;
        for (int gi : sel) {
            int s = kind_slots(gates[gi].kind);
            if (s) { gate_slot_first[gi] = pass_slots; pass_slots += s; }
        }
        P.n_slots = pass_slots;
        out.total_slots += pass_slots;

        // ---- register phases, forward and reverse block sizes
        Pass R = P;
        std::string why = plan_phases(gates, sel, qubit_to_local, m, cfg.rb, gate_slot_first, P, out.phases, out.ops);
        if (!why.empty()) return why;
        why = plan_phases(gates, sel, qubit_to_local, m, cfg.rb_rev, gate_slot_first, R, out.rphases, out.rops);
        if (!why.empty()) return why;
        // ---- rounds, when every gate of the pass is of one rounds kind
        int kind = rounds_ok ? QK_ROT : QK_GENERIC;
        for (int gi : sel)
            if (gates[gi].kind != K_RY && gates[gi].kind != K_RZ && gates[gi].kind != K_CNOT) kind = QK_GENERIC;
        if (rounds_ok && kind == QK_GENERIC) {
            kind = QK_FSIM;
            for (int gi : sel)
                if (gates[gi].kind != K_FSIM && gates[gi].kind != K_H) kind = QK_GENERIC;
        }
        QPass Q{}, QR{};
        Q.phase_begin = Q.phase_end = int(out.qphases.size());
        QR.phase_begin = QR.phase_end = int(out.qrphases.size());
        if (kind == QK_ROT) {
            why = plan_rounds(gates, sel, qubit_to_local, m, cfg.rb, gate_slot_first, out.qphases, out.qsteps, Q);
            if (why.empty())
                why = plan_rounds(gates, sel, qubit_to_local, m, cfg.rb_rev, gate_slot_first, out.qrphases,
                                  out.qrsteps, QR);
        } else if (kind == QK_FSIM) {
            why = plan_rounds_fsim(gates, sel, qubit_to_local, m, cfg.rb, gate_slot_first, out.qphases, out.qsteps,
                                   Q);
            if (why.empty())
                why = plan_rounds_fsim(gates, sel, qubit_to_local, m, cfg.rb_rev, gate_slot_first, out.qrphases,
                                       out.qrsteps, QR);
        }
        if (!why.empty()) return why;
        out.qpasses.push_back(Q);
        out.qrpasses.push_back(QR);
        if (kind != QK_GENERIC) out.rounds = true;
        out.passes.push_back(P);
        out.rpasses.push_back(R);
    }

    // ---- gradient assembly tables
    std::vector<std::vector<int32_t>> per_param(std::max(n_params, 0));
    for (const Pass& P : out.passes)
        for (int f = P.phase_begin; f < P.phase_end; ++f)
            for (int o = out.phases[f].op_begin; o < out.phases[f].op_end; ++o) {
                const Op& op = out.ops[o];
                if (op.slot < 0) continue;
                const int gslot = P.slot_base + op.slot;
                const tcng_gate& g = gates[op.gate];
                if (g.kind == K_U2) {
                    out.gate_slot[op.gate] = gslot;
                } else {
                    if (g.p0 >= 0) per_param[g.p0].push_back(gslot);
                    if (kind_nparams(g.kind) == 2 && g.p1 >= 0) per_param[g.p1].push_back(gslot + 1);
                }
            }
    out.slot_ptr.assign(1, 0);
    for (auto& v : per_param) {
        std::sort(v.begin(), v.end());
        out.slot_idx.insert(out.slot_idx.end(), v.begin(), v.end());
        out.slot_ptr.push_back(int32_t(out.slot_idx.size()));
    }
    return "";
}

void lds_layout(int m, uint32_t v_read, uint32_t v_write, int32_t* img) {
    for (int b = 0; b < MAX_TILE_BITS; ++b) img[b] = 0;
    int pos[MAX_TILE_BITS];
    int k = 0;
    for (int b = 0; b < m; ++b)
        if ((v_read >> b) & 1) pos[b] = k++;
    for (int b = 0; b < m; ++b)
        if (!((v_read >> b) & 1)) pos[b] = k++;
    for (int b = 0; b < m; ++b) img[b] = 1 << pos[b];
    // bits written but not read in the low positions are folded onto the low
    // positions of bits read but not written (XOR: the map stays a bijection)
    int extra[MAX_TILE_BITS], free_pos[MAX_TILE_BITS], ne = 0, nf = 0;
    for (int b = 0; b < m; ++b) {
        const bool r = (v_read >> b) & 1, w = (v_write >> b) & 1;
        if (w && !r) extra[ne++] = b;
        if (r && !w) free_pos[nf++] = pos[b];
    }
    for (int i = 0; i < ne && i < nf; ++i) img[extra[i]] |= 1 << free_pos[i];
}

namespace {

// the 5 lowest column bits of a phase (the bits 32 consecutive columns vary)
uint32_t low_columns(int m, uint32_t rmask) {
    uint32_t v = 0;
    int k = 0;
    for (int b = 0; b < m && k < 5; ++b)
        if (!((rmask >> b) & 1)) { v |= 1u << b; ++k; }
    return v;
}

// column bit c (in increasing order of the non-block bits) of a phase
int column_bit(int m, uint32_t rmask, int c) {
    for (int b = 0; b < m; ++b)
        if (!((rmask >> b) & 1) && c-- == 0) return b;
    return -1;
}

}  // namespace

// The fused reverse keeps one outer product per block and forms every gradient
// slot after the sweep, so a fused pass has no per-pass slot limit (the tiled
// passes reduce their slots inside the pass and keep RED_SLOTS).
constexpr int FUSED_SLOT_BUDGET = 1 << 30;

std::string plan_fused(int n, const std::vector<tcng_gate>& gates, int n_params, int m_max, int lo_cfg,
                       FusedPlan& out, int kb) {
    out = FusedPlan();
    if (kb != 4 && kb != 5) return "fused blocks have 4 or 5 qubits";
    const int m = std::min(n, m_max);
    const int lo = std::min(lo_cfg, m);
    if (m < kb + 5) return "tile too small for fused blocks (needs 2^(K+5) amplitudes)";
    out.m = m;
    out.k = kb;
    const uint64_t lo_mask = (lo >= 64) ? ~uint64_t(0) : ((uint64_t(1) << lo) - 1);
    const uint64_t all_mask = (n >= 64) ? ~uint64_t(0) : ((uint64_t(1) << n) - 1);
    const uint32_t ldst = 0x3Eu;   // tile load / store: 32 lanes vary local bits 1..5

    std::vector<int> rem(gates.size());
    for (size_t i = 0; i < gates.size(); ++i) rem[i] = int(i);
    out.gate_slot.assign(gates.size(), -1);

    while (!rem.empty()) {
        // ---- the tile (same choice as the tiled plan)
        std::vector<uint64_t> cands;
        if (n <= m) {
            cands.push_back(all_mask);
        } else {
            const int h = m - lo;
            for (int a = lo; a + h <= n; ++a) {
                uint64_t w = lo_mask;
                for (int q = a; q < a + h; ++q) w |= uint64_t(1) << q;
                cands.push_back(w);
            }
            uint64_t T = lo_mask, blocked = 0;
            for (int gi : rem) {
                uint64_t qm = gate_qmask(gates[gi]);
                if (!(qm & blocked) && popc(T | qm) <= m) T |= qm;
                else blocked |= qm;
            }
            cands.push_back(fill_tile(T, n, m));
        }
        int best = -1, best_count = -1;
        for (size_t c = 0; c < cands.size(); ++c) {
            int cnt = schedule_into_tile(gates, rem, cands[c], FUSED_SLOT_BUDGET, nullptr);
            if (cnt > best_count) { best_count = cnt; best = int(c); }
        }
        if (best_count <= 0) return "planner made no progress";
        const uint64_t T = cands[best];
        std::vector<char> taken(rem.size(), 0);
        schedule_into_tile(gates, rem, T, FUSED_SLOT_BUDGET, &taken);
        std::vector<int> sel, rest;
        for (size_t i = 0; i < rem.size(); ++i) (taken[i] ? sel : rest).push_back(rem[i]);
        rem.swap(rest);

        FPass P{};
        P.m = m;
        P.lo = lo;
        P.tile_mask = T;
        int qubit_to_local[64];
        for (int q = 0; q < 64; ++q) qubit_to_local[q] = -1;
        for (int i = 0; i < 16; ++i) P.local_qubit[i] = -1;
        int li = 0;
        for (int q = 0; q < n; ++q)
            if ((T >> q) & 1) { qubit_to_local[q] = li; P.local_qubit[li] = q; ++li; }
        if (li != m) return "internal: tile size mismatch";

        // ---- blocks: a gate joins while its qubits fit in kb local bits
        // and no earlier gate of the pass left out shares a qubit with it
        std::vector<uint32_t> rmasks;
        const int first = int(out.phases.size());
        std::vector<int> prem = sel;
        while (!prem.empty()) {
            if (int(out.phases.size()) - first == (kb == 5 ? FUSED5_MAX_BLOCKS : FUSED_MAX_BLOCKS)) {
                // the rest of the pass goes back to the queue (disjoint from
                // everything it overtakes, so order is preserved)
                std::vector<int> back = prem;
                back.insert(back.end(), rem.begin(), rem.end());
                std::sort(back.begin(), back.end());
                rem.swap(back);
                break;
            }
            uint32_t R = 0;
            uint64_t blocked = 0;
            std::vector<int> ph, rest2;
            for (int gi : prem) {
                const tcng_gate& g = gates[gi];
                const uint64_t qm = gate_qmask(g);
                uint32_t need = 1u << qubit_to_local[g.q0];
                if (kind_arity(g.kind) == 2) need |= 1u << qubit_to_local[g.q1];
                if (!(qm & blocked) && popc(R | need) <= kb) {
                    R |= need;
                    ph.push_back(gi);
                } else {
                    blocked |= qm;
                    rest2.push_back(gi);
                }
            }
            prem.swap(rest2);
            for (int b = m - 1; b >= 0 && popc(R) < kb; --b) R |= 1u << b;
            FPhase F{};
            F.k = kb;
            for (int t = 0; t < FUSED_KMAX; ++t) F.R[t] = -1;
            int reg_of_local[MAX_TILE_BITS];
            for (int b = 0; b < MAX_TILE_BITS; ++b) reg_of_local[b] = -1;
            int t = 0, kc = 0;
            for (int i = 0; i < 9; ++i) F.C[i] = -1;
            for (int b = 0; b < m; ++b) {
                if ((R >> b) & 1) { F.R[t] = b; reg_of_local[b] = t; ++t; }
                else if (kc < 9) F.C[kc++] = b;
            }
            F.block = out.n_blocks++;
            F.op_begin = int(out.ops.size());
            for (int gi : ph) {
                const tcng_gate& g = gates[gi];
                Op o{};
                o.kind = g.kind;
                o.p0 = g.p0;
                o.p1 = g.p1;
                o.mat = g.mat;
                o.gate = gi;
                o.slot = -1;
                o.r0 = reg_of_local[qubit_to_local[g.q0]];
                o.r1 = kind_arity(g.kind) == 2 ? reg_of_local[qubit_to_local[g.q1]] : -1;
                o.lb0 = o.lb1 = -1;
                o.type = kind_arity(g.kind);
                out.ops.push_back(o);
            }
            F.op_end = int(out.ops.size());
            out.phases.push_back(F);
            rmasks.push_back(R);
        }
        const int last = int(out.phases.size());
        P.phase_begin = first;
        P.phase_end = last;
        // gradient slots of the gates this pass applies (global numbering)
        P.slot_base = out.total_slots;
        int pass_slots = 0;
        for (size_t o = size_t(out.phases[first].op_begin); o < out.ops.size(); ++o) {
            const int sl = kind_slots(out.ops[o].kind);
            if (sl) { out.ops[o].slot = P.slot_base + pass_slots; pass_slots += sl; }
        }
        P.n_slots = pass_slots;
        out.total_slots += pass_slots;

        // ---- layouts.  Forward: the load writes bits 1..5, phase f reads and
        // writes its 5 lowest column bits, the store reads bits 1..5.
        // Reverse (phases visited last to first): phase f writes its block
        // bits plus column bit 2 (one float per lane, 32 components of two
        // columns per 64 lanes); with 5 block bits, one half at a time (the top
        // block bit is fixed in a write).
        const int F = last - first;
        auto lowc = [&](int i) { return low_columns(m, rmasks[i]); };
        lds_layout(m, lowc(0), ldst, P.ld);
        for (int i = 0; i < F; ++i) {
            FPhase& Ph = out.phases[first + i];
            const uint32_t vw_prev = i == 0 ? ldst : lowc(i - 1);
            lds_layout(m, lowc(i), vw_prev, Ph.rd);
            if (i + 1 < F) lds_layout(m, lowc(i + 1), lowc(i), Ph.wr);
            else lds_layout(m, ldst, lowc(i), Ph.wr);
        }
        lds_layout(m, ldst, lowc(F - 1), P.st);
        out.passes.push_back(P);

        FPass Q = P;
        Q.phase_begin = int(out.rphases.size());
        auto rev_w = [&](int i) {
            const uint32_t half = kb == 5 ? (1u << out.phases[first + i].R[4]) : 0u;
            return (rmasks[i] & ~half) | (1u << column_bit(m, rmasks[i], 2));
        };
        lds_layout(m, lowc(F - 1), ldst, Q.ld);
        for (int i = F - 1; i >= 0; --i) {
            FPhase Ph = out.phases[first + i];
            const uint32_t vw_prev = (i == F - 1) ? ldst : rev_w(i + 1);
            lds_layout(m, lowc(i), vw_prev, Ph.rd);
            if (i > 0) lds_layout(m, lowc(i - 1), rev_w(i), Ph.wr);
            else lds_layout(m, ldst, rev_w(i), Ph.wr);
            out.rphases.push_back(Ph);
        }
        lds_layout(m, ldst, rev_w(0), Q.st);
        Q.phase_end = int(out.rphases.size());
        out.rpasses.push_back(Q);
    }

    // ---- layouts resolved at the column and block bits of every phase
    for (std::vector<FPhase>* v : {&out.phases, &out.rphases})
        for (FPhase& F : *v) {
            for (int k = 0; k < 9; ++k) {
                F.rdc[k] = F.C[k] >= 0 ? F.rd[F.C[k]] : 0;
                F.wrc[k] = F.C[k] >= 0 ? F.wr[F.C[k]] : 0;
            }
            for (int t = 0; t < FUSED_KMAX; ++t) {
                F.rdr[t] = t < F.k ? F.rd[F.R[t]] : 0;
                F.wrr[t] = t < F.k ? F.wr[F.R[t]] : 0;
            }
        }

    // ---- gradient assembly tables
    std::vector<std::vector<int32_t>> per_param(std::max(n_params, 0));
    for (const FPass& P : out.passes)
        for (int f = P.phase_begin; f < P.phase_end; ++f)
            for (int o = out.phases[f].op_begin; o < out.phases[f].op_end; ++o) {
                const Op& op = out.ops[o];
                if (op.slot < 0) continue;
                const int gslot = op.slot;
                const tcng_gate& g = gates[op.gate];
                if (g.kind == K_U2) {
                    out.gate_slot[op.gate] = gslot;
                } else {
                    if (g.p0 >= 0) per_param[g.p0].push_back(gslot);
                    if (kind_nparams(g.kind) == 2 && g.p1 >= 0) per_param[g.p1].push_back(gslot + 1);
                }
            }
    out.slot_ptr.assign(1, 0);
    for (auto& v : per_param) {
        std::sort(v.begin(), v.end());
        out.slot_idx.insert(out.slot_idx.end(), v.begin(), v.end());
        out.slot_ptr.push_back(int32_t(out.slot_idx.size()));
    }
    return "";
}

namespace {

// rank over GF(2) of the vectors v[0..k)
int gf2_rank(std::vector<uint32_t> v) {
    int r = 0;
    for (int bit = 31; bit >= 0; --bit) {
        int piv = -1;
        for (size_t i = r; i < v.size(); ++i)
            if ((v[i] >> bit) & 1) { piv = int(i); break; }
        if (piv < 0) continue;
        std::swap(v[r], v[piv]);
        for (size_t i = 0; i < v.size(); ++i)
            if (int(i) != r && ((v[i] >> bit) & 1)) v[i] ^= v[r];
        ++r;
    }
    return r;
}

// layout img over m bits: a bijection, and 32-lane accesses varying the bits
// of each pattern in `pats` spread over 32 distinct 8-byte bank pairs
bool layout_ok(const int32_t* img, int m, std::initializer_list<uint32_t> pats) {
    std::vector<uint32_t> all;
    for (int b = 0; b < m; ++b) {
        if (img[b] < 0 || img[b] >= (1 << m)) return false;
        all.push_back(uint32_t(img[b]));
    }
    if (gf2_rank(all) != m) return false;
    for (uint32_t p : pats) {
        std::vector<uint32_t> low;
        for (int b = 0; b < m; ++b)
            if ((p >> b) & 1) low.push_back(uint32_t(img[b]) & 31u);
        if (low.size() != 5 || gf2_rank(low) != 5) return false;
    }
    return true;
}

uint32_t phase_rmask(const FPhase& F) {
    uint32_t r = 0;
    for (int t = 0; t < F.k; ++t) r |= 1u << F.R[t];
    return r;
}

}  // namespace

int check_fused_layouts(const FusedPlan& P) {
    const int m = P.m;
    const uint32_t ldst = 0x3Eu;
    int bad = 0;
    for (const FPass& Q : P.passes) {
        const int F = Q.phase_end - Q.phase_begin;
        auto low = [&](int i) { return low_columns(m, phase_rmask(P.phases[Q.phase_begin + i])); };
        bad += !layout_ok(Q.ld, m, {ldst, low(0)});
        for (int i = 0; i < F; ++i) {
            const FPhase& Ph = P.phases[Q.phase_begin + i];
            bad += !layout_ok(Ph.rd, m, {low(i)});
            bad += !layout_ok(Ph.wr, m, {low(i), i + 1 < F ? low(i + 1) : ldst});
        }
        bad += !layout_ok(Q.st, m, {ldst, low(F - 1)});
    }
    for (const FPass& Q : P.rpasses) {
        const int F = Q.phase_end - Q.phase_begin;   // visiting order
        auto low = [&](int i) { return low_columns(m, phase_rmask(P.rphases[Q.phase_begin + i])); };
        auto wpat = [&](int i) {
            const FPhase& Ph = P.rphases[Q.phase_begin + i];
            const uint32_t half = Ph.k == 5 ? (1u << Ph.R[4]) : 0u;
            return (phase_rmask(Ph) & ~half) | (1u << Ph.C[2]);
        };
        bad += !layout_ok(Q.ld, m, {ldst, low(0)});
        for (int i = 0; i < F; ++i) {
            const FPhase& Ph = P.rphases[Q.phase_begin + i];
            bad += !layout_ok(Ph.rd, m, {low(i)});
            bad += !layout_ok(Ph.wr, m, {wpat(i), i + 1 < F ? low(i + 1) : ldst});
        }
        bad += !layout_ok(Q.st, m, {ldst, wpat(F - 1)});
    }
    return bad;
}

std::string plan_pauli(int n, const std::vector<PauliTermHost>& terms, const TileConfig& cfg, PauliPlan& out) {
    out = PauliPlan();
    out.cfg = cfg;
    const int m = std::min(n, cfg.m_max);
    const int lo = std::min(cfg.lo, m);
    const uint64_t lo_mask = (lo >= 64) ? ~uint64_t(0) : ((uint64_t(1) << lo) - 1);
    const uint64_t all_mask = (n >= 64) ? ~uint64_t(0) : ((uint64_t(1) << n) - 1);

    std::map<uint64_t, std::vector<int>> by_x;   // ordered: x = 0 (diagonal) first
    for (size_t t = 0; t < terms.size(); ++t) by_x[terms[t].x].push_back(int(t));
    std::vector<uint64_t> xs;
    for (auto& kv : by_x) {
        if (popc(kv.first & ~lo_mask) > m - lo) return "Pauli term flips more qubits than a tile holds";
        xs.push_back(kv.first);
    }
    std::vector<char> done(xs.size(), 0);
    size_t left = xs.size();
    while (left) {
        uint64_t T = (n <= m) ? all_mask : lo_mask;
        for (size_t i = 0; i < xs.size(); ++i)
            if (!done[i] && popc((T | xs[i]) & all_mask) <= m) T |= xs[i];
        T = fill_tile(T, n, m);
        PPass P{};
        P.m = m;
        P.lo = lo;
        P.tile_mask = T;
        int qubit_to_local[64];
        for (int q = 0; q < 64; ++q) qubit_to_local[q] = -1;
        for (int i = 0; i < 16; ++i) P.local_qubit[i] = -1;
        int li = 0;
        for (int q = 0; q < n; ++q)
            if ((T >> q) & 1) { qubit_to_local[q] = li; P.local_qubit[li] = q; ++li; }
        auto to_local = [&](uint64_t mask) {
            int32_t r = 0;
            for (int q = 0; q < n; ++q)
                if (((mask & T) >> q) & 1) r |= 1 << qubit_to_local[q];
            return r;
        };
        P.group_begin = int(out.groups.size());
        for (size_t i = 0; i < xs.size(); ++i) {
            if (done[i] || (xs[i] & ~T)) continue;
            done[i] = 1;
            --left;
            PGroup G{};
            G.x_local = to_local(xs[i]);
            G.class_begin = int(out.classes.size());
            for (auto& cls : coefficient_classes(terms, by_x[xs[i]])) {
                G.cbr += cls.first.first * double(cls.second.size());
                G.cbi += cls.first.second * double(cls.second.size());
                std::vector<int> zt;   // the terms with Z/Y bits: the others' parities are all even
                for (int t : cls.second)
                    if (terms[t].z) zt.push_back(t);
                for (size_t c0 = 0; c0 < zt.size(); c0 += PCLASS_MAX) {
                    PClass pc{};
                    pc.cre = cls.first.first;
                    pc.cim = cls.first.second;
                    pc.fre = float(pc.cre);
                    pc.fim = float(pc.cim);
                    pc.term_begin = int(out.terms.size());
                    const size_t c1 = std::min(zt.size(), c0 + PCLASS_MAX);
                    for (size_t j = c0; j < c1; ++j) {
                        const int t = zt[j];
                        PTerm pt{};
                        pt.z_local = to_local(terms[t].z);
                        pt.z_out = terms[t].z & ~T;
                        for (int e = 0; m >= PAULI_RB && e < (1 << PAULI_RB); ++e) {   // (below, no tiled pass runs)
                            const uint32_t l = (uint32_t(e) << (m - PAULI_RB)) ^ uint32_t(G.x_local);
                            pt.epar[e >> 2] |= uint32_t(popc(uint64_t(l & uint32_t(pt.z_local))) & 1) << (8 * (e & 3));
                        }
                        out.terms.push_back(pt);
                    }
                    pc.term_end = int(out.terms.size());
                    out.classes.push_back(pc);
                }
            }
            if (int(out.classes.size()) == G.class_begin) {   // no Z/Y bits at all: one class without terms
                PClass pc{};
                pc.term_begin = pc.term_end = int(out.terms.size());
                out.classes.push_back(pc);
                G.no_z = 1;
            }
            G.class_end = int(out.classes.size());
            G.fbr = float(G.cbr);
            G.fbi = float(G.cbi);
            out.groups.push_back(G);
        }
        P.group_end = int(out.groups.size());
        if (P.group_end == P.group_begin) return "internal: Pauli planner made no progress";
        out.passes.push_back(P);
    }
    return "";
}

void group_pauli_full(const std::vector<PauliTermHost>& terms, std::vector<PGroupFull>& groups,
                      std::vector<PClassFull>& classes, std::vector<PTermFull>& out_terms) {
    std::map<uint64_t, std::vector<int>> by_x;
    for (size_t t = 0; t < terms.size(); ++t) by_x[terms[t].x].push_back(int(t));
    groups.clear();
    classes.clear();
    out_terms.clear();
    for (auto& kv : by_x) {
        PGroupFull G{};
        G.x = kv.first;
        G.class_begin = int(classes.size());
        for (auto& cls : coefficient_classes(terms, kv.second)) {
            PClassFull pc{};
            pc.cre = cls.first.first;
            pc.cim = cls.first.second;
            pc.term_begin = int(out_terms.size());
            for (int t : cls.second) out_terms.push_back(PTermFull{terms[t].z});
            pc.term_end = int(out_terms.size());
            classes.push_back(pc);
        }
        G.class_end = int(classes.size());
        groups.push_back(G);
    }
}

}  // namespace tcng
