// Host-side checks of the planner's output (no device code).
#include "plan_check.h"

#include <vector>

namespace tcng {
namespace {

int gf2_rank_of(std::vector<uint32_t> v) {
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

// the LDS slots of lanes 0..s-1's bits differ in their low s bits, s = 3, 4, 5
bool banks_spread(const uint32_t* slot) {
    for (int s = 3; s <= 5; ++s) {
        std::vector<uint32_t> low;
        for (int j = 0; j < s; ++j) low.push_back(slot[j] & ((1u << s) - 1u));
        if (gf2_rank_of(low) != s) return false;
    }
    return true;
}

}  // namespace

int check_rounds_layouts(const CircuitPlan& P) {
    int bad = 0;
    for (int dir = 0; dir < 2; ++dir) {
        const std::vector<QPass>& QP = dir ? P.qrpasses : P.qpasses;
        const std::vector<QPhase>& PH = dir ? P.qrphases : P.qphases;
        for (size_t p = 0; p < QP.size() && p < P.passes.size(); ++p) {
            const int m = P.passes[p].m;
            const uint32_t dim = 1u << m;
            for (int f = QP[p].phase_begin; f < QP[p].phase_end; ++f) {
                const QPhase& F = PH[size_t(f)];
                bool ok = true;
                for (int which = 0; which < 2 && ok; ++which) {   // both image sets: bijections of the tile
                    const int32_t* img = which ? F.cimg : F.uimg;
                    std::vector<uint32_t> v;
                    for (int b = 0; b < m; ++b) {
                        if (uint32_t(img[b]) >= dim) ok = false;
                        v.push_back(uint32_t(img[b]));
                    }
                    if (gf2_rank_of(v) != m) ok = false;
                }
                for (int i = 0; i < QREG && ok; ++i)
                    if (F.R[i] >= 0 && (F.rimg[i] != F.cimg[F.R[i]] || F.ruimg[i] != F.uimg[F.R[i]])) ok = false;
                if (f == QP[p].phase_begin)   // the pass starts from the tile load's layout
                    for (int b = 0; b < m && ok; ++b)
                        if (uint32_t(F.uimg[b]) != tile_swz(1u << b)) ok = false;
                if (f > QP[p].phase_begin && ok) {   // an inner boundary
                    const QPhase& E = PH[size_t(f) - 1];
                    uint32_t rd[5], wr[5];
                    int kr = 0, kw = 0;
                    for (int b = 0; b < m && kr < 5; ++b)
                        if (!((F.rmask >> b) & 1)) rd[kr++] = uint32_t(F.uimg[b]);
                    for (int b = 0; b < m && kw < 5; ++b)
                        if (!((E.rmask >> b) & 1)) wr[kw++] = uint32_t(E.cimg[b]);
                    if (kr < 5 || kw < 5 || !banks_spread(rd) || !banks_spread(wr)) ok = false;
                }
                bad += !ok;
            }
        }
    }
    return bad;
}

}  // namespace tcng
