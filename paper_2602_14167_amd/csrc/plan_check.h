// Host-side checks of the planner's output (no device code).
#pragma once

#include "plan.h"

namespace tcng {

// number of round phases of a tiled plan whose LDS images are not bijections
// of the tile, whose pass does not start from the tile load's swizzle, or that
// put two of 8, 16 or 32 consecutive lanes on one bank at an inner phase
// boundary (the phase's reading lanes, or the writing lanes of the phase
// before it through its CNOT permutation)
int check_rounds_layouts(const CircuitPlan& P);

}  // namespace tcng
