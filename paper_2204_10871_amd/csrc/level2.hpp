// Level-2 pieces shared by the grid interpolation (k_interp.hip) and the
// learned interpolant (k_learn.hip): the per-cell local expansion of the
// distant lenses.
#pragma once

#include "plan.hpp"

namespace irs {

constexpr int kRing = 3;              // the expansion leaves out the (2R+1)^2 block
constexpr int kChunkLens = 65536;     // lenses per partial expansion

// Expansion order P of the plan (0: the paper's per-point sums, no expansion).
int level2_order(const irs_plan_s *p);

// Lens chunks of the plan's partial expansions.
inline int32_t level2_chunks(const irs_plan_s *p)
{
    return p->n_lens > 0 ? (int32_t)((p->n_lens + kChunkLens - 1) / kChunkLens) : 1;
}

// Partial expansions of every cell of level-1 rows [c0, c1] into p->d_part:
// Lt_n of chunk k of cell (cx, cy) at
//   d_part[((((cy - c0) n1x + cx) nchunk + k) P + n) 2 + {0: Re, 1: Im}].
// Grows p->d_part as needed.  Requires level2_order(p) > 0.
irs_status launch_level2_expand(irs_plan_s *p, int64_t c0, int64_t c1);

}  // namespace irs
