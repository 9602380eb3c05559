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

// Order PS of the super-cell expansions (0: the one-level expansion is used).
int super_order(const irs_plan_s *p);

// Parts of each cell expansion in p->d_part: 1 with the two-level field,
// else one per lens chunk.
int32_t level2_chunks(const irs_plan_s *p);

// Expansions of every cell of level-1 rows [c0, c1] into p->d_part: part k of
// Lt_n of cell (cx, cy) at
//   d_part[((((cy - c0) n1x + cx) nchunk + k) P + n) 2 + {0: Re, 1: Im}],
// nchunk = level2_chunks(p); the cell expansion is the sum of its parts in
// order.  Computes the super rows it needs that are not cached.  flops, if
// not null, receives the algorithmic flops of the launches.  Grows the
// buffers as needed.  Requires level2_order(p) > 0.
// fold_sheet: cells away from the rectangle's corners take the sheet's series
// into their expansion (the level-2 points then add only -kappa_* conj(z0))
irs_status launch_level2_expand(irs_plan_s *p, int64_t c0, int64_t c1, double *flops = nullptr,
                                bool fold_sheet = false);

// Forget the cached super rows (the next expansion recomputes them).
void level2_reset(irs_plan_s *p);

// Allocate the buffers a whole-map computation needs (before a capture).
irs_status level2_prepare(irs_plan_s *p);

}  // namespace irs
