// Whole-solve kernel of the coarse strip levels: one work-group per sample,
// PCG state on chip (host-side launchers and fit test).
#pragma once

#include <cstddef>

#include "common.hpp"

namespace mlmc {

// most nodes one thread owns (the 128x32 mesh with 512 threads needs 9)
constexpr int SMALL_MAXN = 9;

int small_threads(const StripGeom &g);
size_t small_lds_bytes(const StripGeom &g);
int small_nodes_per_thread(const StripGeom &g);
// whether the level's PCG state fits one work-group with `lds_per_block` bytes of LDS
bool small_fits(const StripGeom &g, size_t lds_per_block);
// set-up + PCG to completion for slots 0..n-1 of S (angles in S.theta, FP64);
// writes S.x, S.it_b, S.relres, S.status
void launch_small_solve(const StripGeom &g, const StripMat &m, const PcgSlots &S, int n, hipStream_t st);

}  // namespace mlmc
