// External-coordinate Monte Carlo moves (moves.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace bpmf {

// Philox purpose of the external moves' draws
enum : uint32_t { kExternal = 6 };

// n_moves moves in a row for the replica in each state k < k_max of every
// ligand ligs[0..n_lig) that needs `waves` wavefronts (the others, and the
// replicas in other states, are untouched); k_grid = the largest
// min(k_max, K) of those ligands; each ligand's ext_acc / ext_try count
// the attempted and accepted moves per state
hipError_t launch_external_moves(const GridDev& g, const LigDev* ligs,
                                 int n_lig, int k_grid, int waves, int n_moves,
                                 int k_max, float sigma, uint64_t seed,
                                 hipStream_t st);

}  // namespace bpmf
