// External-coordinate Monte Carlo moves (moves.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace bpmf {

// Philox purpose of the external moves' draws
enum : uint32_t { kExternal = 6 };

// n_moves moves in a row for every replica of the ligand whose state is
// below k_max (replicas in other states are untouched); acc / tries: K
// per-state counters, incremented per attempted and accepted move
hipError_t launch_external_move(const GridDev& g, const LigDev* lig, int K,
                                int waves, int n_moves, int k_max,
                                float sigma, unsigned long long* acc,
                                unsigned long long* tries, int lds,
                                uint64_t seed, hipStream_t st);

}  // namespace bpmf
