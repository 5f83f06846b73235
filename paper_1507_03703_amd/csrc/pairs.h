// Intramolecular nonbonded and implicit-solvent terms of a ligand
// (pairs.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bpmf {

constexpr int kPairMaxAtoms = 128;
constexpr int kPairWords = kPairMaxAtoms / 32;  // mask words per atom

struct PairDev {
  int n;
  const float4* p0;       // n: q, sigma, sqrt(eps), rho
  const float2* p1;       // n: rt = rho - 0.09, S * rt
  const uint32_t* excl;   // n x kPairWords: bit j of row i = pair excluded
  const uint32_t* o14;    // n x kPairWords: bit j of row i = 1-4 pair
  float lj14, el14;
  float kc;    // k_e / eps_solute
  float kgb;   // -k_e (1/eps_solute - 1/eps_solvent)
  float sa;    // 4 pi gamma
  float probe;
};

// terms: N x 4 doubles (LJ, Coulomb, GB, SA); forces: N x n x 3 or null
hipError_t launch_pair_terms(const PairDev& P, const float* x, int64_t N,
                             double* terms, float* forces, hipStream_t st);

}  // namespace bpmf
