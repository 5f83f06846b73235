// Intramolecular nonbonded and implicit-solvent terms of a ligand
// (pairs.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bpmf {

constexpr int kPairMaxAtoms = 128;
constexpr int kPairWords = kPairMaxAtoms / 32;  // mask words per atom

// LDS bytes of a ligand's staged pair parameters and per-evaluation pair
// scratch (eval_block): p0 (16 n), p1 (8 n), the excluded and 1-4 masks
// (2 x 16 n), Born radii and their chain-rule factors (2 x 4 n), and 16
// bytes for the alignment of their start
__host__ __device__ inline int pair_lds_bytes(int n) { return 64 * n + 16; }

constexpr float kObcA = 1.0f, kObcB = 0.8f, kObcC = 4.85f;

// descreening integral H(r; a, s) of a ball of radius s at distance r
// outside radius a (Hawkins, Cramer, Truhlar), and dH/dr
__device__ __forceinline__ void hct(float r, float a, float s, float& H,
                                   float& dH) {
  if (a >= r + s) {
    H = 0.f;
    dH = 0.f;
    return;
  }
  const float u = 1.f / (r + s), du = -u * u;
  const float rs = r - s;
  float l, dl;
  if (a > fabsf(rs)) {
    l = 1.f / a;
    dl = 0.f;
  } else {
    l = 1.f / fabsf(rs);
    dl = rs > 0.f ? -l * l : l * l;
  }
  const float ir = 1.f / r;
  const float s2r2 = s * s - r * r;
  const float l2u2 = l * l - u * u;
  const float lg = logf(u / l);
  H = 0.5f * (l - u) + 0.125f * s2r2 * l2u2 * ir + 0.25f * lg * ir;
  dH = 0.5f * (dl - du) + (-0.25f - 0.125f * s2r2 * ir * ir) * l2u2 +
       0.25f * s2r2 * (l * dl - u * du) * ir +
       0.25f * (du / u - dl / l) * ir - 0.25f * lg * ir * ir;
  if (a < s - r) {  // atom i inside the ball: the shells a .. s - r whole
    H += 1.f / a - l;
    dH -= dl;
  }
}

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
