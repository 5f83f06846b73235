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
// plus, for a block of `waves` wavefronts, the per-slice partial sums of
// the three passes (pair_stage): S = waves / ceil(n / 64) slices of the
// partner range, 9 floats per slice and atom
__host__ __device__ inline int pair_slices(int n, int waves) {
  const int a = (n + 63) / 64;
  return waves / a > 0 ? waves / a : 1;
}
__host__ __device__ inline int pair_lds_bytes(int n, int waves) {
  return 64 * n + 16 + 36 * n * pair_slices(n, waves);
}

constexpr float kObcA = 1.0f, kObcB = 0.8f, kObcC = 4.85f;

// descreening integral H(r; a, s) of a ball of radius s at distance r
// outside radius a (Hawkins, Cramer, Truhlar), and dH/dr; ir = 1/r.  The
// reciprocals and the logarithm are the hardware's (1 ulp); du/u = -u and
// dl/l = -+l are used as such.
__device__ __forceinline__ void hct(float r, float ir, float a, float s,
                                   float& H, float& dH) {
  if (a >= r + s) {
    H = 0.f;
    dH = 0.f;
    return;
  }
  const float u = __builtin_amdgcn_rcpf(r + s), du = -u * u;
  const float rs = r - s;
  float l, dl, dll, x;  // dll = dl / l; x = 1 / l
  if (a > fabsf(rs)) {
    x = a;
    l = __builtin_amdgcn_rcpf(a);
    dl = 0.f;
    dll = 0.f;
  } else {
    x = fabsf(rs);
    l = __builtin_amdgcn_rcpf(x);
    dl = rs > 0.f ? -l * l : l * l;
    dll = rs > 0.f ? -l : l;
  }
  const float s2r2 = s * s - r * r;
  const float l2u2 = l * l - u * u;
  const float lg = __logf(u * x);
  H = 0.5f * (l - u) + 0.125f * s2r2 * l2u2 * ir + 0.25f * lg * ir;
  dH = 0.5f * (dl - du) + (-0.25f - 0.125f * s2r2 * ir * ir) * l2u2 +
       0.25f * s2r2 * (l * dl - u * du) * ir +
       0.25f * (-u - dll) * ir - 0.25f * lg * ir * ir;
  if (a < s - r) {  // atom i inside the ball: the shells a .. s - r whole
    H += __builtin_amdgcn_rcpf(a) - l;
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
