// Intramolecular nonbonded and implicit-solvent energy and forces of the
// ligand (Thermodynamic Cycle: the ligand force field with an OBC
// generalised-Born/surface-area solvent).
//   LJ 12-6 and Coulomb over pairs more than two bonds apart (Lorentz-
//   Berthelot; 1-4 pairs scaled), generalised Born over all ordered pairs
//   with f = sqrt(r^2 + R_i R_j exp(-r^2 / 4 R_i R_j)), Born radii from the
//   Hawkins-Cramer-Truhlar descreening integral through the OBC II
//   rescaling (Onufriev, Bashford, Case 2004), and the ACE surface term
//   4 pi gamma (rho + probe)^2 (rho / R)^6.
// One workgroup per configuration, one thread per atom: each thread sums
// its own row of pair terms (every pair is visited from both ends), so the
// forces need no atomics and the result does not depend on scheduling.
// Three passes: (1) LJ, Coulomb and the descreening sum I_i; (2) the Born
// radii known, the GB energy, its explicit force and dE/dR_i; (3) the chain
// rule through dR_i/dI_i and dI/dr.
#include <hip/hip_runtime.h>
#include <math.h>

#include "pairs.h"

namespace bpmf {

namespace {

template <int W, bool FORCES>
__global__ __launch_bounds__(W * 64) void k_pair_terms(
    PairDev P, const float* __restrict__ xs, double* __restrict__ terms,
    float* __restrict__ forces) {
  __shared__ float4 s_x[kPairMaxAtoms], s_p0[kPairMaxAtoms];
  __shared__ float2 s_p1[kPairMaxAtoms];
  __shared__ uint32_t s_ex[kPairMaxAtoms * kPairWords];
  __shared__ uint32_t s_14[kPairMaxAtoms * kPairWords];
  __shared__ float s_R[kPairMaxAtoms], s_b[kPairMaxAtoms];
  __shared__ double s_red[4 * W];
  const int n = P.n;
  const int tid = threadIdx.x;
  const int64_t c = blockIdx.x;
  const bool own = tid < n;
  const float* xc = xs + c * n * 3;
  for (int i = tid; i < n; i += W * 64) {
    s_x[i] = make_float4(xc[3 * i], xc[3 * i + 1], xc[3 * i + 2], 0.f);
    s_p0[i] = P.p0[i];
    s_p1[i] = P.p1[i];
  }
  for (int i = tid; i < n * kPairWords; i += W * 64) {
    s_ex[i] = P.excl[i];
    s_14[i] = P.o14[i];
  }
  __syncthreads();

  float e_lj = 0.f, e_c = 0.f, e_gb = 0.f, e_sa = 0.f;
  float fx = 0.f, fy = 0.f, fz = 0.f;
  float I = 0.f, dRdI = 0.f, Ri = 0.f;
  float4 xi = make_float4(0.f, 0.f, 0.f, 0.f), pi = xi;
  float2 qi1 = make_float2(0.f, 0.f);
  // pass 1: LJ, Coulomb, descreening
  if (own) {
    xi = s_x[tid];
    pi = s_p0[tid];
    qi1 = s_p1[tid];
    for (int j = 0; j < n; ++j) {
      if (j == tid) continue;
      const float4 xj = s_x[j], pj = s_p0[j];
      const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
      const float r2 = dx * dx + dy * dy + dz * dz;
      const float ir = __builtin_amdgcn_rsqf(r2), r = r2 * ir;
      float H, dH;
      hct(r, ir, qi1.x, s_p1[j].y, H, dH);
      I += H;
      const int w = tid * kPairWords + (j >> 5);
      const uint32_t bit = 1u << (j & 31);
      if (s_ex[w] & bit) continue;
      const float sg = 0.5f * (pi.y + pj.y), ep = pi.z * pj.z;
      const float ir2 = ir * ir;
      const float sr2 = sg * sg * ir2, sr6 = sr2 * sr2 * sr2;
      float lj = 4.f * ep * (sr6 * sr6 - sr6);
      float flj = 24.f * ep * (2.f * sr6 * sr6 - sr6) * ir2;
      float cl = P.kc * pi.x * pj.x * ir;
      float fcl = cl * ir2;
      if (s_14[w] & bit) {
        lj *= P.lj14;
        flj *= P.lj14;
        cl *= P.el14;
        fcl *= P.el14;
      }
      e_lj += 0.5f * lj;
      e_c += 0.5f * cl;
      if (FORCES) {
        const float f = flj + fcl;
        fx += f * dx;
        fy += f * dy;
        fz += f * dz;
      }
    }
    // OBC II Born radius
    const float psi = I * qi1.x;
    const float t = psi * (kObcA - psi * (kObcB - kObcC * psi));
    const float th = tanhf(t);
    Ri = 1.f / (1.f / qi1.x - th / pi.w);
    dRdI = Ri * Ri * (1.f - th * th) *
           (kObcA - psi * (2.f * kObcB - 3.f * kObcC * psi)) * qi1.x / pi.w;
    s_R[tid] = Ri;
  }
  __syncthreads();
  // pass 2: GB energy, explicit GB force, dE/dR_i; surface term
  if (own) {
    const float qi = pi.x;
    e_gb = 0.5f * P.kgb * qi * qi / Ri;
    float dEdR = -0.5f * P.kgb * qi * qi / (Ri * Ri);
    for (int j = 0; j < n; ++j) {
      if (j == tid) continue;
      const float4 xj = s_x[j];
      const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
      const float r2 = dx * dx + dy * dy + dz * dz;
      const float Rj = s_R[j];
      const float RR = Ri * Rj;
      const float iRR = __builtin_amdgcn_rcpf(RR);
      const float D = __expf(-0.25f * r2 * iRR);
      const float f2 = r2 + RR * D;
      const float invf = rsqrtf(f2);
      const float invf3 = invf * invf * invf;
      const float kq = P.kgb * qi * s_p0[j].x;
      e_gb += 0.5f * kq * invf;
      if (FORCES) {
        const float g = kq * (1.f - 0.25f * D) * invf3;
        fx += g * dx;
        fy += g * dy;
        fz += g * dz;
        dEdR -= 0.5f * kq * Rj * D * (1.f + 0.25f * r2 * iRR) * invf3;
      }
    }
    const float rp = pi.w + P.probe;
    const float q6 = pi.w / Ri, q3 = q6 * q6 * q6;
    e_sa = P.sa * rp * rp * q3 * q3;
    dEdR -= 6.f * e_sa / Ri;
    s_b[tid] = dEdR * dRdI;
  }
  __syncthreads();
  // pass 3: chain rule through the Born radii
  if (FORCES && own) {
    const float bi = s_b[tid];
    for (int j = 0; j < n; ++j) {
      if (j == tid) continue;
      const float4 xj = s_x[j];
      const float2 pj1 = s_p1[j];
      const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
      const float r2 = dx * dx + dy * dy + dz * dz;
      const float ir = __builtin_amdgcn_rsqf(r2), r = r2 * ir;
      float Hi, dHi, Hj, dHj;
      hct(r, ir, qi1.x, pj1.y, Hi, dHi);
      hct(r, ir, pj1.x, qi1.y, Hj, dHj);
      const float g = -(bi * dHi + s_b[j] * dHj) * ir;
      fx += g * dx;
      fy += g * dy;
      fz += g * dz;
    }
  }
  if (FORCES && own) {
    float* fo = forces + (c * n + tid) * 3;
    fo[0] = fx;
    fo[1] = fy;
    fo[2] = fz;
  }
  // energies: per-wave double sums, then the waves in order
  double v[4] = {(double)e_lj, (double)e_c, (double)e_gb, (double)e_sa};
#pragma unroll
  for (int q = 0; q < 4; ++q)
    for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off);
  if ((tid & 63) == 0)
    for (int q = 0; q < 4; ++q) s_red[4 * (tid >> 6) + q] = v[q];
  __syncthreads();
  if (tid < 4) {
    double s = 0.0;
    for (int w = 0; w < W; ++w) s += s_red[4 * w + tid];
    terms[c * 4 + tid] = s;
  }
}

}  // namespace

hipError_t launch_pair_terms(const PairDev& P, const float* x, int64_t N,
                             double* terms, float* forces, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  if (P.n < 1 || P.n > kPairMaxAtoms || N > 0x7fffffffll)
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)N);
  if (P.n <= 64) {
    if (forces)
      hipLaunchKernelGGL((k_pair_terms<1, true>), grid, dim3(64), 0, st, P, x,
                         terms, forces);
    else
      hipLaunchKernelGGL((k_pair_terms<1, false>), grid, dim3(64), 0, st, P,
                         x, terms, forces);
  } else {
    if (forces)
      hipLaunchKernelGGL((k_pair_terms<2, true>), grid, dim3(128), 0, st, P,
                         x, terms, forces);
    else
      hipLaunchKernelGGL((k_pair_terms<2, false>), grid, dim3(128), 0, st, P,
                         x, terms, forces);
  }
  return hipGetLastError();
}

}  // namespace bpmf
