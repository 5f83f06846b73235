// Device-side building blocks of the BPMF hot path for gfx950 (wave64).
//
// The energy of ligand configuration x in state k (Methodology,
// "Thermodynamic Cycle"):
//   U_k(x) = U_bond + U_angle + U_tors + U_I + sum_c w_kc Psi_c(x)
//   Psi_c(x) = sum_i s_ic v_c(x_i)      (v_c^4 on a quartic-root channel)
// with v_c the trilinear interpolant of grid channel c, clamped to the edge
// outside the grid.  One wavefront evaluates one configuration: lane l owns
// atoms l, l+64, ... (APL atoms per lane); bonded terms are spread over the
// lanes term by term and their per-atom forces meet in LDS "force slots"
// that each atom then sums in a fixed order, so no floating-point atomics
// are used and results are bitwise reproducible.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace bpmf {

// ----------------------------------------------------------------------------
// wave-level helpers
// ----------------------------------------------------------------------------

// Orders this lane's LDS accesses against those of the other lanes of the
// same wavefront.  The hardware executes one wave's LDS instructions in
// order, so only the compiler must be kept from moving them; the
// wavefront-scope fences emit no wait instructions.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Butterfly all-reduce: every lane ends with the same, order-fixed sum.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}
__device__ __forceinline__ float wave_sumf(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, kWave);
  return v;
}

// ----------------------------------------------------------------------------
// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)
// ----------------------------------------------------------------------------
struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1,
                                            uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

__device__ __forceinline__ U4 draw(uint64_t seed, uint32_t index, int lig,
                                   int rep, uint64_t sweep, uint32_t purpose) {
  return philox4x32_10(index, ((uint32_t)lig << 16) | (uint32_t)rep,
                       (uint32_t)sweep, purpose, (uint32_t)seed,
                       (uint32_t)(seed >> 32));
}

// uniform in (0, 1]: (u32 + 1) 2^-32
__device__ __forceinline__ double u01d(uint32_t v) {
  return ((double)v + 1.0) * 2.3283064365386962890625e-10;
}
__device__ __forceinline__ float u01f(uint32_t v) {
  return (float)((double)v + 1.0) * 2.3283064365386962890625e-10f;
}

// three standard normals (Box-Muller on (x,y) and (z,w))
__device__ __forceinline__ void normals3(const U4& o, float& a, float& b,
                                         float& c) {
  const float r1 = sqrtf(-2.0f * logf(u01f(o.x)));
  float s1, c1;
  sincospif(2.0f * u01f(o.y), &s1, &c1);
  const float r2 = sqrtf(-2.0f * logf(u01f(o.z)));
  float s2, c2;
  sincospif(2.0f * u01f(o.w), &s2, &c2);
  a = r1 * c1;
  b = r1 * s1;
  c = r2 * c2;
}

// ----------------------------------------------------------------------------
// trilinear interpolation of all C channels at one point
// ----------------------------------------------------------------------------
struct AxisPos {
  int i;       // cell index, 0..n-2
  float t;     // fraction in [0,1] (NaN propagates)
  float live;  // 1 inside [0, n-1], 0 outside (gradient clamped)
};

__device__ __forceinline__ AxisPos grid_axis(float x, float o, float inv_h,
                                             int n) {
  const float u = (x - o) * inv_h;
  // comparisons are false for NaN, which therefore propagates through t
  const float uc = u < -1.0f ? -1.0f : (u > (float)n ? (float)n : u);
  int i = (int)floorf(uc);
  i = i < 0 ? 0 : (i > n - 2 ? n - 2 : i);
  float t = uc - (float)i;
  t = t < 0.0f ? 0.0f : (t > 1.0f ? 1.0f : t);
  AxisPos a;
  a.i = i;
  a.t = t;
  a.live = (u >= 0.0f && u <= (float)(n - 1)) ? 1.0f : 0.0f;
  return a;
}

// Raw corner values of the cell containing p: g[corner][c], corner bits
// (x, y<<1, z<<2).  Issued as independent loads so that callers can overlap
// their latency with other work before consuming them.
template <int C>
struct Corners {
  float v[8][C];
  AxisPos ax, ay, az;
};

template <int C>
__device__ __forceinline__ void grid_fetch(const GridDev& g, float px,
                                           float py, float pz,
                                           Corners<C>& k) {
  k.ax = grid_axis(px, g.ox, g.inv_h, g.nx);
  k.ay = grid_axis(py, g.oy, g.inv_h, g.ny);
  k.az = grid_axis(pz, g.oz, g.inv_h, g.nz);
  const size_t sx = C, sy = (size_t)g.nx * C, sz = (size_t)g.nx * g.ny * C;
  const float* base = g.nodes + (size_t)k.az.i * sz + (size_t)k.ay.i * sy +
                      (size_t)k.ax.i * sx;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const float* p = base + ((q & 1) ? sx : 0) + ((q & 2) ? sy : 0) +
                     ((q & 4) ? sz : 0);
#pragma unroll
    for (int c = 0; c < C; ++c) k.v[q][c] = __ldg(p + c);
  }
}

// value e_c = s_c * v_c (or s_c * v_c^4) and gradient de_c of every channel
template <int C, bool GRAD>
__device__ __forceinline__ void grid_finish(const GridDev& g,
                                            const Corners<C>& k,
                                            const float* s, float* e,
                                            float (*de)[3]) {
  const float tx = k.ax.t, ty = k.ay.t, tz = k.az.t;
  const float ux = 1.0f - tx, uy = 1.0f - ty, uz = 1.0f - tz;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    // (1-t) a + t b along x, y, z: exact at both ends of every edge, so
    // node values are reproduced exactly
    const float a00 = fmaf(tx, k.v[1][c], ux * k.v[0][c]);
    const float a10 = fmaf(tx, k.v[3][c], ux * k.v[2][c]);
    const float a01 = fmaf(tx, k.v[5][c], ux * k.v[4][c]);
    const float a11 = fmaf(tx, k.v[7][c], ux * k.v[6][c]);
    const float b0 = fmaf(ty, a10, uy * a00);
    const float b1 = fmaf(ty, a11, uy * a01);
    const float v = fmaf(tz, b1, uz * b0);
    float gx = 0.f, gy = 0.f, gz = 0.f;
    if (GRAD) {
      const float d00 = k.v[1][c] - k.v[0][c], d10 = k.v[3][c] - k.v[2][c];
      const float d01 = k.v[5][c] - k.v[4][c], d11 = k.v[7][c] - k.v[6][c];
      const float dx0 = fmaf(ty, d10 - d00, d00);
      const float dx1 = fmaf(ty, d11 - d01, d01);
      const float dy0 = a10 - a00, dy1 = a11 - a01;
      gx = fmaf(tz, dx1 - dx0, dx0) * (k.ax.live * g.inv_h);
      gy = fmaf(tz, dy1 - dy0, dy0) * (k.ay.live * g.inv_h);
      gz = (b1 - b0) * (k.az.live * g.inv_h);
    }
    if ((g.quartic_mask >> c) & 1) {
      const float v2 = v * v;
      e[c] = s[c] * (v2 * v2);
      if (GRAD) {
        const float q = 4.0f * s[c] * v2 * v;
        de[c][0] = q * gx;
        de[c][1] = q * gy;
        de[c][2] = q * gz;
      }
    } else {
      e[c] = s[c] * v;
      if (GRAD) {
        de[c][0] = s[c] * gx;
        de[c][1] = s[c] * gy;
        de[c][2] = s[c] * gz;
      }
    }
  }
}

// ----------------------------------------------------------------------------
// bonded terms (GAFF forms), one term per call; forces into LDS slots
// ----------------------------------------------------------------------------
__device__ __forceinline__ float3 f3(const float4& a) {
  return make_float3(a.x, a.y, a.z);
}
__device__ __forceinline__ float3 sub(float3 a, float3 b) {
  return make_float3(a.x - b.x, a.y - b.y, a.z - b.z);
}
__device__ __forceinline__ float dot(float3 a, float3 b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
__device__ __forceinline__ float3 cross(float3 a, float3 b) {
  return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z,
                     a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float3 scale3(float s, float3 a) {
  return make_float3(s * a.x, s * a.y, s * a.z);
}

struct Slots {
  float* x;
  float* y;
  float* z;
  __device__ __forceinline__ void put(int i, float3 f) const {
    x[i] = f.x;
    y[i] = f.y;
    z[i] = f.z;
  }
};

// K (r - r0)^2
template <bool FORCES>
__device__ __forceinline__ float bond_term(const float4* pos, int2 ij,
                                           float2 par, const Slots& sl,
                                           int slot) {
  const float3 d = sub(f3(pos[ij.x]), f3(pos[ij.y]));
  const float r = sqrtf(dot(d, d));
  const float dr = r - par.y;
  if (FORCES) {
    const float f = -2.0f * par.x * dr / r;
    sl.put(slot, scale3(f, d));
    sl.put(slot + 1, scale3(-f, d));
  }
  return par.x * dr * dr;
}

// K (theta - theta0)^2, theta = atan2(|a x b|, a.b), a = xi-xj, b = xk-xj
template <bool FORCES>
__device__ __forceinline__ float angle_term(const float4* pos, int4 ijk,
                                            float2 par, const Slots& sl,
                                            int slot) {
  const float3 xj = f3(pos[ijk.y]);
  const float3 a = sub(f3(pos[ijk.x]), xj);
  const float3 b = sub(f3(pos[ijk.z]), xj);
  const float3 c = cross(a, b);
  const float s = sqrtf(dot(c, c)), co = dot(a, b);
  const float th = atan2f(s, co);
  const float dth = th - par.y;
  if (FORCES) {
    const float la = sqrtf(dot(a, a)), lb = sqrtf(dot(b, b));
    const float dE = 2.0f * par.x * dth;
    const float ila = 1.0f / la, ilb = 1.0f / lb;
    const float cth = co * ila * ilb, isth = la * lb / s;
    const float3 ah = scale3(ila, a), bh = scale3(ilb, b);
    // d theta / d xi = (cos a^ - b^) / (|a| sin), d theta / d xk likewise
    const float ci = dE * isth * ila, ck = dE * isth * ilb;
    const float3 fi = make_float3(-ci * (cth * ah.x - bh.x),
                                  -ci * (cth * ah.y - bh.y),
                                  -ci * (cth * ah.z - bh.z));
    const float3 fk = make_float3(-ck * (cth * bh.x - ah.x),
                                  -ck * (cth * bh.y - ah.y),
                                  -ck * (cth * bh.z - ah.z));
    sl.put(slot, fi);
    sl.put(slot + 1, make_float3(-(fi.x + fk.x), -(fi.y + fk.y),
                                 -(fi.z + fk.z)));
    sl.put(slot + 2, fk);
  }
  return par.x * dth * dth;
}

// (V/2)(1 + cos(n phi - gamma)), IUPAC phi; forces in the singularity-free
// form of Blondel & Karplus (J. Comput. Chem. 17, 1132, 1996)
template <bool FORCES>
__device__ __forceinline__ float torsion_term(const float4* pos, int4 ijkl,
                                              float4 par, const Slots& sl,
                                              int slot) {
  const float3 xi = f3(pos[ijkl.x]), xj = f3(pos[ijkl.y]);
  const float3 xk = f3(pos[ijkl.z]), xl = f3(pos[ijkl.w]);
  const float3 b1 = sub(xj, xi), b2 = sub(xk, xj), b3 = sub(xl, xk);
  const float3 n1 = cross(b1, b2), n2 = cross(b2, b3);
  const float lb2 = sqrtf(dot(b2, b2));
  const float phi = atan2f(lb2 * dot(b1, n2), dot(n1, n2));
  float sn, cs;
  sincosf(par.y * phi - par.z, &sn, &cs);
  if (FORCES) {
    const float dE = -par.x * par.y * sn;
    const float in1 = 1.0f / dot(n1, n1), in2 = 1.0f / dot(n2, n2);
    const float ilb2 = 1.0f / lb2;
    const float p12 = dot(b1, b2) * ilb2 * in1;
    const float p23 = dot(b2, b3) * ilb2 * in2;
    const float3 gi = scale3(-lb2 * in1, n1);
    const float3 gl = scale3(lb2 * in2, n2);
    const float3 gj = make_float3(-gi.x + p12 * n1.x + p23 * n2.x,
                                  -gi.y + p12 * n1.y + p23 * n2.y,
                                  -gi.z + p12 * n1.z + p23 * n2.z);
    const float3 gk = make_float3(-gl.x - p12 * n1.x - p23 * n2.x,
                                  -gl.y - p12 * n1.y - p23 * n2.y,
                                  -gl.z - p12 * n1.z - p23 * n2.z);
    sl.put(slot, scale3(-dE, gi));
    sl.put(slot + 1, scale3(-dE, gj));
    sl.put(slot + 2, scale3(-dE, gk));
    sl.put(slot + 3, scale3(-dE, gl));
  }
  return par.x * (1.0f + cs);
}

// ----------------------------------------------------------------------------
// one full evaluation of a configuration by one wavefront
// ----------------------------------------------------------------------------
// terms (ENERGY): [U_bond, U_angle, U_tors, U_I, Psi_0..Psi_{C-1}], identical
// on every lane.  f (FORCES): -grad(U_bonded + U_I + sum_c w_c Psi_c) for the
// lane's atoms.  spos: n float4; slots: 3 x n_slots floats.
template <int C, int APL, bool FORCES, bool ENERGY>
__device__ __forceinline__ void eval_conf(const GridDev& g, const LigDev& L,
                                          const float* w,
                                          const float (&x)[APL][3],
                                          const float (&m)[APL],
                                          float (&f)[APL][3],
                                          double (&terms)[4 + C],
                                          float4* spos, const Slots& sl,
                                          int lane) {
  const int n = L.n;
  // publish positions for the bonded pass
#pragma unroll
  for (int a = 0; a < APL; ++a) {
    const int atom = lane + kWave * a;
    if (atom < n) spos[atom] = make_float4(x[a][0], x[a][1], x[a][2], 0.f);
  }
  // issue the grid gathers first; their latency overlaps the bonded pass
  Corners<C> cn[APL];
#pragma unroll
  for (int a = 0; a < APL; ++a) {
    const int atom = lane + kWave * a;
    const int src = atom < n ? a : 0;
    grid_fetch<C>(g, x[src][0], x[src][1], x[src][2], cn[a]);
  }
  wave_lds_sync();

  float eb = 0.f, ea = 0.f, et = 0.f;
  for (int t = lane; t < L.nb; t += kWave)
    eb += bond_term<FORCES>(spos, L.bij[t], L.bpar[t], sl, 2 * t);
  const int sa = 2 * L.nb;
  for (int t = lane; t < L.na; t += kWave)
    ea += angle_term<FORCES>(spos, L.aijk[t], L.apar[t], sl, sa + 3 * t);
  const int st = sa + 3 * L.na;
  for (int t = lane; t < L.nt; t += kWave)
    et += torsion_term<FORCES>(spos, L.tijkl[t], L.tpar[t], sl, st + 4 * t);
  if (FORCES) wave_lds_sync();

  // centre of mass and restraint (Eq. binding_site)
  float cx = 0.f, cy = 0.f, cz = 0.f;
#pragma unroll
  for (int a = 0; a < APL; ++a) {
    cx += m[a] * x[a][0];
    cy += m[a] * x[a][1];
    cz += m[a] * x[a][2];
  }
  cx = wave_sumf(cx) * L.inv_total_mass - L.site[0];
  cy = wave_sumf(cy) * L.inv_total_mass - L.site[1];
  cz = wave_sumf(cz) * L.inv_total_mass - L.site[2];
  const float d = sqrtf(cx * cx + cy * cy + cz * cz);
  const float excess = d - L.d0;
  const bool restrained = excess > 0.f;
  const float fr = restrained ? -L.krest * excess / d * L.inv_total_mass : 0.f;

  float psi[C];
#pragma unroll
  for (int c = 0; c < C; ++c) psi[c] = 0.f;
#pragma unroll
  for (int a = 0; a < APL; ++a) {
    const int atom = lane + kWave * a;
    const bool valid = atom < n;
    float sc[C], e[C], de[C][3];
#pragma unroll
    for (int c = 0; c < C; ++c) sc[c] = valid ? L.scale[atom * C + c] : 0.f;
    grid_finish<C, FORCES>(g, cn[a], sc, e, de);
#pragma unroll
    for (int c = 0; c < C; ++c) psi[c] += e[c];
    if (FORCES) {
      float fx = 0.f, fy = 0.f, fz = 0.f;
      if (valid) {
        const int b = L.gstart[atom], eidx = L.gstart[atom + 1];
        for (int q = b; q < eidx; ++q) {
          const int s = L.gidx[q];
          fx += sl.x[s];
          fy += sl.y[s];
          fz += sl.z[s];
        }
        fx += fr * m[a] * cx;
        fy += fr * m[a] * cy;
        fz += fr * m[a] * cz;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          fx -= w[c] * de[c][0];
          fy -= w[c] * de[c][1];
          fz -= w[c] * de[c][2];
        }
      }
      f[a][0] = fx;
      f[a][1] = fy;
      f[a][2] = fz;
    }
  }
  if (ENERGY) {
    terms[0] = wave_sum((double)eb);
    terms[1] = wave_sum((double)ea);
    terms[2] = wave_sum((double)et);
    terms[3] = restrained ? 0.5 * (double)L.krest * (double)excess *
                                (double)excess
                          : 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) terms[4 + c] = wave_sum((double)psi[c]);
  }
  // keep the next evaluation's position writes behind this one's reads
  wave_lds_sync();
}

}  // namespace bpmf
