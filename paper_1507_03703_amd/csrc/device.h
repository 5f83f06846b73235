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

// Wavefront sums with DPP row operations (quad permutes, half-row and row
// mirrors, then row broadcasts 15 and 31 into the upper rows); the total
// ends in lane 63 and is read back as a wave-uniform value.  The order of
// the additions is fixed, so every lane sees the same, reproducible sum.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL,
                                                    ROWMASK, 0xf, false));
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL,
                                             ROWMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK,
                                             0xf, false);
  return __longlong_as_double(((long long)hi << 32) |
                              (long long)(unsigned)lo);
}

__device__ __forceinline__ float wave_sumf(float v) {
  v += dpp_f<0xB1, 0xf>(v);   // quad_perm [1,0,3,2]
  v += dpp_f<0x4E, 0xf>(v);   // quad_perm [2,3,0,1]
  v += dpp_f<0x141, 0xf>(v);  // row_half_mirror
  v += dpp_f<0x140, 0xf>(v);  // row_mirror: every lane holds its row sum
  v += dpp_f<0x142, 0xa>(v);  // row_bcast:15 into rows 1, 3
  v += dpp_f<0x143, 0xc>(v);  // row_bcast:31 into rows 2, 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// three independent sums with the stages interleaved (each value sees the
// same additions in the same order as wave_sumf)
__device__ __forceinline__ void wave_sumf3(float& a, float& b, float& c) {
  a += dpp_f<0xB1, 0xf>(a);
  b += dpp_f<0xB1, 0xf>(b);
  c += dpp_f<0xB1, 0xf>(c);
  a += dpp_f<0x4E, 0xf>(a);
  b += dpp_f<0x4E, 0xf>(b);
  c += dpp_f<0x4E, 0xf>(c);
  a += dpp_f<0x141, 0xf>(a);
  b += dpp_f<0x141, 0xf>(b);
  c += dpp_f<0x141, 0xf>(c);
  a += dpp_f<0x140, 0xf>(a);
  b += dpp_f<0x140, 0xf>(b);
  c += dpp_f<0x140, 0xf>(c);
  a += dpp_f<0x142, 0xa>(a);
  b += dpp_f<0x142, 0xa>(b);
  c += dpp_f<0x142, 0xa>(c);
  a += dpp_f<0x143, 0xc>(a);
  b += dpp_f<0x143, 0xc>(b);
  c += dpp_f<0x143, 0xc>(c);
  a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(a), 63));
  b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(b), 63));
  c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(c), 63));
}

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<0xB1, 0xf>(v);
  v += dpp_d<0x4E, 0xf>(v);
  v += dpp_d<0x141, 0xf>(v);
  v += dpp_d<0x140, 0xf>(v);
  v += dpp_d<0x142, 0xa>(v);
  v += dpp_d<0x143, 0xc>(v);
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
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

// The Metropolis test ln u < t for u = u01d(v), decided exactly as in double
// precision: u >= 2^-32 puts |ln u| below 22.2, where the single-precision
// logarithm (of u rounded to float) is within 1e-5 of ln u, so outside a
// band of 1e-4 about t its answer is the double one; inside the band the
// double logarithm decides.  t must not be NaN.
__device__ __forceinline__ bool ln_u_below(uint32_t v, double t) {
  const double u = u01d(v);
  const double lf = (double)logf((float)u);
  if (lf < t - 1e-4) return true;
  if (lf > t + 1e-4) return false;
  return log(u) < t;
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
// (x, y<<1, z<<2), read from the cell's record with 16-byte loads.  Issued
// as independent loads so that callers can overlap their latency with other
// work before consuming them.
template <int C>
struct Corners {
  float v[8][C];
  AxisPos ax, ay, az;
};

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int C>
__device__ __forceinline__ void grid_fetch(const GridDev& g, float px,
                                           float py, float pz,
                                           Corners<C>& k) {
  static_assert((8 * C) % 4 == 0, "records are read as float4");
  k.ax = grid_axis(px, g.ox, g.inv_h, g.nx);
  k.ay = grid_axis(py, g.oy, g.inv_h, g.ny);
  k.az = grid_axis(pz, g.oz, g.inv_h, g.nz);
  // fewer than 2^31 cells and at most 2^24 nodes per axis (checked at
  // upload): 24-bit products, a 32-bit index
  const unsigned int cell =
      __umul24(__umul24(k.az.i, g.ny - 1) + k.ay.i, g.nx - 1) + k.ax.i;
  // the grid lives in global memory: say so, so that the gathers are
  // global (not flat) loads and LDS waits do not wait on them
  typedef const f32x4 __attribute__((address_space(1))) gvec;
  gvec* rec = (gvec*)g.cells + (size_t)cell * (cell_stride(C) / 4);
  float b[8 * C];
#pragma unroll
  for (int j = 0; j < 2 * C; ++j) {
    const f32x4 t = rec[j];
    b[4 * j] = t.x;
    b[4 * j + 1] = t.y;
    b[4 * j + 2] = t.z;
    b[4 * j + 3] = t.w;
  }
#pragma unroll
  for (int q = 0; q < 8; ++q)
#pragma unroll
    for (int c = 0; c < C; ++c) k.v[q][c] = b[q * C + c];
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

// Per-atom force accumulators in LDS, in 32-bit fixed point (2^-16
// kJ/mol/A per unit, contributions rounded toward zero): every bonded-term
// thread adds its contribution to each of its atoms with an integer LDS
// atomic.  Integer addition is
// associative, so the sums do not depend on the order in which threads
// arrive and results stay bitwise reproducible.  Quantisation is 1.5e-5
// kJ/mol/A per contribution; a contribution saturates at the int32 range,
// +-32768 kJ/mol/A (a bonded force that large only arises on a diverging
// trajectory, which the exact energy rejects; leapfrog with any
// deterministic force keeps HMC exact).  The term functions hand over
// contributions already in units of 2^-16 (their force factor carries the
// 2^16, and scaling by a power of two commutes with rounding, so the units
// are exact); a NaN contribution becomes 0 (its energy is NaN too, so the
// move is rejected).
constexpr float kFix = 65536.0f;          // 2^16
constexpr float kFixInv = 1.0f / 65536.0f;

// rounds toward zero and saturates out-of-range values, NaN to 0: the
// hardware conversion, written out because a C++ float-to-int conversion
// of an out-of-range value is undefined
__device__ __forceinline__ unsigned int to_fix_units(float f) {
  int r;
  asm("v_cvt_i32_f32 %0, %1" : "=v"(r) : "v"(f));
  return (unsigned int)r;
}

__device__ __forceinline__ float from_fix(unsigned int a) {
  return (float)(int)a * kFixInv;
}

// a word of LDS, addressed with 32-bit arithmetic
typedef __attribute__((address_space(3))) unsigned int lds_u32;

struct Slots {
  lds_u32* acc;  // kAccCopies x n x 3
  int stride;    // 3 n: words per copy
  // f: force contribution in units of 2^-16 kJ/mol/A, into the lane's copy
  __device__ __forceinline__ void put(int atom, float3 f) const {
    lds_u32* a = acc + __umul24(threadIdx.x & (kAccCopies - 1), stride) +
                 __umul24(atom, 3);
    __hip_atomic_fetch_add(a, to_fix_units(f.x), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add(a + 1, to_fix_units(f.y), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
    __hip_atomic_fetch_add(a + 2, to_fix_units(f.z), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
  }
};

// Global-memory view of a device pointer.  Pointers read from a table in
// memory reach a kernel as generic (flat) addresses, and flat loads and
// stores also count against the LDS wait counter: every LDS wait after one
// would wait on memory.  Accesses through this view are global ones.
#define BPMF_GMEM(T, p) ((T __attribute__((address_space(1)))*)(p))

// hardware reciprocal, square root and reciprocal square root (1 ulp, no
// rescaling of denormal arguments: the bonded-term geometry never sees
// one), for the bonded-term geometry
__device__ __forceinline__ float rcp(float x) {
  return __builtin_amdgcn_rcpf(x);
}
__device__ __forceinline__ float hsqrt(float x) {
  return __builtin_amdgcn_sqrtf(x);
}
__device__ __forceinline__ float hrsq(float x) {
  return __builtin_amdgcn_rsqf(x);
}

__device__ __forceinline__ int atom_of(int p) { return p; }
__device__ __forceinline__ int slot_of(int p) { return p; }

// K (r - r0)^2
template <bool FORCES>
__device__ __forceinline__ float bond_term(const float4* pos, int2 ij,
                                           float2 par, const Slots& sl) {
  const float3 d = sub(f3(pos[atom_of(ij.x)]), f3(pos[atom_of(ij.y)]));
  const float d2 = dot(d, d), ir = hrsq(d2);
  const float r = d2 > 0.f ? d2 * ir : 0.f;
  const float dr = r - par.y;
  if (FORCES) {
    const float f = -2.0f * par.x * dr * ir * kFix;
    sl.put(slot_of(ij.x), scale3(f, d));
    sl.put(slot_of(ij.y), scale3(-f, d));
  }
  return par.x * dr * dr;
}

// atan2(y, x) for y >= 0 (an angle in [0, pi]): the octant's ratio
// t = min/max in [0, 1] and atan t = t P(t^2), P of degree 8 fitted to
// atan(t)/t on [0, 1] by reweighted least squares (fit_atan.py beside the
// package; 6e-9 absolute in exact arithmetic, within 1e-7 in float); 0 when
// both arguments are 0
__device__ __forceinline__ float angle_atan2(float y, float x) {
  const float ax = fabsf(x);
  const float lo = fminf(y, ax), hi = fmaxf(y, ax);
  const float t = hi > 0.f ? lo * rcp(hi) : 0.f;
  const float s = t * t;
  float p = 2.456722575e-03f;
  p = fmaf(p, s, -1.440135319e-02f);
  p = fmaf(p, s, 3.978122321e-02f);
  p = fmaf(p, s, -7.234858229e-02f);
  p = fmaf(p, s, 1.049894713e-01f);
  p = fmaf(p, s, -1.416122975e-01f);
  p = fmaf(p, s, 1.998590691e-01f);
  p = fmaf(p, s, -3.333259704e-01f);
  p = fmaf(p, s, 9.999998864e-01f);
  float th = p * t;
  th = y > ax ? 1.57079632679f - th : th;
  return x < 0.f ? 3.14159265359f - th : th;
}

// K (theta - theta0)^2, theta = atan2(|a x b|, a.b), a = xi-xj, b = xk-xj
template <bool FORCES>
__device__ __forceinline__ float angle_term(const float4* pos, int4 ijk,
                                            float2 par, const Slots& sl) {
  const float3 xj = f3(pos[atom_of(ijk.y)]);
  const float3 a = sub(f3(pos[atom_of(ijk.x)]), xj);
  const float3 b = sub(f3(pos[atom_of(ijk.z)]), xj);
  const float3 c = cross(a, b);
  const float cc = dot(c, c), is = hrsq(cc), co = dot(a, b);
  const float s = cc > 0.f ? cc * is : 0.f;
  const float th = angle_atan2(s, co);
  const float dth = th - par.y;
  if (FORCES) {
    const float aa = dot(a, a), bb = dot(b, b);
    const float ila = hrsq(aa), ilb = hrsq(bb);
    const float dE = 2.0f * par.x * dth;
    const float cth = co * ila * ilb;
    const float3 ah = scale3(ila, a), bh = scale3(ilb, b);
    // d theta / d xi = (cos a^ - b^) / (|a| sin), d theta / d xk likewise;
    // 1 / (|a| sin) = |b| / |a x b|
    const float ci = dE * (bb * ilb) * is * kFix;
    const float ck = dE * (aa * ila) * is * kFix;
    const float3 fi = make_float3(-ci * (cth * ah.x - bh.x),
                                  -ci * (cth * ah.y - bh.y),
                                  -ci * (cth * ah.z - bh.z));
    const float3 fk = make_float3(-ck * (cth * bh.x - ah.x),
                                  -ck * (cth * bh.y - ah.y),
                                  -ck * (cth * bh.z - ah.z));
    sl.put(slot_of(ijk.x), fi);
    sl.put(slot_of(ijk.y), make_float3(-(fi.x + fk.x), -(fi.y + fk.y),
                                       -(fi.z + fk.z)));
    sl.put(slot_of(ijk.z), fk);
  }
  return par.x * dth * dth;
}

// (V/2)(1 + cos(n phi - gamma)), IUPAC phi; forces in the singularity-free
// form of Blondel & Karplus (J. Comput. Chem. 17, 1132, 1996).  With
// x = n1.n2 and y = |b2| b1.n2 one has x^2 + y^2 = |n1|^2 |n2|^2, so
// cos phi = x/r and sin phi = y/r (r = |n1||n2|); for integer
// multiplicities 1..6 (par.w = n, else 0) cos(n phi) and sin(n phi) follow
// by complex multiplication and no inverse trigonometric call is needed.
template <bool FORCES>
__device__ __forceinline__ float torsion_term(const float4* pos, int4 ijkl,
                                              float4 par, const Slots& sl) {
  const float3 xi = f3(pos[atom_of(ijkl.x)]), xj = f3(pos[atom_of(ijkl.y)]);
  const float3 xk = f3(pos[atom_of(ijkl.z)]), xl = f3(pos[atom_of(ijkl.w)]);
  const float3 b1 = sub(xj, xi), b2 = sub(xk, xj), b3 = sub(xl, xk);
  const float3 n1 = cross(b1, b2), n2 = cross(b2, b3);
  const float b22 = dot(b2, b2), ilb2 = hrsq(b22);
  const float lb2 = b22 * ilb2;
  const float xx = dot(n1, n2), yy = lb2 * dot(b1, n2);
  // par: V/2, n, cos gamma, sin gamma; integer multiplicity in the sign-free
  // upper bits is not needed: n is an integer 1..6 (checked at setup)
  const int mult = (int)par.y;
  const float ir = hrsq(xx * xx + yy * yy);
  const float c1 = xx * ir, s1 = yy * ir;
  float cn = c1, sn = s1;
  for (int q = 1; q < mult; ++q) {
    const float c2 = cn * c1 - sn * s1;
    sn = sn * c1 + cn * s1;
    cn = c2;
  }
  // cos(n phi - gamma), sin(n phi - gamma)
  const float cg = par.z, sg = par.w;
  const float cs = cn * cg + sn * sg;
  const float snm = sn * cg - cn * sg;
  if (FORCES) {
    // -dE/dphi in force units of 2^-16, folded into the four scalars of
    // the gradient: F_i = ai n1, F_l = al n2, F_j = -F_i + P n1 + Q n2,
    // F_k = -F_l - P n1 - Q n2
    const float dEs = par.x * par.y * snm * kFix;
    const float in1 = rcp(dot(n1, n1)), in2 = rcp(dot(n2, n2));
    const float lin1 = lb2 * in1, lin2 = lb2 * in2;
    const float P = dot(b1, b2) * ilb2 * in1 * dEs;
    const float Q = dot(b2, b3) * ilb2 * in2 * dEs;
    const float ai = -lin1 * dEs, al = lin2 * dEs;
    const float3 fi = scale3(ai, n1), fl = scale3(al, n2);
    sl.put(slot_of(ijkl.x), fi);
    sl.put(slot_of(ijkl.y),
           make_float3(fmaf(P, n1.x, fmaf(Q, n2.x, -fi.x)),
                       fmaf(P, n1.y, fmaf(Q, n2.y, -fi.y)),
                       fmaf(P, n1.z, fmaf(Q, n2.z, -fi.z))));
    sl.put(slot_of(ijkl.z),
           make_float3(fmaf(-P, n1.x, fmaf(-Q, n2.x, -fl.x)),
                       fmaf(-P, n1.y, fmaf(-Q, n2.y, -fl.y)),
                       fmaf(-P, n1.z, fmaf(-Q, n2.z, -fl.z))));
    sl.put(slot_of(ijkl.w), fl);
  }
  return par.x * (1.0f + cs);
}

// ----------------------------------------------------------------------------
// one full evaluation of a configuration by one workgroup of W wavefronts
// ----------------------------------------------------------------------------
// Thread t owns atom t (n <= 64 W); the A = ceil(n / 64) wavefronts that
// hold atoms are the atom waves.  Bonded terms come in chunks of 64 of one
// kind, so a wavefront never diverges over term kinds, and the ligand's
// schedule deals the chunks to the wavefronts so that their work is
// balanced (each wavefront of a workgroup runs on its own SIMD, so the
// busiest one sets the pace of the step); an atom wave takes chunks only
// once the others carry as much as its grid work.  With four or more
// wavefronts and at least as many spare as atom waves
// (bonded_first_wave(..) > 0) the atom waves issue their gathers after the
// first barrier, so that the spare waves start their chunks without waiting
// for the address work; otherwise the owners' grid gathers are issued before the
// first barrier so that their latency overlaps the bonded pass (a workgroup
// barrier on gfx950 waits on LDS traffic only, not on outstanding global
// loads).
//
// Shared memory (Shared): positions, force slots, per-wave partial sums.
struct Shared {
  float4* pos;     // 64 W
  Slots sl;        // n x 3 fixed-point force accumulators
  float* com;      // W x 3
  double* red;     // W x kRed
  // ligand topology staged once per launch (stage_topology)
  const int2* bij;
  const float2* bpar;
  const int4* aijk;
  const float2* apar;
  const int4* tijkl;
  const float4* tpar;
  const unsigned short* sched;  // this launch width's schedule row
  // pair terms in the energy (L.pairs_on): staged parameters and scratch
  const float4* pp0;        // n: q, sigma, sqrt(eps), rho
  const float2* pp1;        // n: rt, S rt
  const uint32_t* pex;      // n x kPairWords excluded-pair masks
  const uint32_t* p14;      // n x kPairWords 1-4 masks
  float* pR;                // n Born radii
  float* pb;                // n chain-rule factors dE/dR_i dR_i/dI_i
  float* pscr;              // slices x n x 9 partial sums (pair_stage)
};

// Copy a ligand's constant topology into LDS (all threads; caller syncs).
// `raw` points past the per-evaluation areas; layout: tpar (nt float4),
// tijkl (nt int4), aijk (na int4), apar (na float2), bij (nb int2), bpar
// (nb float2).
__device__ __forceinline__ void stage_topology(const LigDev& L,
                                               unsigned char* raw, Shared& sh,
                                               int tid, int nthreads) {
  float4* tpar = reinterpret_cast<float4*>(raw);
  int4* tijkl = reinterpret_cast<int4*>(tpar + L.nt);
  int4* aijk = tijkl + L.nt;
  float2* apar = reinterpret_cast<float2*>(aijk + L.na);
  int2* bij = reinterpret_cast<int2*>(apar + L.na);
  float2* bpar = reinterpret_cast<float2*>(bij + L.nb);
  unsigned short* sched = reinterpret_cast<unsigned short*>(bpar + L.nb);
  // global (not flat) loads: they cannot alias the LDS stores, so several
  // stay in flight at once
  typedef float f4v __attribute__((ext_vector_type(4)));
  typedef int i4v __attribute__((ext_vector_type(4)));
  typedef float f2v __attribute__((ext_vector_type(2)));
  typedef int i2v __attribute__((ext_vector_type(2)));
  typedef const f4v __attribute__((address_space(1))) gf4;
  typedef const i4v __attribute__((address_space(1))) gi4;
  typedef const f2v __attribute__((address_space(1))) gf2;
  typedef const i2v __attribute__((address_space(1))) gi2;
  for (int i = tid; i < L.nt; i += nthreads) {
    const f4v p = ((gf4*)L.tpar)[i];
    const i4v q = ((gi4*)L.tijkl)[i];
    tpar[i] = make_float4(p.x, p.y, p.z, p.w);
    tijkl[i] = make_int4(q.x, q.y, q.z, q.w);
  }
  for (int i = tid; i < L.na; i += nthreads) {
    const i4v q = ((gi4*)L.aijk)[i];
    const f2v p = ((gf2*)L.apar)[i];
    aijk[i] = make_int4(q.x, q.y, q.z, q.w);
    apar[i] = make_float2(p.x, p.y);
  }
  for (int i = tid; i < L.nb; i += nthreads) {
    const i2v q = ((gi2*)L.bij)[i];
    const f2v p = ((gf2*)L.bpar)[i];
    bij[i] = make_int2(q.x, q.y);
    bpar[i] = make_float2(p.x, p.y);
  }
  // the schedule row of this launch width (nthreads / 64 wavefronts)
  const int row = sched_row(L.nb, L.na, L.nt);
  const int q = nthreads <= kWave ? 0 : nthreads <= 2 * kWave ? 1
                : nthreads <= 4 * kWave ? 2 : 3;
  for (int i = tid; i < row; i += nthreads)
    sched[i] = BPMF_GMEM(const unsigned short, L.bsched)[q * row + i];
  sh.sched = sched;
  sh.bij = bij;
  sh.bpar = bpar;
  if (L.pairs_on) {
    // pair parameters after the schedule row, 16-byte aligned (raw is)
    unsigned char* pb0 =
        raw + ((32 * L.nt + 24 * L.na + 16 * L.nb + 2 * row + 15) & ~15);
    const int n = L.n;
    float4* p0 = reinterpret_cast<float4*>(pb0);
    float2* p1 = reinterpret_cast<float2*>(p0 + n);
    uint32_t* ex = reinterpret_cast<uint32_t*>(p1 + n);
    uint32_t* o4 = ex + n * kPairWords;
    float* R = reinterpret_cast<float*>(o4 + n * kPairWords);
    typedef float f4v __attribute__((ext_vector_type(4)));
    typedef float f2v __attribute__((ext_vector_type(2)));
    typedef const f4v __attribute__((address_space(1))) gf4;
    typedef const f2v __attribute__((address_space(1))) gf2;
    for (int i = tid; i < n; i += nthreads) {
      const f4v a = ((gf4*)L.pair.p0)[i];
      const f2v b = ((gf2*)L.pair.p1)[i];
      p0[i] = make_float4(a.x, a.y, a.z, a.w);
      p1[i] = make_float2(b.x, b.y);
    }
    for (int i = tid; i < n * kPairWords; i += nthreads) {
      ex[i] = BPMF_GMEM(const uint32_t, L.pair.excl)[i];
      o4[i] = BPMF_GMEM(const uint32_t, L.pair.o14)[i];
    }
    sh.pp0 = p0;
    sh.pp1 = p1;
    sh.pex = ex;
    sh.p14 = o4;
    sh.pR = R;
    sh.pb = R + n;
    sh.pscr = R + 2 * n;
  }
  sh.aijk = aijk;
  sh.apar = apar;
  sh.tijkl = tijkl;
  sh.tpar = tpar;
}

constexpr int kRedMax = kRedSlots;  // U_bond..U_tors, Psi_c, two extras

// Force assembly of one atom, shared by eval_block and the sweep kernel's
// start-of-trajectory reuse so that both give the same bits:
// ge = -sum_c w_c grad e_c (channels in order), then + the restraint force
// fr m (c - c0), then f = bonded + ge.
template <int C>
__device__ __forceinline__ void grid_force(const float* w,
                                           const float (&de)[C][3],
                                           float (&ge)[3]) {
#pragma unroll
  for (int c = 0; c < C; ++c) {
    ge[0] -= w[c] * de[c][0];
    ge[1] -= w[c] * de[c][1];
    ge[2] -= w[c] * de[c][2];
  }
}
__device__ __forceinline__ void restraint_force(float fr, float m, float cx,
                                                float cy, float cz,
                                                float (&ge)[3]) {
  ge[0] += fr * m * cx;
  ge[1] += fr * m * cy;
  ge[2] += fr * m * cz;
}

// number of leading wavefronts (the atom waves) that issue their grid
// gathers after the first barrier, 0 when they issue them before it (see
// eval_block)
__device__ __forceinline__ int bonded_first_wave(int waves, int atom_waves) {
  return (waves >= 4 && waves >= 2 * atom_waves) ? atom_waves : 0;
}

__device__ __forceinline__ void block_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// The ligand's intramolecular nonbonded and OBC GB/SA energy (the terms of
// bpmf_pair_evaluate) for the configuration in sh.pos.  Every atom's row of
// pair terms (each pair is visited from both ends, so forces need no
// atomics) is split over the block's wavefronts: thread t takes atom
// i = lane + 64 (wave mod A) (A = atom waves) and slice k = wave / A of its
// partners j (S = waves / A slices of [0, n)), and writes its partial sums
// to LDS; the atom's owner adds the S partials in slice order.  Three
// passes, each followed by a workgroup barrier and a combine (which every
// thread of the block calls): (1) LJ, Coulomb and the descreening sum,
// giving the Born radius, and v_i = sum_j dH(r_ij; a_i, s_j) (x_i - x_j) /
// r_ij; (2) GB energy, its explicit force and dE/dR_i, then the self and
// surface terms; (3) the chain rule through the Born radii (FORCES):
// -b_i v_i - sum_j b_j dH(r_ij; a_j, s_i) (x_i - x_j) / r_ij, with
// b = dE/dR dR/dI.  e: the owner's share of the energy; pf: the force on
// its atom (FORCES); both 0 on other threads.
template <bool FORCES>
__device__ __forceinline__ void pair_stage(const Shared& sh, const PairDev& P,
                                           int n, int tid, int nthreads,
                                           float& e, float (&pf)[3]) {
  const int A = (n + kWave - 1) / kWave;
  const int S = pair_slices(n, nthreads / kWave);
  const int wv = tid >> 6;
  const int i = (tid & (kWave - 1)) + kWave * (wv % A);
  const int k = wv / A;
  const bool act = k < S && i < n;
  const bool own = tid < n;  // slice 0's thread of atom tid
  const int j0 = k * n / S, j1 = (k + 1) * n / S;
  float* const part = sh.pscr + (size_t)(k * n + i) * 9;
  float4 xi = make_float4(0.f, 0.f, 0.f, 0.f), pi = xi;
  float2 qi1 = make_float2(0.f, 0.f);
  if (act) {
    xi = sh.pos[i];
    pi = sh.pp0[i];
    qi1 = sh.pp1[i];
  }
  // (1) LJ, Coulomb, descreening
  if (act) {
    float I = 0.f, e_lj = 0.f, e_c = 0.f, fx = 0.f, fy = 0.f, fz = 0.f;
    float vx = 0.f, vy = 0.f, vz = 0.f;
    for (int j = j0; j < j1; ++j) {
      if (j == i) continue;
      const float4 xj = sh.pos[j], pj = sh.pp0[j];
      const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
      const float r2 = dx * dx + dy * dy + dz * dz;
      const float ir = __builtin_amdgcn_rsqf(r2), r = r2 * ir;
      float H, dH;
      hct(r, ir, qi1.x, sh.pp1[j].y, H, dH);
      I += H;
      if (FORCES) {
        const float h = dH * ir;
        vx += h * dx;
        vy += h * dy;
        vz += h * dz;
      }
      const int w = i * kPairWords + (j >> 5);
      const uint32_t bit = 1u << (j & 31);
      if (sh.pex[w] & bit) continue;
      const float sg = 0.5f * (pi.y + pj.y), ep = pi.z * pj.z;
      const float ir2 = ir * ir;
      const float sr2 = sg * sg * ir2, sr6 = sr2 * sr2 * sr2;
      float lj = 4.f * ep * (sr6 * sr6 - sr6);
      float flj = 24.f * ep * (2.f * sr6 * sr6 - sr6) * ir2;
      float cl = P.kc * pi.x * pj.x * ir;
      float fcl = cl * ir2;
      if (sh.p14[w] & bit) {
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
    part[0] = I;
    part[1] = e_lj;
    part[2] = e_c;
    part[3] = fx;
    part[4] = fy;
    part[5] = fz;
    part[6] = vx;
    part[7] = vy;
    part[8] = vz;
  }
  block_sync();
  float e_lj = 0.f, e_c = 0.f, fx = 0.f, fy = 0.f, fz = 0.f;
  float vx = 0.f, vy = 0.f, vz = 0.f;
  float Ri = 0.f, dRdI = 0.f;
  if (own) {
    float I = 0.f;
    for (int q = 0; q < S; ++q) {
      const float* o = sh.pscr + (size_t)(q * n + tid) * 9;
      I += o[0];
      e_lj += o[1];
      e_c += o[2];
      fx += o[3];
      fy += o[4];
      fz += o[5];
      vx += o[6];
      vy += o[7];
      vz += o[8];
    }
    const float psi = I * qi1.x;
    const float t = psi * (kObcA - psi * (kObcB - kObcC * psi));
    const float th = tanhf(t);
    Ri = 1.f / (1.f / qi1.x - th / pi.w);
    dRdI = Ri * Ri * (1.f - th * th) *
           (kObcA - psi * (2.f * kObcB - 3.f * kObcC * psi)) * qi1.x / pi.w;
    sh.pR[tid] = Ri;
  }
  block_sync();
  // (2) generalised Born pairs
  if (act) {
    const float qi = pi.x, Rii = sh.pR[i];
    float e_gb = 0.f, dEdR = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
    for (int j = j0; j < j1; ++j) {
      if (j == i) continue;
      const float4 xj = sh.pos[j];
      const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
      const float r2 = dx * dx + dy * dy + dz * dz;
      const float Rj = sh.pR[j];
      const float RR = Rii * Rj;
      const float iRR = __builtin_amdgcn_rcpf(RR);
      const float D = __expf(-0.25f * r2 * iRR);
      const float f2 = r2 + RR * D;
      const float invf = rsqrtf(f2);
      const float invf3 = invf * invf * invf;
      const float kq = P.kgb * qi * sh.pp0[j].x;
      e_gb += 0.5f * kq * invf;
      if (FORCES) {
        const float g = kq * (1.f - 0.25f * D) * invf3;
        gx += g * dx;
        gy += g * dy;
        gz += g * dz;
        dEdR -= 0.5f * kq * Rj * D * (1.f + 0.25f * r2 * iRR) * invf3;
      }
    }
    part[0] = e_gb;
    part[1] = dEdR;
    part[2] = gx;
    part[3] = gy;
    part[4] = gz;
  }
  block_sync();
  float e_gb = 0.f, e_sa = 0.f;
  if (own) {
    const float qi = pi.x;
    float dEdR = 0.f;
    for (int q = 0; q < S; ++q) {
      const float* o = sh.pscr + (size_t)(q * n + tid) * 9;
      e_gb += o[0];
      dEdR += o[1];
      fx += o[2];
      fy += o[3];
      fz += o[4];
    }
    // the atom's self term
    e_gb += 0.5f * P.kgb * qi * qi / Ri;
    dEdR -= 0.5f * P.kgb * qi * qi / (Ri * Ri);
    const float rp = pi.w + P.probe;
    const float q6 = pi.w / Ri, q3 = q6 * q6 * q6;
    e_sa = P.sa * rp * rp * q3 * q3;
    dEdR -= 6.f * e_sa / Ri;
    sh.pb[tid] = dEdR * dRdI;
  }
  if (FORCES) {
    block_sync();
    // (3) the chain rule through the Born radii: the partners' radii here,
    // the atom's own from v_i
    if (act) {
      float gx = 0.f, gy = 0.f, gz = 0.f;
      for (int j = j0; j < j1; ++j) {
        if (j == i) continue;
        const float4 xj = sh.pos[j];
        const float2 pj1 = sh.pp1[j];
        const float dx = xi.x - xj.x, dy = xi.y - xj.y, dz = xi.z - xj.z;
        const float r2 = dx * dx + dy * dy + dz * dz;
        const float ir = __builtin_amdgcn_rsqf(r2), r = r2 * ir;
        float Hj, dHj;
        hct(r, ir, pj1.x, qi1.y, Hj, dHj);
        const float g = -sh.pb[j] * dHj * ir;
        gx += g * dx;
        gy += g * dy;
        gz += g * dz;
      }
      part[0] = gx;
      part[1] = gy;
      part[2] = gz;
    }
    block_sync();
    if (own) {
      const float bi = sh.pb[tid];
      fx -= bi * vx;
      fy -= bi * vy;
      fz -= bi * vz;
      for (int q = 0; q < S; ++q) {
        const float* o = sh.pscr + (size_t)(q * n + tid) * 9;
        fx += o[0];
        fy += o[1];
        fz += o[2];
      }
    }
  }
  e = own ? e_lj + e_c + e_gb + e_sa : 0.f;
  pf[0] = own ? fx : 0.f;
  pf[1] = own ? fy : 0.f;
  pf[2] = own ? fz : 0.f;
}

// sc: per-atom grid factors of the thread's atom (0 for non-owners).
// terms (ENERGY): [U_bond, U_angle, U_tors, U_I, Psi_0..Psi_{C-1}, X0, X1]
// (LEAN: [U_bond + U_angle + U_tors, 0, 0, U_I, Psi_c, 0, 0])
// where X0, X1 are block sums of the caller's per-thread extras; identical
// on every thread.  f (FORCES): -grad(U_bonded + U_I + sum_c w_c Psi_c) of
// the thread's atom.
// BONDED false: the grid terms and the restraint only (terms[0..2] = 0; no
// topology needs to be staged), for rigid moves, which leave the bonded
// energy unchanged.
// PAIRS: the ligand's pair terms join the energy when L.pairs_on (their
// energy is summed with the bonded terms, in terms[0]; their force is part
// of the state-independent force).
template <int C, int W, bool FORCES, bool ENERGY, bool LEAN = false,
          bool BONDED = true, bool PAIRS = false, bool TERMS0 = false>
__device__ __forceinline__ void eval_block(const GridDev& g, const LigDev& L,
                                           const float* w, const float (&x)[3],
                                           float m, const float (&sc)[C],
                                           float (&f)[3],
                                           double (&terms)[6 + C],
                                           float ex0, float ex1,
                                           const Shared& sh, int tid,
                                           float* cache_atom = nullptr,
                                           float* cache_rep = nullptr) {
  const int n = L.n;
  const int lane = tid & (kWave - 1), wv = tid >> 6;
  const bool owner = tid < n;
  const int n_atom_waves = (n + kWave - 1) / kWave;
  const bool wave_has_atoms = wv < n_atom_waves;
  const int first = bonded_first_wave(W, n_atom_waves);
  // positions with the atom's mass (w), for the centre of mass
  if (owner) sh.pos[tid] = make_float4(x[0], x[1], x[2], m);
  // grid gathers: before the barrier when the atom waves also take bonded
  // terms (the loads fly during them), after it when they do not (the
  // bonded waves then start without waiting for the address work)
  Corners<C> cn;
  if (wave_has_atoms && first == 0) grid_fetch<C>(g, x[0], x[1], x[2], cn);
  block_sync();
  if (wave_has_atoms && first != 0) grid_fetch<C>(g, x[0], x[1], x[2], cn);

  // bonded terms: the chunks the ligand's schedule gives this wavefront
  float eb = 0.f, ea = 0.f, et = 0.f;
  if (BONDED) {
    const int bw = __builtin_amdgcn_readfirstlane(wv);
    {
      const int ntc = (L.nt + kWave - 1) / kWave;
      const int nac = (L.na + kWave - 1) / kWave;
      const int j0 = sh.sched[bw], j1 = sh.sched[bw + 1];
      // the wavefront's chunk list, one entry per lane, read once
      const int mine = j0 + lane < j1 ? sh.sched[9 + j0 + lane] : 0;
      for (int j = j0; j < j1; ++j) {
        const int ch = __builtin_amdgcn_readlane(mine, j - j0);
        if (ch < ntc) {
          const int t = ch * kWave + lane;
          if (t < L.nt)
            et += torsion_term<FORCES>(sh.pos, sh.tijkl[t], sh.tpar[t],
                                       sh.sl);
        } else if (ch < ntc + nac) {
          const int t = (ch - ntc) * kWave + lane;
          if (t < L.na)
            ea += angle_term<FORCES>(sh.pos, sh.aijk[t], sh.apar[t], sh.sl);
        } else {
          const int t = (ch - ntc - nac) * kWave + lane;
          if (t < L.nb)
            eb += bond_term<FORCES>(sh.pos, sh.bij[t], sh.bpar[t], sh.sl);
        }
      }
    }
  }

  // atom waves: mass-weighted position sums of all atoms (restraint; with
  // two atom waves each sums both halves from the staged positions, lane l
  // taking atoms l and l + 64, so that both hold the same total without a
  // barrier) and the grid values and gradients, beside the bonded waves
  float psi[C];
#pragma unroll
  for (int c = 0; c < C; ++c) psi[c] = 0.f;
  float ge[3] = {0.f, 0.f, 0.f};
  float de[C][3];
  float px = 0.f, py = 0.f, pz = 0.f;
  if (wave_has_atoms) {
    if (n_atom_waves == 1) {
      px = m * x[0];
      py = m * x[1];
      pz = m * x[2];
    } else {
      const float4 a = sh.pos[lane];
      px = a.w * a.x;
      py = a.w * a.y;
      pz = a.w * a.z;
      if (lane + kWave < n) {
        const float4 b = sh.pos[lane + kWave];
        px += b.w * b.x;
        py += b.w * b.y;
        pz += b.w * b.z;
      }
    }
    wave_sumf3(px, py, pz);
    // for the waves without atoms (restraint energy)
    if (tid == 0) {
      sh.com[0] = px;
      sh.com[1] = py;
      sh.com[2] = pz;
    }
    float e[C];
    grid_finish<C, FORCES>(g, cn, sc, e, de);
#pragma unroll
    for (int c = 0; c < C; ++c) psi[c] = e[c];
    if (FORCES) grid_force<C>(w, de, ge);
  }
  // intramolecular nonbonded and implicit-solvent terms
  float epair = 0.f, fpair[3] = {0.f, 0.f, 0.f};
  const bool pairs = PAIRS && L.pairs_on;
  if (pairs) pair_stage<FORCES>(sh, L.pair, n, tid, W * kWave, epair, fpair);
  // centre of mass offset from the site (an atom wave's own total, which
  // wave 0 publishes for the others)
  float cx, cy, cz;
  auto com_offset = [&]() {
    if (wave_has_atoms) {
      cx = px;
      cy = py;
      cz = pz;
    } else {
      cx = sh.com[0];
      cy = sh.com[1];
      cz = sh.com[2];
    }
    cx = cx * L.inv_total_mass - L.site[0];
    cy = cy * L.inv_total_mass - L.site[1];
    cz = cz * L.inv_total_mass - L.site[2];
  };
  if (FORCES) {
    // restraint force -(m_i/M) k (d - d0) (c - c0)/d, before the barrier
    float fr = 0.f;
    if (wave_has_atoms) {
      com_offset();
      const float d = hsqrt(cx * cx + cy * cy + cz * cz);
      const float excess = d - L.d0;
      fr = excess > 0.f ? -L.krest * excess * rcp(d) * L.inv_total_mass
                        : 0.f;
      restraint_force(fr, m, cx, cy, cz, ge);
    }
    block_sync();
    if (owner) {
      // bonded forces: read and clear the atom's fixed-point accumulators
      // (the next evaluation adds into them only after its first barrier);
      // the copies' integer sum does not depend on which lane used which
      unsigned int s3[3] = {0u, 0u, 0u};
#pragma unroll
      for (int q = 0; q < kAccCopies; ++q) {
        lds_u32* a3 = sh.sl.acc + q * sh.sl.stride + 3 * tid;
        s3[0] += a3[0];
        s3[1] += a3[1];
        s3[2] += a3[2];
        a3[0] = 0u;
        a3[1] = 0u;
        a3[2] = 0u;
      }
      const float b[3] = {from_fix(s3[0]) + fpair[0],
                          from_fix(s3[1]) + fpair[1],
                          from_fix(s3[2]) + fpair[2]};
      f[0] = b[0] + ge[0];
      f[1] = b[1] + ge[1];
      f[2] = b[2] + ge[2];
      // the parts of the force that do not depend on the state weights
      if (cache_atom) {
        auto ca = BPMF_GMEM(float, cache_atom);
        ca[0] = b[0];
        ca[1] = b[1];
        ca[2] = b[2];
#pragma unroll
        for (int c = 0; c < C; ++c) {
          ca[3 + 3 * c] = de[c][0];
          ca[4 + 3 * c] = de[c][1];
          ca[5 + 3 * c] = de[c][2];
        }
      }
      if (cache_rep && tid == 0) {
        auto cr = BPMF_GMEM(float, cache_rep);
        cr[0] = fr;
        cr[1] = cx;
        cr[2] = cy;
        cr[3] = cz;
      }
    } else {
      f[0] = f[1] = f[2] = 0.f;
    }
  }
  if (ENERGY) {
    // per-wave sums in double, then a fixed-order sum over the waves.
    // LEAN: only the bonded total (in terms[0]) and the grid sums; the
    // extras are not reduced (their terms are 0)
    // a wavefront without bonded terms (or without atoms) contributes exact
    // zeros to those sums: it skips them (wave-uniform branches)
    const bool wave_bonded = (BONDED && sh.sched[wv + 1] > sh.sched[wv]) ||
                             (pairs && wave_has_atoms);
    double v[6 + C];
    v[0] = v[1] = v[2] = 0.0;
    if (wave_bonded) {
      if (LEAN) {
        v[0] = wave_sum((double)eb + (double)ea + (double)et +
                        (double)epair);
      } else {
        v[0] = wave_sum((double)eb + (double)epair);
        v[1] = wave_sum((double)ea);
        v[2] = wave_sum((double)et);
      }
    }
    v[3] = 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c)
      v[4 + c] = wave_has_atoms ? wave_sum((double)psi[c]) : 0.0;
    v[4 + C] = LEAN ? 0.0 : wave_sum((double)ex0);
    v[5 + C] = LEAN ? 0.0 : wave_sum((double)ex1);
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < 6 + C; ++q) sh.red[wv * kRedMax + q] = v[q];
    }
    block_sync();
    double acc[6 + C];
#pragma unroll
    for (int q = 0; q < 6 + C; ++q) acc[q] = 0.0;
    // TERMS0: the caller reads the terms in wavefront 0 only
    if (TERMS0 && wv != 0) {
#pragma unroll
      for (int q = 0; q < 6 + C; ++q) terms[q] = 0.0;
      return;
    }
    // waves one at a time: an unrolled loop would hold W x (6 + C)
    // doubles in registers at once
#pragma unroll 1
    for (int ww = 0; ww < W; ++ww) {
#pragma unroll
      for (int q = 0; q < 6 + C; ++q) acc[q] += sh.red[ww * kRedMax + q];
    }
#pragma unroll
    for (int q = 0; q < 6 + C; ++q) terms[q] = acc[q];
    // restraint energy: every thread from the published partials
    com_offset();
    const float d = sqrtf(cx * cx + cy * cy + cz * cz);
    const float excess = d - L.d0;
    terms[3] = excess > 0.f
                   ? 0.5 * (double)L.krest * (double)excess * (double)excess
                   : 0.0;
    // the next evaluation overwrites red[] and com[] only after at least
    // one more barrier
  }
  if (!FORCES && !ENERGY) block_sync();
}

}  // namespace bpmf
