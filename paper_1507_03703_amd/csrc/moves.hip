// External-coordinate Monte Carlo moves of the ligand (Sampling: external
// coordinate Markov chain Monte Carlo).  A move rotates the ligand rigidly
// about its centre of mass by the rotation of a random unit quaternion,
// translates it by sigma z (z standard normal per axis; the paper uses
// sigma = 0.6 A) and is accepted by the Metropolis criterion at the
// replica's state.  The proposal is symmetric (the rotation is uniform on
// SO(3), so a rotation and its inverse are equally likely, and so are t and
// -t), so no proposal-density ratio enters.
#include <hip/hip_runtime.h>
#include <math.h>

#include "device.h"
#include "internal.h"
#include "moves.h"

namespace bpmf {

namespace {

// One workgroup of W waves per (state k < k_max, ligand): the blocks of
// grid row y move ligand ligs[y] when it needs W waves (else they return),
// the replica in state k of it (the paper attempts the moves only where the
// grids are nearly off).  Move m of the call uses Philox draw 3m (three
// uniforms: the quaternion by Shoemake's construction), 3m + 1 (three
// normals: the translation) and 3m + 2 (the acceptance uniform), keyed by
// the ligand, the replica and the sweep counter.  The moves are a chain, but their
// random numbers are not: each batch of up to kBatch moves has its
// rotations, translations and ln u made first, one lane per move.
constexpr int kBatch = 64;
template <int C, int W>
__global__ __launch_bounds__(W * kWave) void k_external_move(
    GridDev g, const LigDev* __restrict__ ligs, int n_moves, int k_max,
    float sigma, uint64_t seed) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ float sRm[kBatch][9], stm[kBatch][3], sc0[3], st[3];
  __shared__ double s_lnu[kBatch];
  __shared__ double s_cp[4 * W];
  __shared__ double s_ui;  // restraint energy of the current pose
  __shared__ int s_acc;
  const LigDev L = ligs[blockIdx.y];
  const int tid = threadIdx.x;
  const int n = L.n;
  const int k = blockIdx.x;
  // uniform over the block: another launch's ligand, or no such state
  if ((n <= kWave ? 1 : 2) != W || k >= k_max || k >= L.K) return;
  const int r = L.replica_of_state[k];
  const unsigned long long s = *L.counter;
  Shared sh;
  {
    sh.pos = reinterpret_cast<float4*>(smem);
    sh.red = reinterpret_cast<double*>(smem + 16 * kWave * W);
    sh.com = reinterpret_cast<float*>(smem + 16 * kWave * W + 8 * W * kRedMax);
    const int acc0 = 16 * kWave * W + 8 * W * kRedMax + 16 * W;
    sh.sl = Slots{(lds_u32*)(smem + acc0), 0};  // no forces
    stage_topology(L, smem + acc0, sh, tid, W * kWave);
    __syncthreads();
  }
  const bool owner = tid < n;
  float x[3] = {0.f, 0.f, 0.f}, f[3];
  if (owner)
    for (int d = 0; d < 3; ++d) x[d] = L.x[(size_t)r * n * 3 + 3 * tid + d];
  const float m = owner ? L.mass[tid] : 0.f;
  float sc[C], w[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    sc[c] = owner ? L.scale[tid * C + c] : 0.f;
    w[c] = L.wf[k * C + c];
  }
  const double beta = L.beta[k];
  // energy and components of the current configuration (stored)
  double comp[1 + C];
  {
    const double* cp = L.comps + (size_t)r * (1 + C);
#pragma unroll
    for (int e = 0; e <= C; ++e) comp[e] = cp[e];
  }
  double e_cur = comp[0];
#pragma unroll
  for (int c = 0; c < C; ++c) e_cur += L.wd[k * C + c] * comp[1 + c];
  bool moved = false;
  for (int mv = 0; mv < n_moves; ++mv) {
    const int j = mv % kBatch;
    if (j == 0) {
      // this batch's rotations, translations and ln u (the previous
      // batch's last reader passed the barrier that ended its move)
      const int b = mv + tid;
      if (tid < kBatch && b < n_moves) {
        // uniform unit quaternion (w, x, y, z) from three uniforms
        const U4 o = draw(seed, 3u * b, L.id, r, s, kExternal);
        const double u1 = u01d(o.x), u2 = u01d(o.y), u3 = u01d(o.z);
        const double a = sqrt(1.0 - u1), bb = sqrt(u1);
        double s2, c2, s3, c3;
        sincos(2.0 * M_PI * u2, &s2, &c2);
        sincos(2.0 * M_PI * u3, &s3, &c3);
        const double qw = bb * c3, qx = a * s2, qy = a * c2, qz = bb * s3;
        const double R[9] = {1 - 2 * (qy * qy + qz * qz),
                             2 * (qx * qy - qz * qw), 2 * (qx * qz + qy * qw),
                             2 * (qx * qy + qz * qw),
                             1 - 2 * (qx * qx + qz * qz),
                             2 * (qy * qz - qx * qw), 2 * (qx * qz - qy * qw),
                             2 * (qy * qz + qx * qw),
                             1 - 2 * (qx * qx + qy * qy)};
        for (int e = 0; e < 9; ++e) sRm[tid][e] = (float)R[e];
        float z[3];
        normals3(draw(seed, 3u * b + 1u, L.id, r, s, kExternal), z[0], z[1],
                 z[2]);
        for (int d = 0; d < 3; ++d) stm[tid][d] = sigma * z[d];
        s_lnu[tid] =
            log(u01d(draw(seed, 3u * b + 2u, L.id, r, s, kExternal).x));
      }
    }
    // centre of mass in double (fixed-order: wave sums, then waves)
    {
      const double mi = (double)m;
      const double cx = wave_sum(mi * x[0]), cy = wave_sum(mi * x[1]);
      const double cz = wave_sum(mi * x[2]), cm = wave_sum(mi);
      if ((tid & (kWave - 1)) == 0) {
        const int wv = tid >> 6;
        s_cp[4 * wv] = cx;
        s_cp[4 * wv + 1] = cy;
        s_cp[4 * wv + 2] = cz;
        s_cp[4 * wv + 3] = cm;
      }
    }
    __syncthreads();
    if (tid == 0) {
      double c[3] = {0.0, 0.0, 0.0}, M = 0.0;
      for (int q = 0; q < W; ++q) {
        for (int d = 0; d < 3; ++d) c[d] += s_cp[4 * q + d];
        M += s_cp[4 * q + 3];
      }
      double d2 = 0.0;
      for (int d = 0; d < 3; ++d) {
        c[d] /= M;
        sc0[d] = (float)c[d];
        st[d] = (float)(c[d] + (double)stm[j][d]);
        d2 += (c[d] - (double)L.site[d]) * (c[d] - (double)L.site[d]);
      }
      // restraint energy at the current centre of mass (Eq. binding_site)
      const double ex = sqrt(d2) - (double)L.d0;
      s_ui = ex > 0.0 ? 0.5 * (double)L.krest * ex * ex : 0.0;
    }
    __syncthreads();
    const float* sR = sRm[j];
    // x' = c + sigma z + R (x - c)
    float xn[3] = {0.f, 0.f, 0.f};
    if (owner) {
      const float y[3] = {x[0] - sc0[0], x[1] - sc0[1], x[2] - sc0[2]};
      for (int a = 0; a < 3; ++a)
        xn[a] = st[a] + sR[3 * a] * y[0] + sR[3 * a + 1] * y[1] +
                sR[3 * a + 2] * y[2];
    }
    // the move is rigid: the bonded (and pair) energy is the cached one, the
    // stored first component less the restraint energy of the current
    // centre of mass; only the grid terms and the restraint are evaluated
    double t[6 + C];
    eval_block<C, W, false, true, true, false>(g, L, w, xn, m, sc, f, t, 0.f,
                                               0.f, sh, tid);
    const double u0 = (comp[0] - s_ui) + t[3];
    double e_new = u0;
#pragma unroll
    for (int c = 0; c < C; ++c) e_new += L.wd[k * C + c] * t[4 + c];
    if (tid == 0) {
      const double ln_a = -beta * (e_new - e_cur);
      s_acc = (isfinite(ln_a) && s_lnu[j] < ln_a) ? 1 : 0;
      atomicAdd(&L.ext_try[k], 1ull);
      if (s_acc) atomicAdd(&L.ext_acc[k], 1ull);
    }
    __syncthreads();
    if (s_acc) {
      for (int d = 0; d < 3; ++d) x[d] = xn[d];
      e_cur = e_new;
      comp[0] = u0;
#pragma unroll
      for (int c = 0; c < C; ++c) comp[1 + c] = t[4 + c];
      moved = true;
    }
  }
  if (moved) {
    if (owner)
      for (int d = 0; d < 3; ++d) L.x[(size_t)r * n * 3 + 3 * tid + d] = x[d];
    if (tid == 0) {
      double* cw = L.comps + (size_t)r * (1 + C);
#pragma unroll
      for (int e = 0; e <= C; ++e) cw[e] = comp[e];
      L.fvalid[r] = 0;  // the stored start-of-trajectory forces are stale
    }
  }
}

template <int C>
hipError_t launch_c(const GridDev& g, const LigDev* ligs, int n_lig, int kg,
                    int waves, int n_moves, int k_max, float sigma, int lds,
                    uint64_t seed, hipStream_t st) {
  const dim3 grid(kg, n_lig);
  if (waves == 1)
    hipLaunchKernelGGL((k_external_move<C, 1>), grid, dim3(kWave), lds, st, g,
                       ligs, n_moves, k_max, sigma, seed);
  else if (waves == 2)
    hipLaunchKernelGGL((k_external_move<C, 2>), grid, dim3(2 * kWave), lds,
                       st, g, ligs, n_moves, k_max, sigma, seed);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace

hipError_t launch_external_moves(const GridDev& g, const LigDev* ligs,
                                 int n_lig, int k_grid, int waves, int n_moves,
                                 int k_max, float sigma, int lds,
                                 uint64_t seed, hipStream_t st) {
  if (n_lig <= 0 || k_grid <= 0 || n_moves <= 0 || k_max <= 0)
    return hipSuccess;
  if (n_lig > 65535) return hipErrorInvalidValue;
  switch (g.C) {
    case 3:
      return launch_c<3>(g, ligs, n_lig, k_grid, waves, n_moves, k_max, sigma,
                         lds, seed, st);
    case 5:
      return launch_c<5>(g, ligs, n_lig, k_grid, waves, n_moves, k_max, sigma,
                         lds, seed, st);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace bpmf

// ----------------------------------------------------------------------------
// Random placements in the binding site (Initialization: configurations put
// at random centre-of-mass positions in the site, each with random
// orientations).  Site position i: radius d0 u^(1/3), cos(theta) = 2u - 1,
// phi = 2 pi u about the site centre; orientation o: the rotation of a
// uniform unit quaternion, applied about the configuration's centre of mass.
// ----------------------------------------------------------------------------
#include "protocol.h"

namespace bpmf {

namespace {

// centre of mass of each configuration, in double
__global__ __launch_bounds__(64) void k_conf_com(const LigDev* __restrict__ lig,
                                                 const float* __restrict__ confs,
                                                 int n_conf, double* com) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_conf) return;
  const LigDev& L = *lig;
  const int n = L.n;
  double sx = 0, sy = 0, sz = 0, sm = 0;
  for (int a = 0; a < n; ++a) {
    const double m = L.mass[a];
    const float* p = confs + ((size_t)c * n + a) * 3;
    sx += m * p[0];
    sy += m * p[1];
    sz += m * p[2];
    sm += m;
  }
  com[3 * c] = sx / sm;
  com[3 * c + 1] = sy / sm;
  com[3 * c + 2] = sz / sm;
}

// one thread per (pose, atom)
__global__ __launch_bounds__(256) void k_place_poses(
    const LigDev* __restrict__ lig, const float* __restrict__ confs,
    const double* __restrict__ com, int n_com, int n_orient, int64_t first,
    int64_t total, uint64_t seed, float* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const LigDev& L = *lig;
  const int n = L.n;
  const int64_t q = t / n;
  const int a = (int)(t - q * n);
  const int64_t p = first + q;
  const int o = (int)(p % n_orient);
  const int64_t ci = p / n_orient;
  const int i = (int)(ci % n_com);
  const int c = (int)(ci / n_com);
  // site position i
  const U4 up = draw(seed, (uint32_t)i, L.id, 0, 0, kInit | (kSubCom << 8));
  const double r = (double)L.d0 * cbrt(u01d(up.x));
  const double ct = 2.0 * u01d(up.y) - 1.0;
  const double stt = sqrt(fmax(0.0, 1.0 - ct * ct));
  double sp, cp;
  sincos(2.0 * M_PI * u01d(up.z), &sp, &cp);
  const double tx = (double)L.site[0] + r * stt * cp;
  const double ty = (double)L.site[1] + r * stt * sp;
  const double tz = (double)L.site[2] + r * ct;
  // orientation o: uniform unit quaternion (w, x, y, z) from three uniforms
  const U4 uo = draw(seed, (uint32_t)o, L.id, 0, 0, kInit | (kSubOrient << 8));
  const double u1 = u01d(uo.x), u2 = u01d(uo.y), u3 = u01d(uo.z);
  const double qa = sqrt(1.0 - u1), qb = sqrt(u1);
  double s2, c2, s3, c3;
  sincos(2.0 * M_PI * u2, &s2, &c2);
  sincos(2.0 * M_PI * u3, &s3, &c3);
  const double qw = qb * c3, qx = qa * s2, qy = qa * c2, qz = qb * s3;
  const float* src = confs + ((size_t)c * n + a) * 3;
  const double dx = src[0] - com[3 * c], dy = src[1] - com[3 * c + 1],
               dz = src[2] - com[3 * c + 2];
  float* dst = out + t * 3;
  dst[0] = (float)(tx + (1 - 2 * (qy * qy + qz * qz)) * dx +
                   2 * (qx * qy - qz * qw) * dy + 2 * (qx * qz + qy * qw) * dz);
  dst[1] = (float)(ty + 2 * (qx * qy + qz * qw) * dx +
                   (1 - 2 * (qx * qx + qz * qz)) * dy +
                   2 * (qy * qz - qx * qw) * dz);
  dst[2] = (float)(tz + 2 * (qx * qz - qy * qw) * dx +
                   2 * (qy * qz + qx * qw) * dy +
                   (1 - 2 * (qx * qx + qy * qy)) * dz);
}

}  // namespace

hipError_t launch_place_poses(const LigDev* lig, int n, const float* confs,
                              int n_conf, int n_com, int n_orient,
                              int64_t first, int64_t count, double* com,
                              uint64_t seed, float* out, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_conf_com, dim3((n_conf + 63) / 64), dim3(64), 0, st,
                     lig, confs, n_conf, com);
  const int64_t total = count * n;
  const int64_t blocks = (total + 255) / 256;
  if (blocks > (1ll << 24) - 1) return hipErrorInvalidValue;  // 2^32 threads
  hipLaunchKernelGGL(k_place_poses, dim3((unsigned)blocks), dim3(256), 0, st,
                     lig, confs, com, n_com, n_orient, first, total, seed,
                     out);
  return hipGetLastError();
}

}  // namespace bpmf
