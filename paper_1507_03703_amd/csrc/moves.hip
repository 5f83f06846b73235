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
// the ligand, the replica and the sweep counter.
//
// The moves form a chain, but a candidate's position does not depend on
// any energy: the candidates of the next kSpec moves, each made from the
// one before as if that one were accepted, are built first and their grid
// energies evaluated together (their gathers in flight at once); the
// Metropolis decisions then run in order, and the round ends at the first
// rejection (the later candidates were made from a configuration the chain
// does not reach and are dropped).  The accepted chain is the sequential
// one.  A move is rigid: the bonded (and pair) energy keeps its cached
// value, the centre of mass moves by the translation (rotation is about
// it), so only the grid terms and the restraint change.  The centre of mass
// is summed from the positions at the start of every round and carried in
// double within it.
constexpr int kBatch = 64;  // moves whose random numbers are made at once
constexpr int kSpec = 4;    // candidates per round
template <int C, int W>
__global__ __launch_bounds__(W * kWave) void k_external_move(
    GridDev g, const LigDev* __restrict__ ligs, int n_moves, int k_max,
    float sigma, uint64_t seed) {
  __shared__ float sRm[kBatch][9], stm[kBatch][3];
  __shared__ double s_lnu[kBatch];
  __shared__ double s_red[2][W][kSpec + 4];
  const LigDev L = ligs[blockIdx.y];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1), wv = tid >> 6;
  const int n = L.n;
  const int k = blockIdx.x;
  // uniform over the block: another launch's ligand, or no such state
  if ((n <= kWave ? 1 : 2) != W || k >= k_max || k >= L.K) return;
  const int r = L.replica_of_state[k];
  const unsigned long long s = *L.counter;
  const bool owner = tid < n;
  float x[3] = {0.f, 0.f, 0.f};
  if (owner)
    for (int d = 0; d < 3; ++d) x[d] = L.x[(size_t)r * n * 3 + 3 * tid + d];
  const double m = owner ? (double)L.mass[tid] : 0.0;
  float sc[C];
  double wd[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    sc[c] = owner ? L.scale[tid * C + c] : 0.f;
    wd[c] = L.wd[k * C + c];
  }
  const double beta = L.beta[k];
  const double site[3] = {(double)L.site[0], (double)L.site[1],
                          (double)L.site[2]};
  const double d0 = (double)L.d0, krest = (double)L.krest;
  // restraint energy at centre of mass c (Eq. binding_site)
  auto restraint = [&](const double* c) {
    double d2 = 0.0;
    for (int d = 0; d < 3; ++d) d2 += (c[d] - site[d]) * (c[d] - site[d]);
    const double ex = sqrt(d2) - d0;
    return ex > 0.0 ? 0.5 * krest * ex * ex : 0.0;
  };
  // stored components of the current configuration and its energy
  double comp[1 + C];
  {
    const double* cp = L.comps + (size_t)r * (1 + C);
#pragma unroll
    for (int e = 0; e <= C; ++e) comp[e] = cp[e];
  }
  double e_cur = comp[0];
#pragma unroll
  for (int c = 0; c < C; ++c) e_cur += wd[c] * comp[1 + c];
  // grid values of this lane's atom in the current configuration (filled
  // at the first acceptance; the stored channel sums hold until then)
  float psi[C];
#pragma unroll
  for (int c = 0; c < C; ++c) psi[c] = 0.f;
  bool moved = false;
  int batch0 = 0, batch1 = 0;  // moves whose random numbers are in LDS
  int round = 0;
  for (int mv = 0; mv < n_moves; ++round) {
    if (mv + kSpec > batch1 && batch1 < n_moves) {
      // random numbers of moves [mv, mv + kBatch), once every wave has
      // taken the previous round's decisions from the old batch
      __syncthreads();
      batch0 = mv;
      batch1 = mv + kBatch;
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
      __syncthreads();
    }
    const int nd = min(kSpec, n_moves - mv);
    // centre of mass of the current configuration, in double (fixed
    // order: wave sums, then the waves in order); the round's partial slots
    // alternate, so a wave one round ahead never overwrites what another
    // still reads
    double (*red)[kSpec + 4] = s_red[round & 1];
    {
      const double cx = wave_sum(m * x[0]), cy = wave_sum(m * x[1]);
      const double cz = wave_sum(m * x[2]), cm = wave_sum(m);
      if (lane == 0) {
        red[wv][kSpec] = cx;
        red[wv][kSpec + 1] = cy;
        red[wv][kSpec + 2] = cz;
        red[wv][kSpec + 3] = cm;
      }
    }
    __syncthreads();
    double c0[3] = {0.0, 0.0, 0.0}, M = 0.0;
    for (int q = 0; q < W; ++q) {
      for (int d = 0; d < 3; ++d) c0[d] += red[q][kSpec + d];
      M += red[q][kSpec + 3];
    }
    for (int d = 0; d < 3; ++d) c0[d] /= M;
    // candidates: y_j = c_j + t_j + R_j (y_{j-1} - c_j), c_j the centre of
    // mass of y_{j-1} (c_0 of the current configuration, then carried).
    // Every step below runs for all kSpec candidates without branches, so
    // that the independent candidates interleave; those past the call's
    // last move (j >= nd) repeat its random numbers and are never accepted.
    float y[kSpec][3];
    double cj[kSpec][3];
    {
      double c[3] = {c0[0], c0[1], c0[2]};
      float p[3] = {x[0], x[1], x[2]};
#pragma unroll
      for (int j = 0; j < kSpec; ++j) {
        const int q = min(j, nd - 1) + mv - batch0;
        const float* R = sRm[q];
        float cf[3], tf[3];
        for (int d = 0; d < 3; ++d) {
          cf[d] = (float)c[d];
          tf[d] = (float)(c[d] + (double)stm[q][d]);
          c[d] += (double)stm[q][d];
        }
        const float u[3] = {p[0] - cf[0], p[1] - cf[1], p[2] - cf[2]};
        for (int a = 0; a < 3; ++a)
          p[a] = tf[a] + R[3 * a] * u[0] + R[3 * a + 1] * u[1] +
                 R[3 * a + 2] * u[2];
        for (int d = 0; d < 3; ++d) {
          y[j][d] = p[d];
          cj[j][d] = c[d];
        }
      }
    }
    // grid energies of every candidate: the gathers first (the restraint
    // energies are computed while they fly), then the interpolation; per
    // atom the weighted sum over channels
    Corners<C> cn[kSpec];
#pragma unroll
    for (int j = 0; j < kSpec; ++j)
      grid_fetch<C>(g, y[j][0], y[j][1], y[j][2], cn[j]);
    double ui[kSpec];
#pragma unroll
    for (int j = 0; j < kSpec; ++j) ui[j] = restraint(cj[j]);
    const double base = comp[0] - restraint(c0);
    float pj[kSpec][C];
    double gj[kSpec];
#pragma unroll
    for (int j = 0; j < kSpec; ++j) {
      grid_finish<C, false>(g, cn[j], sc, pj[j], nullptr);
      gj[j] = 0.0;
#pragma unroll
      for (int c = 0; c < C; ++c) gj[j] += wd[c] * (double)pj[j][c];
    }
#pragma unroll
    for (int j = 0; j < kSpec; ++j) gj[j] = wave_sum(gj[j]);
    if (lane == 0)
#pragma unroll
      for (int j = 0; j < kSpec; ++j) red[wv][j] = gj[j];
    __syncthreads();
    // the decisions in order, by every thread from the same sums: move j
    // is accepted when every earlier one of the round was and its own test
    // passes against the energy of candidate j - 1
    double e_new[kSpec];
#pragma unroll
    for (int j = 0; j < kSpec; ++j) {
      double G = 0.0;
      for (int q = 0; q < W; ++q) G += red[q][j];
      e_new[j] = (base + ui[j]) + G;
    }
    int acc = 0;
    bool go = true;
#pragma unroll
    for (int j = 0; j < kSpec; ++j) {
      const double ln_a = -beta * (e_new[j] - (j ? e_new[j - 1] : e_cur));
      const double lnu = s_lnu[min(j, nd - 1) + mv - batch0];
      go = go && j < nd && isfinite(ln_a) && lnu < ln_a;
      acc += go ? 1 : 0;
    }
    double e_acc = e_cur, u_acc = comp[0];
#pragma unroll
    for (int j = 0; j < kSpec; ++j)
      if (j == acc - 1) {
        e_acc = e_new[j];
        u_acc = base + ui[j];
      }
    const int used = acc < nd ? acc + 1 : nd;
    if (tid == 0) {
      atomicAdd(&L.ext_try[k], (unsigned long long)used);
      if (acc) atomicAdd(&L.ext_acc[k], (unsigned long long)acc);
    }
    if (acc > 0) {
#pragma unroll
      for (int j = 0; j < kSpec; ++j)
        if (j == acc - 1) {
          for (int d = 0; d < 3; ++d) x[d] = y[j][d];
#pragma unroll
          for (int c = 0; c < C; ++c) psi[c] = pj[j][c];
        }
      e_cur = e_acc;
      comp[0] = u_acc;
      moved = true;
    }
    mv += used;
  }
  if (moved) {
    // channel sums of the final configuration, in the slots the last round
    // did not use (their readers, two rounds back, are done)
    double (*red)[kSpec + 4] = s_red[round & 1];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const double v = wave_sum((double)psi[c]);
      if (lane == 0) red[wv][c] = v;
    }
    __syncthreads();
    if (owner)
      for (int d = 0; d < 3; ++d) L.x[(size_t)r * n * 3 + 3 * tid + d] = x[d];
    if (tid == 0) {
      double* cw = L.comps + (size_t)r * (1 + C);
      cw[0] = comp[0];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        double v = 0.0;
        for (int q = 0; q < W; ++q) v += red[q][c];
        cw[1 + c] = v;
      }
      L.fvalid[r] = 0;  // the stored start-of-trajectory forces are stale
    }
  }
}

template <int C>
hipError_t launch_c(const GridDev& g, const LigDev* ligs, int n_lig, int kg,
                    int waves, int n_moves, int k_max, float sigma,
                    uint64_t seed, hipStream_t st) {
  const dim3 grid(kg, n_lig);
  if (waves == 1)
    hipLaunchKernelGGL((k_external_move<C, 1>), grid, dim3(kWave), 0, st, g,
                       ligs, n_moves, k_max, sigma, seed);
  else if (waves == 2)
    hipLaunchKernelGGL((k_external_move<C, 2>), grid, dim3(2 * kWave), 0, st,
                       g, ligs, n_moves, k_max, sigma, seed);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace

hipError_t launch_external_moves(const GridDev& g, const LigDev* ligs,
                                 int n_lig, int k_grid, int waves, int n_moves,
                                 int k_max, float sigma, uint64_t seed,
                                 hipStream_t st) {
  if (n_lig <= 0 || k_grid <= 0 || n_moves <= 0 || k_max <= 0)
    return hipSuccess;
  if (n_lig > 65535) return hipErrorInvalidValue;
  switch (g.C) {
    case 3:
      return launch_c<3>(g, ligs, n_lig, k_grid, waves, n_moves, k_max, sigma,
                         seed, st);
    case 5:
      return launch_c<5>(g, ligs, n_lig, k_grid, waves, n_moves, k_max, sigma,
                         seed, st);
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
