// MBAR on the device in double precision (Shirts & Chodera 2008; the paper
// estimates f_BC,L and f_CD' with it, Methodology "Estimation").
//
// The free energies minimise the convex function
//   F(f) = sum_n ln sum_k N_k exp(f_k - u_kn) - sum_i N_i f_i,   f_0 = 0,
// whose gradient is g_i = N_i (sum_n W_ni - 1) and Hessian
//   H_ij = N_i delta_ij sum_n W_ni - N_i N_j sum_n W_ni W_nj,
// W_ni = exp(f_i - u_in) / sum_k N_k exp(f_k - u_kn).  Newton steps solve the
// gauge-fixed system; var(f_k - f_0) = (H~^-1)_kk - 1/N_k - 1/N_0.
//
// Every kernel serves a list of independent problems (one per ligand):
// blockIdx.y picks the problem, and each problem keeps its own block count
// for every grid-wide loop, so a problem's arithmetic -- and its result --
// is the same whether it is solved alone or in a batch.  All reductions run
// over a fixed block grid in a fixed order, so results do not depend on
// scheduling either.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "internal.h"

namespace bpmf {

namespace {

constexpr int kT = 256;

__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_max(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ const MbarProb& prob(const MbarProb* P,
                                                const int* list) {
  return P[list[blockIdx.y]];
}

// logD_n = ln sum_k exp(logN_k + f_k - u_kn) at f (or ftry); obj_part[b] =
// sum over block b's samples of logD_n (p.nb blocks per problem)
__global__ __launch_bounds__(kT) void k_logD(const MbarProb* __restrict__ P,
                                             const int* __restrict__ list,
                                             int use_try) {
  const MbarProb& p = prob(P, list);
  if ((int)blockIdx.x >= p.nb) return;
  __shared__ double a[BPMF_MAX_MBAR_STATES_DEV];
  __shared__ double red[kT];
  const int K = p.K;
  const int64_t N = p.N, ld = p.ld;
  const double* __restrict__ ukn = p.ukn;
  const double* f = use_try ? p.ftry : p.f;
  for (int k = threadIdx.x; k < K; k += blockDim.x) a[k] = p.logN[k] + f[k];
  __syncthreads();
  double acc = 0.0;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
       n += (int64_t)p.nb * blockDim.x) {
    double m = -INFINITY;
    for (int k = 0; k < K; ++k) m = fmax(m, a[k] - ukn[(size_t)k * ld + n]);
    double s = 0.0;
    for (int k = 0; k < K; ++k) s += exp(a[k] - ukn[(size_t)k * ld + n] - m);
    const double v = m + log(s);
    p.logD[n] = v;
    acc += v;
  }
  const double b = block_sum(acc, red);
  if (threadIdx.x == 0) p.obj_part[blockIdx.x] = b;
}

// scalars[0] = sum_b obj_part[b] - sum_k N_k f_k (one block per problem)
__global__ __launch_bounds__(kT) void k_objective(
    const MbarProb* __restrict__ P, const int* __restrict__ list,
    int use_try) {
  const MbarProb& p = prob(P, list);
  __shared__ double red[kT];
  const double* f = use_try ? p.ftry : p.f;
  double acc = 0.0;
  for (int b = threadIdx.x; b < p.nb; b += blockDim.x) acc += p.obj_part[b];
  const double s1 = block_sum(acc, red);
  acc = 0.0;
  for (int k = threadIdx.x; k < p.K; k += blockDim.x) acc += p.Nk[k] * f[k];
  const double s2 = block_sum(acc, red);
  if (threadIdx.x == 0) p.scalars[0] = s1 - s2;
}

// self-consistent update step_i = -ln sum_n exp(-u_in - logD_n), one block
// per state (logD current for f)
__global__ __launch_bounds__(kT) void k_self_consistent(
    const MbarProb* __restrict__ P, const int* __restrict__ list) {
  const MbarProb& p = prob(P, list);
  const int i = blockIdx.x;
  if (i >= p.K) return;
  __shared__ double red[kT];
  const int64_t N = p.N;
  const double* __restrict__ row = p.ukn + (size_t)i * p.ld;
  double m = -INFINITY;
  for (int64_t n = threadIdx.x; n < N; n += blockDim.x)
    m = fmax(m, -row[n] - p.logD[n]);
  const double M = block_max(m, red);
  double acc = 0.0;
  for (int64_t n = threadIdx.x; n < N; n += blockDim.x)
    acc += exp(-row[n] - p.logD[n] - M);
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) p.step[i] = -(M + log(s));
}

// gauge shift f = step - step_0 of the fixed-point update, with
// scalars[4] = max_k |f_new - f_old|
__global__ __launch_bounds__(kT) void k_gauge(const MbarProb* __restrict__ P,
                                              const int* __restrict__ list) {
  const MbarProb& p = prob(P, list);
  __shared__ double red[kT];
  double ch = 0.0;
  for (int k = threadIdx.x; k < p.K; k += blockDim.x) {
    const double v = p.step[k] - p.step[0];
    ch = fmax(ch, fabs(v - p.f[k]));
    p.f[k] = v;
  }
  const double c = block_max(ch, red);
  if (threadIdx.x == 0) p.scalars[4] = c;
}

// partial[b] = [colsum_i (K) | M_ij (K*K)] over the block's sample chunks,
// M = W W^T with W_in = exp(f_i - u_in - logD_n).  A chunk of W sits in LDS
// sample-major, row stride Kp + 2 doubles (16-byte aligned rows, staggered
// banks); the 256 threads form a 16 x 16 grid of TS x TS register tiles of
// M (Kp = 16 TS >= K, rows and columns past K are zero).  Every problem of
// the launch has this TS; it uses p.nb_acc blocks.
template <int TS>
__global__ __launch_bounds__(kT) void k_accumulate(
    const MbarProb* __restrict__ P, const int* __restrict__ list) {
  constexpr int Kp = 16 * TS, RS = Kp + 2;
  constexpr int chunk = 4096 / Kp;
  const MbarProb& p = prob(P, list);
  if ((int)blockIdx.x >= p.nb_acc) return;
  extern __shared__ __align__(16) double W[];  // chunk x RS
  __shared__ double fk[Kp];
  const int K = p.K;
  const int64_t N = p.N, ld = p.ld;
  const double* __restrict__ ukn = p.ukn;
  const double* __restrict__ logD = p.logD;
  const int tid = threadIdx.x;
  const int ta = tid >> 4, tb = tid & 15;
  for (int k = tid; k < Kp; k += kT) fk[k] = k < K ? p.f[k] : 0.0;
  double acc[TS][TS];
#pragma unroll
  for (int i = 0; i < TS; ++i)
#pragma unroll
    for (int j = 0; j < TS; ++j) acc[i][j] = 0.0;
  double col = 0.0;
  const int64_t n_chunks = (N + chunk - 1) / chunk;
  for (int64_t ch = blockIdx.x; ch < n_chunks; ch += p.nb_acc) {
    const int64_t n0 = ch * chunk;
    const int cnt = (int)((N - n0) < chunk ? (N - n0) : chunk);
    __syncthreads();
    // fill: consecutive threads take consecutive samples of one state
    for (int e = tid; e < Kp * chunk; e += kT) {
      const int k = e / chunk, t = e - k * chunk;
      double v = 0.0;
      if (k < K && t < cnt)
        v = exp(fk[k] - ukn[(size_t)k * ld + n0 + t] - logD[n0 + t]);
      W[t * RS + k] = v;
    }
    __syncthreads();
    if (tid < Kp)
      for (int t = 0; t < cnt; ++t) col += W[t * RS + tid];
    for (int t = 0; t < cnt; ++t) {
      const double* row = W + t * RS;
      double wi[TS], wj[TS];
#pragma unroll
      for (int i = 0; i < TS; ++i) wi[i] = row[ta * TS + i];
#pragma unroll
      for (int j = 0; j < TS; ++j) wj[j] = row[tb * TS + j];
#pragma unroll
      for (int i = 0; i < TS; ++i)
#pragma unroll
        for (int j = 0; j < TS; ++j) acc[i][j] = fma(wi[i], wj[j], acc[i][j]);
    }
  }
  const int KK = K * K;
  double* out = p.partial + (size_t)blockIdx.x * (K + KK);
  if (tid < K) out[tid] = col;
#pragma unroll
  for (int i = 0; i < TS; ++i)
#pragma unroll
    for (int j = 0; j < TS; ++j) {
      const int r = ta * TS + i, c = tb * TS + j;
      if (r < K && c < K) out[K + r * K + c] = acc[i][j];
    }
}

// red[e] = sum over blocks of partial[b][e], in block order (small blocks:
// many of them keep enough loads in flight)
constexpr int kRedT = 64;
__global__ __launch_bounds__(kRedT) void k_reduce_partials(
    const MbarProb* __restrict__ P, const int* __restrict__ list) {
  const MbarProb& p = prob(P, list);
  const int width = p.K + p.K * p.K;
  const int e = blockIdx.x * kRedT + threadIdx.x;
  if (e >= width) return;
  const double* __restrict__ part = p.partial;
  const int nb = p.nb_acc;
  double s = 0.0;
#pragma unroll 16
  for (int b = 0; b < nb; ++b) s += part[(size_t)b * width + e];
  p.red[e] = s;
}

// Newton step (one block per problem): from the reduced sums build the
// gauge-fixed system [H~ | -g~ (| I)], Gauss-Jordan eliminate it (H~ is
// symmetric positive definite), write step, max|step|, g.step and, on
// request, var(f_k - f_0).  The system lives in LDS (dynamic) when every
// problem's fits, else in each problem's global `mat`.
constexpr int kNewtonT = 256;
template <bool LDS>
__global__ __launch_bounds__(kNewtonT) void k_newton(
    const MbarProb* __restrict__ P, const int* __restrict__ list,
    int want_inverse) {
  const MbarProb& p = prob(P, list);
  extern __shared__ __align__(16) double lmat[];
  double* mat = LDS ? lmat : p.mat;
  __shared__ double fac[BPMF_MAX_MBAR_STATES_DEV];
  __shared__ double gsh[BPMF_MAX_MBAR_STATES_DEV];
  __shared__ double piv_sh, dmax_sh;
  __shared__ int bad;
  const int K = p.K;
  const double* __restrict__ red = p.red;
  const double* __restrict__ Nk = p.Nk;
  if (threadIdx.x == 0) bad = 0;
  const int m = K - 1;
  const int wcols = m + 1 + (want_inverse ? m : 0);
  for (int k = threadIdx.x; k < K; k += blockDim.x)
    gsh[k] = Nk[k] * (red[k] - 1.0);
  __syncthreads();
  for (int e = threadIdx.x; e < m * wcols; e += blockDim.x) {
    const int r = e / wcols, c = e - r * wcols;
    const int i = r + 1;
    double v;
    if (c < m) {
      const int j = c + 1;
      v = -Nk[i] * Nk[j] * red[K + i * K + j];
      if (i == j) v += Nk[i] * red[i];
    } else if (c == m) {
      v = -gsh[i];
    } else {
      v = (c - m - 1 == r) ? 1.0 : 0.0;
    }
    mat[e] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double dm = 0.0;
    for (int q = 0; q < m; ++q) dm = fmax(dm, mat[(size_t)q * wcols + q]);
    dmax_sh = dm;
  }
  __syncthreads();
  // a pivot below 1e-13 of the largest diagonal entry marks the system as
  // not numerically positive definite (the caller then takes a fixed-point
  // step instead)
  const double pmin = 1e-13 * dmax_sh;
  for (int q = 0; q < m; ++q) {
    if (threadIdx.x == 0) {
      piv_sh = mat[(size_t)q * wcols + q];
      if (!(piv_sh > pmin)) bad = 1;
    }
    __syncthreads();
    const double piv = piv_sh;
    for (int c = threadIdx.x; c < wcols; c += blockDim.x)
      mat[(size_t)q * wcols + c] /= piv;
    for (int r = threadIdx.x; r < m; r += blockDim.x)
      fac[r] = mat[(size_t)r * wcols + q];
    __syncthreads();
    for (int e = threadIdx.x; e < m * wcols; e += blockDim.x) {
      const int r = e / wcols, c = e - r * wcols;
      if (r != q) mat[e] -= fac[r] * mat[(size_t)q * wcols + c];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double mx = 0.0, gs = 0.0;
    p.step[0] = 0.0;
    for (int i = 1; i < K; ++i) {
      const double s = mat[(size_t)(i - 1) * wcols + m];
      p.step[i] = s;
      mx = fmax(mx, fabs(s));
      gs += gsh[i] * s;
    }
    p.scalars[1] = mx;
    p.scalars[2] = gs;
    p.scalars[3] = bad ? 1.0 : 0.0;
    if (want_inverse) {
      p.var[0] = 0.0;
      for (int i = 1; i < K; ++i)
        p.var[i] = mat[(size_t)(i - 1) * wcols + m + 1 + (i - 1)] -
                   1.0 / Nk[i] - 1.0 / Nk[0];
    }
  }
}

// line-search trial ftry = f + t * step, t = tvec[problem]
__global__ __launch_bounds__(kT) void k_axpy(const MbarProb* __restrict__ P,
                                             const int* __restrict__ list,
                                             const double* __restrict__ tvec) {
  const MbarProb& p = prob(P, list);
  const double t = tvec[list[blockIdx.y]];
  for (int k = threadIdx.x; k < p.K; k += blockDim.x)
    p.ftry[k] = p.f[k] + t * p.step[k];
}

// an accepted trial becomes the current point: f = ftry
__global__ __launch_bounds__(kT) void k_accept(const MbarProb* __restrict__ P,
                                               const int* __restrict__ list) {
  const MbarProb& p = prob(P, list);
  for (int k = threadIdx.x; k < p.K; k += blockDim.x) p.f[k] = p.ftry[k];
}

template <int TS>
hipError_t accumulate_ts(const MbarProb* P, const int* list, int n,
                         int max_blocks, hipStream_t st) {
  const size_t lds = (size_t)(4096 / (16 * TS)) * (16 * TS + 2) *
                     sizeof(double);
  hipLaunchKernelGGL(k_accumulate<TS>, dim3(max_blocks, n), dim3(kT), lds, st,
                     P, list);
  return hipGetLastError();
}

}  // namespace

int mbar_logD_blocks(int64_t N) {
  return (int)std::min<int64_t>(256, std::max<int64_t>(1, (N + 255) / 256));
}

int mbar_acc_ts(int K) { return K <= 16 ? 1 : K <= 32 ? 2 : K <= 64 ? 4 : 8; }

int mbar_acc_blocks(int K, int64_t N) {
  const int chunk = 4096 / (16 * mbar_acc_ts(K));
  const int64_t chunks = (N + chunk - 1) / chunk;
  return (int)(chunks < 256 ? chunks : 256);
}

size_t mbar_newton_lds(int K, int want_inverse) {
  const size_t m = K - 1;
  return m * (m + 1 + (want_inverse ? m : 0)) * sizeof(double);
}

hipError_t mbar_objective(const MbarProb* P, const int* list, int n,
                          int max_nb, int use_try, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_logD, dim3(max_nb, n), dim3(kT), 0, st, P, list,
                     use_try);
  hipLaunchKernelGGL(k_objective, dim3(1, n), dim3(kT), 0, st, P, list,
                     use_try);
  return hipGetLastError();
}

hipError_t mbar_fixed_point(const MbarProb* P, const int* list, int n,
                            int max_K, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_self_consistent, dim3(max_K, n), dim3(kT), 0, st, P,
                     list);
  hipLaunchKernelGGL(k_gauge, dim3(1, n), dim3(kT), 0, st, P, list);
  return hipGetLastError();
}

hipError_t mbar_accumulate(const MbarProb* P, const int* list, int n, int ts,
                           int max_blocks, hipStream_t st) {
  if (n == 0) return hipSuccess;
  switch (ts) {
    case 1: return accumulate_ts<1>(P, list, n, max_blocks, st);
    case 2: return accumulate_ts<2>(P, list, n, max_blocks, st);
    case 4: return accumulate_ts<4>(P, list, n, max_blocks, st);
    default: return accumulate_ts<8>(P, list, n, max_blocks, st);
  }
}

hipError_t mbar_newton(const MbarProb* P, const int* list, int n, int max_K,
                       int want_inverse, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int width = max_K + max_K * max_K;
  hipLaunchKernelGGL(k_reduce_partials, dim3((width + kRedT - 1) / kRedT, n),
                     dim3(kRedT), 0, st, P, list);
  const size_t bytes = mbar_newton_lds(max_K, want_inverse);
  // LDS when the largest system fits beside the kernel's static arrays
  if (bytes <= 60 * 1024)
    hipLaunchKernelGGL(k_newton<true>, dim3(1, n), dim3(kNewtonT), bytes, st,
                       P, list, want_inverse);
  else
    hipLaunchKernelGGL(k_newton<false>, dim3(1, n), dim3(kNewtonT), 0, st, P,
                       list, want_inverse);
  return hipGetLastError();
}

hipError_t mbar_axpy(const MbarProb* P, const int* list, int n,
                     const double* tvec, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy, dim3(1, n), dim3(kT), 0, st, P, list, tvec);
  return hipGetLastError();
}

hipError_t mbar_accept(const MbarProb* P, const int* list, int n,
                       hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_accept, dim3(1, n), dim3(kT), 0, st, P, list);
  return hipGetLastError();
}

}  // namespace bpmf
