// MBAR on the device in double precision (Shirts & Chodera 2008; the paper
// estimates f_BC,L and f_CD' with it, Methodology "Estimation").
//
// The free energies minimise the convex function
//   F(f) = sum_n ln sum_k N_k exp(f_k - u_kn) - sum_i N_i f_i,   f_0 = 0,
// whose gradient is g_i = N_i (sum_n W_ni - 1) and Hessian
//   H_ij = N_i delta_ij sum_n W_ni - N_i N_j sum_n W_ni W_nj,
// W_ni = exp(f_i - u_in) / sum_k N_k exp(f_k - u_kn).  Newton steps solve the
// gauge-fixed system; var(f_k - f_0) = (H~^-1)_kk - 1/N_k - 1/N_0.
// All reductions run over a fixed block grid in a fixed order, so results do
// not depend on scheduling.
#include <hip/hip_runtime.h>
#include <math.h>

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

// logD_n = ln sum_k exp(logN_k + f_k - u_kn); obj_part[b] = sum over the
// block's samples of logD_n
__global__ __launch_bounds__(kT) void k_logD(const double* __restrict__ ukn,
                                             int K, int64_t N, int64_t ld,
                                             const double* __restrict__ f,
                                             const double* __restrict__ logN,
                                             double* __restrict__ logD,
                                             double* __restrict__ obj_part) {
  __shared__ double a[BPMF_MAX_MBAR_STATES_DEV];
  __shared__ double red[kT];
  for (int k = threadIdx.x; k < K; k += blockDim.x) a[k] = logN[k] + f[k];
  __syncthreads();
  double acc = 0.0;
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N;
       n += (int64_t)gridDim.x * blockDim.x) {
    double m = -INFINITY;
    for (int k = 0; k < K; ++k) m = fmax(m, a[k] - ukn[(size_t)k * ld + n]);
    double s = 0.0;
    for (int k = 0; k < K; ++k) s += exp(a[k] - ukn[(size_t)k * ld + n] - m);
    const double v = m + log(s);
    logD[n] = v;
    acc += v;
  }
  const double b = block_sum(acc, red);
  if (threadIdx.x == 0) obj_part[blockIdx.x] = b;
}

// scalars[0] = sum_b obj_part[b] - sum_k N_k f_k
__global__ __launch_bounds__(kT) void k_objective(
    const double* __restrict__ obj_part, int nb, const double* __restrict__ f,
    const double* __restrict__ Nk, int K, double* __restrict__ scalars) {
  __shared__ double red[kT];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += obj_part[b];
  const double s1 = block_sum(acc, red);
  acc = 0.0;
  for (int k = threadIdx.x; k < K; k += blockDim.x) acc += Nk[k] * f[k];
  const double s2 = block_sum(acc, red);
  if (threadIdx.x == 0) scalars[0] = s1 - s2;
}

// self-consistent update f_i = -ln sum_n exp(-u_in - logD_n), one block per
// state, followed by the gauge shift (k_gauge)
__global__ __launch_bounds__(kT) void k_self_consistent(
    const double* __restrict__ ukn, int64_t N, int64_t ld,
    const double* __restrict__ logD, double* __restrict__ fnew) {
  __shared__ double red[kT];
  const int i = blockIdx.x;
  double m = -INFINITY;
  for (int64_t n = threadIdx.x; n < N; n += blockDim.x)
    m = fmax(m, -ukn[(size_t)i * ld + n] - logD[n]);
  // block max
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const double M = red[0];
  __syncthreads();
  double acc = 0.0;
  for (int64_t n = threadIdx.x; n < N; n += blockDim.x)
    acc += exp(-ukn[(size_t)i * ld + n] - logD[n] - M);
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) fnew[i] = -(M + log(s));
}

__global__ void k_gauge(const double* __restrict__ fnew, int K,
                        double* __restrict__ f) {
  for (int k = threadIdx.x; k < K; k += blockDim.x) f[k] = fnew[k] - fnew[0];
}

// partial[b] = [colsum_i (K) | M_ij (K*K)] over the block's sample chunks,
// M = W W^T with W_in = exp(f_i - u_in - logD_n).  A chunk of W sits in LDS
// sample-major, row stride Kp + 2 doubles (16-byte aligned rows, staggered
// banks); the 256 threads form a 16 x 16 grid of TS x TS register tiles of
// M (Kp = 16 TS >= K, rows and columns past K are zero).
template <int TS>
__global__ __launch_bounds__(kT) void k_accumulate(
    const double* __restrict__ ukn, int K, int64_t N, int64_t ld,
    const double* __restrict__ f, const double* __restrict__ logD,
    double* __restrict__ partial, int chunk) {
  constexpr int Kp = 16 * TS, RS = Kp + 2;
  extern __shared__ __align__(16) double W[];  // chunk x RS
  __shared__ double fk[Kp];
  const int tid = threadIdx.x;
  const int ta = tid >> 4, tb = tid & 15;
  for (int k = tid; k < Kp; k += kT) fk[k] = k < K ? f[k] : 0.0;
  double acc[TS][TS];
#pragma unroll
  for (int i = 0; i < TS; ++i)
#pragma unroll
    for (int j = 0; j < TS; ++j) acc[i][j] = 0.0;
  double col = 0.0;
  const int64_t n_chunks = (N + chunk - 1) / chunk;
  for (int64_t ch = blockIdx.x; ch < n_chunks; ch += gridDim.x) {
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
  double* out = partial + (size_t)blockIdx.x * (K + KK);
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
    const double* __restrict__ partial, int nb, int width,
    double* __restrict__ red) {
  const int e = blockIdx.x * kRedT + threadIdx.x;
  if (e >= width) return;
  double s = 0.0;
#pragma unroll 16
  for (int b = 0; b < nb; ++b) s += partial[(size_t)b * width + e];
  red[e] = s;
}

// Newton step (single block): from the reduced sums build the gauge-fixed
// system [H~ | -g~ (| I)], Gauss-Jordan eliminate it (H~ is symmetric
// positive definite), write step, max|step|, g.step and, on request,
// var(f_k - f_0).  `mat` is LDS (dynamic) when the system fits, else global.
constexpr int kNewtonT = 256;
template <bool LDS>
__global__ __launch_bounds__(kNewtonT) void k_newton(
    const double* __restrict__ red, int K, const double* __restrict__ Nk,
    double* __restrict__ gmat, double* __restrict__ step,
    double* __restrict__ scalars, int want_inverse,
    double* __restrict__ var_out) {
  extern __shared__ __align__(16) double lmat[];
  double* mat = LDS ? lmat : gmat;
  __shared__ double fac[BPMF_MAX_MBAR_STATES_DEV];
  __shared__ double gsh[BPMF_MAX_MBAR_STATES_DEV];
  __shared__ double piv_sh, dmax_sh;
  __shared__ int bad;
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
    for (int p = 0; p < m; ++p) dm = fmax(dm, mat[(size_t)p * wcols + p]);
    dmax_sh = dm;
  }
  __syncthreads();
  // a pivot below 1e-13 of the largest diagonal entry marks the system as
  // not numerically positive definite (the caller then takes a fixed-point
  // step instead)
  const double pmin = 1e-13 * dmax_sh;
  for (int p = 0; p < m; ++p) {
    if (threadIdx.x == 0) {
      piv_sh = mat[(size_t)p * wcols + p];
      if (!(piv_sh > pmin)) bad = 1;
    }
    __syncthreads();
    const double piv = piv_sh;
    for (int c = threadIdx.x; c < wcols; c += blockDim.x)
      mat[(size_t)p * wcols + c] /= piv;
    for (int r = threadIdx.x; r < m; r += blockDim.x)
      fac[r] = mat[(size_t)r * wcols + p];
    __syncthreads();
    for (int e = threadIdx.x; e < m * wcols; e += blockDim.x) {
      const int r = e / wcols, c = e - r * wcols;
      if (r != p) mat[e] -= fac[r] * mat[(size_t)p * wcols + c];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double mx = 0.0, gs = 0.0;
    step[0] = 0.0;
    for (int i = 1; i < K; ++i) {
      const double s = mat[(size_t)(i - 1) * wcols + m];
      step[i] = s;
      mx = fmax(mx, fabs(s));
      gs += gsh[i] * s;
    }
    scalars[1] = mx;
    scalars[2] = gs;
    scalars[3] = bad ? 1.0 : 0.0;
    if (want_inverse && var_out) {
      var_out[0] = 0.0;
      for (int i = 1; i < K; ++i)
        var_out[i] = mat[(size_t)(i - 1) * wcols + m + 1 + (i - 1)] -
                     1.0 / Nk[i] - 1.0 / Nk[0];
    }
  }
}

__global__ void k_axpy(const double* __restrict__ f,
                       const double* __restrict__ s, double t, int K,
                       double* __restrict__ out) {
  for (int k = threadIdx.x; k < K; k += blockDim.x) out[k] = f[k] + t * s[k];
}

}  // namespace

hipError_t mbar_logD(const double* ukn, int K, int64_t N, int64_t ld,
                     const double* f, const MbarScratch& s, hipStream_t st) {
  hipLaunchKernelGGL(k_logD, dim3(s.n_blocks), dim3(kT), 0, st, ukn, K, N, ld,
                     f, s.logN, s.logD, s.obj_part);
  return hipGetLastError();
}

hipError_t mbar_objective(int K, const int64_t*, const MbarScratch& s,
                          const double* f, double* N_k_dev, hipStream_t st) {
  hipLaunchKernelGGL(k_objective, dim3(1), dim3(kT), 0, st, s.obj_part,
                     s.n_blocks, f, N_k_dev, K, s.scalars);
  return hipGetLastError();
}

hipError_t mbar_self_consistent(const double* ukn, int K, int64_t N,
                                int64_t ld, const MbarScratch& s,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_self_consistent, dim3(K), dim3(kT), 0, st, ukn, N, ld,
                     s.logD, s.step);
  hipLaunchKernelGGL(k_gauge, dim3(1), dim3(kT), 0, st, s.step, K, s.f);
  return hipGetLastError();
}

int mbar_acc_chunk(int K) {
  const int TS = K <= 16 ? 1 : K <= 32 ? 2 : K <= 64 ? 4 : 8;
  return 4096 / (16 * TS);
}

int mbar_acc_blocks(int K, int64_t N) {
  const int64_t chunks = (N + mbar_acc_chunk(K) - 1) / mbar_acc_chunk(K);
  return (int)(chunks < 256 ? chunks : 256);
}

hipError_t mbar_accumulate(const double* ukn, int K, int64_t N, int64_t ld,
                           const double* f, const MbarScratch& s,
                           hipStream_t st) {
  const int chunk = mbar_acc_chunk(K);
  const int nb = mbar_acc_blocks(K, N);
  const int TS = K <= 16 ? 1 : K <= 32 ? 2 : K <= 64 ? 4 : 8;
  const size_t lds = (size_t)chunk * (16 * TS + 2) * sizeof(double);
  if (TS == 1)
    hipLaunchKernelGGL(k_accumulate<1>, dim3(nb), dim3(kT), lds, st, ukn, K,
                       N, ld, f, s.logD, s.partial, chunk);
  else if (TS == 2)
    hipLaunchKernelGGL(k_accumulate<2>, dim3(nb), dim3(kT), lds, st, ukn, K,
                       N, ld, f, s.logD, s.partial, chunk);
  else if (TS == 4)
    hipLaunchKernelGGL(k_accumulate<4>, dim3(nb), dim3(kT), lds, st, ukn, K,
                       N, ld, f, s.logD, s.partial, chunk);
  else
    hipLaunchKernelGGL(k_accumulate<8>, dim3(nb), dim3(kT), lds, st, ukn, K,
                       N, ld, f, s.logD, s.partial, chunk);
  const int width = K + K * K;
  hipLaunchKernelGGL(k_reduce_partials, dim3((width + kRedT - 1) / kRedT),
                     dim3(kRedT), 0, st, s.partial, nb, width, s.red);
  return hipGetLastError();
}

hipError_t mbar_newton(int K, const double* N_k_dev, const MbarScratch& s,
                       int want_inverse, double* var_out, hipStream_t st) {
  const int m = K - 1;
  const size_t bytes =
      (size_t)m * (m + 1 + (want_inverse ? m : 0)) * sizeof(double);
  // LDS when the system fits beside the kernel's static arrays
  if (bytes <= 60 * 1024)
    hipLaunchKernelGGL(k_newton<true>, dim3(1), dim3(kNewtonT), bytes, st,
                       s.red,
                       K, N_k_dev, s.mat, s.step, s.scalars, want_inverse,
                       var_out);
  else
    hipLaunchKernelGGL(k_newton<false>, dim3(1), dim3(kNewtonT), 0, st, s.red,
                       K,
                       N_k_dev, s.mat, s.step, s.scalars, want_inverse,
                       var_out);
  return hipGetLastError();
}

hipError_t mbar_axpy(int K, const double* f, const double* step, double t,
                     double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy, dim3(1), dim3(kT), 0, st, f, step, t, K, out);
  return hipGetLastError();
}

}  // namespace bpmf
