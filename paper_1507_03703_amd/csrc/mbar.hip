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

// partial[b] = [colsum_i (K) | M_ij (K*K)] over the block's sample chunks;
// PER = entries of M per thread (K*K <= PER * blockDim)
template <int PER>
__global__ __launch_bounds__(kT) void k_accumulate(
    const double* __restrict__ ukn, int K, int64_t N, int64_t ld,
    const double* __restrict__ f, const double* __restrict__ logD,
    double* __restrict__ partial, int chunk) {
  extern __shared__ double W[];  // K x chunk
  double acc[PER];
  double col = 0.0;
  const int KK = K * K;
#pragma unroll
  for (int q = 0; q < PER; ++q) acc[q] = 0.0;
  const int64_t n_chunks = (N + chunk - 1) / chunk;
  for (int64_t ch = blockIdx.x; ch < n_chunks; ch += gridDim.x) {
    const int64_t n0 = ch * chunk;
    const int cnt = (int)((N - n0) < chunk ? (N - n0) : chunk);
    __syncthreads();
    for (int e = threadIdx.x; e < K * chunk; e += blockDim.x) {
      const int k = e / chunk, j = e - k * chunk;
      W[e] = j < cnt ? exp(f[k] - ukn[(size_t)k * ld + n0 + j] - logD[n0 + j])
                     : 0.0;
    }
    __syncthreads();
    if ((int)threadIdx.x < K) {
      const double* wi = W + threadIdx.x * chunk;
      for (int j = 0; j < cnt; ++j) col += wi[j];
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + kT * q;
      if (e < KK) {
        const int i = e / K, j = e - i * K;
        const double* wi = W + i * chunk;
        const double* wj = W + j * chunk;
        double s = 0.0;
        for (int t = 0; t < cnt; ++t) s += wi[t] * wj[t];
        acc[q] += s;
      }
    }
  }
  double* out = partial + (size_t)blockIdx.x * (K + KK);
  if ((int)threadIdx.x < K) out[threadIdx.x] = col;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + kT * q;
    if (e < KK) out[K + e] = acc[q];
  }
}

// Newton step (single block): reduce partials, build the gauge-fixed system
// [H~ | -g~ | I], Gauss-Jordan eliminate (H~ is symmetric positive definite),
// write step, max|step|, g.step and, on request, var(f_k - f_0).
__global__ __launch_bounds__(1024) void k_newton(
    const double* __restrict__ partial, int nb, int K,
    const double* __restrict__ Nk, double* __restrict__ red,
    double* __restrict__ mat, double* __restrict__ step,
    double* __restrict__ scalars, int want_inverse,
    double* __restrict__ var_out) {
  __shared__ double fac[BPMF_MAX_MBAR_STATES_DEV];
  __shared__ double gsh[BPMF_MAX_MBAR_STATES_DEV];
  __shared__ double piv_sh, dmax_sh;
  __shared__ int bad;
  const int KK = K * K, stride = K + KK;
  for (int e = threadIdx.x; e < stride; e += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[(size_t)b * stride + e];
    red[e] = s;
  }
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
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

hipError_t mbar_accumulate(const double* ukn, int K, int64_t N, int64_t ld,
                           const double* f, const MbarScratch& s,
                           hipStream_t st) {
  const int chunk = 4096 / K < 1 ? 1 : 4096 / K;
  const size_t lds = (size_t)K * chunk * sizeof(double);
  const int KK = K * K;
  if (KK <= kT)
    hipLaunchKernelGGL(k_accumulate<1>, dim3(s.n_blocks), dim3(kT), lds, st,
                       ukn, K, N, ld, f, s.logD, s.partial, chunk);
  else if (KK <= 4 * kT)
    hipLaunchKernelGGL(k_accumulate<4>, dim3(s.n_blocks), dim3(kT), lds, st,
                       ukn, K, N, ld, f, s.logD, s.partial, chunk);
  else if (KK <= 16 * kT)
    hipLaunchKernelGGL(k_accumulate<16>, dim3(s.n_blocks), dim3(kT), lds, st,
                       ukn, K, N, ld, f, s.logD, s.partial, chunk);
  else if (KK <= 64 * kT)
    hipLaunchKernelGGL(k_accumulate<64>, dim3(s.n_blocks), dim3(kT), lds, st,
                       ukn, K, N, ld, f, s.logD, s.partial, chunk);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t mbar_newton(int K, const double* N_k_dev, const MbarScratch& s,
                       int want_inverse, double* var_out, hipStream_t st) {
  hipLaunchKernelGGL(k_newton, dim3(1), dim3(1024), 0, st, s.partial,
                     s.n_blocks, K, N_k_dev, s.red, s.mat, s.step, s.scalars,
                     want_inverse, var_out);
  return hipGetLastError();
}

hipError_t mbar_axpy(int K, const double* f, const double* step, double t,
                     double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy, dim3(1), dim3(kT), 0, st, f, step, t, K, out);
  return hipGetLastError();
}

}  // namespace bpmf
