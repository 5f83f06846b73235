// Learned rigid-body pose proposal on gfx950: a conditional Gaussian-mixture
// density q(t, omega | tau) from an MLP 16 -> 256 -> 256 -> 104 (SiLU), its
// training (negative log-likelihood, Adam) and the independence
// Metropolis-Hastings pose move it drives.  The paper's own pose move is a
// random rotation about the centre of mass plus a Gaussian translation with
// Metropolis acceptance (Sampling section); here the proposal is learned and
// the acceptance carries the exact proposal density on SE(3).
//
// Dense layers run on the matrix cores: v_mfma_f32_16x16x32_bf16 with bf16
// operands rounded from fp32 when they are staged in LDS and fp32
// accumulation.
#include <hip/hip_runtime.h>
#include <math.h>

#include "deferred.h"
#include "device.h"
#include "internal.h"
#include "mlp.h"

namespace bpmf {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// fp32 -> bf16 bits, round to nearest even (finite inputs); NaN stays NaN
__device__ __forceinline__ unsigned short bf16_bits(float f) {
  const unsigned int u = __float_as_uint(f);
  const unsigned int rn = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
  const unsigned int qn = (u >> 16) | 0x40u;
  return (unsigned short)((u & 0x7fffffffu) > 0x7f800000u ? qn : rn);
}

constexpr int kTile = 64;   // output tile edge per workgroup
constexpr int kKStep = 32;  // K per MFMA
constexpr int kPad = 8;     // LDS row padding (bf16 elements)

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// C[m, n] = sum_k A(m, k) B(k, n) with epilogue (see GemmArgs).  A block of
// 256 threads computes a 64 x 64 tile; wave (wm, wn) owns a 32 x 32 quarter
// as 2 x 2 MFMA tiles of 16 x 16.  Operand layout of the 16x16x32 bf16 MFMA:
// lane l supplies row (l % 16) of A and column (l % 16) of B, each with the
// 8 consecutive k = 8 (l / 16) .. + 7; it receives D rows 4 (l / 16) .. + 3
// of column l % 16.
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  __shared__ __align__(16) unsigned short As[kTile][kKStep + kPad];
  __shared__ __align__(16) unsigned short Bs[kTile][kKStep + kPad];  // [n][k]
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int m0 = blockIdx.y * kTile, n0 = blockIdx.x * kTile;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int k0 = 0; k0 < g.K; k0 += kKStep) {
    // stage: 64 x 32 elements of A and of B, 8 per thread
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = tid + 256 * q;       // 0 .. 2047
      const int r = e >> 5, kk = e & 31;  // row/col of tile, k in step
      const int m = m0 + r, n = n0 + r, k = k0 + kk;
      float av = 0.f, bv = 0.f;
      if (m < g.M && k < g.K) av = g.A[(int64_t)m * g.sam + (int64_t)k * g.sak];
      if (n < g.N && k < g.K) bv = g.B[(int64_t)k * g.sbk + (int64_t)n * g.sbn];
      As[r][kk] = bf16_bits(av);
      Bs[r][kk] = bf16_bits(bv);
    }
    __syncthreads();
    const int kg = (lane >> 4) * 8;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int ar = wm * 32 + i * 16 + (lane & 15);
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[ar][kg]);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int bc = wn * 32 + j * 16 + (lane & 15);
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[bc][kg]);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i][j], 0,
                                                            0, 0);
      }
    }
    __syncthreads();
  }
  // epilogue
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wm * 32 + i * 16 + (lane >> 4) * 4 + q;
        const int n = n0 + wn * 32 + j * 16 + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        float v = acc[i][j][q];
        const int64_t o = (int64_t)m * g.ldc + n;
        if (g.bias) v += g.bias[n];
        if (g.epi == kEpiSilu) {
          g.Zout[o] = v;
          g.C[o] = silu(v);
        } else if (g.epi == kEpiDsilu) {
          g.C[o] = v * dsilu(g.Zin[o]);
        } else {
          g.C[o] = v;
        }
      }
}

// The three dense layers for kFRows rows per workgroup.  A row's path
// through the network does not involve the other rows, so one workgroup
// takes its rows through all three layers with the activations held in LDS
// as the next layer's bf16 operand; each wave owns every kFWaves-th
// 16-column output tile.  Every tile is accumulated by the same MFMA over the same
// 32-wide k chunks in the same order, from operands rounded to bf16 in the
// same way, and finished by the same epilogue as k_gemm, so the outputs are
// those of three k_gemm launches.
constexpr int kFRows = 16;
constexpr int kFWaves = 16;  // wavefronts per workgroup
constexpr int kFLd = kNHid + kPad;  // LDS row length (bf16 elements)

// one layer: out(16 x N) = act(A(16 x Kin) W(Kin x N) + bias), A in LDS.
// A wave accumulates all its tiles in one pass over k, so the weight loads
// of every tile of a k chunk are in flight together.
template <int KIN, int N, bool HIDDEN>
__device__ __forceinline__ void dense_rows(
    const unsigned short (*A)[kFLd], const float* __restrict__ W,
    const float* __restrict__ bias, int row0, int B, float* __restrict__ Z,
    float* __restrict__ H, unsigned short (*Hn)[kFLd], int lane, int wv) {
  constexpr int kTiles = (N + 15) / 16;
  constexpr int kTPW = (kTiles + kFWaves - 1) / kFWaves;
  const int kg = (lane >> 4) * 8;
  f32x4 acc[kTPW];
#pragma unroll
  for (int i = 0; i < kTPW; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
  for (int k0 = 0; k0 < KIN; k0 += kKStep) {
    bf16x8 a, b[kTPW];
    // loads at clamped (in-bounds) indices, unconditionally, so that they
    // issue together; out-of-range operands are then zeroed
    float w[kTPW][8];
    unsigned short av[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = k0 + kg + e, kc = k < KIN ? k : KIN - 1;
      av[e] = A[lane & 15][kc];
#pragma unroll
      for (int i = 0; i < kTPW; ++i) {
        const int n = (wv + kFWaves * i) * 16 + (lane & 15);
        const int nc = n < N ? n : N - 1;
        w[i][e] = W[(int64_t)kc * N + nc];
      }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const bool in = k0 + kg + e < KIN;
      a[e] = __builtin_bit_cast(__bf16, in ? av[e] : (unsigned short)0);
#pragma unroll
      for (int i = 0; i < kTPW; ++i) {
        const int n = (wv + kFWaves * i) * 16 + (lane & 15);
        b[i][e] = __builtin_bit_cast(
            __bf16, (in && n < N) ? bf16_bits(w[i][e]) : (unsigned short)0);
      }
    }
#pragma unroll
    for (int i = 0; i < kTPW; ++i)
      if (wv + kFWaves * i < kTiles)  // uniform over the wave
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[i], acc[i], 0,
                                                         0, 0);
  }
#pragma unroll
  for (int i = 0; i < kTPW; ++i) {
    const int n = (wv + kFWaves * i) * 16 + (lane & 15);
    if (n >= N) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = (lane >> 4) * 4 + q, m = row0 + r;
      const float v = acc[i][q] + bias[n];
      if (HIDDEN) {
        const float h = silu(v);
        Hn[r][n] = bf16_bits(h);
        if (m < B) {
          Z[(int64_t)m * N + n] = v;
          H[(int64_t)m * N + n] = h;
        }
      } else if (m < B) {
        H[(int64_t)m * N + n] = v;
      }
    }
  }
}

// dense_rows with the weights from their bf16 transposed copy (row n of WT
// holds column n of W, KLD elements, zero past KIN and past N): a lane's
// eight k values of a tile are one 16-byte load.  The operands, the k order
// and the epilogue are dense_rows', so the results are the same bits.
template <int KIN, int KLD, int N, bool HIDDEN>
__device__ __forceinline__ void dense_rows_t(
    const unsigned short (*A)[kFLd], const unsigned short* __restrict__ WT,
    const float* __restrict__ bias, int row0, int B, float* __restrict__ H,
    unsigned short (*Hn)[kFLd], int lane, int wv) {
  constexpr int kTiles = (N + 15) / 16;
  constexpr int kTPW = (kTiles + kFWaves - 1) / kFWaves;
  typedef const bf16x8 __attribute__((address_space(1))) gbf;
  const int kg = (lane >> 4) * 8;
  f32x4 acc[kTPW];
#pragma unroll
  for (int i = 0; i < kTPW; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  // every k step's weight loads in flight at once (one 16-byte load per
  // tile and step): one round trip to L2 per layer
#pragma unroll
  for (int k0 = 0; k0 < KIN; k0 += kKStep) {
    bf16x8 b[kTPW];
#pragma unroll
    for (int i = 0; i < kTPW; ++i) {
      const int n = (wv + kFWaves * i) * 16 + (lane & 15);
      if (wv + kFWaves * i < kTiles)  // uniform over the wave
        b[i] = *(gbf*)(WT + (int64_t)n * KLD + k0 + kg);
    }
    bf16x8 a;
    if (k0 + kg < KIN) {
      a = *reinterpret_cast<const bf16x8*>(&A[lane & 15][k0 + kg]);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) a[e] = __builtin_bit_cast(__bf16,
                                                           (unsigned short)0);
    }
#pragma unroll
    for (int i = 0; i < kTPW; ++i)
      if (wv + kFWaves * i < kTiles)
        acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[i], acc[i], 0,
                                                         0, 0);
  }
#pragma unroll
  for (int i = 0; i < kTPW; ++i) {
    const int n = (wv + kFWaves * i) * 16 + (lane & 15);
    if (n >= N) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = (lane >> 4) * 4 + q, m = row0 + r;
      const float v = acc[i][q] + bias[n];
      if (HIDDEN)
        Hn[r][n] = bf16_bits(silu(v));
      else if (m < B)
        H[(int64_t)m * N + n] = v;
    }
  }
}

__device__ float dihedral_angle(const float* x, int4 q);

// The network on the current configurations of pose-move tasks, for groups
// of up to 16 rows (row m = task m), group b with its own parameters (bf16
// transposed weights), outputs only; each row's features (sin and cos of
// the conditioning torsions, the dihedral angles of the replica's
// configuration) are computed in place, one thread per (row, torsion slot).
// Blocks past n_groups close a run of neighbour-scheme sweeps instead, one
// ligand of `fin` each (finish_ligand): the features need only positions,
// which that leaves unchanged.
__global__ __launch_bounds__(kFWaves * 64) void k_pose_network(
    const MlpGroup* __restrict__ groups, int n_groups,
    const LigDev* __restrict__ ligs, const PropDev* __restrict__ props,
    const PoseTask* __restrict__ tasks, float* __restrict__ out,
    const LigDev* __restrict__ fin, int exchange_every, int sample_every,
    uint64_t seed) {
  if ((int)blockIdx.x >= n_groups) {
    finish_ligand(fin[blockIdx.x - n_groups], exchange_every, sample_every,
                  seed);
    return;
  }
  __shared__ __align__(16) unsigned short S[2][kFRows][kFLd];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const MlpGroup gr = groups[blockIdx.x];
  const int row0 = gr.row0, B = gr.row0 + gr.rows;
  static_assert(kNFeat == 16, "eight torsion slots of sin, cos");
  for (int e = tid; e < kFRows * 8; e += kFWaves * 64) {
    const int r = e >> 3, q = e & 7, m = row0 + r;
    float sn = 0.f, cs = 0.f;
    if (m < B) {
      const PoseTask t = tasks[m];
      const LigDev& L = ligs[t.lig];
      const PropDev& P = props[t.lig];
      if (q < P.n_cond) {
        const float phi =
            dihedral_angle(L.x + (size_t)t.r * L.n * 3, P.cond[q]);
        sincosf(phi, &sn, &cs);
      }
    }
    S[0][r][2 * q] = bf16_bits(sn);
    S[0][r][2 * q + 1] = bf16_bits(cs);
  }
  __syncthreads();
  dense_rows_t<kNFeat, kT1Ld, kNHid, true>(S[0], gr.WT + kTOff1,
                                           gr.P + kOffB1, row0, B, nullptr,
                                           S[1], lane, wv);
  __syncthreads();
  dense_rows_t<kNHid, kT2Ld, kNHid, true>(S[1], gr.WT + kTOff2,
                                          gr.P + kOffB2, row0, B, nullptr,
                                          S[0], lane, wv);
  __syncthreads();
  dense_rows_t<kNHid, kT3Ld, kNOut, false>(S[0], gr.WT + kTOff3,
                                           gr.P + kOffB3, row0, B, out,
                                           nullptr, lane, wv);
}

// WT from the fp32 parameters: element (n, k) of each transposed matrix is
// the bf16 rounding of W[k][n] (0 in the padding)
__global__ __launch_bounds__(256) void k_weights_bf16(
    const float* __restrict__ P, unsigned short* __restrict__ WT) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kTSize) return;
  int off, ld, kin, nout;
  const float* W;
  if (i < kTOff2) {
    off = kTOff1; ld = kT1Ld; kin = kNFeat; nout = kNHid; W = P + kOffW1;
  } else if (i < kTOff3) {
    off = kTOff2; ld = kT2Ld; kin = kNHid; nout = kNHid; W = P + kOffW2;
  } else {
    off = kTOff3; ld = kT3Ld; kin = kNHid; nout = kNOut; W = P + kOffW3;
  }
  const int n = (i - off) / ld, k = (i - off) - n * ld;
  WT[i] = (n < nout && k < kin) ? bf16_bits(W[(int64_t)k * nout + n])
                                : (unsigned short)0;
}

__global__ __launch_bounds__(kFWaves * 64) void k_mlp_forward(
    const float* __restrict__ P, const float* __restrict__ X, int B,
    float* __restrict__ Z1, float* __restrict__ H1, float* __restrict__ Z2,
    float* __restrict__ H2, float* __restrict__ out) {
  __shared__ __align__(16) unsigned short S[2][kFRows][kFLd];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int row0 = blockIdx.x * kFRows;
  for (int e = tid; e < kFRows * kNFeat; e += kFWaves * 64) {
    const int r = e / kNFeat, k = e - r * kNFeat, m = row0 + r;
    S[0][r][k] = bf16_bits(m < B ? X[(int64_t)m * kNFeat + k] : 0.f);
  }
  __syncthreads();
  dense_rows<kNFeat, kNHid, true>(S[0], P + kOffW1, P + kOffB1, row0, B, Z1,
                                  H1, S[1], lane, wv);
  __syncthreads();
  dense_rows<kNHid, kNHid, true>(S[1], P + kOffW2, P + kOffB2, row0, B, Z2,
                                 H2, S[0], lane, wv);
  __syncthreads();
  dense_rows<kNHid, kNOut, false>(S[0], P + kOffW3, P + kOffB3, row0, B,
                                  nullptr, out, nullptr, lane, wv);
}

// column sums of X (rows x cols, row stride ld): out[c] = sum_r X[r, c].
// 64 columns per block, each summed by 4 threads over interleaved rows and
// the 4 partials added in a fixed order.
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ X,
                                                int rows, int cols, int64_t ld,
                                                float* __restrict__ out) {
  __shared__ double part[4][64];
  const int cl = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + cl;
  double s = 0.0;
  if (c < cols) {
#pragma unroll 8
    for (int r = g; r < rows; r += 4) s += X[(int64_t)r * ld + c];
  }
  part[g][cl] = s;
  __syncthreads();
  if (g == 0 && c < cols)
    out[c] = (float)(((part[0][cl] + part[1][cl]) + part[2][cl]) + part[3][cl]);
}

__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + expf(-z)); }

// Mixture parameters of one output row (13 numbers per component).
struct Mix {
  float lw[kNComp];  // log weights (normalised by mixture_of; the pose move
                     // keeps the raw logits and normalises them, mix_lse)
  float mt[kNComp][3], mw[kNComp][3], st[kNComp][3], sw[kNComp][3];
};

// log-normaliser of the raw mixture logits (the log-softmax's lse, float)
__device__ __forceinline__ float mix_lse(const Mix& p) {
  float mx = -INFINITY;
  for (int j = 0; j < kNComp; ++j) mx = fmaxf(mx, p.lw[j]);
  float sm = 0.f;
  for (int j = 0; j < kNComp; ++j) sm += expf(p.lw[j] - mx);
  return mx + logf(sm);
}

__device__ __forceinline__ void mixture_of(const float* o, Mix& p) {
  float mx = -INFINITY;
  for (int j = 0; j < kNComp; ++j) mx = fmaxf(mx, o[13 * j]);
  float s = 0.f;
  for (int j = 0; j < kNComp; ++j) s += expf(o[13 * j] - mx);
  const float lse = mx + logf(s);
  for (int j = 0; j < kNComp; ++j) {
    const float* r = o + 13 * j;
    p.lw[j] = r[0] - lse;
    for (int a = 0; a < 3; ++a) {
      p.mt[j][a] = r[1 + a];
      p.mw[j][a] = (float)M_PI * tanhf(r[4 + a]);
      p.st[j][a] = kSt0 + (kSt1 - kSt0) * sigm(r[7 + a]);
      p.sw[j][a] = kSw0 + (kSw1 - kSw0) * sigm(r[10 + a]);
    }
  }
}

// negative log-likelihood of (t, w) and d loss / d out (scaled by 1/B)
__global__ __launch_bounds__(256) void k_nll(const float* __restrict__ out,
                                             const float* __restrict__ pose,
                                             int B, float inv_b,
                                             float* __restrict__ dout,
                                             double* __restrict__ loss_part) {
  __shared__ double red[256];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double li = 0.0;
  if (i < B) {
    const float* o = out + (int64_t)i * kNOut;
    const float* ps = pose + (int64_t)i * 6;
    Mix p;
    mixture_of(o, p);
    float a[kNComp], zt[kNComp][3], zw[kNComp][3];
    float mx = -INFINITY;
    for (int j = 0; j < kNComp; ++j) {
      float lg = p.lw[j] - 3.0f * logf(2.0f * (float)M_PI);
      for (int d = 0; d < 3; ++d) {
        zt[j][d] = (ps[d] - p.mt[j][d]) / p.st[j][d];
        zw[j][d] = (ps[3 + d] - p.mw[j][d]) / p.sw[j][d];
        lg += -0.5f * (zt[j][d] * zt[j][d] + zw[j][d] * zw[j][d]) -
              logf(p.st[j][d]) - logf(p.sw[j][d]);
      }
      a[j] = lg;
      mx = fmaxf(mx, lg);
    }
    float s = 0.f;
    for (int j = 0; j < kNComp; ++j) s += expf(a[j] - mx);
    const float ll = mx + logf(s);
    li = -(double)ll;
    float* d = dout + (int64_t)i * kNOut;
    for (int j = 0; j < kNComp; ++j) {
      const float r = expf(a[j] - ll);
      const float pi = expf(p.lw[j]);
      const float* oj = o + 13 * j;
      float* dj = d + 13 * j;
      dj[0] = -(r - pi) * inv_b;
      for (int q = 0; q < 3; ++q) {
        dj[1 + q] = -r * zt[j][q] / p.st[j][q] * inv_b;
        const float th = tanhf(oj[4 + q]);
        dj[4 + q] = -r * zw[j][q] / p.sw[j][q] * (float)M_PI *
                    (1.f - th * th) * inv_b;
        float sg = sigm(oj[7 + q]);
        dj[7 + q] = -r * (zt[j][q] * zt[j][q] - 1.f) / p.st[j][q] *
                    (kSt1 - kSt0) * sg * (1.f - sg) * inv_b;
        sg = sigm(oj[10 + q]);
        dj[10 + q] = -r * (zw[j][q] * zw[j][q] - 1.f) / p.sw[j][q] *
                     (kSw1 - kSw0) * sg * (1.f - sg) * inv_b;
      }
    }
  }
  red[threadIdx.x] = li;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// Adam (Kingma & Ba) on fp32 master parameters
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p,
                                              const float* __restrict__ g,
                                              float* __restrict__ m,
                                              float* __restrict__ v, int n,
                                              float lr, float b1, float b2,
                                              float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ----------------------------------------------------------------------------
// pose of a configuration: t = COM - c0, R = body frame, omega = log R,
// features = sin/cos of the conditioning torsions
// ----------------------------------------------------------------------------
struct Frame {
  float R[3][3];  // columns e1, e2, e3
};

__device__ void body_frame(const float* x, const int* fa, Frame& F) {
  float e1[3], v[3], e2[3];
  for (int a = 0; a < 3; ++a) {
    e1[a] = x[3 * fa[1] + a] - x[3 * fa[0] + a];
    v[a] = x[3 * fa[2] + a] - x[3 * fa[0] + a];
  }
  float l = rsqrtf(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
  for (int a = 0; a < 3; ++a) e1[a] *= l;
  const float pr = v[0] * e1[0] + v[1] * e1[1] + v[2] * e1[2];
  for (int a = 0; a < 3; ++a) e2[a] = v[a] - pr * e1[a];
  l = rsqrtf(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
  for (int a = 0; a < 3; ++a) e2[a] *= l;
  const float e3[3] = {e1[1] * e2[2] - e1[2] * e2[1],
                       e1[2] * e2[0] - e1[0] * e2[2],
                       e1[0] * e2[1] - e1[1] * e2[0]};
  for (int a = 0; a < 3; ++a) {
    F.R[a][0] = e1[a];
    F.R[a][1] = e2[a];
    F.R[a][2] = e3[a];
  }
}

// rotation vector of R (double), |omega| in [0, pi]: theta from
// atan2(|v|/2, (tr R - 1)/2) with v the axial vector of R - R^T, axis
// v/|v| (well conditioned up to theta -> pi); within ~5e-5 of pi the axis
// comes from the symmetric part (R + R^T)/4 + I/2 = n n^T
__device__ void log_rot(const double R[3][3], double w[3]) {
  const double c = (R[0][0] + R[1][1] + R[2][2] - 1.0) * 0.5;
  const double v[3] = {R[2][1] - R[1][2], R[0][2] - R[2][0], R[1][0] - R[0][1]};
  const double s2 = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  const double th = atan2(0.5 * s2, c);
  if (s2 < 1e-12 && c > 0) {
    for (int a = 0; a < 3; ++a) w[a] = 0.5 * v[a];
    return;
  }
  if (s2 >= 1e-12 && (s2 > 1e-4 || c > 0)) {
    for (int a = 0; a < 3; ++a) w[a] = th * v[a] / s2;
    return;
  }
  double B[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      B[a][b] = 0.25 * (R[a][b] + R[b][a]) + (a == b ? 0.5 : 0.0);
  int k = 0;
  if (B[1][1] > B[k][k]) k = 1;
  if (B[2][2] > B[k][k]) k = 2;
  double n[3] = {B[0][k], B[1][k], B[2][k]};
  const double ln = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  const double dn = n[0] * v[0] + n[1] * v[1] + n[2] * v[2];
  const double sgn = dn < 0 ? -1.0 : 1.0;
  for (int a = 0; a < 3; ++a) w[a] = sgn * th * n[a] / ln;
}

__device__ void rodrigues(const double w[3], double R[3][3]) {
  const double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  const double K[3][3] = {{0, -w[2], w[1]}, {w[2], 0, -w[0]}, {-w[1], w[0], 0}};
  double a, b;
  if (th < 1e-8) {
    a = 1.0;
    b = 0.5;
  } else {
    a = sin(th) / th;
    b = (1.0 - cos(th)) / (th * th);
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double kk = 0.0;
      for (int q = 0; q < 3; ++q) kk += K[i][q] * K[q][j];
      R[i][j] = (i == j ? 1.0 : 0.0) + a * K[i][j] + b * kk;
    }
}

__device__ float dihedral_angle(const float* x, int4 q) {
  float b1[3], b2[3], b3[3];
  for (int a = 0; a < 3; ++a) {
    b1[a] = x[3 * q.y + a] - x[3 * q.x + a];
    b2[a] = x[3 * q.z + a] - x[3 * q.y + a];
    b3[a] = x[3 * q.w + a] - x[3 * q.z + a];
  }
  const float n1[3] = {b1[1] * b2[2] - b1[2] * b2[1], b1[2] * b2[0] - b1[0] * b2[2],
                       b1[0] * b2[1] - b1[1] * b2[0]};
  const float n2[3] = {b2[1] * b3[2] - b2[2] * b3[1], b2[2] * b3[0] - b2[0] * b3[2],
                       b2[0] * b3[1] - b2[1] * b3[0]};
  const float lb2 = sqrtf(b2[0] * b2[0] + b2[1] * b2[1] + b2[2] * b2[2]);
  const float y = lb2 * (b1[0] * n2[0] + b1[1] * n2[1] + b1[2] * n2[2]);
  const float xx = n1[0] * n2[0] + n1[1] * n2[1] + n1[2] * n2[2];
  return atan2f(y, xx);
}

// pose (t, omega) and features of one configuration x of ligand L
__device__ void pose_features_one(const LigDev& L, const PropDev& P,
                                  const float* x, float* po, float* fo) {
  const int n = L.n;
  double c[3] = {0, 0, 0}, M = 0;
  for (int a = 0; a < n; ++a) {
    const double m = L.mass[a];
    M += m;
    for (int d = 0; d < 3; ++d) c[d] += m * x[3 * a + d];
  }
  Frame F;
  body_frame(x, P.frame, F);
  double R[3][3], w[3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) R[a][b] = F.R[a][b];
  log_rot(R, w);
  for (int d = 0; d < 3; ++d) {
    po[d] = (float)(c[d] / M - L.site[d]);
    po[3 + d] = (float)w[d];
  }
  for (int q = 0; q < kNFeat; ++q) fo[q] = 0.f;
  for (int q = 0; q < P.n_cond; ++q) {
    const float phi = dihedral_angle(x, P.cond[q]);
    float s, cs;
    sincosf(phi, &s, &cs);
    fo[2 * q] = s;
    fo[2 * q + 1] = cs;
  }
}

// one thread per configuration xs[i] of one ligand
__global__ __launch_bounds__(128) void k_pose_features(
    const LigDev* __restrict__ lig, const PropDev* __restrict__ prop,
    const float* __restrict__ xs, int64_t N, float* __restrict__ feats,
    float* __restrict__ poses) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const LigDev& L = *lig;
  pose_features_one(L, *prop, xs + i * L.n * 3, poses + i * 6,
                    feats + i * kNFeat);
}

// wavefront maximum of a double (DPP tree as in wave_sum)
__device__ __forceinline__ double wave_max_d(double v) {
  v = fmax(v, dpp_d<0xB1, 0xf>(v));
  v = fmax(v, dpp_d<0x4E, 0xf>(v));
  v = fmax(v, dpp_d<0x141, 0xf>(v));
  v = fmax(v, dpp_d<0x140, 0xf>(v));
  // rows that receive no broadcast keep their value (bound_ctrl off): the
  // update_dpp "old" operand is 0 there, so take max with the lane's own
  const double b15 = dpp_d<0x142, 0xa>(v);
  if ((threadIdx.x & 63) >= 16 && ((threadIdx.x >> 4) & 1)) v = fmax(v, b15);
  const double b31 = dpp_d<0x143, 0xc>(v);
  if ((threadIdx.x & 63) >= 32) v = fmax(v, b31);
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// log q_SE3(t, omega): the mixture density of (t, omega') summed over the
// preimages omega' = omega/|omega| (|omega| + 2 pi m), m = -kFold..kFold, of
// the same rotation, each with the Haar-measure factor |omega'|^2 /
// (2 (1 - cos|omega|)); one (preimage, component) term per lane of the
// calling wavefront (all 64 lanes call; lanes past the terms add nothing)
// and a log-sum-exp across the wavefront.  |omega| < 1e-9: the identity
// rotation, one term per component.  c0[j]: the pose-free part of
// component j's log-density, its normalised log weight less 3 ln 2 pi and
// the logs of its six standard deviations.
__device__ double log_q_se3_wave(const Mix& p, const double* c0,
                                 const double t[3], const double w0[3]) {
  const int lane = threadIdx.x & 63;
  const double th = sqrt(w0[0] * w0[0] + w0[1] * w0[1] + w0[2] * w0[2]);
  const bool small = th < 1e-9;
  const int n_terms = small ? kNComp : (2 * kFold + 1) * kNComp;
  double term = -INFINITY;
  if (lane < n_terms) {
    const int j = lane % kNComp, m = lane / kNComp - kFold;
    double s = c0[j];
    for (int d = 0; d < 3; ++d) {
      const double z = (t[d] - p.mt[j][d]) / p.st[j][d];
      s += -0.5 * z * z;
    }
    if (small) {
      for (int d = 0; d < 3; ++d) {
        const double z = (0.0 - p.mw[j][d]) / p.sw[j][d];
        s += -0.5 * z * z;
      }
    } else {
      const double a = th + 2.0 * M_PI * m;
      s += 2.0 * log(fabs(a)) - log(2.0 * (1.0 - cos(th)));
      for (int d = 0; d < 3; ++d) {
        const double z = (a * w0[d] / th - p.mw[j][d]) / p.sw[j][d];
        s += -0.5 * z * z;
      }
    }
    term = s;
  }
  const double mx = wave_max_d(term);
  const double e = lane < n_terms ? exp(term - mx) : 0.0;
  return mx + log(wave_sum(e));
}

// Independence MH pose move, one workgroup of W waves per task (replica
// t.r of ligand t.lig, network outputs in row t.row).  The move is rigid, so
// the bonded energy does not change: only the grid terms and the restraint
// are evaluated at the proposed pose, and the bonded part of the energy is
// the cached one (the cached U_bond + U_angle + U_tors + U_I less the
// restraint energy of the current centre of mass).
template <int C, int W>
__global__ __launch_bounds__(W * kWave) void k_pose_move(
    GridDev g, const LigDev* __restrict__ ligs,
    const PropDev* __restrict__ props, const PoseTask* __restrict__ tasks,
    const float* __restrict__ out, uint64_t seed, int begin_next) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ float sR[9], st[3], scom[3];
  __shared__ int s_ok;
  __shared__ double s_ui0;
  const PoseTask task = tasks[blockIdx.x];
  const LigDev L = ligs[task.lig];
  const PropDev& P = props[task.lig];
  const int tid = threadIdx.x;
  const int r = task.r;
  const int n = L.n;
  const unsigned long long s = *L.counter;
  const int k = L.state_of_replica[r];
  const float* xr = L.x + (size_t)r * n * 3;
  // current pose, proposal and the proposal-density ratio (double): the
  // centre of mass by a block reduction, the mixture parsed one component
  // per lane, the two proposal densities one term per lane of wave 0, the
  // frames and the draws on thread 0
  __shared__ double s_cp[2 * W * 3];
  __shared__ Mix s_mix;
  __shared__ double s_pose[12];  // t0, w0, t1, w1p
  // per component: -3 ln 2 pi - sum_d (ln st + ln sw), then (once the
  // weights are normalised) plus its normalised log weight
  __shared__ double s_c0[kNComp];
  double lq_ratio = 0.0;
  {
    const bool own = tid < n;
    const double mi = own ? (double)L.mass[tid] : 0.0;
    const double cx = wave_sum(own ? mi * xr[3 * tid] : 0.0);
    const double cy = wave_sum(own ? mi * xr[3 * tid + 1] : 0.0);
    const double cz = wave_sum(own ? mi * xr[3 * tid + 2] : 0.0);
    const double cm = wave_sum(mi);
    if ((tid & 63) == 0) {
      const int wv = tid >> 6;
      s_cp[4 * wv] = cx;
      s_cp[4 * wv + 1] = cy;
      s_cp[4 * wv + 2] = cz;
      s_cp[4 * wv + 3] = cm;
    }
    // the mixture on the last wavefront (the one with the fewest atoms),
    // with each component's log-density constant but its weight
    const int j = tid - (W - 1) * kWave;
    if (j >= 0 && j < kNComp) {
      const float* o = out + (size_t)task.row * kNOut + 13 * j;
      s_mix.lw[j] = o[0];
      double c = -3.0 * log(2.0 * M_PI);
      for (int a = 0; a < 3; ++a) {
        s_mix.mt[j][a] = o[1 + a];
        s_mix.mw[j][a] = (float)M_PI * tanhf(o[4 + a]);
        const float sd_t = kSt0 + (kSt1 - kSt0) * sigm(o[7 + a]);
        const float sd_w = kSw0 + (kSw1 - kSw0) * sigm(o[10 + a]);
        s_mix.st[j][a] = sd_t;
        s_mix.sw[j][a] = sd_w;
        // single-precision logs: within 1e-6 of the double ones on the
        // deviations' range, far inside ln q's float error elsewhere
        c += -(double)logf(sd_t) - (double)logf(sd_w);
      }
      s_c0[j] = c;
    }
  }
  __syncthreads();
  // Two independent chains: A (thread 0) the current pose and the restraint
  // energy at the current centre of mass, B (thread 64, or thread 0 after A
  // in a one-wavefront block) the proposal; with two wavefronts they run
  // side by side.  Each computes the log-normaliser of the mixture weights
  // (log-softmax of the raw logits, float) with the same operations.
  __shared__ double s_R[2][9];  // R0, R1
  __shared__ double s_lq[2];
  const int tb = W >= 2 ? kWave : 0;
  if (tid == 0) {
    double c[3] = {0, 0, 0}, M = 0;
    for (int q = 0; q < W; ++q) {
      for (int d = 0; d < 3; ++d) c[d] += s_cp[4 * q + d];
      M += s_cp[4 * q + 3];
    }
    Frame F;
    body_frame(xr, P.frame, F);
    double R0[3][3], w0[3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) R0[a][b] = F.R[a][b];
    log_rot(R0, w0);
    double d2 = 0.0;
    for (int d = 0; d < 3; ++d) {
      c[d] /= M;
      s_pose[d] = c[d] - L.site[d];
      s_pose[3 + d] = w0[d];
      d2 += s_pose[d] * s_pose[d];
      scom[d] = (float)c[d];
    }
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) s_R[0][3 * a + b] = R0[a][b];
    // restraint energy at the current centre of mass (Eq. binding_site)
    const double ex0 = sqrt(d2) - (double)L.d0;
    s_ui0 = ex0 > 0.0 ? 0.5 * (double)L.krest * ex0 * ex0 : 0.0;
  }
  // the wavefront of lane tb: the components' weights and log-density
  // constants, one component per lane; the weights then go to every lane
  double wt[kNComp];
  if ((tid >> 6) == (tb >> 6)) {
    const float lse = mix_lse(s_mix);
    const int jj = tid - tb;
    double wj = 0.0;
    if (jj < kNComp) {
      const double lw = (double)(s_mix.lw[jj] - lse);
      wj = exp(lw);
      s_c0[jj] += lw;
    }
    for (int j = 0; j < kNComp; ++j) {
      const long long b = __double_as_longlong(wj);
      const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), j);
      const int hi = __builtin_amdgcn_readlane((int)(b >> 32), j);
      wt[j] = __longlong_as_double(((long long)hi << 32) |
                                   (long long)(unsigned)lo);
    }
  }
  if (tid == tb) {
    // component by inverse CDF, then (t, omega) by Gaussian draws
    const U4 o0 = draw(seed, 0u, L.id, r, s, kPose);
    const double u = u01d(o0.x);
    double cum[kNComp], tot = 0.0;
    for (int j = 0; j < kNComp; ++j) {
      tot += wt[j];
      cum[j] = tot;
    }
    int j = 0;
    while (j < kNComp - 1 && cum[j] < u * tot) ++j;
    float z[6];
    normals3(draw(seed, 1u, L.id, r, s, kPose), z[0], z[1], z[2]);
    normals3(draw(seed, 2u, L.id, r, s, kPose), z[3], z[4], z[5]);
    double t1[3], w1[3];
    for (int d = 0; d < 3; ++d) {
      t1[d] = (double)s_mix.mt[j][d] + (double)s_mix.st[j][d] * z[d];
      w1[d] = (double)s_mix.mw[j][d] + (double)s_mix.sw[j][d] * z[3 + d];
    }
    double R1[3][3];
    rodrigues(w1, R1);
    double w1p[3];
    log_rot(R1, w1p);  // principal rotation vector of the proposal
    for (int d = 0; d < 3; ++d) {
      s_pose[6 + d] = t1[d];
      s_pose[9 + d] = w1p[d];
      st[d] = (float)(L.site[d] + t1[d]);
    }
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) s_R[1][3 * a + b] = R1[a][b];
  }
  __syncthreads();
  // the two proposal densities, one term per lane: wave 0 at the current
  // pose, wave 1 (or wave 0 after that) at the proposal
  {
    const int wv = tid >> 6;
    if (W >= 2) {
      if (wv < 2) {
        const double lq = log_q_se3_wave(s_mix, s_c0, s_pose + 6 * wv,
                                         s_pose + 6 * wv + 3);
        if ((tid & 63) == 0) s_lq[wv] = lq;
      }
    } else {
      const double lq0 = log_q_se3_wave(s_mix, s_c0, s_pose, s_pose + 3);
      const double lq1 = log_q_se3_wave(s_mix, s_c0, s_pose + 6, s_pose + 9);
      if (tid == 0) {
        s_lq[0] = lq0;
        s_lq[1] = lq1;
      }
    }
  }
  if (tid == 0) {
    // x'_i = c0 + t' + R' R0^T (x_i - c): the rotation applied is R' R0^T
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double v = 0.0;
        for (int q = 0; q < 3; ++q) v += s_R[1][3 * a + q] * s_R[0][3 * b + q];
        sR[3 * a + b] = (float)v;
      }
  }
  __syncthreads();
  lq_ratio = s_lq[0] - s_lq[1];
  if (tid == 0) s_ok = isfinite(lq_ratio) ? 1 : 0;
  Shared sh{};
  sh.pos = reinterpret_cast<float4*>(smem);
  sh.red = reinterpret_cast<double*>(smem + 16 * kWave * W);
  sh.com = reinterpret_cast<float*>(smem + 16 * kWave * W + 8 * W * kRedMax);
  const bool owner = tid < n;
  float x2[3] = {0.f, 0.f, 0.f}, f[3];
  if (owner) {
    float y[3];
    for (int d = 0; d < 3; ++d) y[d] = xr[3 * tid + d] - scom[d];
    for (int a = 0; a < 3; ++a)
      x2[a] = st[a] + sR[3 * a] * y[0] + sR[3 * a + 1] * y[1] + sR[3 * a + 2] * y[2];
  }
  const float m = owner ? L.mass[tid] : 0.f;
  float sc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) sc[c] = owner ? L.scale[tid * C + c] : 0.f;
  float w[C];
  for (int c = 0; c < C; ++c) w[c] = L.wf[k * C + c];
  double t1e[6 + C];
  eval_block<C, W, false, true, true, false>(g, L, w, x2, m, sc, f, t1e, 0.f,
                                             0.f, sh, tid);
  const double* cp = L.comps + (size_t)r * (1 + C);
  const double ub = cp[0] - s_ui0;  // bonded energy, unchanged by the move
  double E1 = ub + t1e[3], E0 = cp[0];
  for (int c = 0; c < C; ++c) {
    E1 += L.wd[k * C + c] * t1e[4 + c];
    E0 += L.wd[k * C + c] * cp[1 + c];
  }
  __shared__ int s_acc;
  if (tid == 0) {
    const double ln_a = -L.beta[k] * (E1 - E0) + lq_ratio;
    const U4 ou = draw(seed, 3u, L.id, r, s, kPose);
    s_acc = (s_ok && isfinite(ln_a) && ln_u_below(ou.x, ln_a)) ? 1 : 0;
    P.last_ln_alpha[r] = ln_a;
    atomicAdd(&P.pose_try[k], 1ull);
    if (s_acc) atomicAdd(&P.pose_acc[k], 1ull);
  }
  __syncthreads();
  if (s_acc) {
    if (owner)
      for (int d = 0; d < 3; ++d) L.x[(size_t)r * n * 3 + 3 * tid + d] = x2[d];
    if (tid == 0) {
      double* cw = L.comps + (size_t)r * (1 + C);
      cw[0] = ub + t1e[3];
      for (int c = 0; c < C; ++c) cw[1 + c] = t1e[4 + c];
      L.fvalid[r] = 0;  // the stored start-of-trajectory forces are stale
    }
  }
  // the next run of neighbour-scheme sweeps starts from this replica's
  // state and (new or kept) components
  if (begin_next && tid == 0)
    begin_replica(L, r, k, s, *L.n_rec, L.comps + (size_t)r * (1 + C));
}

}  // namespace

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------
hipError_t launch_gemm(const GemmArgs& a, hipStream_t st) {
  if (a.M <= 0 || a.N <= 0) return hipSuccess;
  dim3 grid((a.N + kTile - 1) / kTile, (a.M + kTile - 1) / kTile);
  hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* P, const float* X, int B,
                              float* Z1, float* H1, float* Z2, float* H2,
                              float* out, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_forward, dim3((B + kFRows - 1) / kFRows),
                     dim3(kFWaves * 64), 0, st, P, X, B, Z1, H1, Z2, H2, out);
  return hipGetLastError();
}

hipError_t launch_pose_network(const MlpGroup* groups, int n_groups,
                               const LigDev* ligs, const PropDev* props,
                               const PoseTask* tasks, float* out,
                               const LigDev* fin, int n_fin,
                               int exchange_every, int sample_every,
                               uint64_t seed, hipStream_t st) {
  if (n_groups + n_fin <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pose_network, dim3(n_groups + n_fin),
                     dim3(kFWaves * 64), 0, st, groups, n_groups, ligs, props,
                     tasks, out, fin, exchange_every, sample_every, seed);
  return hipGetLastError();
}

hipError_t launch_weights_bf16(const float* P, unsigned short* WT,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_weights_bf16, dim3((kTSize + 255) / 256), dim3(256), 0,
                     st, P, WT);
  return hipGetLastError();
}

hipError_t launch_colsum(const float* X, int rows, int cols, int64_t ld,
                         float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_colsum, dim3((cols + 63) / 64), dim3(256), 0, st, X,
                     rows, cols, ld, out);
  return hipGetLastError();
}

hipError_t launch_nll(const float* out, const float* pose, int B,
                      float* dout, double* loss_part, hipStream_t st) {
  hipLaunchKernelGGL(k_nll, dim3((B + 255) / 256), dim3(256), 0, st, out,
                     pose, B, 1.0f / (float)B, dout, loss_part);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n,
                       float lr, float b1, float b2, float eps, float c1,
                       float c2, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, p, g, m,
                     v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_pose_features(const LigDev* lig, const PropDev* prop,
                                const float* xs, int64_t N, float* feats,
                                float* poses, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pose_features, dim3((unsigned)((N + 127) / 128)),
                     dim3(128), 0, st, lig, prop, xs, N, feats, poses);
  return hipGetLastError();
}


hipError_t launch_pose_move(const GridDev& g, const LigDev* ligs,
                            const PropDev* props, const PoseTask* tasks,
                            int n, const float* out, int waves, int lds,
                            uint64_t seed, bool begin_next, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  switch (g.C) {
    case 3:
      if (waves == 1)
        hipLaunchKernelGGL((k_pose_move<3, 1>), dim3(n), dim3(64), lds, st, g,
                           ligs, props, tasks, out, seed, begin_next ? 1 : 0);
      else
        hipLaunchKernelGGL((k_pose_move<3, 2>), dim3(n), dim3(128), lds, st, g,
                           ligs, props, tasks, out, seed, begin_next ? 1 : 0);
      break;
    case 5:
      if (waves == 1)
        hipLaunchKernelGGL((k_pose_move<5, 1>), dim3(n), dim3(64), lds, st, g,
                           ligs, props, tasks, out, seed, begin_next ? 1 : 0);
      else
        hipLaunchKernelGGL((k_pose_move<5, 2>), dim3(n), dim3(128), lds, st, g,
                           ligs, props, tasks, out, seed, begin_next ? 1 : 0);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace bpmf

namespace bpmf {
namespace {
// minibatch gather: row i of step s is row philox(s, i) mod N (sampling with
// replacement)
__global__ __launch_bounds__(256) void k_gather(
    const float* __restrict__ feats, const float* __restrict__ poses,
    int64_t N, int B, uint64_t seed, uint64_t step, float* __restrict__ bf,
    float* __restrict__ bp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  const U4 o = philox4x32_10((uint32_t)i, (uint32_t)(step >> 32),
                             (uint32_t)step, kBatch, (uint32_t)seed,
                             (uint32_t)(seed >> 32));
  const uint64_t r = ((uint64_t)o.x << 32) | o.y;
  const int64_t j = (int64_t)(r % (uint64_t)N);
  for (int q = 0; q < kNFeat; ++q) bf[(int64_t)i * kNFeat + q] = feats[j * kNFeat + q];
  for (int q = 0; q < 6; ++q) bp[(int64_t)i * 6 + q] = poses[j * 6 + q];
}
}  // namespace

hipError_t launch_gather_batch(const float* feats, const float* poses,
                               int64_t N, int B, uint64_t seed,
                               uint64_t step, float* bf, float* bp,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_gather, dim3((B + 255) / 256), dim3(256), 0, st, feats,
                     poses, N, B, seed, step, bf, bp);
  return hipGetLastError();
}
}  // namespace bpmf
