// Learned pose proposal: network shape, parameter layout, device state and
// launchers (mlp.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace bpmf {

constexpr int kNFeat = 16, kNHid = 256, kNComp = 8, kNOut = kNComp * 13;
constexpr int kFold = 3;  // preimages (theta + 2 pi m) n, m = -3..3
constexpr float kSt0 = 0.02f, kSt1 = 3.0f;  // translation sigma range (A)
constexpr float kSw0 = 0.02f, kSw1 = 1.5f;  // rotation sigma range (rad)

// flat fp32 parameter vector: W1 (16x256) b1 W2 (256x256) b2 W3 (256x104) b3,
// weights row-major [in][out]
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kNFeat * kNHid;
constexpr int kOffW2 = kOffB1 + kNHid;
constexpr int kOffB2 = kOffW2 + kNHid * kNHid;
constexpr int kOffW3 = kOffB2 + kNHid;
constexpr int kOffB3 = kOffW3 + kNHid * kNOut;
constexpr int kNParams = kOffB3 + kNOut;

// bf16 copy of the weights for the pose moves' forward pass, each matrix
// transposed ([out][in]) with rows padded so that a lane's eight
// consecutive k values are one 16-byte load and every 16-column output tile
// is in range: W1^T 256 x 32, W2^T 256 x 256, W3^T 112 x 256 (padding 0)
constexpr int kT1Ld = 32, kT2Ld = kNHid, kT3Ld = kNHid, kT3Rows = 112;
constexpr int kTOff1 = 0;
constexpr int kTOff2 = kTOff1 + kNHid * kT1Ld;
constexpr int kTOff3 = kTOff2 + kNHid * kT2Ld;
constexpr int kTSize = kTOff3 + kT3Rows * kT3Ld;

enum Purpose2 : uint32_t { kPose = 4, kBatch = 5 };

// Device state of one ligand's proposal.
struct PropDev {
  int frame[3];
  int n_cond;
  int4 cond[8];
  unsigned long long* pose_acc;  // K
  unsigned long long* pose_try;  // K
  double* last_ln_alpha;         // K, ln alpha of each replica's last move
};

// One replica of a batch of pose moves over several ligands: its ligand's
// table index, the replica, and its row in the batch's features, poses and
// network outputs.
struct PoseTask {
  int lig, r, row, pad;
};

// One workgroup of a batched forward pass: rows [row0, row0 + rows) (at
// most 16) through the network whose parameters start at P.
struct MlpGroup {
  const float* P;             // fp32 parameters (the biases are read here)
  const unsigned short* WT;   // bf16 transposed weights (kTSize)
  int row0, rows;
};

enum { kEpiStore = 0, kEpiSilu = 1, kEpiDsilu = 2 };

// C[m, n] = sum_k A(m, k) B(k, n) (+ bias[n]); A(m, k) = A[m*sam + k*sak],
// B(k, n) = B[k*sbk + n*sbn]; bf16 operands, fp32 accumulation.
// kEpiSilu: Zout = acc + bias, C = silu(Zout).  kEpiDsilu: C = acc *
// silu'(Zin).  Row stride of C, Zout, Zin: ldc.
struct GemmArgs {
  int M, N, K;
  const float* A;
  int64_t sam, sak;
  const float* B;
  int64_t sbk, sbn;
  float* C;
  int64_t ldc;
  const float* bias;
  int epi;
  float* Zout;
  const float* Zin;
};

hipError_t launch_gemm(const GemmArgs& a, hipStream_t st);
// the whole network for B rows (features B x kNFeat): Z1, H1, Z2, H2 (B x
// kNHid) and out (B x kNOut), equal to three launch_gemm calls
hipError_t launch_mlp_forward(const float* P, const float* X, int B,
                              float* Z1, float* H1, float* Z2, float* H2,
                              float* out, hipStream_t st);
hipError_t launch_colsum(const float* X, int rows, int cols, int64_t ld,
                         float* out, hipStream_t st);
hipError_t launch_nll(const float* out, const float* pose, int B, float* dout,
                      double* loss_part, hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n,
                       float lr, float b1, float b2, float eps, float c1,
                       float c2, hipStream_t st);
hipError_t launch_pose_features(const LigDev* lig, const PropDev* prop,
                                const float* xs, int64_t N, float* feats,
                                float* poses, hipStream_t st);
// the network on the current configurations of tasks [row0, row0 + rows)
// of every group (features computed in place), outputs only; n_fin further
// blocks close the neighbour-scheme run of ligands fin[0..n_fin) as
// launch_sweep_finish does
hipError_t launch_pose_network(const MlpGroup* groups, int n_groups,
                               const LigDev* ligs, const PropDev* props,
                               const PoseTask* tasks, float* out,
                               const LigDev* fin, int n_fin,
                               int exchange_every, int sample_every,
                               uint64_t seed, hipStream_t st);
// the bf16 transposed copy of the weights of parameter vector P
hipError_t launch_weights_bf16(const float* P, unsigned short* WT,
                               hipStream_t st);
// one pose move of each of the n tasks (all of `waves` wavefronts; props
// indexed by ligand table index, out by task row); begin_next: each task's
// replica then starts the next run of neighbour-scheme sweeps
// (begin_replica), in place of launch_sweep_begin
hipError_t launch_pose_move(const GridDev& g, const LigDev* ligs,
                            const PropDev* props, const PoseTask* tasks,
                            int n, const float* out, int waves, int lds,
                            uint64_t seed, bool begin_next, hipStream_t st);
hipError_t launch_gather_batch(const float* feats, const float* poses,
                               int64_t N, int B, uint64_t seed,
                               uint64_t step, float* bf, float* bp,
                               hipStream_t st);

}  // namespace bpmf
