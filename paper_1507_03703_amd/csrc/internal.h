// Structures shared by the host side of libbpmf and its gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pairs.h"

namespace bpmf {

constexpr int kWave = 64;
constexpr double kRGas = 8.314462618e-3;  // kJ/(mol K)
#define BPMF_MAX_MBAR_STATES_DEV 128
constexpr int kRedSlots = 4 + 8 + 2;  // per-wave partial sums (see Shared)

// copies of the fixed-point force accumulators: a bonded-term lane adds
// into copy (lane mod kAccCopies), which divides the lanes of one LDS
// atomic instruction that meet the same atom among that many addresses
constexpr int kAccCopies = 4;

// LDS bytes of the fixed-point force accumulators (kAccCopies x n x 3
// int32), rounded up to 16 so that the topology staged after them stays
// 16-byte aligned
__host__ __device__ inline int acc_lds_bytes(int n) {
  return (kAccCopies * 12 * n + 15) & ~15;
}

// Bonded terms are taken in chunks of 64 terms of one kind (a wavefront
// takes a chunk in one pass): torsion chunks, then angle chunks, then bond
// chunks.  The schedule of a ligand gives, for each launch width (1, 2, 4,
// 8 wavefronts), the chunks of each wavefront: a row of 9 offsets
// (wavefront w takes entries off[w] .. off[w+1]-1) followed by the chunk
// ids, stored as 16-bit values.
__host__ __device__ inline int bonded_chunks(int nb, int na, int nt) {
  return (nt + kWave - 1) / kWave + (na + kWave - 1) / kWave +
         (nb + kWave - 1) / kWave;
}
__host__ __device__ inline int sched_row(int nb, int na, int nt) {
  return 9 + bonded_chunks(nb, na, nt);
}

// dynamic LDS bytes of a W-wave evaluation block: per-evaluation areas,
// force accumulators (forces only), the staged topology (with the schedule
// row of this width) and, with pair terms in the energy, the pair
// parameters and scratch
__host__ __device__ inline int block_lds_bytes(int waves, bool forces, int n,
                                                int nb, int na, int nt,
                                                bool pairs = false) {
  const int head = 16 * kWave * waves + 8 * waves * kRedSlots + 16 * waves +
                   (forces ? acc_lds_bytes(n) : 0);
  const int topo = 32 * nt + 24 * na + 16 * nb +
                   ((2 * sched_row(nb, na, nt) + 15) & ~15);
  return head + topo + (pairs ? pair_lds_bytes(n, waves) : 0);
}

// LDS of a k_energy_matrix_wave block: the states' weights and beta_k, then
// per wavefront its positions (64 AP float4) and the columns of a group of
// kUknWaveGroup samples, then the ligand's topology (as stage_topology lays
// it out)
constexpr int kUknWaves = 4, kUknWaveGroup = 8;
__host__ __device__ inline int ukn_wave_head_bytes(int K, int C) {
  return (K * (C + 1) * 8 + 15) & ~15;
}
__host__ __device__ inline int ukn_wave_slot_bytes(int K, int ap) {
  return 16 * kWave * ap + kUknWaveGroup * K * 8;
}
__host__ __device__ inline int ukn_wave_lds_bytes(int K, int C, int ap,
                                                  int nb, int na, int nt) {
  return ukn_wave_head_bytes(K, C) + kUknWaves * ukn_wave_slot_bytes(K, ap) +
         32 * nt + 24 * na + 16 * nb +
         ((2 * sched_row(nb, na, nt) + 15) & ~15);
}

enum Purpose : uint32_t { kMomenta = 1, kAccept = 2, kExchange = 3 };

// Floats per cell record of the cell-major grid: the 8 corners x C channels
// rounded up to a power of two, so that a record of up to 4 channels is one
// aligned 128-byte cache line.
constexpr int cell_stride(int C) {
  return 8 * C <= 8 ? 8 : 8 * C <= 16 ? 16 : 8 * C <= 32 ? 32 : 64;
}

// Receptor grid as the kernels see it, cell-major: cell (i, j, k) (i < nx-1,
// j < ny-1, k < nz-1) owns the record at cells + ((k*(ny-1) + j)*(nx-1) + i)
// * cell_stride(C) holding the values of its corners, corner q = (i + (q&1),
// j + ((q>>1)&1), k + (q>>2)) at [q*C + c] for channel c.  Each node value
// appears in up to 8 records: one interpolation reads one record instead of
// 8 scattered corners.  Channel c holds a quartic root when bit c of
// quartic_mask is set.
struct GridDev {
  const float* cells;
  int nx, ny, nz, C;
  float ox, oy, oz, inv_h;
  int quartic_mask;
};

// One ligand: force field, state ladder, replica state, statistics and the
// sample store, all resident in device memory.  Replica r of a ligand with
// K states owns x[r*n*3 .. (r+1)*n*3).
struct LigDev {
  int n, K, C;
  int nb, na, nt, n_slots;
  int id;     // ligand id (enters the random-number counter)
  int cap;    // recorded samples per state
  float site[3];
  float d0, krest, inv_total_mass;
  const float* mass;      // n
  const float* inv_mass;  // n
  const float* scale;     // n*C
  const int2* bij;        // nb
  const float2* bpar;     // nb: K_r, r0
  const int4* aijk;       // na: i, j(vertex), k, -
  const float2* apar;     // na: K_theta, theta0
  const int4* tijkl;      // nt
  const float4* tpar;     // nt: V/2, n (integer 1..6), cos gamma, sin gamma
  const unsigned short* bsched;  // 4 x sched_row: bonded chunks per wavefront
  const double* beta;     // K: 1/(R T_k)
  const float* Tf;        // K
  const float* dtf;       // K
  const float* wf;        // K*C
  const double* wd;       // K*C
  float* x;               // K*n*3
  double* comps;          // K*(1+C)
  int* state_of_replica;  // K
  int* replica_of_state;  // K
  unsigned long long* counter;    // sweeps done
  unsigned long long* n_rec;      // recorded rounds
  unsigned long long* hmc_acc;    // K
  unsigned long long* hmc_try;    // K
  unsigned long long* ex_acc;     // max(K-1,1)
  unsigned long long* ex_try;     // max(K-1,1)
  unsigned long long* nonfinite;  // 1
  unsigned long long* ext_acc;    // K: external moves accepted per state
  unsigned long long* ext_try;    // K: external moves tried per state
  // Neighbour-scheme sweeps apply the exchange (and record) that ends sweep
  // s-1 at the start of sweep s, in every replica's own block: sweep s
  // reads buffer (s-1)&1 and writes buffer s&1 (k_sweep_begin fills the
  // first from the canonical arrays above, k_sweep_finish applies the last
  // pending exchange and writes them back).
  unsigned long long* rcnt;   // K: sweep counter of each replica
  unsigned long long* rnrec;  // K: recorded rounds seen by each replica
  int* rpend;                 // 2K: exchange/record of the previous sweep due
  int* rsor;                  // 2K: state of each replica
  double* scomp;              // 2K(1+C): components of the replica in each state
  // start-of-trajectory force reuse: per replica two slots of the parts of
  // the force at its current positions that do not depend on the state
  // (per atom: bonded force, grid gradients of every channel; per replica:
  // restraint factor and centre-of-mass offset); fvalid[r] = 0 (none) or
  // 1 + the slot holding the current positions' parts
  float* fcache;              // 2K x n x (3 + 3C)
  float* frc;                 // 2K x 4
  int* fvalid;                // K
  float* samp_x;                  // cap*K*n*3
  double* samp_c;                 // cap*K*(1+C)
  // intramolecular nonbonded and OBC GB/SA terms in the sampled energy
  // (bpmf_pair_sample): on when pairs_on, parameters in `pair`
  int pairs_on;
  PairDev pair;
};

// Every region of a ligand's device arena starts on a 256-byte boundary.
constexpr size_t kArenaAlign = 256;

// Round-trip bookkeeping (kept out of the table, whose every field the
// sweep kernel holds in scalar registers), in the arena region right after
// fvalid: per replica the extreme state it last visited on its way (0 =
// state 0, 1 = state K-1, -1 = neither yet), then, 8-byte aligned, the
// ligand's trip count.
__host__ __device__ inline int* rt_end_of(const LigDev& L) {
  const size_t b = ((size_t)L.K * 4 + kArenaAlign - 1) & ~(kArenaAlign - 1);
  return (int*)((char*)L.fvalid + b);
}
__host__ __device__ inline unsigned long long* round_trips_of(
    const LigDev& L) {
  return (unsigned long long*)(rt_end_of(L) + ((L.K + 1) & ~1));
}
__host__ __device__ inline size_t rt_region_bytes(int K) {
  return (size_t)((K + 1) & ~1) * 4 + 8;
}

// Launch wrappers (kernels.hip).  All return hipError_t of the launch.
// waves = wavefronts per replica (1, 2 or 4); n_atoms <= 64 * waves
// exchange/record schedule of a sweep (scheme 0: deferred into the next
// sweep's blocks; scheme 1: a tail kernel after every sweep, running
// exchange_sweeps exchange sweeps when an exchange is due)
struct TailArgs {
  int exchange_every, scheme, max_sep, sample_every, exchange_sweeps;
};
// one: the host copy of the table entry when the launch covers a single
// ligand (its replicas 0..n_tasks-1 in order), else null
// pairs: some ligand of the launch has its pair terms in the energy
hipError_t launch_hmc_sweep(const GridDev& g, const LigDev* d_ligs,
                            const int2* d_tasks, int n_tasks, int waves,
                            int lds_bytes, int nleap, uint64_t seed,
                            TailArgs tail, const LigDev* one, bool pairs,
                            hipStream_t st);
hipError_t launch_sweep_tail(const LigDev* d_ligs, int n_ligs,
                             int exchange_every, int scheme, int max_sep,
                             int n_sub, int sample_every, uint64_t seed,
                             hipStream_t st);
hipError_t launch_sweep_begin(const LigDev* d_ligs, int n_ligs,
                              hipStream_t st);
hipError_t launch_sweep_finish(const LigDev* d_ligs, int n_ligs,
                               int exchange_every, int sample_every,
                               uint64_t seed, hipStream_t st);
// n_sub exchange sweeps in a row (sweep j draws with replica field j)
hipError_t launch_exchange(const LigDev* d_lig, int n_ligs, int scheme,
                           int max_sep, int n_sub, uint64_t seed,
                           hipStream_t st);
// one ligand's share of an energy-matrix launch: samples xs (n x n_atoms x
// 3), output u_kn (K x ld); its samples are [first, first + n) of the
// launch's flat sample index
struct UknJob {
  int lig;   // index into the ligand table
  int cost;  // estimated cost of one sample (instruction-issue units)
  const float* xs;
  double* ukn;
  int64_t n, ld;
  int64_t first;   // flat index of the job's first sample
  int64_t cfirst;  // cost of the launch's samples before the job's first
};
// d_jobs: n_jobs jobs in flat order, every ligand needing `waves`
// wavefronts, then a sentinel with first = total and cfirst = the launch's
// total cost (each block takes a contiguous share of equal cost); group = samples whose
// columns are staged in LDS before they are written.  per_wave: one
// wavefront per sample (k_energy_matrix_wave, for ligands whose pair terms
// are not in the energy; `waves` is then the atoms per lane, 1 or 2, and
// lds_bytes comes from ukn_wave_lds_bytes)
hipError_t launch_energy_matrix(const GridDev& g, const LigDev* d_ligs,
                                int waves, const UknJob* d_jobs, int n_jobs,
                                int64_t total, int group, int lds_bytes,
                                int n_cu, bool pairs, bool per_wave,
                                hipStream_t st);
// copy n jobs from host memory into the device table dst by kernels that
// take the jobs as arguments (no host staging buffer, no copy engine)
hipError_t launch_put_jobs(UknJob* dst, const UknJob* jobs, int n,
                           hipStream_t st);
hipError_t launch_evaluate(const GridDev& g, const LigDev* d_lig,
                           int waves, const float* xs, int64_t N,
                           const double* w, double* terms, float* forces,
                           int lds_bytes, hipStream_t st);
// cell-major records (GridDev) from a node-major grid nodes[((k*ny + j)*nx +
// i)*C + c]
hipError_t launch_expand_cells(const float* nodes, int nx, int ny, int nz,
                               int C, float* cells, hipStream_t st);
hipError_t launch_grid_eval(const GridDev& g, const float* pos,
                            const float* scale, int64_t n, const double* w,
                            float* energy, float* force, hipStream_t st);
hipError_t launch_recompute_comps(const GridDev& g, const LigDev* d_lig,
                                  int waves, int K, int lds_bytes, bool pairs,
                                  hipStream_t st);

// MBAR kernels (mbar.hip).  One entry per problem of a batch, in device
// memory; kernels take the table and a device list of problem indices and
// put the list position in blockIdx.y.
struct MbarProb {
  const double* ukn;  // K x N, leading dimension ld
  int64_t N, ld;
  int K;
  int nb;             // blocks of the logD / objective pass
  int nb_acc;         // blocks of the W W^T accumulation
  int ts;             // register tile of the accumulation (mbar_acc_ts)
  double* f;          // K current point (f_0 = 0)
  double* ftry;       // K line-search trial
  double* logN;       // K
  double* Nk;         // K
  double* logD;       // N
  double* partial;    // max(nb, nb_acc) x (K + K*K)
  double* red;        // K + K*K reduced sums
  double* mat;        // (K-1) x (2K-1) augmented system (large K only)
  double* step;       // K Newton step / fixed-point values
  double* scalars;    // [0] objective [1] max|step| [2] g.step [3] status
                      // [4] fixed-point change
  double* var;        // K variances
  double* obj_part;   // nb
};
int mbar_logD_blocks(int64_t N);
int mbar_acc_ts(int K);
int mbar_acc_blocks(int K, int64_t N);
size_t mbar_newton_lds(int K, int want_inverse);
// logD and scalars[0] at f (use_try = 0) or ftry
hipError_t mbar_objective(const MbarProb* P, const int* list, int n,
                          int max_nb, int use_try, hipStream_t st);
// fixed-point update of f in place (logD current for f), change in [4]
hipError_t mbar_fixed_point(const MbarProb* P, const int* list, int n,
                            int max_K, hipStream_t st);
// partial sums of W W^T at f; every listed problem has register tile ts
hipError_t mbar_accumulate(const MbarProb* P, const int* list, int n, int ts,
                           int max_blocks, hipStream_t st);
// reduce the partial sums and solve for the Newton step (and variances)
hipError_t mbar_newton(const MbarProb* P, const int* list, int n, int max_K,
                       int want_inverse, hipStream_t st);
hipError_t mbar_axpy(const MbarProb* P, const int* list, int n,
                     const double* tvec, hipStream_t st);
hipError_t mbar_accept(const MbarProb* P, const int* list, int n,
                       hipStream_t st);

}  // namespace bpmf
