// gfx950 kernels of the BPMF sampling hot path: HMC sweep, replica exchange,
// sample recording, per-sample energy components, u_kn expansion, and the
// exposed energy/force and grid evaluators.
#include <hip/hip_runtime.h>
#include <math.h>

#include "deferred.h"
#include "device.h"
#include "internal.h"

namespace bpmf {

namespace {

// Dynamic LDS of a W-wave block: positions (64 W float4), per-wave partial
// sums, centre-of-mass partials, n_acc x 3 fixed-point force accumulators,
// then the ligand's topology (staged once per launch).
template <int W, bool SYNC = true>
__device__ __forceinline__ Shared carve(unsigned char* raw, const LigDev& L,
                                        int n_acc, int tid) {
  Shared sh;
  sh.pos = reinterpret_cast<float4*>(raw);
  sh.red = reinterpret_cast<double*>(raw + 16 * kWave * W);
  sh.com = reinterpret_cast<float*>(raw + 16 * kWave * W +
                                    8 * W * kRedMax);
  // offset arithmetic on the LDS base keeps the pointers in LDS space;
  // force accumulators exist when n_acc > 0 (force-evaluating kernels)
  const int acc0 = 16 * kWave * W + 8 * W * kRedMax + 16 * W;
  sh.sl = Slots{(lds_u32*)(raw + acc0), 3 * n_acc};
  for (int i = tid; i < kAccCopies * 3 * n_acc; i += W * kWave)
    sh.sl.acc[i] = 0u;
  stage_topology(L, raw + acc0 + acc_lds_bytes(n_acc), sh, tid, W * kWave);
  // SYNC false: the caller issues more work before its own barrier
  if (SYNC) __syncthreads();
  return sh;
}

// block-wide double sums of two per-thread floats (fixed order); W0: the
// sums are needed (and formed) in wavefront 0 only, 0 elsewhere
template <int W, bool W0 = false>
__device__ __forceinline__ void block_sum2(float a, float b, double* buf,
                                           int tid, double& sa, double& sb) {
  const double wa = wave_sum((double)a), wb = wave_sum((double)b);
  if ((tid & (kWave - 1)) == 0) {
    buf[2 * (tid >> 6)] = wa;
    buf[2 * (tid >> 6) + 1] = wb;
  }
  block_sync();
  sa = 0.0;
  sb = 0.0;
  if (W0 && tid >= kWave) return;
#pragma unroll
  for (int q = 0; q < W; ++q) {
    sa += buf[2 * q];
    sb += buf[2 * q + 1];
  }
}

// ----------------------------------------------------------------------------
// replica exchange (Eq. repXacc), state labels swapped
// ----------------------------------------------------------------------------
#pragma clang fp contract(off)
__device__ double state_energy(const LigDev& L, int k, int rep) {
  const double* cp = L.comps + (size_t)rep * (1 + L.C);
  double E = cp[0];
  for (int c = 0; c < L.C; ++c) E += L.wd[k * L.C + c] * cp[1 + c];
  return E;
}

__device__ bool attempt_pair(const LigDev& L, int a, int b, int sep,
                             uint64_t sweep, int sub, uint64_t seed) {
  const int ra = L.replica_of_state[a], rb = L.replica_of_state[b];
  const double ba = L.beta[a], bb = L.beta[b];
  const double delta =
      ba * (state_energy(L, a, rb) - state_energy(L, a, ra)) +
      bb * (state_energy(L, b, ra) - state_energy(L, b, rb));
  const uint32_t purpose = (uint32_t)kExchange | ((uint32_t)sep << 8);
  const U4 o = draw(seed, (uint32_t)a, L.id, sub, sweep, purpose);
  const double lnu = log(u01d(o.x));
  const bool ok = isfinite(delta) && (lnu < -delta);
  if (sep == 1) atomicAdd(&L.ex_try[a], 1ull);
  if (ok) {
    L.replica_of_state[a] = rb;
    L.replica_of_state[b] = ra;
    L.state_of_replica[ra] = b;
    L.state_of_replica[rb] = a;
    if (sep == 1) atomicAdd(&L.ex_acc[a], 1ull);
  }
  return ok;
}

// The all-separations sweep with the state data staged in LDS.  Within one
// separation d, pair (a, a + d) only touches states of residue a mod d, so
// the d residue classes are independent chains, each taken in ascending a.
// A chain is a sequence of runs: the replica of the run's first state q is
// carried up the chain while its swaps are accepted and stays at the state
// where one is rejected (or where the chain ends); the next run starts one
// step further up with that state's own replica.  When pair (a, a + d) is
// attempted, state a + d still holds its replica from the start of the
// pass, so the run that starts at q depends only on q and the labels at
// the start of the pass.  Every possible run is therefore followed at once,
// one thread per first state; then one thread per class walks the runs that
// actually happen (first state of the class, then one state past each
// run's end) and every state takes its new replica.  The energies are the
// same double sums as state_energy and each attempt sees the replicas the
// one-thread order gives it, so every decision is that order's.
constexpr int kXStates = 256, kXChannels = 5;
struct XStage {
  double cp[kXStates * (1 + kXChannels)];  // components per replica
  double wd[kXStates * kXChannels];        // weights per state
  double beta[kXStates];
  double ecur[2][kXStates];  // energy of the replica in state k at state k
  double lnu[2][kXStates];   // ln u of a pass, by lower state (two buffers)
  double eo[kXStates];       // energy of the replica in a + d at state a
  double erest[kXStates];    // run from q: energy of its replica where it stays
  int ros[2][kXStates];      // replica of each state (two buffers)
  int rest[kXStates];        // run from q: the state where its replica stays
  int owner[kXStates];       // first state of the run that ends at k, or -1
  int ntry[kXStates], nacc[kXStates];  // separation-1 counts, by lower state
};

// state-k energy of components v, in the order of state_energy
template <int C>
__device__ __forceinline__ double staged_sum(const double (&v)[1 + C],
                                             const double (&u)[C]) {
  double E = v[0];
#pragma unroll
  for (int c = 0; c < C; ++c) E += u[c] * v[1 + c];
  return E;
}
template <int C>
__device__ __forceinline__ double staged_energy(const XStage& X, int k,
                                                int r) {
  double v[1 + C], u[C];
#pragma unroll
  for (int e = 0; e <= C; ++e) v[e] = X.cp[r * (1 + C) + e];
#pragma unroll
  for (int c = 0; c < C; ++c) u[c] = X.wd[k * C + c];
  return staged_sum<C>(v, u);
}

// ladders of up to kXTable states also keep the whole table E(k, r) of
// every replica's energy at every state, computed once per call: a run
// step then reads one entry instead of summing components
constexpr int kXTable = 64;

template <int C, bool TABLE>
__device__ void exchange_all_staged(const LigDev& L, uint64_t sweep,
                                    int max_sep, int n_sub, uint64_t seed,
                                    XStage& X, double* em) {
  const int K = L.K, C1 = 1 + C;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i < K * C1; i += nt) X.cp[i] = L.comps[i];
  for (int i = tid; i < K * C; i += nt) X.wd[i] = L.wd[i];
  for (int k = tid; k < K; k += nt) {
    X.beta[k] = L.beta[k];
    X.ros[0][k] = L.replica_of_state[k];
    X.ntry[k] = 0;
    X.nacc[k] = 0;
  }
  __syncthreads();
  for (int k = tid; k < K; k += nt)
    X.ecur[0][k] = staged_energy<C>(X, k, X.ros[0][k]);
  if (TABLE)
    for (int q = tid; q < K * K; q += nt)
      em[(q / K) * kXTable + q % K] = staged_energy<C>(X, q / K, q % K);
  __syncthreads();
  int cur = 0, lb = 0;
  const int dmax = max_sep < K - 1 ? max_sep : K - 1;
  // ln u of the pass (j, d) into buffer b, by threads t0, t0 + stride, ...
  auto draw_pass = [&](int j, int d, int b, int t0, int stride) {
    const uint32_t purpose = (uint32_t)kExchange | ((uint32_t)d << 8);
    for (int a = t0; a + d < K; a += stride)
      X.lnu[b][a] =
          log(u01d(draw(seed, (uint32_t)a, L.id, j, sweep, purpose).x));
  };
  if (n_sub > 0 && dmax > 0) draw_pass(0, 1, 0, tid, nt);
  for (int j = 0; j < n_sub; ++j) {
    for (int d = 1; d <= dmax; ++d) {
      const int* ros = X.ros[cur];
      const double* ecur = X.ecur[cur];
      const double* lnu = X.lnu[lb];
      // the upper replica's energy at the lower state
      for (int a = tid; a < K; a += nt) {
        X.owner[a] = -1;
        if (a + d < K)
          X.eo[a] = TABLE ? em[a * kXTable + ros[a + d]]
                          : staged_energy<C>(X, a, ros[a + d]);
      }
      __syncthreads();
      // the run that starts at q, for every q; each step's operands are
      // loaded while the step before it is decided
      for (int q = tid; q < K; q += nt) {
        int a = q;
        double e = ecur[q];  // energy of the carried replica at state a
        if (q + d < K) {
          const int r = ros[q];
          double v[1 + C], wb[C], et = 0.0;
          if (!TABLE)
#pragma unroll
            for (int i = 0; i <= C; ++i) v[i] = X.cp[r * C1 + i];
          int b = a + d;
          double ba = X.beta[a], eoa = X.eo[a], lna = lnu[a];
          double bb = X.beta[b], ebb = ecur[b];
          if (TABLE)
            et = em[b * kXTable + r];
          else
#pragma unroll
            for (int c = 0; c < C; ++c) wb[c] = X.wd[b * C + c];
          for (;;) {
            // the next step's operands (unused when this step ends the run)
            const int b2 = b + d < K ? b + d : b;
            const double neo = X.eo[b], nln = lnu[b];
            const double nbb = X.beta[b2], neb = ecur[b2];
            double nwb[C], net = 0.0;
            if (TABLE)
              net = em[b2 * kXTable + r];
            else
#pragma unroll
              for (int c = 0; c < C; ++c) nwb[c] = X.wd[b2 * C + c];
            // the carried replica at state b
            const double eba = TABLE ? et : staged_sum<C>(v, wb);
            const double delta = ba * (eoa - e) + bb * (eba - ebb);
            const bool ok = isfinite(delta) && (lna < -delta);
            if (!ok) break;
            e = eba;
            a = b;
            if (a + d >= K) break;
            b = b2;
            ba = bb;
            eoa = neo;
            lna = nln;
            bb = nbb;
            ebb = neb;
            et = net;
#pragma unroll
            for (int c = 0; c < C; ++c) wb[c] = nwb[c];
          }
        }
        X.rest[q] = a;
        X.erest[q] = e;
      }
      __syncthreads();
      // the next pass's uniforms, by the threads past the first wavefront
      // while it walks (by every thread, before its walk, in a block of
      // one wavefront)
      {
        const int dn = d < dmax ? d + 1 : 1, jn = d < dmax ? j : j + 1;
        const int t0 = nt > kWave ? kWave : 0;
        if (jn < n_sub && tid >= t0)
          draw_pass(jn, dn, lb ^ 1, tid - t0, nt - t0);
      }
      // the runs that happen: from the class's first state, each one
      // starting one step past the previous one's end
      for (int rho = tid; rho < d; rho += nt)
        for (int q = rho; q < K;) {
          const int a = X.rest[q];
          X.owner[a] = q;
          q = a + d;
        }
      __syncthreads();
      // a state where a run ends takes the run's replica; any other state
      // had its swap with the state d above accepted
      int* nros = X.ros[cur ^ 1];
      double* necur = X.ecur[cur ^ 1];
      for (int a = tid; a < K; a += nt) {
        const int q = X.owner[a];
        if (q >= 0) {
          nros[a] = ros[q];
          necur[a] = X.erest[q];
        } else {
          nros[a] = ros[a + d];
          necur[a] = X.eo[a];
        }
        if (d == 1 && a + 1 < K) {
          X.ntry[a] += 1;
          X.nacc[a] += (int)(q < 0);
        }
      }
      cur ^= 1;
      lb ^= 1;
      __syncthreads();
    }
  }
  for (int k = tid; k < K; k += nt) {
    const int r = X.ros[cur][k];
    L.replica_of_state[k] = r;
    L.state_of_replica[r] = k;
    if (k + 1 < K && X.ntry[k]) {
      atomicAdd(&L.ex_try[k], (unsigned long long)X.ntry[k]);
      if (X.nacc[k]) atomicAdd(&L.ex_acc[k], (unsigned long long)X.nacc[k]);
    }
  }
}
#pragma clang fp contract(fast)

// block-wide exchange for one ligand (called by all threads): n_sub
// exchange sweeps in a row, sweep j drawing its uniforms with replica field j
__device__ void exchange_block(const LigDev& L, uint64_t sweep, int scheme,
                               int max_sep, int n_sub, uint64_t seed) {
  __shared__ XStage X;
  __shared__ double em[kXTable * kXTable];
  const int K = L.K;
  if (K < 2) return;
  if (scheme == 0) {
    // disjoint neighbour pairs: independent, one thread each
    const int a0 = (int)(sweep & 1ull);
    for (int j = 0; j < n_sub; ++j) {
      if (j > 0) __syncthreads();
      for (int a = a0 + 2 * (int)threadIdx.x; a + 1 < K; a += 2 * blockDim.x)
        attempt_pair(L, a, a + 1, 1, sweep, j, seed);
    }
  } else if (K <= kXTable && L.C == 3) {
    exchange_all_staged<3, true>(L, sweep, max_sep, n_sub, seed, X, em);
  } else if (K <= kXTable && L.C == 5) {
    exchange_all_staged<5, true>(L, sweep, max_sep, n_sub, seed, X, em);
  } else if (K <= kXStates && L.C == 3) {
    exchange_all_staged<3, false>(L, sweep, max_sep, n_sub, seed, X, em);
  } else if (K <= kXStates && L.C == 5) {
    exchange_all_staged<5, false>(L, sweep, max_sep, n_sub, seed, X, em);
  } else if (threadIdx.x == 0) {
    const int dmax = max_sep < K - 1 ? max_sep : K - 1;
    for (int j = 0; j < n_sub; ++j)
      for (int d = 1; d <= dmax; ++d)
        for (int a = 0; a + d < K; ++a)
          attempt_pair(L, a, a + d, d, sweep, j, seed);
  }
  // every replica's state after the exchange (round-trip bookkeeping)
  __syncthreads();
  for (int r = threadIdx.x; r < K; r += blockDim.x)
    note_state(L, r, L.state_of_replica[r]);
}

// Tail of one ligand's sweep, run by one whole block: exchange (if due),
// record one sample per state (if due), counter += 1.
__device__ void sweep_tail(const LigDev& L, int exchange_every, int scheme,
                           int max_sep, int n_sub, int sample_every,
                           uint64_t seed) {
  const unsigned long long s = *L.counter;
  if (exchange_every > 0 && s % (unsigned long long)exchange_every == 0ull)
    exchange_block(L, s, scheme, max_sep, n_sub, seed);
  __syncthreads();
  const unsigned long long rec = *L.n_rec;
  const bool record = sample_every > 0 &&
                      (s + 1ull) % (unsigned long long)sample_every == 0ull &&
                      rec < (unsigned long long)L.cap;
  if (record) {
    const int n3 = L.n * 3, C1 = 1 + L.C;
    float* dx = L.samp_x + (size_t)rec * L.K * n3;
    double* dc = L.samp_c + (size_t)rec * L.K * C1;
    for (int q = threadIdx.x; q < L.K * n3; q += blockDim.x) {
      const int k = q / n3, e = q - k * n3;
      dx[q] = L.x[(size_t)L.replica_of_state[k] * n3 + e];
    }
    for (int q = threadIdx.x; q < L.K * C1; q += blockDim.x) {
      const int k = q / C1, e = q - k * C1;
      dc[q] = L.comps[(size_t)L.replica_of_state[k] * C1 + e];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    *L.counter = s + 1ull;
    if (record) *L.n_rec = rec + 1ull;
  }
}

// One block per ligand: the tail as a kernel of its own.
__global__ __launch_bounds__(256) void k_sweep_tail(
    const LigDev* __restrict__ ligs, int exchange_every, int scheme,
    int max_sep, int n_sub, int sample_every, uint64_t seed) {
  sweep_tail(ligs[blockIdx.x], exchange_every, scheme, max_sep, n_sub,
             sample_every, seed);
}

// Start of a run of neighbour-scheme sweeps: buffer (s-1)&1 from the
// canonical state, nothing pending.  One block per ligand.
__global__ __launch_bounds__(256) void k_sweep_begin(
    const LigDev* __restrict__ ligs) {
  begin_ligand(ligs[blockIdx.x]);
}

// End of a run: the pending exchange and record of the last sweep, the
// canonical state written back.  One block per ligand.
__global__ __launch_bounds__(256) void k_sweep_finish(
    const LigDev* __restrict__ ligs, int exchange_every, int sample_every,
    uint64_t seed) {
  finish_ligand(ligs[blockIdx.x], exchange_every, sample_every, seed);
}

// ----------------------------------------------------------------------------
// HMC: one trial move per replica, one workgroup of W wavefronts per replica.
// (Sampling: HMC trial moves from velocity-Verlet molecular dynamics.)
// ----------------------------------------------------------------------------
// ONE: the launch covers the replicas of a single ligand, whose table entry
// comes in the kernel arguments (block b = replica b) instead of through the
// task list.
// PAIRS: ligands whose pair terms are in the energy (L.pairs_on) evaluate
// them too.
template <int C, int W, bool ONE, bool PAIRS>
__global__ __launch_bounds__(W * kWave) void k_hmc_sweep(
    GridDev g, const LigDev* __restrict__ ligs, const int2* __restrict__ tasks,
    LigDev one, int nleap, uint64_t seed, TailArgs tail) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const int2 task = ONE ? make_int2(0, (int)blockIdx.x) : tasks[blockIdx.x];
  const LigDev L = ONE ? one : ligs[task.x];  // kernel-lifetime copy
  const int r = task.y;
  const int n = L.n;
  const bool deferred = tail.scheme == 0;

  // per-replica state and per-atom data: issued before the topology is
  // staged so that both latencies overlap
  unsigned long long s;
  int a = 0, pin = 0, ain = 0;
  bool pend = false;
  if (deferred) {
    s = BPMF_GMEM(const unsigned long long, L.rcnt)[r];
    auto rsor = BPMF_GMEM(const int, L.rsor);
    auto rpend = BPMF_GMEM(const int, L.rpend);
    const int a0 = rsor[r], a1 = rsor[L.K + r];
    const int p0 = rpend[r], p1 = rpend[L.K + r];
    pin = (int)((s - 1ull) & 1ull);
    ain = pin ? a1 : a0;
    a = rsor_state(ain);
    pend = (pin ? p1 : p0) != 0;
  } else {
    s = *BPMF_GMEM(const unsigned long long, L.counter);
    a = BPMF_GMEM(const int, L.state_of_replica)[r];
  }
  const int fv = BPMF_GMEM(const int, L.fvalid)[r];
  const bool owner = tid < n;
  float x[3], v[3], f[3];
  const float m = owner ? BPMF_GMEM(const float, L.mass)[tid] : 0.f;
  float sc[C];
#pragma unroll
  for (int c = 0; c < C; ++c)
    sc[c] = owner ? BPMF_GMEM(const float, L.scale)[tid * C + c] : 0.f;
  const float im = owner ? BPMF_GMEM(const float, L.inv_mass)[tid] : 0.f;
  auto xr = BPMF_GMEM(const float, L.x) + (size_t)r * n * 3;
#pragma unroll
  for (int d = 0; d < 3; ++d) x[d] = owner ? xr[tid * 3 + d] : 0.f;

  // the ligand's topology goes to LDS now: its loads need only the table
  // entry, so they overlap the replica's; the barrier comes after the
  // loads below have been issued as well
  const Shared sh = carve<W, false>(smem, L, L.n, tid);

  // scheme 0 first applies the exchange (and record) that ended the previous
  // sweep, from the double buffer; the parameters of both states of the
  // replica's pair are loaded with the pair's components
  const Pair pr = (deferred && pend) ? own_pair(L.K, a, s, tail.exchange_every)
                                     : Pair{a, a, false};
  const int kb = pr.active ? (a == pr.lo ? pr.hi : pr.lo) : a;
  float wa[C], wb[C];
  double wda[C], wdb[C];
  auto wf = BPMF_GMEM(const float, L.wf);
  auto wdp = BPMF_GMEM(const double, L.wd);
#pragma unroll
  for (int c = 0; c < C; ++c) {
    wa[c] = wf[a * C + c];
    wb[c] = wf[kb * C + c];
    wda[c] = wdp[a * C + c];
    wdb[c] = wdp[kb * C + c];
  }
  auto Tf = BPMF_GMEM(const float, L.Tf);
  auto dtf = BPMF_GMEM(const float, L.dtf);
  auto bt = BPMF_GMEM(const double, L.beta);
  const float Ta = Tf[a], Tb = Tf[kb];
  const float dta = dtf[a], dtb = dtf[kb];
  const double ba = bt[a], bb = bt[kb];
  // the start of the trajectory's stored parts (state-independent force of
  // the current positions, restraint factor, components), loaded beside
  // the exchange's operands
  constexpr int kFC = 3 + 3 * C;
  const int C1 = 1 + C;
  const int cur = fv > 0 ? fv - 1 : 0, nxt = 1 - cur;
  float* const fc_cur = L.fcache + ((size_t)cur * L.K + r) * n * kFC;
  float* const fc_nxt = L.fcache + ((size_t)nxt * L.K + r) * n * kFC;
  float ca[kFC], cr[4];
  double cp[1 + C];
  if (fv > 0) {
    if (owner) {
      auto cap = BPMF_GMEM(const float, fc_cur + (size_t)tid * kFC);
#pragma unroll
      for (int q = 0; q < kFC; ++q) ca[q] = cap[q];
    } else {
#pragma unroll
      for (int q = 0; q < kFC; ++q) ca[q] = 0.f;
    }
    auto crp = BPMF_GMEM(const float, L.frc + ((size_t)cur * L.K + r) * 4);
#pragma unroll
    for (int q = 0; q < 4; ++q) cr[q] = crp[q];
    auto cpp = BPMF_GMEM(const double,
                         deferred ? L.scomp + ((size_t)pin * L.K + a) * C1
                                  : L.comps + (size_t)r * C1);
#pragma unroll
    for (int q = 0; q < 1 + C; ++q) cp[q] = cpp[q];
  }
  // the decision is the block's: the last wavefront (the one with the
  // fewest atoms) takes it and publishes it with the barrier that ends the
  // staging
  // The replica's next state-map entry (its state after this decision and
  // its round-trip mark) is written here: only this block reads it, in the
  // next sweep.
  __shared__ int s_swap;
  int* const rsor_out = L.rsor + (1 - pin) * L.K + r;
  if (pr.active && (tid >> 6) == W - 1) {
    const bool sw = pair_accepts<C>(L, pr, pin, s, seed);
    if (tid == (W - 1) * kWave) {
      s_swap = sw ? 1 : 0;
      if (a == pr.lo) {
        atomicAdd(&L.ex_try[pr.lo], 1ull);
        if (sw) atomicAdd(&L.ex_acc[pr.lo], 1ull);
      }
      *rsor_out = sw ? rsor_pack(kb, rt_step(L, rsor_mark(ain), kb)) : ain;
    }
  }
  if (deferred && !pr.active && tid == 0) *rsor_out = ain;
  // the momenta's standard normals do not depend on the state: drawn
  // beside the decision
  float z[3] = {0.f, 0.f, 0.f};
  if (owner) {
    const U4 o = draw(seed, (uint32_t)tid, L.id, r, s, kMomenta);
    normals3(o, z[0], z[1], z[2]);
  }
  __syncthreads();  // the staged topology and the decision
  const bool swap = pr.active && s_swap != 0;
  const int k = swap ? kb : a;
  float w[C];
  double wdk[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    w[c] = swap ? wb[c] : wa[c];
    wdk[c] = swap ? wdb[c] : wda[c];
  }
  const float T = swap ? Tb : Ta;
  const float dt = swap ? dtb : dta;
  const double beta = swap ? bb : ba;

  __shared__ double fin[2 * W];
  // the previous sweep's round: this replica's configuration and components
  // go to the slot of its state after that exchange.  The replica's record
  // counter is advanced at the end of the kernel, after the barriers, so that
  // every wavefront has read it first.
  bool recorded = false;
  unsigned long long rec = 0ull;
  if (deferred && pend && record_due(s, tail.sample_every)) {
    rec = BPMF_GMEM(const unsigned long long, L.rnrec)[r];
    if (rec < (unsigned long long)L.cap) {
      recorded = true;
      if (owner)
#pragma unroll
        for (int d = 0; d < 3; ++d)
          BPMF_GMEM(float, L.samp_x)[((size_t)rec * L.K + k) * n * 3 +
                                     tid * 3 + d] = x[d];
      if (tid < C1)
        BPMF_GMEM(double, L.samp_c)[((size_t)rec * L.K + k) * C1 + tid] =
            BPMF_GMEM(const double, L.scomp)[((size_t)pin * L.K + a) * C1 +
                                             tid];
    }
  }
  {
    const float sd = owner ? sqrtf((float)kRGas * T * im * 1e-4f) : 0.f;
    v[0] = sd * z[0];
    v[1] = sd * z[1];
    v[2] = sd * z[2];
  }
  const float ke0 = 0.5f * m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);

  // start of the trajectory: force and energy at the current positions,
  // rebuilt from the state-independent parts stored when these positions
  // were last evaluated (same arithmetic, same bits), or evaluated
  double U0, KE0;
  if (fv > 0) {
    U0 = cp[0];
#pragma unroll
    for (int c = 0; c < C; ++c) U0 += wdk[c] * cp[1 + c];
    if (owner) {
      float de[C][3], ge[3] = {0.f, 0.f, 0.f};
#pragma unroll
      for (int c = 0; c < C; ++c)
#pragma unroll
        for (int d = 0; d < 3; ++d) de[c][d] = ca[3 + 3 * c + d];
      grid_force<C>(w, de, ge);
      restraint_force(cr[0], m, cr[1], cr[2], cr[3], ge);
      f[0] = ca[0] + ge[0];
      f[1] = ca[1] + ge[1];
      f[2] = ca[2] + ge[2];
    } else {
      f[0] = f[1] = f[2] = 0.f;
    }
    double ke, unused;
    block_sum2<W, true>(ke0, 0.f, fin, tid, ke, unused);
    KE0 = ke * 1e4;
  } else {
    double t0[6 + C];
    eval_block<C, W, true, true, false, true, PAIRS>(
        g, L, w, x, m, sc, f, t0, ke0, 0.f, sh, tid,
        owner ? fc_cur + (size_t)tid * kFC : nullptr,
        L.frc + ((size_t)cur * L.K + r) * 4);
    U0 = t0[0] + t0[1] + t0[2] + t0[3];
#pragma unroll
    for (int c = 0; c < C; ++c) U0 += wdk[c] * t0[4 + c];
    KE0 = t0[4 + C] * 1e4;
  }

  // nleap velocity-Verlet steps; the last one also evaluates the energy
  const float hk = 0.5f * dt * 1e-4f * im;
  double t1[6 + C];
  for (int step = 0; step < nleap - 1; ++step) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      v[d] = fmaf(hk, f[d], v[d]);
      x[d] = fmaf(dt, v[d], x[d]);
    }
    eval_block<C, W, true, false, false, true, PAIRS>(g, L, w, x, m, sc, f,
                                                      t1, 0.f, 0.f, sh, tid);
#pragma unroll
    for (int d = 0; d < 3; ++d) v[d] = fmaf(hk, f[d], v[d]);
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    v[d] = fmaf(hk, f[d], v[d]);
    x[d] = fmaf(dt, v[d], x[d]);
  }
  // lean sums: the bonded total (the sweep needs no single bonded term),
  // formed in wavefront 0 only (its lanes take the decision and write the
  // components)
  eval_block<C, W, true, true, true, true, PAIRS, true>(
      g, L, w, x, m, sc, f, t1, 0.f, 0.f, sh, tid,
      owner ? fc_nxt + (size_t)tid * kFC : nullptr,
      L.frc + ((size_t)nxt * L.K + r) * 4);
#pragma unroll
  for (int d = 0; d < 3; ++d) v[d] = fmaf(hk, f[d], v[d]);
  double U1 = t1[0] + t1[1] + t1[2] + t1[3];
#pragma unroll
  for (int c = 0; c < C; ++c) U1 += wdk[c] * t1[4 + c];
  const float ke1 = 0.5f * m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  const float bad =
      (!isfinite(x[0]) || !isfinite(x[1]) || !isfinite(x[2])) ? 1.f : 0.f;
  double KE1, nbad;
  block_sum2<W, true>(ke1, bad, fin, tid, KE1, nbad);
  // the Metropolis decision in wavefront 0, published through LDS
  __shared__ int s_acc;
  bool finite = true;
  if (tid < kWave) {
    KE1 *= 1e4;
    const double dH = (U1 + KE1) - (U0 + KE0);
    const U4 o = draw(seed, 0u, L.id, r, s, kAccept);
    finite = isfinite(dH) && nbad == 0.0;
    const bool acc0 = finite && ln_u_below(o.x, -beta * dH);
    if (tid == 0) s_acc = acc0 ? 1 : 0;
  }
  block_sync();
  const bool accept = s_acc != 0;
  if (accept) {
    auto xw = BPMF_GMEM(float, L.x) + (size_t)r * n * 3;
    if (owner)
#pragma unroll
      for (int d = 0; d < 3; ++d) xw[tid * 3 + d] = x[d];
  }
  // components of the replica after the move (scheme 0: into the output
  // buffer, indexed by state)
  if (tid < C1 && (accept || deferred)) {
    double cv;
    if (accept) {
      // select without a register-array index
      cv = t1[0] + t1[1] + t1[2] + t1[3];
#pragma unroll
      for (int c = 0; c < C; ++c)
        if (tid == 1 + c) cv = t1[4 + c];
    } else {
      cv = BPMF_GMEM(const double, L.scomp)[((size_t)pin * L.K + a) * C1 +
                                            tid];
    }
    if (deferred)
      BPMF_GMEM(double, L.scomp)[((size_t)(s & 1ull) * L.K + k) * C1 + tid] =
          cv;
    else
      BPMF_GMEM(double, L.comps)[(size_t)r * C1 + tid] = cv;
  }
  if (tid == 0) {
    // the stored parts of the replica's (new or kept) positions
    BPMF_GMEM(int, L.fvalid)[r] = 1 + (accept ? nxt : cur);
    atomicAdd(&L.hmc_try[k], 1ull);
    if (accept) atomicAdd(&L.hmc_acc[k], 1ull);
    if (!finite) atomicAdd(L.nonfinite, 1ull);
    if (deferred) {
      const int pout = (int)(s & 1ull);
      BPMF_GMEM(int, L.rpend)[pout * L.K + r] = 1;
      BPMF_GMEM(unsigned long long, L.rcnt)[r] = s + 1ull;
      if (recorded) BPMF_GMEM(unsigned long long, L.rnrec)[r] = rec + 1ull;
    }
  }
}

__global__ __launch_bounds__(256) void k_exchange(
    const LigDev* __restrict__ ligs, int scheme, int max_sep, int n_sub,
    uint64_t seed) {
  const LigDev& L = ligs[blockIdx.x];
  exchange_block(L, *L.counter, scheme, max_sep, n_sub, seed);
}

// ----------------------------------------------------------------------------
// reduced-energy matrix u_kn = beta_k (U0_n + sum_c w_kc Psi_cn) of samples
// of one or many ligands (Estimation), energy only
// ----------------------------------------------------------------------------
// First sample of block b's share of a launch (b = nblocks: the end): the
// shares are contiguous runs of the flat sample index of equal estimated
// cost, so a block holding a large ligand's samples takes fewer of them.
// Position P = b * total_cost / nblocks falls in job j (jobs[j].cfirst <= P
// < jobs[j + 1].cfirst; the sentinel ends the list) and the share starts at
// the first of its samples whose cost starts at or after P.  j: that job.
__device__ __forceinline__ int64_t ukn_share_start(
    const UknJob* __restrict__ jobs, int n_jobs, int b, int nblocks, int& j) {
  const int64_t P = (int64_t)b * jobs[n_jobs].cfirst / nblocks;
  int lo = 0, hi = n_jobs;
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (jobs[mid].cfirst <= P) lo = mid; else hi = mid;
  }
  const int64_t c = jobs[lo].cost;
  int64_t k = (P - jobs[lo].cfirst + c - 1) / c;
  if (k > jobs[lo].n) k = jobs[lo].n;
  // block-uniform results, held in scalar registers (the 64-bit division
  // is vector code)
  j = __builtin_amdgcn_readfirstlane(lo);
  const int64_t r = jobs[lo].first + k;
  const uint32_t rlo = __builtin_amdgcn_readfirstlane((uint32_t)r);
  const uint32_t rhi = __builtin_amdgcn_readfirstlane((uint32_t)(r >> 32));
  return (int64_t)(((uint64_t)rhi << 32) | rlo);
}

// One W-wave block evaluates one sample at a time, persistent over the
// launch: block b takes the b-th contiguous share (by cost) of the flat
// sample index over all jobs (job j's samples are [jobs[j].first, jobs[j+1].first); a
// sentinel ends the list), so it stages a ligand's topology once per
// segment.  Each sample's column (K entries) goes to LDS; every `group`
// samples (at most 16: a 128-byte line of each row) the columns are written
// out row by row by consecutive lanes.
template <int C, int W, bool PAIRS>
__global__ __launch_bounds__(W * kWave) void k_energy_matrix(
    GridDev g, const LigDev* __restrict__ ligs,
    const UknJob* __restrict__ jobs, int n_jobs, int64_t total,
    int group) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const float w0[C] = {};
  // ligands and jobs come from restrict arguments: the u_kn stores cannot
  // clobber them, so they load into scalar registers
  int j, j_end;
  const int64_t b0 = ukn_share_start(jobs, n_jobs, blockIdx.x, gridDim.x, j);
  const int64_t b1 =
      ukn_share_start(jobs, n_jobs, blockIdx.x + 1, gridDim.x, j_end);
  if (b0 >= b1) return;
  typedef const float __attribute__((address_space(1))) gfloat;
  typedef const double __attribute__((address_space(1))) gcdouble;
  for (int64_t s = b0; s < b1; ++j) {
    const UknJob J = jobs[j];
    const int64_t e = jobs[j + 1].first < b1 ? jobs[j + 1].first : b1;
    if (s >= e) continue;  // empty job
    const LigDev L = ligs[J.lig];
    // topology staged for the segment; the barrier in carve also keeps the
    // previous segment's readers ahead of the copy
    const Shared sh = carve<W>(smem, L, 0, tid);
    // state weights and beta_k after the topology, for the expansion, then
    // the group's columns (the evaluation's first barrier orders these
    // writes before their reads)
    const int K = L.K;
    double* ew = reinterpret_cast<double*>(
        smem + block_lds_bytes(W, false, L.n, L.nb, L.na, L.nt,
                               PAIRS && L.pairs_on));
    double* col = ew + K * (C + 1);
    for (int i = tid; i < K * (C + 1); i += W * kWave)
      ew[i] = i < K * C ? ((gcdouble*)L.wd)[i]
                        : ((gcdouble*)L.beta)[i - K * C];
    // per-lane data through global (not flat) loads, so that the waits of
    // the evaluation's LDS reads do not wait on them
    const int n = L.n;
    const bool owner = tid < n;
    const float m = owner ? ((gfloat*)L.mass)[tid] : 0.f;
    float sc[C];
#pragma unroll
    for (int c = 0; c < C; ++c)
      sc[c] = owner ? ((gfloat*)L.scale)[tid * C + c] : 0.f;
    const gfloat* xb = (const gfloat*)J.xs + (size_t)tid * 3;
    // positions of the next sample load during the current evaluation
    float xn[3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
      xn[d] = owner ? xb[(size_t)(s - J.first) * n * 3 + d] : 0.f;
    for (; s < e;) {
      const int64_t g1 = s + group < e ? s + group : e;
      for (int64_t q = s; q < g1; ++q) {
        float x[3] = {xn[0], xn[1], xn[2]}, f[3];
        if (q + 1 < e) {
#pragma unroll
          for (int d = 0; d < 3; ++d)
            xn[d] = owner ? xb[(size_t)(q + 1 - J.first) * n * 3 + d] : 0.f;
        }
        double t[6 + C];
        eval_block<C, W, false, true, true, true, PAIRS>(
            g, L, w0, x, m, sc, f, t, 0.f, 0.f, sh, tid);
        const double U0 = t[0] + t[1] + t[2] + t[3];
        double* cs = col + (q - s) * K;
        for (int k = tid; k < K; k += W * kWave) {
          double E = U0;
#pragma unroll
          for (int c = 0; c < C; ++c) E = fma(ew[k * C + c], t[4 + c], E);
          cs[k] = ew[K * C + k] * E;
        }
      }
      // the group's columns: each row's run of consecutive samples written
      // by consecutive lanes (global stores: no wait of the next LDS access
      // depends on them)
      block_sync();
      const int cnt = (int)(g1 - s);
      const int64_t n0 = s - J.first;
      auto out = BPMF_GMEM(double, J.ukn);
      for (int i = tid; i < cnt * K; i += W * kWave) {
        const int k = i / cnt, qq = i - k * cnt;
        out[(size_t)k * J.ld + n0 + qq] = col[qq * K + k];
      }
      s = g1;
    }
  }
}

// The same u_kn with one wavefront per sample and no workgroup barrier
// inside a sample: for ligands whose pair terms are not in the energy.  A
// block of kUknWaves wavefronts stages the topology of its current job once
// (shared by its wavefronts); the job's samples are dealt to the wavefronts
// in groups of kUknWaveGroup consecutive ones.  A wavefront evaluates a
// sample alone: lane l owns atoms l and l + 64 (AP = 2) or l; the grid terms
// of its atoms, every bonded chunk of the ligand (energies only), the
// mass-weighted position sums of the restraint, then double sums over the
// wavefront, as the lean block evaluation forms them: U0 = (bonded total) +
// U_I, and the C channel sums.  Its LDS (positions, the group's columns) is
// its own; LDS operations of one wavefront complete in order, so its lanes
// see each other's stores after a wavefront-scope fence.
template <int C, int AP>
__global__ __launch_bounds__(kUknWaves * kWave) void k_energy_matrix_wave(
    GridDev g, const LigDev* __restrict__ ligs,
    const UknJob* __restrict__ jobs, int n_jobs, int64_t total) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid >> 6;
  int j, j_end;
  const int64_t b0 = ukn_share_start(jobs, n_jobs, blockIdx.x, gridDim.x, j);
  const int64_t b1 =
      ukn_share_start(jobs, n_jobs, blockIdx.x + 1, gridDim.x, j_end);
  if (b0 >= b1) return;
  typedef const float __attribute__((address_space(1))) gfloat;
  typedef const double __attribute__((address_space(1))) gcdouble;
  auto wave_fence = []() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  const Slots no_forces{nullptr, 0};
  for (int64_t s = b0; s < b1; ++j) {
    const UknJob J = jobs[j];
    const int64_t e = jobs[j + 1].first < b1 ? jobs[j + 1].first : b1;
    if (s >= e) continue;  // empty job
    const LigDev L = ligs[J.lig];
    const int K = L.K, n = L.n;
    double* ew = reinterpret_cast<double*>(smem);
    unsigned char* slot =
        smem + ukn_wave_head_bytes(K, C) + wv * ukn_wave_slot_bytes(K, AP);
    float4* pos = reinterpret_cast<float4*>(slot);
    double* col = reinterpret_cast<double*>(slot + 16 * kWave * AP);
    unsigned char* topo = smem + ukn_wave_head_bytes(K, C) +
                          kUknWaves * ukn_wave_slot_bytes(K, AP);
    __syncthreads();  // the previous job's readers are done
    Shared sh{};
    stage_topology(L, topo, sh, tid, kUknWaves * kWave);
    for (int i = tid; i < K * (C + 1); i += kUknWaves * kWave)
      ew[i] = i < K * C ? ((gcdouble*)L.wd)[i]
                        : ((gcdouble*)L.beta)[i - K * C];
    __syncthreads();
    const int ntc = (L.nt + kWave - 1) / kWave;
    const int nac = (L.na + kWave - 1) / kWave;
    const int nbc = (L.nb + kWave - 1) / kWave;
    float m[AP], sc[AP][C];
    bool own[AP];
#pragma unroll
    for (int a = 0; a < AP; ++a) {
      const int at = lane + kWave * a;
      own[a] = at < n;
      m[a] = own[a] ? ((gfloat*)L.mass)[at] : 0.f;
#pragma unroll
      for (int c = 0; c < C; ++c)
        sc[a][c] = own[a] ? ((gfloat*)L.scale)[at * C + c] : 0.f;
    }
    const int64_t nseg = e - s;
    for (int64_t gi = wv; gi * kUknWaveGroup < nseg; gi += kUknWaves) {
      const int64_t q0 = s + gi * kUknWaveGroup;
      const int64_t q1 = q0 + kUknWaveGroup < e ? q0 + kUknWaveGroup : e;
      for (int64_t q = q0; q < q1; ++q) {
        const gfloat* xq = (const gfloat*)J.xs + (size_t)(q - J.first) * n * 3;
        float x[AP][3];
#pragma unroll
        for (int a = 0; a < AP; ++a)
#pragma unroll
          for (int d = 0; d < 3; ++d)
            x[a][d] = own[a] ? xq[(lane + kWave * a) * 3 + d] : 0.f;
#pragma unroll
        for (int a = 0; a < AP; ++a)
          if (own[a])
            pos[lane + kWave * a] =
                make_float4(x[a][0], x[a][1], x[a][2], m[a]);
        // the first atom's cell records load during the torsions, the
        // second's (AP = 2) during the angles and bonds: one record set in
        // registers at a time
        float psi[C];
#pragma unroll
        for (int c = 0; c < C; ++c) psi[c] = 0.f;
        Corners<C> cn;
        if (own[0]) grid_fetch<C>(g, x[0][0], x[0][1], x[0][2], cn);
        wave_fence();
        // bonded terms, energies only, every chunk of the ligand
        float eb = 0.f, ea = 0.f, et = 0.f;
        for (int ch = 0; ch < ntc; ++ch) {
          const int t = ch * kWave + lane;
          if (t < L.nt)
            et += torsion_term<false>(pos, sh.tijkl[t], sh.tpar[t],
                                      no_forces);
        }
#pragma unroll
        for (int a = 0; a < AP; ++a) {
          if (own[a]) {
            float ev[C], dv[C][3];
            grid_finish<C, false>(g, cn, sc[a], ev, dv);
#pragma unroll
            for (int c = 0; c < C; ++c) psi[c] += ev[c];
          }
          if (a + 1 < AP && own[a + 1])
            grid_fetch<C>(g, x[a + 1][0], x[a + 1][1], x[a + 1][2], cn);
          if (a + 1 < AP) {
            for (int ch = 0; ch < nac; ++ch) {
              const int t = ch * kWave + lane;
              if (t < L.na)
                ea += angle_term<false>(pos, sh.aijk[t], sh.apar[t],
                                        no_forces);
            }
            for (int ch = 0; ch < nbc; ++ch) {
              const int t = ch * kWave + lane;
              if (t < L.nb)
                eb += bond_term<false>(pos, sh.bij[t], sh.bpar[t], no_forces);
            }
          }
        }
        for (int ch = 0; AP == 1 && ch < nac; ++ch) {
          const int t = ch * kWave + lane;
          if (t < L.na)
            ea += angle_term<false>(pos, sh.aijk[t], sh.apar[t], no_forces);
        }
        for (int ch = 0; AP == 1 && ch < nbc; ++ch) {
          const int t = ch * kWave + lane;
          if (t < L.nb)
            eb += bond_term<false>(pos, sh.bij[t], sh.bpar[t], no_forces);
        }
        // the centre of mass
        float px = 0.f, py = 0.f, pz = 0.f;
#pragma unroll
        for (int a = 0; a < AP; ++a) {
          px += m[a] * x[a][0];
          py += m[a] * x[a][1];
          pz += m[a] * x[a][2];
        }
        wave_sumf3(px, py, pz);
        const double U0b = wave_sum((double)eb + (double)ea + (double)et);
        double ps[C];
#pragma unroll
        for (int c = 0; c < C; ++c) ps[c] = wave_sum((double)psi[c]);
        const float cx = px * L.inv_total_mass - L.site[0];
        const float cy = py * L.inv_total_mass - L.site[1];
        const float cz = pz * L.inv_total_mass - L.site[2];
        const float d = sqrtf(cx * cx + cy * cy + cz * cz);
        const float excess = d - L.d0;
        const double ui =
            excess > 0.f
                ? 0.5 * (double)L.krest * (double)excess * (double)excess
                : 0.0;
        const double U0 = U0b + 0.0 + 0.0 + ui;
        double* cs = col + (q - q0) * K;
        for (int k = lane; k < K; k += kWave) {
          double E = U0;
#pragma unroll
          for (int c = 0; c < C; ++c) E = fma(ew[k * C + c], ps[c], E);
          cs[k] = ew[K * C + k] * E;
        }
        // the next sample's position stores come after every lane's
        // reads of this one
        wave_fence();
      }
      // the group's columns, row by row: a run of consecutive samples of
      // each row by consecutive lanes
      wave_fence();
      const int cnt = (int)(q1 - q0);
      const int64_t n0 = q0 - J.first;
      auto out = BPMF_GMEM(double, J.ukn);
      for (int i = lane; i < cnt * K; i += kWave) {
        const int k = i / cnt, qq = i - k * cnt;
        out[(size_t)k * J.ld + n0 + qq] = col[qq * K + k];
      }
      wave_fence();
    }
    s = e;
  }
}

// ----------------------------------------------------------------------------
// exposed evaluator: terms and forces for arbitrary configurations/weights
// ----------------------------------------------------------------------------
template <int C, int W>
__global__ __launch_bounds__(W * kWave) void k_evaluate(
    GridDev g, const LigDev* __restrict__ lig, const float* __restrict__ xs,
    int64_t N, const double* __restrict__ wconf, double* __restrict__ terms,
    float* __restrict__ forces) {
  extern __shared__ __align__(16) unsigned char smem[];
  const LigDev L = *lig;
  const int tid = threadIdx.x;
  const int n = L.n;
  const Shared sh = carve<W>(smem, L, L.n, tid);
  const bool owner = tid < n;
  const float m = owner ? L.mass[tid] : 0.f;
  float sc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) sc[c] = owner ? L.scale[tid * C + c] : 0.f;
  for (int64_t cf = blockIdx.x; cf < N; cf += gridDim.x) {
    float w[C];
#pragma unroll
    for (int c = 0; c < C; ++c) w[c] = (float)wconf[cf * C + c];
    float x[3], f[3];
    const float* xr = xs + (size_t)cf * n * 3;
#pragma unroll
    for (int d = 0; d < 3; ++d) x[d] = owner ? xr[tid * 3 + d] : 0.f;
    double t[6 + C];
    eval_block<C, W, true, true>(g, L, w, x, m, sc, f, t, 0.f, 0.f, sh, tid);
    if (tid == 0)
      for (int q = 0; q < 4 + C; ++q) terms[(size_t)cf * (4 + C) + q] = t[q];
    if (forces && owner) {
      float* fo = forces + (size_t)cf * n * 3;
#pragma unroll
      for (int d = 0; d < 3; ++d) fo[tid * 3 + d] = f[d];
    }
  }
}

// recompute cached components of every replica from its positions
template <int C, int W, bool PAIRS>
__global__ __launch_bounds__(W * kWave) void k_recompute(
    GridDev g, const LigDev* __restrict__ lig) {
  extern __shared__ __align__(16) unsigned char smem[];
  const LigDev L = *lig;
  const int tid = threadIdx.x;
  const int n = L.n;
  const Shared sh = carve<W>(smem, L, 0, tid);
  const int r = blockIdx.x;
  const bool owner = tid < n;
  const float m = owner ? L.mass[tid] : 0.f;
  float sc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) sc[c] = owner ? L.scale[tid * C + c] : 0.f;
  float x[3], f[3];
  const float w0[C] = {};
#pragma unroll
  for (int d = 0; d < 3; ++d)
    x[d] = owner ? L.x[((size_t)r * n + tid) * 3 + d] : 0.f;
  double t[6 + C];
  eval_block<C, W, false, true, false, true, PAIRS>(g, L, w0, x, m, sc, f, t,
                                                    0.f, 0.f, sh, tid);
  if (tid == 0) {
    double* cp = L.comps + (size_t)r * (1 + C);
    cp[0] = t[0] + t[1] + t[2] + t[3];
#pragma unroll
    for (int c = 0; c < C; ++c) cp[1 + c] = t[4 + c];
  }
}

// ----------------------------------------------------------------------------
// grid term alone, one thread per point
// ----------------------------------------------------------------------------
template <int C>
struct WeightsC {
  float w[C];
};

template <int C>
__global__ __launch_bounds__(256) void k_grid_eval(
    GridDev g, const float* __restrict__ pos, const float* __restrict__ scale,
    int64_t n, WeightsC<C> wc, float* __restrict__ energy,
    float* __restrict__ force) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    Corners<C> cn;
    grid_fetch<C>(g, pos[3 * i], pos[3 * i + 1], pos[3 * i + 2], cn);
    float s[C], e[C], de[C][3];
#pragma unroll
    for (int c = 0; c < C; ++c) s[c] = scale[i * C + c];
    grid_finish<C, true>(g, cn, s, e, de);
    if (energy)
#pragma unroll
      for (int c = 0; c < C; ++c) energy[i * C + c] = e[c];
    if (force) {
      float fx = 0.f, fy = 0.f, fz = 0.f;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        fx -= wc.w[c] * de[c][0];
        fy -= wc.w[c] * de[c][1];
        fz -= wc.w[c] * de[c][2];
      }
      force[3 * i] = fx;
      force[3 * i + 1] = fy;
      force[3 * i + 2] = fz;
    }
  }
}

// cell-major records from the node-major grid (one thread per record float,
// pads zero)
__global__ __launch_bounds__(256) void k_expand_cells(
    const float* __restrict__ nodes, int nx, int ny, int nz, int C,
    float* __restrict__ cells) {
  const int stride = cell_stride(C);
  const size_t cx = nx - 1, cy = ny - 1;
  const size_t total = cx * cy * (size_t)(nz - 1) * stride;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t cell = e / stride;
    const int o = (int)(e - cell * stride);
    float v = 0.f;
    if (o < 8 * C) {
      const int q = o / C, c = o - q * C;
      const size_t i = cell % cx + (q & 1);
      const size_t j = (cell / cx) % cy + ((q >> 1) & 1);
      const size_t k = cell / (cx * cy) + (q >> 2);
      v = nodes[((k * ny + j) * nx + i) * C + c];
    }
    cells[e] = v;
  }
}

int grid_blocks(int64_t work, int per_block, int cap) {
  int64_t b = (work + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

}  // namespace

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------
#define BPMF_DISPATCH_C(C_, ...)                                   \
  switch (C_) {                                                    \
    case 3: {                                                      \
      constexpr int C = 3;                                         \
      __VA_ARGS__;                                                 \
    } break;                                                       \
    case 5: {                                                      \
      constexpr int C = 5;                                         \
      __VA_ARGS__;                                                 \
    } break;                                                       \
    default:                                                       \
      return hipErrorInvalidValue;                                 \
  }

#define BPMF_DISPATCH_W(W_, ...)                                   \
  switch (W_) {                                                    \
    case 1: {                                                      \
      constexpr int W = 1;                                         \
      __VA_ARGS__;                                                 \
    } break;                                                       \
    case 2: {                                                      \
      constexpr int W = 2;                                         \
      __VA_ARGS__;                                                 \
    } break;                                                       \
    case 4: {                                                      \
      constexpr int W = 4;                                         \
      __VA_ARGS__;                                                 \
    } break;                                                       \
    case 8: {                                                      \
      constexpr int W = 8;                                         \
      __VA_ARGS__;                                                 \
    } break;                                                       \
    default:                                                       \
      return hipErrorInvalidValue;                                 \
  }

hipError_t launch_hmc_sweep(const GridDev& g, const LigDev* d_ligs,
                            const int2* d_tasks, int n_tasks, int waves,
                            int lds_bytes, int nleap, uint64_t seed,
                            TailArgs tail, const LigDev* one, bool pairs,
                            hipStream_t st) {
  if (n_tasks <= 0) return hipSuccess;
  const LigDev none{};
  const LigDev& arg = one ? *one : none;
#define BPMF_SWEEP(ONE_, PAIRS_)                                            \
  BPMF_DISPATCH_C(g.C, BPMF_DISPATCH_W(waves, {                             \
    hipLaunchKernelGGL((k_hmc_sweep<C, W, ONE_, PAIRS_>), dim3(n_tasks),    \
                       dim3(W * kWave), lds_bytes, st, g, d_ligs, d_tasks,  \
                       arg, nleap, seed, tail);                             \
  }))
  if (one && pairs) {
    BPMF_SWEEP(true, true);
  } else if (one) {
    BPMF_SWEEP(true, false);
  } else if (pairs) {
    BPMF_SWEEP(false, true);
  } else {
    BPMF_SWEEP(false, false);
  }
#undef BPMF_SWEEP
  return hipGetLastError();
}

hipError_t launch_sweep_tail(const LigDev* d_ligs, int n_ligs,
                             int exchange_every, int scheme, int max_sep,
                             int n_sub, int sample_every, uint64_t seed,
                             hipStream_t st) {
  if (n_ligs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sweep_tail, dim3(n_ligs), dim3(256), 0, st, d_ligs,
                     exchange_every, scheme, max_sep, n_sub, sample_every,
                     seed);
  return hipGetLastError();
}

hipError_t launch_sweep_begin(const LigDev* d_ligs, int n_ligs,
                              hipStream_t st) {
  if (n_ligs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sweep_begin, dim3(n_ligs), dim3(256), 0, st, d_ligs);
  return hipGetLastError();
}

hipError_t launch_sweep_finish(const LigDev* d_ligs, int n_ligs,
                               int exchange_every, int sample_every,
                               uint64_t seed, hipStream_t st) {
  if (n_ligs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sweep_finish, dim3(n_ligs), dim3(256), 0, st, d_ligs,
                     exchange_every, sample_every, seed);
  return hipGetLastError();
}

hipError_t launch_exchange(const LigDev* d_lig, int n_ligs, int scheme,
                           int max_sep, int n_sub, uint64_t seed,
                           hipStream_t st) {
  if (n_ligs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_exchange, dim3(n_ligs), dim3(256), 0, st, d_lig,
                     scheme, max_sep, n_sub, seed);
  return hipGetLastError();
}

namespace {
constexpr int kJobChunk = 32;
struct JobChunk {
  UknJob j[kJobChunk];
  int n;
};
__global__ __launch_bounds__(kJobChunk) void k_put_jobs(UknJob* dst,
                                                        JobChunk ch) {
  if ((int)threadIdx.x < ch.n) dst[threadIdx.x] = ch.j[threadIdx.x];
}
}  // namespace

hipError_t launch_put_jobs(UknJob* dst, const UknJob* jobs, int n,
                           hipStream_t st) {
  for (int first = 0; first < n; first += kJobChunk) {
    JobChunk ch;
    ch.n = n - first < kJobChunk ? n - first : kJobChunk;
    for (int i = 0; i < ch.n; ++i) ch.j[i] = jobs[first + i];
    hipLaunchKernelGGL(k_put_jobs, dim3(1), dim3(kJobChunk), 0, st,
                       dst + first, ch);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_energy_matrix(const GridDev& g, const LigDev* d_ligs,
                                int waves, const UknJob* d_jobs, int n_jobs,
                                int64_t total, int group, int lds_bytes,
                                int n_cu, bool pairs, bool per_wave,
                                hipStream_t st) {
  if (total <= 0) return hipSuccess;
  if (per_wave) {
    if (waves != 1 && waves != 2) return hipErrorInvalidValue;
    BPMF_DISPATCH_C(g.C, {
      auto kern = waves == 1 ? k_energy_matrix_wave<C, 1>
                             : k_energy_matrix_wave<C, 2>;
      int per_cu = 0;
      hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, kern, kUknWaves * kWave, lds_bytes);
      if (e != hipSuccess) return e;
      int64_t blocks = (int64_t)(per_cu > 0 ? per_cu : 1) * n_cu;
      // at least a group per wavefront
      const int64_t most =
          (total + kUknWaves * kUknWaveGroup - 1) / (kUknWaves * kUknWaveGroup);
      if (blocks > most) blocks = most;
      hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kUknWaves * kWave),
                         lds_bytes, st, g, d_ligs, d_jobs, n_jobs, total);
    });
    return hipGetLastError();
  }
  BPMF_DISPATCH_C(g.C, BPMF_DISPATCH_W(waves, {
    auto kern = pairs ? k_energy_matrix<C, W, true>
                      : k_energy_matrix<C, W, false>;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, kern, W * kWave, lds_bytes);
    if (e != hipSuccess) return e;
    int64_t blocks = (int64_t)(per_cu > 0 ? per_cu : 1) * n_cu;
    if (blocks > total) blocks = total;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(W * kWave),
                       lds_bytes, st, g, d_ligs, d_jobs, n_jobs, total,
                       group);
  }));
  return hipGetLastError();
}

hipError_t launch_evaluate(const GridDev& g, const LigDev* d_lig,
                           int waves, const float* xs, int64_t N,
                           const double* w, double* terms, float* forces,
                           int lds_bytes, hipStream_t st) {
  if (N <= 0) return hipSuccess;
  const int blocks = grid_blocks(N, 1, 1 << 20);
  BPMF_DISPATCH_C(g.C, BPMF_DISPATCH_W(waves, {
    hipLaunchKernelGGL((k_evaluate<C, W>), dim3(blocks), dim3(W * kWave),
                       lds_bytes, st, g, d_lig, xs, N, w, terms, forces);
  }));
  return hipGetLastError();
}

hipError_t launch_recompute_comps(const GridDev& g, const LigDev* d_lig,
                                  int waves, int K, int lds_bytes, bool pairs,
                                  hipStream_t st) {
  if (pairs) {
    BPMF_DISPATCH_C(g.C, BPMF_DISPATCH_W(waves, {
      hipLaunchKernelGGL((k_recompute<C, W, true>), dim3(K), dim3(W * kWave),
                         lds_bytes, st, g, d_lig);
    }));
  } else {
    BPMF_DISPATCH_C(g.C, BPMF_DISPATCH_W(waves, {
      hipLaunchKernelGGL((k_recompute<C, W, false>), dim3(K), dim3(W * kWave),
                         lds_bytes, st, g, d_lig);
    }));
  }
  return hipGetLastError();
}

hipError_t launch_expand_cells(const float* nodes, int nx, int ny, int nz,
                               int C, float* cells, hipStream_t st) {
  const int64_t total =
      (int64_t)(nx - 1) * (ny - 1) * (nz - 1) * cell_stride(C);
  hipLaunchKernelGGL(k_expand_cells, dim3(grid_blocks(total, 256, 1 << 16)),
                     dim3(256), 0, st, nodes, nx, ny, nz, C, cells);
  return hipGetLastError();
}

hipError_t launch_grid_eval(const GridDev& g, const float* pos,
                            const float* scale, int64_t n, const double* w,
                            float* energy, float* force, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int blocks = grid_blocks(n, 256, 1 << 20);
  BPMF_DISPATCH_C(g.C, {
    WeightsC<C> wc;
    for (int c = 0; c < C; ++c) wc.w[c] = (float)w[c];
    hipLaunchKernelGGL((k_grid_eval<C>), dim3(blocks), dim3(256), 0, st, g,
                       pos, scale, n, wc, energy, force);
  });
  return hipGetLastError();
}

}  // namespace bpmf
