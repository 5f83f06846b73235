// Neighbour-scheme replica exchange deferred into the next kernel: the
// exchange (and sample record) that ends sweep s - 1 is taken at the start of
// the next sweep, by both replicas of each pair, from double-buffered
// components indexed by state (Sampling: replica exchange between
// neighbouring states, Eq. repXacc).  Shared by the sweep kernels and the
// kernels that close a unit of sweeps.
#pragma once
#include <hip/hip_runtime.h>

#include "device.h"
#include "internal.h"

namespace bpmf {
namespace {

// State after the exchange that ends sweep s - 1 of the replica that held
// state a during it, from buffer `pin` (components indexed by state).  Only
// the replica's own pair (a, a +- 1) matters in the even/odd scheme; both
// replicas of a pair evaluate the same expression as attempt_pair on the same
// numbers and take the same decision.  `stats`: count the attempt (once per
// pair, by its lower state).
#pragma clang fp contract(off)

// The neighbour pair (lo, hi) of state a in the exchange that ends sweep
// s - 1, if that exchange is due and a has a partner.
struct Pair {
  int lo, hi;
  bool active;
};
__device__ __forceinline__ Pair own_pair(int K, int a, unsigned long long s,
                                         int exchange_every) {
  Pair p{a, a, false};
  if (exchange_every <= 0 || s == 0ull || K < 2) return p;
  const unsigned long long sw = s - 1ull;
  if (sw % (unsigned long long)exchange_every != 0ull) return p;
  const int a0 = (int)(sw & 1ull);
  if (a < a0) return p;
  if (((a - a0) & 1) == 0) {
    if (a + 1 >= K) return p;
    p.lo = a;
    p.hi = a + 1;
  } else {
    p.lo = a - 1;
    p.hi = a;
  }
  p.active = true;
  return p;
}

// Metropolis decision on pair p from buffer `pin` (attempt_pair's expression
// on the same numbers), every operand loaded before the arithmetic.
template <int C>
__device__ bool pair_accepts(const LigDev& L, Pair p, int pin,
                             unsigned long long s, uint64_t seed) {
  constexpr int C1 = 1 + C;
  auto sc = BPMF_GMEM(const double, L.scomp);
  auto wd = BPMF_GMEM(const double, L.wd);
  double clo[C1], chi[C1], wlo[C], whi[C];
#pragma unroll
  for (int e = 0; e < C1; ++e) {
    clo[e] = sc[((size_t)pin * L.K + p.lo) * C1 + e];
    chi[e] = sc[((size_t)pin * L.K + p.hi) * C1 + e];
  }
#pragma unroll
  for (int c = 0; c < C; ++c) {
    wlo[c] = wd[p.lo * C + c];
    whi[c] = wd[p.hi * C + c];
  }
  const double blo = BPMF_GMEM(const double, L.beta)[p.lo];
  const double bhi = BPMF_GMEM(const double, L.beta)[p.hi];
  // E_k(x) = U0 + sum_c w_kc Psi_c, channels in order
  auto energy = [](const double* w, const double* cp) {
    double E = cp[0];
#pragma unroll
    for (int c = 0; c < C; ++c) E += w[c] * cp[1 + c];
    return E;
  };
  const double delta = blo * (energy(wlo, chi) - energy(wlo, clo)) +
                       bhi * (energy(whi, clo) - energy(whi, chi));
  const uint32_t purpose = (uint32_t)kExchange | (1u << 8);
  const U4 o = draw(seed, (uint32_t)p.lo, L.id, 0, s - 1ull, purpose);
  return isfinite(delta) && ln_u_below(o.x, -delta);
}

__device__ int deferred_state(const LigDev& L, int a, unsigned long long s,
                              int pin, int exchange_every, uint64_t seed,
                              bool stats) {
  const Pair p = own_pair(L.K, a, s, exchange_every);
  if (!p.active) return a;
  // the sweep kernels run 3 or 5 channels only
  const bool ok = L.C == 5 ? pair_accepts<5>(L, p, pin, s, seed)
                           : pair_accepts<3>(L, p, pin, s, seed);
  if (stats && a == p.lo) {
    atomicAdd(&L.ex_try[p.lo], 1ull);
    if (ok) atomicAdd(&L.ex_acc[p.lo], 1ull);
  }
  return ok ? (a == p.lo ? p.hi : p.lo) : a;
}
#pragma clang fp contract(fast)

// Round trips (Sampling: the replica-exchange walk between the end
// states): replica r has just entered state k.  A trip counts when a
// replica that has visited state K-1 since it was last in state 0 returns
// to state 0.  Only the replica's own thread writes its rt_end; entering
// the same state again changes nothing.
// The mark after entering state k with mark e (a trip completes: counted).
__device__ __forceinline__ int rt_step(const LigDev& L, int e, int k) {
  if (L.K < 2) return e;
  if (k == 0) {
    if (e == 1) atomicAdd(round_trips_of(L), 1ull);
    return 0;
  }
  return (k == L.K - 1 && e == 0) ? 1 : e;
}
// the same on the canonical marks
__device__ __forceinline__ void note_state(const LigDev& L, int r, int k) {
  int* e = rt_end_of(L) + r;
  const int e0 = *e, e1 = rt_step(L, e0, k);
  if (e1 != e0) *e = e1;
}

// During a run of neighbour-scheme sweeps the state map's buffers also
// carry each replica's mark: entry = state | (mark + 1) << 16.
__device__ __forceinline__ int rsor_pack(int k, int e) {
  return k | ((e + 1) << 16);
}
__device__ __forceinline__ int rsor_state(int v) { return v & 0xffff; }
__device__ __forceinline__ int rsor_mark(int v) { return (v >> 16) - 1; }

// the exchange ending sweep s - 1 records a round when s % every == 0
__device__ __forceinline__ bool record_due(unsigned long long s, int every) {
  return every > 0 && s > 0ull && s % (unsigned long long)every == 0ull;
}


// Start of a run of neighbour-scheme sweeps for one replica: buffer (s-1)&1
// from the replica's canonical state k and components, nothing pending.
__device__ __forceinline__ void begin_replica(const LigDev& L, int r, int k,
                                              unsigned long long s,
                                              unsigned long long nrec,
                                              const double* comps_r) {
  const int pin = (int)((s - 1ull) & 1ull), K = L.K, C1 = 1 + L.C;
  L.rsor[pin * K + r] = rsor_pack(k, rt_end_of(L)[r]);
  L.rpend[pin * K + r] = 0;
  L.rcnt[r] = s;
  L.rnrec[r] = nrec;
  for (int e = 0; e < C1; ++e)
    L.scomp[((size_t)pin * K + k) * C1 + e] = comps_r[e];
}

// begin_replica for every replica of a ligand (all threads of a block)
__device__ __forceinline__ void begin_ligand(const LigDev& L) {
  const unsigned long long s = *L.counter, nrec = *L.n_rec;
  const int C1 = 1 + L.C;
  for (int r = threadIdx.x; r < L.K; r += blockDim.x)
    begin_replica(L, r, L.state_of_replica[r], s, nrec,
                  L.comps + (size_t)r * C1);
}

// End of a run for one ligand (all threads of a block): apply the pending
// exchange and record of the last sweep and write the canonical state maps,
// components and counters back.
__device__ __forceinline__ void finish_ligand(const LigDev& L,
                                              int exchange_every,
                                              int sample_every,
                                              uint64_t seed) {
  const unsigned long long s = L.rcnt[0];
  const int pin = (int)((s - 1ull) & 1ull), K = L.K, C1 = 1 + L.C;
  const bool pend = L.rpend[pin * K] != 0;
  for (int r = threadIdx.x; r < K; r += blockDim.x) {
    const int v = L.rsor[pin * K + r];
    const int a = rsor_state(v), e = rsor_mark(v);
    const int k =
        pend ? deferred_state(L, a, s, pin, exchange_every, seed, true) : a;
    rt_end_of(L)[r] = k != a ? rt_step(L, e, k) : e;
    L.state_of_replica[r] = k;
    L.replica_of_state[k] = r;
    for (int e = 0; e < C1; ++e)
      L.comps[(size_t)r * C1 + e] = L.scomp[((size_t)pin * K + a) * C1 + e];
  }
  __syncthreads();
  const unsigned long long rec = L.rnrec[0];
  const bool record =
      pend && record_due(s, sample_every) && rec < (unsigned long long)L.cap;
  if (record) {
    const int n3 = L.n * 3;
    float* dx = L.samp_x + (size_t)rec * K * n3;
    double* dc = L.samp_c + (size_t)rec * K * C1;
    for (int q = threadIdx.x; q < K * n3; q += blockDim.x) {
      const int k = q / n3, e = q - k * n3;
      dx[q] = L.x[(size_t)L.replica_of_state[k] * n3 + e];
    }
    for (int q = threadIdx.x; q < K * C1; q += blockDim.x) {
      const int k = q / C1, e = q - k * C1;
      dc[q] = L.comps[(size_t)L.replica_of_state[k] * C1 + e];
    }
  }
  if (threadIdx.x == 0) {
    *L.counter = s;
    *L.n_rec = record ? rec + 1ull : rec;
  }
}

}  // namespace
}  // namespace bpmf
