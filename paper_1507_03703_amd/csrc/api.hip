// Host side of libbpmf: argument validation, device-memory layout, kernel
// sequencing.  Every entry point is declared in include/bpmf.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/bpmf.h"
#include "internal.h"
#include "moves.h"
#include "mlp.h"
#include "protocol.h"
#include "pairs.h"

using namespace bpmf;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                      \
  do {                                                                     \
    hipError_t e_ = (expr);                                                \
    if (e_ != hipSuccess)                                                  \
      return fail(BPMF_E_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                  __FILE__, __LINE__);                                     \
  } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Carves one device allocation into aligned sub-arrays.
struct Arena {
  std::vector<size_t> offsets;
  size_t total = 0;
  size_t add(size_t bytes) {
    total = align_up(total, kArenaAlign);
    const size_t o = total;
    offsets.push_back(o);
    total += bytes > 0 ? bytes : 1;
    return o;
  }
};

struct LigHost {
  LigDev dev;      // device pointers inside the ligand's arena
  void* arena;     // owning allocation
  size_t state_bytes;  // arena prefix holding everything but the samples
  int min_waves;   // wavefronts needed to give every atom a thread
  int sweep_waves; // wavefronts per replica in the HMC sweep
  int waves_pin = 0;  // the ligand's own choice (bpmf_set_ligand_waves), 0 =
                      // none: the context-wide one applies
  uint64_t counter;   // host mirror of *dev.counter
  int64_t n_rec;      // host mirror of *dev.n_rec
  std::vector<double> beta, wd;
  // external-move statistics per state (in the arena's state region)
  unsigned long long* ext_acc = nullptr;
  unsigned long long* ext_try = nullptr;
  // learned pose proposal (bpmf_proposal_setup)
  bool has_prop = false;
  void* prop_arena = nullptr;
  PropDev* d_prop = nullptr;  // device copy of PropDev
  float* params = nullptr;    // kNParams fp32 master weights
  float* grad = nullptr;      // kNParams
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  int64_t adam_t = 0;
  PropDev prop{};
  // place in the batched pose-move tables (build_pose_tables): first task
  // (= first row), first forward group and their count
  int ptask0 = -1, pgroup0 = 0, n_pgroups = 0;
  // bf16 transposed weights of the pose moves' forward pass (kTSize), stale
  // while wt_dirty (after the fp32 parameters change)
  unsigned short* wt = nullptr;
  bool wt_dirty = true;
  // intramolecular nonbonded / implicit-solvent terms (bpmf_pair_setup)
  bool has_pairs = false;
  void* pair_arena = nullptr;
  PairDev pair{};
};

}  // namespace

struct bpmf_ctx {
  int device = 0;
  uint64_t seed = 0;
  hipStream_t stream = nullptr;
  bpmf_alloc_fn alloc = nullptr;
  bpmf_free_fn free_fn = nullptr;
  void* user = nullptr;
  // grid
  bool has_grid = false;
  GridDev grid{};
  void* grid_mem = nullptr;
  // ligands
  std::vector<LigHost> ligs;
  LigDev* d_ligs = nullptr;  // device copy of every LigDev
  int2* d_tasks = nullptr;   // sweep tasks grouped by wavefronts per replica
  static constexpr int kWaveClasses = 4;  // W = 1, 2, 4, 8
  int class_off[kWaveClasses] = {0, 0, 0, 0};
  int class_n[kWaveClasses] = {0, 0, 0, 0};
  int class_lds[kWaveClasses] = {0, 0, 0, 0};
  int class_single[kWaveClasses] = {-1, -1, -1, -1};  // sole ligand or -1
  bool class_pairs[kWaveClasses] = {false, false, false, false};
  int waves_override = 0;  // 0 = automatic choice
  int task_order = 1;      // 0 = ligand by ligand, 1 = heaviest first
  int n_cu = 1;  // compute units of the device
  // scratch
  void* comps_mem = nullptr;  // energy-matrix job table (device)
  size_t comps_bytes = 0;
  UknJob* jobs_host = nullptr;  // pinned staging of the job table
  size_t jobs_host_n = 0;
  hipEvent_t jobs_copied = nullptr;  // last upload of the staging buffer
  void* mbar_mem = nullptr;
  size_t mbar_bytes = 0;
  void* mlp_mem = nullptr;   // activations of the proposal network
  size_t mlp_bytes = 0;
  void* place_mem = nullptr;  // centres of mass of placed configurations
  size_t place_bytes = 0;
  // this device's address of the no-allocation job table (or null)
  void* scratch_addr = nullptr;
  // batched pose moves over every ligand with a proposal: per-ligand
  // proposal entries (zero without a proposal), tasks ordered by wavefront
  // class, then ligand, then replica (a task's row is its index), and the
  // forward pass's groups of up to 16 rows of one ligand
  bool pose_dirty = true;
  PropDev* d_props = nullptr;
  PoseTask* d_ptasks = nullptr;
  MlpGroup* d_pgroups = nullptr;
  int n_ptasks = 0, n_pgroups = 0;
  int ptask_off[kWaveClasses] = {0, 0, 0, 0};
  int ptask_n[kWaveClasses] = {0, 0, 0, 0};
  // kernel timing
  static constexpr int kTimers = 4;
  static constexpr size_t kMaxPairs = 8192;
  bool timing = false;
  int timing_every = 1;
  uint64_t launches[kTimers] = {0, 0, 0, 0};
  std::vector<hipEvent_t> ev_pool[kTimers];  // start/stop pairs
  std::vector<int> ev_weight[kTimers];       // launches covered by a pair
  size_t ev_used[kTimers] = {0, 0, 0, 0};
  // hipGraph of a chunk of sweeps (captured on a private stream, launched on
  // `stream`)
  int graph_chunk = 64;  // 0 disables
  hipStream_t cap_stream = nullptr;
  // the sweep's wavefront classes after the first run on streams of their
  // own, forked from and joined to the launching stream (default priority)
  hipStream_t class_stream[kWaveClasses] = {};
  hipEvent_t class_fork = nullptr, class_join[kWaveClasses] = {};
  hipGraphExec_t graph_exec = nullptr;
  hipGraph_t graph = nullptr;
  uint64_t table_version = 0, graph_version = ~0ull;
  static constexpr int kKey = 14;
  int graph_key[kKey] = {0};

  void drop_graph() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    graph_exec = nullptr;
    graph = nullptr;
    graph_version = ~0ull;
  }

  // returns the event pair to bracket this launch of `k`, or false
  bool timer_begin(int k, hipEvent_t* a, hipEvent_t* b, int weight = 1) {
    if (!timing) return false;
    const uint64_t idx = launches[k]++;
    if (idx % (uint64_t)timing_every != 0) return false;
    if (ev_used[k] >= kMaxPairs) return false;
    if (ev_used[k] * 2 + 2 > ev_pool[k].size()) {
      hipEvent_t e0, e1;
      if (hipEventCreate(&e0) != hipSuccess) return false;
      if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return false;
      }
      ev_pool[k].push_back(e0);
      ev_pool[k].push_back(e1);
    }
    *a = ev_pool[k][ev_used[k] * 2];
    *b = ev_pool[k][ev_used[k] * 2 + 1];
    if (ev_weight[k].size() <= ev_used[k]) ev_weight[k].resize(ev_used[k] + 1);
    ev_weight[k][ev_used[k]] = weight;
    ++ev_used[k];
    return true;
  }

  void* dalloc(size_t bytes) {
    if (bytes == 0) bytes = 1;
    if (alloc) return alloc(bytes, user);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
  }
  void dfree(void* p) {
    if (!p) return;
    if (free_fn)
      free_fn(p, user);
    else
      (void)hipFree(p);
  }
};

namespace {

int check_ctx(bpmf_ctx* c) {
  if (!c) return fail(BPMF_E_INVAL, "null context");
  if (hipSetDevice(c->device) != hipSuccess)
    return fail(BPMF_E_HIP, "hipSetDevice(%d) failed", c->device);
  return BPMF_OK;
}

int check_lig(bpmf_ctx* c, int id) {
  if (id < 0 || id >= (int)c->ligs.size())
    return fail(BPMF_E_INVAL, "ligand id %d out of range [0, %d)", id,
                (int)c->ligs.size());
  return BPMF_OK;
}

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!isfinite(p[i])) return false;
  return true;
}

int wave_class(int w) { return w == 1 ? 0 : (w == 2 ? 1 : (w == 4 ? 2 : 3)); }

int lds_of(const LigHost& h, int waves, bool forces) {
  const LigDev& L = h.dev;
  return block_lds_bytes(waves, forces, L.n, L.nb, L.na, L.nt,
                         L.pairs_on != 0);
}

// wavefronts per replica for the HMC sweep: enough to own every atom; when
// few replicas are in flight (latency-bound) spread each over up to four
// wavefronts so that the bonded terms of a step run in parallel
int choose_waves(const bpmf_ctx* c, const LigHost& h, int total_replicas) {
  if (h.waves_pin) return std::max(h.waves_pin, h.min_waves);
  int w = c->waves_override ? c->waves_override : 1;
  if (!c->waves_override) {
    // enough waves to give every slot of the wave-aligned bonded index its
    // own thread while the chip has room for them (latency-bound ladders),
    // fewer when replicas alone fill the chip; from four waves on the atom
    // waves leave the bonded terms to the others
    const int pad = kWave - 1;
    const int index = ((h.dev.nt + pad) & ~pad) + ((h.dev.na + pad) & ~pad) +
                      h.dev.nb;
    const int atom_waves = (h.dev.n + pad) / kWave;
    auto bonded_threads = [&](int waves) {
      const int first =
          (waves >= 4 && waves >= 2 * atom_waves) ? atom_waves : 0;
      return (waves - first) * kWave;
    };
    int want = 1;
    while (want < 8 && bonded_threads(want) < index) want *= 2;
    while (want > 1 && total_replicas * want > 4096) want /= 2;
    w = want;
  }
  if (w < h.min_waves) w = h.min_waves;
  return w;
}

// rebuild the device ligand table and the sweep task lists
int rebuild_tables(bpmf_ctx* c) {
  const int nl = (int)c->ligs.size();
  std::vector<LigDev> table(nl);
  std::vector<int2> cls[bpmf_ctx::kWaveClasses];
  int lds[bpmf_ctx::kWaveClasses] = {0, 0, 0, 0};
  bool pairs[bpmf_ctx::kWaveClasses] = {false, false, false, false};
  int total = 0;
  for (int l = 0; l < nl; ++l) total += c->ligs[l].dev.K;
  for (int l = 0; l < nl; ++l) {
    LigHost& h = c->ligs[l];
    table[l] = h.dev;
    h.sweep_waves = choose_waves(c, h, total);
    const int q = wave_class(h.sweep_waves);
    for (int r = 0; r < h.dev.K; ++r) cls[q].push_back(make_int2(l, r));
    lds[q] = std::max(lds[q], lds_of(h, h.sweep_waves, true));
    pairs[q] = pairs[q] || h.dev.pairs_on;
  }
  if (c->task_order == 1) {
    // the replicas of the ligands with the most work per sweep first (a
    // rough per-block cost: bonded terms by kind, and atoms): workgroups
    // start in launch order, so the longest ones start earliest and the
    // short ones fill in behind them (config 5: 42.2 -> 36.9 us per sweep)
    auto cost = [&](int l) {
      const LigDev& d = c->ligs[l].dev;
      return 4L * d.nt + 2L * d.na + d.nb + 2L * d.n;
    };
    for (auto& v : cls)
      std::stable_sort(v.begin(), v.end(), [&](int2 u, int2 w) {
        return cost(u.x) > cost(w.x);
      });
  }
  std::vector<int2> all;
  int off[bpmf_ctx::kWaveClasses];
  for (int q = 0; q < bpmf_ctx::kWaveClasses; ++q) {
    off[q] = (int)all.size();
    all.insert(all.end(), cls[q].begin(), cls[q].end());
  }
  void* nd = c->dalloc(sizeof(LigDev) * std::max(nl, 1));
  void* nt = c->dalloc(sizeof(int2) * std::max<size_t>(all.size(), 1));
  if (!nd || !nt) {
    c->dfree(nd);
    c->dfree(nt);
    return fail(BPMF_E_NOMEM, "ligand table allocation failed");
  }
  if (nl)
    HIP_TRY(hipMemcpyAsync(nd, table.data(), sizeof(LigDev) * nl,
                           hipMemcpyHostToDevice, c->stream));
  if (!all.empty())
    HIP_TRY(hipMemcpyAsync(nt, all.data(), sizeof(int2) * all.size(),
                           hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->drop_graph();
  ++c->table_version;
  c->dfree(c->d_ligs);
  c->dfree(c->d_tasks);
  c->d_ligs = (LigDev*)nd;
  c->d_tasks = (int2*)nt;
  c->pose_dirty = true;
  for (int q = 0; q < bpmf_ctx::kWaveClasses; ++q) {
    c->class_off[q] = off[q];
    c->class_n[q] = (int)cls[q].size();
    c->class_lds[q] = lds[q];
    c->class_pairs[q] = pairs[q];
    // a class holding the replicas of one ligand (0..K-1 in order) passes
    // that ligand's table entry as a kernel argument
    c->class_single[q] = -1;
    if (!cls[q].empty() && cls[q].front().x == cls[q].back().x)
      c->class_single[q] = cls[q].front().x;
  }
  return BPMF_OK;
}

int ensure_scratch(bpmf_ctx* c, void** mem, size_t* have, size_t need) {
  if (*have >= need) return BPMF_OK;
  HIP_TRY(hipStreamSynchronize(c->stream));
  // a captured graph may address the old buffer: capture again
  c->drop_graph();
  c->dfree(*mem);
  *mem = c->dalloc(need);
  if (!*mem) {
    *have = 0;
    return fail(BPMF_E_NOMEM, "scratch allocation of %zu bytes failed", need);
  }
  *have = need;
  return BPMF_OK;
}

}  // namespace

// ============================================================================
// lifecycle
// ============================================================================
namespace {
int scratch_address(int device, void** out);
}  // namespace

extern "C" int bpmf_version(void) { return 100; }

extern "C" const char* bpmf_last_error(void) { return g_err.c_str(); }

extern "C" int bpmf_create(bpmf_ctx** out, int device, uint64_t seed,
                           void* hip_stream, bpmf_alloc_fn alloc,
                           bpmf_free_fn free_fn, void* alloc_user) {
  if (!out) return fail(BPMF_E_INVAL, "null output pointer");
  *out = nullptr;
  if ((alloc == nullptr) != (free_fn == nullptr))
    return fail(BPMF_E_INVAL, "alloc and free must both be given or both NULL");
  int n_dev = 0;
  if (hipGetDeviceCount(&n_dev) != hipSuccess || n_dev == 0)
    return fail(BPMF_E_HIP, "no HIP device available");
  if (device < 0 || device >= n_dev)
    return fail(BPMF_E_INVAL, "device %d out of range [0, %d)", device, n_dev);
  HIP_TRY(hipSetDevice(device));
  bpmf_ctx* c = new (std::nothrow) bpmf_ctx();
  if (!c) return fail(BPMF_E_NOMEM, "context allocation failed");
  c->device = device;
  if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount,
                            device) != hipSuccess ||
      c->n_cu < 1)
    c->n_cu = 1;
  c->seed = seed;
  c->stream = (hipStream_t)hip_stream;
  c->alloc = alloc;
  c->free_fn = free_fn;
  c->user = alloc_user;
  const int src = scratch_address(device, &c->scratch_addr);
  if (src) {
    delete c;
    return src;
  }
  *out = c;
  return BPMF_OK;
}

extern "C" int bpmf_destroy(bpmf_ctx* c) {
  if (!c) return BPMF_OK;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  for (auto& l : c->ligs) {
    c->dfree(l.arena);
    c->dfree(l.prop_arena);
    c->dfree(l.pair_arena);
  }
  c->dfree(c->mlp_mem);
  c->dfree(c->place_mem);
  c->dfree(c->grid_mem);
  c->dfree(c->d_ligs);
  c->dfree(c->d_tasks);
  c->dfree(c->d_props);
  c->dfree(c->d_ptasks);
  c->dfree(c->d_pgroups);
  c->dfree(c->comps_mem);
  if (c->jobs_host) (void)hipHostFree(c->jobs_host);
  if (c->jobs_copied) (void)hipEventDestroy(c->jobs_copied);
  c->dfree(c->mbar_mem);
  for (int k = 0; k < bpmf_ctx::kTimers; ++k)
    for (hipEvent_t e : c->ev_pool[k]) (void)hipEventDestroy(e);
  c->drop_graph();
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (int q = 0; q < bpmf_ctx::kWaveClasses; ++q) {
    if (c->class_stream[q]) (void)hipStreamDestroy(c->class_stream[q]);
    if (c->class_join[q]) (void)hipEventDestroy(c->class_join[q]);
  }
  if (c->class_fork) (void)hipEventDestroy(c->class_fork);
  delete c;
  return BPMF_OK;
}

extern "C" int bpmf_sync(bpmf_ctx* c) {
  int rc = check_ctx(c);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return BPMF_OK;
}

// ============================================================================
// grid
// ============================================================================
extern "C" int bpmf_grid_upload(bpmf_ctx* c, const bpmf_grid_desc* d,
                                const float* nodes) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!d || !nodes) return fail(BPMF_E_INVAL, "null grid descriptor or nodes");
  if (!c->ligs.empty())
    return fail(BPMF_E_STATE, "grid cannot change after ligand setup");
  if (d->nx < 2 || d->ny < 2 || d->nz < 2)
    return fail(BPMF_E_INVAL, "grid needs >= 2 nodes per axis (got %d %d %d)",
                d->nx, d->ny, d->nz);
  if (d->nx > (1 << 24) || d->ny > (1 << 24) || d->nz > (1 << 24))
    return fail(BPMF_E_INVAL,
                "grid has more than 2^24 nodes on an axis (%d %d %d)", d->nx,
                d->ny, d->nz);
  if (d->n_channels < 1 || d->n_channels > BPMF_MAX_CHANNELS)
    return fail(BPMF_E_INVAL, "n_channels %d outside 1..%d", d->n_channels,
                BPMF_MAX_CHANNELS);
  if (!(d->spacing > 0) || !isfinite(d->spacing))
    return fail(BPMF_E_INVAL, "grid spacing must be positive and finite");
  if (!finite_all(d->origin, 3))
    return fail(BPMF_E_INVAL, "grid origin must be finite");
  if (!d->transform) return fail(BPMF_E_INVAL, "null transform array");
  const size_t nn = (size_t)d->nx * d->ny * d->nz;
  if (nn * d->n_channels > (size_t)INT32_MAX)
    return fail(BPMF_E_INVAL, "grid too large (%zu values)", nn * d->n_channels);
  int mask = 0;
  for (int ch = 0; ch < d->n_channels; ++ch) {
    if (d->transform[ch] == 4)
      mask |= 1 << ch;
    else if (d->transform[ch] != 0)
      return fail(BPMF_E_INVAL, "channel %d: transform %d (0 or 4 allowed)", ch,
                  d->transform[ch]);
  }
  for (size_t i = 0; i < nn * d->n_channels; ++i) {
    const float v = nodes[i];
    if (!isfinite(v))
      return fail(BPMF_E_INVAL, "non-finite grid value at index %zu", i);
    if (((mask >> (i % d->n_channels)) & 1) && v < 0.f)
      return fail(BPMF_E_INVAL,
                  "negative value %g at index %zu of a quartic-root channel", v,
                  i);
  }
  // the kernels read the cell-major copy (8 corners of a cell in one
  // record); the node-major upload is a staging buffer
  const size_t cell_bytes = (size_t)(d->nx - 1) * (d->ny - 1) * (d->nz - 1) *
                            cell_stride(d->n_channels) * sizeof(float);
  if (cell_bytes > ((size_t)64 << 30))
    return fail(BPMF_E_INVAL, "grid too large: %zu bytes of cell records",
                cell_bytes);
  void* stage = c->dalloc(nn * d->n_channels * sizeof(float));
  if (!stage) return fail(BPMF_E_NOMEM, "grid staging allocation failed");
  void* mem = c->dalloc(cell_bytes);
  if (!mem) {
    c->dfree(stage);
    return fail(BPMF_E_NOMEM, "grid allocation failed (%zu bytes)",
                cell_bytes);
  }
  hipError_t e = hipMemcpyAsync(stage, nodes,
                                nn * d->n_channels * sizeof(float),
                                hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = launch_expand_cells((const float*)stage, d->nx, d->ny, d->nz,
                            d->n_channels, (float*)mem, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  c->dfree(stage);
  if (e != hipSuccess) {
    c->dfree(mem);
    return fail(BPMF_E_HIP, "grid upload: %s", hipGetErrorString(e));
  }
  c->dfree(c->grid_mem);
  c->grid_mem = mem;
  c->grid.cells = (const float*)mem;
  c->grid.nx = d->nx;
  c->grid.ny = d->ny;
  c->grid.nz = d->nz;
  c->grid.C = d->n_channels;
  c->grid.ox = (float)d->origin[0];
  c->grid.oy = (float)d->origin[1];
  c->grid.oz = (float)d->origin[2];
  c->grid.inv_h = (float)(1.0 / d->spacing);
  c->grid.quartic_mask = mask;
  c->has_grid = true;
  return BPMF_OK;
}

// Order of a ligand's terms of one kind (arity atoms each, t-th term's
// atoms at idx[arity t ..]) that spreads every atom over the 64-term
// chunks: a chunk adds the force on its terms' atoms at one position
// (first atom, second, ...) with one LDS atomic instruction per component,
// and lanes of one such instruction that add into the same accumulator are
// serialised.  Terms go, in their order, to the chunk with room where their
// atoms have been met least so far at the same positions (ties: the lower
// chunk); the terms of a chunk keep their relative order.  The order of the
// terms does not change any force (integer accumulation), only which lane
// sums which energy term.
static std::vector<int> spread_order(const int* idx, int n_terms, int arity,
                                     int n_atoms) {
  const int nc = (n_terms + kWave - 1) / kWave;
  std::vector<std::vector<int>> chunk(nc);
  // seen[(c arity + a) n_atoms + atom]: terms of chunk c with `atom` at
  // position a
  std::vector<int> seen((size_t)nc * arity * n_atoms, 0);
  auto cell = [&](int c, int a, int atom) -> int& {
    return seen[((size_t)c * arity + a) * n_atoms + atom];
  };
  for (int t = 0; t < n_terms; ++t) {
    int best = -1, best_score = 0;
    for (int c = 0; c < nc; ++c) {
      if ((int)chunk[c].size() >= kWave) continue;
      int score = 0;
      for (int a = 0; a < arity; ++a) score += cell(c, a, idx[arity * t + a]);
      if (best < 0 || score < best_score) {
        best = c;
        best_score = score;
      }
    }
    chunk[best].push_back(t);
    for (int a = 0; a < arity; ++a) ++cell(best, a, idx[arity * t + a]);
  }
  std::vector<int> order;
  order.reserve(n_terms);
  for (auto& ch : chunk) order.insert(order.end(), ch.begin(), ch.end());
  return order;
}

// Balanced deal of a ligand's bonded chunks (see sched_row) to the
// wavefronts of each launch width: chunks longest first, each to the
// wavefront with the least work so far (ties: the lower one), the
// wavefronts that hold atoms starting with their grid work.  The costs are the wave64 instruction counts of one
// chunk of each kind in the sweep kernel (roughly: torsion 175, angle 135,
// bond 45, an atom wavefront's grid work 250).  Each wavefront takes its
// chunks in kind order.
static std::vector<unsigned short> bonded_schedule(int n, int nb, int na,
                                                   int nt) {
  const int ntc = (nt + kWave - 1) / kWave, nac = (na + kWave - 1) / kWave;
  const int nch = bonded_chunks(nb, na, nt), row = sched_row(nb, na, nt);
  const int atom_waves = (n + kWave - 1) / kWave;
  std::vector<unsigned short> out(4 * (size_t)row, 0);
  auto cost = [&](int ch) { return ch < ntc ? 175 : ch < ntc + nac ? 135 : 45; };
  std::vector<int> order(nch);
  for (int ch = 0; ch < nch; ++ch) order[ch] = ch;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return cost(a) > cost(b); });
  for (int q = 0; q < 4; ++q) {
    const int W = 1 << q;
    const int nbw = W;
    std::vector<int> load(nbw, 0);
    std::vector<std::vector<int>> mine(nbw);
    for (int w = 0; w < nbw && w < atom_waves; ++w) load[w] = 250;
    for (int ch : order) {
      int best = 0;
      for (int w = 1; w < nbw; ++w)
        if (load[w] < load[best]) best = w;
      load[best] += cost(ch);
      mine[best].push_back(ch);
    }
    unsigned short* r = out.data() + (size_t)q * row;
    int j = 0;
    for (int w = 0; w < 9; ++w) {
      r[w] = (unsigned short)j;
      if (w < nbw) {
        std::sort(mine[w].begin(), mine[w].end());
        for (int ch : mine[w]) r[9 + j++] = (unsigned short)ch;
      }
    }
  }
  return out;
}

static bool supported_channels(int C) { return C == 3 || C == 5; }

// ============================================================================
// ligands
// ============================================================================
extern "C" int bpmf_ligand_setup(bpmf_ctx* c, const bpmf_ligand_desc* d,
                                 int* ligand_id) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!d || !ligand_id) return fail(BPMF_E_INVAL, "null descriptor or id");
  if (!c->has_grid) return fail(BPMF_E_STATE, "upload the grid first");
  const int C = c->grid.C;
  if (!supported_channels(C))
    return fail(BPMF_E_UNIMPL, "the sampler takes 3 or 5 channels, not %d",
                C);
  const int n = d->n_atoms, K = d->n_states;
  if (n < 1 || n > BPMF_MAX_ATOMS)
    return fail(BPMF_E_INVAL, "n_atoms %d outside 1..%d", n, BPMF_MAX_ATOMS);
  if (K < 1 || K > BPMF_MAX_STATES)
    return fail(BPMF_E_INVAL, "n_states %d outside 1..%d", K, BPMF_MAX_STATES);
  if ((int)c->ligs.size() >= 65535)
    return fail(BPMF_E_INVAL, "too many ligands");
  if (!d->mass || !d->scale || !d->T || !d->w || !d->dt_fs || !d->x0)
    return fail(BPMF_E_INVAL, "null per-atom or per-state array");
  if (d->n_bonds < 0 || d->n_angles < 0 || d->n_tors < 0 ||
      d->sample_capacity < 0)
    return fail(BPMF_E_INVAL, "negative count");
  if ((d->n_bonds && (!d->bond_ij || !d->bond_k_r0)) ||
      (d->n_angles && (!d->angle_ijk || !d->angle_k_t0)) ||
      (d->n_tors && (!d->tors_ijkl || !d->tors_v_n_g)))
    return fail(BPMF_E_INVAL, "null term array with nonzero count");
  for (int i = 0; i < n; ++i)
    if (!(d->mass[i] > 0) || !isfinite(d->mass[i]))
      return fail(BPMF_E_INVAL, "mass[%d] must be positive and finite", i);
  if (!finite_all(d->scale, (size_t)n * C))
    return fail(BPMF_E_INVAL, "non-finite scale factor");
  for (int k = 0; k < K; ++k) {
    if (!(d->T[k] > 0) || !isfinite(d->T[k]))
      return fail(BPMF_E_INVAL, "T[%d] must be positive and finite", k);
    if (!(d->dt_fs[k] > 0) || !isfinite(d->dt_fs[k]))
      return fail(BPMF_E_INVAL, "dt[%d] must be positive and finite", k);
  }
  if (!finite_all(d->w, (size_t)K * C))
    return fail(BPMF_E_INVAL, "non-finite state weight");
  if (!finite_all(d->site_center, 3) || !(d->d0 >= 0) || !isfinite(d->d0) ||
      !(d->k_restraint >= 0) || !isfinite(d->k_restraint))
    return fail(BPMF_E_INVAL, "bad restraint parameters");
  for (size_t i = 0; i < (size_t)K * n * 3; ++i)
    if (!isfinite(d->x0[i]))
      return fail(BPMF_E_INVAL, "non-finite start coordinate at %zu", i);
  auto check_idx = [&](const int* idx, int cnt, int ar, const char* what) -> int {
    for (int t = 0; t < cnt; ++t)
      for (int a = 0; a < ar; ++a) {
        const int v = idx[t * ar + a];
        if (v < 0 || v >= n)
          return fail(BPMF_E_INVAL, "%s %d: atom index %d out of range", what,
                      t, v);
        for (int b = 0; b < a; ++b)
          if (idx[t * ar + b] == v)
            return fail(BPMF_E_INVAL, "%s %d: repeated atom %d", what, t, v);
      }
    return BPMF_OK;
  };
  if ((rc = check_idx(d->bond_ij, d->n_bonds, 2, "bond"))) return rc;
  if ((rc = check_idx(d->angle_ijk, d->n_angles, 3, "angle"))) return rc;
  if ((rc = check_idx(d->tors_ijkl, d->n_tors, 4, "torsion"))) return rc;
  if (!finite_all(d->bond_k_r0, (size_t)d->n_bonds * 2) ||
      !finite_all(d->angle_k_t0, (size_t)d->n_angles * 2) ||
      !finite_all(d->tors_v_n_g, (size_t)d->n_tors * 3))
    return fail(BPMF_E_INVAL, "non-finite force-field parameter");

  const int nb = d->n_bonds, na = d->n_angles, nt = d->n_tors;
  const int n_slots = 2 * nb + 3 * na + 4 * nt;
  const int min_waves = n <= kWave ? 1 : 2;
  const int cap = d->sample_capacity;
  const int C1 = 1 + C;
  const int Km1 = std::max(K - 1, 1);

  // host staging of every device array
  std::vector<float> mass(n), inv_mass(n), scale((size_t)n * C);
  double M = 0;
  for (int i = 0; i < n; ++i) {
    mass[i] = (float)d->mass[i];
    inv_mass[i] = (float)(1.0 / d->mass[i]);
    M += d->mass[i];
  }
  for (size_t i = 0; i < (size_t)n * C; ++i) scale[i] = (float)d->scale[i];
  for (int t = 0; t < nt; ++t) {
    const double mult = d->tors_v_n_g[3 * t + 1];
    if (mult != floor(mult) || mult < 1 || mult > 6)
      return fail(BPMF_E_INVAL,
                  "torsion %d: multiplicity %g is not an integer in 1..6", t,
                  mult);
  }
  // device order of the terms: spread over the chunks (spread_order)
  const std::vector<int> bo = spread_order(d->bond_ij, nb, 2, n);
  const std::vector<int> ao = spread_order(d->angle_ijk, na, 3, n);
  const std::vector<int> to = spread_order(d->tors_ijkl, nt, 4, n);
  std::vector<int2> bij(nb);
  std::vector<float2> bpar(nb);
  for (int u = 0; u < nb; ++u) {
    const int t = bo[u];
    const int* q = d->bond_ij + 2 * t;
    bij[u] = make_int2(q[0], q[1]);
    bpar[u] = make_float2((float)d->bond_k_r0[2 * t],
                          (float)d->bond_k_r0[2 * t + 1]);
  }
  std::vector<int4> aijk(na);
  std::vector<float2> apar(na);
  for (int u = 0; u < na; ++u) {
    const int t = ao[u];
    const int* q = d->angle_ijk + 3 * t;
    aijk[u] = make_int4(q[0], q[1], q[2], 0);
    apar[u] = make_float2((float)d->angle_k_t0[2 * t],
                          (float)d->angle_k_t0[2 * t + 1]);
  }
  std::vector<int4> tijkl(nt);
  std::vector<float4> tpar(nt);
  for (int u = 0; u < nt; ++u) {
    const int t = to[u];
    const int* q = d->tors_ijkl + 4 * t;
    tijkl[u] = make_int4(q[0], q[1], q[2], q[3]);
    const double gam = d->tors_v_n_g[3 * t + 2];
    tpar[u] = make_float4((float)d->tors_v_n_g[3 * t],
                          (float)d->tors_v_n_g[3 * t + 1], (float)cos(gam),
                          (float)sin(gam));
  }
  std::vector<double> beta(K), wd((size_t)K * C);
  std::vector<float> Tf(K), dtf(K), wf((size_t)K * C);
  for (int k = 0; k < K; ++k) {
    beta[k] = 1.0 / (kRGas * d->T[k]);
    Tf[k] = (float)d->T[k];
    dtf[k] = (float)d->dt_fs[k];
  }
  for (size_t i = 0; i < (size_t)K * C; ++i) {
    wd[i] = d->w[i];
    wf[i] = (float)d->w[i];
  }
  std::vector<int> sor(K), ros(K);
  for (int k = 0; k < K; ++k) sor[k] = ros[k] = k;

  // one arena per ligand
  Arena A;
  const size_t o_mass = A.add(n * 4), o_imass = A.add(n * 4),
               o_scale = A.add((size_t)n * C * 4), o_bij = A.add(nb * 8),
               o_bpar = A.add(nb * 8), o_aijk = A.add(na * 16),
               o_apar = A.add(na * 8), o_tijkl = A.add(nt * 16),
               o_tpar = A.add(nt * 16),
               o_sched = A.add((size_t)4 * sched_row(nb, na, nt) * 2),
               o_beta = A.add(K * 8),
               o_Tf = A.add(K * 4), o_dt = A.add(K * 4),
               o_wf = A.add((size_t)K * C * 4), o_wd = A.add((size_t)K * C * 8),
               o_x = A.add((size_t)K * n * 12), o_comps = A.add((size_t)K * C1 * 8),
               o_sor = A.add(K * 4), o_ros = A.add(K * 4),
               o_counters = A.add(8 * 4), o_hacc = A.add(K * 8),
               o_htry = A.add(K * 8), o_eacc = A.add(Km1 * 8),
               o_etry = A.add(Km1 * 8), o_rcnt = A.add(K * 8),
               o_rnrec = A.add(K * 8), o_rpend = A.add(2 * K * 4),
               o_rsor = A.add(2 * K * 4),
               o_scomp = A.add((size_t)2 * K * C1 * 8),
               o_fcache = A.add((size_t)2 * K * n * (3 + 3 * C) * 4),
               o_frc = A.add((size_t)2 * K * 4 * 4), o_fvalid = A.add(K * 4),
               // right after fvalid: the kernels find it from that pointer
               o_rtend = A.add(rt_region_bytes(K)),
               o_xacc = A.add(K * 8), o_xtry = A.add(K * 8),
               o_sx = A.add((size_t)cap * K * n * 12),
               o_sc = A.add((size_t)cap * K * C1 * 8);
  {
    // every kernel stages the topology in LDS next to its working areas
    const int need = block_lds_bytes(min_waves, true, n, nb, na, nt);
    if (need > 65536)
      return fail(BPMF_E_INVAL,
                  "topology too large: %d bytes of LDS per replica (max 65536)",
                  need);
  }
  char* base = (char*)c->dalloc(A.total);
  if (!base) return fail(BPMF_E_NOMEM, "ligand allocation of %zu bytes failed",
                         A.total);
  auto up = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(base + off, src, bytes, hipMemcpyHostToDevice,
                          c->stream);
  };
  hipError_t e = hipSuccess;
  auto chain = [&](hipError_t x) {
    if (e == hipSuccess) e = x;
  };
  chain(up(o_mass, mass.data(), n * 4));
  chain(up(o_imass, inv_mass.data(), n * 4));
  chain(up(o_scale, scale.data(), (size_t)n * C * 4));
  chain(up(o_bij, bij.data(), nb * 8));
  chain(up(o_bpar, bpar.data(), nb * 8));
  chain(up(o_aijk, aijk.data(), na * 16));
  chain(up(o_apar, apar.data(), na * 8));
  chain(up(o_tijkl, tijkl.data(), nt * 16));
  chain(up(o_tpar, tpar.data(), nt * 16));
  const std::vector<unsigned short> sched = bonded_schedule(n, nb, na, nt);
  chain(up(o_sched, sched.data(), sched.size() * 2));
  chain(up(o_beta, beta.data(), K * 8));
  chain(up(o_Tf, Tf.data(), K * 4));
  chain(up(o_dt, dtf.data(), K * 4));
  chain(up(o_wf, wf.data(), (size_t)K * C * 4));
  chain(up(o_wd, wd.data(), (size_t)K * C * 8));
  chain(up(o_x, d->x0, (size_t)K * n * 12));
  chain(up(o_sor, sor.data(), K * 4));
  chain(up(o_ros, ros.data(), K * 4));
  chain(hipMemsetAsync(base + o_counters, 0, 8 * 4, c->stream));
  chain(hipMemsetAsync(base + o_hacc, 0, K * 8, c->stream));
  chain(hipMemsetAsync(base + o_htry, 0, K * 8, c->stream));
  chain(hipMemsetAsync(base + o_eacc, 0, Km1 * 8, c->stream));
  chain(hipMemsetAsync(base + o_etry, 0, Km1 * 8, c->stream));
  chain(hipMemsetAsync(base + o_rcnt, 0, o_sx - o_rcnt, c->stream));
  // round trips: replica r starts in state r
  std::vector<int> rte(rt_region_bytes(K) / 4, 0);  // trip count 0
  for (int r = 0; r < K; ++r) rte[r] = r == 0 ? 0 : -1;
  chain(up(o_rtend, rte.data(), rt_region_bytes(K)));
  chain(hipStreamSynchronize(c->stream));
  if (e != hipSuccess) {
    c->dfree(base);
    return fail(BPMF_E_HIP, "ligand upload: %s", hipGetErrorString(e));
  }
  LigHost h{};
  LigDev& L = h.dev;
  L.n = n;
  L.K = K;
  L.C = C;
  L.nb = nb;
  L.na = na;
  L.nt = nt;
  L.n_slots = n_slots;
  L.id = (int)c->ligs.size();
  L.cap = cap;
  for (int a = 0; a < 3; ++a) L.site[a] = (float)d->site_center[a];
  L.d0 = (float)d->d0;
  L.krest = (float)d->k_restraint;
  L.inv_total_mass = (float)(1.0 / M);
  L.mass = (const float*)(base + o_mass);
  L.inv_mass = (const float*)(base + o_imass);
  L.scale = (const float*)(base + o_scale);
  L.bij = (const int2*)(base + o_bij);
  L.bpar = (const float2*)(base + o_bpar);
  L.aijk = (const int4*)(base + o_aijk);
  L.apar = (const float2*)(base + o_apar);
  L.tijkl = (const int4*)(base + o_tijkl);
  L.tpar = (const float4*)(base + o_tpar);
  L.bsched = (const unsigned short*)(base + o_sched);
  L.beta = (const double*)(base + o_beta);
  L.Tf = (const float*)(base + o_Tf);
  L.dtf = (const float*)(base + o_dt);
  L.wf = (const float*)(base + o_wf);
  L.wd = (const double*)(base + o_wd);
  L.x = (float*)(base + o_x);
  L.comps = (double*)(base + o_comps);
  L.state_of_replica = (int*)(base + o_sor);
  L.replica_of_state = (int*)(base + o_ros);
  L.counter = (unsigned long long*)(base + o_counters);
  L.n_rec = L.counter + 1;
  L.nonfinite = L.counter + 2;

  L.rcnt = (unsigned long long*)(base + o_rcnt);
  L.rnrec = (unsigned long long*)(base + o_rnrec);
  L.rpend = (int*)(base + o_rpend);
  L.rsor = (int*)(base + o_rsor);
  L.scomp = (double*)(base + o_scomp);
  L.fcache = (float*)(base + o_fcache);
  L.frc = (float*)(base + o_frc);
  L.fvalid = (int*)(base + o_fvalid);
  L.hmc_acc = (unsigned long long*)(base + o_hacc);
  L.hmc_try = (unsigned long long*)(base + o_htry);
  L.ex_acc = (unsigned long long*)(base + o_eacc);
  L.ex_try = (unsigned long long*)(base + o_etry);
  L.samp_x = (float*)(base + o_sx);
  L.samp_c = (double*)(base + o_sc);
  h.arena = base;
  h.state_bytes = o_sx;
  L.ext_acc = (unsigned long long*)(base + o_xacc);
  L.ext_try = (unsigned long long*)(base + o_xtry);
  h.ext_acc = L.ext_acc;
  h.ext_try = L.ext_try;
  h.min_waves = min_waves;
  h.sweep_waves = min_waves;
  h.counter = 0;
  h.n_rec = 0;
  h.beta = beta;
  h.wd = wd;
  c->ligs.push_back(h);
  rc = rebuild_tables(c);
  if (rc) {
    c->dfree(base);
    c->ligs.pop_back();
    return rc;
  }
  // initial cached components
  const LigDev* dl = c->d_ligs + (c->ligs.size() - 1);
  HIP_TRY(launch_recompute_comps(c->grid, dl, min_waves, K,
                                 lds_of(c->ligs.back(), min_waves, false),
                                 false, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  *ligand_id = L.id;
  return BPMF_OK;
}

namespace {
// proposal network scratch (see mlp_scratch); pose moves of one ligand
struct MlpBufs {
  float *Z1, *H1, *Z2, *H2, *out, *dout, *dZ2, *dZ1, *bf, *bp;
  double* loss_part;
};
int mlp_scratch(bpmf_ctx* c, int B, MlpBufs* b);
int build_pose_tables(bpmf_ctx* c);
int refresh_pose_weights(bpmf_ctx* c);
int pair_sample_refresh(bpmf_ctx* c, int lid);
// closing a unit of neighbour-scheme sweeps inside the pose-move launches:
// the ligands [l0, l1) whose run ends there and the run's parameters
struct UnitClose {
  int l0 = 0, l1 = 0;
  int exchange_every = 0, sample_every = 0;
};
int pose_move_batch(bpmf_ctx* c, int only, hipStream_t st,
                    const UnitClose* close = nullptr);
int external_moves_range(bpmf_ctx* c, int l0, int l1, int n_moves,
                         int k_max, double sigma, hipStream_t st);
int check_external(int n_moves, int k_max, double sigma);
}  // namespace

// ============================================================================
// sampling
// ============================================================================
// sweeps of every ligand (only = -1) or of ligand `only` alone
static int hmc_sweep_impl(bpmf_ctx* c, const bpmf_sweep_args* a, int only) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!a) return fail(BPMF_E_INVAL, "null sweep arguments");
  if (c->ligs.empty()) return fail(BPMF_E_STATE, "no ligand set up");
  if (only >= 0 && (rc = check_lig(c, only))) return rc;
  // the ligands this call advances: [l0, l1)
  const int l0 = only >= 0 ? only : 0;
  const int l1 = only >= 0 ? only + 1 : (int)c->ligs.size();
  if (a->n_sweeps < 0 || a->n_leapfrog < 1 || a->exchange_every < 0 ||
      a->sample_every < 0)
    return fail(BPMF_E_INVAL, "bad sweep arguments (n_sweeps %d, n_leapfrog %d,"
                " exchange_every %d, sample_every %d)", a->n_sweeps,
                a->n_leapfrog, a->exchange_every, a->sample_every);
  if (a->exchange_scheme != 0 && a->exchange_scheme != 1)
    return fail(BPMF_E_INVAL, "exchange_scheme must be 0 or 1");
  if (a->exchange_scheme == 1 && a->max_sep < 1)
    return fail(BPMF_E_INVAL, "max_sep must be >= 1");
  if (a->exchange_sweeps < 0 || a->exchange_sweeps > BPMF_MAX_EXCHANGE_SWEEPS)
    return fail(BPMF_E_INVAL, "exchange_sweeps must be in 0..%d",
                BPMF_MAX_EXCHANGE_SWEEPS);
  const int n_sub = a->exchange_sweeps > 1 ? a->exchange_sweeps : 1;
  if (n_sub > 1 && a->exchange_scheme != 1)
    return fail(BPMF_E_INVAL, "exchange_sweeps > 1 needs exchange_scheme 1");
  if (a->pose_move_every < 0)
    return fail(BPMF_E_INVAL, "pose_move_every must be >= 0");
  if ((rc = check_external(a->external_moves, a->external_k_max,
                           a->external_sigma)))
    return rc;
  // sample capacity check (host mirrors of the device counters)
  std::vector<int64_t> add(c->ligs.size(), 0);
  if (a->sample_every > 0) {
    for (int l = l0; l < l1; ++l) {
      const LigHost& h = c->ligs[l];
      const int64_t se = a->sample_every;
      add[l] = (int64_t)((h.counter + a->n_sweeps) / se) -
               (int64_t)(h.counter / se);
      if (h.n_rec + add[l] > h.dev.cap)
        return fail(BPMF_E_INVAL,
                    "ligand %d: %lld recorded + %lld new samples per state "
                    "exceed capacity %d", l, (long long)h.n_rec,
                    (long long)add[l], h.dev.cap);
    }
  }
  TailArgs tail{a->exchange_every, a->exchange_scheme, a->max_sep,
                a->sample_every, n_sub};
  const int nl = l1 - l0;
  const LigDev* dl = c->d_ligs + l0;  // table entries of the call's ligands
  // scheme 0: each sweep applies the previous one's exchange and record in
  // its own blocks (begin/finish kernels bracket the run); scheme 1: a tail
  // kernel after every sweep
  auto enqueue_sweep = [&](hipStream_t st) -> int {
    if (only >= 0) {
      const LigHost& h = c->ligs[only];
      HIP_TRY(launch_hmc_sweep(c->grid, c->d_ligs, nullptr, h.dev.K,
                               h.sweep_waves, lds_of(h, h.sweep_waves, true),
                               a->n_leapfrog, c->seed, tail, &h.dev,
                               h.dev.pairs_on != 0, st));
    } else {
      // classes hold different ligands: the first runs on `st`, each other
      // one on a stream of its own forked from `st` and joined back after
      // it, so that the launches overlap (in a captured graph: parallel
      // branches)
      int nq = 0;
      for (int q = 0; q < bpmf_ctx::kWaveClasses; ++q) nq += c->class_n[q] > 0;
      if (nq > 1) {
        if (!c->class_fork)
          HIP_TRY(hipEventCreateWithFlags(&c->class_fork,
                                          hipEventDisableTiming));
        for (int q = 0; q < bpmf_ctx::kWaveClasses; ++q) {
          if (!c->class_n[q]) continue;
          if (!c->class_stream[q])
            HIP_TRY(hipStreamCreateWithFlags(&c->class_stream[q],
                                             hipStreamNonBlocking));
          if (!c->class_join[q])
            HIP_TRY(hipEventCreateWithFlags(&c->class_join[q],
                                            hipEventDisableTiming));
        }
        HIP_TRY(hipEventRecord(c->class_fork, st));
      }
      bool forked[bpmf_ctx::kWaveClasses] = {false, false, false, false};
      bool first = true;
      // widest class first: it usually holds the heaviest ligands
      for (int qi = 0; qi < bpmf_ctx::kWaveClasses; ++qi) {
        const int q = bpmf_ctx::kWaveClasses - 1 - qi;
        if (!c->class_n[q]) continue;
        hipStream_t sq = st;
        if (!first) {
          sq = c->class_stream[q];
          HIP_TRY(hipStreamWaitEvent(sq, c->class_fork, 0));
          forked[q] = true;
        }
        first = false;
        HIP_TRY(launch_hmc_sweep(
            c->grid, c->d_ligs, c->d_tasks + c->class_off[q], c->class_n[q],
            1 << q, c->class_lds[q], a->n_leapfrog, c->seed, tail,
            c->class_single[q] >= 0 ? &c->ligs[c->class_single[q]].dev
                                    : nullptr,
            c->class_pairs[q], sq));
        if (forked[q]) HIP_TRY(hipEventRecord(c->class_join[q], sq));
      }
      for (int q = 0; q < bpmf_ctx::kWaveClasses; ++q)
        if (forked[q]) HIP_TRY(hipStreamWaitEvent(st, c->class_join[q], 0));
    }
    if (tail.scheme == 1)
      HIP_TRY(launch_sweep_tail(dl, nl, tail.exchange_every, tail.scheme,
                                tail.max_sep, n_sub, tail.sample_every,
                                c->seed, st));
    return BPMF_OK;
  };
  if (a->n_sweeps == 0) return BPMF_OK;
  // units of P sweeps closed by pose moves and/or external moves
  const int NX = a->external_moves;
  const int P = a->pose_move_every > 0 ? a->pose_move_every : (NX > 0 ? 1 : 0);
  // a run of `count` sweeps with its exchange/record bookkeeping
  auto enqueue_run = [&](hipStream_t st, int count) -> int {
    if (tail.scheme == 0) HIP_TRY(launch_sweep_begin(dl, nl, st));
    for (int s = 0; s < count; ++s) {
      const int r = enqueue_sweep(st);
      if (r) return r;
    }
    if (tail.scheme == 0)
      HIP_TRY(launch_sweep_finish(dl, nl, tail.exchange_every,
                                  tail.sample_every, c->seed, st));
    return BPMF_OK;
  };
  // units closed by pose moves alone, with every ligand of the call
  // carrying a proposal: the run's end and the next run's start are folded
  // into the pose-move launches (pose_move_batch with a UnitClose)
  bool fused = a->pose_move_every > 0 && NX == 0 && tail.scheme == 0;
  for (int l = l0; l < l1 && fused; ++l) fused = c->ligs[l].has_prop;
  UnitClose uc;
  uc.l0 = l0;
  uc.l1 = l1;
  uc.exchange_every = tail.exchange_every;
  uc.sample_every = tail.sample_every;
  // one pose move of every ligand that has a proposal (when asked), then
  // the external moves of every ligand
  auto enqueue_pose = [&](hipStream_t st) -> int {
    if (a->pose_move_every > 0) {
      const int r = pose_move_batch(c, only, st);
      if (r) return r;
    }
    if (NX > 0)
      return external_moves_range(c, l0, l1, NX, a->external_k_max,
                                  a->external_sigma, st);
    return BPMF_OK;
  };
  // (re)capture `fn` into the context's graph under `key`; the kernels read
  // every per-sweep quantity (counters, state maps) from device memory, so
  // one capture replays unchanged
  auto ensure_graph = [&](const int (&key)[bpmf_ctx::kKey], auto&& fn) -> int {
    if (c->graph_exec && c->graph_version == c->table_version &&
        memcmp(key, c->graph_key, sizeof(key)) == 0)
      return BPMF_OK;
    c->drop_graph();
    if (!c->cap_stream)
      HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(c->cap_stream,
                                  hipStreamCaptureModeThreadLocal));
    const int crc = fn(c->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(c->cap_stream, &g);
    if (crc) {
      if (g) (void)hipGraphDestroy(g);
      return crc;
    }
    if (ec != hipSuccess)
      return fail(BPMF_E_HIP, "graph capture: %s", hipGetErrorString(ec));
    c->graph = g;
    HIP_TRY(hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0));
    c->graph_version = c->table_version;
    memcpy(c->graph_key, key, sizeof(key));
    return BPMF_OK;
  };
  auto launch_timed = [&](int weight, auto&& fn) -> int {
    hipEvent_t t0, t1;
    const bool timed = c->timer_begin(BPMF_TIMER_HMC, &t0, &t1, weight);
    if (timed) HIP_TRY(hipEventRecord(t0, c->stream));
    const int r = fn();
    if (r) return r;
    if (timed) HIP_TRY(hipEventRecord(t1, c->stream));
    return BPMF_OK;
  };
  const int chunk = c->graph_chunk;
  if (P > 0) {
    // units of P sweeps, each followed by the unit's moves; the network's
    // scratch is sized before any capture
    if (a->pose_move_every > 0) {
      if ((rc = build_pose_tables(c)) || (rc = refresh_pose_weights(c)))
        return rc;
      MlpBufs b;
      if (c->n_ptasks > 0 && (rc = mlp_scratch(c, c->n_ptasks, &b))) return rc;
    }
    const int units = a->n_sweeps / P, rest = a->n_sweeps % P;
    auto unit = [&](hipStream_t st) -> int {
      if (fused) {
        for (int s = 0; s < P; ++s) {
          const int r = enqueue_sweep(st);
          if (r) return r;
        }
        return pose_move_batch(c, only, st, &uc);
      }
      const int r = enqueue_run(st, P);
      return r ? r : enqueue_pose(st);
    };
    // a fused unit's first sweep reads the run state its predecessor's
    // pose moves leave; the first unit's comes from a begin launch
    if (fused && units > 0) HIP_TRY(launch_sweep_begin(dl, nl, c->stream));
    // G units per captured graph (about `chunk` sweeps), so that the host
    // launches one graph per chunk however short the units are; the units
    // left over run as plain launches (the same kernels, the same bits)
    const int G = chunk > 0 ? std::max(1, chunk / P) : 0;
    int u = 0;
    if (G > 0 && units >= G) {
      int sg[2];
      memcpy(sg, &a->external_sigma, sizeof(sg));
      const int key[bpmf_ctx::kKey] = {
          a->n_leapfrog, a->exchange_every, a->exchange_scheme, a->max_sep,
          a->sample_every, fused ? -G : G, P, a->pose_move_every, NX,
          a->external_k_max, sg[0], sg[1], n_sub, only};
      if ((rc = ensure_graph(key, [&](hipStream_t st) -> int {
             for (int q = 0; q < G; ++q) {
               const int r = unit(st);
               if (r) return r;
             }
             return BPMF_OK;
           })))
        return rc;
      for (; u + G <= units; u += G)
        if ((rc = launch_timed(G * P, [&]() -> int {
               HIP_TRY(hipGraphLaunch(c->graph_exec, c->stream));
               return BPMF_OK;
             })))
          return rc;
    }
    for (; u < units; ++u)
      if ((rc = launch_timed(P, [&] { return unit(c->stream); }))) return rc;
    if (rest > 0 &&
        (rc = launch_timed(rest, [&] { return enqueue_run(c->stream, rest); })))
      return rc;
  } else {
    if (tail.scheme == 0) HIP_TRY(launch_sweep_begin(dl, nl, c->stream));
    int done = 0;
    if (chunk > 0 && a->n_sweeps >= chunk) {
      const int key[bpmf_ctx::kKey] = {
          a->n_leapfrog, a->exchange_every, a->exchange_scheme, a->max_sep,
          a->sample_every, chunk, 0, 0, 0, 0, 0, -1, n_sub, only};
      if ((rc = ensure_graph(key, [&](hipStream_t st) -> int {
             for (int s = 0; s < chunk; ++s) {
               const int r = enqueue_sweep(st);
               if (r) return r;
             }
             return BPMF_OK;
           })))
        return rc;
      for (; done + chunk <= a->n_sweeps; done += chunk)
        if ((rc = launch_timed(chunk, [&]() -> int {
               HIP_TRY(hipGraphLaunch(c->graph_exec, c->stream));
               return BPMF_OK;
             })))
          return rc;
    }
    for (; done < a->n_sweeps; ++done)
      if ((rc = launch_timed(1, [&] { return enqueue_sweep(c->stream); })))
        return rc;
    if (tail.scheme == 0) {
      hipEvent_t t0, t1;
      const bool timed = c->timer_begin(BPMF_TIMER_TAIL, &t0, &t1);
      if (timed) HIP_TRY(hipEventRecord(t0, c->stream));
      HIP_TRY(launch_sweep_finish(dl, nl, tail.exchange_every,
                                  tail.sample_every, c->seed, c->stream));
      if (timed) HIP_TRY(hipEventRecord(t1, c->stream));
    }
  }
  for (int l = l0; l < l1; ++l) {
    c->ligs[l].counter += (uint64_t)a->n_sweeps;
    c->ligs[l].n_rec += add[l];
  }
  return BPMF_OK;
}

extern "C" int bpmf_hmc_sweep(bpmf_ctx* c, const bpmf_sweep_args* a) {
  return hmc_sweep_impl(c, a, -1);
}

extern "C" int bpmf_hmc_sweep_ligand(bpmf_ctx* c, int ligand_id,
                                     const bpmf_sweep_args* a) {
  if (c && check_lig(c, ligand_id)) return BPMF_E_INVAL;
  return hmc_sweep_impl(c, a, ligand_id);
}

extern "C" int bpmf_exchange(bpmf_ctx* c, int ligand_id, int scheme,
                             int max_sep, int n_sweeps) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (c->ligs.empty()) return fail(BPMF_E_STATE, "no ligand set up");
  if (ligand_id != -1 && (rc = check_lig(c, ligand_id))) return rc;
  if (scheme != 0 && scheme != 1)
    return fail(BPMF_E_INVAL, "scheme must be 0 or 1");
  if (scheme == 1 && max_sep < 1) return fail(BPMF_E_INVAL, "max_sep must be >= 1");
  if (n_sweeps < 1 || n_sweeps > BPMF_MAX_EXCHANGE_SWEEPS)
    return fail(BPMF_E_INVAL, "n_sweeps must be in 1..%d",
                BPMF_MAX_EXCHANGE_SWEEPS);
  if (ligand_id == -1)
    HIP_TRY(launch_exchange(c->d_ligs, (int)c->ligs.size(), scheme, max_sep,
                            n_sweeps, c->seed, c->stream));
  else
    HIP_TRY(launch_exchange(c->d_ligs + ligand_id, 1, scheme, max_sep,
                            n_sweeps, c->seed, c->stream));
  return BPMF_OK;
}

// ============================================================================
// u_kn, MBAR
// ============================================================================
// u_kn of several ligands: one persistent launch per wavefront class, the
// job table staged through pinned memory (the previous upload must have
// left it before it is rewritten)
namespace {
// launch plan of an energy-matrix batch: jobs grouped by wavefront class,
// each group followed by a sentinel
struct UknPlan {
  int group = 16;  // samples whose columns are staged before being written
  int n_jobs = 0;  // table entries, sentinels included (0: nothing to do)
  int64_t total[bpmf_ctx::kWaveClasses] = {0, 0, 0, 0};
  int off[bpmf_ctx::kWaveClasses] = {0, 0, 0, 0};
  int cnt[bpmf_ctx::kWaveClasses] = {0, 0, 0, 0};
  int lds[bpmf_ctx::kWaveClasses] = {0, 0, 0, 0};
  bool pairs[bpmf_ctx::kWaveClasses] = {false, false, false, false};
  // one wavefront per sample (k_energy_matrix_wave) and its LDS
  bool per_wave[bpmf_ctx::kWaveClasses] = {false, false, false, false};
  int wave_lds[bpmf_ctx::kWaveClasses] = {0, 0, 0, 0};
};

// Estimated issue cost of one u_kn sample of a ligand whose atoms need W
// wavefronts (one wavefront per sample: W atoms per lane): the grid terms
// of each lane's atoms, the 64-term chunks of each bonded kind (roughly
// 150, 90 and 40 instructions per term), the sums and the column.  Only
// its proportions matter: it splits a launch's samples into shares of
// equal work.
int ukn_sample_cost(const LigDev& d, int W) {
  auto chunks = [](int m) { return (m + kWave - 1) / kWave; };
  return 100 * W + 150 * chunks(d.nt) + 90 * chunks(d.na) +
         40 * chunks(d.nb) + 200 + 4 * d.K;
}

// Validates an energy-matrix batch and writes its job table into `jobs`
// (room for n + kWaveClasses entries); allocates nothing.
int ukn_plan(bpmf_ctx* c, int n, const int* ligand_ids,
             const float* const* dev_samples, const int64_t* n_samples,
             double* const* dev_ukn, const int64_t* ld, UknJob* jobs,
             UknPlan* p) {
  int rc = check_ctx(c);
  if (rc) return rc;
  *p = UknPlan{};
  if (n < 0) return fail(BPMF_E_INVAL, "negative batch size");
  if (n == 0) return BPMF_OK;
  if (!ligand_ids || !n_samples || !dev_ukn || !ld)
    return fail(BPMF_E_INVAL, "null energy-matrix argument");
  int64_t total = 0;
  for (int i = 0; i < n; ++i) {
    if ((rc = check_lig(c, ligand_ids[i]))) return rc;
    const LigHost& h = c->ligs[ligand_ids[i]];
    const int64_t ns = n_samples[i];
    if (ns < 0)
      return fail(BPMF_E_INVAL, "entry %d: negative n_samples", i);
    if (!dev_ukn[i] && ns > 0)
      return fail(BPMF_E_INVAL, "entry %d: null u_kn output", i);
    if (ld[i] < ns)
      return fail(BPMF_E_INVAL, "entry %d: ld %lld < n_samples %lld", i,
                  (long long)ld[i], (long long)ns);
    if ((!dev_samples || !dev_samples[i]) && ns != h.n_rec * h.dev.K)
      return fail(BPMF_E_INVAL,
                  "entry %d: recorded samples: n_samples must be %lld "
                  "(records x K)",
                  i, (long long)(h.n_rec * h.dev.K));
    total += ns;
  }
  if (total == 0) return BPMF_OK;
  // columns staged in groups of up to 16 samples (a 128-byte line of each
  // u_kn row), fewer when group x K doubles would exceed 16 KB of LDS
  int group = 16, max_K = 0;
  for (int i = 0; i < n; ++i)
    max_K = std::max(max_K, c->ligs[ligand_ids[i]].dev.K);
  while (group > 1 && (int64_t)group * max_K * 8 > 16384) group /= 2;
  // LDS of a block: evaluation areas and topology, the states' weights and
  // beta_k, the group's columns
  auto ukn_lds = [&](const LigHost& h, int W) {
    return lds_of(h, W, false) +
           (int)((size_t)h.dev.K * (h.dev.C + 1 + group) * sizeof(double));
  };
  for (int i = 0; i < n; ++i) {
    const LigHost& h = c->ligs[ligand_ids[i]];
    const int need = ukn_lds(h, h.min_waves);
    if (need > 65536)
      return fail(BPMF_E_UNIMPL,
                  "entry %d: %d bytes of LDS per block (topology and %d "
                  "states' weights and columns; max 65536)",
                  i, need, h.dev.K);
  }
  // Ligands of up to 64 and of 65-128 atoms run as two launches side by
  // side, or, when the larger ones hold at least 40 % of the estimated
  // cost, as one launch of the two-atoms-per-lane kernel (its occupancy
  // equals the one-atom kernel's; a lane without a second atom skips it):
  // a minority of large ligands fits in the tail of the small ligands'
  // launch, a majority would leave two tails (config-3 sample set, 27 %:
  // 3.9e10 atom-evals/s side by side against 3.7e10 merged; config 5,
  // 60 %: 2.9e10 against 3.1e10).  Not when one of them has pair terms in
  // its energy or needs more LDS per wavefront than that kernel has.
  bool merge = true;
  double cost1 = 0.0, cost2 = 0.0;
  for (int i = 0; i < n; ++i) {
    const LigHost& h = c->ligs[ligand_ids[i]];
    if (h.min_waves > 2) continue;
    if (h.dev.pairs_on ||
        ukn_wave_lds_bytes(h.dev.K, h.dev.C, 2, h.dev.nb, h.dev.na,
                           h.dev.nt) > 65536)
      merge = false;
    (h.min_waves == 1 ? cost1 : cost2) +=
        (double)ukn_sample_cost(h.dev, h.min_waves) * (double)n_samples[i];
  }
  if (cost2 < 0.4 * (cost1 + cost2)) merge = false;
  auto class_waves = [&](const LigHost& h) {
    return merge && h.min_waves <= 2 ? 2 : h.min_waves;
  };
  int nj = 0;
  for (int q = 0; q < bpmf_ctx::kWaveClasses; ++q) {
    const int W = 1 << q;
    p->off[q] = nj;
    int64_t first = 0, cfirst = 0;
    for (int i = 0; i < n; ++i) {
      const LigHost& h = c->ligs[ligand_ids[i]];
      if (class_waves(h) != W || n_samples[i] == 0) continue;
      UknJob J;
      J.lig = ligand_ids[i];
      J.cost = ukn_sample_cost(h.dev, h.min_waves);
      J.cfirst = cfirst;
      cfirst += J.cost * n_samples[i];
      J.xs = dev_samples && dev_samples[i] ? dev_samples[i] : h.dev.samp_x;
      J.ukn = dev_ukn[i];
      J.n = n_samples[i];
      J.ld = ld[i];
      J.first = first;
      first += J.n;
      jobs[nj++] = J;
      p->lds[q] = std::max(p->lds[q], ukn_lds(h, W));
      p->pairs[q] = p->pairs[q] || h.dev.pairs_on;
      if (W <= 2)
        p->wave_lds[q] = std::max(
            p->wave_lds[q],
            ukn_wave_lds_bytes(h.dev.K, h.dev.C, W, h.dev.nb, h.dev.na,
                               h.dev.nt));
    }
    // a class whose ligands have no pair terms in their energy and whose
    // per-wavefront LDS fits runs one wavefront per sample
    p->per_wave[q] = W <= 2 && !p->pairs[q] && p->wave_lds[q] <= 65536;
    p->cnt[q] = nj - p->off[q];
    p->total[q] = first;
    UknJob end{};
    end.first = first;
    end.cfirst = cfirst;
    end.cost = 1;
    jobs[nj++] = end;
  }
  p->group = group;
  p->n_jobs = nj;
  return BPMF_OK;
}

// the launches of a planned batch, the job table at d_jobs on the device.
// overlap: the classes' launches run side by side, the first on the
// context's stream and each other one on a stream of its own forked from
// it and joined back (the streams and events are created on first use);
// otherwise one after the other.  Timed as one interval.
int ukn_launch(bpmf_ctx* c, const UknPlan& p, const UknJob* d_jobs,
               bool timed_ok, bool overlap) {
  int act[bpmf_ctx::kWaveClasses], na = 0;
  for (int q = 0; q < bpmf_ctx::kWaveClasses; ++q)
    if (p.total[q] != 0) act[na++] = q;
  if (na == 0) return BPMF_OK;
  hipEvent_t t0, t1;
  const bool timed =
      timed_ok && c->timer_begin(BPMF_TIMER_COMPONENTS, &t0, &t1);
  if (timed) HIP_TRY(hipEventRecord(t0, c->stream));
  const bool fork = overlap && na > 1;
  if (fork) {
    if (!c->class_fork)
      HIP_TRY(hipEventCreateWithFlags(&c->class_fork, hipEventDisableTiming));
    for (int i = 1; i < na; ++i) {
      const int q = act[i];
      if (!c->class_stream[q])
        HIP_TRY(hipStreamCreateWithFlags(&c->class_stream[q],
                                         hipStreamNonBlocking));
      if (!c->class_join[q])
        HIP_TRY(hipEventCreateWithFlags(&c->class_join[q],
                                        hipEventDisableTiming));
    }
    HIP_TRY(hipEventRecord(c->class_fork, c->stream));
  }
  for (int i = 0; i < na; ++i) {
    const int q = act[i];
    hipStream_t sq = c->stream;
    if (fork && i > 0) {
      sq = c->class_stream[q];
      HIP_TRY(hipStreamWaitEvent(sq, c->class_fork, 0));
    }
    HIP_TRY(launch_energy_matrix(
        c->grid, c->d_ligs, 1 << q, d_jobs + p.off[q], p.cnt[q], p.total[q],
        p.group, p.per_wave[q] ? p.wave_lds[q] : p.lds[q], c->n_cu,
        p.pairs[q], p.per_wave[q], sq));
    if (fork && i > 0) HIP_TRY(hipEventRecord(c->class_join[q], sq));
  }
  if (fork)
    for (int i = 1; i < na; ++i)
      HIP_TRY(hipStreamWaitEvent(c->stream, c->class_join[act[i]], 0));
  if (timed) HIP_TRY(hipEventRecord(t1, c->stream));
  return BPMF_OK;
}
}  // namespace

extern "C" int bpmf_energy_matrix_batch(bpmf_ctx* c, int n,
                                        const int* ligand_ids,
                                        const float* const* dev_samples,
                                        const int64_t* n_samples,
                                        double* const* dev_ukn,
                                        const int64_t* ld) {
  std::vector<UknJob> jobs((size_t)std::max(n, 0) + bpmf_ctx::kWaveClasses);
  UknPlan p;
  int rc = ukn_plan(c, n, ligand_ids, dev_samples, n_samples, dev_ukn, ld,
                    jobs.data(), &p);
  if (rc || p.n_jobs == 0) return rc;
  rc = ensure_scratch(c, &c->comps_mem, &c->comps_bytes,
                      p.n_jobs * sizeof(UknJob));
  if (rc) return rc;
  if (!c->jobs_copied) HIP_TRY(hipEventCreate(&c->jobs_copied));
  HIP_TRY(hipEventSynchronize(c->jobs_copied));
  if (c->jobs_host_n < (size_t)p.n_jobs) {
    if (c->jobs_host) HIP_TRY(hipHostFree(c->jobs_host));
    c->jobs_host = nullptr;
    c->jobs_host_n = 0;
    HIP_TRY(hipHostMalloc((void**)&c->jobs_host, p.n_jobs * sizeof(UknJob)));
    c->jobs_host_n = p.n_jobs;
  }
  memcpy(c->jobs_host, jobs.data(), p.n_jobs * sizeof(UknJob));
  UknJob* d_jobs = (UknJob*)c->comps_mem;
  HIP_TRY(hipMemcpyAsync(d_jobs, c->jobs_host, p.n_jobs * sizeof(UknJob),
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipEventRecord(c->jobs_copied, c->stream));
  return ukn_launch(c, p, d_jobs, true, true);
}

// ----------------------------------------------------------------------------
// energy matrix without allocation: the job table lives in `scratch`, a
// file-scope device array of BPMF_NOALLOC_MAX_JOBS entries plus the
// sentinels; every device that runs the library holds its own copy until the
// process ends.  Host code never uses the array's name as an address: its
// per-device address comes from hipGetSymbolAddress at context creation.
// ----------------------------------------------------------------------------
static __device__ __align__(256) UknJob
    scratch[BPMF_NOALLOC_MAX_JOBS + bpmf_ctx::kWaveClasses];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// address of `scratch` on `device` (the current device), looked up once per
// device; null where the lookup failed or the device index is too large
int scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return BPMF_OK;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(BPMF_E_HIP, "address of the no-allocation job table: %s",
                  hipGetErrorString(e));
    g_scratch_addr[device] = ptr;
  }
  *out = g_scratch_addr[device];
  return BPMF_OK;
}
}  // namespace

extern "C" int bpmf_energy_matrix_batch_noalloc(
    bpmf_ctx* c, int n, const int* ligand_ids,
    const float* const* dev_samples, const int64_t* n_samples,
    double* const* dev_ukn, const int64_t* ld) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (n > BPMF_NOALLOC_MAX_JOBS)
    return fail(BPMF_E_INVAL,
                "no-allocation energy matrix: %d entries exceed the limit %d",
                n, BPMF_NOALLOC_MAX_JOBS);
  if (!c->scratch_addr)
    return fail(BPMF_E_UNIMPL,
                "no-allocation energy matrix: no job table on device %d",
                c->device);
  UknJob jobs[BPMF_NOALLOC_MAX_JOBS + bpmf_ctx::kWaveClasses];
  UknPlan p;
  if ((rc = ukn_plan(c, n, ligand_ids, dev_samples, n_samples, dev_ukn, ld,
                     jobs, &p)) ||
      p.n_jobs == 0)
    return rc;
  UknJob* d_jobs = (UknJob*)c->scratch_addr;
  HIP_TRY(launch_put_jobs(d_jobs, jobs, p.n_jobs, c->stream));
  return ukn_launch(c, p, d_jobs, false, false);
}

extern "C" int bpmf_energy_matrix(bpmf_ctx* c, int ligand_id,
                                  const float* dev_samples, int64_t n_samples,
                                  double* dev_ukn, int64_t ld) {
  return bpmf_energy_matrix_batch(c, 1, &ligand_id, &dev_samples, &n_samples,
                                  &dev_ukn, &ld);
}

namespace {
// host side of one problem of an MBAR batch
struct MbarSolve {
  enum Phase { kNewtonStep, kSearch, kFixedPoint, kDone };
  Phase phase = kNewtonStep;
  int it = 1;         // current iteration (1-based)
  int ls = 0;         // line-search trials made in this iteration
  bool accept = false;  // ftry becomes f at the start of the next round
  double trust = INFINITY, Fcur = 0.0, t = 1.0, maxstep = 0.0, gs = 0.0;
  int n_iter = 0;
};
}  // namespace

// Solves every problem of the batch with the same sequence of steps a lone
// solve takes, advancing all unfinished problems by one step per round (one
// host synchronisation per round for the whole batch).  Per problem and
// iteration: a Newton step with backtracking on the objective when the
// gauge-fixed Hessian is numerically positive definite, otherwise one
// fixed-point step (far from the solution whole states' weights can
// underflow, leaving the Hessian singular).  While accepted moves are large
// (>= 1 kT) the first trial of a Newton step moves no component by more than
// twice the last accepted move (far from the solution full Newton steps
// overshoot and would be halved many times).
extern "C" int bpmf_mbar_batch(bpmf_ctx* c, int n_problems,
                               const double* const* dev_ukn, const int* Ks,
                               const int64_t* Ns, const int64_t* lds,
                               const int64_t* N_k, double tol, int max_iter,
                               double* f, double* var, int* n_iter,
                               int warm_start) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (n_problems < 0 || n_problems > BPMF_MAX_MBAR_BATCH)
    return fail(BPMF_E_INVAL, "MBAR batch of %d problems outside 0..%d",
                n_problems, BPMF_MAX_MBAR_BATCH);
  if (n_problems == 0) return BPMF_OK;
  if (!dev_ukn || !Ks || !Ns || !lds || !N_k || !f)
    return fail(BPMF_E_INVAL, "null MBAR argument");
  if (!(tol > 0) || max_iter < 1)
    return fail(BPMF_E_INVAL, "tol must be > 0 and max_iter >= 1");
  const int P = n_problems;
  std::vector<int64_t> koff(P + 1, 0);
  for (int p = 0; p < P; ++p) {
    const int K = Ks[p];
    const int64_t N = Ns[p];
    if (!dev_ukn[p]) return fail(BPMF_E_INVAL, "null u_kn of problem %d", p);
    if (K < 1 || K > BPMF_MAX_MBAR_STATES)
      return fail(BPMF_E_INVAL, "MBAR K %d of problem %d outside 1..%d", K, p,
                  BPMF_MAX_MBAR_STATES);
    if (N < 1 || lds[p] < N)
      return fail(BPMF_E_INVAL, "bad N or ld of problem %d", p);
    int64_t tot = 0;
    for (int k = 0; k < K; ++k) {
      if (N_k[koff[p] + k] <= 0)
        return fail(BPMF_E_INVAL, "N_k[%d] of problem %d must be > 0", k, p);
      tot += N_k[koff[p] + k];
    }
    if (tot != N)
      return fail(BPMF_E_INVAL, "problem %d: sum N_k = %lld != N = %lld", p,
                  (long long)tot, (long long)N);
    if (warm_start)
      for (int k = 0; k < K; ++k)
        if (!std::isfinite(f[koff[p] + k]))
          return fail(BPMF_E_INVAL, "non-finite initial f[%d] of problem %d",
                      k, p);
    koff[p + 1] = koff[p] + K;
  }
  // problems with one state are solved by definition
  std::vector<int> act;
  for (int p = 0; p < P; ++p) {
    if (Ks[p] == 1) {
      f[koff[p]] = 0.0;
      if (var) var[koff[p]] = 0.0;
      if (n_iter) n_iter[p] = 0;
    } else {
      act.push_back(p);
    }
  }
  if (act.empty()) return BPMF_OK;
  const int64_t sumK = koff[P];
  int max_K = 0, max_nb = 0, max_acc[9] = {0};
  size_t n_logD = 0, n_obj = 0, n_part = 0, n_red = 0, n_mat = 0;
  for (int p : act) {
    const int K = Ks[p];
    const int ts = mbar_acc_ts(K);
    max_K = std::max(max_K, K);
    max_nb = std::max(max_nb, mbar_logD_blocks(Ns[p]));
    max_acc[ts] = std::max(max_acc[ts], mbar_acc_blocks(K, Ns[p]));
    n_logD += Ns[p];
    n_obj += mbar_logD_blocks(Ns[p]);
    n_part += (size_t)mbar_acc_blocks(K, Ns[p]) * (K + (size_t)K * K);
    n_red += K + (size_t)K * K;
    n_mat += (size_t)(K - 1) * (2 * K - 1);
  }
  Arena A;
  const size_t o_tab = A.add(P * sizeof(MbarProb)),
               o_vec = A.add((size_t)6 * sumK * 8),
               o_sc = A.add((size_t)P * 8 * 8), o_logD = A.add(n_logD * 8),
               o_obj = A.add(n_obj * 8), o_part = A.add(n_part * 8),
               o_red = A.add(n_red * 8), o_mat = A.add(n_mat * 8),
               o_list = A.add((size_t)P * 4 * sizeof(int)),
               o_t = A.add((size_t)P * 8);
  rc = ensure_scratch(c, &c->mbar_mem, &c->mbar_bytes, A.total);
  if (rc) return rc;
  char* base = (char*)c->mbar_mem;
  double* vec = (double*)(base + o_vec);
  double *d_f = vec, *d_ftry = vec + sumK, *d_logN = vec + 2 * sumK,
         *d_Nk = vec + 3 * sumK, *d_step = vec + 4 * sumK,
         *d_var = vec + 5 * sumK;
  double* d_sc = (double*)(base + o_sc);
  const MbarProb* d_tab = (const MbarProb*)(base + o_tab);
  int* d_list = (int*)(base + o_list);
  double* d_t = (double*)(base + o_t);
  std::vector<MbarProb> tab(P);
  std::vector<double> h_logN(sumK, 0.0), h_Nk(sumK, 1.0), h_f(sumK, 0.0);
  {
    size_t qd = 0, qo = 0, qp = 0, qr = 0, qm = 0;
    for (int p : act) {
      const int K = Ks[p];
      MbarProb& q = tab[p];
      q.ukn = dev_ukn[p];
      q.N = Ns[p];
      q.ld = lds[p];
      q.K = K;
      q.nb = mbar_logD_blocks(Ns[p]);
      q.nb_acc = mbar_acc_blocks(K, Ns[p]);
      q.ts = mbar_acc_ts(K);
      q.f = d_f + koff[p];
      q.ftry = d_ftry + koff[p];
      q.logN = d_logN + koff[p];
      q.Nk = d_Nk + koff[p];
      q.step = d_step + koff[p];
      q.var = d_var + koff[p];
      q.scalars = d_sc + (size_t)p * 8;
      q.logD = (double*)(base + o_logD) + qd;
      q.obj_part = (double*)(base + o_obj) + qo;
      q.partial = (double*)(base + o_part) + qp;
      q.red = (double*)(base + o_red) + qr;
      q.mat = (double*)(base + o_mat) + qm;
      qd += Ns[p];
      qo += q.nb;
      qp += (size_t)q.nb_acc * (K + (size_t)K * K);
      qr += K + (size_t)K * K;
      qm += (size_t)(K - 1) * (2 * K - 1);
      for (int k = 0; k < K; ++k) {
        h_Nk[koff[p] + k] = (double)N_k[koff[p] + k];
        h_logN[koff[p] + k] = log(h_Nk[koff[p] + k]);
        if (warm_start) h_f[koff[p] + k] = f[koff[p] + k] - f[koff[p]];
      }
    }
  }
  HIP_TRY(hipMemcpyAsync(base + o_tab, tab.data(), P * sizeof(MbarProb),
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(d_f, h_f.data(), sumK * 8, hipMemcpyHostToDevice,
                         c->stream));
  HIP_TRY(hipMemcpyAsync(d_logN, h_logN.data(), sumK * 8,
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(d_Nk, h_Nk.data(), sumK * 8, hipMemcpyHostToDevice,
                         c->stream));
  std::vector<MbarSolve> S(P);
  std::vector<double> sc((size_t)P * 8);
  // lists of one round, uploaded together: [accept | newton (by tile) |
  // line search | fixed point]
  std::vector<int> lists;
  std::vector<double> tv(P, 0.0);
  auto upload = [&]() -> int {
    HIP_TRY(hipMemcpyAsync(d_list, lists.data(), lists.size() * sizeof(int),
                           hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(d_t, tv.data(), P * 8, hipMemcpyHostToDevice,
                           c->stream));
    return BPMF_OK;
  };
  auto fetch = [&]() -> int {
    HIP_TRY(hipMemcpyAsync(sc.data(), d_sc, (size_t)P * 64,
                           hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return BPMF_OK;
  };
  // objective (and logD) at every starting point
  lists = act;
  if ((rc = upload())) return rc;
  HIP_TRY(mbar_objective(d_tab, d_list, (int)act.size(), max_nb, 0,
                         c->stream));
  if ((rc = fetch())) return rc;
  for (int p : act) S[p].Fcur = sc[(size_t)p * 8];
  auto finish = [&](MbarSolve& s, double change) {
    if (!(change >= tol)) {
      s.phase = MbarSolve::kDone;
      s.n_iter = s.it;
    } else if (s.it >= max_iter) {
      s.phase = MbarSolve::kDone;
      s.n_iter = max_iter;
    } else {
      ++s.it;
      s.phase = MbarSolve::kNewtonStep;
    }
  };
  static const int kTiles[4] = {1, 2, 4, 8};
  for (;;) {
    lists.clear();
    std::vector<int> newt, search, fixed;
    for (int p : act)
      if (S[p].accept) lists.push_back(p);
    const int n_acc = (int)lists.size();
    int n_tile[4] = {0, 0, 0, 0};
    for (int i = 0; i < 4; ++i)
      for (int p : act)
        if (S[p].phase == MbarSolve::kNewtonStep && tab[p].ts == kTiles[i]) {
          lists.push_back(p);
          newt.push_back(p);
          ++n_tile[i];
        }
    for (int p : act)
      if (S[p].phase == MbarSolve::kSearch) {
        lists.push_back(p);
        search.push_back(p);
        tv[p] = S[p].t;
      }
    for (int p : act)
      if (S[p].phase == MbarSolve::kFixedPoint) {
        lists.push_back(p);
        fixed.push_back(p);
      }
    if (newt.empty() && search.empty() && fixed.empty()) break;
    if ((rc = upload())) return rc;
    const int* L = d_list;
    HIP_TRY(mbar_accept(d_tab, L, n_acc, c->stream));
    L += n_acc;
    for (int p : act) S[p].accept = false;
    const int* Ln = L;
    for (int i = 0; i < 4; ++i) {
      HIP_TRY(mbar_accumulate(d_tab, L, n_tile[i], kTiles[i],
                              max_acc[kTiles[i]], c->stream));
      L += n_tile[i];
    }
    HIP_TRY(mbar_newton(d_tab, Ln, (int)newt.size(), max_K, 0, c->stream));
    HIP_TRY(mbar_axpy(d_tab, L, (int)search.size(), d_t, c->stream));
    HIP_TRY(mbar_objective(d_tab, L, (int)search.size(), max_nb, 1,
                           c->stream));
    L += search.size();
    HIP_TRY(mbar_fixed_point(d_tab, L, (int)fixed.size(), max_K, c->stream));
    HIP_TRY(mbar_objective(d_tab, L, (int)fixed.size(), max_nb, 0,
                           c->stream));
    if ((rc = fetch())) return rc;
    for (int p : newt) {
      MbarSolve& s = S[p];
      const double* q = &sc[(size_t)p * 8];
      if (q[3] == 0.0) {
        s.maxstep = q[1];
        s.gs = q[2];
        s.t = s.trust >= 1.0 ? std::min(1.0, 2.0 * s.trust / s.maxstep) : 1.0;
        s.ls = 0;
        s.phase = MbarSolve::kSearch;
      } else {
        s.phase = MbarSolve::kFixedPoint;
      }
    }
    for (int p : search) {
      MbarSolve& s = S[p];
      const double Ftry = sc[(size_t)p * 8];
      const bool ok = Ftry <= s.Fcur + 1e-4 * s.t * s.gs + 1e-13 * fabs(s.Fcur)
                      || s.t * s.maxstep < tol;
      if (!ok) {
        s.t *= 0.5;
        // after 60 trials the last one is taken anyway
        if (++s.ls < 60) continue;
      }
      s.accept = true;
      s.Fcur = Ftry;
      const double change = s.t * s.maxstep;
      s.trust = change;
      finish(s, change);
    }
    for (int p : fixed) {
      MbarSolve& s = S[p];
      s.Fcur = sc[(size_t)p * 8];
      finish(s, sc[(size_t)p * 8 + 4]);
    }
  }
  // variances at the solutions (logD recomputed at f)
  lists.clear();
  for (int p : act)
    if (S[p].accept) lists.push_back(p);
  const int n_acc = (int)lists.size();
  int n_tile[4] = {0, 0, 0, 0};
  for (int i = 0; i < 4; ++i)
    for (int p : act)
      if (tab[p].ts == kTiles[i]) {
        lists.push_back(p);
        ++n_tile[i];
      }
  if ((rc = upload())) return rc;
  HIP_TRY(mbar_accept(d_tab, d_list, n_acc, c->stream));
  const int* Ln = d_list + n_acc;
  HIP_TRY(mbar_objective(d_tab, Ln, (int)act.size(), max_nb, 0, c->stream));
  const int* L = Ln;
  for (int i = 0; i < 4; ++i) {
    HIP_TRY(mbar_accumulate(d_tab, L, n_tile[i], kTiles[i],
                            max_acc[kTiles[i]], c->stream));
    L += n_tile[i];
  }
  HIP_TRY(mbar_newton(d_tab, Ln, (int)act.size(), max_K, 1, c->stream));
  std::vector<double> hf(sumK), hv(sumK);
  HIP_TRY(hipMemcpyAsync(hf.data(), d_f, sumK * 8, hipMemcpyDeviceToHost,
                         c->stream));
  HIP_TRY(hipMemcpyAsync(hv.data(), d_var, sumK * 8, hipMemcpyDeviceToHost,
                         c->stream));
  if ((rc = fetch())) return rc;
  for (int p : act) {
    const int K = Ks[p];
    memcpy(f + koff[p], hf.data() + koff[p], K * 8);
    // a Hessian that is not positive definite at the solution means states
    // without overlap: their differences are not determined
    if (sc[(size_t)p * 8 + 3] != 0.0)
      for (int k = 1; k < K; ++k) hv[koff[p] + k] = INFINITY;
    if (var) memcpy(var + koff[p], hv.data() + koff[p], K * 8);
    if (n_iter) n_iter[p] = S[p].n_iter;
  }
  return BPMF_OK;
}

extern "C" int bpmf_mbar(bpmf_ctx* c, const double* dev_ukn, int K, int64_t N,
                         int64_t ld, const int64_t* N_k, double tol,
                         int max_iter, double* f, double* var, int* n_iter,
                         int warm_start) {
  return bpmf_mbar_batch(c, 1, &dev_ukn, &K, &N, &ld, N_k, tol, max_iter, f,
                         var, n_iter, warm_start);
}

// ============================================================================
// direct evaluation
// ============================================================================
extern "C" int bpmf_evaluate(bpmf_ctx* c, int ligand_id, const float* dev_x,
                             int64_t n_conf, const double* dev_w,
                             double* dev_terms, float* dev_forces) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_lig(c, ligand_id))) return rc;
  if (n_conf < 0) return fail(BPMF_E_INVAL, "negative n_conf");
  if (n_conf == 0) return BPMF_OK;
  if (!dev_x || !dev_w || !dev_terms)
    return fail(BPMF_E_INVAL, "null evaluate argument");
  const LigHost& h = c->ligs[ligand_id];
  const int wv = c->waves_override ? std::max(c->waves_override, h.min_waves)
                                   : h.min_waves;
  HIP_TRY(launch_evaluate(c->grid, c->d_ligs + ligand_id, wv, dev_x, n_conf,
                          dev_w, dev_terms, dev_forces,
                          lds_of(h, wv, true), c->stream));
  return BPMF_OK;
}

extern "C" int bpmf_grid_eval(bpmf_ctx* c, const float* dev_pos,
                              const float* dev_scale, int64_t n,
                              const double* w, float* dev_energy,
                              float* dev_force) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!c->has_grid) return fail(BPMF_E_STATE, "upload the grid first");
  if (!supported_channels(c->grid.C))
    return fail(BPMF_E_UNIMPL, "grid_eval supports 3 or 5 channels");
  if (n < 0) return fail(BPMF_E_INVAL, "negative n");
  if (n == 0) return BPMF_OK;
  if (!dev_pos || !dev_scale || !w)
    return fail(BPMF_E_INVAL, "null grid_eval argument");
  if (!finite_all(w, c->grid.C)) return fail(BPMF_E_INVAL, "non-finite weight");
  hipEvent_t t0, t1;
  const bool timed = c->timer_begin(BPMF_TIMER_GRID_EVAL, &t0, &t1);
  if (timed) HIP_TRY(hipEventRecord(t0, c->stream));
  HIP_TRY(launch_grid_eval(c->grid, dev_pos, dev_scale, n, w, dev_energy,
                           dev_force, c->stream));
  if (timed) HIP_TRY(hipEventRecord(t1, c->stream));
  return BPMF_OK;
}

// ============================================================================
// replica state, statistics, samples
// ============================================================================
extern "C" int bpmf_get_replicas(bpmf_ctx* c, int ligand_id, float* x,
                                 int* sor, double* comps, uint64_t* counter) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_lig(c, ligand_id))) return rc;
  const LigDev& L = c->ligs[ligand_id].dev;
  if (x)
    HIP_TRY(hipMemcpyAsync(x, L.x, (size_t)L.K * L.n * 12,
                           hipMemcpyDeviceToHost, c->stream));
  if (sor)
    HIP_TRY(hipMemcpyAsync(sor, L.state_of_replica, L.K * 4,
                           hipMemcpyDeviceToHost, c->stream));
  if (comps)
    HIP_TRY(hipMemcpyAsync(comps, L.comps, (size_t)L.K * (1 + L.C) * 8,
                           hipMemcpyDeviceToHost, c->stream));
  unsigned long long cnt = 0;
  HIP_TRY(hipMemcpyAsync(&cnt, L.counter, 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (counter) *counter = cnt;
  return BPMF_OK;
}

extern "C" int bpmf_set_replicas(bpmf_ctx* c, int ligand_id, const float* x,
                                 const int* sor, const double* comps,
                                 uint64_t counter) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_lig(c, ligand_id))) return rc;
  LigHost& h = c->ligs[ligand_id];
  const LigDev& L = h.dev;
  if (!x || !sor) return fail(BPMF_E_INVAL, "null x or state_of_replica");
  std::vector<int> ros(L.K, -1);
  for (int r = 0; r < L.K; ++r) {
    if (sor[r] < 0 || sor[r] >= L.K || ros[sor[r]] != -1)
      return fail(BPMF_E_INVAL, "state_of_replica is not a permutation");
    ros[sor[r]] = r;
  }
  HIP_TRY(hipMemcpyAsync(L.x, x, (size_t)L.K * L.n * 12, hipMemcpyHostToDevice,
                         c->stream));
  HIP_TRY(hipMemcpyAsync(L.state_of_replica, sor, L.K * 4,
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(L.replica_of_state, ros.data(), L.K * 4,
                         hipMemcpyHostToDevice, c->stream));
  unsigned long long cnt = counter;
  HIP_TRY(hipMemcpyAsync(L.counter, &cnt, 8, hipMemcpyHostToDevice, c->stream));
  // round-trip tracking restarts from the given states (the count is kept)
  std::vector<int> rte(L.K);
  for (int r = 0; r < L.K; ++r) rte[r] = sor[r] == 0 ? 0 : -1;
  HIP_TRY(hipMemcpyAsync(rt_end_of(L), rte.data(), L.K * 4,
                         hipMemcpyHostToDevice, c->stream));
  // new positions: no reusable start-of-trajectory forces
  HIP_TRY(hipMemsetAsync(L.fvalid, 0, (size_t)L.K * 4, c->stream));
  if (comps)
    HIP_TRY(hipMemcpyAsync(L.comps, comps, (size_t)L.K * (1 + L.C) * 8,
                           hipMemcpyHostToDevice, c->stream));
  else
    HIP_TRY(launch_recompute_comps(c->grid, c->d_ligs + ligand_id,
                                   h.min_waves, L.K,
                                   lds_of(h, h.min_waves, false),
                                   L.pairs_on != 0, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  h.counter = counter;
  return BPMF_OK;
}

extern "C" int bpmf_ligand_info(bpmf_ctx* c, int ligand_id, int* n_atoms,
                                int* n_states, int* n_channels,
                                int* sample_capacity) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_lig(c, ligand_id))) return rc;
  const LigDev& L = c->ligs[ligand_id].dev;
  if (n_atoms) *n_atoms = L.n;
  if (n_states) *n_states = L.K;
  if (n_channels) *n_channels = L.C;
  if (sample_capacity) *sample_capacity = L.cap;
  return BPMF_OK;
}

extern "C" int bpmf_set_states(bpmf_ctx* c, int ligand_id, const double* T,
                               const double* w, const double* dt_fs) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_lig(c, ligand_id))) return rc;
  if (!T || !w || !dt_fs) return fail(BPMF_E_INVAL, "null state array");
  LigHost& h = c->ligs[ligand_id];
  const LigDev& L = h.dev;
  const int K = L.K, C = L.C;
  for (int k = 0; k < K; ++k) {
    if (!(T[k] > 0) || !isfinite(T[k]))
      return fail(BPMF_E_INVAL, "T[%d] must be positive and finite", k);
    if (!(dt_fs[k] > 0) || !isfinite(dt_fs[k]))
      return fail(BPMF_E_INVAL, "dt[%d] must be positive and finite", k);
  }
  if (!finite_all(w, (size_t)K * C))
    return fail(BPMF_E_INVAL, "non-finite state weight");
  std::vector<double> beta(K), wd(w, w + (size_t)K * C);
  std::vector<float> Tf(K), dtf(K), wf((size_t)K * C);
  for (int k = 0; k < K; ++k) {
    beta[k] = 1.0 / (kRGas * T[k]);
    Tf[k] = (float)T[k];
    dtf[k] = (float)dt_fs[k];
  }
  for (size_t i = 0; i < wf.size(); ++i) wf[i] = (float)w[i];
  // the arrays are read by kernels already in the stream: replace them in
  // stream order, then wait so that the host buffers can go
  HIP_TRY(hipMemcpyAsync((void*)L.beta, beta.data(), K * 8,
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync((void*)L.Tf, Tf.data(), K * 4, hipMemcpyHostToDevice,
                         c->stream));
  HIP_TRY(hipMemcpyAsync((void*)L.dtf, dtf.data(), K * 4,
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync((void*)L.wf, wf.data(), wf.size() * 4,
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync((void*)L.wd, wd.data(), wd.size() * 8,
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  h.beta = beta;
  h.wd = wd;
  return BPMF_OK;
}

extern "C" int bpmf_place_poses(bpmf_ctx* c, int ligand_id,
                                const float* dev_confs, int n_conf, int n_com,
                                int n_orient, int64_t first, int64_t count,
                                float* dev_out) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_lig(c, ligand_id))) return rc;
  if (n_conf < 1 || n_com < 1 || n_orient < 1)
    return fail(BPMF_E_INVAL, "n_conf, n_com and n_orient must be >= 1");
  if (n_com > (1 << 24) || n_orient > (1 << 24))
    return fail(BPMF_E_INVAL, "n_com and n_orient are limited to 2^24");
  const int64_t total = (int64_t)n_conf * n_com * n_orient;
  if (first < 0 || count < 0 || first + count > total)
    return fail(BPMF_E_INVAL, "poses [%lld, %lld) outside [0, %lld)",
                (long long)first, (long long)(first + count),
                (long long)total);
  if (count == 0) return BPMF_OK;
  if (!dev_confs || !dev_out) return fail(BPMF_E_INVAL, "null pose buffer");
  if ((rc = ensure_scratch(c, &c->place_mem, &c->place_bytes,
                           (size_t)n_conf * 3 * sizeof(double))))
    return rc;
  HIP_TRY(launch_place_poses(c->d_ligs + ligand_id, c->ligs[ligand_id].dev.n,
                             dev_confs, n_conf, n_com, n_orient, first, count,
                             (double*)c->place_mem, c->seed, dev_out,
                             c->stream));
  return BPMF_OK;
}

extern "C" int bpmf_pair_setup(bpmf_ctx* c, int ligand_id,
                               const bpmf_pair_desc* d) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_lig(c, ligand_id))) return rc;
  if (!d || !d->charge || !d->lj_sigma || !d->lj_eps || !d->gb_radius ||
      !d->gb_scale)
    return fail(BPMF_E_INVAL, "null pair parameter array");
  LigHost& h = c->ligs[ligand_id];
  const int n = h.dev.n;
  if (n > kPairMaxAtoms)
    return fail(BPMF_E_UNIMPL, "pair terms support up to %d atoms, not %d",
                kPairMaxAtoms, n);
  for (int i = 0; i < n; ++i) {
    if (!isfinite(d->charge[i]) || !(d->lj_sigma[i] > 0) ||
        !(d->lj_eps[i] >= 0) || !isfinite(d->lj_eps[i]) ||
        !isfinite(d->lj_sigma[i]))
      return fail(BPMF_E_INVAL, "atom %d: bad charge or LJ parameters", i);
    if (!(d->gb_radius[i] > 0.09 + 1e-6) || !isfinite(d->gb_radius[i]) ||
        !(d->gb_scale[i] > 0) || !isfinite(d->gb_scale[i]))
      return fail(BPMF_E_INVAL,
                  "atom %d: GB radius must exceed 0.09 A and scale be > 0", i);
  }
  if (d->n_exclusions < 0 || d->n_pairs14 < 0 ||
      (d->n_exclusions && !d->exclusions) || (d->n_pairs14 && !d->pairs14))
    return fail(BPMF_E_INVAL, "bad exclusion or 1-4 list");
  if (!(d->eps_solute > 0) || !(d->eps_solvent > 0) || !(d->sa_gamma >= 0) ||
      !(d->probe_radius >= 0) || !isfinite(d->lj14) || !isfinite(d->el14))
    return fail(BPMF_E_INVAL, "bad dielectric, surface or 1-4 constants");
  std::vector<uint32_t> ex((size_t)n * kPairWords, 0u),
      o4((size_t)n * kPairWords, 0u);
  auto set = [&](std::vector<uint32_t>& m, int i, int j) {
    m[(size_t)i * kPairWords + (j >> 5)] |= 1u << (j & 31);
    m[(size_t)j * kPairWords + (i >> 5)] |= 1u << (i & 31);
  };
  auto get = [&](const std::vector<uint32_t>& m, int i, int j) {
    return (m[(size_t)i * kPairWords + (j >> 5)] >> (j & 31)) & 1u;
  };
  for (int t = 0; t < d->n_exclusions; ++t) {
    const int i = d->exclusions[2 * t], j = d->exclusions[2 * t + 1];
    if (i < 0 || j < 0 || i >= n || j >= n || i == j)
      return fail(BPMF_E_INVAL, "exclusion %d: bad pair (%d, %d)", t, i, j);
    set(ex, i, j);
  }
  for (int t = 0; t < d->n_pairs14; ++t) {
    const int i = d->pairs14[2 * t], j = d->pairs14[2 * t + 1];
    if (i < 0 || j < 0 || i >= n || j >= n || i == j)
      return fail(BPMF_E_INVAL, "1-4 pair %d: bad pair (%d, %d)", t, i, j);
    if (!get(ex, i, j)) set(o4, i, j);
  }
  std::vector<float4> p0(n);
  std::vector<float2> p1(n);
  for (int i = 0; i < n; ++i) {
    const double rt = d->gb_radius[i] - 0.09;
    p0[i] = make_float4((float)d->charge[i], (float)d->lj_sigma[i],
                        (float)sqrt(d->lj_eps[i]), (float)d->gb_radius[i]);
    p1[i] = make_float2((float)rt, (float)(d->gb_scale[i] * rt));
  }
  Arena A;
  const size_t o_p0 = A.add((size_t)n * 16), o_p1 = A.add((size_t)n * 8),
               o_ex = A.add(ex.size() * 4), o_o4 = A.add(o4.size() * 4);
  char* base = (char*)c->dalloc(A.total);
  if (!base) return fail(BPMF_E_NOMEM, "pair parameter allocation failed");
  hipError_t e = hipMemcpyAsync(base + o_p0, p0.data(), (size_t)n * 16,
                                hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(base + o_p1, p1.data(), (size_t)n * 8,
                       hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(base + o_ex, ex.data(), ex.size() * 4,
                       hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(base + o_o4, o4.data(), o4.size() * 4,
                       hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    c->dfree(base);
    return fail(BPMF_E_HIP, "pair parameter upload: %s", hipGetErrorString(e));
  }
  c->dfree(h.pair_arena);
  h.pair_arena = base;
  PairDev& P = h.pair;
  P.n = n;
  P.p0 = (const float4*)(base + o_p0);
  P.p1 = (const float2*)(base + o_p1);
  P.excl = (const uint32_t*)(base + o_ex);
  P.o14 = (const uint32_t*)(base + o_o4);
  P.lj14 = (float)d->lj14;
  P.el14 = (float)d->el14;
  const double ke = 1389.35457644382;  // e^2 / (4 pi eps0), kJ/mol A
  P.kc = (float)(ke / d->eps_solute);
  P.kgb = (float)(-ke * (1.0 / d->eps_solute - 1.0 / d->eps_solvent));
  P.sa = (float)(4.0 * M_PI * d->sa_gamma);
  P.probe = (float)d->probe_radius;
  h.has_pairs = true;
  // pair terms already in the sampled energy: the new parameters take over
  if (h.dev.pairs_on) return pair_sample_refresh(c, ligand_id);
  return BPMF_OK;
}

namespace {
// After the pair terms of a ligand's energy changed (switched on or off, new
// parameters): device table entry, LDS sizes, captured graphs, the cached
// start-of-trajectory forces (invalid) and the cached energy components
// (recomputed).  Synchronises.
int pair_sample_refresh(bpmf_ctx* c, int lid) {
  LigHost& h = c->ligs[lid];
  h.dev.pair = h.pair;
  int rc = rebuild_tables(c);
  if (rc) return rc;
  LigDev& L = h.dev;
  HIP_TRY(hipMemsetAsync(L.fvalid, 0, (size_t)L.K * 4, c->stream));
  HIP_TRY(launch_recompute_comps(c->grid, c->d_ligs + lid, h.min_waves, L.K,
                                 lds_of(h, h.min_waves, false),
                                 L.pairs_on != 0, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return BPMF_OK;
}
}  // namespace

extern "C" int bpmf_pair_sample(bpmf_ctx* c, int ligand_id, int on) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_lig(c, ligand_id))) return rc;
  LigHost& h = c->ligs[ligand_id];
  if (on && !h.has_pairs)
    return fail(BPMF_E_STATE, "ligand %d has no pair parameters (call "
                "bpmf_pair_setup)", ligand_id);
  const LigDev& L = h.dev;
  if (on) {
    const int need = block_lds_bytes(8, true, L.n, L.nb, L.na, L.nt, true);
    if (need > 65536)
      return fail(BPMF_E_UNIMPL,
                  "ligand %d: %d bytes of LDS per replica with pair terms "
                  "(max 65536)", ligand_id, need);
  }
  h.dev.pairs_on = on ? 1 : 0;
  return pair_sample_refresh(c, ligand_id);
}

extern "C" int bpmf_pair_evaluate(bpmf_ctx* c, int ligand_id,
                                  const float* dev_x, int64_t n_conf,
                                  double* dev_terms, float* dev_forces) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_lig(c, ligand_id))) return rc;
  const LigHost& h = c->ligs[ligand_id];
  if (!h.has_pairs)
    return fail(BPMF_E_STATE, "ligand %d has no pair parameters", ligand_id);
  if (n_conf < 0 || n_conf > 0x7fffffffll)
    return fail(BPMF_E_INVAL, "n_conf %lld outside 0..2^31-1",
                (long long)n_conf);
  if (n_conf == 0) return BPMF_OK;
  if (!dev_x || !dev_terms) return fail(BPMF_E_INVAL, "null pair buffer");
  HIP_TRY(launch_pair_terms(h.pair, dev_x, n_conf, dev_terms, dev_forces,
                            c->stream));
  return BPMF_OK;
}

// accessors for the ladder initialisation (protocol.hip)
namespace bpmf {
void* ctx_alloc(bpmf_ctx* c, size_t bytes) { return c->dalloc(bytes); }
void ctx_free(bpmf_ctx* c, void* p) { c->dfree(p); }
hipStream_t ctx_stream(bpmf_ctx* c) { return c->stream; }
uint64_t ctx_seed(bpmf_ctx* c) { return c->seed; }
int ctx_fail(int code, const char* msg) { return fail(code, "%s", msg); }
}  // namespace bpmf

extern "C" int bpmf_get_round_trips(bpmf_ctx* c, int ligand_id,
                                    int64_t* trips) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_lig(c, ligand_id))) return rc;
  if (!trips) return fail(BPMF_E_INVAL, "null trips");
  unsigned long long v = 0;
  HIP_TRY(hipMemcpyAsync(&v, round_trips_of(c->ligs[ligand_id].dev), 8,
                         hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  *trips = (int64_t)v;
  return BPMF_OK;
}

extern "C" int bpmf_get_stats(bpmf_ctx* c, int ligand_id, int64_t* hmc_acc,
                              int64_t* hmc_try, int64_t* ex_acc,
                              int64_t* ex_try, int64_t* nonfinite) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_lig(c, ligand_id))) return rc;
  const LigDev& L = c->ligs[ligand_id].dev;
  const int Km1 = std::max(L.K - 1, 1);
  std::vector<unsigned long long> ex_a(Km1), ex_t(Km1);
  if (hmc_acc)
    HIP_TRY(hipMemcpyAsync(hmc_acc, L.hmc_acc, L.K * 8, hipMemcpyDeviceToHost,
                           c->stream));
  if (hmc_try)
    HIP_TRY(hipMemcpyAsync(hmc_try, L.hmc_try, L.K * 8, hipMemcpyDeviceToHost,
                           c->stream));
  HIP_TRY(hipMemcpyAsync(ex_a.data(), L.ex_acc, Km1 * 8, hipMemcpyDeviceToHost,
                         c->stream));
  HIP_TRY(hipMemcpyAsync(ex_t.data(), L.ex_try, Km1 * 8, hipMemcpyDeviceToHost,
                         c->stream));
  unsigned long long nf = 0;
  HIP_TRY(hipMemcpyAsync(&nf, L.nonfinite, 8, hipMemcpyDeviceToHost,
                         c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (int q = 0; q < L.K - 1; ++q) {
    if (ex_acc) ex_acc[q] = (int64_t)ex_a[q];
    if (ex_try) ex_try[q] = (int64_t)ex_t[q];
  }
  if (nonfinite) *nonfinite = (int64_t)nf;
  return BPMF_OK;
}

extern "C" int bpmf_get_samples(bpmf_ctx* c, int ligand_id, int64_t* n_records,
                                float* x, double* comps) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_lig(c, ligand_id))) return rc;
  const LigHost& h = c->ligs[ligand_id];
  const LigDev& L = h.dev;
  unsigned long long nr = 0;
  HIP_TRY(hipMemcpyAsync(&nr, L.n_rec, 8, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (x && nr)
    HIP_TRY(hipMemcpyAsync(x, L.samp_x, (size_t)nr * L.K * L.n * 12,
                           hipMemcpyDeviceToHost, c->stream));
  if (comps && nr)
    HIP_TRY(hipMemcpyAsync(comps, L.samp_c, (size_t)nr * L.K * (1 + L.C) * 8,
                           hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (n_records) *n_records = (int64_t)nr;
  return BPMF_OK;
}

extern "C" int bpmf_reset_samples(bpmf_ctx* c, int ligand_id) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (ligand_id != -1 && (rc = check_lig(c, ligand_id))) return rc;
  for (size_t l = 0; l < c->ligs.size(); ++l) {
    if (ligand_id != -1 && (int)l != ligand_id) continue;
    HIP_TRY(hipMemsetAsync(c->ligs[l].dev.n_rec, 0, 8, c->stream));
    c->ligs[l].n_rec = 0;
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  return BPMF_OK;
}

// ============================================================================
// kernel timing
// ============================================================================
extern "C" int bpmf_set_timing(bpmf_ctx* c, int enable, int every) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (every < 1) return fail(BPMF_E_INVAL, "every must be >= 1");
  c->timing = enable != 0;
  c->timing_every = every;
  for (int k = 0; k < bpmf_ctx::kTimers; ++k) {
    c->launches[k] = 0;
    c->ev_used[k] = 0;
  }
  return BPMF_OK;
}

extern "C" int bpmf_get_timing(bpmf_ctx* c, int kernel, double* mean_ms,
                               int64_t* n_timed) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (kernel < 0 || kernel >= bpmf_ctx::kTimers)
    return fail(BPMF_E_INVAL, "unknown timer %d", kernel);
  HIP_TRY(hipStreamSynchronize(c->stream));
  double tot = 0.0;
  int64_t cnt = 0;
  const size_t n = c->ev_used[kernel];
  for (size_t i = 0; i < n; ++i) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, c->ev_pool[kernel][2 * i],
                                c->ev_pool[kernel][2 * i + 1]));
    tot += ms;
    cnt += c->ev_weight[kernel][i];
  }
  if (mean_ms) *mean_ms = cnt ? tot / (double)cnt : 0.0;
  if (n_timed) *n_timed = cnt;
  c->ev_used[kernel] = 0;
  c->launches[kernel] = 0;
  return BPMF_OK;
}

// ============================================================================
// launch shape
// ============================================================================
extern "C" int bpmf_set_waves(bpmf_ctx* c, int waves) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (waves != 0 && waves != 1 && waves != 2 && waves != 4 && waves != 8)
    return fail(BPMF_E_INVAL, "waves must be 0 (automatic), 1, 2, 4 or 8");
  c->waves_override = waves;
  return rebuild_tables(c);
}

extern "C" int bpmf_set_task_order(bpmf_ctx* c, int order) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (order != 0 && order != 1)
    return fail(BPMF_E_INVAL, "task order must be 0 or 1");
  c->task_order = order;
  return rebuild_tables(c);
}

extern "C" int bpmf_get_task_order(bpmf_ctx* c, int* order) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (!order) return fail(BPMF_E_INVAL, "null order");
  *order = c->task_order;
  return BPMF_OK;
}

extern "C" int bpmf_set_ligand_waves(bpmf_ctx* c, int ligand_id, int waves) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_lig(c, ligand_id))) return rc;
  if (waves != 0 && waves != 1 && waves != 2 && waves != 4 && waves != 8)
    return fail(BPMF_E_INVAL, "waves must be 0 (none), 1, 2, 4 or 8");
  c->ligs[ligand_id].waves_pin = waves;
  return rebuild_tables(c);
}

extern "C" int bpmf_get_waves(bpmf_ctx* c, int ligand_id, int* waves) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_lig(c, ligand_id))) return rc;
  if (!waves) return fail(BPMF_E_INVAL, "null output");
  *waves = c->ligs[ligand_id].sweep_waves;
  return BPMF_OK;
}

// ============================================================================
// learned pose proposal
// ============================================================================
namespace {



int mlp_scratch(bpmf_ctx* c, int B, MlpBufs* b) {
  Arena A;
  const size_t o_z1 = A.add((size_t)B * kNHid * 4), o_h1 = A.add((size_t)B * kNHid * 4),
               o_z2 = A.add((size_t)B * kNHid * 4), o_h2 = A.add((size_t)B * kNHid * 4),
               o_out = A.add((size_t)B * kNOut * 4), o_do = A.add((size_t)B * kNOut * 4),
               o_dz2 = A.add((size_t)B * kNHid * 4), o_dz1 = A.add((size_t)B * kNHid * 4),
               o_bf = A.add((size_t)B * kNFeat * 4), o_bp = A.add((size_t)B * 6 * 4),
               o_lp = A.add((size_t)((B + 255) / 256) * 8);
  int rc = ensure_scratch(c, &c->mlp_mem, &c->mlp_bytes, A.total);
  if (rc) return rc;
  char* base = (char*)c->mlp_mem;
  b->Z1 = (float*)(base + o_z1);
  b->H1 = (float*)(base + o_h1);
  b->Z2 = (float*)(base + o_z2);
  b->H2 = (float*)(base + o_h2);
  b->out = (float*)(base + o_out);
  b->dout = (float*)(base + o_do);
  b->dZ2 = (float*)(base + o_dz2);
  b->dZ1 = (float*)(base + o_dz1);
  b->bf = (float*)(base + o_bf);
  b->bp = (float*)(base + o_bp);
  b->loss_part = (double*)(base + o_lp);
  return BPMF_OK;
}

GemmArgs gemm(int M, int N, int K, const float* A, int64_t sam, int64_t sak,
              const float* B, int64_t sbk, int64_t sbn, float* C, int64_t ldc,
              const float* bias, int epi, float* Zout, const float* Zin) {
  GemmArgs g;
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.sam = sam; g.sak = sak;
  g.B = B; g.sbk = sbk; g.sbn = sbn;
  g.C = C; g.ldc = ldc; g.bias = bias; g.epi = epi; g.Zout = Zout; g.Zin = Zin;
  return g;
}

// out = MLP(feats) for B rows
int mlp_forward(bpmf_ctx* c, const float* P, const float* feats, int B,
                const MlpBufs& b, float* out, hipStream_t st) {
  HIP_TRY(launch_mlp_forward(P, feats, B, b.Z1, b.H1, b.Z2, b.H2, out, st));
  return BPMF_OK;
}

// gradient of the mean NLL of (feats, poses) into G; loss partials in b
int mlp_grad(bpmf_ctx* c, const float* P, const float* feats,
             const float* poses, int B, const MlpBufs& b, float* G) {
  int rc = mlp_forward(c, P, feats, B, b, b.out, c->stream);
  if (rc) return rc;
  HIP_TRY(launch_nll(b.out, poses, B, b.dout, b.loss_part, c->stream));
  // dZ2 = (dout W3^T) * silu'(Z2); dZ1 = (dZ2 W2^T) * silu'(Z1)
  HIP_TRY(launch_gemm(gemm(B, kNHid, kNOut, b.dout, kNOut, 1, P + kOffW3, 1,
                           kNOut, b.dZ2, kNHid, nullptr, kEpiDsilu, nullptr, b.Z2),
                      c->stream));
  HIP_TRY(launch_gemm(gemm(B, kNHid, kNHid, b.dZ2, kNHid, 1, P + kOffW2, 1, kNHid,
                           b.dZ1, kNHid, nullptr, kEpiDsilu, nullptr, b.Z1),
                      c->stream));
  // weight gradients: H2^T dout, H1^T dZ2, feats^T dZ1
  HIP_TRY(launch_gemm(gemm(kNHid, kNOut, B, b.H2, 1, kNHid, b.dout, kNOut, 1,
                           G + kOffW3, kNOut, nullptr, kEpiStore, nullptr, nullptr),
                      c->stream));
  HIP_TRY(launch_gemm(gemm(kNHid, kNHid, B, b.H1, 1, kNHid, b.dZ2, kNHid, 1,
                           G + kOffW2, kNHid, nullptr, kEpiStore, nullptr, nullptr),
                      c->stream));
  HIP_TRY(launch_gemm(gemm(kNFeat, kNHid, B, feats, 1, kNFeat, b.dZ1, kNHid, 1,
                           G + kOffW1, kNHid, nullptr, kEpiStore, nullptr, nullptr),
                      c->stream));
  HIP_TRY(launch_colsum(b.dout, B, kNOut, kNOut, G + kOffB3, c->stream));
  HIP_TRY(launch_colsum(b.dZ2, B, kNHid, kNHid, G + kOffB2, c->stream));
  HIP_TRY(launch_colsum(b.dZ1, B, kNHid, kNHid, G + kOffB1, c->stream));
  return BPMF_OK;
}

int read_loss(bpmf_ctx* c, const MlpBufs& b, int B, double* loss) {
  const int nb = (B + 255) / 256;
  std::vector<double> lp(nb);
  HIP_TRY(hipMemcpyAsync(lp.data(), b.loss_part, nb * 8, hipMemcpyDeviceToHost,
                         c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  double s = 0.0;
  for (double v : lp) s += v;
  *loss = s / B;
  return BPMF_OK;
}

int check_prop(bpmf_ctx* c, int lid) {
  int rc = check_lig(c, lid);
  if (rc) return rc;
  if (!c->ligs[lid].has_prop)
    return fail(BPMF_E_STATE, "ligand %d has no pose proposal (call "
                "bpmf_proposal_setup)", lid);
  return BPMF_OK;
}

}  // namespace

extern "C" int bpmf_proposal_setup(bpmf_ctx* c, int lid, const int* frame_atoms,
                                   int n_cond, const int* cond_ijkl,
                                   const float* params) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_lig(c, lid))) return rc;
  LigHost& h = c->ligs[lid];
  const int n = h.dev.n;
  if (!frame_atoms || !params)
    return fail(BPMF_E_INVAL, "null frame atoms or parameters");
  if (n_cond < 0 || n_cond > 8 || (n_cond && !cond_ijkl))
    return fail(BPMF_E_INVAL, "n_cond must be 0..8 with a torsion list");
  if (n < 3) return fail(BPMF_E_INVAL, "a pose frame needs >= 3 atoms");
  for (int a = 0; a < 3; ++a) {
    if (frame_atoms[a] < 0 || frame_atoms[a] >= n)
      return fail(BPMF_E_INVAL, "frame atom %d out of range", frame_atoms[a]);
    for (int b = 0; b < a; ++b)
      if (frame_atoms[a] == frame_atoms[b])
        return fail(BPMF_E_INVAL, "repeated frame atom");
  }
  for (int q = 0; q < 4 * n_cond; ++q)
    if (cond_ijkl[q] < 0 || cond_ijkl[q] >= n)
      return fail(BPMF_E_INVAL, "conditioning torsion atom out of range");
  for (int q = 0; q < kNParams; ++q)
    if (!isfinite(params[q])) return fail(BPMF_E_INVAL, "non-finite parameter");
  const int K = h.dev.K;
  Arena A;
  const size_t o_p = A.add(kNParams * 4), o_g = A.add(kNParams * 4),
               o_m = A.add(kNParams * 4), o_v = A.add(kNParams * 4),
               o_acc = A.add(K * 8), o_try = A.add(K * 8), o_la = A.add(K * 8),
               o_dev = A.add(sizeof(PropDev)),
               o_wt = A.add((size_t)kTSize * sizeof(unsigned short));
  char* base = (char*)c->dalloc(A.total);
  if (!base) return fail(BPMF_E_NOMEM, "proposal allocation failed");
  PropDev pd{};
  for (int a = 0; a < 3; ++a) pd.frame[a] = frame_atoms[a];
  pd.n_cond = n_cond;
  for (int q = 0; q < n_cond; ++q)
    pd.cond[q] = make_int4(cond_ijkl[4 * q], cond_ijkl[4 * q + 1],
                           cond_ijkl[4 * q + 2], cond_ijkl[4 * q + 3]);
  pd.pose_acc = (unsigned long long*)(base + o_acc);
  pd.pose_try = (unsigned long long*)(base + o_try);
  pd.last_ln_alpha = (double*)(base + o_la);
  hipError_t e = hipMemcpyAsync(base + o_p, params, kNParams * 4,
                                hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(base + o_m, 0, kNParams * 4, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(base + o_v, 0, kNParams * 4, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(base + o_acc, 0, K * 8, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(base + o_try, 0, K * 8, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(base + o_la, 0, K * 8, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(base + o_dev, &pd, sizeof(PropDev), hipMemcpyHostToDevice,
                       c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    c->dfree(base);
    return fail(BPMF_E_HIP, "proposal upload: %s", hipGetErrorString(e));
  }
  c->dfree(h.prop_arena);
  h.prop_arena = base;
  h.params = (float*)(base + o_p);
  h.grad = (float*)(base + o_g);
  h.adam_m = (float*)(base + o_m);
  h.adam_v = (float*)(base + o_v);
  h.d_prop = (PropDev*)(base + o_dev);
  h.wt = (unsigned short*)(base + o_wt);
  h.wt_dirty = true;
  h.prop = pd;
  h.adam_t = 0;
  h.has_prop = true;
  c->pose_dirty = true;
  return BPMF_OK;
}

extern "C" int bpmf_proposal_params(bpmf_ctx* c, int lid, float* out,
                                    const float* in) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_prop(c, lid))) return rc;
  LigHost& h = c->ligs[lid];
  if (in) {
    HIP_TRY(hipMemcpyAsync(h.params, in, kNParams * 4, hipMemcpyHostToDevice,
                           c->stream));
    h.wt_dirty = true;
  }
  if (out)
    HIP_TRY(hipMemcpyAsync(out, h.params, kNParams * 4, hipMemcpyDeviceToHost,
                           c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return BPMF_OK;
}

extern "C" int bpmf_pose_features(bpmf_ctx* c, int lid, const float* dev_x,
                                  int64_t N, float* dev_feats,
                                  float* dev_poses) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_prop(c, lid))) return rc;
  if (N < 0) return fail(BPMF_E_INVAL, "negative N");
  if (N == 0) return BPMF_OK;
  if (!dev_x || !dev_feats || !dev_poses)
    return fail(BPMF_E_INVAL, "null pose_features argument");
  HIP_TRY(launch_pose_features(c->d_ligs + lid, c->ligs[lid].d_prop, dev_x, N,
                               dev_feats, dev_poses, c->stream));
  return BPMF_OK;
}

extern "C" int bpmf_proposal_forward(bpmf_ctx* c, int lid,
                                     const float* dev_feats, int64_t N,
                                     float* dev_out) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_prop(c, lid))) return rc;
  if (N < 0 || N > (1 << 24)) return fail(BPMF_E_INVAL, "N outside 0..2^24");
  if (N == 0) return BPMF_OK;
  if (!dev_feats || !dev_out) return fail(BPMF_E_INVAL, "null argument");
  MlpBufs b;
  if ((rc = mlp_scratch(c, (int)N, &b))) return rc;
  return mlp_forward(c, c->ligs[lid].params, dev_feats, (int)N, b, dev_out,
                     c->stream);
}

extern "C" int bpmf_proposal_grad(bpmf_ctx* c, int lid, const float* dev_feats,
                                  const float* dev_poses, int64_t N,
                                  float* dev_grad, double* loss) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_prop(c, lid))) return rc;
  if (N < 1 || N > (1 << 24)) return fail(BPMF_E_INVAL, "N outside 1..2^24");
  if (!dev_feats || !dev_poses || !dev_grad)
    return fail(BPMF_E_INVAL, "null argument");
  MlpBufs b;
  if ((rc = mlp_scratch(c, (int)N, &b))) return rc;
  if ((rc = mlp_grad(c, c->ligs[lid].params, dev_feats, dev_poses, (int)N, b,
                     dev_grad)))
    return rc;
  if (loss) return read_loss(c, b, (int)N, loss);
  return BPMF_OK;
}

extern "C" int bpmf_proposal_train(bpmf_ctx* c, int lid, const float* dev_feats,
                                   const float* dev_poses, int64_t N, int batch,
                                   int steps, double lr, double* loss_out) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_prop(c, lid))) return rc;
  if (N < 1 || batch < 1 || batch > (1 << 20) || steps < 0 || !(lr > 0))
    return fail(BPMF_E_INVAL, "bad training arguments");
  if (!dev_feats || !dev_poses) return fail(BPMF_E_INVAL, "null data");
  LigHost& h = c->ligs[lid];
  MlpBufs b;
  if ((rc = mlp_scratch(c, batch, &b))) return rc;
  if (steps > 0) h.wt_dirty = true;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  for (int s = 0; s < steps; ++s) {
    HIP_TRY(launch_gather_batch(dev_feats, dev_poses, N, batch, c->seed,
                                (uint64_t)h.adam_t, b.bf, b.bp, c->stream));
    if ((rc = mlp_grad(c, h.params, b.bf, b.bp, batch, b, h.grad))) return rc;
    ++h.adam_t;
    const float c1 = 1.f - powf(b1, (float)h.adam_t);
    const float c2 = 1.f - powf(b2, (float)h.adam_t);
    HIP_TRY(launch_adam(h.params, h.grad, h.adam_m, h.adam_v, kNParams,
                        (float)lr, b1, b2, eps, c1, c2, c->stream));
    if (loss_out && (rc = read_loss(c, b, batch, &loss_out[s]))) return rc;
  }
  return BPMF_OK;
}

namespace {
// Tables of the batched pose move (see bpmf_ctx), rebuilt when ligands or
// proposals have changed; a rebuild invalidates captured graphs.
int build_pose_tables(bpmf_ctx* c) {
  if (!c->pose_dirty) return BPMF_OK;
  const int nl = (int)c->ligs.size();
  std::vector<PropDev> props(std::max(nl, 1));
  std::vector<PoseTask> tasks;
  std::vector<MlpGroup> groups;
  int off[bpmf_ctx::kWaveClasses], cnt[bpmf_ctx::kWaveClasses];
  for (int q = 0; q < bpmf_ctx::kWaveClasses; ++q) {
    off[q] = (int)tasks.size();
    for (int l = 0; l < nl; ++l) {
      LigHost& h = c->ligs[l];
      if (!h.has_prop || wave_class(h.min_waves) != q) continue;
      props[l] = h.prop;
      h.ptask0 = (int)tasks.size();
      h.pgroup0 = (int)groups.size();
      for (int r = 0; r < h.dev.K; ++r) {
        const int row = (int)tasks.size();
        tasks.push_back(PoseTask{l, r, row, 0});
      }
      for (int r = 0; r < h.dev.K; r += 16)
        groups.push_back(MlpGroup{h.params, h.wt, h.ptask0 + r,
                                  std::min(16, h.dev.K - r)});
      h.n_pgroups = (int)groups.size() - h.pgroup0;
    }
    cnt[q] = (int)tasks.size() - off[q];
  }
  void* np = c->dalloc(sizeof(PropDev) * props.size());
  void* nt = c->dalloc(sizeof(PoseTask) * std::max<size_t>(tasks.size(), 1));
  void* ng = c->dalloc(sizeof(MlpGroup) * std::max<size_t>(groups.size(), 1));
  if (!np || !nt || !ng) {
    c->dfree(np);
    c->dfree(nt);
    c->dfree(ng);
    return fail(BPMF_E_NOMEM, "pose-move table allocation failed");
  }
  HIP_TRY(hipMemcpyAsync(np, props.data(), sizeof(PropDev) * props.size(),
                         hipMemcpyHostToDevice, c->stream));
  if (!tasks.empty())
    HIP_TRY(hipMemcpyAsync(nt, tasks.data(), sizeof(PoseTask) * tasks.size(),
                           hipMemcpyHostToDevice, c->stream));
  if (!groups.empty())
    HIP_TRY(hipMemcpyAsync(ng, groups.data(),
                           sizeof(MlpGroup) * groups.size(),
                           hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->drop_graph();
  ++c->table_version;
  c->dfree(c->d_props);
  c->dfree(c->d_ptasks);
  c->dfree(c->d_pgroups);
  c->d_props = (PropDev*)np;
  c->d_ptasks = (PoseTask*)nt;
  c->d_pgroups = (MlpGroup*)ng;
  c->n_ptasks = (int)tasks.size();
  c->n_pgroups = (int)groups.size();
  for (int q = 0; q < bpmf_ctx::kWaveClasses; ++q) {
    c->ptask_off[q] = off[q];
    c->ptask_n[q] = cnt[q];
  }
  c->pose_dirty = false;
  return BPMF_OK;
}

// Refresh the bf16 weight copies that are stale (enqueued on the stream;
// called outside graph capture, before the moves that read them).
int refresh_pose_weights(bpmf_ctx* c) {
  for (auto& h : c->ligs)
    if (h.has_prop && h.wt_dirty) {
      HIP_TRY(launch_weights_bf16(h.params, h.wt, c->stream));
      h.wt_dirty = false;
    }
  return BPMF_OK;
}

// One pose move of every replica of ligand `only` (-1: of every ligand
// with a proposal): features, the network and the move, each one launch
// over all of the ligands (the move one per wavefront class).  The tables
// and the network's scratch must be ready (not rebuilt under capture).
// One pose move of every replica of every ligand with a proposal (or of
// ligand `only`): the network on the current configurations, then the
// moves.  close: the run of sweeps before it ends in the network launch
// (its extra blocks apply the last exchange and record of ligands
// [l0, l1)) and the next one starts in the move launch, so that no begin or
// finish kernel brackets the unit; every ligand in that range must have a
// proposal.
int pose_move_batch(bpmf_ctx* c, int only, hipStream_t st,
                    const UnitClose* close) {
  int t0 = 0, nt = c->n_ptasks, g0 = 0, ng = c->n_pgroups;
  if (only >= 0) {
    const LigHost& h = c->ligs[only];
    if (!h.has_prop) return BPMF_OK;
    t0 = h.ptask0;
    nt = h.dev.K;
    g0 = h.pgroup0;
    ng = h.n_pgroups;
  }
  if (nt == 0) return BPMF_OK;
  MlpBufs b;
  int rc = mlp_scratch(c, c->n_ptasks, &b);
  if (rc) return rc;
  const int n_fin = close ? close->l1 - close->l0 : 0;
  HIP_TRY(launch_pose_network(
      c->d_pgroups + g0, ng, c->d_ligs, c->d_props, c->d_ptasks, b.out,
      close ? c->d_ligs + close->l0 : nullptr, n_fin,
      close ? close->exchange_every : 0, close ? close->sample_every : 0,
      c->seed, st));
  // one launch at the widest class in the range: the move is latency-bound
  // (one workgroup per replica), and narrower ligands run with idle
  // wavefronts rather than in a launch of their own
  int qmax = 0;
  for (int q = 0; q < bpmf_ctx::kWaveClasses; ++q) {
    const int a = std::max(t0, c->ptask_off[q]);
    const int e = std::min(t0 + nt, c->ptask_off[q] + c->ptask_n[q]);
    if (e > a) qmax = q;
  }
  HIP_TRY(launch_pose_move(c->grid, c->d_ligs, c->d_props, c->d_ptasks + t0,
                           nt, b.out, 1 << qmax,
                           block_lds_bytes(1 << qmax, false, 0, 0, 0, 0),
                           c->seed, close != nullptr, st));
  return BPMF_OK;
}
}  // namespace

extern "C" int bpmf_pose_move(bpmf_ctx* c, int lid, int rounds) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (rounds < 0) return fail(BPMF_E_INVAL, "negative rounds");
  if (lid != -1 && (rc = check_prop(c, lid))) return rc;
  if ((rc = build_pose_tables(c)) || (rc = refresh_pose_weights(c))) return rc;
  for (int r = 0; r < rounds; ++r)
    if ((rc = pose_move_batch(c, lid, c->stream))) return rc;
  return BPMF_OK;
}

// ============================================================================
// external-coordinate moves
// ============================================================================
namespace {
// the moves of ligands [l0, l1) in one launch per wavefront count present
// (a ligand's blocks run in the launch of its own count)
int external_moves_range(bpmf_ctx* c, int l0, int l1, int n_moves,
                         int k_max, double sigma, hipStream_t st) {
  for (int W = 1; W <= 2; ++W) {
    int kg = 0;
    for (int l = l0; l < l1; ++l) {
      const LigHost& h = c->ligs[l];
      if (h.min_waves == W) kg = std::max(kg, std::min(k_max, h.dev.K));
    }
    if (kg == 0) continue;
    HIP_TRY(launch_external_moves(c->grid, c->d_ligs + l0, l1 - l0, kg, W,
                                  n_moves, k_max, (float)sigma, c->seed, st));
  }
  return BPMF_OK;
}

int check_external(int n_moves, int k_max, double sigma) {
  if (n_moves < 0) return fail(BPMF_E_INVAL, "negative n_moves");
  if (k_max < 0) return fail(BPMF_E_INVAL, "negative k_max");
  if (n_moves > 0 && !(sigma > 0 && std::isfinite(sigma)))
    return fail(BPMF_E_INVAL, "translation sigma must be positive and finite");
  return BPMF_OK;
}
}  // namespace

extern "C" int bpmf_external_move(bpmf_ctx* c, int lid, int n_moves,
                                  int k_max, double sigma) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (lid != -1 && (rc = check_lig(c, lid))) return rc;
  if ((rc = check_external(n_moves, k_max, sigma))) return rc;
  const int l0 = lid == -1 ? 0 : lid;
  const int l1 = lid == -1 ? (int)c->ligs.size() : lid + 1;
  return external_moves_range(c, l0, l1, n_moves, k_max, sigma, c->stream);
}

extern "C" int bpmf_get_external_stats(bpmf_ctx* c, int lid, int64_t* acc,
                                       int64_t* tries) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_lig(c, lid))) return rc;
  const LigHost& h = c->ligs[lid];
  const int K = h.dev.K;
  std::vector<unsigned long long> a(K), t(K);
  HIP_TRY(hipMemcpyAsync(a.data(), h.ext_acc, K * 8, hipMemcpyDeviceToHost,
                         c->stream));
  HIP_TRY(hipMemcpyAsync(t.data(), h.ext_try, K * 8, hipMemcpyDeviceToHost,
                         c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (int k = 0; k < K; ++k) {
    if (acc) acc[k] = (int64_t)a[k];
    if (tries) tries[k] = (int64_t)t[k];
  }
  return BPMF_OK;
}

extern "C" int bpmf_get_pose_stats(bpmf_ctx* c, int lid, int64_t* acc,
                                   int64_t* tries, double* last_ln_alpha) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if ((rc = check_prop(c, lid))) return rc;
  const LigHost& h = c->ligs[lid];
  const int K = h.dev.K;
  if (acc)
    HIP_TRY(hipMemcpyAsync(acc, h.prop.pose_acc, K * 8, hipMemcpyDeviceToHost,
                           c->stream));
  if (tries)
    HIP_TRY(hipMemcpyAsync(tries, h.prop.pose_try, K * 8,
                           hipMemcpyDeviceToHost, c->stream));
  if (last_ln_alpha)
    HIP_TRY(hipMemcpyAsync(last_ln_alpha, h.prop.last_ln_alpha, K * 8,
                           hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return BPMF_OK;
}

extern "C" int bpmf_set_graph(bpmf_ctx* c, int chunk) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (chunk < 0 || chunk > 4096)
    return fail(BPMF_E_INVAL, "chunk must be 0 (no graph) .. 4096");
  c->graph_chunk = chunk;
  c->drop_graph();
  return BPMF_OK;
}

// ============================================================================
// autotuner: wavefronts per replica
// ============================================================================
extern "C" int bpmf_autotune(bpmf_ctx* c, int n_sweeps, int n_leapfrog,
                             double* ms_out, int* chosen) {
  int rc = check_ctx(c);
  if (rc) return rc;
  if (c->ligs.empty()) return fail(BPMF_E_STATE, "no ligand set up");
  if (n_sweeps < 1 || n_leapfrog < 1)
    return fail(BPMF_E_INVAL, "n_sweeps and n_leapfrog must be >= 1");
  // snapshot every ligand's state (all but its sample store) on the device
  size_t total = 0;
  for (auto& h : c->ligs) total += (h.state_bytes + 255) / 256 * 256;
  char* snap = (char*)c->dalloc(total);
  if (!snap) return fail(BPMF_E_NOMEM, "autotune snapshot allocation failed");
  std::vector<std::pair<uint64_t, int64_t>> mirror;
  for (auto& h : c->ligs) mirror.emplace_back(h.counter, h.n_rec);
  auto copy_all = [&](bool save) -> int {
    size_t off = 0;
    if (!save)
      for (size_t l = 0; l < c->ligs.size(); ++l) {
        c->ligs[l].counter = mirror[l].first;
        c->ligs[l].n_rec = mirror[l].second;
      }
    for (auto& h : c->ligs) {
      char* a = (char*)h.arena;
      HIP_TRY(hipMemcpyAsync(save ? snap + off : a, save ? a : snap + off,
                             h.state_bytes, hipMemcpyDeviceToDevice,
                             c->stream));
      off += (h.state_bytes + 255) / 256 * 256;
    }
    return BPMF_OK;
  };
  const int old_override = c->waves_override;
  const int old_order = c->task_order;
  c->task_order = 1;  // shapes are timed heaviest first
  std::vector<int> old_pins;
  for (auto& h : c->ligs) old_pins.push_back(h.waves_pin);
  const bool old_timing = c->timing;
  const int old_every = c->timing_every;
  // mean sweep time of the current launch shape, the state restored after
  auto trial = [&](double* ms) -> int {
    int r;
    if ((r = rebuild_tables(c))) return r;
    bpmf_sweep_args a{2, n_leapfrog, 1, 0, 1, 0, 0};
    if ((r = bpmf_hmc_sweep(c, &a))) return r;
    c->timing = true;
    c->timing_every = 1;
    c->launches[BPMF_TIMER_HMC] = 0;
    c->ev_used[BPMF_TIMER_HMC] = 0;
    a.n_sweeps = n_sweeps;
    if ((r = bpmf_hmc_sweep(c, &a))) return r;
    int64_t cnt = 0;
    if ((r = bpmf_get_timing(c, BPMF_TIMER_HMC, ms, &cnt))) return r;
    return copy_all(false);
  };
  const int cand[5] = {0, 1, 2, 4, 8};
  double best = INFINITY;
  int best_w = 0;
  if ((rc = copy_all(true))) {
    c->dfree(snap);
    return rc;
  }
  for (auto& h : c->ligs) h.waves_pin = 0;
  for (int q = 0; q < 5 && !rc; ++q) {
    double ms = INFINITY;
    c->waves_override = cand[q];
    if ((rc = trial(&ms))) break;
    if (ms < best) {
      best = ms;
      best_w = cand[q];
    }
    if (ms_out) ms_out[q] = ms;
  }
  // refinement: per atom-count class (up to 16, 32, 48, 64, 96, 128 atoms),
  // one class at a time, the other wavefront counts with the rest kept;
  // a change stays when it saves more than 2 % (the classes' launches run
  // side by side, so mixed shapes cost no serialisation)
  c->waves_override = best_w;
  auto size_class = [](int n) {
    return n <= 16 ? 0 : n <= 32 ? 1 : n <= 48 ? 2 : n <= 64 ? 3
           : n <= 96 ? 4 : 5;
  };
  bool present[6] = {false, false, false, false, false, false};
  for (auto& h : c->ligs) present[size_class(h.dev.n)] = true;
  for (int sc = 5; sc >= 0 && !rc; --sc) {
    if (!present[sc]) continue;
    int keep = 0;  // the class's pin so far (0: the context-wide choice)
    for (int w : {1, 2, 4, 8}) {
      if (w == (best_w ? best_w : -1)) continue;
      for (auto& h : c->ligs)
        if (size_class(h.dev.n) == sc) h.waves_pin = w;
      double ms = INFINITY;
      if ((rc = trial(&ms))) break;
      if (ms < 0.98 * best) {
        best = ms;
        keep = w;
      }
    }
    for (auto& h : c->ligs)
      if (size_class(h.dev.n) == sc) h.waves_pin = keep;
  }
  // the workgroup order, with the shapes chosen (heaviest first unless
  // ligand by ligand saves more than 2 %)
  int best_order = 1;
  if (!rc && c->ligs.size() > 1) {
    const double with_order = best;  // the last trials ran heaviest first
    c->task_order = 0;
    double ms = INFINITY;
    rc = trial(&ms);
    if (!rc && ms < 0.98 * with_order) best_order = 0;
  }
  c->task_order = best_order;
  c->timing = old_timing;
  c->timing_every = old_every;
  if (!rc) (void)copy_all(false);
  (void)hipStreamSynchronize(c->stream);
  c->dfree(snap);
  if (rc) {
    c->waves_override = old_override;
    c->task_order = old_order;
    for (size_t l = 0; l < c->ligs.size(); ++l)
      c->ligs[l].waves_pin = old_pins[l];
    (void)rebuild_tables(c);
    return rc;
  }
  if ((rc = rebuild_tables(c))) return rc;
  if (chosen) *chosen = best_w;
  return BPMF_OK;
}
