// Initialisation and adaptation of the thermodynamic-state ladder
// (Initialization; state insertion and equilibration detection from
// Equilibration and production).  Host logic: the arithmetic of each step is
// a function of its own below, and bpmf_initialize_ladder drives them with
// the library's sampler (bpmf_hmc_sweep_ligand), evaluation and placement
// kernels.  Every statistic comes from the energy components the sampler
// records with each sample (U0 = bonded + restraint, then Psi_c per grid
// channel), in double.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/bpmf.h"
#include "protocol.h"

using namespace bpmf;

namespace {

constexpr double kR = 8.314462618e-3;  // kJ/(mol K)
// the paper's constants (Initialization)
constexpr double kPLow = 0.4, kPHigh = 0.99, kSpeedFactor = 0.8;
constexpr double kAccLow = 0.4, kAccHigh = 0.8, kAccVeryLow = 0.1;
constexpr double kDtUp = 0.125, kDtDown = 0.25, kDtDownMore = 0.5;

int bad(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
int bad(const char* fmt, ...) {
  char buf[384];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  return ctx_fail(BPMF_E_INVAL, buf);
}

// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) for host-side draws:
// ten rounds of two multiply/xor boxes, keys bumped by the Weyl constants
struct H4 {
  uint32_t x, y, z, w;
};
H4 philox_host(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
               uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c0 = n0;
    c1 = (uint32_t)p1;
    c2 = n2;
    c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return H4{c0, c1, c2, c3};
}
// uniform in (0, 1] of draw (index, ligand<<16 | rep, sweep, purpose)
double uniform_host(uint64_t seed, uint32_t index, int lig, int rep,
                    uint64_t sweep, uint32_t purpose) {
  const H4 o = philox_host(index, ((uint32_t)lig << 16) | (uint32_t)rep,
                           (uint32_t)sweep, purpose, (uint32_t)seed,
                           (uint32_t)(seed >> 32));
  return ((double)o.x + 1.0) * 2.3283064365386962890625e-10;
}

// schedule of the grid path (Thermodynamic Cycle)
double temperature(double a, double TH, double TT) { return (TT - TH) * a + TH; }
double alpha_sg(double a) { return 1.0 - (2.0 * a - 1.0) * (2.0 * a - 1.0); }
double alpha_g(double a) {
  return (2.0 * a - 1.0) * (2.0 * a - 1.0) /
         (1.0 + exp(-1000.0 * (a - 0.5)));
}
double d_alpha_sg(double a) { return -4.0 * (2.0 * a - 1.0); }
double d_alpha_g(double a) {
  // logistic sig and its derivative 1000 sig (1 - sig)
  const double sig = 1.0 / (1.0 + exp(-1000.0 * (a - 0.5)));
  return 4.0 * (2.0 * a - 1.0) * sig +
         (2.0 * a - 1.0) * (2.0 * a - 1.0) * 1000.0 * sig * (1.0 - sig);
}

void state_of(double a, int kind, int C, double TH, double TT, double* T,
              double* w) {
  *T = temperature(a, TH, TT);
  if (kind == BPMF_SCHEDULE_LINEAR) {
    for (int c = 0; c < C; ++c) w[c] = a;
  } else {
    const double g = alpha_g(a), sg = alpha_sg(a);
    for (int c = 0; c < C; ++c) w[c] = c < 3 ? g : sg;
  }
}

int check_kind(int kind, int C) {
  if (kind != BPMF_SCHEDULE_LINEAR && kind != BPMF_SCHEDULE_SOFT)
    return bad("schedule kind %d is neither linear (0) nor soft (1)", kind);
  if (C < 1 || C > BPMF_MAX_CHANNELS)
    return bad("n_channels %d outside 1..%d", C, BPMF_MAX_CHANNELS);
  if (kind == BPMF_SCHEDULE_SOFT && C != 5)
    return bad("the soft schedule needs 5 channels (rep, att, ele, soft rep, "
               "soft ele), not %d", C);
  return BPMF_OK;
}

// reduced energy of one sample's components at (T, w)
double reduced(const double* comp, int C, double T, const double* w) {
  double E = comp[0];
  for (int c = 0; c < C; ++c) E += w[c] * comp[1 + c];
  return E / (kR * T);
}

// population standard deviation (two passes)
double stdev(const std::vector<double>& v) {
  if (v.empty()) return 0.0;
  double m = 0;
  for (double x : v) m += x;
  m /= (double)v.size();
  double s = 0;
  for (double x : v) s += (x - m) * (x - m);
  return sqrt(s / (double)v.size());
}

// g of a series: 1 + 2 sum_t (1 - t/N) C_t / C_0, stopped at the first
// C_t <= 0
double stat_inefficiency(const double* a, int64_t N) {
  double m = 0;
  for (int64_t i = 0; i < N; ++i) m += a[i];
  m /= (double)N;
  std::vector<double> d(N);
  for (int64_t i = 0; i < N; ++i) d[i] = a[i] - m;
  double c0 = 0;
  for (int64_t i = 0; i < N; ++i) c0 += d[i] * d[i];
  c0 /= (double)N;
  if (c0 <= 0) return 1.0;
  double g = 1.0;
  for (int64_t t = 1; t < N - 1; ++t) {
    double ct = 0;
    for (int64_t i = 0; i + t < N; ++i) ct += d[i] * d[i + t];
    ct /= (double)(N - t);
    if (ct <= 0) break;
    g += 2.0 * (1.0 - (double)t / (double)N) * ct / c0;
  }
  return g > 1.0 ? g : 1.0;
}

}  // namespace

// ============================================================================
// the steps
// ============================================================================
extern "C" int bpmf_protocol_state(double alpha, int kind, int n_channels,
                                   double T_hot, double T_cold, double* T,
                                   double* w) {
  int rc = check_kind(kind, n_channels);
  if (rc) return rc;
  if (!T || !w) return bad("null output");
  if (!(alpha >= 0.0 && alpha <= 1.0)) return bad("alpha %g outside [0, 1]", alpha);
  state_of(alpha, kind, n_channels, T_hot, T_cold, T, w);
  return BPMF_OK;
}

extern "C" int bpmf_protocol_sigmas(const double* comps, int64_t n,
                                    int n_channels, double alpha, int kind,
                                    double T_hot, double T_cold,
                                    double* sigma) {
  int rc = check_kind(kind, n_channels);
  if (rc) return rc;
  if (!comps || !sigma || n < 1) return bad("need samples and an output");
  const int C = n_channels, C1 = 1 + C;
  double T, w[BPMF_MAX_CHANNELS];
  state_of(alpha, kind, C, T_hot, T_cold, &T, w);
  std::vector<double> pg(n), psg(n), u(n);
  for (int64_t i = 0; i < n; ++i) {
    const double* cp = comps + i * C1;
    double g = 0, sg = 0;
    for (int c = 0; c < C; ++c) {
      if (kind == BPMF_SCHEDULE_SOFT && c >= 3)
        sg += cp[1 + c];
      else
        g += cp[1 + c];
    }
    pg[i] = g;
    psg[i] = sg;
    u[i] = reduced(cp, C, T, w);
  }
  sigma[0] = stdev(pg);
  sigma[1] = stdev(psg);
  sigma[2] = stdev(u);
  return BPMF_OK;
}

extern "C" int bpmf_protocol_next_alpha(double alpha, const double* sigma,
                                        int kind, double speed, double T_hot,
                                        double T_cold, double* next) {
  if (!sigma || !next) return bad("null argument");
  if (kind != BPMF_SCHEDULE_LINEAR && kind != BPMF_SCHEDULE_SOFT)
    return bad("bad schedule kind %d", kind);
  if (!(speed > 0)) return bad("speed must be positive");
  const double T = temperature(alpha, T_hot, T_cold), kT = kR * T;
  const double dg = kind == BPMF_SCHEDULE_LINEAR ? 1.0 : d_alpha_g(alpha);
  const double dsg = kind == BPMF_SCHEDULE_LINEAR ? 0.0 : d_alpha_sg(alpha);
  const double denom = fabs(dsg) * sigma[1] / kT + fabs(dg) * sigma[0] / kT +
                       fabs(T_cold - T_hot) * sigma[2] / T;
  if (!(denom > 0.0)) {
    *next = 1.0;
    return BPMF_OK;
  }
  const double a = alpha + speed / denom;
  *next = a < 1.0 ? a : 1.0;
  return BPMF_OK;
}

extern "C" int bpmf_protocol_next_temperature(double T, double sigma_U,
                                              double speed, double T_target,
                                              double* next) {
  if (!next) return bad("null output");
  if (!(T > 0) || !(speed > 0)) return bad("T and speed must be positive");
  if (!(sigma_U > 0.0)) {
    *next = T_target;
    return BPMF_OK;
  }
  const double step = speed * kR * T * T / sigma_U;
  *next = T_target >= T ? std::min(T + step, T_target)
                        : std::max(T - step, T_target);
  return BPMF_OK;
}

extern "C" int bpmf_protocol_sir(const double* log_w, int64_t n, int n_draw,
                                 uint64_t seed, int ligand_id, int state,
                                 int64_t* idx) {
  if (!log_w || !idx || n < 1 || n_draw < 0) return bad("bad SIR arguments");
  double m = -INFINITY;
  for (int64_t i = 0; i < n; ++i)
    if (isfinite(log_w[i]) && log_w[i] > m) m = log_w[i];
  if (!isfinite(m)) return bad("no finite weight");
  std::vector<double> cum(n);
  double acc = 0;
  for (int64_t i = 0; i < n; ++i) {
    acc += isfinite(log_w[i]) ? exp(log_w[i] - m) : 0.0;
    cum[i] = acc;
  }
  for (int j = 0; j < n_draw; ++j) {
    const double u = uniform_host(seed, (uint32_t)j, ligand_id, 0,
                                  (uint64_t)state, kInit | (kSubSir << 8));
    const int64_t i =
        std::lower_bound(cum.begin(), cum.end(), u * acc) - cum.begin();
    idx[j] = i < n ? i : n - 1;
  }
  return BPMF_OK;
}

extern "C" int bpmf_protocol_adapt_dt(double dt, double acc, double dt_min,
                                      double* new_dt, int* done) {
  if (!new_dt || !done) return bad("null output");
  if (acc > kAccHigh) {
    *new_dt = dt + kDtUp;
    *done = 0;
  } else if (acc < kAccLow) {
    if (dt <= dt_min) {
      *new_dt = dt;
      *done = 1;
    } else {
      const double step = acc < kAccVeryLow ? kDtDownMore : kDtDown;
      *new_dt = std::max(dt - step, dt_min);
      *done = 0;
    }
  } else {
    *new_dt = dt;
    *done = 1;
  }
  return BPMF_OK;
}

extern "C" int bpmf_protocol_mean_pacc(const double* uk_x, const double* uk1_x,
                                       const double* uk_y, const double* uk1_y,
                                       int64_t n, double* mean) {
  if (!uk_x || !uk1_x || !uk_y || !uk1_y || !mean || n < 1)
    return bad("bad p_acc arguments");
  double s = 0;
  for (int64_t i = 0; i < n; ++i) {
    const double d = uk_y[i] + uk1_x[i] - uk_x[i] - uk1_y[i];
    s += isfinite(d) ? exp(-(d > 0 ? d : 0.0)) : 0.0;
  }
  *mean = s / (double)n;
  return BPMF_OK;
}

extern "C" int bpmf_protocol_insert(const double* alpha, int K,
                                    const double* pacc, double threshold,
                                    int max_out, double* out, int* K_out) {
  if (!alpha || !out || !K_out || K < 1 || (K > 1 && !pacc))
    return bad("bad insertion arguments");
  int m = 0;
  auto put = [&](double v) -> bool {
    if (m >= max_out) return false;
    out[m++] = v;
    return true;
  };
  if (!put(alpha[0])) return bad("max_out %d too small", max_out);
  for (int k = 0; k + 1 < K; ++k) {
    if (pacc[k] < threshold && !put(0.5 * (alpha[k] + alpha[k + 1])))
      return bad("max_out %d too small", max_out);
    if (!put(alpha[k + 1])) return bad("max_out %d too small", max_out);
  }
  *K_out = m;
  return BPMF_OK;
}

extern "C" int bpmf_detect_equilibration(const double* a, int64_t n,
                                         int n_candidates, int64_t* t0,
                                         double* g, double* n_eff) {
  if (!a || n < 2 || n_candidates < 1 || !t0 || !g || !n_eff)
    return bad("bad equilibration-detection arguments");
  int64_t bt = 0;
  double bg = 1.0, bn = -1.0;
  for (int i = 0; i < n_candidates; ++i) {
    const int64_t t = (int64_t)i * n / n_candidates;
    if (n - t < 2) break;
    const double gi = stat_inefficiency(a + t, n - t);
    const double ne = (double)(n - t) / gi;
    if (ne > bn) {
      bt = t;
      bg = gi;
      bn = ne;
    }
  }
  *t0 = bt;
  *g = bg;
  *n_eff = bn;
  return BPMF_OK;
}

// ============================================================================
// bpmf_initialize_ladder: the steps run on the sampler
// ============================================================================
namespace {

#define TRY(expr)                 \
  do {                            \
    const int r_ = (expr);        \
    if (r_ != BPMF_OK) return r_; \
  } while (0)

// device buffers of one initialisation, released on every exit
struct DevBufs {
  bpmf_ctx* c;
  std::vector<void*> held;
  explicit DevBufs(bpmf_ctx* cc) : c(cc) {}
  void* get(size_t bytes) {
    void* p = ctx_alloc(c, bytes);
    if (p) held.push_back(p);
    return p;
  }
  ~DevBufs() {
    (void)hipStreamSynchronize(ctx_stream(c));
    for (void* p : held) ctx_free(c, p);
  }
};

// a state's sample set: components (N x (1 + C)); coordinates either on the
// host (N x n x 3) or implicit in the placements of device configurations
struct Samples {
  int64_t N = 0;
  std::vector<double> comps;
  std::vector<float> x;
  const float* d_confs = nullptr;  // placements: n_conf x n x 3 (device)
  int n_conf = 0, n_com = 0, n_orient = 0;
};

struct Driver {
  bpmf_ctx* c;
  const bpmf_init_args* a;
  int lid, n, K, C;
  DevBufs bufs;
  int n_runs = 0;
  Driver(bpmf_ctx* cc, const bpmf_init_args* aa, int nn, int KK, int CC)
      : c(cc), a(aa), lid(aa->ligand_id), n(nn), K(KK), C(CC), bufs(cc) {}

  // K runs of n_trials HMC trials from seeds (K x n x 3) at (T, w), the time
  // step adapted by the paper's rule; the samples and final configurations
  // of the last run
  int run_state(double T, const double* w, double dt_in, const float* seeds,
                Samples* S, std::vector<float>* fx, double* dt_out,
                double* acc_out) {
    std::vector<double> Tv(K, T), wv((size_t)K * C), dtv(K);
    for (int k = 0; k < K; ++k)
      for (int ch = 0; ch < C; ++ch) wv[(size_t)k * C + ch] = w[ch];
    std::vector<int> sor(K);
    for (int k = 0; k < K; ++k) sor[k] = k;
    std::vector<int64_t> ha(K), ht(K);
    double dt = dt_in, acc = 0;
    for (int round = 0; round < a->max_dt_rounds; ++round) {
      for (int k = 0; k < K; ++k) dtv[k] = dt;
      TRY(bpmf_set_states(c, lid, Tv.data(), wv.data(), dtv.data()));
      uint64_t counter = 0;
      TRY(bpmf_get_replicas(c, lid, nullptr, nullptr, nullptr, &counter));
      TRY(bpmf_set_replicas(c, lid, seeds, sor.data(), nullptr, counter));
      TRY(bpmf_reset_samples(c, lid));
      TRY(bpmf_get_stats(c, lid, ha.data(), ht.data(), nullptr, nullptr,
                         nullptr));
      int64_t a0 = 0, t0 = 0;
      for (int k = 0; k < K; ++k) {
        a0 += ha[k];
        t0 += ht[k];
      }
      bpmf_sweep_args sa;
      memset(&sa, 0, sizeof(sa));
      sa.n_sweeps = a->n_trials;
      sa.n_leapfrog = a->n_leapfrog;
      sa.exchange_every = 0;
      sa.max_sep = 1;
      sa.sample_every = 1;
      sa.external_sigma = 0.6;
      TRY(bpmf_hmc_sweep_ligand(c, lid, &sa));
      ++n_runs;
      TRY(bpmf_get_stats(c, lid, ha.data(), ht.data(), nullptr, nullptr,
                         nullptr));
      int64_t a1 = 0, t1 = 0;
      for (int k = 0; k < K; ++k) {
        a1 += ha[k];
        t1 += ht[k];
      }
      acc = t1 > t0 ? (double)(a1 - a0) / (double)(t1 - t0) : 0.0;
      double nd;
      int done;
      TRY(bpmf_protocol_adapt_dt(dt, acc, a->dt_min, &nd, &done));
      if (done || round + 1 == a->max_dt_rounds) break;
      dt = nd;
    }
    int64_t nrec = 0;
    TRY(bpmf_get_samples(c, lid, &nrec, nullptr, nullptr));
    S->N = nrec * K;
    S->comps.assign((size_t)S->N * (1 + C), 0.0);
    S->x.assign((size_t)S->N * n * 3, 0.f);
    S->d_confs = nullptr;
    TRY(bpmf_get_samples(c, lid, &nrec, S->x.data(), S->comps.data()));
    fx->assign((size_t)K * n * 3, 0.f);
    TRY(bpmf_get_replicas(c, lid, fx->data(), nullptr, nullptr, nullptr));
    *dt_out = dt;
    *acc_out = acc;
    return BPMF_OK;
  }

  // state 0's sample set replaced by placements of n_conf of its final
  // configurations, components from the evaluation kernel
  int place(const std::vector<float>& fx, Samples* S) {
    const int64_t N = (int64_t)a->n_conf * a->n_com * a->n_orient;
    float* d_confs = (float*)bufs.get((size_t)a->n_conf * n * 12);
    const int64_t chunk = std::min<int64_t>(N, 1 << 18);
    float* d_x = (float*)bufs.get((size_t)chunk * n * 12);
    double* d_w = (double*)bufs.get((size_t)chunk * C * 8);
    double* d_t = (double*)bufs.get((size_t)chunk * (4 + C) * 8);
    if (!d_confs || !d_x || !d_w || !d_t)
      return ctx_fail(BPMF_E_NOMEM, "placement buffers");
    hipStream_t st = ctx_stream(c);
    if (hipMemcpyAsync(d_confs, fx.data(), (size_t)a->n_conf * n * 12,
                       hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemsetAsync(d_w, 0, (size_t)chunk * C * 8, st) != hipSuccess)
      return ctx_fail(BPMF_E_HIP, "placement upload failed");
    S->N = N;
    S->comps.assign((size_t)N * (1 + C), 0.0);
    S->x.clear();
    S->d_confs = d_confs;
    S->n_conf = a->n_conf;
    S->n_com = a->n_com;
    S->n_orient = a->n_orient;
    std::vector<double> t((size_t)chunk * (4 + C));
    for (int64_t f = 0; f < N; f += chunk) {
      const int64_t m = std::min(chunk, N - f);
      TRY(bpmf_place_poses(c, lid, d_confs, a->n_conf, a->n_com, a->n_orient,
                           f, m, d_x));
      TRY(bpmf_evaluate(c, lid, d_x, m, d_w, d_t, nullptr));
      if (hipMemcpyAsync(t.data(), d_t, (size_t)m * (4 + C) * 8,
                         hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return ctx_fail(BPMF_E_HIP, "placement energies: copy failed");
      for (int64_t i = 0; i < m; ++i) {
        const double* ti = t.data() + (size_t)i * (4 + C);
        double* cp = S->comps.data() + (size_t)(f + i) * (1 + C);
        cp[0] = ti[0] + ti[1] + ti[2] + ti[3];
        for (int ch = 0; ch < C; ++ch) cp[1 + ch] = ti[4 + ch];
      }
    }
    return BPMF_OK;
  }

  // coordinates of samples idx (K of them) of S, into seeds (K x n x 3)
  int gather(const Samples& S, const std::vector<int64_t>& idx,
             std::vector<float>* seeds) {
    seeds->assign((size_t)K * n * 3, 0.f);
    if (!S.d_confs) {
      for (int j = 0; j < K; ++j)
        memcpy(seeds->data() + (size_t)j * n * 3,
               S.x.data() + (size_t)idx[j] * n * 3, (size_t)n * 12);
      return BPMF_OK;
    }
    float* d_s = (float*)bufs.get((size_t)K * n * 12);
    if (!d_s) return ctx_fail(BPMF_E_NOMEM, "seed buffer");
    for (int j = 0; j < K; ++j)
      TRY(bpmf_place_poses(c, lid, S.d_confs, S.n_conf, S.n_com, S.n_orient,
                           idx[j], 1, d_s + (size_t)j * n * 3));
    hipStream_t st = ctx_stream(c);
    if (hipMemcpyAsync(seeds->data(), d_s, (size_t)K * n * 12,
                       hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return ctx_fail(BPMF_E_HIP, "seed copy failed");
    return BPMF_OK;
  }

  // mean exchange acceptance between the sample sets of two states, pairs
  // spread evenly over both sets (the same index when they are equal)
  double pacc(const Samples& A, double TA, const double* wA, const Samples& B,
              double TB, const double* wB) {
    const int64_t M = std::min(A.N, B.N);
    std::vector<double> ax(M), bx(M), ay(M), by(M);
    for (int64_t i = 0; i < M; ++i) {
      const double* x = A.comps.data() + (size_t)(i * A.N / M) * (1 + C);
      const double* y = B.comps.data() + (size_t)(i * B.N / M) * (1 + C);
      ax[i] = reduced(x, C, TA, wA);
      bx[i] = reduced(x, C, TB, wB);
      ay[i] = reduced(y, C, TA, wA);
      by[i] = reduced(y, C, TB, wB);
    }
    double m = 0;
    (void)bpmf_protocol_mean_pacc(ax.data(), bx.data(), ay.data(), by.data(),
                                  M, &m);
    return m;
  }
};

}  // namespace

extern "C" int bpmf_initialize_ladder(bpmf_ctx* c, const bpmf_init_args* a,
                                      bpmf_init_result* res) {
  if (!c || !a || !res) return bad("null argument");
  int n = 0, K = 0, C = 0, cap = 0;
  TRY(bpmf_ligand_info(c, a->ligand_id, &n, &K, &C, &cap));
  TRY(check_kind(a->kind, C));
  if (!(a->T_hot > 0) || !(a->T_cold > 0)) return bad("temperatures must be positive");
  if (!(a->speed > 0)) return bad("speed must be positive");
  if (a->n_trials < 1 || a->n_trials > cap)
    return bad("n_trials %d outside 1..sample capacity %d", a->n_trials, cap);
  if (a->n_leapfrog < 1) return bad("n_leapfrog must be >= 1");
  if (!(a->dt_start > 0) || !(a->dt_min > 0)) return bad("time steps must be positive");
  if (a->max_dt_rounds < 1 || a->max_selections < 1)
    return bad("max_dt_rounds and max_selections must be >= 1");
  if (a->max_states < 2) return bad("max_states must be >= 2");
  if (a->n_com < 0 || a->n_orient < 0 || a->n_conf < 0)
    return bad("negative placement count");
  if (a->n_com > 0 && (a->n_conf < 1 || a->n_conf > K || a->n_orient < 1))
    return bad("placements need 1 <= n_conf <= %d and n_orient >= 1", K);
  if (!res->alpha || !res->T || !res->w || !res->dt || !res->acc || !res->pacc)
    return bad("null result array");
  if (res->trace && res->trace_cap < 0) return bad("negative trace_cap");

  Driver d(c, a, n, K, C);
  const uint64_t seed = ctx_seed(c);
  int ns = 0, n_sel = 0, n_tr = 0;
  res->n_removed = 0;
  res->reached_target = 0;
  auto store = [&](int k, double alpha, double T, const double* w, double dt,
                   double acc, double p, const double* sig,
                   const std::vector<float>& fx) {
    res->alpha[k] = alpha;
    res->T[k] = T;
    for (int ch = 0; ch < C; ++ch) res->w[(size_t)k * C + ch] = w[ch];
    res->dt[k] = dt;
    res->acc[k] = acc;
    res->pacc[k] = p;
    if (res->sigma)
      for (int e = 0; e < 3; ++e) res->sigma[3 * k + e] = sig[e];
    if (res->x)
      memcpy(res->x + (size_t)k * K * n * 3, fx.data(), (size_t)K * n * 12);
  };

  // state 0 from the ligand's current replicas
  std::vector<float> seeds((size_t)K * n * 3), fx;
  TRY(bpmf_get_replicas(c, a->ligand_id, seeds.data(), nullptr, nullptr,
                        nullptr));
  double T0, w0[BPMF_MAX_CHANNELS], dt0, acc0, sig0[3];
  state_of(0.0, a->kind, C, a->T_hot, a->T_cold, &T0, w0);
  Samples S;
  TRY(d.run_state(T0, w0, a->dt_start, seeds.data(), &S, &fx, &dt0, &acc0));
  if (a->n_com > 0) TRY(d.place(fx, &S));
  TRY(bpmf_protocol_sigmas(S.comps.data(), S.N, C, 0.0, a->kind, a->T_hot,
                           a->T_cold, sig0));
  store(0, 0.0, T0, w0, dt0, acc0, 1.0, sig0, fx);
  ns = 1;
  double aK = 0.0, TK = T0, dtK = dt0, sigK[3] = {sig0[0], sig0[1], sig0[2]};
  double wK[BPMF_MAX_CHANNELS];
  memcpy(wK, w0, sizeof(wK));

  while (aK < 1.0 && ns < a->max_states) {
    double s = a->speed;
    double an = 0, Tn = 0, wn[BPMF_MAX_CHANNELS], dtn = 0, accn = 0, pn = 0;
    Samples Sn;
    std::vector<float> fxn;
    for (int sel = 0; sel < a->max_selections; ++sel) {
      TRY(bpmf_protocol_next_alpha(aK, sigK, a->kind, s, a->T_hot, a->T_cold,
                                   &an));
      state_of(an, a->kind, C, a->T_hot, a->T_cold, &Tn, wn);
      std::vector<double> logw(S.N);
      for (int64_t i = 0; i < S.N; ++i) {
        const double* cp = S.comps.data() + (size_t)i * (1 + C);
        logw[i] = reduced(cp, C, TK, wK) - reduced(cp, C, Tn, wn);
      }
      std::vector<int64_t> idx(K);
      TRY(bpmf_protocol_sir(logw.data(), S.N, K, seed, a->ligand_id, ns,
                            idx.data()));
      TRY(d.gather(S, idx, &seeds));
      TRY(d.run_state(Tn, wn, dtK, seeds.data(), &Sn, &fxn, &dtn, &accn));
      pn = d.pacc(S, TK, wK, Sn, Tn, wn);
      ++n_sel;
      const bool retry = pn < kPLow && sel + 1 < a->max_selections;
      const int outcome = retry ? 1 : (pn > kPHigh && ns > 1 ? 2 : 0);
      if (res->trace && n_tr < res->trace_cap) {
        double* tr = res->trace + (size_t)n_tr * BPMF_TRACE_FIELDS;
        tr[0] = aK;
        tr[1] = sigK[0];
        tr[2] = sigK[1];
        tr[3] = sigK[2];
        tr[4] = s;
        tr[5] = an;
        tr[6] = dtn;
        tr[7] = accn;
        tr[8] = pn;
        tr[9] = outcome;
        ++n_tr;
      }
      if (!retry) break;
      s *= kSpeedFactor;
    }
    double sn[3];
    TRY(bpmf_protocol_sigmas(Sn.comps.data(), Sn.N, C, an, a->kind, a->T_hot,
                             a->T_cold, sn));
    // above p_high the previous state adds nothing: the new one replaces it
    // (the end state alpha = 0 is kept)
    const int k = (pn > kPHigh && ns > 1) ? ns - 1 : ns;
    if (k < ns) ++res->n_removed;
    store(k, an, Tn, wn, dtn, accn, pn, sn, fxn);
    ns = k + 1;
    aK = an;
    TK = Tn;
    dtK = dtn;
    memcpy(wK, wn, sizeof(wK));
    memcpy(sigK, sn, sizeof(sigK));
    S = std::move(Sn);
  }
  res->n_states = ns;
  res->reached_target = aK >= 1.0 ? 1 : 0;
  res->n_selections = n_sel;
  res->n_runs = d.n_runs;
  res->n_trace = n_tr;
  return BPMF_OK;
}
