// Host plan and C ABI of the ESP reciprocal-space library (see include/esp.h).
//
// Plan-time work is FP64 on the host: parameter selection (paper Sec. 5.1),
// the PSWF of the split and of the window (App. A.1), the per-subinterval
// window polynomials (Sec. 4.3), Chebyshev fits of psi and x psi' for the
// scaling (Sec. 4.3, "polynomial approximation" of the Fourier kernel), the
// deconvolution tables 1/w_hat^2 (Sec. 4.2) and the FFT factorisations.  All
// device memory is allocated here; the per-step calls only enqueue kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/esp.h"
#include "esp_device.h"
#include "esp_internal.h"
#include "pswf.h"

using namespace espx;

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

struct Resolved {
  int precision = ESP_FP32;
  int64_t n = 0;
  double h[9], hinv[9], V = 0;
  double tol = 0, delta = 0, rc = 0.9, c_split = 0, c_spread = 0, sigma = 1.07, coulomb_k = 1;
  int P = 0, M[3] = {0, 0, 0}, T[3] = {0, 0, 0}, nt[3] = {0, 0, 0}, ntiles = 0;
  int params_source = ESP_ANALYTIC;
  int coupling = ESP_ISO;
  double window_tol = 0;
  int gather = ESP_GATHER_AUTO;
  int force = ESP_FORCE_AD;
  int local = 0;
  int fft_split = 0;
  int spread_accum = ESP_SPREAD_AUTO;
  int deterministic = 0;
  double pred[4] = {0, 0, 0, 0};
  double pred_cost = 0;
};

bool smooth235(int m) {
  if (m < 1) return false;
  for (int p : {2, 3, 5})
    while (m % p == 0) m /= p;
  return m == 1;
}

int next_smooth(int m) {
  while (!smooth235(m)) ++m;
  return m;
}

bool invert3(const double* h, double* inv, double* det) {
  const double a = h[0], b = h[1], c = h[2], d = h[3], e = h[4], f = h[5], g = h[6], k = h[7], l = h[8];
  const double A = e * l - f * k, B = -(d * l - f * g), C = d * k - e * g;
  const double D = a * A + b * B + c * C;
  *det = D;
  if (!std::isfinite(D) || D <= 0) return false;
  inv[0] = A / D;
  inv[1] = -(b * l - c * k) / D;
  inv[2] = (b * f - c * e) / D;
  inv[3] = B / D;
  inv[4] = (a * l - c * g) / D;
  inv[5] = -(a * f - c * d) / D;
  inv[6] = C / D;
  inv[7] = -(a * k - b * g) / D;
  inv[8] = (a * e - b * d) / D;
  return true;
}

double col_norm(const double* h, int j) {
  return std::sqrt(h[j] * h[j] + h[3 + j] * h[3 + j] + h[6 + j] * h[6 + j]);
}

// distance between the faces spanned by the other two cell vectors
double perp_width(const double* h, int j, double V) {
  const int a = (j + 1) % 3, b = (j + 2) % 3;
  const double u[3] = {h[a], h[3 + a], h[6 + a]}, v[3] = {h[b], h[3 + b], h[6 + b]};
  const double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2], cz = u[0] * v[1] - u[1] * v[0];
  return V / std::sqrt(cx * cx + cy * cy + cz * cz);
}

int grid_rule(const double* h, int d, double c, double rc, double sigma) {
  return static_cast<int>(std::ceil(sigma * col_norm(h, d) * c / (M_PI * rc) - 1e-9));
}

esp_status check_box(const double* h, double rc, double* hinv, double* V, std::string& err) {
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(h[i])) {
      err = "cell matrix has a non-finite entry";
      return ESP_EBOX;
    }
  if (!invert3(h, hinv, V)) {
    err = "cell matrix must have a positive determinant";
    return ESP_EBOX;
  }
  double wmin = 1e300;
  for (int j = 0; j < 3; ++j) wmin = std::min(wmin, perp_width(h, j, *V));
  if (!(rc > 0) || rc >= 0.5 * wmin) {
    char b[160];
    std::snprintf(b, sizeof b, "rc = %g must be positive and below half the smallest cell width (%g)", rc,
                  0.5 * wmin);
    err = b;
    return ESP_ECUTOFF;
  }
  return ESP_OK;
}

// ---- learned parameter proposer -------------------------------------------
}  // namespace
namespace espx {
esp_status mlp_predict_host(esp_mlp_t* p, const float* xh, int64_t B, float* yh);
int mlp_dim(const esp_mlp_t* p, int which);
}  // namespace espx
namespace {
struct ProposerState {
  bool set = false;
  esp_proposer cfg{};
  std::vector<double> deltas, cs;   // candidate Delta grid and c(Delta)
};
ProposerState g_prop;
std::mutex g_prop_mu;

constexpr double kSigmas[] = {0.85, 0.9, 0.95, 1.0, 1.07, 1.15, 1.22, 1.3};

struct Proposal {
  double delta, c, sigma, cost;
  int P, M[3];
  double pred[4];
};

// Score the candidate grid with the registered MLP (on the GPU) and return the
// cheapest candidate predicted to meet tol; false if none does.
// Score the candidate grid (plus the analytic choice) with the registered
// MLP on the GPU.  Returns 1 with the cheapest candidate predicted to meet
// tol, 2 with the candidate of smallest predicted excess when none does, and
// 0 (err set) when no proposer is usable.
int propose(const double* h, int64_t n, double tol, int coupling, double rc, double V, double sigma_rule,
            Proposal& best, std::string& err) {
  std::lock_guard<std::mutex> lock(g_prop_mu);
  if (!g_prop.set) {
    err = "no proposer registered";
    return 0;
  }
  const esp_proposer& cfg = g_prop.cfg;
  constexpr int NF = ESP_PROPOSER_FEATURES;
  const double fdens = std::log10(static_cast<double>(n) / V);
  std::vector<Proposal> cand;
  std::vector<float> feat;
  auto add = [&](double delta, double c, int P, double sg) {
    Proposal pr{};
    pr.delta = delta;
    pr.c = c;
    pr.sigma = sg;
    pr.P = P;
    for (int d = 0; d < 3; ++d) pr.M[d] = next_smooth(std::max({grid_rule(h, d, c, rc, sg), P, 2}));
    const double f[NF] = {std::log10(delta), double(P), sg, fdens};
    for (int j = 0; j < NF; ++j) feat.push_back(static_cast<float>((f[j] - cfg.in_mean[j]) / cfg.in_std[j]));
    cand.push_back(pr);
  };
  for (size_t k = 0; k < g_prop.deltas.size(); ++k) {
    const double delta = g_prop.deltas[k];
    const int D = static_cast<int>(std::ceil(-std::log10(delta) - 1e-9));
    for (int P = std::max(3, D - 1); P <= std::min(kMaxP, D + 2); ++P)
      for (double sg : kSigmas) add(delta, g_prop.cs[k], P, sg);
  }
  {
    // the analytic rule's own choice competes on the same terms
    const double delta = coupling == ESP_FLEX ? tol / 5 : tol;
    const int P = std::min(kMaxP, static_cast<int>(std::ceil(-std::log10(delta) - 1e-9)) + 1);
    add(delta, c_from_delta(delta), P, sigma_rule);
  }
  const int64_t B = static_cast<int64_t>(cand.size());
  std::vector<float> y(B * 4);
  if (mlp_predict_host(const_cast<esp_mlp_t*>(cfg.mlp), feat.data(), B, y.data()) != ESP_OK) {
    err = "proposer evaluation failed on the device";
    return 0;
  }
  double lim[4];
  for (int j = 0; j < 4; ++j) lim[j] = std::log10(tol) - cfg.margin[j];
  int found = 0;
  double best_excess = 0;
  for (int64_t b = 0; b < B; ++b) {
    Proposal& pr = cand[b];
    for (int j = 0; j < 4; ++j) pr.pred[j] = y[b * 4 + j] * cfg.out_std[j] + cfg.out_mean[j];
    double excess = std::max({pr.pred[0] - lim[0], pr.pred[1] - lim[1], pr.pred[3] - lim[3]});
    if (coupling == ESP_FLEX) excess = std::max(excess, pr.pred[2] - lim[2]);
    const double G = double(pr.M[0]) * pr.M[1] * pr.M[2];
    pr.cost = cfg.cost[0] + cfg.cost[1] * n * double(pr.P) * pr.P * pr.P + cfg.cost[2] * G * std::log2(G) +
              cfg.cost[3] * n + cfg.cost[4] * G;
    if (excess <= 0) {
      if (found != 1 || pr.cost < best.cost) {
        best = pr;
        found = 1;
      }
    } else if (found != 1 && (found == 0 || excess < best_excess)) {
      best = pr;
      best_excess = excess;
      found = 2;
    }
  }
  if (found == 2) {
    char b[160];
    std::snprintf(b, sizeof b, "no candidate is predicted to meet tol; the most accurate one is %.2f decades short",
                  best_excess);
    err = b;
  }
  return found;
}

void choose_tiles(Resolved& r, int tile) {
  int T = tile;
  if (T <= 0) {
    // smallest tile edge in {4,...,12} giving at most ~4 tiles per CU and
    // at least 256 tiles, else the largest tile that keeps 256 tiles
    T = 6;
    const int cand[] = {12, 10, 8, 6, 5, 4};
    for (int t : cand) {
      long nt = 1;
      for (int d = 0; d < 3; ++d) nt *= (r.M[d] + std::min(t, r.M[d]) - 1) / std::min(t, r.M[d]);
      T = t;
      if (nt >= 256) break;
    }
  }
  // the scatter pass keeps all tile offsets in LDS: at most 32768 tiles
  for (;; ++T) {
    r.ntiles = 1;
    for (int d = 0; d < 3; ++d) {
      r.T[d] = std::min(T, r.M[d]);
      r.nt[d] = (r.M[d] + r.T[d] - 1) / r.T[d];
      r.ntiles *= r.nt[d];
    }
    if (r.ntiles <= 32768) break;
  }
}

esp_status resolve(const double* h, int64_t n, double tol, const esp_opts* o, Resolved& r, std::string& err) {
  esp_opts def;
  esp_opts_default(&def);
  if (!o) o = &def;
  if (!h) {
    err = "null cell";
    return ESP_EINVAL;
  }
  if (n < 1 || n > (int64_t(1) << 30)) {
    err = "n must be in [1, 2^30]";
    return ESP_EINVAL;
  }
  if (!(tol >= 1e-12 && tol < 0.1)) {
    err = "tol must be in [1e-12, 1e-1)";
    return ESP_EINVAL;
  }
  if (o->precision != ESP_FP32 && o->precision != ESP_FP64) {
    err = "precision must be ESP_FP32 or ESP_FP64";
    return ESP_EINVAL;
  }
  if (o->coupling < ESP_ISO || o->coupling > ESP_FLEX) {
    err = "coupling must be ESP_ISO .. ESP_FLEX";
    return ESP_EINVAL;
  }
  r.precision = o->precision;
  r.n = n;
  r.tol = tol;
  r.rc = o->rc > 0 ? o->rc : 0.9;
  r.sigma = o->grid_sigma > 0 ? o->grid_sigma : 1.07;
  r.coulomb_k = o->coulomb_k != 0 ? o->coulomb_k : 1.0;
  r.coupling = o->coupling;
  if (o->window_tol < 0 || o->window_tol >= 1e-2) {
    err = "window_tol must be 0 (automatic) or in (0, 1e-2)";
    return ESP_EINVAL;
  }
  r.window_tol = o->window_tol;
  if (o->gather < ESP_GATHER_AUTO || o->gather > ESP_GATHER_LANE) {
    err = "gather must be ESP_GATHER_AUTO, ESP_GATHER_PARTICLE, ESP_GATHER_TILE or ESP_GATHER_LANE";
    return ESP_EINVAL;
  }
  r.gather = o->gather;
  if (o->force != ESP_FORCE_AD && o->force != ESP_FORCE_IK) {
    err = "force must be ESP_FORCE_AD or ESP_FORCE_IK";
    return ESP_EINVAL;
  }
  r.force = o->force;
  r.local = o->local_virial ? 1 : 0;
  r.fft_split = o->fft_split ? 1 : 0;
  if (o->spread_accum < ESP_SPREAD_AUTO || o->spread_accum > ESP_SPREAD_FP64) {
    err = "spread_accum must be ESP_SPREAD_AUTO, ESP_SPREAD_FIXED or ESP_SPREAD_FP64";
    return ESP_EINVAL;
  }
  r.spread_accum = o->spread_accum;
  r.deterministic = o->deterministic ? 1 : 0;
  std::memcpy(r.h, h, 9 * sizeof(double));
  esp_status st = check_box(h, r.rc, r.hinv, &r.V, err);
  if (st != ESP_OK) return st;

  esp_status warn = ESP_OK;
  int src = o->params;
  if (src == ESP_LEARNED) {
    Proposal pr{};
    std::string why;
    const int got = propose(h, n, tol, o->coupling, r.rc, r.V, r.sigma, pr, why);
    if (got) {
      r.delta = pr.delta;
      r.c_split = r.c_spread = pr.c;
      r.P = pr.P;
      r.sigma = pr.sigma;
      for (int d = 0; d < 3; ++d) r.M[d] = pr.M[d];
      for (int j = 0; j < 4; ++j) r.pred[j] = pr.pred[j];
      r.pred_cost = pr.cost;
      r.params_source = ESP_LEARNED;
      if (got == 2) {
        err = "learned parameters: " + why;
        warn = ESP_WARN_FALLBACK;
      }
    } else {
      err = "learned parameters unavailable (" + why + "); analytic rule used";
      warn = ESP_WARN_FALLBACK;
      src = ESP_ANALYTIC;
    }
  }
  if (src == ESP_ANALYTIC) {
    r.delta = o->coupling == ESP_FLEX ? tol / 5.0 : tol;
    r.c_split = r.c_spread = c_from_delta(r.delta);
    r.P = std::min(kMaxP, static_cast<int>(std::ceil(-std::log10(r.delta) - 1e-9)) + 1);
    r.P = std::max(r.P, 2);
    for (int d = 0; d < 3; ++d) r.M[d] = next_smooth(std::max({grid_rule(h, d, r.c_split, r.rc, r.sigma), r.P, 2}));
    r.params_source = ESP_ANALYTIC;
  } else if (src == ESP_EXPLICIT) {
    if (!(o->c_split > 0 && o->c_spread > 0) || o->P < 2 || o->P > kMaxP) {
      err = "explicit parameters need c_split > 0, c_spread > 0 and 2 <= P <= 12";
      return ESP_EINVAL;
    }
    r.c_split = o->c_split;
    r.c_spread = o->c_spread;
    r.P = o->P;
    r.delta = tol;
    for (int d = 0; d < 3; ++d) {
      if (o->M[d] < r.P || o->M[d] < 2 || !smooth235(o->M[d])) {
        err = "explicit grid sizes must be 2,3,5-smooth and at least P";
        return ESP_EINVAL;
      }
      r.M[d] = o->M[d];
    }
    r.params_source = ESP_EXPLICIT;
  } else if (src != ESP_LEARNED) {
    err = "params must be ESP_ANALYTIC, ESP_EXPLICIT or ESP_LEARNED";
    return ESP_EINVAL;
  }
  if (o->tile < 0 || o->tile > 32) {
    err = "tile must be 0 (automatic) or in [1, 32]";
    return ESP_EINVAL;
  }
  choose_tiles(r, o->tile);
  if (r.precision == ESP_FP32 && tol < kFp32TolFloor && warn == ESP_OK) {
    // FP32 spreading, transforms and gather carry relative rounding errors of
    // a few 1e-7 (energy, RMS force) up to ~3e-6 (a small virial component)
    // at identical parameters: a tighter tol is planned for, but the result
    // is not expected to meet it
    char b[160];
    std::snprintf(b, sizeof b, "tol %.3g is below the FP32 floor %.0e: FP32 rounding may exceed it (use ESP_FP64)",
                  tol, kFp32TolFloor);
    err = b;
    warn = ESP_WARN_PRECISION;
  }
  return warn;
}

// radices for a 2,3,5-smooth length: 8s, 6s, 4s, then a 2, then 3s and 5s
void factor(int n, FftLen& f) {
  f.n = n;
  f.nstage = 0;
  int m = n;
  while (m % 8 == 0) { f.rad[f.nstage++] = 8; m /= 8; }
  while (m % 6 == 0) { f.rad[f.nstage++] = 6; m /= 6; }
  while (m % 4 == 0) { f.rad[f.nstage++] = 4; m /= 4; }
  while (m % 2 == 0) { f.rad[f.nstage++] = 2; m /= 2; }
  while (m % 3 == 0) { f.rad[f.nstage++] = 3; m /= 3; }
  while (m % 5 == 0) { f.rad[f.nstage++] = 5; m /= 5; }
  if (n == 1) { f.rad[f.nstage++] = 1; }
}

}  // namespace

enum StageId { ST_BIN, ST_SCATTER, ST_SPREAD, ST_FFT_XY, ST_FFT_Z, ST_FFT_XY_INV, ST_GATHER, ST_REAL, ST_COUNT };
const char* kStageNames[ST_COUNT] = {"bin", "scatter", "spread", "fft_xy", "fft_z", "fft_xy_inv", "gather",
                                     "real"};

// Optional per-stage timing with HIP events recorded on the plan's stream.
struct Profiler {
  unsigned mask = 0;
  int cap = 0;
  int stride = 1;                // time every stride-th launch of a stage
  long long seen[ST_COUNT] = {};
  std::vector<hipEvent_t> ev[ST_COUNT];
  int used[ST_COUNT] = {};
  double ms[ST_COUNT] = {};
  long long cnt[ST_COUNT] = {};
  void release() {
    for (auto& v : ev) {
      for (hipEvent_t e : v) (void)hipEventDestroy(e);
      v.clear();
    }
  }
};

struct esp_plan_s {
  Resolved r;
  Profiler prof;
  std::unique_ptr<Pswf> split, spread;
  int nw = 0, nw_fitted = 0, nker = 0, nseg = 0;
  double A = 0, self_coef = 0, Ic = 0;
  hipStream_t stream = nullptr;
  // esp_coulomb: the real-space part runs on its own stream (made on first
  // use, default priority), forked from and joined back to `stream` by events
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::vector<void*> allocs;
  // device memory from a caller-provided region instead of hipMalloc (the
  // allocation-free entry point): bump allocation, nothing freed by the plan;
  // such a plan holds only what the force path needs
  unsigned char* arena = nullptr;
  size_t arena_cap = 0, arena_used = 0;
  DevPlan<float> d32{};
  DevPlan<double> d64{};
  std::string err;
  ~esp_plan_s() {
    prof.release();
    if (side) (void)hipStreamSynchronize(side);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (side) (void)hipStreamDestroy(side);
    for (void* p : allocs) (void)hipFree(p);
  }
};

namespace espx {
LaunchTiming& launch_timing() {
  thread_local LaunchTiming t;
  return t;
}
}  // namespace espx

namespace {

template <typename R>
DevPlan<R>& dev(esp_plan_t* p);
template <>
DevPlan<float>& dev<float>(esp_plan_t* p) { return p->d32; }
template <>
DevPlan<double>& dev<double>(esp_plan_t* p) { return p->d64; }

esp_status hip_fail(esp_plan_t* p, hipError_t e, const char* what) {
  p->err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? ESP_ENOMEM : ESP_EDEVICE;
}

template <typename T>
esp_status dalloc(esp_plan_t* p, T** ptr, size_t count) {
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  if (p->arena) {
    const size_t off = (p->arena_used + 255) & ~static_cast<size_t>(255);
    if (off + bytes > p->arena_cap) {
      char b[200];
      std::snprintf(b, sizeof b, "the plan needs more than the %zu bytes of its preallocated device region",
                    p->arena_cap);
      p->err = b;
      *ptr = nullptr;
      return ESP_ENOMEM;
    }
    p->arena_used = off + bytes;
    *ptr = reinterpret_cast<T*>(p->arena + off);
    return ESP_OK;
  }
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) return hip_fail(p, e, "hipMalloc");
  p->allocs.push_back(q);
  *ptr = static_cast<T*>(q);
  return ESP_OK;
}

FinalConsts final_consts(const esp_plan_t* p) {
  FinalConsts c;
  c.inv2V = 0.5 / p->r.V;
  c.self_coef = p->self_coef;
  c.bg_coef = kTwoPi * p->Ic / p->r.V;
  c.coulomb_k = p->r.coulomb_k;
  return c;
}

// Box-dependent fields of the device plan.
template <typename R>
void set_box_fields(esp_plan_t* p, DevPlan<R>& d) {
  const Resolved& r = p->r;
  for (int i = 0; i < 9; ++i) {
    d.hinv[i] = r.hinv[i];
    d.hinv_hi[i] = static_cast<float>(r.hinv[i]);
    d.hinv_lo[i] = static_cast<float>(r.hinv[i] - static_cast<double>(d.hinv_hi[i]));
  }
  for (int a = 0; a < 3; ++a)
    for (int m = 0; m < 3; ++m) {
      d.B[3 * a + m] = static_cast<R>(kTwoPi * r.hinv[3 * m + a]);
      d.G[3 * a + m] = static_cast<R>(-r.hinv[3 * m + a] * r.M[m]);
    }
  d.inv_vol = static_cast<R>(1.0 / r.V);
  d.fin = final_consts(p);
  // real-space cells: floor(w_d / rc) per dimension (at least 2, since rc is
  // below half of every width), merged along the most divided dimension while
  // there are more than kMaxCells
  int cn[3];
  for (int k = 0; k < 3; ++k) cn[k] = std::max(2, static_cast<int>(perp_width(r.h, k, r.V) / r.rc));
  while (static_cast<int64_t>(cn[0]) * cn[1] * cn[2] > kMaxCells) {
    const int k = cn[0] >= cn[1] && cn[0] >= cn[2] ? 0 : (cn[1] >= cn[2] ? 1 : 2);
    --cn[k];
  }
  d.cn1 = cn[0];
  d.cn2 = cn[1];
  d.cn3 = cn[2];
  for (int i = 0; i < 9; ++i) d.hmat[i] = static_cast<R>(r.h[i]);
  {
    auto g = [&](int a, int b) { return r.h[a] * r.h[b] + r.h[3 + a] * r.h[3 + b] + r.h[6 + a] * r.h[6 + b]; };
    const double sc = sizeof(R) == 4 ? std::ldexp(1.0, -64) : 1.0;
    const double gm[6] = {g(0, 0), g(1, 1), g(2, 2), 2 * g(0, 1), 2 * g(0, 2), 2 * g(1, 2)};
    for (int k = 0; k < 6; ++k) d.gmet[k] = static_cast<R>(gm[k] * sc);
  }
  d.rc2 = static_cast<R>(r.rc * r.rc);
  d.inv_rc = static_cast<R>(1.0 / r.rc);
}

// Per-subinterval window polynomials (Sec. 4.3): polynomial p approximates
// W(tau + (P-1)/2 - p) = psi((tau + (P-1)/2 - p) / omega), tau in [-1/2, 1/2],
// omega = P/2, by Chebyshev interpolation converted to monomials in tau.  The
// smallest degree meeting eps (values) and 4 eps (derivatives), relative to
// psi(0), is chosen, then padded with zeros to the kernel class 8, 12 or 16.
// Table layout: coef[j * P + p] multiplies tau^j in polynomial p.
int fit_window(esp_plan_t* p, double eps, std::vector<double>& coef, int* fitted) {
  const Pswf& ps = *p->spread;
  const int P = p->r.P;
  const double omega = 0.5 * P;
  std::vector<std::vector<double>> best;
  int deg = 3;
  for (; deg <= kMaxWinDeg; ++deg) {
    best.assign(P, {});
    double maxerr = 0, maxderr = 0;
    for (int q = 0; q < P; ++q) {
      const double shift = 0.5 * (P - 1) - q;
      auto f = [&](double tau) { return ps.psi((tau + shift) / omega); };
      best[q] = fit_monomial(f, -0.5, 0.5, deg);
      const std::vector<double>& c = best[q];
      for (int s = 0; s <= 64; ++s) {
        const double tau = -0.5 + s / 64.0;
        double v = 0, dv = 0;
        for (int j = deg; j >= 0; --j) {
          dv = dv * tau + v;
          v = v * tau + c[j];
        }
        maxerr = std::max(maxerr, std::fabs(v - f(tau)));
        maxderr = std::max(maxderr, std::fabs(dv - ps.dpsi((tau + shift) / omega) / omega));
      }
    }
    if (maxerr <= eps * ps.psi0() && maxderr <= 4 * eps * ps.psi0()) break;
  }
  deg = std::min(deg, kMaxWinDeg);
  *fitted = deg;
  const int cls = deg <= 8 ? 8 : (deg <= 12 ? 12 : 16);
  coef.assign(static_cast<size_t>(cls + 1) * P, 0.0);
  for (int q = 0; q < P; ++q)
    for (int j = 0; j <= deg; ++j) coef[static_cast<size_t>(j) * P + q] = best[q][j];
  return cls;
}

// Chebyshev fits of the two kernel functions in z = 2y - 1, to 1e-13 psi(0)
// for FP64 plans and to 1e-9 psi(0) for FP32 plans (far below FP32 rounding;
// two to four degrees fewer).
int fit_kernel(esp_plan_t* p, std::vector<double>& cf, std::vector<double>& cg) {
  const Pswf& ps = *p->split;
  const double rel = p->r.precision == ESP_FP32 ? 1e-9 : 1e-13;
  auto f = [&](double z) {
    const double y = 0.5 * (z + 1.0);
    return ps.psi(std::sqrt(y));
  };
  auto g = [&](double z) {
    const double y = 0.5 * (z + 1.0), x = std::sqrt(y);
    return x * ps.dpsi(x);
  };
  for (int deg = 8; deg <= kMaxKerDeg; deg += 2) {
    cf = fit_chebyshev(f, deg);
    cg = fit_chebyshev(g, deg);
    double err = 0;
    for (int s = 0; s <= 200; ++s) {
      const double z = -1.0 + s / 100.0;
      double b1 = 0, b2 = 0, c1 = 0, c2 = 0;
      for (int k = deg; k >= 1; --k) {
        double b0 = 2 * z * b1 - b2 + cf[k];
        b2 = b1; b1 = b0;
        double e0 = 2 * z * c1 - c2 + cg[k];
        c2 = c1; c1 = e0;
      }
      err = std::max(err, std::fabs(z * b1 - b2 + cf[0] - f(z)));
      err = std::max(err, std::fabs(z * c1 - c2 + cg[0] - g(z)));
    }
    if (err <= rel * ps.psi0()) return deg;
  }
  return kMaxKerDeg;
}

// Near-part split functions (Sec. 3.1, eq. UN and eq. mathFN) of x = r / rc
// as piecewise polynomials of degree kRealDeg on nseg equal segments of
// [0, 1]: the fewest segments (a power of two) whose fits stay within eps of
// both functions; layout seg x {1 - phi0, F_N} x (deg + 1) coefficients of
// t = nseg x - seg - 1/2 in [-1/2, 1/2].
int fit_near(esp_plan_t* p, int deg, double eps, int max_seg, std::vector<double>& coef) {
  const Pswf& ps = *p->split;
  const double C0 = ps.C0();
  auto gN = [&](double x) { return 1.0 - ps.int_psi(x) / C0; };
  auto gF = [&](double x) { return 1.0 - ps.int_psi(x) / C0 + x * ps.psi(x) / C0; };
  int nseg = 8;
  for (;; nseg *= 2) {
    coef.assign(static_cast<size_t>(nseg) * 2 * (deg + 1), 0.0);
    double err = 0;
    for (int sgm = 0; sgm < nseg && (err <= eps || nseg >= max_seg); ++sgm)
      for (int fn = 0; fn < 2; ++fn) {
        auto g = [&](double t) {
          const double x = std::min(1.0, std::max(0.0, (sgm + 0.5 + t) / nseg));
          return fn == 0 ? gN(x) : gF(x);
        };
        const std::vector<double> m = fit_monomial(g, -0.5, 0.5, deg);
        for (int k = 0; k <= deg; ++k) coef[(static_cast<size_t>(sgm) * 2 + fn) * (deg + 1) + k] = m[k];
        for (int s2 = 0; s2 <= 16; ++s2) {
          const double t = -0.5 + s2 / 16.0;
          double v = 0;
          for (int k = deg; k >= 0; --k) v = v * t + m[k];
          err = std::max(err, std::fabs(v - g(t)));
        }
      }
    if (err <= eps || nseg >= max_seg) return nseg;
  }
}

// Binning blocks: 256, 512 or 1,024 particles per block of kBinThreads
// threads, more where tiles are many, since every block clears and reads the
// whole tile histogram (10^6 slab, 3,328 tiles: that work was ~70 % of the
// binning kernel's VALU issue at 256 particles per block).
template <typename R>
void set_bin_blocks(DevPlan<R>& d) {
  d.binppt = d.ntiles >= 2048 ? 4 : (d.ntiles >= 1024 ? 2 : 1);
  const int64_t per = static_cast<int64_t>(kBinThreads) * d.binppt;
  d.nbin = static_cast<int>((d.n + per - 1) / per);
}

// partial-sum slots for any block size set_bin_blocks picks
size_t bin_blocks_max(int64_t n) { return static_cast<size_t>((n + kBinThreads - 1) / kBinThreads); }

template <typename R>
esp_status build_device(esp_plan_t* p) {
  const Resolved& r = p->r;
  DevPlan<R>& d = dev<R>(p);
  d = DevPlan<R>{};
  d.n = r.n;
  d.M1 = r.M[0];
  d.M2 = r.M[1];
  d.M3 = r.M[2];
  d.H = r.M[0] / 2 + 1;
  d.P = r.P;
  d.T1 = r.T[0]; d.T2 = r.T[1]; d.T3 = r.T[2];
  d.nt1 = r.nt[0]; d.nt2 = r.nt[1]; d.nt3 = r.nt[2];
  d.ntiles = r.ntiles;
  // columns per z-pass workgroup: ~256 elements, at least 16 columns
  // (128-byte rows of the spectrum) for long columns (10^6 slab, 160 x 160 x
  // 128: 34.0 us with 8 columns, 31.5 with 16, 39.9 with 32)
  {
    const int per = 256 / std::max(1, d.M3);
    d.cz = std::max(1, std::min(d.H, per >= 6 ? per : 16));
  }
  d.nzblk = ((d.H + d.cz - 1) / d.cz) * d.M2;
  set_bin_blocks(d);
  d.ik = r.force == ESP_FORCE_IK ? 1 : 0;
  d.local = r.local;
  d.ncomp = d.local ? 6 : (d.ik ? 3 : 1);
  d.kcut2 = static_cast<R>((r.c_split / r.rc) * (r.c_split / r.rc));
  d.ysc = static_cast<R>((r.rc / r.c_split) * (r.rc / r.c_split));
  d.A = static_cast<R>(p->A);
  d.coulomb_k = static_cast<R>(r.coulomb_k);
  set_box_fields(p, d);

  // ---- tables ---------------------------------------------------------
  std::vector<double> win;
  double eps = r.precision == ESP_FP32 ? std::max(1e-2 * r.delta, 2e-8) : 1e-3 * r.delta;
  if (r.window_tol > 0) eps = r.window_tol;
  int fitted = 0;
  p->nw = fit_window(p, std::min(eps, 1e-4), win, &fitted);
  p->nw_fitted = fitted;
  {
    // largest |w_q(tau)| of the fitted polynomials over tau in [-1/2, 1/2],
    // sampled, with 1% added (the values lie below psi(0); the bound only
    // sets the fixed-point scale, which keeps another factor of two spare)
    double wm = 0;
    for (int q = 0; q < r.P; ++q)
      for (int s = 0; s <= 256; ++s) {
        const double tau = -0.5 + s / 256.0;
        double v = 0;
        for (int j = p->nw; j >= 0; --j) v = v * tau + win[static_cast<size_t>(j) * r.P + q];
        wm = std::max(wm, std::fabs(v));
      }
    d.wmax = static_cast<float>(1.01 * wm);
    d.wmax3 = static_cast<float>(1.01 * wm * wm * wm);
  }
  std::vector<double> cf, cg;
  p->nker = fit_kernel(p, cf, cg);
  d.nw = p->nw;
  d.nker = (p->nker + 3) / 4 * 4;
  std::vector<double> iw[3];
  const Pswf& sp = *p->spread;
  const double omega = 0.5 * r.P;
  for (int k = 0; k < 3; ++k) {
    const int M = r.M[k];
    iw[k].resize(M);
    for (int m = 0; m < M; ++m) {
      const int ms = m <= (M - 1) / 2 ? m : m - M;
      const double kappa = kTwoPi * ms / M;
      const double wh = omega * sp.lambda0() * sp.psi(omega * kappa / r.c_spread);
      iw[k][m] = 1.0 / (wh * wh);
    }
  }
  for (int k = 0; k < 3; ++k) factor(r.M[k], (k == 0 ? d.f1 : k == 1 ? d.f2 : d.f3));
  d.f1.tw = 0;
  d.f2.tw = r.M[0];
  d.f3.tw = r.M[0] + r.M[1];
  const int ntw = r.M[0] + r.M[1] + r.M[2];
  std::vector<Cplx<R>> tw(ntw);
  for (int k = 0; k < 3; ++k) {
    const int M = r.M[k], off = (k == 0 ? d.f1.tw : k == 1 ? d.f2.tw : d.f3.tw);
    for (int j = 0; j < M; ++j)
      tw[off + j] = {static_cast<R>(std::cos(kTwoPi * j / M)), static_cast<R>(-std::sin(kTwoPi * j / M))};
  }
  // pack all real tables into one allocation
  std::vector<R> tab;
  auto push = [&](const std::vector<double>& v) {
    size_t off = tab.size();
    for (double x : v) tab.push_back(static_cast<R>(x));
    while (tab.size() % 4) tab.push_back(R(0));
    return off;
  };
  std::vector<double> near;
  int max_seg = 8;                  // segment tables of at most 40 KiB of LDS
  while (2 * max_seg * 2 * (kRealDeg<R> + 1) * static_cast<int>(sizeof(R)) <= 40 * 1024) max_seg *= 2;
  p->nseg = fit_near(p, kRealDeg<R>, r.precision == ESP_FP32 ? 2e-8 : 1e-14, max_seg, near);
  d.nrs = p->nseg;
  std::vector<double> kfg(2 * static_cast<size_t>(d.nker + 1), 0.0);   // (f_k, g_k) pairs, zero past the fit
  for (int k = 0; k <= p->nker; ++k) {
    kfg[2 * k] = cf[k];
    kfg[2 * k + 1] = cg[k];
  }
  const size_t o_win = push(win), o_kfg = push(kfg);
  const size_t o_i1 = push(iw[0]), o_i2 = push(iw[1]), o_i3 = push(iw[2]), o_near = push(near);
  R* dtab;
  Cplx<R>* dtw;
  esp_status st;
  if ((st = dalloc(p, &dtab, tab.size())) != ESP_OK) return st;
  if ((st = dalloc(p, &dtw, tw.size())) != ESP_OK) return st;
  hipError_t e = hipSuccess;
  d.win = dtab + o_win;
  d.kerfg = reinterpret_cast<const Cplx<R>*>(dtab + o_kfg);   // offsets are multiples of 4 reals
  d.iw1 = dtab + o_i1;
  d.iw2 = dtab + o_i2;
  d.iw3 = dtab + o_i3;
  d.rsN = dtab + o_near;
  d.tw = dtw;

  // ---- LDS limits --------------------------------------------------------
  int dev_id = 0, maxlds = 65536;
  if (hipGetDevice(&dev_id) == hipSuccess)
    (void)hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev_id);
  // xy transforms: one workgroup per plane when the plane fits in LDS, else
  // separate x and y passes with as many row pairs / columns per workgroup
  // (up to 8) as fit (10^6 slab, 160 x 160 planes: forward and inverse xy
  // 28.8 / 31.8 us with 8 and 8, 33.6 / 36.2 with 16 and 16, 55.9 / 59.8
  // with 32 row pairs)
  d.xy_split = r.fft_split || lds_fft_xy(d) > static_cast<size_t>(maxlds) ? 1 : 0;
  // fixed-point spreading: FP32 terms are integer products (two VALU
  // instructions), faster than the FP64 adds on every shape measured (729
  // tiles of ~40 particles to 1,296 of ~770).  FP64 terms need the long
  // f64 -> i64 conversion, which pays only where the LDS atomics bound the
  // kernel: crowded tiles, and enough of them to keep every CU busy.
  d.spread_fixed = r.spread_accum == ESP_SPREAD_FIXED ||
                   (r.spread_accum == ESP_SPREAD_AUTO &&
                    (r.precision == ESP_FP32 || (r.ntiles >= kSpreadFixedMinTiles &&
                                                 r.n >= static_cast<int64_t>(kSpreadFixedMin) * r.ntiles)));
  // deterministic FP32 plans: fixed-point tiles add their integers into an
  // int64 grid (results that repeat bit for bit); other plans keep the R grid
  d.grid_fixed = r.deterministic && r.precision == ESP_FP32 && d.spread_fixed ? 1 : 0;
  d.xpairs = d.ycols = 8;
  while (d.xpairs > 1 && lds_fft_x(d, d.xpairs) > static_cast<size_t>(maxlds)) d.xpairs /= 2;
  while (d.ycols > 1 && lds_fft_y(d, d.ycols) > static_cast<size_t>(maxlds)) d.ycols /= 2;
  const size_t need_xy = d.xy_split ? std::max(lds_fft_x(d, d.xpairs), lds_fft_y(d, d.ycols)) : lds_fft_xy(d);
  const size_t need[3] = {need_xy, lds_fft_z(d), lds_spread(d)};
  const char* what[3] = {"xy-plane FFT", "z-column FFT", "spreading tile"};
  for (int k = 0; k < 3; ++k)
    if (need[k] > static_cast<size_t>(maxlds)) {
      char b[200];
      std::snprintf(b, sizeof b, "%s needs %zu bytes of LDS, the device allows %d (grid %dx%dx%d too large for this precision)",
                    what[k], need[k], maxlds, r.M[0], r.M[1], r.M[2]);
      p->err = b;
      return ESP_EINVAL;
    }

  // ---- buffers -----------------------------------------------------------
  const size_t G = static_cast<size_t>(r.M[0]) * r.M[1] * r.M[2];
  const size_t S = static_cast<size_t>(d.H) * r.M[1] * r.M[2];
  // counter copies: about kBinContention same-address atomics per counter at most
  {
    const double per = static_cast<double>(d.nbin) * std::min(kBinThreads * d.binppt, r.ntiles) / r.ntiles;
    d.nsub = std::max(1, std::min(kMaxCounterCopies, static_cast<int>(std::ceil(per / kBinContention))));
  }
  const size_t ncount = static_cast<size_t>(r.ntiles) * d.nsub;
  const bool want_near = !p->arena;   // a region plan serves the force path only
  if ((st = dalloc(p, &d.counts, ncount)) || (st = dalloc(p, &d.sbase, d.nsub > 1 ? ncount : 1)) ||
      (st = dalloc(p, &d.offsets, r.ntiles + 1)) ||
      (want_near && ((st = dalloc(p, &d.nr_counts, kMaxCells)) || (st = dalloc(p, &d.nr_offsets, kMaxCells + 1)) ||
                (st = dalloc(p, &d.nr_keys, r.n)) || (st = dalloc(p, &d.nr_ranks, r.n)) ||
                (st = dalloc(p, &d.nr_perm, r.n)) || (st = dalloc(p, &d.nr_tmp, r.n)) ||
                (st = dalloc(p, &d.nr_sorted, r.n)) ||
                (st = dalloc(p, &d.nr_qpart, bin_blocks_max(r.n) * 3)) ||
                (st = dalloc(p, &d.rpart, static_cast<size_t>(std::max(kMaxCells, 2 * kRealBlocks)) * kNumSums)) ||
                (st = dalloc(p, &d.fpart, static_cast<size_t>(kMaxRealSplit) * r.n * 3)) ||
                (st = dalloc(p, &d.facc, static_cast<size_t>(r.n) * 3)))) ||
      (st = dalloc(p, &d.keys, r.n)) || (st = dalloc(p, &d.ranks, r.n)) || (st = dalloc(p, &d.perm, r.n)) ||
      (st = dalloc(p, &d.tmp, r.n)) || (st = dalloc(p, &d.sorted, r.n)) || (st = dalloc(p, &d.rho, d.grid_fixed ? 1 : G)) ||
      (st = dalloc(p, &d.rhofix, d.grid_fixed ? G : 1)) || (st = dalloc(p, &d.gexp, 1)) ||
      (st = dalloc(p, &d.spec, S * d.ncomp)) || (st = dalloc(p, &d.phi, G * d.ncomp)) ||
      (st = dalloc(p, &d.zpart, static_cast<size_t>(d.nzblk) * kNumSums)) ||
      (st = dalloc(p, &d.qpart, bin_blocks_max(r.n) * 3)) || (st = dalloc(p, &d.flags, 4)))
    return st;
  d.bin_lds = r.ntiles <= 8192 ? 1 : 0;
  // dense tiles: stage each tile's potential box in LDS for the gather
  const size_t gather_base = ((p->nw + 1) * r.P + (256 / gather_lanes(r.P)) * 6 * r.P) * sizeof(R);
  const bool box_fits = gather_base + lds_gather_box(d) <= static_cast<size_t>(maxlds);
  const size_t lane_base = ((p->nw + 1) * r.P + 3) / 4 * 4 * sizeof(R);
  const bool lane_fits = lane_base + lds_gather_box(d) <= static_cast<size_t>(maxlds);
  if ((r.gather == ESP_GATHER_TILE && !box_fits) || (r.gather == ESP_GATHER_LANE && !lane_fits)) {
    p->err = "the tile-staged gather's potential box does not fit in LDS for this tile";
    return ESP_EINVAL;
  }
  // automatic choice: dense tiles (kTiledGatherMin+ particles on average)
  // stage their potential box and take one particle per lane (10^6 slab:
  // 72 us against 110 us for lane groups per particle and 272 us unstaged)
  const bool auto_tiled = r.gather == ESP_GATHER_AUTO && lane_fits &&
                          r.n >= static_cast<int64_t>(kTiledGatherMin) * r.ntiles;
  d.gather_lane = r.gather == ESP_GATHER_LANE || auto_tiled ? 1 : 0;
  d.gather_tiled = r.gather == ESP_GATHER_TILE || d.gather_lane ? 1 : 0;
  // the ik and virial gathers stage three component boxes per tile once
  // tiles hold kCompLaneMin+ particles on average and the boxes fit in LDS
  // (their per-particle form reads 3 or 6 grids at random: 10^6 slab 1.4 /
  // 2.4 ms); the virial takes two launches of three components
  d.comp_lane = 0;
  if (r.gather != ESP_GATHER_PARTICLE && r.n >= static_cast<int64_t>(kCompLaneMin) * r.ntiles &&
      lane_base + 3 * lds_gather_box(d) <= static_cast<size_t>(maxlds))
    d.comp_lane = 3;
  // tables: uploaded once every buffer has its place, so that a plan that
  // does not fit its region fails before it writes any device memory; the
  // copies are ordered on the plan's stream after earlier work there (a
  // region's previous user may still be reading its tables) and waited for
  // before the host copies go out of scope
  e = hipMemcpyAsync(dtab, tab.data(), tab.size() * sizeof(R), hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dtw, tw.data(), tw.size() * sizeof(Cplx<R>), hipMemcpyHostToDevice, p->stream);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(p->stream);
    return hip_fail(p, e, "table upload");
  }
  if (p->arena) {
    // the region holds whatever its previous user left: clear, stream-ordered
    // with fill kernels, what the force path needs zero at its start
    e = launch_fill(d.counts, ncount, p->stream);
    if (e == hipSuccess) e = d.grid_fixed ? launch_fill(d.rhofix, G, p->stream) : launch_fill(d.rho, G, p->stream);
    if (e == hipSuccess) e = launch_fill(d.flags, 4, p->stream);
    const hipError_t es = hipStreamSynchronize(p->stream);
    if (e == hipSuccess) e = es;
    if (e != hipSuccess) return hip_fail(p, e, "buffer initialisation");
    return ESP_OK;
  }
  e = hipMemset(d.counts, 0, ncount * sizeof(int));
  if (e == hipSuccess) e = hipMemset(d.nr_counts, 0, kMaxCells * sizeof(int));
  if (e == hipSuccess)
    e = d.grid_fixed ? hipMemset(d.rhofix, 0, G * sizeof(long long)) : hipMemset(d.rho, 0, G * sizeof(R));
  if (e == hipSuccess) e = hipMemset(d.facc, 0, static_cast<size_t>(r.n) * 3 * sizeof(double));
  if (e == hipSuccess) e = hipMemset(d.flags, 0, 4 * sizeof(int));
  const hipError_t es = hipDeviceSynchronize();
  if (e == hipSuccess) e = es;
  if (e != hipSuccess) return hip_fail(p, e, "buffer initialisation");
  return ESP_OK;
}

// Launch one stage, bracketed by profiling events when that stage is profiled.
template <class F>
hipError_t stage(esp_plan_t* p, int st, F&& launch, hipStream_t s) {
  Profiler& pr = p->prof;
  const bool on = ((pr.mask >> st) & 1u) && pr.used[st] < pr.cap && pr.seen[st]++ % pr.stride == 0;
  LaunchTiming& lt = launch_timing();
  if (on) lt = {pr.ev[st][2 * pr.used[st]], pr.ev[st][2 * pr.used[st] + 1]};
  (void)s;
  hipError_t e = launch();
  if (on) {
    // a stage that launched nothing (an error) leaves its events unrecorded
    if (!lt.start) ++pr.used[st];
    lt = {};
  }
  return e;
}

template <class F>
hipError_t stage(esp_plan_t* p, int st, F&& launch) {
  return stage(p, st, launch, p->stream);
}

// Cell sort.  Leaves the tile counts set; the spreading pass clears them.
template <typename R>
hipError_t run_sort(esp_plan_t* p, const R* xyz, const R* q) {
  DevPlan<R>& d = dev<R>(p);
  hipError_t e = stage(p, ST_BIN, [&] {
    hipError_t eb = launch_bin(d, xyz, q, p->stream);
    if (eb == hipSuccess && d.nsub > 1) eb = launch_scan_sub(d, p->stream);
    return eb;
  });
  if (e == hipSuccess) e = stage(p, ST_SCATTER, [&] { return launch_scatter(d, p->stream); });
  return e;
}

template <typename R>
esp_status run_sort_spread(esp_plan_t* p, const R* xyz, const R* q) {
  DevPlan<R>& d = dev<R>(p);
  hipError_t e = run_sort(p, xyz, q);
  if (e == hipSuccess) e = stage(p, ST_SPREAD, [&] { return launch_spread(d, p->stream); });
  return e == hipSuccess ? ESP_OK : hip_fail(p, e, "kernel launch");
}

template <typename R>
esp_status energy_virial(esp_plan_t* p, const R* xyz, const R* q, double* out7) {
  if (!xyz || !q || !out7) {
    p->err = "null pointer argument";
    return ESP_EINVAL;
  }
  DevPlan<R>& d = dev<R>(p);
  esp_status st = run_sort_spread(p, xyz, q);
  if (st != ESP_OK) return st;
  hipError_t e = stage(p, ST_FFT_XY, [&] { return launch_fft_xy(d, static_cast<const R*>(nullptr), d.spec, true, p->stream); });
  if (e == hipSuccess) e = stage(p, ST_FFT_Z, [&] { return launch_fft_z(d, Z_ENERGY, p->stream); });
  if (e == hipSuccess) e = launch_finalize(d, out7, p->stream);
  return e == hipSuccess ? ESP_OK : hip_fail(p, e, "kernel launch");
}

// Sort, spread, forward FFT and the z pass in the given mode (Z_POTENTIAL:
// the potential grid; Z_IK: the three field components), then the inverse
// xy pass of every component.
template <typename R>
esp_status potential(esp_plan_t* p, const R* xyz, const R* q, ZMode mode = Z_POTENTIAL) {
  DevPlan<R>& d = dev<R>(p);
  esp_status st = run_sort_spread(p, xyz, q);
  if (st != ESP_OK) return st;
  hipError_t e = stage(p, ST_FFT_XY, [&] { return launch_fft_xy(d, static_cast<const R*>(nullptr), d.spec, true, p->stream); });
  if (e == hipSuccess) e = stage(p, ST_FFT_Z, [&] { return launch_fft_z(d, mode, p->stream); });
  const int ncomp = mode == Z_IK ? 3 : (mode == Z_LOCAL ? 6 : 1);
  if (e == hipSuccess) e = stage(p, ST_FFT_XY_INV, [&] { return launch_fft_xy_inv(d, ncomp, p->stream); });
  return e == hipSuccess ? ESP_OK : hip_fail(p, e, "kernel launch");
}

template <typename R>
esp_status forces(esp_plan_t* p, const R* xyz, const R* q, R* f, double* out7) {
  if (!xyz || !q || !f) {
    p->err = "null pointer argument";
    return ESP_EINVAL;
  }
  DevPlan<R>& d = dev<R>(p);
  esp_status st = potential(p, xyz, q, d.ik ? Z_IK : Z_POTENTIAL);
  if (st != ESP_OK) return st;
  hipError_t e = stage(p, ST_GATHER, [&] { return launch_gather(d, f, out7, p->stream); });
  return e == hipSuccess ? ESP_OK : hip_fail(p, e, "kernel launch");
}

template <typename R>
esp_status local_virial(esp_plan_t* p, const R* xyz, const R* q, R* w6, double* out7) {
  if (!xyz || !q || !w6) {
    p->err = "null pointer argument";
    return ESP_EINVAL;
  }
  DevPlan<R>& d = dev<R>(p);
  if (!d.local) {
    p->err = "the plan was made without local_virial";
    return ESP_EINVAL;
  }
  esp_status st = potential(p, xyz, q, Z_LOCAL);
  if (st != ESP_OK) return st;
  hipError_t e = stage(p, ST_GATHER, [&] { return launch_gather_local(d, w6, out7, p->stream); });
  return e == hipSuccess ? ESP_OK : hip_fail(p, e, "kernel launch");
}

// The real-space part's launch description: the plan with the real-space
// cells as sort keys and the real-space sort buffers.
template <typename R>
DevPlan<R> near_plan(esp_plan_t* p) {
  DevPlan<R> c = dev<R>(p);
  c.cellsort = 1;
  c.grid_fixed = 0;                   // the near part's sort publishes no grid scale
  c.ntiles = c.cn1 * c.cn2 * c.cn3;
  c.nsub = 1;
  c.bin_lds = c.ntiles <= 8192 ? 1 : 0;
  set_bin_blocks(c);
  c.counts = c.nr_counts;
  c.offsets = c.nr_offsets;
  c.keys = c.nr_keys;
  c.ranks = c.nr_ranks;
  c.perm = c.nr_perm;
  c.tmp = c.nr_tmp;
  c.sorted = c.nr_sorted;
  c.qpart = c.nr_qpart;
  // enough workgroups to fill the chip: rsplit x cells <= max(cells, 2 kRealBlocks)
  c.rsplit = std::max(1, std::min(kMaxRealSplit, (kRealBlocks + c.ntiles / 2) / c.ntiles));
  return c;
}

// Cell sort with the real-space cells and the pair kernel on stream s (the
// pair kernel clears the cell counters); forces and sums stay in the plan.
template <typename R>
hipError_t launch_near(const DevPlan<R>& c, const R* xyz, const R* q, hipStream_t s) {
  hipError_t e = launch_bin(c, xyz, q, s);
  if (e == hipSuccess) e = launch_scatter(c, s);
  if (e == hipSuccess) e = launch_real_pairs(c, s);
  return e;
}

// Real-space part on the plan's stream.
template <typename R>
esp_status real_space(esp_plan_t* p, const R* xyz, const R* q, R* f, int accumulate, double* out7) {
  if (!xyz || !q || !f || !out7) {
    p->err = "null pointer argument";
    return ESP_EINVAL;
  }
  const DevPlan<R> c = near_plan<R>(p);
  hipError_t e = stage(p, ST_REAL, [&] {
    hipError_t eb = launch_near(c, xyz, q, p->stream);
    if (eb == hipSuccess) eb = launch_real_forces(c, f, accumulate, p->stream);
    if (eb == hipSuccess) eb = launch_real_finalize(c, out7, 0, p->stream);
    return eb;
  });
  return e == hipSuccess ? ESP_OK : hip_fail(p, e, "kernel launch");
}

// Total Coulomb: the real-space part on the side stream, the Fourier forces
// on the plan's stream at the same time (they share only the read-only
// inputs and the error flags), then, after the join, the near forces and
// sums added to f and out7.
template <typename R>
esp_status coulomb(esp_plan_t* p, const R* xyz, const R* q, R* f, double* out7) {
  if (!xyz || !q || !f || !out7) {
    p->err = "null pointer argument";
    return ESP_EINVAL;
  }
  hipError_t e = hipSuccess;
  if (!p->side) {
    e = hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(p, e, "side stream creation");
  }
  const DevPlan<R> c = near_plan<R>(p);
  e = hipEventRecord(p->ev_fork, p->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(p->side, p->ev_fork, 0);
  if (e == hipSuccess) e = stage(p, ST_REAL, [&] { return launch_near(c, xyz, q, p->side); }, p->side);
  if (e == hipSuccess) e = hipEventRecord(p->ev_join, p->side);
  if (e != hipSuccess) return hip_fail(p, e, "real-space launch");
  const esp_status st = forces<R>(p, xyz, q, f, out7);
  // joined whatever the Fourier part returned, so that later work on the
  // plan's stream stays ordered after the side stream's
  e = hipStreamWaitEvent(p->stream, p->ev_join, 0);
  if (st != ESP_OK) return st;
  if (e == hipSuccess) e = launch_real_forces(c, f, 1, p->stream);
  if (e == hipSuccess) e = launch_real_finalize(c, out7, 1, p->stream);
  return e == hipSuccess ? ESP_OK : hip_fail(p, e, "kernel launch");
}

esp_status want_precision(esp_plan_t* p, int prec) {
  if (!p) return ESP_EINVAL;
  if (p->r.precision != prec) {
    p->err = prec == ESP_FP32 ? "FP64 plan: use the _f64 entry points" : "FP32 plan: use the float entry points";
    return ESP_EINVAL;
  }
  return ESP_OK;
}

template <typename R>
size_t real_bytes() { return sizeof(R); }

}  // namespace

// ============================================================================ C ABI
namespace {

esp_status plan_create(const double h[9], int64_t n, double tol, const esp_opts* o, void* region, size_t cap,
                       esp_plan_t** out) {
  if (!out) return ESP_EINVAL;
  *out = nullptr;
  std::unique_ptr<esp_plan_s> p(new esp_plan_s());
  p->arena = static_cast<unsigned char*>(region);
  p->arena_cap = region ? cap : 0;
  esp_status warn;
  try {
    warn = resolve(h, n, tol, o, p->r, p->err);
    if (warn < 0) {
      std::fprintf(stderr, "esp_plan: %s\n", p->err.c_str());
      return warn;
    }
    p->split.reset(new Pswf(p->r.c_split));
    p->spread.reset(new Pswf(p->r.c_spread));
  } catch (const std::exception& ex) {
    std::fprintf(stderr, "esp_plan: %s\n", ex.what());
    return ESP_EINVAL;
  }
  const Pswf& s = *p->split;
  p->A = kTwoPi * s.lambda0() / s.C0();
  p->self_coef = s.psi0() / (2.0 * s.C0() * p->r.rc);
  {
    // Ic = rc^2 / 2 - int_0^rc r phi0(r) dr, phi0(r) = int_0^{r/rc} psi / C0 (Sec. 3.4)
    std::vector<double> x, w;
    gauss_legendre(96, x, w);
    double acc = 0;
    for (size_t j = 0; j < x.size(); ++j) {
      const double t = 0.5 * (x[j] + 1.0);
      acc += 0.5 * w[j] * t * s.int_psi(t) / s.C0();
    }
    p->Ic = p->r.rc * p->r.rc * (0.5 - acc);
  }
  p->stream = o ? static_cast<hipStream_t>(o->stream) : nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
    p->err = "no HIP device";
    std::fprintf(stderr, "esp_plan: no HIP device\n");
    return ESP_EDEVICE;
  }
  esp_status st = p->r.precision == ESP_FP32 ? build_device<float>(p.get()) : build_device<double>(p.get());
  if (st != ESP_OK) {
    std::fprintf(stderr, "esp_plan: %s\n", p->err.c_str());
    return st;
  }
  *out = p.release();
  return warn;
}

}  // namespace


extern "C" {

void esp_opts_default(esp_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->precision = ESP_FP32;
  o->params = ESP_ANALYTIC;
  o->coupling = ESP_ISO;
  o->rc = 0.9;
  o->grid_sigma = 1.07;
  o->coulomb_k = 1.0;
}

esp_status esp_resolve_params(const double h[9], int64_t n, double tol, const esp_opts* o, esp_params* out) {
  if (!out) return ESP_EINVAL;
  Resolved r;
  std::string err;
  esp_status st;
  try {
    st = resolve(h, n, tol, o, r, err);
  } catch (const std::exception& ex) {
    return ESP_EINVAL;
  }
  if (st < 0) return st;
  std::memset(out, 0, sizeof *out);
  out->precision = r.precision;
  out->n = r.n;
  out->tol = r.tol;
  out->delta = r.delta;
  out->rc = r.rc;
  out->c_split = r.c_split;
  out->c_spread = r.c_spread;
  out->P = r.P;
  for (int d = 0; d < 3; ++d) {
    out->M[d] = r.M[d];
    out->tile[d] = r.T[d];
  }
  out->ntiles = r.ntiles;
  out->volume = r.V;
  out->params_source = r.params_source;
  for (int j = 0; j < 4; ++j) out->predicted_log10_err[j] = r.pred[j];
  out->predicted_cost = r.pred_cost;
  Pswf ps(r.c_split);
  out->lambda0_split = ps.lambda0();
  out->C0_split = ps.C0();
  out->psi0_split = ps.psi0();
  return st;
}


esp_status esp_plan(const double h[9], int64_t n, double tol, const esp_opts* o, esp_plan_t** out) {
  return plan_create(h, n, tol, o, nullptr, 0, out);
}

esp_status esp_set_box(esp_plan_t* p, const double h[9]) {
  if (!p || !h) return ESP_EINVAL;
  double hinv[9], V;
  esp_status st = check_box(h, p->r.rc, hinv, &V, p->err);
  if (st != ESP_OK) return st;
  std::memcpy(p->r.h, h, sizeof p->r.h);
  std::memcpy(p->r.hinv, hinv, sizeof hinv);
  p->r.V = V;
  if (p->r.precision == ESP_FP32) set_box_fields(p, p->d32); else set_box_fields(p, p->d64);
  for (int d = 0; d < 3; ++d)
    if (p->r.M[d] * 1.1 < grid_rule(h, d, p->r.c_split, p->r.rc, p->r.sigma)) {
      p->err = "the cell grew by more than 10% beyond the grid rule; consider a new plan";
      return ESP_WARN_REPLAN;
    }
  return ESP_OK;
}

esp_status esp_set_stream(esp_plan_t* p, void* stream) {
  if (!p) return ESP_EINVAL;
  p->stream = static_cast<hipStream_t>(stream);
  return ESP_OK;
}

esp_status esp_energy_virial(esp_plan_t* p, const float* xyz, const float* q, double* out7) {
  esp_status st = want_precision(p, ESP_FP32);
  return st != ESP_OK ? st : energy_virial<float>(p, xyz, q, out7);
}

esp_status esp_energy_virial_f64(esp_plan_t* p, const double* xyz, const double* q, double* out7) {
  esp_status st = want_precision(p, ESP_FP64);
  return st != ESP_OK ? st : energy_virial<double>(p, xyz, q, out7);
}

esp_status esp_forces(esp_plan_t* p, const float* xyz, const float* q, float* f, double* out7) {
  esp_status st = want_precision(p, ESP_FP32);
  return st != ESP_OK ? st : forces<float>(p, xyz, q, f, out7);
}

esp_status esp_forces_f64(esp_plan_t* p, const double* xyz, const double* q, double* f, double* out7) {
  esp_status st = want_precision(p, ESP_FP64);
  return st != ESP_OK ? st : forces<double>(p, xyz, q, f, out7);
}

esp_status esp_local_virial(esp_plan_t* p, const float* xyz, const float* q, float* w6, double* out7) {
  esp_status st = want_precision(p, ESP_FP32);
  return st != ESP_OK ? st : local_virial<float>(p, xyz, q, w6, out7);
}

esp_status esp_local_virial_f64(esp_plan_t* p, const double* xyz, const double* q, double* w6, double* out7) {
  esp_status st = want_precision(p, ESP_FP64);
  return st != ESP_OK ? st : local_virial<double>(p, xyz, q, w6, out7);
}

esp_status esp_real_space(esp_plan_t* p, const float* xyz, const float* q, float* f, int accumulate,
                          double* out7) {
  esp_status st = want_precision(p, ESP_FP32);
  return st != ESP_OK ? st : real_space<float>(p, xyz, q, f, accumulate, out7);
}

esp_status esp_real_space_f64(esp_plan_t* p, const double* xyz, const double* q, double* f, int accumulate,
                              double* out7) {
  esp_status st = want_precision(p, ESP_FP64);
  return st != ESP_OK ? st : real_space<double>(p, xyz, q, f, accumulate, out7);
}

esp_status esp_coulomb(esp_plan_t* p, const float* xyz, const float* q, float* f, double* out7) {
  esp_status st = want_precision(p, ESP_FP32);
  return st != ESP_OK ? st : coulomb<float>(p, xyz, q, f, out7);
}

esp_status esp_coulomb_f64(esp_plan_t* p, const double* xyz, const double* q, double* f, double* out7) {
  esp_status st = want_precision(p, ESP_FP64);
  return st != ESP_OK ? st : coulomb<double>(p, xyz, q, f, out7);
}

esp_status esp_check(esp_plan_t* p) {
  if (!p) return ESP_EINVAL;
  hipError_t e = hipStreamSynchronize(p->stream);
  if (e == hipSuccess && p->side) e = hipStreamSynchronize(p->side);
  if (e != hipSuccess) return hip_fail(p, e, "stream synchronise");
  int* flags = p->r.precision == ESP_FP32 ? p->d32.flags : p->d64.flags;
  int h = 0;
  e = hipMemcpy(&h, flags, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(p, e, "flag read");
  if (h) {
    (void)hipMemset(flags, 0, sizeof(int));
    if (h & 2) {
      p->err = "inconsistent tile counts in the cell sort (results of the affected calls are invalid)";
      return ESP_EDEVICE;
    }
    p->err = "non-finite position or charge (treated as an uncharged particle)";
    return ESP_ENONFINITE;
  }
  return ESP_OK;
}

esp_status esp_get_params(const esp_plan_t* p, esp_params* out) {
  if (!p || !out) return ESP_EINVAL;
  const Resolved& r = p->r;
  std::memset(out, 0, sizeof *out);
  out->precision = r.precision;
  out->n = r.n;
  out->tol = r.tol;
  out->delta = r.delta;
  out->rc = r.rc;
  out->c_split = r.c_split;
  out->c_spread = r.c_spread;
  out->P = r.P;
  for (int d = 0; d < 3; ++d) {
    out->M[d] = r.M[d];
    out->tile[d] = r.T[d];
  }
  out->ntiles = r.ntiles;
  out->window_degree = p->nw_fitted;
  out->kernel_degree = p->nker;
  out->lambda0_split = p->split->lambda0();
  out->C0_split = p->split->C0();
  out->psi0_split = p->split->psi0();
  out->volume = r.V;
  out->params_source = r.params_source;
  for (int j = 0; j < 4; ++j) out->predicted_log10_err[j] = r.pred[j];
  out->predicted_cost = r.pred_cost;
  out->gather_tiled = r.precision == ESP_FP32 ? p->d32.gather_tiled : p->d64.gather_tiled;
  out->gather_lane = r.precision == ESP_FP32 ? p->d32.gather_lane : p->d64.gather_lane;
  out->grid_fixed = r.precision == ESP_FP32 ? p->d32.grid_fixed : 0;
  out->counter_copies = r.precision == ESP_FP32 ? p->d32.nsub : p->d64.nsub;
  out->force = r.force;
  out->local_virial = r.local;
  {
    const bool f32 = r.precision == ESP_FP32;
    out->real_cells[0] = f32 ? p->d32.cn1 : p->d64.cn1;
    out->real_cells[1] = f32 ? p->d32.cn2 : p->d64.cn2;
    out->real_cells[2] = f32 ? p->d32.cn3 : p->d64.cn3;
    out->real_segments = p->nseg;
    out->fft_split = f32 ? p->d32.xy_split : p->d64.xy_split;
    out->spread_fixed = f32 ? p->d32.spread_fixed : p->d64.spread_fixed;
  }
  for (int i = 0; i < 9; ++i) out->hinv[i] = r.hinv[i];
  return ESP_OK;
}

const char* esp_last_error(const esp_plan_t* p) { return p ? p->err.c_str() : "null plan"; }

void esp_destroy(esp_plan_t* p) {
  if (!p) return;
  (void)hipStreamSynchronize(p->stream);
  if (p->side) (void)hipStreamSynchronize(p->side);
  delete p;
}

esp_status esp_stage_sort(esp_plan_t* p, const void* xyz, const void* q, int32_t* perm_out,
                          int32_t* offsets_out) {
  if (!p || !xyz || !q || !perm_out || !offsets_out) return ESP_EINVAL;
  hipError_t e;
  const int* perm;
  const int* off;
  int* counts;
  if (p->r.precision == ESP_FP32) {
    e = run_sort(p, static_cast<const float*>(xyz), static_cast<const float*>(q));
    perm = p->d32.perm;
    off = p->d32.offsets;
    counts = p->d32.counts;
  } else {
    e = run_sort(p, static_cast<const double*>(xyz), static_cast<const double*>(q));
    perm = p->d64.perm;
    off = p->d64.offsets;
    counts = p->d64.counts;
  }
  // no spreading pass follows: clear the tile counts here
  const int nsub = p->r.precision == ESP_FP32 ? p->d32.nsub : p->d64.nsub;
  if (e == hipSuccess) e = launch_fill(counts, static_cast<size_t>(p->r.ntiles) * nsub, p->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(perm_out, perm, p->r.n * sizeof(int), hipMemcpyDeviceToDevice, p->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(offsets_out, off, (p->r.ntiles + 1) * sizeof(int), hipMemcpyDeviceToDevice, p->stream);
  return e == hipSuccess ? ESP_OK : hip_fail(p, e, "stage sort");
}

esp_status esp_stage_spread(esp_plan_t* p, const void* xyz, const void* q, void* grid_out) {
  if (!p || !xyz || !q || !grid_out) return ESP_EINVAL;
  const size_t G = static_cast<size_t>(p->r.M[0]) * p->r.M[1] * p->r.M[2];
  esp_status st;
  hipError_t e = hipSuccess;
  if (p->r.precision == ESP_FP32) {
    st = run_sort_spread(p, static_cast<const float*>(xyz), static_cast<const float*>(q));
    if (st != ESP_OK) return st;
    if (p->d32.grid_fixed) {
      e = launch_grid_out(p->d32, static_cast<float*>(grid_out), p->stream);
    } else {
      e = hipMemcpyAsync(grid_out, p->d32.rho, G * sizeof(float), hipMemcpyDeviceToDevice, p->stream);
      if (e == hipSuccess) e = launch_fill(p->d32.rho, G, p->stream);
    }
  } else {
    st = run_sort_spread(p, static_cast<const double*>(xyz), static_cast<const double*>(q));
    if (st != ESP_OK) return st;
    e = hipMemcpyAsync(grid_out, p->d64.rho, G * sizeof(double), hipMemcpyDeviceToDevice, p->stream);
    if (e == hipSuccess) e = launch_fill(p->d64.rho, G, p->stream);
  }
  return e == hipSuccess ? ESP_OK : hip_fail(p, e, "stage spread");
}

esp_status esp_stage_fft(esp_plan_t* p, const void* grid_in, void* spec_out) {
  if (!p || !grid_in || !spec_out) return ESP_EINVAL;
  const size_t S = static_cast<size_t>(p->r.M[0] / 2 + 1) * p->r.M[1] * p->r.M[2];
  hipError_t e;
  if (p->r.precision == ESP_FP32) {
    DevPlan<float>& d = p->d32;
    e = launch_fft_xy(d, static_cast<const float*>(grid_in), d.spec, false, p->stream);
    if (e == hipSuccess) e = launch_fft_z(d, Z_FFT_ONLY, p->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(spec_out, d.spec, S * sizeof(Cplx<float>), hipMemcpyDeviceToDevice, p->stream);
  } else {
    DevPlan<double>& d = p->d64;
    e = launch_fft_xy(d, static_cast<const double*>(grid_in), d.spec, false, p->stream);
    if (e == hipSuccess) e = launch_fft_z(d, Z_FFT_ONLY, p->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(spec_out, d.spec, S * sizeof(Cplx<double>), hipMemcpyDeviceToDevice, p->stream);
  }
  return e == hipSuccess ? ESP_OK : hip_fail(p, e, "stage fft");
}

esp_status esp_stage_potential(esp_plan_t* p, const void* xyz, const void* q, void* phi_out) {
  if (!p || !xyz || !q || !phi_out) return ESP_EINVAL;
  const size_t G = static_cast<size_t>(p->r.M[0]) * p->r.M[1] * p->r.M[2];
  esp_status st;
  hipError_t e;
  if (p->r.precision == ESP_FP32) {
    st = potential(p, static_cast<const float*>(xyz), static_cast<const float*>(q));
    if (st != ESP_OK) return st;
    e = hipMemcpyAsync(phi_out, p->d32.phi, G * sizeof(float), hipMemcpyDeviceToDevice, p->stream);
  } else {
    st = potential(p, static_cast<const double*>(xyz), static_cast<const double*>(q));
    if (st != ESP_OK) return st;
    e = hipMemcpyAsync(phi_out, p->d64.phi, G * sizeof(double), hipMemcpyDeviceToDevice, p->stream);
  }
  return e == hipSuccess ? ESP_OK : hip_fail(p, e, "stage potential");
}

esp_status esp_pswf_eval(double c, int64_t m, const double* x, double* psi, double* dpsi, double* ipsi,
                         double* consts3) {
  if (!(c > 0) || m < 0 || (m > 0 && !x)) return ESP_EINVAL;
  try {
    Pswf ps(c);
    for (int64_t i = 0; i < m; ++i) {
      if (psi) psi[i] = ps.psi(x[i]);
      if (dpsi) dpsi[i] = ps.dpsi(x[i]);
      if (ipsi) ipsi[i] = std::fabs(x[i]) <= 1.0 ? ps.int_psi(x[i]) : std::nan("");
    }
    if (consts3) {
      consts3[0] = ps.psi0();
      consts3[1] = ps.C0();
      consts3[2] = ps.lambda0();
    }
  } catch (const std::exception&) {
    return ESP_EINVAL;
  }
  return ESP_OK;
}

double esp_c_from_delta(double delta) {
  try {
    return c_from_delta(delta);
  } catch (const std::exception&) {
    return std::nan("");
  }
}

esp_status esp_profile_enable(esp_plan_t* p, unsigned stage_mask, int max_launches, int stride) {
  if (!p || max_launches < 0 || max_launches > (1 << 20) || stride < 1) return ESP_EINVAL;
  hipError_t e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return hip_fail(p, e, "stream synchronise");
  Profiler& pr = p->prof;
  pr.release();
  pr.mask = stage_mask & ((1u << ST_COUNT) - 1);
  pr.cap = pr.mask ? max_launches : 0;
  pr.stride = stride;
  for (int s = 0; s < ST_COUNT; ++s) {
    pr.used[s] = 0;
    pr.seen[s] = 0;
    pr.ms[s] = 0;
    pr.cnt[s] = 0;
    if (!((pr.mask >> s) & 1u)) continue;
    pr.ev[s].resize(2 * static_cast<size_t>(pr.cap));
    for (auto& ev : pr.ev[s]) {
      e = hipEventCreate(&ev);
      if (e != hipSuccess) {
        pr.release();
        pr.mask = 0;
        pr.cap = 0;
        return hip_fail(p, e, "hipEventCreate");
      }
    }
  }
  return ESP_OK;
}

esp_status esp_profile_read(esp_plan_t* p, double* total_ms, int64_t* launches) {
  if (!p) return ESP_EINVAL;
  hipError_t e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return hip_fail(p, e, "stream synchronise");
  Profiler& pr = p->prof;
  for (int s = 0; s < ST_COUNT; ++s) {
    for (int k = 0; k < pr.used[s]; ++k) {
      float ms = 0;
      e = hipEventElapsedTime(&ms, pr.ev[s][2 * k], pr.ev[s][2 * k + 1]);
      if (e != hipSuccess) return hip_fail(p, e, "hipEventElapsedTime");
      pr.ms[s] += ms;
      ++pr.cnt[s];
    }
    pr.used[s] = 0;
    if (total_ms) total_ms[s] = pr.ms[s];
    if (launches) launches[s] = pr.cnt[s];
  }
  return ESP_OK;
}

const char* esp_stage_name(int stage) {
  return stage >= 0 && stage < ST_COUNT ? kStageNames[stage] : "";
}

esp_status esp_proposer_set(const esp_proposer* p) {
  std::lock_guard<std::mutex> lock(g_prop_mu);
  if (!p) {
    g_prop = ProposerState{};
    return ESP_OK;
  }
  if (!p->mlp || esp_mlp_num_params(p->mlp) <= 0 || mlp_dim(p->mlp, 0) != ESP_PROPOSER_FEATURES ||
      mlp_dim(p->mlp, 1) != 4)
    return ESP_EINVAL;
  for (int j = 0; j < ESP_PROPOSER_FEATURES; ++j)
    if (!(p->in_std[j] > 0)) return ESP_EINVAL;
  for (int j = 0; j < 4; ++j)
    if (!(p->out_std[j] > 0) || !(p->margin[j] >= 0)) return ESP_EINVAL;
  ProposerState st;
  st.cfg = *p;
  try {
    for (int k = 0; k <= 20; ++k) {
      const double delta = std::pow(10.0, -2.0 - 0.25 * k);
      st.deltas.push_back(delta);
      st.cs.push_back(c_from_delta(delta));
    }
  } catch (const std::exception&) {
    return ESP_EINVAL;
  }
  st.set = true;
  g_prop = st;
  return ESP_OK;
}

const char* esp_version(void) { return "esp-mi355x 0.1.0 (gfx950)"; }

}  // extern "C"

namespace espx {

esp_status plan_in_region(const double h[9], int64_t n, double tol, const esp_opts* o, void* base, size_t cap,
                          esp_plan_t** out, size_t* used) {
  if (!base || cap == 0) return ESP_EINVAL;
  const esp_status st = plan_create(h, n, tol, o, base, cap, out);
  if (used) *used = st >= 0 && *out ? (*out)->arena_used : 0;
  return st;
}

void plan_release(esp_plan_t* p) { delete p; }

bool plan_same_grid(const esp_plan_t* p, const double h[9]) {
  const Resolved& r = p->r;
  if (r.params_source == ESP_EXPLICIT) return true;
  if (r.params_source != ESP_ANALYTIC) return false;
  for (int d = 0; d < 3; ++d)
    if (next_smooth(std::max({grid_rule(h, d, r.c_split, r.rc, r.sigma), r.P, 2})) != r.M[d]) return false;
  return true;
}

}  // namespace espx

// ============================================================================ batches
// A batch holds one ordinary plan per replica (its tables and buffers) plus a
// device array of their DevPlans, ordered so that replicas sharing a window
// support P and window degree are adjacent.  Each stage is one launch over a
// contiguous range of that array; a workgroup finds its replica by bisecting
// the stage's block offsets.
struct BatchStage {
  size_t at = 0;          // index of this stage's offsets in the shared table
  int* boff = nullptr;    // device: count + 1 block offsets
  int nblk = 0, nth = 256;
  size_t lds = 0;
  int first = 0, count = 0;
  int P = 0, nw = 0;
  int ppt = 1;            // binning stage: largest binppt of its replicas
  int grid_fixed = 0;     // xy stage: the replicas keep int64 grids
  int lane = 0;           // gather stage: tile-staged, one particle per lane
};

struct esp_batch_s {
  int nrep = 0, precision = ESP_FP32;
  std::vector<esp_plan_t*> reps;
  std::vector<int> order;         // position in the device array -> replica
  std::vector<int> pos;           // replica -> position
  std::vector<int64_t> pofs;      // first particle of each replica (nrep + 1)
  hipStream_t stream = nullptr;
  void* dplans = nullptr;
  int* dboff = nullptr;
  unsigned char* hstage = nullptr;    // pinned staging of box updates, one slot per replica
  std::vector<hipEvent_t> staged;
  size_t plan_bytes = 0;
  BatchStage bin, scatter, fxy, fz, fxyi, fin;
  std::vector<BatchStage> spread, gather;
  bool any_sub = false;           // some replica bins into counter copies
  bool use_graph = false;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* key[5] = {};
  std::string err;
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  ~esp_batch_s() {
    (void)hipStreamSynchronize(stream);
    drop_graph();
    if (cap) (void)hipStreamDestroy(cap);
    for (hipEvent_t e : staged)
      if (e) (void)hipEventDestroy(e);
    if (hstage) (void)hipHostFree(hstage);
    if (dplans) (void)hipFree(dplans);
    if (dboff) (void)hipFree(dboff);
    for (esp_plan_t* p : reps) delete p;
  }
};

namespace {

template <typename R>
DevPlan<R> batch_entry(const esp_batch_t* b, int r) {
  DevPlan<R> d = dev<R>(b->reps[r]);
  d.pofs = b->pofs[r];
  d.rep = r;
  // the batch's binning launch has blocks enough for the chip from all its
  // replicas together: every replica takes kBinMaxPpt particles per thread
  d.binppt = kBinMaxPpt;
  d.nbin = static_cast<int>((d.n + kBinThreads * kBinMaxPpt - 1) / (kBinThreads * kBinMaxPpt));
  return d;
}

template <typename R>
esp_status batch_build(esp_batch_t* b) {
  const int nrep = b->nrep;
  std::vector<DevPlan<R>> hp(nrep);
  for (int k = 0; k < nrep; ++k) hp[k] = batch_entry<R>(b, b->order[k]);
  for (int k = 0; k < nrep; ++k)
    if (hp[k].xy_split) {
      b->err = "a replica's grid plane exceeds one workgroup's LDS; batched launches need the one-pass xy transform";
      return ESP_EINVAL;
    }
  // batched FP32 spreading is fixed point: a deterministic batch needs every
  // replica's int64 grid (batch options are shared, so all or none have one)
  for (int k = 0; k < nrep; ++k)
    if (hp[k].grid_fixed != hp[0].grid_fixed || (hp[k].grid_fixed && sizeof(R) != 4)) {
      b->err = "replicas differ in their grid accumulation (deterministic FP32 batches need fixed-point tiles)";
      return ESP_EINVAL;
    }
  std::vector<int> offs;
  auto make = [&](BatchStage& st, int first, int count, auto nblk_of, auto lds_of, int nth) {
    st.first = first;
    st.count = count;
    st.at = offs.size();
    st.nth = nth;
    st.lds = 0;
    offs.push_back(0);
    for (int k = first; k < first + count; ++k) {
      offs.push_back(offs.back() + nblk_of(hp[k]));
      st.lds = std::max(st.lds, lds_of(hp[k]));
    }
    st.nblk = offs.back();
    st.P = hp[first].P;
    st.nw = hp[first].nw;
  };
  auto zero = [](const DevPlan<R>&) { return size_t(0); };
  make(b->bin, 0, nrep, [](const DevPlan<R>& d) { return d.nbin; },
       [](const DevPlan<R>& d) { return d.bin_lds ? static_cast<size_t>(d.ntiles) * sizeof(int) : size_t(0); },
       kBinThreads);
  for (const DevPlan<R>& d : hp) b->bin.ppt = std::max(b->bin.ppt, d.binppt);
  make(b->scatter, 0, nrep, [](const DevPlan<R>& d) { return static_cast<int>((d.n + 1023) / 1024); },
       [](const DevPlan<R>& d) { return (static_cast<size_t>(d.ntiles) + 1) * sizeof(int); }, 1024);
  int nth_xy = 256;
  for (const DevPlan<R>& d : hp) nth_xy = std::max(nth_xy, fft_threads(d.M1 * d.M2));
  make(b->fxy, 0, nrep, [](const DevPlan<R>& d) { return d.M3; }, [](const DevPlan<R>& d) { return lds_fft_xy(d); },
       nth_xy);
  b->fxy.grid_fixed = hp[0].grid_fixed;
  make(b->fz, 0, nrep, [](const DevPlan<R>& d) { return d.nzblk; }, [](const DevPlan<R>& d) { return lds_fft_z(d); },
       256);
  make(b->fxyi, 0, nrep, [](const DevPlan<R>& d) { return d.M3; }, [](const DevPlan<R>& d) { return lds_fft_xy(d); },
       nth_xy);
  make(b->fin, 0, nrep, [](const DevPlan<R>&) { return 1; }, zero, 256);
  b->any_sub = false;
  for (const DevPlan<R>& d : hp) b->any_sub = b->any_sub || d.nsub > 1;
  b->spread.clear();
  b->gather.clear();
  int dev_id = 0, maxlds = 65536;
  if (hipGetDevice(&dev_id) == hipSuccess)
    (void)hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev_id);
  for (int k = 0; k < nrep;) {
    int e = k + 1;
    while (e < nrep && hp[e].P == hp[k].P && hp[e].nw == hp[k].nw) ++e;
    BatchStage sp, ga;
    make(sp, k, e - k, [](const DevPlan<R>& d) { return d.ntiles; },
         [](const DevPlan<R>& d) { return lds_spread(d); }, 256);
    // gather: tile-staged with one particle per lane (one workgroup per tile)
    // where every replica's potential box fits in LDS, else per particle
    auto lane_lds = [](const DevPlan<R>& d) {
      return static_cast<size_t>(((d.nw + 1) * d.P + 3) / 4 * 4) * sizeof(R) + lds_gather_box(d);
    };
    bool lane = true;
    for (int j = k; j < e; ++j) lane = lane && lane_lds(hp[j]) <= static_cast<size_t>(maxlds);
    if (lane) {
      make(ga, k, e - k, [](const DevPlan<R>& d) { return d.ntiles; }, lane_lds, 256);
      ga.lane = 1;
    } else {
      const int G = 256 / gather_lanes(hp[k].P);
      make(ga, k, e - k, [G](const DevPlan<R>& d) { return static_cast<int>((d.n + G - 1) / G); }, zero, 256);
    }
    b->spread.push_back(sp);
    b->gather.push_back(ga);
    k = e;
  }
  b->plan_bytes = sizeof(DevPlan<R>);
  void* dp = nullptr;
  hipError_t e = hipMalloc(&dp, hp.size() * sizeof(DevPlan<R>));
  if (e == hipSuccess) {
    b->dplans = dp;
    e = hipMalloc(&b->dboff, offs.size() * sizeof(int));
  }
  if (e == hipSuccess) e = hipMemcpy(b->dplans, hp.data(), hp.size() * sizeof(DevPlan<R>), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->dboff, offs.data(), offs.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&b->hstage), hp.size() * sizeof(DevPlan<R>));
  if (e != hipSuccess) {
    b->err = std::string("batch set-up: ") + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? ESP_ENOMEM : ESP_EDEVICE;
  }
  b->staged.assign(nrep, nullptr);
  for (BatchStage* st : {&b->bin, &b->scatter, &b->fxy, &b->fz, &b->fxyi, &b->fin}) st->boff = b->dboff + st->at;
  for (auto* v : {&b->spread, &b->gather})
    for (BatchStage& st : *v) st.boff = b->dboff + st.at;
  return ESP_OK;
}

template <typename R>
BatchLaunch<R> batch_launch(const esp_batch_t* b, const BatchStage& st) {
  return BatchLaunch<R>{static_cast<const DevPlan<R>*>(b->dplans) + st.first, st.boff, st.count, st.nblk, st.nth,
                        st.lds, st.P, st.nw, st.ppt, st.grid_fixed, st.lane};
}

template <typename R>
hipError_t batch_launches(const esp_batch_t* b, const R* xyz, const R* q, R* f, double* out7, bool forces,
                          hipStream_t s) {
  hipError_t e = launch_bin_batch(batch_launch<R>(b, b->bin), xyz, q, s);
  if (e == hipSuccess && b->any_sub) e = launch_scan_sub_batch(batch_launch<R>(b, b->fin), s);
  if (e == hipSuccess) e = launch_scatter_batch(batch_launch<R>(b, b->scatter), s);
  for (const BatchStage& g : b->spread)
    if (e == hipSuccess) e = launch_spread_batch(batch_launch<R>(b, g), s);
  if (e == hipSuccess) e = launch_fft_xy_batch(batch_launch<R>(b, b->fxy), s);
  if (e == hipSuccess) e = launch_fft_z_batch(batch_launch<R>(b, b->fz), forces ? Z_POTENTIAL : Z_ENERGY, s);
  if (forces) {
    if (e == hipSuccess) e = launch_fft_xy_inv_batch(batch_launch<R>(b, b->fxyi), s);
    for (const BatchStage& g : b->gather)
      if (e == hipSuccess) e = launch_gather_batch(batch_launch<R>(b, g), f, out7, s);
  } else if (e == hipSuccess) {
    e = launch_finalize_batch(batch_launch<R>(b, b->fin), out7, s);
  }
  return e;
}

esp_status batch_fail(esp_batch_t* b, hipError_t e, const char* what) {
  b->err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? ESP_ENOMEM : ESP_EDEVICE;
}

template <typename R>
esp_status batch_call(esp_batch_t* b, const R* xyz, const R* q, R* f, double* out7, bool forces) {
  if (!b) return ESP_EINVAL;
  if ((b->precision == ESP_FP32) != std::is_same<R, float>::value) {
    b->err = "precision of the entry point differs from the batch's";
    return ESP_EINVAL;
  }
  if (!xyz || !q || (forces && !f) || (!forces && !out7)) {
    b->err = "null pointer argument";
    return ESP_EINVAL;
  }
  if (!b->use_graph) {
    const hipError_t e = batch_launches(b, xyz, q, f, out7, forces, b->stream);
    return e == hipSuccess ? ESP_OK : batch_fail(b, e, "kernel launch");
  }
  const void* key[5] = {xyz, q, f, out7, forces ? b : nullptr};
  if (b->exec && std::equal(key, key + 5, b->key)) {
    const hipError_t e = hipGraphLaunch(b->exec, b->stream);
    return e == hipSuccess ? ESP_OK : batch_fail(b, e, "graph launch");
  }
  // New pointers or kind of call: run eagerly (this call's result), then record
  // the same launches on a private stream for the following calls.
  hipError_t e = batch_launches(b, xyz, q, f, out7, forces, b->stream);
  if (e != hipSuccess) return batch_fail(b, e, "kernel launch");
  b->drop_graph();
  if (!b->cap && (e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)) != hipSuccess)
    return batch_fail(b, e, "capture stream");
  if ((e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return batch_fail(b, e, "begin capture");
  const hipError_t el = batch_launches(b, xyz, q, f, out7, forces, b->cap);
  e = hipStreamEndCapture(b->cap, &b->graph);
  if (el != hipSuccess || e != hipSuccess) {
    b->drop_graph();
    return batch_fail(b, el != hipSuccess ? el : e, "graph capture");
  }
  if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess) {
    b->drop_graph();
    return batch_fail(b, e, "graph instantiate");
  }
  std::copy(key, key + 5, b->key);
  return ESP_OK;
}

}  // namespace

extern "C" {

esp_status esp_batch_plan(int nrep, const double* h, const int64_t* n, const double* tol, const esp_opts* o,
                          const int* tiles, esp_batch_t** out) {
  if (!out) return ESP_EINVAL;
  *out = nullptr;
  if (nrep < 1 || !h || !n || !tol) return ESP_EINVAL;
  esp_opts base;
  esp_opts_default(&base);
  if (o) base = *o;
  if (base.force != ESP_FORCE_AD) {
    std::fprintf(stderr, "esp_batch_plan: batched forces use analytic differentiation\n");
    return ESP_EINVAL;
  }
  std::unique_ptr<esp_batch_s> b(new (std::nothrow) esp_batch_s());
  if (!b) return ESP_ENOMEM;
  b->nrep = nrep;
  b->precision = base.precision;
  b->stream = static_cast<hipStream_t>(base.stream);
  b->reps.assign(nrep, nullptr);
  b->pofs.assign(nrep + 1, 0);
  esp_status warn = ESP_OK;
  for (int r = 0; r < nrep; ++r) {
    esp_opts opt = base;
    if (tiles) opt.tile = tiles[r];
    const esp_status st = esp_plan(h + 9 * r, n[r], tol[r], &opt, &b->reps[r]);
    if (st < 0) {
      std::fprintf(stderr, "esp_batch_plan: replica %d rejected (status %d)\n", r, st);
      return st;
    }
    if (st > 0) warn = st;
    b->pofs[r + 1] = b->pofs[r] + n[r];
  }
  b->order.resize(nrep);
  for (int r = 0; r < nrep; ++r) b->order[r] = r;
  std::stable_sort(b->order.begin(), b->order.end(), [&](int a, int c) {
    const esp_plan_t* pa = b->reps[a];
    const esp_plan_t* pc = b->reps[c];
    return pa->r.P != pc->r.P ? pa->r.P < pc->r.P : pa->nw < pc->nw;
  });
  b->pos.resize(nrep);
  for (int k = 0; k < nrep; ++k) b->pos[b->order[k]] = k;
  const esp_status st = b->precision == ESP_FP32 ? batch_build<float>(b.get()) : batch_build<double>(b.get());
  if (st != ESP_OK) {
    std::fprintf(stderr, "esp_batch_plan: %s\n", b->err.c_str());
    return st;
  }
  *out = b.release();
  return warn;
}

esp_status esp_batch_energy_virial(esp_batch_t* b, const float* xyz, const float* q, double* out7) {
  return batch_call<float>(b, xyz, q, nullptr, out7, false);
}

esp_status esp_batch_forces(esp_batch_t* b, const float* xyz, const float* q, float* f, double* out7) {
  return batch_call<float>(b, xyz, q, f, out7, true);
}

esp_status esp_batch_energy_virial_f64(esp_batch_t* b, const double* xyz, const double* q, double* out7) {
  return batch_call<double>(b, xyz, q, nullptr, out7, false);
}

esp_status esp_batch_forces_f64(esp_batch_t* b, const double* xyz, const double* q, double* f, double* out7) {
  return batch_call<double>(b, xyz, q, f, out7, true);
}

esp_status esp_batch_set_box(esp_batch_t* b, int r, const double h[9]) {
  if (!b || r < 0 || r >= b->nrep || !h) return ESP_EINVAL;
  const esp_status st = esp_set_box(b->reps[r], h);
  if (st < 0) {
    b->err = "replica " + std::to_string(r) + ": " + b->reps[r]->err;
    return st;
  }
  hipError_t e = hipSuccess;
  if (b->staged[r]) e = hipEventSynchronize(b->staged[r]);      // slot r free again
  else e = hipEventCreateWithFlags(&b->staged[r], hipEventDisableTiming);
  if (e != hipSuccess) return batch_fail(b, e, "box staging");
  unsigned char* slot = b->hstage + static_cast<size_t>(r) * b->plan_bytes;
  const size_t at = static_cast<size_t>(b->pos[r]) * b->plan_bytes;
  if (b->precision == ESP_FP32) {
    const DevPlan<float> d = batch_entry<float>(b, r);
    std::memcpy(slot, &d, sizeof d);
  } else {
    const DevPlan<double> d = batch_entry<double>(b, r);
    std::memcpy(slot, &d, sizeof d);
  }
  e = hipMemcpyAsync(static_cast<unsigned char*>(b->dplans) + at, slot, b->plan_bytes, hipMemcpyHostToDevice,
                     b->stream);
  if (e == hipSuccess) e = hipEventRecord(b->staged[r], b->stream);
  return e == hipSuccess ? st : batch_fail(b, e, "box upload");
}

esp_status esp_batch_set_stream(esp_batch_t* b, void* stream) {
  if (!b) return ESP_EINVAL;
  b->stream = static_cast<hipStream_t>(stream);
  return ESP_OK;
}

esp_status esp_batch_set_graph(esp_batch_t* b, int enable) {
  if (!b) return ESP_EINVAL;
  b->use_graph = enable != 0;
  if (!b->use_graph) {
    (void)hipStreamSynchronize(b->stream);
    b->drop_graph();
  }
  return ESP_OK;
}

esp_status esp_batch_check(esp_batch_t* b) {
  if (!b) return ESP_EINVAL;
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return batch_fail(b, e, "stream synchronise");
  esp_status worst = ESP_OK;
  for (int r = 0; r < b->nrep; ++r) {
    b->reps[r]->stream = b->stream;
    const esp_status st = esp_check(b->reps[r]);
    if (st != ESP_OK && (worst == ESP_OK || st == ESP_EDEVICE)) {
      worst = st;
      b->err = "replica " + std::to_string(r) + ": " + b->reps[r]->err;
    }
  }
  return worst;
}

esp_status esp_batch_get_params(const esp_batch_t* b, int r, esp_params* out) {
  if (!b || r < 0 || r >= b->nrep) return ESP_EINVAL;
  return esp_get_params(b->reps[r], out);
}

int esp_batch_num_launches(const esp_batch_t* b, int forces) {
  if (!b) return -1;
  const int groups = static_cast<int>(b->spread.size());
  const int sort = b->any_sub ? 3 : 2;
  return forces ? sort + groups + 3 + groups : sort + groups + 3;
}

const char* esp_batch_last_error(const esp_batch_t* b) { return b ? b->err.c_str() : "null batch"; }

void esp_batch_destroy(esp_batch_t* b) { delete b; }

}  // extern "C"
