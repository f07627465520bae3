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
#include <string>
#include <vector>

#include "../../include/esp.h"
#include "esp_device.h"
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

// Learned proposer hook (set from the learned-parameter module).
typedef int (*proposer_fn)(const double* features, int nfeat, double* out, void* ctx);
proposer_fn g_proposer = nullptr;
void* g_proposer_ctx = nullptr;

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
  std::memcpy(r.h, h, 9 * sizeof(double));
  esp_status st = check_box(h, r.rc, r.hinv, &r.V, err);
  if (st != ESP_OK) return st;

  esp_status warn = ESP_OK;
  int src = o->params;
  if (src == ESP_LEARNED) {
    bool ok = false;
    if (g_proposer) {
      // features: log10 tol, log10 N, edges / V^(1/3), coupling, rc
      double V13 = std::cbrt(r.V);
      double feat[8] = {std::log10(tol), std::log10(double(n)), col_norm(h, 0) / V13, col_norm(h, 1) / V13,
                        col_norm(h, 2) / V13, double(o->coupling), r.rc, n / r.V};
      double out[6];
      if (g_proposer(feat, 8, out, g_proposer_ctx) == 0) {
        // out: delta, P, sigma
        double dl = out[0];
        int P = static_cast<int>(std::lround(out[1]));
        double sg = out[2];
        if (dl >= 1e-14 && dl < 0.5 && P >= 2 && P <= kMaxP && sg >= 0.6 && sg <= 3.0) {
          r.delta = dl;
          r.c_split = r.c_spread = c_from_delta(dl);
          r.P = P;
          for (int d = 0; d < 3; ++d)
            r.M[d] = next_smooth(std::max({grid_rule(h, d, r.c_split, r.rc, sg), P, 2}));
          r.params_source = ESP_LEARNED;
          ok = true;
        }
      }
    }
    if (!ok) {
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
  return warn;
}

// radices for a 2,3,5-smooth length: 4s first, then a 2, then 3s and 5s
void factor(int n, FftLen& f) {
  f.n = n;
  f.nstage = 0;
  int m = n;
  while (m % 4 == 0) { f.rad[f.nstage++] = 4; m /= 4; }
  while (m % 2 == 0) { f.rad[f.nstage++] = 2; m /= 2; }
  while (m % 3 == 0) { f.rad[f.nstage++] = 3; m /= 3; }
  while (m % 5 == 0) { f.rad[f.nstage++] = 5; m /= 5; }
  if (n == 1) { f.rad[f.nstage++] = 1; }
}

}  // namespace

enum StageId { ST_BIN, ST_SCATTER, ST_SPREAD, ST_FFT_XY, ST_FFT_Z, ST_FFT_XY_INV, ST_GATHER, ST_COUNT };
const char* kStageNames[ST_COUNT] = {"bin", "scatter", "spread", "fft_xy", "fft_z", "fft_xy_inv", "gather"};

// Optional per-stage timing with HIP events recorded on the plan's stream.
struct Profiler {
  unsigned mask = 0;
  int cap = 0;
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
  int nw = 0, nw_fitted = 0, nker = 0;
  double A = 0, self_coef = 0, Ic = 0;
  hipStream_t stream = nullptr;
  std::vector<void*> allocs;
  DevPlan<float> d32{};
  DevPlan<double> d64{};
  std::string err;
  ~esp_plan_s() {
    prof.release();
    for (void* p : allocs) (void)hipFree(p);
  }
};

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
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) return hip_fail(p, e, "hipMalloc");
  p->allocs.push_back(q);
  *ptr = static_cast<T*>(q);
  return ESP_OK;
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

int fit_kernel(esp_plan_t* p, std::vector<double>& cf, std::vector<double>& cg) {
  const Pswf& ps = *p->split;
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
    if (err <= 1e-13 * ps.psi0()) return deg;
  }
  return kMaxKerDeg;
}

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
  d.cz = std::max(1, std::min(d.H, 256 / std::max(1, d.M3)));
  d.nzblk = ((d.H + d.cz - 1) / d.cz) * d.M2;
  d.nbin = static_cast<int>((r.n + 255) / 256);
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
  std::vector<double> cf, cg;
  p->nker = fit_kernel(p, cf, cg);
  d.nw = p->nw;
  d.nker = p->nker;
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
  const size_t o_win = push(win), o_kf = push(cf), o_kg = push(cg);
  const size_t o_i1 = push(iw[0]), o_i2 = push(iw[1]), o_i3 = push(iw[2]);
  R* dtab;
  Cplx<R>* dtw;
  esp_status st;
  if ((st = dalloc(p, &dtab, tab.size())) != ESP_OK) return st;
  if ((st = dalloc(p, &dtw, tw.size())) != ESP_OK) return st;
  hipError_t e = hipMemcpy(dtab, tab.data(), tab.size() * sizeof(R), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dtw, tw.data(), tw.size() * sizeof(Cplx<R>), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(p, e, "table upload");
  d.win = dtab + o_win;
  d.kerf = dtab + o_kf;
  d.kerg = dtab + o_kg;
  d.iw1 = dtab + o_i1;
  d.iw2 = dtab + o_i2;
  d.iw3 = dtab + o_i3;
  d.tw = dtw;

  // ---- LDS limits --------------------------------------------------------
  int dev_id = 0, maxlds = 65536;
  if (hipGetDevice(&dev_id) == hipSuccess)
    (void)hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev_id);
  const size_t need[3] = {lds_fft_xy(d), lds_fft_z(d), lds_spread(d)};
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
  if ((st = dalloc(p, &d.counts, r.ntiles)) || (st = dalloc(p, &d.offsets, r.ntiles + 1)) ||
      (st = dalloc(p, &d.keys, r.n)) || (st = dalloc(p, &d.ranks, r.n)) || (st = dalloc(p, &d.perm, r.n)) ||
      (st = dalloc(p, &d.tmp, r.n)) || (st = dalloc(p, &d.sorted, r.n)) || (st = dalloc(p, &d.rho, G)) ||
      (st = dalloc(p, &d.spec, S)) || (st = dalloc(p, &d.phi, G)) ||
      (st = dalloc(p, &d.zpart, static_cast<size_t>(d.nzblk) * kNumSums)) ||
      (st = dalloc(p, &d.qpart, static_cast<size_t>(d.nbin) * 2)) || (st = dalloc(p, &d.flags, 4)))
    return st;
  d.bin_lds = r.ntiles <= 8192 ? 1 : 0;
  e = hipMemset(d.counts, 0, r.ntiles * sizeof(int));
  if (e == hipSuccess) e = hipMemset(d.rho, 0, G * sizeof(R));
  if (e == hipSuccess) e = hipMemset(d.flags, 0, 4 * sizeof(int));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(p, e, "buffer initialisation");
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

// Launch one stage, bracketed by profiling events when that stage is profiled.
template <class F>
hipError_t stage(esp_plan_t* p, int st, F&& launch) {
  Profiler& pr = p->prof;
  const bool on = ((pr.mask >> st) & 1u) && pr.used[st] < pr.cap;
  if (on) (void)hipEventRecord(pr.ev[st][2 * pr.used[st]], p->stream);
  hipError_t e = launch();
  if (on) {
    (void)hipEventRecord(pr.ev[st][2 * pr.used[st] + 1], p->stream);
    ++pr.used[st];
  }
  return e;
}

// Cell sort.  Leaves the tile counts set; the spreading pass clears them.
template <typename R>
hipError_t run_sort(esp_plan_t* p, const R* xyz, const R* q) {
  DevPlan<R>& d = dev<R>(p);
  hipError_t e = stage(p, ST_BIN, [&] { return launch_bin(d, xyz, q, p->stream); });
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
  hipError_t e = stage(p, ST_FFT_XY, [&] { return launch_fft_xy(d, d.rho, d.spec, true, p->stream); });
  if (e == hipSuccess) e = stage(p, ST_FFT_Z, [&] { return launch_fft_z(d, Z_ENERGY, p->stream); });
  if (e == hipSuccess) e = launch_finalize(d, final_consts(p), out7, p->stream);
  return e == hipSuccess ? ESP_OK : hip_fail(p, e, "kernel launch");
}

template <typename R>
esp_status potential(esp_plan_t* p, const R* xyz, const R* q) {
  DevPlan<R>& d = dev<R>(p);
  esp_status st = run_sort_spread(p, xyz, q);
  if (st != ESP_OK) return st;
  hipError_t e = stage(p, ST_FFT_XY, [&] { return launch_fft_xy(d, d.rho, d.spec, true, p->stream); });
  if (e == hipSuccess) e = stage(p, ST_FFT_Z, [&] { return launch_fft_z(d, Z_POTENTIAL, p->stream); });
  if (e == hipSuccess) e = stage(p, ST_FFT_XY_INV, [&] { return launch_fft_xy_inv(d, p->stream); });
  return e == hipSuccess ? ESP_OK : hip_fail(p, e, "kernel launch");
}

template <typename R>
esp_status forces(esp_plan_t* p, const R* xyz, const R* q, R* f, double* out7) {
  if (!xyz || !q || !f) {
    p->err = "null pointer argument";
    return ESP_EINVAL;
  }
  esp_status st = potential(p, xyz, q);
  if (st != ESP_OK) return st;
  DevPlan<R>& d = dev<R>(p);
  hipError_t e = stage(p, ST_GATHER, [&] { return launch_gather(d, f, final_consts(p), out7, p->stream); });
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
  Pswf ps(r.c_split);
  out->lambda0_split = ps.lambda0();
  out->C0_split = ps.C0();
  out->psi0_split = ps.psi0();
  return st;
}

esp_status esp_plan(const double h[9], int64_t n, double tol, const esp_opts* o, esp_plan_t** out) {
  if (!out) return ESP_EINVAL;
  *out = nullptr;
  std::unique_ptr<esp_plan_s> p(new esp_plan_s());
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

esp_status esp_check(esp_plan_t* p) {
  if (!p) return ESP_EINVAL;
  hipError_t e = hipStreamSynchronize(p->stream);
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
  return ESP_OK;
}

const char* esp_last_error(const esp_plan_t* p) { return p ? p->err.c_str() : "null plan"; }

void esp_destroy(esp_plan_t* p) {
  if (!p) return;
  (void)hipStreamSynchronize(p->stream);
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
  if (e == hipSuccess) e = launch_fill(counts, p->r.ntiles, p->stream);
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
    e = hipMemcpyAsync(grid_out, p->d32.rho, G * sizeof(float), hipMemcpyDeviceToDevice, p->stream);
    if (e == hipSuccess) e = launch_fill(p->d32.rho, G, p->stream);
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

esp_status esp_profile_enable(esp_plan_t* p, unsigned stage_mask, int max_launches) {
  if (!p || max_launches < 0 || max_launches > (1 << 20)) return ESP_EINVAL;
  hipError_t e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return hip_fail(p, e, "stream synchronise");
  Profiler& pr = p->prof;
  pr.release();
  pr.mask = stage_mask & ((1u << ST_COUNT) - 1);
  pr.cap = pr.mask ? max_launches : 0;
  for (int s = 0; s < ST_COUNT; ++s) {
    pr.used[s] = 0;
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

const char* esp_version(void) { return "esp-mi355x 0.1.0 (gfx950)"; }

}  // extern "C"
