// Device helpers shared by the kernel translation units: complex arithmetic,
// the LDS Stockham FFT, block reductions, reduced coordinates and stencil
// placement, and the final FP64 sums.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "esp_device.h"

// Kernel launch; timed with the stage's events while its stage is profiled
// (see LaunchTiming).
#define ESP_LAUNCH(K, G, B, L, S, ...)                                                        \
  do {                                                                                        \
    ::espx::LaunchTiming& lt_ = ::espx::launch_timing();                                      \
    if (lt_.stop) {                                                                           \
      hipExtLaunchKernelGGL(K, G, B, L, S, lt_.start, lt_.stop, 0, __VA_ARGS__);              \
      lt_.start = nullptr;                                                                    \
    } else {                                                                                  \
      hipLaunchKernelGGL(K, G, B, L, S, __VA_ARGS__);                                         \
    }                                                                                         \
  } while (0)

namespace espx {

// ------------------------------------------------------------------ complex
template <typename R>
__device__ __forceinline__ Cplx<R> cadd(Cplx<R> a, Cplx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ Cplx<R> csub(Cplx<R> a, Cplx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ Cplx<R> cmul(Cplx<R> a, Cplx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ Cplx<R> cscale(Cplx<R> a, R s) { return {a.x * s, a.y * s}; }
// a + sgn * i * b
template <typename R>
__device__ __forceinline__ Cplx<R> cadd_i(Cplx<R> a, Cplx<R> b, R sgn) {
  return {a.x - sgn * b.y, a.y + sgn * b.x};
}

// ------------------------------------------------------------- butterflies
// sgn = -1: forward DFT (exp(-2 pi i jk/R)); sgn = +1: inverse (unnormalised).
template <typename R, int RAD>
struct Dft;

template <typename R>
struct Dft<R, 2> {
  __device__ static void run(Cplx<R>* v, R) {
    Cplx<R> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <typename R>
struct Dft<R, 3> {
  __device__ static void run(Cplx<R>* v, R sgn) {
    const R s60 = R(0.86602540378443864676);
    Cplx<R> t1 = cadd(v[1], v[2]);
    Cplx<R> t2 = csub(v[0], cscale(t1, R(0.5)));
    Cplx<R> t3 = cscale(csub(v[1], v[2]), s60);
    v[0] = cadd(v[0], t1);
    v[1] = cadd_i(t2, t3, sgn);
    v[2] = cadd_i(t2, t3, -sgn);
  }
};

template <typename R>
struct Dft<R, 4> {
  __device__ static void run(Cplx<R>* v, R sgn) {
    Cplx<R> a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    Cplx<R> b0 = cadd(v[1], v[3]), b1 = csub(v[1], v[3]);
    v[0] = cadd(a0, b0);
    v[2] = csub(a0, b0);
    v[1] = cadd_i(a1, b1, sgn);
    v[3] = cadd_i(a1, b1, -sgn);
  }
};

template <typename R>
struct Dft<R, 5> {
  __device__ static void run(Cplx<R>* v, R sgn) {
    const R c1 = R(0.30901699437494742410), c2 = R(-0.80901699437494742410);
    const R s1 = R(0.95105651629515357212), s2 = R(0.58778525229247312917);
    Cplx<R> t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    Cplx<R> t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    Cplx<R> a1 = {v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y};
    Cplx<R> a2 = {v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y};
    Cplx<R> b1 = {s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y};
    Cplx<R> b2 = {s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y};
    v[0] = cadd(v[0], cadd(t1, t2));
    v[1] = cadd_i(a1, b1, sgn);
    v[4] = cadd_i(a1, b1, -sgn);
    v[2] = cadd_i(a2, b2, sgn);
    v[3] = cadd_i(a2, b2, -sgn);
  }
};

// Radix 6 = 2 x 3: X[k] = E[k mod 3] + w^k O[k mod 3], w = exp(sgn 2 pi i / 6),
// with E, O the 3-point transforms of the even and odd samples.
template <typename R>
struct Dft<R, 6> {
  __device__ static void run(Cplx<R>* v, R sgn) {
    const R s60 = R(0.86602540378443864676);
    Cplx<R> e[3] = {v[0], v[2], v[4]}, o[3] = {v[1], v[3], v[5]};
    Dft<R, 3>::run(e, sgn);
    Dft<R, 3>::run(o, sgn);
    const Cplx<R> w1 = {R(0.5), sgn * s60}, w2 = {R(-0.5), sgn * s60};
    const Cplx<R> o1 = cmul(o[1], w1), o2 = cmul(o[2], w2);
    v[0] = cadd(e[0], o[0]);
    v[3] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[4] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[5] = csub(e[2], o2);
  }
};

// Radix 8 = 2 x 4, w = exp(sgn 2 pi i / 8).
template <typename R>
struct Dft<R, 8> {
  __device__ static void run(Cplx<R>* v, R sgn) {
    const R h = R(0.70710678118654752440);
    Cplx<R> e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    Dft<R, 4>::run(e, sgn);
    Dft<R, 4>::run(o, sgn);
    const Cplx<R> o1 = cmul(o[1], Cplx<R>{h, sgn * h});
    const Cplx<R> o2 = cadd_i(Cplx<R>{R(0), R(0)}, o[2], sgn);      // i sgn o2
    const Cplx<R> o3 = cmul(o[3], Cplx<R>{-h, sgn * h});
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

// floor(a / b) and a mod b for 0 <= a < 2^24, 1 <= b, with rb = 1 / b
// (a float product plus one integer correction instead of a division).
__device__ __forceinline__ int fast_div(int a, int b, float rb, int& rem) {
  int q = static_cast<int>(static_cast<float>(a) * rb);
  int r = a - q * b;
  if (r >= b) {
    ++q;
    r -= b;
  } else if (r < 0) {
    --q;
    r += b;
  }
  rem = r;
  return q;
}

// Division by a divisor fixed for the workgroup (grid sizes, column counts),
// for dividends 0 <= a < 2^24: fast_div with the reciprocal formed once.
struct Divisor {
  int b;
  float rb;
  __device__ explicit Divisor(int b_) : b(b_), rb(1.0f / static_cast<float>(b_)) {}
  __device__ __forceinline__ int div(int a, int& rem) const { return fast_div(a, b, rb, rem); }
};

// One Stockham stage of nlines independent length-n transforms held in LDS:
// element e of line l lives at base[l * lstride + e * estride].  Adjacent
// threads take adjacent elements of a line when elements are contiguous
// (estride 1), else adjacent lines (lstride 1), so LDS accesses stay
// unit-stride and free of bank conflicts either way.
// nth: threads of the workgroup (passed in, so that no stage re-reads the
// workgroup size from the dispatch packet).
template <typename R, int RAD>
__device__ void fft_stage(const Cplx<R>* __restrict__ in, Cplx<R>* __restrict__ out, int n, int Ns,
                          int nlines, int lstride, int estride, const Cplx<R>* __restrict__ tw,
                          R sgn, int nth) {
  const int nb = n / RAD;
  const int total = nlines * nb;
  const int tunit = n / (Ns * RAD);
  const bool by_line = estride != 1;
  const int inner = by_line ? nlines : nb;
  const float rin = 1.0f / static_cast<float>(inner), rns = 1.0f / static_cast<float>(Ns);
  for (int id = threadIdx.x; id < total; id += nth) {
    int rem, j;
    const int q = fast_div(id, inner, rin, rem);
    const int line = by_line ? rem : q;
    const int i = by_line ? q : rem;
    const int blk = fast_div(i, Ns, rns, j);
    const Cplx<R>* src = in + line * lstride;
    Cplx<R>* dst = out + line * lstride;
    Cplx<R> v[RAD];
#pragma unroll
    for (int r = 0; r < RAD; ++r) v[r] = src[(i + r * nb) * estride];
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < RAD; ++r) {
        Cplx<R> w = tw[tunit * j * r];      // j r < Ns RAD, so the index is < n
        w.y = sgn < 0 ? w.y : -w.y;
        v[r] = cmul(v[r], w);
      }
    }
    Dft<R, RAD>::run(v, sgn);
    const int ob = blk * Ns * RAD + j;
#pragma unroll
    for (int r = 0; r < RAD; ++r) dst[(ob + r * Ns) * estride] = v[r];
  }
  __syncthreads();
}

// All stages; ping-pongs between a and b and returns the buffer holding the result.
template <typename R>
__device__ __forceinline__ Cplx<R>* fft_lines(Cplx<R>* a, Cplx<R>* b, const FftLen& f, int nlines, int lstride,
                                              int estride, const Cplx<R>* tw, bool inverse, int nth) {
  const R sgn = inverse ? R(1) : R(-1);
  int Ns = 1;
  Cplx<R>* in = a;
  Cplx<R>* out = b;
  for (int s = 0; s < f.nstage; ++s) {
    switch (f.rad[s]) {
      case 2: fft_stage<R, 2>(in, out, f.n, Ns, nlines, lstride, estride, tw, sgn, nth); break;
      case 3: fft_stage<R, 3>(in, out, f.n, Ns, nlines, lstride, estride, tw, sgn, nth); break;
      case 4: fft_stage<R, 4>(in, out, f.n, Ns, nlines, lstride, estride, tw, sgn, nth); break;
      case 5: fft_stage<R, 5>(in, out, f.n, Ns, nlines, lstride, estride, tw, sgn, nth); break;
      case 6: fft_stage<R, 6>(in, out, f.n, Ns, nlines, lstride, estride, tw, sgn, nth); break;
      default: fft_stage<R, 8>(in, out, f.n, Ns, nlines, lstride, estride, tw, sgn, nth); break;
    }
    Ns *= f.rad[s];
    Cplx<R>* t = in;
    in = out;
    out = t;
  }
  return in;
}

// ------------------------------------------------------------- reductions
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One DPP step on a double (both 32-bit halves moved the same way); lanes of
// rows outside ROWMASK, or without a source lane, read 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_double(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, ROWMASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, ROWMASK, 0xf, false);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Sum over aligned groups of L lanes (L = 2, 4, 8 or 16), left in every lane
// of the group, with DPP moves only: quad swaps, then half-row and row
// mirrors (each pairs lanes of the two halves of the next larger group).
template <int CTRL>
__device__ __forceinline__ float dpp_float(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int L, typename R>
__device__ __forceinline__ R lane_group_sum(R v) {
  static_assert(L == 1 || L == 2 || L == 4 || L == 8 || L == 16, "groups within one DPP row");
  auto step = [](R x, auto ctrl) {
    constexpr int C = decltype(ctrl)::value;
    if constexpr (sizeof(R) == 8)
      return x + dpp_double<C, 0xf>(x);
    else
      return x + dpp_float<C>(x);
  };
  if constexpr (L >= 2) v = step(v, std::integral_constant<int, 0xb1>{});    // quad_perm [1, 0, 3, 2]
  if constexpr (L >= 4) v = step(v, std::integral_constant<int, 0x4e>{});    // quad_perm [2, 3, 0, 1]
  if constexpr (L >= 8) v = step(v, std::integral_constant<int, 0x141>{});   // row_half_mirror
  if constexpr (L >= 16) v = step(v, std::integral_constant<int, 0x140>{});  // row_mirror
  return v;
}

// Sum of a double over the 64 lanes, left in lane 63, with DPP moves only
// (no LDS permutes): quad swaps, half-row and row mirrors give every lane its
// row's sum; row broadcasts of lanes 15 and 31 then carry rows 0 + 1 and
// rows 0..2 into row 3.
__device__ __forceinline__ double wave_sum_to_last(double v) {
  v += dpp_double<0xb1, 0xf>(v);     // quad_perm [1, 0, 3, 2]
  v += dpp_double<0x4e, 0xf>(v);     // quad_perm [2, 3, 0, 1]
  v += dpp_double<0x141, 0xf>(v);    // row_half_mirror
  v += dpp_double<0x140, 0xf>(v);    // row_mirror
  v += dpp_double<0x142, 0xa>(v);    // row_bcast:15 into rows 1 and 3
  v += dpp_double<0x143, 0xc>(v);    // row_bcast:31 into rows 2 and 3
  return v;
}

// Orders a wave's LDS accesses on either side: what its lanes wrote before is
// seen by its lanes' accesses after (LDS operations of one wave complete in
// issue order; this keeps the compiler from moving accesses across it).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum of a float over the 64 lanes, left in lane 63 (DPP moves, as above).
__device__ __forceinline__ float wave_sum_to_last(float v) {
  v += dpp_float<0xb1>(v);
  v += dpp_float<0x4e>(v);
  v += dpp_float<0x141>(v);
  v += dpp_float<0x140>(v);
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xa, 0xf, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xc, 0xf, false));
  return v;
}

// Block-wide sums of NV doubles (fixed order, deterministic).  red: LDS of
// at least NV * 16 doubles.  Result valid in thread 0.
template <int NV>
__device__ void block_sum(double* v, double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum_to_last(v[k]);
  if (lane == 63)
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k * 16 + wid] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0;
      for (int w = 0; w < nw; ++w) s += red[k * 16 + w];
      v[k] = s;
    }
  }
}

// ----------------------------------------------------------- coordinates
// The error-free transformations below must not be contracted: a product
// fused into the subtraction of two_sum would be rounded differently from the
// product that fed the sum, and its rounding error would be counted twice.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
#pragma clang fp contract(off)
  s = a + b;
  float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// s_d = (h^-1 r)_d in float-float arithmetic, wrapped to [0, 1) and returned as
// 32-bit fixed point floor(frac(s_d) 2^32).
__device__ __forceinline__ uint32_t fixed_reduced(const float* hi, const float* lo, float x, float y,
                                                  float z) {
#pragma clang fp contract(off)
  const float r[3] = {x, y, z};
  float sh = 0.f, sl = 0.f;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    float p = hi[j] * r[j];
    float pe = fmaf(hi[j], r[j], -p);          // exact product error
    float t, e;
    two_sum(sh, p, t, e);
    sh = t;
    sl += e + pe + lo[j] * r[j];
  }
  float fh, e2;
  two_sum(sh, -floorf(sh), fh, e2);            // fractional part, error kept in e2
  sl += e2;
  const float scale = 4294967296.0f;           // 2^32
  float xh = fh * scale;                       // exact (power of two)
  float ih = floorf(xh);
  float rem = xh - ih;                         // exact
  float t = rem + sl * scale;
  long long S = static_cast<long long>(ih) + static_cast<long long>(floorf(t));
  return static_cast<uint32_t>(S & 0xffffffffLL);
}

// Stencil base g0 = ceil(u - P/2) (wrapped into [0, M)) and the local offset
// tau = u - g0 - (P-1)/2 in (-1/2, 1/2] of the first stencil point, from the
// fixed-point reduced coordinate S (u = M S / 2^32).
__device__ __forceinline__ void stencil_fixed(uint32_t S, int M, int P, int& gm, float& tau) {
  const long long U = static_cast<long long>(static_cast<unsigned long long>(M) * S);
  const long long a = U - (static_cast<long long>(P) << 31);
  const long long g0 = (a + 0xffffffffLL) >> 32;                    // ceil(a / 2^32)
  const long long tf = U - (g0 << 32) - (static_cast<long long>(P - 1) << 31);
  tau = static_cast<float>(tf) * 2.3283064365386963e-10f;           // 2^-32
  int g = static_cast<int>(g0);
  gm = g < 0 ? g + M : g;
}

// Not contracted: u = s M and u - P/2 are rounded separately, so that the tile
// key is a plain function of the FP64 reduced coordinate.
__device__ __forceinline__ void stencil_f64(double s, int M, int P, int& gm, double& tau) {
#pragma clang fp contract(off)
  const double u = s * M;
  const double g0 = ceil(u - 0.5 * P);
  tau = u - g0 - 0.5 * (P - 1);
  int g = static_cast<int>(g0);
  gm = g < 0 ? g + M : (g >= M ? g - M : g);
}

template <typename R>
struct Coord;

template <>
struct Coord<float> {
  __device__ static void make(const DevPlan<float>& d, float x, float y, float z, float q,
                              Record<float>& rec) {
#pragma unroll
    for (int k = 0; k < 3; ++k) rec.S[k] = fixed_reduced(d.hinv_hi + 3 * k, d.hinv_lo + 3 * k, x, y, z);
    rec.q = q;
  }
  __device__ static void stencil(const Record<float>& rec, int dim, int M, int P, int& gm, float& tau) {
    const uint32_t S = dim == 0 ? rec.S[0] : (dim == 1 ? rec.S[1] : rec.S[2]);
    stencil_fixed(S, M, P, gm, tau);
  }
  // real-space cell of s_dim among n equal cells: floor(n S / 2^32), exact
  __device__ static int cell(const Record<float>& rec, int dim, int n) {
    const uint32_t S = dim == 0 ? rec.S[0] : (dim == 1 ? rec.S[1] : rec.S[2]);
    return static_cast<int>((static_cast<unsigned long long>(S) * static_cast<unsigned>(n)) >> 32);
  }
  // reduced displacement a - b, minimum image in [-1/2, 1/2): the 32-bit
  // difference of the fixed-point coordinates wraps by itself
  __device__ static void disp(const Record<float>& a, const Record<float>& b, float* ds) {
#pragma unroll
    for (int k = 0; k < 3; ++k)
      ds[k] = static_cast<float>(static_cast<int>(a.S[k] - b.S[k])) * 2.3283064365386963e-10f;
  }
  // the same displacement in units of 2^-32 (unscaled)
  __device__ static void disp_raw(const Record<float>& a, const Record<float>& b, float* n) {
#pragma unroll
    for (int k = 0; k < 3; ++k) n[k] = static_cast<float>(static_cast<int>(a.S[k] - b.S[k]));
  }
};

template <>
struct Coord<double> {
  __device__ static void make(const DevPlan<double>& d, double x, double y, double z, double q,
                              Record<double>& rec) {
    // plain products and sums (no contraction): s = (h00 x + h01 y) + h02 z
#pragma clang fp contract(off)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      double s = d.hinv[3 * k] * x + d.hinv[3 * k + 1] * y + d.hinv[3 * k + 2] * z;
      s -= floor(s);
      rec.s[k] = s < 1.0 ? s : 0.0;
    }
    rec.q = q;
  }
  __device__ static void stencil(const Record<double>& rec, int dim, int M, int P, int& gm, double& tau) {
    const double sd = dim == 0 ? rec.s[0] : (dim == 1 ? rec.s[1] : rec.s[2]);
    stencil_f64(sd, M, P, gm, tau);
  }
  __device__ static int cell(const Record<double>& rec, int dim, int n) {
    const double sd = dim == 0 ? rec.s[0] : (dim == 1 ? rec.s[1] : rec.s[2]);
    return min(n - 1, static_cast<int>(sd * n));
  }
  __device__ static void disp(const Record<double>& a, const Record<double>& b, double* ds) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double v = a.s[k] - b.s[k];
      ds[k] = v - rint(v);
    }
  }
  __device__ static void disp_raw(const Record<double>& a, const Record<double>& b, double* n) { disp(a, b, n); }
};

template <typename R>
__device__ __forceinline__ bool finite_r(R v) { return isfinite(v); }

template <typename R>
__device__ __forceinline__ void atomic_add_global(R* p, R v) {
  unsafeAtomicAdd(p, v);
}

// Final FP64 sums: the z-pass block partials (eq. diag / eq. PFfinal summed
// over modes), the self-energy (eq. selfen) and, for a net charge, the
// neutralising-background terms (eq. Corr).  Run by one workgroup of a kernel
// launched after the z-pass, in a fixed order.
template <typename R>
__device__ void finalize_sums(const DevPlan<R>& d, double* __restrict__ out, double* red) {
  const FinalConsts& fc = d.fin;
  double v[kNumSums];
#pragma unroll
  for (int k = 0; k < kNumSums; ++k) v[k] = 0.0;
  for (int b = threadIdx.x; b < d.nzblk; b += blockDim.x)
#pragma unroll
    for (int k = 0; k < kNumSums; ++k) v[k] += d.zpart[static_cast<size_t>(b) * kNumSums + k];
  block_sum<kNumSums>(v, red);
  __syncthreads();
  double qv[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < d.nbin; b += blockDim.x) {
    qv[0] += d.qpart[3 * b];
    qv[1] += d.qpart[3 * b + 1];
  }
  block_sum<2>(qv, red + kNumSums * 16 - 32);
  if (threadIdx.x == 0) {
    const double Q = qv[0], Q2 = qv[1];
    const double Uself = -fc.self_coef * Q2;
    const double Ucorr = -fc.bg_coef * Q * Q;
    const double k = fc.coulomb_k;
    out[0] = k * (v[0] * fc.inv2V + Uself + Ucorr);
    out[1] = k * (v[1] * fc.inv2V + Ucorr);
    out[2] = k * (v[2] * fc.inv2V + Ucorr);
    out[3] = k * (v[3] * fc.inv2V + Ucorr);
    out[4] = k * v[4] * fc.inv2V;
    out[5] = k * v[5] * fc.inv2V;
    out[6] = k * v[6] * fc.inv2V;
  }
}


// The plan of the current workgroup and the block index within that plan's
// range: the kernel argument itself, or (batched launch) the plan whose block
// range holds blockIdx.x, found by bisection of the block offsets.
//
// Workgroup i of a launch is dispatched to XCD i mod 8 (round robin over the
// 8 XCDs, each with its own L2).  Blocks are renumbered so that each XCD
// takes runs of kXcdRun consecutive block numbers (tiles along x, column
// groups of a spectrum row): neighbours that read the same halo cells or the
// same 128-byte lines then share an L2, while the runs still alternate over
// the XCDs for load balance.  The ragged last round keeps its order.
__device__ __forceinline__ int xcd_block(int i, int n) {
  constexpr int X = kNumXcd, C = kXcdRun;
  const int full = n / (X * C) * (X * C);
  if (i >= full) return i;
  const int round = i / (X * C), k = i - round * X * C;
  return round * X * C + (k % X) * C + k / X;
}

// Batched launches read their plans from a device array that is written only
// between kernels, so a kernel may read it through the constant address
// space: uniform field reads then become scalar loads hoisted past the
// kernel's stores, as for kernel arguments.  (The integer round trip keeps
// the compiler from folding the two address-space casts away.)
template <typename R>
__device__ __forceinline__ const DevPlan<R>& plan_at(const DevPlan<R>* p) {
  using CP = const __attribute__((address_space(4))) DevPlan<R>*;
  return *(const DevPlan<R>*)(CP)reinterpret_cast<uintptr_t>(p);
}

template <typename R>
__device__ __forceinline__ const DevPlan<R>& plan_of(const KArg<R, false>& a, int& blk) {
  blk = xcd_block(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
  return a.d;
}
template <typename R>
__device__ __forceinline__ const DevPlan<R>& plan_of(const KArg<R, true>& a, int& blk) {
  const int b = xcd_block(static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x));
  int lo = 0, hi = a.nrep;                  // boff[lo] <= b < boff[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (a.boff[mid] <= b) lo = mid; else hi = mid;
  }
  blk = b - a.boff[lo];
  return plan_at(a.plans + lo);
}

// Spreading and gather launchers for one window support P (one translation
// unit per P, see esp_stencil.hip).
template <typename R, int P>
hipError_t spread_launch(const DevPlan<R>& d, hipStream_t s);
template <typename R, int P>
hipError_t gather_launch(const DevPlan<R>& d, R* f, double* out7, hipStream_t s);
template <typename R, int P>
hipError_t gather_ik_launch(const DevPlan<R>& d, R* f, double* out7, hipStream_t s);
template <typename R, int P>
hipError_t gather_local_launch(const DevPlan<R>& d, R* w6, double* out7, hipStream_t s);
template <typename R, int P>
hipError_t spread_launch_batch(const BatchLaunch<R>& b, hipStream_t s);
template <typename R, int P>
hipError_t gather_launch_batch(const BatchLaunch<R>& b, R* f, double* out7, hipStream_t s);

}  // namespace espx
