// gfx950 kernels of the ESP reciprocal-space path.
//
//   sort      bin (fixed-point reduced coordinates, tile key, rank), scan, scatter
//   spread    one workgroup per tile: PSWF weights, LDS accumulation, atomic write-back
//   fft_xy    one workgroup per z-plane: real-to-complex x transform (two rows per
//             complex transform), then the y transform, all in LDS (Stockham)
//   fft_z     one workgroup per group of x-columns: z transform fused with the
//             diagonal scaling / Fourier collection, and for forces the
//             multiplication by G and the inverse z transform
//   fft_xy_inv  inverse of fft_xy (complex-to-real)
//   gather    one thread per sorted particle: window gradient against phi
//   finalize  FP64 sums of the block partials plus self / background terms
//
// The spreading and stencil follow the paper's Sec. 4.2-4.3 with the base
// index g0 = ceil(u - P/2); the scaling follows eq. diag / eq. PFfinal; the
// force path follows App. C (analytic differentiation).
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "esp_device.h"

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

// One Stockham stage of nlines independent length-n transforms held in LDS:
// element e of line l lives at base[l * lstride + e * estride].
template <typename R, int RAD>
__device__ void fft_stage(const Cplx<R>* __restrict__ in, Cplx<R>* __restrict__ out, int n, int Ns,
                          int nlines, int lstride, int estride, const Cplx<R>* __restrict__ tw,
                          R sgn) {
  const int nb = n / RAD;
  const int total = nlines * nb;
  const int tunit = n / (Ns * RAD);
  for (int id = threadIdx.x; id < total; id += blockDim.x) {
    const int line = id / nb;
    const int i = id - line * nb;
    const int j = i % Ns;
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
    const int ob = (i / Ns) * Ns * RAD + j;
#pragma unroll
    for (int r = 0; r < RAD; ++r) dst[(ob + r * Ns) * estride] = v[r];
  }
  __syncthreads();
}

// All stages; ping-pongs between a and b and returns the buffer holding the result.
template <typename R>
__device__ Cplx<R>* fft_lines(Cplx<R>* a, Cplx<R>* b, const FftLen& f, int nlines, int lstride,
                              int estride, const Cplx<R>* tw, bool inverse) {
  const R sgn = inverse ? R(1) : R(-1);
  int Ns = 1;
  Cplx<R>* in = a;
  Cplx<R>* out = b;
  for (int s = 0; s < f.nstage; ++s) {
    switch (f.rad[s]) {
      case 2: fft_stage<R, 2>(in, out, f.n, Ns, nlines, lstride, estride, tw, sgn); break;
      case 3: fft_stage<R, 3>(in, out, f.n, Ns, nlines, lstride, estride, tw, sgn); break;
      case 4: fft_stage<R, 4>(in, out, f.n, Ns, nlines, lstride, estride, tw, sgn); break;
      default: fft_stage<R, 5>(in, out, f.n, Ns, nlines, lstride, estride, tw, sgn); break;
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

// Block-wide sums of NV doubles (fixed order, deterministic).  red: LDS of
// at least NV * (blockDim / 64) doubles.  Result valid in thread 0.
template <int NV>
__device__ void block_sum(double* v, double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0)
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
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// s_d = (h^-1 r)_d in float-float arithmetic, wrapped to [0, 1) and returned as
// 32-bit fixed point floor(frac(s_d) 2^32).
__device__ __forceinline__ uint32_t fixed_reduced(const float* hi, const float* lo, float x, float y,
                                                  float z) {
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

__device__ __forceinline__ void stencil_f64(double s, int M, int P, int& gm, double& tau) {
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
};

template <>
struct Coord<double> {
  __device__ static void make(const DevPlan<double>& d, double x, double y, double z, double q,
                              Record<double>& rec) {
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
};

template <typename R>
__device__ __forceinline__ bool finite_r(R v) { return isfinite(v); }

// ------------------------------------------------------------------- sort
template <typename R>
__global__ void __launch_bounds__(256) k_bin(DevPlan<R> d, const R* __restrict__ xyz,
                                             const R* __restrict__ q) {
  __shared__ double red[2 * 16];
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (i < d.n) {
    R x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2], qi = q[i];
    if (!(finite_r(x) && finite_r(y) && finite_r(z) && finite_r(qi))) {
      atomicOr(d.flags, 1);
      x = y = z = qi = R(0);
    }
    Record<R> rec;
    Coord<R>::make(d, x, y, z, qi, rec);
    d.tmp[i] = rec;
    int g1, g2, g3;
    R t;
    Coord<R>::stencil(rec, 0, d.M1, d.P, g1, t);
    Coord<R>::stencil(rec, 1, d.M2, d.P, g2, t);
    Coord<R>::stencil(rec, 2, d.M3, d.P, g3, t);
    const int key = ((g3 / d.T3) * d.nt2 + g2 / d.T2) * d.nt1 + g1 / d.T1;
    d.keys[i] = key;
    d.ranks[i] = atomicAdd(d.counts + key, 1);
    v[0] = static_cast<double>(qi);
    v[1] = static_cast<double>(qi) * static_cast<double>(qi);
  }
  block_sum<2>(v, red);
  if (threadIdx.x == 0) {
    d.qpart[2 * blockIdx.x] = v[0];
    d.qpart[2 * blockIdx.x + 1] = v[1];
  }
}

// Exclusive scan of the tile counts (one workgroup, fixed order); clears counts.
__global__ void __launch_bounds__(1024) k_scan(int* __restrict__ counts, int* __restrict__ offsets,
                                               int ntiles) {
  __shared__ int part[1024];
  const int nth = blockDim.x;
  const int chunk = (ntiles + nth - 1) / nth;
  const int b0 = threadIdx.x * chunk;
  const int b1 = min(ntiles, b0 + chunk);
  int s = 0;
  for (int k = b0; k < b1; ++k) s += counts[k];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int off = 1; off < nth; off <<= 1) {
    int add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  int run = part[threadIdx.x] - s;   // exclusive prefix of this chunk
  for (int k = b0; k < b1; ++k) {
    const int c = counts[k];
    offsets[k] = run;
    run += c;
    counts[k] = 0;
  }
  if (threadIdx.x == nth - 1) offsets[ntiles] = part[nth - 1];
}

template <typename R>
__global__ void __launch_bounds__(256) k_scatter(DevPlan<R> d) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const int pos = d.offsets[d.keys[i]] + d.ranks[i];
  d.sorted[pos] = d.tmp[i];
  d.perm[pos] = static_cast<int>(i);
}

// ----------------------------------------------------------------- window
// Value (and derivative) of the P window polynomials at tau, coefficients
// win[p * (nw + 1) + j] of tau^j.
template <typename R, int P>
__device__ __forceinline__ void window_weights(const R* __restrict__ win, int nw, R tau, R* w) {
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const R* c = win + p * (nw + 1);
    R v = c[nw];
    for (int j = nw - 1; j >= 0; --j) v = v * tau + c[j];
    w[p] = v;
  }
}

template <typename R, int P>
__device__ __forceinline__ void window_weights_d(const R* __restrict__ win, int nw, R tau, R* w, R* dw) {
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const R* c = win + p * (nw + 1);
    R v = c[nw], dv = R(0);
    for (int j = nw - 1; j >= 0; --j) {
      dv = dv * tau + v;
      v = v * tau + c[j];
    }
    w[p] = v;
    dw[p] = dv;
  }
}

// ----------------------------------------------------------------- spread
template <typename R>
__device__ __forceinline__ void atomic_add_global(R* p, R v) {
  unsafeAtomicAdd(p, v);
}

template <typename R, int P>
__global__ void __launch_bounds__(256) k_spread(DevPlan<R> d) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tile = blockIdx.x;
  const int start = d.offsets[tile], end = d.offsets[tile + 1];
  if (start == end) return;
  const int t1 = tile % d.nt1, t2 = (tile / d.nt1) % d.nt2, t3 = tile / (d.nt1 * d.nt2);
  const int o1 = t1 * d.T1, o2 = t2 * d.T2, o3 = t3 * d.T3;
  const int E1 = min(d.T1, d.M1 - o1) + P - 1;
  const int E2 = min(d.T2, d.M2 - o2) + P - 1;
  const int E3 = min(d.T3, d.M3 - o3) + P - 1;
  const int ncell = E1 * E2 * E3;
  const int maxcell = (d.T1 + P - 1) * (d.T2 + P - 1) * (d.T3 + P - 1);
  R* grid = reinterpret_cast<R*>(smem);
  R* wts = grid + maxcell;                           // kSpreadChunk x 3 x P
  R* win = wts + kSpreadChunk * 3 * P;               // P x (nw + 1)
  int* base = reinterpret_cast<int*>(win + P * (d.nw + 1));   // kSpreadChunk x 3
  for (int k = threadIdx.x; k < ncell; k += blockDim.x) grid[k] = R(0);
  for (int k = threadIdx.x; k < P * (d.nw + 1); k += blockDim.x) win[k] = d.win[k];
  __syncthreads();
  for (int c0 = start; c0 < end; c0 += kSpreadChunk) {
    const int nc = min(kSpreadChunk, end - c0);
    for (int t = threadIdx.x; t < nc * 3; t += blockDim.x) {
      const int j = t / 3, dim = t - 3 * j;
      const Record<R> rec = d.sorted[c0 + j];
      int gm;
      R tau;
      const int Md = dim == 0 ? d.M1 : (dim == 1 ? d.M2 : d.M3);
      const int od = dim == 0 ? o1 : (dim == 1 ? o2 : o3);
      Coord<R>::stencil(rec, dim, Md, P, gm, tau);
      R w[P];
      window_weights<R, P>(win, d.nw, tau, w);
      const R sc = dim == 0 ? rec.q : R(1);
#pragma unroll
      for (int p = 0; p < P; ++p) wts[(j * 3 + dim) * P + p] = w[p] * sc;
      base[j * 3 + dim] = gm - od;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nc * P * P; t += blockDim.x) {
      const int j = t / (P * P);
      const int r = t - j * P * P;
      const int cz = r / P, by = r - cz * P;
      const R* wj = wts + j * 3 * P;
      const R v = wj[P + by] * wj[2 * P + cz];
      R* row = grid + ((base[j * 3 + 2] + cz) * E2 + base[j * 3 + 1] + by) * E1 + base[j * 3];
#pragma unroll
      for (int a = 0; a < P; ++a) atomicAdd(row + a, v * wj[a]);
    }
    __syncthreads();
  }
  for (int k = threadIdx.x; k < ncell; k += blockDim.x) {
    const R val = grid[k];
    if (val != R(0)) {
      const int x = k % E1, y = (k / E1) % E2, z = k / (E1 * E2);
      int gx = o1 + x, gy = o2 + y, gz = o3 + z;
      gx -= gx >= d.M1 ? d.M1 : 0;
      gy -= gy >= d.M2 ? d.M2 : 0;
      gz -= gz >= d.M3 ? d.M3 : 0;
      atomic_add_global(d.rho + (static_cast<size_t>(gz) * d.M2 + gy) * d.M1 + gx, val);
    }
  }
}

// ------------------------------------------------------------------ FFT xy
template <typename R>
__global__ void __launch_bounds__(1024) k_fft_xy(DevPlan<R> d, const R* __restrict__ grid,
                                                 Cplx<R>* __restrict__ spec, int clear) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int M1 = d.M1, M2 = d.M2, H = d.H;
  const int npairs = (M2 + 1) / 2;
  const int L = max(npairs * M1, M2 * H);
  Cplx<R>* A = reinterpret_cast<Cplx<R>*>(smem);
  Cplx<R>* B = A + L;
  Cplx<R>* tw1 = B + L;
  Cplx<R>* tw2 = tw1 + M1;
  const int nth = blockDim.x, tid = threadIdx.x;
  for (int k = tid; k < M1; k += nth) tw1[k] = d.tw[d.f1.tw + k];
  for (int k = tid; k < M2; k += nth) tw2[k] = d.tw[d.f2.tw + k];
  const size_t zoff = static_cast<size_t>(blockIdx.x) * M2 * M1;
  const R* plane = grid + zoff;
  R* wplane = const_cast<R*>(grid) + zoff;
  for (int k = tid; k < npairs * M1; k += nth) {
    const int p = k / M1, x = k - p * M1;
    const int y0 = 2 * p;
    const R re = plane[y0 * M1 + x];
    const R im = y0 + 1 < M2 ? plane[(y0 + 1) * M1 + x] : R(0);
    A[k] = {re, im};
    if (clear) {
      wplane[y0 * M1 + x] = R(0);
      if (y0 + 1 < M2) wplane[(y0 + 1) * M1 + x] = R(0);
    }
  }
  __syncthreads();
  Cplx<R>* res = fft_lines(A, B, d.f1, npairs, M1, 1, tw1, false);
  Cplx<R>* oth = res == A ? B : A;
  // rows 2p (real part) and 2p+1 (imaginary part) were transformed together:
  // X_a[k] = (Z[k] + conj Z[-k]) / 2,  X_b[k] = (Z[k] - conj Z[-k]) / (2 i)
  for (int k = tid; k < npairs * H; k += nth) {
    const int p = k / H, m = k - p * H;
    const Cplx<R> Z = res[p * M1 + m];
    const Cplx<R> Zm = res[p * M1 + (m == 0 ? 0 : M1 - m)];
    oth[(2 * p) * H + m] = {R(0.5) * (Z.x + Zm.x), R(0.5) * (Z.y - Zm.y)};
    if (2 * p + 1 < M2) oth[(2 * p + 1) * H + m] = {R(0.5) * (Z.y + Zm.y), R(0.5) * (Zm.x - Z.x)};
  }
  __syncthreads();
  res = fft_lines(oth, res, d.f2, H, 1, H, tw2, false);
  Cplx<R>* out = spec + static_cast<size_t>(blockIdx.x) * M2 * H;
  for (int k = tid; k < M2 * H; k += nth) out[k] = res[k];
}

template <typename R>
__global__ void __launch_bounds__(1024) k_fft_xy_inv(DevPlan<R> d) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int M1 = d.M1, M2 = d.M2, H = d.H;
  const int npairs = (M2 + 1) / 2;
  const int L = max(npairs * M1, M2 * H);
  Cplx<R>* A = reinterpret_cast<Cplx<R>*>(smem);
  Cplx<R>* B = A + L;
  Cplx<R>* tw1 = B + L;
  Cplx<R>* tw2 = tw1 + M1;
  const int nth = blockDim.x, tid = threadIdx.x;
  for (int k = tid; k < M1; k += nth) tw1[k] = d.tw[d.f1.tw + k];
  for (int k = tid; k < M2; k += nth) tw2[k] = d.tw[d.f2.tw + k];
  const Cplx<R>* in = d.spec + static_cast<size_t>(blockIdx.x) * M2 * H;
  for (int k = tid; k < M2 * H; k += nth) A[k] = in[k];
  __syncthreads();
  Cplx<R>* res = fft_lines(A, B, d.f2, H, 1, H, tw2, true);
  Cplx<R>* oth = res == A ? B : A;
  // Hermitian rows a (= row 2p) and b (= row 2p+1): Z[x] = X_a[x] + i X_b[x]
  for (int k = tid; k < npairs * M1; k += nth) {
    const int p = k / M1, x = k - p * M1;
    const bool lo = x < H;
    const int xs = lo ? x : M1 - x;
    Cplx<R> a = res[(2 * p) * H + xs];
    Cplx<R> b = 2 * p + 1 < M2 ? res[(2 * p + 1) * H + xs] : Cplx<R>{R(0), R(0)};
    if (!lo) {
      a.y = -a.y;
      b.y = -b.y;
    }
    oth[k] = {a.x - b.y, a.y + b.x};
  }
  __syncthreads();
  res = fft_lines(oth, res, d.f1, npairs, M1, 1, tw1, true);
  R* plane = d.phi + static_cast<size_t>(blockIdx.x) * M2 * M1;
  for (int k = tid; k < npairs * M1; k += nth) {
    const int p = k / M1, x = k - p * M1;
    plane[(2 * p) * M1 + x] = res[k].x;
    if (2 * p + 1 < M2) plane[(2 * p + 1) * M1 + x] = res[k].y;
  }
}

// ------------------------------------------------------------------- FFT z
template <typename R>
__device__ __forceinline__ R chebyshev(const R* __restrict__ c, int deg, R z) {
  R b1 = R(0), b2 = R(0);
  for (int k = deg; k >= 1; --k) {
    const R b0 = R(2) * z * b1 - b2 + c[k];
    b2 = b1;
    b1 = b0;
  }
  return z * b1 - b2 + c[0];
}

// Compensated accumulator: FP32 Kahan sums for the production path, plain
// sums for FP64.
template <typename R>
struct Acc {
  R s = R(0), c = R(0);
  __device__ __forceinline__ void add(R v) {
    const R y = v - c;
    const R t = s + y;
    c = (t - s) - y;
    s = t;
  }
  __device__ __forceinline__ double value() const {
    return static_cast<double>(s) - static_cast<double>(c);
  }
};

template <typename R>
__global__ void __launch_bounds__(256) k_fft_z(DevPlan<R> d, int mode) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int M1 = d.M1, M2 = d.M2, M3 = d.M3, H = d.H, cz = d.cz;
  const int ngrp = (H + cz - 1) / cz;
  const int y = blockIdx.x / ngrp;
  const int k0 = (blockIdx.x - y * ngrp) * cz;
  const int nc = min(cz, H - k0);
  double* red = reinterpret_cast<double*>(smem);                   // kNumSums x 16
  Cplx<R>* A = reinterpret_cast<Cplx<R>*>(red + kNumSums * 16);
  Cplx<R>* B = A + cz * M3;
  Cplx<R>* tw3 = B + cz * M3;
  R* kf = reinterpret_cast<R*>(tw3 + M3);
  R* kg = kf + d.nker + 1;
  const int nth = blockDim.x, tid = threadIdx.x;
  for (int k = tid; k < M3; k += nth) tw3[k] = d.tw[d.f3.tw + k];
  for (int k = tid; k <= d.nker; k += nth) {
    kf[k] = d.kerf[k];
    kg[k] = d.kerg[k];
  }
  const size_t colstride = static_cast<size_t>(M2) * H;
  Cplx<R>* col = d.spec + static_cast<size_t>(y) * H + k0;
  for (int k = tid; k < nc * M3; k += nth) {
    const int z = k / nc, c = k - z * nc;
    A[k] = col[z * colstride + c];
  }
  __syncthreads();
  Cplx<R>* res = fft_lines(A, B, d.f3, nc, 1, nc, tw3, false);
  if (mode == Z_FFT_ONLY) {
    for (int k = tid; k < nc * M3; k += nth) {
      const int z = k / nc, c = k - z * nc;
      col[z * colstride + c] = res[k];
    }
    return;
  }
  Acc<R> acc[kNumSums];
  const int m2 = y <= (M2 - 1) / 2 ? y : y - M2;
  for (int k = tid; k < nc * M3; k += nth) {
    const int z = k / nc, c = k - z * nc;
    const int i1 = k0 + c;
    const int m1 = i1 <= (M1 - 1) / 2 ? i1 : i1 - M1;
    const int m3 = z <= (M3 - 1) / 2 ? z : z - M3;
    const Cplx<R> v = res[k];
    const R fm1 = R(m1), fm2 = R(m2), fm3 = R(m3);
    const R kx = d.B[0] * fm1 + d.B[1] * fm2 + d.B[2] * fm3;
    const R ky = d.B[3] * fm1 + d.B[4] * fm2 + d.B[5] * fm3;
    const R kz = d.B[6] * fm1 + d.B[7] * fm2 + d.B[8] * fm3;
    const R kk = kx * kx + ky * ky + kz * kz;
    const bool inside = (m1 | m2 | m3) != 0 && kk <= d.kcut2;
    R g = R(0);
    if (inside) {
      const R zc = R(2) * kk * d.ysc - R(1);
      const R f = chebyshev(kf, d.nker, zc);
      const R xg = chebyshev(kg, d.nker, zc);
      const R ik = R(1) / kk;
      const R Fh = d.A * f * ik;
      const R beta = (d.A * xg * ik - R(2) * Fh) * ik;
      const R iw = d.iw1[i1] * d.iw2[y] * d.iw3[z];
      const R wgt = (i1 == 0 || 2 * i1 == M1) ? R(1) : R(2);
      const R e = wgt * (v.x * v.x + v.y * v.y) * iw;
      const R Fe = Fh * e, be = beta * e;
      acc[0].add(Fe);
      acc[1].add(Fe + be * kx * kx);
      acc[2].add(Fe + be * ky * ky);
      acc[3].add(Fe + be * kz * kz);
      acc[4].add(be * kx * ky);
      acc[5].add(be * kx * kz);
      acc[6].add(be * ky * kz);
      g = Fh * iw * d.inv_vol;
    }
    if (mode == Z_POTENTIAL) res[k] = cscale(v, g);
  }
  double sums[kNumSums];
#pragma unroll
  for (int k = 0; k < kNumSums; ++k) sums[k] = acc[k].value();
  block_sum<kNumSums>(sums, red);
  if (tid == 0)
#pragma unroll
    for (int k = 0; k < kNumSums; ++k) d.zpart[static_cast<size_t>(blockIdx.x) * kNumSums + k] = sums[k];
  if (mode != Z_POTENTIAL) return;
  __syncthreads();
  Cplx<R>* oth = res == A ? B : A;
  res = fft_lines(res, oth, d.f3, nc, 1, nc, tw3, true);
  for (int k = tid; k < nc * M3; k += nth) {
    const int z = k / nc, c = k - z * nc;
    col[z * colstride + c] = res[k];
  }
}

// ------------------------------------------------------------------ gather
template <typename R, int P>
__global__ void __launch_bounds__(256) k_gather(DevPlan<R> d, R* __restrict__ f) {
  extern __shared__ __align__(16) unsigned char smem[];
  R* win = reinterpret_cast<R*>(smem);
  for (int k = threadIdx.x; k < P * (d.nw + 1); k += blockDim.x) win[k] = d.win[k];
  __syncthreads();
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const Record<R> rec = d.sorted[i];
  int g1, g2, g3;
  R t1, t2, t3;
  Coord<R>::stencil(rec, 0, d.M1, P, g1, t1);
  Coord<R>::stencil(rec, 1, d.M2, P, g2, t2);
  Coord<R>::stencil(rec, 2, d.M3, P, g3, t3);
  R w1[P], d1[P], w2[P], d2[P], w3[P], d3[P];
  window_weights_d<R, P>(win, d.nw, t1, w1, d1);
  window_weights_d<R, P>(win, d.nw, t2, w2, d2);
  window_weights_d<R, P>(win, d.nw, t3, w3, d3);
  int xi[P];
#pragma unroll
  for (int a = 0; a < P; ++a) {
    const int x = g1 + a;
    xi[a] = x >= d.M1 ? x - d.M1 : x;
  }
  R gx = R(0), gy = R(0), gz = R(0);
  for (int c = 0; c < P; ++c) {
    int z = g3 + c;
    z -= z >= d.M3 ? d.M3 : 0;
    R sx3 = R(0), s03 = R(0), sy3 = R(0);
#pragma unroll
    for (int b = 0; b < P; ++b) {
      int y = g2 + b;
      y -= y >= d.M2 ? d.M2 : 0;
      const R* row = d.phi + (static_cast<size_t>(z) * d.M2 + y) * d.M1;
      R sx = R(0), s0 = R(0);
#pragma unroll
      for (int a = 0; a < P; ++a) {
        const R v = row[xi[a]];
        sx += v * d1[a];
        s0 += v * w1[a];
      }
      sx3 += sx * w2[b];
      s03 += s0 * w2[b];
      sy3 += s0 * d2[b];
    }
    gx += sx3 * w3[c];
    gy += sy3 * w3[c];
    gz += s03 * d3[c];
  }
  const R qk = rec.q * d.coulomb_k;
  const int j = d.perm[i];
  f[3 * static_cast<int64_t>(j) + 0] = qk * (d.G[0] * gx + d.G[1] * gy + d.G[2] * gz);
  f[3 * static_cast<int64_t>(j) + 1] = qk * (d.G[3] * gx + d.G[4] * gy + d.G[5] * gz);
  f[3 * static_cast<int64_t>(j) + 2] = qk * (d.G[6] * gx + d.G[7] * gy + d.G[8] * gz);
}

// ---------------------------------------------------------------- finalize
template <typename R>
__global__ void __launch_bounds__(256) k_finalize(DevPlan<R> d, FinalConsts fc, double* __restrict__ out) {
  __shared__ double red[kNumSums * 16];
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
    qv[0] += d.qpart[2 * b];
    qv[1] += d.qpart[2 * b + 1];
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

template <typename R>
__global__ void k_fill(R* __restrict__ p, size_t count) {
  for (size_t k = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < count;
       k += static_cast<size_t>(gridDim.x) * blockDim.x)
    p[k] = R(0);
}

// ---------------------------------------------------------------- launchers
int fft_threads(int work) {
  if (work <= 2048) return 256;
  if (work <= 8192) return 512;
  return 1024;
}

template <typename R>
size_t lds_fft_xy(const DevPlan<R>& d) {
  const int npairs = (d.M2 + 1) / 2;
  const size_t L = static_cast<size_t>(std::max(npairs * d.M1, d.M2 * d.H));
  return (2 * L + d.M1 + d.M2) * sizeof(Cplx<R>);
}

template <typename R>
size_t lds_fft_z(const DevPlan<R>& d) {
  return (2 * static_cast<size_t>(d.cz) * d.M3 + d.M3) * sizeof(Cplx<R>) +
         (2 * (d.nker + 1) + 2) * sizeof(R) + kNumSums * 16 * sizeof(double) + 16;
}

template <typename R>
size_t lds_spread(const DevPlan<R>& d) {
  const size_t cells = static_cast<size_t>(d.T1 + d.P - 1) * (d.T2 + d.P - 1) * (d.T3 + d.P - 1);
  return (cells + kSpreadChunk * 3 * d.P + d.P * (d.nw + 1)) * sizeof(R) + kSpreadChunk * 3 * sizeof(int) + 16;
}

template <typename R>
hipError_t launch_bin(const DevPlan<R>& d, const R* xyz, const R* q, hipStream_t s) {
  hipLaunchKernelGGL(k_bin<R>, dim3(d.nbin), dim3(256), 0, s, d, xyz, q);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_scan(const DevPlan<R>& d, hipStream_t s) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, d.counts, d.offsets, d.ntiles);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_scatter(const DevPlan<R>& d, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter<R>, dim3(d.nbin), dim3(256), 0, s, d);
  return hipGetLastError();
}

template <typename R, int P>
static hipError_t spread_p(const DevPlan<R>& d, hipStream_t s) {
  const size_t lds = lds_spread(d);
  if (lds > 65536) (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_spread<R, P>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  hipLaunchKernelGGL((k_spread<R, P>), dim3(d.ntiles), dim3(256), lds, s, d);
  return hipGetLastError();
}

template <typename R, int P>
static hipError_t gather_p(const DevPlan<R>& d, R* f, hipStream_t s) {
  const int nb = static_cast<int>((d.n + 255) / 256);
  const size_t lds = P * (d.nw + 1) * sizeof(R);
  hipLaunchKernelGGL((k_gather<R, P>), dim3(nb), dim3(256), lds, s, d, f);
  return hipGetLastError();
}

#define ESP_P_SWITCH(FN, ...)                 \
  switch (d.P) {                              \
    case 2: return FN<R, 2>(__VA_ARGS__);     \
    case 3: return FN<R, 3>(__VA_ARGS__);     \
    case 4: return FN<R, 4>(__VA_ARGS__);     \
    case 5: return FN<R, 5>(__VA_ARGS__);     \
    case 6: return FN<R, 6>(__VA_ARGS__);     \
    case 7: return FN<R, 7>(__VA_ARGS__);     \
    case 8: return FN<R, 8>(__VA_ARGS__);     \
    case 9: return FN<R, 9>(__VA_ARGS__);     \
    case 10: return FN<R, 10>(__VA_ARGS__);   \
    case 11: return FN<R, 11>(__VA_ARGS__);   \
    case 12: return FN<R, 12>(__VA_ARGS__);   \
    default: return hipErrorInvalidValue;     \
  }

template <typename R>
hipError_t launch_spread(const DevPlan<R>& d, hipStream_t s) {
  ESP_P_SWITCH(spread_p, d, s)
}

template <typename R>
hipError_t launch_gather(const DevPlan<R>& d, R* f, hipStream_t s) {
  ESP_P_SWITCH(gather_p, d, f, s)
}

template <typename R>
hipError_t launch_fft_xy(const DevPlan<R>& d, const R* grid, Cplx<R>* spec, bool clear_input,
                         hipStream_t s) {
  const size_t lds = lds_fft_xy(d);
  if (lds > 65536) (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_xy<R>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  const int nth = fft_threads(d.M1 * d.M2);
  hipLaunchKernelGGL(k_fft_xy<R>, dim3(d.M3), dim3(nth), lds, s, d, grid, spec, clear_input ? 1 : 0);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_fft_xy_inv(const DevPlan<R>& d, hipStream_t s) {
  const size_t lds = lds_fft_xy(d);
  if (lds > 65536) (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_xy_inv<R>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  const int nth = fft_threads(d.M1 * d.M2);
  hipLaunchKernelGGL(k_fft_xy_inv<R>, dim3(d.M3), dim3(nth), lds, s, d);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_fft_z(const DevPlan<R>& d, ZMode mode, hipStream_t s) {
  const size_t lds = lds_fft_z(d);
  if (lds > 65536) (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_z<R>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  hipLaunchKernelGGL(k_fft_z<R>, dim3(d.nzblk), dim3(256), lds, s, d, static_cast<int>(mode));
  return hipGetLastError();
}

template <typename R>
hipError_t launch_finalize(const DevPlan<R>& d, FinalConsts c, double* out7, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize<R>, dim3(1), dim3(256), 0, s, d, c, out7);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_fill(R* p, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const int nb = static_cast<int>(std::min<size_t>((count + 255) / 256, 4096));
  hipLaunchKernelGGL(k_fill<R>, dim3(nb), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

#define ESP_INSTANTIATE(R)                                                                    \
  template hipError_t launch_bin<R>(const DevPlan<R>&, const R*, const R*, hipStream_t);      \
  template hipError_t launch_scan<R>(const DevPlan<R>&, hipStream_t);                         \
  template hipError_t launch_scatter<R>(const DevPlan<R>&, hipStream_t);                      \
  template hipError_t launch_spread<R>(const DevPlan<R>&, hipStream_t);                       \
  template hipError_t launch_fft_xy<R>(const DevPlan<R>&, const R*, Cplx<R>*, bool, hipStream_t); \
  template hipError_t launch_fft_z<R>(const DevPlan<R>&, ZMode, hipStream_t);                 \
  template hipError_t launch_fft_xy_inv<R>(const DevPlan<R>&, hipStream_t);                   \
  template hipError_t launch_gather<R>(const DevPlan<R>&, R*, hipStream_t);                   \
  template hipError_t launch_finalize<R>(const DevPlan<R>&, FinalConsts, double*, hipStream_t); \
  template hipError_t launch_fill<R>(R*, size_t, hipStream_t);                                \
  template size_t lds_fft_xy<R>(const DevPlan<R>&);                                           \
  template size_t lds_fft_z<R>(const DevPlan<R>&);                                            \
  template size_t lds_spread<R>(const DevPlan<R>&);

ESP_INSTANTIATE(float)
ESP_INSTANTIATE(double)

}  // namespace espx
