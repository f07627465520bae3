// PSWF spreading (paper Sec. 4.1 Step 1, Sec. 4.2-4.3) and the gather of the
// analytic-differentiation force (App. C), for one window support P.
//
// This file is compiled once per P (-DESP_P=2..12) so that the per-P
// instantiations build in parallel.  Every kernel is also specialised on the
// padded degree NW of the window polynomials (8, 12 or 16) so that the Horner
// loops unroll completely and the coefficient reads are issued up front.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "esp_common.h"

#ifndef ESP_P
#error "compile with -DESP_P=<window support>"
#endif

namespace espx {

// Window polynomials.  Coefficient-major table: win[j * P + p] multiplies
// tau^j in polynomial p (the window on the stencil point g0 + p, whose offset
// from the particle is tau + (P - 1)/2 - p).  psi is even and the P points
// lie symmetric about the particle, so polynomial P - 1 - q at tau is
// polynomial q at -tau: writing c_q(tau) = E(u) + tau O(u), u = tau^2 (even
// and odd coefficients), one evaluation of E and O gives both members of a
// mirror pair, E(u) +- tau O(u), in half the FMAs of evaluating each
// polynomial.  Only the tables of q < P/2 (and the middle one for odd P)
// are read.  NW is even: E has NW/2 + 1 coefficients, O has NW/2.
template <typename R, int NW>
__device__ __forceinline__ void even_odd(const R* __restrict__ c, int stride, R u, R& e, R& o) {
  static_assert(NW % 2 == 0, "even padded degree");
  e = c[NW * stride];
  o = c[(NW - 1) * stride];
#pragma unroll
  for (int j = NW - 2; j >= 0; j -= 2) {
    e = e * u + c[j * stride];
    if (j >= 2) o = o * u + c[(j - 1) * stride];
  }
}

// ... and with the derivatives E'(u), O'(u)
template <typename R, int NW>
__device__ __forceinline__ void even_odd_d(const R* __restrict__ c, int stride, R u, R& e, R& de, R& o, R& dO) {
  static_assert(NW % 2 == 0, "even padded degree");
  e = c[NW * stride];
  o = c[(NW - 1) * stride];
  de = R(0);
  dO = R(0);
#pragma unroll
  for (int j = NW - 2; j >= 0; j -= 2) {
    de = de * u + e;
    e = e * u + c[j * stride];
    if (j >= 2) {
      dO = dO * u + o;
      o = o * u + c[(j - 1) * stride];
    }
  }
}

// Values of the P window polynomials at tau.
template <typename R, int P, int NW>
__device__ __forceinline__ void eval_window(const R* __restrict__ win, R tau, R* w) {
  const R u = tau * tau;
#pragma unroll
  for (int q = 0; q < (P + 1) / 2; ++q) {
    R e, o;
    even_odd<R, NW>(win + q, P, u, e, o);
    const R to = tau * o;
    w[q] = e + to;
    if (P - 1 - q != q) w[P - 1 - q] = e - to;
  }
}

// Values and tau-derivatives: d/dtau [E(u) +- tau O(u)] = 2 tau E'(u) +-
// (O(u) + 2 u O'(u)).
template <typename R, int P, int NW>
__device__ __forceinline__ void window_pair_d(const R* __restrict__ win, int q, R tau, R& w, R& dw, R& wm, R& dwm) {
  const R u = tau * tau;
  R e, de, o, dO;
  even_odd_d<R, NW>(win + q, P, u, e, de, o, dO);
  const R to = tau * o;
  const R a = R(2) * tau * de, b = o + R(2) * u * dO;
  w = e + to;
  dw = a + b;
  wm = e - to;
  dwm = a - b;
}

// The 3 P window values and derivatives of one particle, shared out over its
// L lanes (mirror pair k = lane, lane + L, ...: dimension k / H, pair k % H,
// H = (P + 1) / 2), stored as my[2 d P + p] (value) and my[(2 d + 1) P + p]
// (derivative).
template <typename R, int P, int NW, int L>
__device__ __forceinline__ void window_d_lanes(const R* __restrict__ win, R t1, R t2, R t3, int lane, R* my) {
  constexpr int H = (P + 1) / 2;
#pragma unroll
  for (int r = 0; r < (3 * H + L - 1) / L; ++r) {
    const int k = lane + r * L;
    if (k < 3 * H) {
      const int dim = k / H, q = k - dim * H;
      const R tau = dim == 0 ? t1 : (dim == 1 ? t2 : t3);
      R v, dv, vm, dvm;
      window_pair_d<R, P, NW>(win, q, tau, v, dv, vm, dvm);
      my[2 * dim * P + q] = v;
      my[(2 * dim + 1) * P + q] = dv;
      if (P - 1 - q != q) {
        my[2 * dim * P + P - 1 - q] = vm;
        my[(2 * dim + 1) * P + P - 1 - q] = dvm;
      }
    }
  }
}

// Walk over the elements tid, tid + nth, tid + 2 nth, ... of a tile's
// E1 x E2 x E3 box (x fastest) that carries the box coordinates along: a step
// of nth adds fixed increments with at most one carry per coordinate, so
// only the first element costs divisions (the staging loops were dominated
// by three integer divisions per element).
struct BoxWalk {
  int k, x, y, z;
  int dx, dy, dz, E1, E2;
  // offset of (x, y, z) from the box origin in the grid, for boxes that do
  // not wrap around the periodic grid: advanced with the walk, so that such
  // a box is staged without per-element wrap tests or index products
  int off, doff, rowfix, planefix;
  bool wrap;                     // the box crosses the grid's upper edge in some dimension
  size_t base;                   // grid index of the box origin
  __device__ BoxWalk(int k0, int nth, int e1, int e2, int e3, int o1, int o2, int o3, int m1, int m2, int m3)
      : k(k0), E1(e1), E2(e2) {
    const int e12 = e1 * e2;
    z = k0 / e12;
    y = (k0 - z * e12) / e1;
    x = k0 - z * e12 - y * e1;
    dz = nth / e12;
    dy = (nth - dz * e12) / e1;
    dx = nth - dz * e12 - dy * e1;
    const int m12 = m1 * m2;
    off = z * m12 + y * m1 + x;
    doff = dz * m12 + dy * m1 + dx;
    rowfix = m1 - e1;
    planefix = m12 - e2 * m1;
    wrap = o1 + e1 > m1 || o2 + e2 > m2 || o3 + e3 > m3;
    base = (static_cast<size_t>(o3) * m2 + o2) * m1 + o1;
  }
  __device__ __forceinline__ void step(int nth) {
    k += nth;
    x += dx;
    y += dy;
    z += dz;
    off += doff;
    if (x >= E1) {
      x -= E1;
      ++y;
      off += rowfix;
    }
    if (y >= E2) {
      y -= E2;
      ++z;
      off += planefix;
    }
  }
};

// Stage the potential values of the box at grid point (o1, o2, o3) (periodic)
// into box[(z E2 + y) E1 + x]: rounds of U loads per thread, issued before
// their stores (elements past the box load the box's first value).  `first`
// stages only the first round, so that a kernel can put other loads behind
// it; `w` keeps the position for the remaining rounds.
template <typename R, int U>
__device__ __forceinline__ void stage_box_round(const DevPlan<R>& d, const R* __restrict__ src, R* __restrict__ box,
                                                BoxWalk& w, int nbox, int o1, int o2, int o3, int nth) {
  R v[U];
  int kk[U];
  if (!w.wrap) {
    const R* s0 = src + w.base;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      kk[u] = w.k;
      v[u] = s0[w.k < nbox ? w.off : 0];
      w.step(nth);
    }
  } else {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool in = w.k < nbox;
      int gx = o1 + (in ? w.x : 0), gy = o2 + (in ? w.y : 0), gz = o3 + (in ? w.z : 0);
      gx -= gx >= d.M1 ? d.M1 : 0;
      gy -= gy >= d.M2 ? d.M2 : 0;
      gz -= gz >= d.M3 ? d.M3 : 0;
      kk[u] = w.k;
      v[u] = src[(static_cast<size_t>(gz) * d.M2 + gy) * d.M1 + gx];
      w.step(nth);
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (kk[u] < nbox) box[kk[u]] = v[u];
}

// ----------------------------------------------------------------- spread
// Particles a spreading wave stages at a time, at most kWaveChunk (one weight
// task per (particle, dimension) lane): the size whose (particle, z offset)
// tasks fill the 64-lane accumulation passes best, i.e. the most particles per
// pass, c / ceil(c P / 64), the larger c on a tie (P = 6: 21, two passes of
// 63 tasks; P = 4: 16, one full pass, where 21 left a second pass of 20
// lanes; P = 5: 12; P = 7: 18; P = 8: 16).
constexpr int spread_chunk(int P) {
  int best = 1, num = 1, den = 1;                  // best particles per pass as num / den
  for (int c = 1; c <= kWaveChunk; ++c) {
    const int passes = (c * P + 63) / 64;
    if (c * den >= num * passes) {
      best = c;
      num = c;
      den = passes;
    }
  }
  return best;
}
static_assert(spread_chunk(6) == 21 && spread_chunk(4) == 16 && spread_chunk(7) == 18, "chunk sizes");

// One workgroup per tile of T1 x T2 x T3 grid cells.  Its particles (those
// whose stencil base lies in the tile, contiguous after the cell sort) are
// spread into an LDS copy of the tile plus its (P - 1)-wide upper halo, which
// is then added to the periodic grid.  The LDS tile accumulates in 8-byte
// cells (ds_add_f32 is several times slower on gfx950 than the 8-byte LDS
// adds):
//  * FIX = false: FP64 (ds_add_f64) of products formed in R.
//  * FIX = true: 64-bit fixed point (ds_add_u64).  The scale 2^e is the
//    tile's own: with b = wmax^3 sum |q_j| over its particles no cell can
//    exceed b in magnitude, and 2^e b <= 2^59 (FP32) or < 2^62 (FP64) keeps the int64
//    sums in range.  The integer sums are exact, so a cell does not depend
//    on the order of the atomics.  FP64 plans round each product q wx wy wz
//    2^e to an integer.  FP32 plans form each term as an exact integer
//    product: B_a = q wx_a 2^eq and A = wy wz 2^ka are rounded to int32
//    (|B|, |A| < 2^31; the float products before the rounding are the same
//    two roundings as the float path's), and A B 2^-s, s = eq + ka - e >= 1,
//    is taken with one rounding shift: two VALU instructions per term, and
//    faster than the FP64 tile on every tile shape measured.  For FP64 plans
//    the pass over the tile's charges and the longer f64 -> i64 rounding pay
//    only on crowded tiles.
template <typename R>
__device__ __forceinline__ long long to_fixed(R y) {
  return static_cast<long long>(rint(y));
}

template <typename R, int P, int NW, bool BATCH, bool FIX>
__global__ void __launch_bounds__(256) k_spread(KArg<R, BATCH> ka) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ float qabs[4];                          // FIX: per-wave sums of |q| (256 threads)
  constexpr bool IPROD = FIX && sizeof(R) == 4;      // integer-product terms (FP32)
  int tile;
  const DevPlan<R>& d = plan_of(ka, tile);
  const int t1 = tile % d.nt1, t2 = (tile / d.nt1) % d.nt2, t3 = tile / (d.nt1 * d.nt2);
  const int o1 = t1 * d.T1, o2 = t2 * d.T2, o3 = t3 * d.T3;
  const int E1 = min(d.T1, d.M1 - o1) + P - 1;
  const int E2 = min(d.T2, d.M2 - o2) + P - 1;
  const int E3 = min(d.T3, d.M3 - o3) + P - 1;
  // plane stride made odd: the P z-planes of one particle are touched by P
  // adjacent lanes, and an even stride of 8-byte cells maps them onto few banks
  const int S = (E1 * E2) | 1;
  const int ncell = S * E3;
  const int maxcell = (((d.T1 + P - 1) * (d.T2 + P - 1)) | 1) * (d.T3 + P - 1);
  using Cell = typename std::conditional<FIX, unsigned long long, double>::type;
  Cell* grid = reinterpret_cast<Cell*>(smem);
  R* wts = reinterpret_cast<R*>(grid + maxcell);     // per wave: kWaveChunk x 3 x P (IPROD: x slots hold B)
  R* win = wts + kSpreadWaves * kWaveChunk * 3 * P;  // (NW + 1) x P
  int* base = reinterpret_cast<int*>(win + (NW + 1) * P);   // per wave: kWaveChunk x 3
  int* shf = base + kSpreadWaves * kWaveChunk * 3;   // IPROD, per wave: kWaveChunk shifts s
  const int start = d.offsets[tile], end = d.offsets[tile + 1];
  const R wv = d.win[min(static_cast<int>(threadIdx.x), (NW + 1) * P - 1)];   // in flight with the offsets
  if (threadIdx.x == 0) d.counts[tile] = 0;        // ready for the next binning pass
  if (start == end) return;
  // Each wave spreads chunks of csz particles of its own (chunk c of the
  // tile goes to wave c mod 4): its lanes evaluate the chunk's weights (one
  // task per (particle, dimension)), stage them in the wave's LDS slots and
  // then add the chunk's (particle, z offset) tasks into the shared tile.
  // Only the tile clear and the write-back are workgroup barriers, so one
  // wave's weight evaluation overlaps another's LDS atomics.
  // The chunk size and the wave index are read into scalar registers, so the
  // chunk loop below is a uniform (scalar) loop of the wave.  Held in vector
  // registers they made it a divergent loop, whose compiled form gave wrong
  // grids for P = 8 with fewer than 21 particles per chunk (measured).
  static_assert(kWaveChunk * 3 <= 64, "one weight task per lane");
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  const int n = end - start;
  const int csz = __builtin_amdgcn_readfirstlane(max(1, min(spread_chunk(P), (n + kSpreadWaves - 1) / kSpreadWaves)));
  const int step = kSpreadWaves * csz;
  R* wts_w = wts + wave * kWaveChunk * 3 * P;
  int* base_w = base + wave * kWaveChunk * 3;
  int* shf_w = shf + wave * kWaveChunk;
  const int tj = lane / 3, tdim = lane - 3 * (lane / 3);
  int c0 = start + wave * csz;
  Record<R> rec;
  if (c0 < end && tj < min(csz, end - c0)) rec = d.sorted[c0 + tj];
  float qs = 0.f;
  if constexpr (FIX)
    for (int k = start + threadIdx.x; k < end; k += blockDim.x) qs += fabsf(static_cast<float>(d.sorted[k].q));
  for (int k = threadIdx.x; k < ncell; k += blockDim.x) grid[k] = Cell(0);
  if (static_cast<int>(threadIdx.x) < (NW + 1) * P) win[threadIdx.x] = wv;
  for (int k = threadIdx.x + blockDim.x; k < (NW + 1) * P; k += blockDim.x) win[k] = d.win[k];
  if constexpr (FIX) {
    qs = wave_sum_to_last(qs);
    if ((threadIdx.x & 63) == 63) qabs[threadIdx.x >> 6] = qs;
  }
  __syncthreads();
  R scale = R(1);
  double unscale = 1.0;
  int e = 0, kA = 0;
  if constexpr (FIX) {
    // the float sum of |q| is within n 2^-24 (relative) of the exact one,
    // far inside the margins of the exponents below
    const float bnd = (qabs[0] + qabs[1] + qabs[2] + qabs[3]) * d.wmax3;
    e = max(-100, min(120, (IPROD ? 58 : 61) - ilogbf(fmaxf(bnd, 1e-30f))));
    scale = static_cast<R>(ldexpf(1.f, e));
    unscale = ldexp(1.0, -e);
    kA = 30 - ilogbf(d.wmax * d.wmax);               // |wy wz| 2^kA < 2^31
  }
  for (; c0 < end; c0 += step) {
    const int nc = min(csz, end - c0);
    // weights: q (and the fixed-point scale) folded into x
    if (tj < nc) {
      const int j = tj, dim = tdim;
      int gm;
      R tau;
      const int Md = dim == 0 ? d.M1 : (dim == 1 ? d.M2 : d.M3);
      const int od = dim == 0 ? o1 : (dim == 1 ? o2 : o3);
      Coord<R>::stencil(rec, dim, Md, P, gm, tau);
      R w[P];
      eval_window<R, P, NW>(win, tau, w);
      if constexpr (IPROD) {
        if (dim == 0) {
          // B_p = q w_p 2^eq with |q| wmax 2^eq < 2^31; s = eq + kA - e
          const float qa = fabsf(static_cast<float>(rec.q)) * d.wmax;
          const int eq = qa > 0.f ? 30 - ilogbf(qa) : 0;
          const float sq = ldexpf(static_cast<float>(rec.q), eq);
          int* bw = reinterpret_cast<int*>(wts_w + j * 3 * P);
#pragma unroll
          for (int p = 0; p < P; ++p) bw[p] = __float2int_rn(static_cast<float>(w[p]) * sq);
          shf_w[j] = qa > 0.f ? max(0, min(63, eq + kA - e)) : 0;
        } else {
          const R sc = dim == 2 ? static_cast<R>(ldexpf(1.f, kA)) : R(1);
#pragma unroll
          for (int p = 0; p < P; ++p) wts_w[(j * 3 + dim) * P + p] = w[p] * sc;
        }
      } else {
        const R sc = dim == 0 ? (FIX ? rec.q * scale : rec.q) : R(1);
#pragma unroll
        for (int p = 0; p < P; ++p) wts_w[(j * 3 + dim) * P + p] = w[p] * sc;
      }
      base_w[j * 3 + dim] = gm - od;
    }
    wave_lds_sync();
    {
      const int c1 = c0 + step;
      if (c1 < end && tj < min(csz, end - c1)) rec = d.sorted[c1 + tj];
    }
    // accumulation: one task per (particle, z offset), the P x P block of that plane
    for (int t = lane; t < nc * P; t += 64) {
      const int j = t / P, cz = t - j * P;
      const R* wj = wts_w + j * 3 * P;
      R wy[P];
#pragma unroll
      for (int a = 0; a < P; ++a) wy[a] = wj[P + a];
      const R wz = wj[2 * P + cz];
      Cell* plane = grid + (base_w[j * 3 + 2] + cz) * S + base_w[j * 3 + 1] * E1 + base_w[j * 3];
      if constexpr (IPROD) {
        const int* bj = reinterpret_cast<const int*>(wj);
        int bx[P];
#pragma unroll
        for (int a = 0; a < P; ++a) bx[a] = bj[a];
        const int sh = shf_w[j];
        const long long rnd = sh > 0 ? (1ll << (sh - 1)) : 0ll;
#pragma unroll
        for (int by = 0; by < P; ++by) {
          const long long A = __float2int_rn(static_cast<float>(wy[by] * wz));
#pragma unroll
          for (int a = 0; a < P; ++a)
            atomicAdd(plane + by * E1 + a, static_cast<unsigned long long>((A * bx[a] + rnd) >> sh));
        }
      } else {
        R wx[P];
#pragma unroll
        for (int a = 0; a < P; ++a) wx[a] = wj[a];
#pragma unroll
        for (int by = 0; by < P; ++by) {
          const R v = wy[by] * wz;
#pragma unroll
          for (int a = 0; a < P; ++a) {
            if constexpr (FIX)
              atomicAdd(plane + by * E1 + a, static_cast<unsigned long long>(to_fixed(v * wx[a])));
            else
              atomicAdd(plane + by * E1 + a, static_cast<double>(v * wx[a]));
          }
        }
      }
    }
    // the next chunk's weight writes come after this chunk's reads
    wave_lds_sync();
  }
  __syncthreads();
  // write-back: each thread owns one (x, y) column of the tile and walks z.
  // Deterministic FP32 plans: the tile's integers, rescaled from 2^e to the
  // grid's 2^gexp by a rounding shift, are added to the int64 grid (order-
  // independent sums); otherwise the cells are added to the R grid.
  const int E12 = E1 * E2;
  const size_t planesz = static_cast<size_t>(d.M1) * d.M2;
  if (IPROD && d.grid_fixed) {
    const int sh = max(0, min(63, e - d.gexp[0]));    // >= 1 unless both scales are clamped
    const long long half = sh > 0 ? (1ll << (sh - 1)) : 0ll;
    for (int k0 = threadIdx.x; k0 < E12; k0 += blockDim.x) {
      const int y = k0 / E1, x = k0 - y * E1;
      int gx = o1 + x, gy = o2 + y;
      gx -= gx >= d.M1 ? d.M1 : 0;
      gy -= gy >= d.M2 ? d.M2 : 0;
      unsigned long long* col =
          reinterpret_cast<unsigned long long*>(d.rhofix) + static_cast<size_t>(gy) * d.M1 + gx;
      for (int z = 0; z < E3; ++z) {
        const long long v = static_cast<long long>(grid[z * S + k0]);
        const long long g = sh == 63 ? 0ll : (v + half) >> sh;
        int gz = o3 + z;
        gz -= gz >= d.M3 ? d.M3 : 0;
        if (g != 0) atomicAdd(col + gz * planesz, static_cast<unsigned long long>(g));
      }
    }
    return;
  }
  for (int k0 = threadIdx.x; k0 < E12; k0 += blockDim.x) {
    const int y = k0 / E1, x = k0 - y * E1;
    int gx = o1 + x, gy = o2 + y;
    gx -= gx >= d.M1 ? d.M1 : 0;
    gy -= gy >= d.M2 ? d.M2 : 0;
    R* col = d.rho + static_cast<size_t>(gy) * d.M1 + gx;
    for (int z = 0; z < E3; ++z) {
      R val;
      if constexpr (FIX)
        val = static_cast<R>(static_cast<double>(static_cast<long long>(grid[z * S + k0])) * unscale);
      else
        val = static_cast<R>(grid[z * S + k0]);
      int gz = o3 + z;
      gz -= gz >= d.M3 ? d.M3 : 0;
      if (val != R(0)) atomic_add_global(col + gz * planesz, val);
    }
  }
}

// ------------------------------------------------------------------ gather
// L = 2^k >= P lanes per particle.  Lanes 0..2 evaluate the P window values
// and derivatives of one dimension each and stage them in LDS; lane c < P
// then sums z-plane c of the stencil against phi; the L partial gradients are
// reduced with DPP lane moves.  F = q G grad_u, G = -h^-T diag(M).
template <int P>
struct GatherLanes {
  static constexpr int L = gather_lanes(P);
};

template <typename R, int P, int NW, bool BATCH>
__global__ void __launch_bounds__(256) k_gather(KArg<R, BATCH> ka, R* __restrict__ f,
                                                double* __restrict__ out7) {
  constexpr int L = GatherLanes<P>::L;
  constexpr int G = 256 / L;                          // particles per block
  int blk;
  const DevPlan<R>& d = plan_of(ka, blk);
  f += 3 * d.pofs;
  if (out7 && blk == 0) {
    __shared__ double red[kNumSums * 16];
    finalize_sums(d, out7 + kNumSums * d.rep, red);
  }
  extern __shared__ __align__(16) unsigned char smem[];
  R* win = reinterpret_cast<R*>(smem);                // (NW + 1) x P
  R* wt = win + (NW + 1) * P;                         // G x 6 x P: w1 d1 w2 d2 w3 d3
  // the particle's record and destination are fetched before the table
  // barrier, so the two global round trips overlap
  const int grp = threadIdx.x / L, lane = threadIdx.x - grp * L;
  const int64_t i = static_cast<int64_t>(blk) * G + grp;
  const bool valid = i < d.n;
  const Record<R> rec = d.sorted[valid ? i : 0];
  const int64_t j = valid ? d.perm[i] : 0;
  for (int k = threadIdx.x; k < (NW + 1) * P; k += blockDim.x) win[k] = d.win[k];
  __syncthreads();
  int g1, g2, g3;
  R t1, t2, t3;
  Coord<R>::stencil(rec, 0, d.M1, P, g1, t1);
  Coord<R>::stencil(rec, 1, d.M2, P, g2, t2);
  Coord<R>::stencil(rec, 2, d.M3, P, g3, t3);
  R* my = wt + grp * 6 * P;
  window_d_lanes<R, P, NW, L>(win, t1, t2, t3, lane, my);
  __syncthreads();
  R gx = R(0), gy = R(0), gz = R(0);
  if (lane < P) {
    int xi[P];
#pragma unroll
    for (int a = 0; a < P; ++a) {
      const int x = g1 + a;
      xi[a] = x >= d.M1 ? x - d.M1 : x;
    }
    R w1[P], d1[P];
#pragma unroll
    for (int a = 0; a < P; ++a) {
      w1[a] = my[a];
      d1[a] = my[P + a];
    }
    int z = g3 + lane;
    z -= z >= d.M3 ? d.M3 : 0;
    R sxz = R(0), syz = R(0), s0z = R(0);
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
      const R w2 = my[2 * P + b], d2 = my[3 * P + b];
      sxz += sx * w2;
      s0z += s0 * w2;
      syz += s0 * d2;
    }
    gx = sxz * my[4 * P + lane];
    gy = syz * my[4 * P + lane];
    gz = s0z * my[5 * P + lane];
  }
  gx = lane_group_sum<L>(gx);
  gy = lane_group_sum<L>(gy);
  gz = lane_group_sum<L>(gz);
  if (lane == 0 && valid) {
    const R qk = rec.q * d.coulomb_k;
    f[3 * j + 0] = qk * (d.G[0] * gx + d.G[1] * gy + d.G[2] * gz);
    f[3 * j + 1] = qk * (d.G[3] * gx + d.G[4] * gy + d.G[5] * gz);
    f[3 * j + 2] = qk * (d.G[6] * gx + d.G[7] * gy + d.G[8] * gz);
  }
}

// Gather of the ik-differentiated field (App. C, eq. rhodiagforce): the three
// Cartesian components E_a of the gradient of the smoothed potential are
// separate grids (phi + a M1 M2 M3); the force is F = -q sum_g W(u - g) E(g)
// with the plain window.  Lane layout as in k_gather.
template <typename R, int P, int NW, bool BATCH>
__global__ void __launch_bounds__(256) k_gather_ik(KArg<R, BATCH> ka, R* __restrict__ f,
                                                   double* __restrict__ out7) {
  constexpr int L = GatherLanes<P>::L;
  constexpr int G = 256 / L;
  int blk;
  const DevPlan<R>& d = plan_of(ka, blk);
  f += 3 * d.pofs;
  if (out7 && blk == 0) {
    __shared__ double red[kNumSums * 16];
    finalize_sums(d, out7 + kNumSums * d.rep, red);
  }
  extern __shared__ __align__(16) unsigned char smem[];
  R* win = reinterpret_cast<R*>(smem);                // (NW + 1) x P
  R* wt = win + (NW + 1) * P;                         // G x 3 x P: w1 w2 w3
  // the particle's record and destination are fetched before the table
  // barrier, so the two global round trips overlap
  const int grp = threadIdx.x / L, lane = threadIdx.x - grp * L;
  const int64_t i = static_cast<int64_t>(blk) * G + grp;
  const bool valid = i < d.n;
  const Record<R> rec = d.sorted[valid ? i : 0];
  const int64_t j = valid ? d.perm[i] : 0;
  for (int k = threadIdx.x; k < (NW + 1) * P; k += blockDim.x) win[k] = d.win[k];
  __syncthreads();
  int g1, g2, g3;
  R t1, t2, t3;
  Coord<R>::stencil(rec, 0, d.M1, P, g1, t1);
  Coord<R>::stencil(rec, 1, d.M2, P, g2, t2);
  Coord<R>::stencil(rec, 2, d.M3, P, g3, t3);
  R* my = wt + grp * 3 * P;
  if (lane < 3) {
    R w[P];
    eval_window<R, P, NW>(win, lane == 0 ? t1 : (lane == 1 ? t2 : t3), w);
#pragma unroll
    for (int p = 0; p < P; ++p) my[lane * P + p] = w[p];
  }
  __syncthreads();
  R ex = R(0), ey = R(0), ez = R(0);
  if (lane < P) {
    const size_t G3 = static_cast<size_t>(d.M1) * d.M2 * d.M3;
    int xi[P];
#pragma unroll
    for (int a = 0; a < P; ++a) {
      const int x = g1 + a;
      xi[a] = x >= d.M1 ? x - d.M1 : x;
    }
    R w1[P];
#pragma unroll
    for (int a = 0; a < P; ++a) w1[a] = my[a];
    int z = g3 + lane;
    z -= z >= d.M3 ? d.M3 : 0;
#pragma unroll
    for (int b = 0; b < P; ++b) {
      int y = g2 + b;
      y -= y >= d.M2 ? d.M2 : 0;
      const R* row = d.phi + (static_cast<size_t>(z) * d.M2 + y) * d.M1;
      R sx = R(0), sy = R(0), sz = R(0);
#pragma unroll
      for (int a = 0; a < P; ++a) {
        sx += row[xi[a]] * w1[a];
        sy += row[G3 + xi[a]] * w1[a];
        sz += row[2 * G3 + xi[a]] * w1[a];
      }
      const R w2 = my[P + b];
      ex += sx * w2;
      ey += sy * w2;
      ez += sz * w2;
    }
    const R w3 = my[2 * P + lane];
    ex *= w3;
    ey *= w3;
    ez *= w3;
  }
  ex = lane_group_sum<L>(ex);
  ey = lane_group_sum<L>(ey);
  ez = lane_group_sum<L>(ez);
  if (lane == 0 && valid) {
    const R qk = -rec.q * d.coulomb_k;
    f[3 * j + 0] = qk * ex;
    f[3 * j + 1] = qk * ey;
    f[3 * j + 2] = qk * ez;
  }
}

// Per-particle Fourier virial (Sec. 4.4, eq. PinsFind): the six grids
// Pi_c = inverse FFT of P_hat_c rho_hat / (2 V W_hat^2) (phi + c M1 M2 M3) are
// gathered with the plain window; w6[6 j + c] = q_j sum_g W(u_j - g) Pi_c(g),
// components xx, yy, zz, xy, xz, yz, in input order.  Lane layout as in
// k_gather.
template <typename R, int P, int NW, bool BATCH>
__global__ void __launch_bounds__(256) k_gather_local(KArg<R, BATCH> ka, R* __restrict__ w6,
                                                      double* __restrict__ out7) {
  constexpr int L = GatherLanes<P>::L;
  constexpr int G = 256 / L;
  int blk;
  const DevPlan<R>& d = plan_of(ka, blk);
  w6 += 6 * d.pofs;
  if (out7 && blk == 0) {
    __shared__ double red[kNumSums * 16];
    finalize_sums(d, out7 + kNumSums * d.rep, red);
  }
  extern __shared__ __align__(16) unsigned char smem[];
  R* win = reinterpret_cast<R*>(smem);                // (NW + 1) x P
  R* wt = win + (NW + 1) * P;                         // G x 3 x P: w1 w2 w3
  // the particle's record and destination are fetched before the table
  // barrier, so the two global round trips overlap
  const int grp = threadIdx.x / L, lane = threadIdx.x - grp * L;
  const int64_t i = static_cast<int64_t>(blk) * G + grp;
  const bool valid = i < d.n;
  const Record<R> rec = d.sorted[valid ? i : 0];
  const int64_t j = valid ? d.perm[i] : 0;
  for (int k = threadIdx.x; k < (NW + 1) * P; k += blockDim.x) win[k] = d.win[k];
  __syncthreads();
  int g1, g2, g3;
  R t1, t2, t3;
  Coord<R>::stencil(rec, 0, d.M1, P, g1, t1);
  Coord<R>::stencil(rec, 1, d.M2, P, g2, t2);
  Coord<R>::stencil(rec, 2, d.M3, P, g3, t3);
  R* my = wt + grp * 3 * P;
  if (lane < 3) {
    R w[P];
    eval_window<R, P, NW>(win, lane == 0 ? t1 : (lane == 1 ? t2 : t3), w);
#pragma unroll
    for (int p = 0; p < P; ++p) my[lane * P + p] = w[p];
  }
  __syncthreads();
  R acc[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
  if (lane < P) {
    const size_t G3 = static_cast<size_t>(d.M1) * d.M2 * d.M3;
    int xi[P];
#pragma unroll
    for (int a = 0; a < P; ++a) {
      const int x = g1 + a;
      xi[a] = x >= d.M1 ? x - d.M1 : x;
    }
    R w1[P];
#pragma unroll
    for (int a = 0; a < P; ++a) w1[a] = my[a];
    int z = g3 + lane;
    z -= z >= d.M3 ? d.M3 : 0;
#pragma unroll
    for (int b = 0; b < P; ++b) {
      int y = g2 + b;
      y -= y >= d.M2 ? d.M2 : 0;
      const R* row = d.phi + (static_cast<size_t>(z) * d.M2 + y) * d.M1;
      const R w2 = my[P + b];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        R sc = R(0);
#pragma unroll
        for (int a = 0; a < P; ++a) sc += row[c * G3 + xi[a]] * w1[a];
        acc[c] += sc * w2;
      }
    }
    const R w3 = my[2 * P + lane];
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[c] *= w3;
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) acc[c] = lane_group_sum<L>(acc[c]);
  if (lane == 0 && valid) {
    const R qk = rec.q * d.coulomb_k;
#pragma unroll
    for (int c = 0; c < 6; ++c) w6[6 * j + c] = qk * acc[c];
  }
}

// Tile-staged gathers of NC plain-window components, one particle per lane:
// components c0 .. c0 + NC - 1 of the field grids (component c at phi + c M1
// M2 M3) go to out[stride j + c], scaled by sgn q_j.  The ik field (App. C,
// eq. rhodiagforce) is one launch of three, f_j = -q_j sum_g W E_c(g); the
// per-particle virial (Sec. 4.4, eq. PinsFind), w6_j = q_j sum_g W Pi_c(g), is
// one launch of six for small boxes and two of three for large ones (three
// boxes in LDS instead of six keep three workgroups per CU: 10^6 slab 694 ->
// 342 us; at 30k the second launch costs more than it saves).  One workgroup
// per tile stages the tile's component boxes, then each lane evaluates its
// particle's 3 P window values and sums the components over its P^3 stencil.  The per-particle kernels read the grids from L2 at random
// (10^6 slab: 1.4 ms for the ik gather, 2.4 ms for the virial gather).
template <typename R, int P, int NW, int NC, bool BATCH>
__global__ void __launch_bounds__(256) k_gather_comp_lane(KArg<R, BATCH> ka, R* __restrict__ out,
                                                          double* __restrict__ out7, int c0, int stride, R sgn) {
  static_assert(NC == 3 || NC == 6, "three or six components");
  int tile;
  const DevPlan<R>& d = plan_of(ka, tile);
  out += static_cast<int64_t>(stride) * d.pofs;
  if (out7 && tile == 0) {
    __shared__ double red[kNumSums * 16];
    finalize_sums(d, out7 + kNumSums * d.rep, red);
  }
  extern __shared__ __align__(16) unsigned char smem[];
  R* win = reinterpret_cast<R*>(smem);                // (NW + 1) x P
  R* box = win + ((NW + 1) * P + 3) / 4 * 4;          // NC x E1 x E2 x E3 component values
  const int tid = threadIdx.x, nth = blockDim.x;
  const int t1 = tile % d.nt1, t2 = (tile / d.nt1) % d.nt2, t3 = tile / (d.nt1 * d.nt2);
  const int o1 = t1 * d.T1, o2 = t2 * d.T2, o3 = t3 * d.T3;
  const int E1 = min(d.T1, d.M1 - o1) + P - 1;
  const int E2 = min(d.T2, d.M2 - o2) + P - 1;
  const int E3 = min(d.T3, d.M3 - o3) + P - 1;
  const int E12 = E1 * E2;
  const int nbox = E12 * E3;
  const int start = d.offsets[tile], end = d.offsets[tile + 1];
  if (start == end) return;
  const size_t G3 = static_cast<size_t>(d.M1) * d.M2 * d.M3;
  const bool deep = nbox > 4 * nth;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const R* src = d.phi + (c0 + c) * G3;
    BoxWalk walk(tid, nth, E1, E2, E3, o1, o2, o3, d.M1, d.M2, d.M3);
    while (walk.k < nbox) {
      if (deep)
        stage_box_round<R, 16>(d, src, box + c * nbox, walk, nbox, o1, o2, o3, nth);
      else
        stage_box_round<R, 4>(d, src, box + c * nbox, walk, nbox, o1, o2, o3, nth);
    }
  }
  for (int k = tid; k < (NW + 1) * P; k += nth) win[k] = d.win[k];
  __syncthreads();
  const R qk0 = sgn * d.coulomb_k;
  for (int i = start + tid; i < end; i += nth) {
    const Record<R> rec = d.sorted[i];
    const int64_t j = d.perm[i];
    int g1, g2, g3;
    R u1, u2, u3;
    Coord<R>::stencil(rec, 0, d.M1, P, g1, u1);
    Coord<R>::stencil(rec, 1, d.M2, P, g2, u2);
    Coord<R>::stencil(rec, 2, d.M3, P, g3, u3);
    R w1[P], w2[P], w3[P];
    eval_window<R, P, NW>(win, u1, w1);
    eval_window<R, P, NW>(win, u2, w2);
    eval_window<R, P, NW>(win, u3, w3);
    // the base lies in this tile: box-local base = g0 - o (no wrap)
    const R* p0 = box + (g3 - o3) * E12 + (g2 - o2) * E1 + (g1 - o1);
    R acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = R(0);
#pragma unroll
    for (int cz = 0; cz < P; ++cz) {
      R accz[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) accz[c] = R(0);
#pragma unroll
      for (int b = 0; b < P; ++b) {
        const R* row = p0 + cz * E12 + b * E1;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          R s = R(0);
#pragma unroll
          for (int a = 0; a < P; ++a) s += row[c * nbox + a] * w1[a];
          accz[c] += s * w2[b];
        }
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] += accz[c] * w3[cz];
    }
    const R qk = rec.q * qk0;
#pragma unroll
    for (int c = 0; c < NC; ++c) out[static_cast<int64_t>(stride) * j + c0 + c] = qk * acc[c];
  }
}

// Tile-staged gather, for dense tiles: one workgroup per tile.  The
// potential on the tile's stencil box (its cells plus P - 1 more along each
// cell vector, cyclically) is staged in LDS once, then the tile's particles
// (contiguous after the sort) are processed as in k_gather, reading the
// potential from LDS instead of L2.
template <typename R, int P, int NW, bool BATCH>
__global__ void __launch_bounds__(256) k_gather_tile(KArg<R, BATCH> ka, R* __restrict__ f,
                                                double* __restrict__ out7) {
  constexpr int L = GatherLanes<P>::L;
  constexpr int G = 256 / L;                          // particles per round
  int tile;
  const DevPlan<R>& d = plan_of(ka, tile);
  f += 3 * d.pofs;
  if (out7 && tile == 0) {
    __shared__ double red[kNumSums * 16];
    finalize_sums(d, out7 + kNumSums * d.rep, red);
  }
  extern __shared__ __align__(16) unsigned char smem[];
  R* win = reinterpret_cast<R*>(smem);                // (NW + 1) x P
  R* wt = win + (NW + 1) * P;                         // G x 6 x P: w1 d1 w2 d2 w3 d3
  R* box = wt + G * 6 * P;                            // E1 x E2 x E3 potential values
  const int tid = threadIdx.x, nth = blockDim.x;
  const int t1 = tile % d.nt1, t2 = (tile / d.nt1) % d.nt2, t3 = tile / (d.nt1 * d.nt2);
  const int o1 = t1 * d.T1, o2 = t2 * d.T2, o3 = t3 * d.T3;
  const int E1 = min(d.T1, d.M1 - o1) + P - 1;
  const int E2 = min(d.T2, d.M2 - o2) + P - 1;
  const int E3 = min(d.T3, d.M3 - o3) + P - 1;
  const int nbox = E1 * E2 * E3;
  // the offsets, the window table and the potential box are fetched in rounds
  // of U loads per thread, the first together with the offsets (clamped
  // indices: no branches)
  // box loads in flight per thread: 16 for large boxes (10^6 slab, 15^3: the
  // staging is latency-bound, 66.4 -> 64.2 us), 4 for small ones (30k water,
  // 9^3: deeper rounds cost 2 us there)
  BoxWalk walk(tid, nth, E1, E2, E3, o1, o2, o3, d.M1, d.M2, d.M3);
  const bool deep = nbox > 4 * nth;
  auto stage_round = [&] {
    if (deep)
      stage_box_round<R, 16>(d, d.phi, box, walk, nbox, o1, o2, o3, nth);
    else
      stage_box_round<R, 4>(d, d.phi, box, walk, nbox, o1, o2, o3, nth);
  };
  const int start = d.offsets[tile], end = d.offsets[tile + 1];
  const R wv = d.win[min(tid, (NW + 1) * P - 1)];
  stage_round();
  if (start == end) return;
  if (tid < (NW + 1) * P) win[tid] = wv;
  for (int k = tid + nth; k < (NW + 1) * P; k += nth) win[k] = d.win[k];
  while (walk.k < nbox) stage_round();
  const int grp = tid / L, lane = tid - grp * L;
  R* my = wt + grp * 6 * P;
  for (int base = start; base < end; base += G) {
    const int i = base + grp;
    const bool valid = i < end;
    const Record<R> rec = d.sorted[valid ? i : start];
    const int64_t j = valid ? d.perm[i] : 0;        // fetched early: used at the end
    int g1, g2, g3;
    R u1, u2, u3;
    Coord<R>::stencil(rec, 0, d.M1, P, g1, u1);
    Coord<R>::stencil(rec, 1, d.M2, P, g2, u2);
    Coord<R>::stencil(rec, 2, d.M3, P, g3, u3);
    __syncthreads();                                  // box staged / previous round done with wt
    window_d_lanes<R, P, NW, L>(win, u1, u2, u3, lane, my);
    __syncthreads();
    // the base lies in this tile: box-local base = g0 - o (no wrap)
    const int b1 = g1 - o1, b2 = g2 - o2, b3 = g3 - o3;
    R gx = R(0), gy = R(0), gz = R(0);
    if (lane < P) {
      R w1[P], d1[P];
#pragma unroll
      for (int a = 0; a < P; ++a) {
        w1[a] = my[a];
        d1[a] = my[P + a];
      }
      const R* plane = box + (b3 + lane) * E1 * E2 + b2 * E1 + b1;
      R sxz = R(0), syz = R(0), s0z = R(0);
#pragma unroll
      for (int b = 0; b < P; ++b) {
        const R* row = plane + b * E1;
        R sx = R(0), s0 = R(0);
#pragma unroll
        for (int a = 0; a < P; ++a) {
          const R v = row[a];
          sx += v * d1[a];
          s0 += v * w1[a];
        }
        const R w2 = my[2 * P + b], d2 = my[3 * P + b];
        sxz += sx * w2;
        s0z += s0 * w2;
        syz += s0 * d2;
      }
      gx = sxz * my[4 * P + lane];
      gy = syz * my[4 * P + lane];
      gz = s0z * my[5 * P + lane];
    }
    gx = lane_group_sum<L>(gx);
    gy = lane_group_sum<L>(gy);
    gz = lane_group_sum<L>(gz);
    if (lane == 0 && valid) {
      const R qk = rec.q * d.coulomb_k;
      f[3 * j + 0] = qk * (d.G[0] * gx + d.G[1] * gy + d.G[2] * gz);
      f[3 * j + 1] = qk * (d.G[3] * gx + d.G[4] * gy + d.G[5] * gz);
      f[3 * j + 2] = qk * (d.G[6] * gx + d.G[7] * gy + d.G[8] * gz);
    }
  }
}

// Tile-staged gather with one particle per lane: the tile's potential box is
// staged in LDS as in k_gather_tile, then each thread takes whole particles
// of the tile (contiguous after the sort) in strides of the workgroup size.
// A lane evaluates its particle's 3 P window values and derivatives itself
// (the coefficients are read at the same LDS address by every lane, a
// broadcast) and sums its P^3 stencil; no barrier or cross-lane reduction
// per particle.  The P^3 potential reads of a wave go to 64 independent
// stencils of the box.
template <typename R, int P, int NW>
__device__ __forceinline__ void eval_window_d(const R* __restrict__ win, R tau, R* w, R* dw) {
#pragma unroll
  for (int q = 0; q < (P + 1) / 2; ++q) {
    R v, dv, vm, dvm;
    window_pair_d<R, P, NW>(win, q, tau, v, dv, vm, dvm);
    w[q] = v;
    dw[q] = dv;
    if (P - 1 - q != q) {
      w[P - 1 - q] = vm;
      dw[P - 1 - q] = dvm;
    }
  }
}

template <typename R, int P, int NW, bool BATCH>
__global__ void __launch_bounds__(256) k_gather_lane(KArg<R, BATCH> ka, R* __restrict__ f,
                                                     double* __restrict__ out7) {
  int tile;
  const DevPlan<R>& d = plan_of(ka, tile);
  f += 3 * d.pofs;
  if (out7 && tile == 0) {
    __shared__ double red[kNumSums * 16];
    finalize_sums(d, out7 + kNumSums * d.rep, red);
  }
  extern __shared__ __align__(16) unsigned char smem[];
  R* win = reinterpret_cast<R*>(smem);                // (NW + 1) x P
  R* box = win + ((NW + 1) * P + 3) / 4 * 4;          // E1 x E2 x E3 potential values
  const int tid = threadIdx.x, nth = blockDim.x;
  const int t1 = tile % d.nt1, t2 = (tile / d.nt1) % d.nt2, t3 = tile / (d.nt1 * d.nt2);
  const int o1 = t1 * d.T1, o2 = t2 * d.T2, o3 = t3 * d.T3;
  const int E1 = min(d.T1, d.M1 - o1) + P - 1;
  const int E2 = min(d.T2, d.M2 - o2) + P - 1;
  const int E3 = min(d.T3, d.M3 - o3) + P - 1;
  const int E12 = E1 * E2;
  const int nbox = E12 * E3;
  // box loads in flight per thread: 16 for large boxes (10^6 slab, 15^3: the
  // staging is latency-bound, 66.4 -> 64.2 us), 4 for small ones (30k water,
  // 9^3: deeper rounds cost 2 us there)
  BoxWalk walk(tid, nth, E1, E2, E3, o1, o2, o3, d.M1, d.M2, d.M3);
  const bool deep = nbox > 4 * nth;
  auto stage_round = [&] {
    if (deep)
      stage_box_round<R, 16>(d, d.phi, box, walk, nbox, o1, o2, o3, nth);
    else
      stage_box_round<R, 4>(d, d.phi, box, walk, nbox, o1, o2, o3, nth);
  };
  const int start = d.offsets[tile], end = d.offsets[tile + 1];
  const R wv = d.win[min(tid, (NW + 1) * P - 1)];
  stage_round();
  if (start == end) return;
  // this thread's first particle, fetched while the box is staged
  int i = start + tid;
  Record<R> rec = d.sorted[i < end ? i : start];
  int64_t j = i < end ? d.perm[i] : 0;
  if (tid < (NW + 1) * P) win[tid] = wv;
  for (int k = tid + nth; k < (NW + 1) * P; k += nth) win[k] = d.win[k];
  while (walk.k < nbox) stage_round();
  __syncthreads();
  const R qk0 = d.coulomb_k;
  for (; i < end; i += nth) {
    const int inext = i + nth;
    const Record<R> rn = d.sorted[inext < end ? inext : start];
    const int64_t jn = inext < end ? d.perm[inext] : 0;
    int g1, g2, g3;
    R u1, u2, u3;
    Coord<R>::stencil(rec, 0, d.M1, P, g1, u1);
    Coord<R>::stencil(rec, 1, d.M2, P, g2, u2);
    Coord<R>::stencil(rec, 2, d.M3, P, g3, u3);
    R w1[P], d1[P], w2[P], d2[P], w3[P], d3[P];
    eval_window_d<R, P, NW>(win, u1, w1, d1);
    eval_window_d<R, P, NW>(win, u2, w2, d2);
    eval_window_d<R, P, NW>(win, u3, w3, d3);
    // the base lies in this tile: box-local base = g0 - o (no wrap)
    const R* p0 = box + (g3 - o3) * E12 + (g2 - o2) * E1 + (g1 - o1);
    R gx = R(0), gy = R(0), gz = R(0);
#pragma unroll
    for (int c = 0; c < P; ++c) {
      R sxz = R(0), syz = R(0), s0z = R(0);
#pragma unroll
      for (int b = 0; b < P; ++b) {
        const R* row = p0 + c * E12 + b * E1;
        R sx = R(0), s0 = R(0);
#pragma unroll
        for (int a = 0; a < P; ++a) {
          const R v = row[a];
          sx += v * d1[a];
          s0 += v * w1[a];
        }
        sxz += sx * w2[b];
        s0z += s0 * w2[b];
        syz += s0 * d2[b];
      }
      gx += sxz * w3[c];
      gy += syz * w3[c];
      gz += s0z * d3[c];
    }
    const R qk = rec.q * qk0;
    f[3 * j + 0] = qk * (d.G[0] * gx + d.G[1] * gy + d.G[2] * gz);
    f[3 * j + 1] = qk * (d.G[3] * gx + d.G[4] * gy + d.G[5] * gz);
    f[3 * j + 2] = qk * (d.G[6] * gx + d.G[7] * gy + d.G[8] * gz);
    rec = rn;
    j = jn;
  }
}

// ---------------------------------------------------------------- launchers
template <typename R, int P, int NW, bool FIX>
static hipError_t spread_acc(const DevPlan<R>& d, hipStream_t s) {
  const size_t lds = lds_spread(d);
  if (lds > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_spread<R, P, NW, false, FIX>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  ESP_LAUNCH((k_spread<R, P, NW, false, FIX>), dim3(d.ntiles), dim3(256), lds, s, KArg<R, false>{d});
  return hipGetLastError();
}

template <typename R, int P, int NW>
static hipError_t spread_nw(const DevPlan<R>& d, hipStream_t s) {
  return d.spread_fixed ? spread_acc<R, P, NW, true>(d, s) : spread_acc<R, P, NW, false>(d, s);
}

template <typename R, int P, int NW>
static size_t gather_lds() {
  return ((NW + 1) * P + (256 / GatherLanes<P>::L) * 6 * P) * sizeof(R);
}

template <typename R, int P, int NW>
static hipError_t gather_nw(const DevPlan<R>& d, R* f, double* out7, hipStream_t s) {
  if (d.gather_lane) {
    const size_t lds = ((NW + 1) * P + 3) / 4 * 4 * sizeof(R) + lds_gather_box(d);
    if (lds > 65536)
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gather_lane<R, P, NW, false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    ESP_LAUNCH((k_gather_lane<R, P, NW, false>), dim3(d.ntiles), dim3(256), lds, s, KArg<R, false>{d},
                       f, out7);
    return hipGetLastError();
  }
  if (d.gather_tiled) {
    const size_t lds = gather_lds<R, P, NW>() + lds_gather_box(d);
    if (lds > 65536)
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gather_tile<R, P, NW, false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    ESP_LAUNCH((k_gather_tile<R, P, NW, false>), dim3(d.ntiles), dim3(256), lds, s, KArg<R, false>{d},
                       f, out7);
    return hipGetLastError();
  }
  constexpr int G = 256 / GatherLanes<P>::L;
  const int nb = static_cast<int>((d.n + G - 1) / G);
  ESP_LAUNCH((k_gather<R, P, NW, false>), dim3(nb), dim3(256), (gather_lds<R, P, NW>()), s,
                     KArg<R, false>{d}, f, out7);
  return hipGetLastError();
}

template <typename R, int P, int NW>
static hipError_t spread_nw_batch(const BatchLaunch<R>& b, hipStream_t s) {
  // FP32 batches spread in fixed point (integer-product terms), FP64 batches
  // with FP64 adds: the automatic choice of single plans for tiles of the
  // replica sizes (2,000 to 60,000 particles)
  constexpr bool FIX = sizeof(R) == 4;
  if (b.lds > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_spread<R, P, NW, true, FIX>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(b.lds));
  ESP_LAUNCH((k_spread<R, P, NW, true, FIX>), dim3(b.nblk), dim3(256), b.lds, s,
                     KArg<R, true>{b.plans, b.boff, b.nrep});
  return hipGetLastError();
}

template <typename R, int P, int NW>
static hipError_t gather_nw_batch(const BatchLaunch<R>& b, R* f, double* out7, hipStream_t s) {
  if (b.lane) {
    // tile-staged, one particle per lane: one workgroup per tile of every replica
    if (b.lds > 65536)
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gather_lane<R, P, NW, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(b.lds));
    ESP_LAUNCH((k_gather_lane<R, P, NW, true>), dim3(b.nblk), dim3(256), b.lds, s,
               KArg<R, true>{b.plans, b.boff, b.nrep}, f, out7);
    return hipGetLastError();
  }
  ESP_LAUNCH((k_gather<R, P, NW, true>), dim3(b.nblk), dim3(256), (gather_lds<R, P, NW>()), s,
                     KArg<R, true>{b.plans, b.boff, b.nrep}, f, out7);
  return hipGetLastError();
}

#define ESP_NW_SWITCH(NWV, FN, ...)                  \
  switch (NWV) {                                     \
    case 8: return FN<R, P, 8>(__VA_ARGS__);         \
    case 12: return FN<R, P, 12>(__VA_ARGS__);       \
    case 16: return FN<R, P, 16>(__VA_ARGS__);       \
    default: return hipErrorInvalidValue;            \
  }

template <typename R, int P>
hipError_t spread_launch(const DevPlan<R>& d, hipStream_t s) {
  ESP_NW_SWITCH(d.nw, spread_nw, d, s)
}

template <typename R, int P>
hipError_t gather_launch(const DevPlan<R>& d, R* f, double* out7, hipStream_t s) {
  ESP_NW_SWITCH(d.nw, gather_nw, d, f, out7, s)
}

template <typename R, int P, int NW>
static hipError_t gather_ik_nw(const DevPlan<R>& d, R* f, double* out7, hipStream_t s) {
  if (d.comp_lane & 1) {
    const size_t lds = ((NW + 1) * P + 3) / 4 * 4 * sizeof(R) + 3 * lds_gather_box(d);
    if (lds > 65536)
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gather_comp_lane<R, P, NW, 3, false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    ESP_LAUNCH((k_gather_comp_lane<R, P, NW, 3, false>), dim3(d.ntiles), dim3(256), lds, s, KArg<R, false>{d},
               f, out7, 0, 3, R(-1));
    return hipGetLastError();
  }
  constexpr int G = 256 / GatherLanes<P>::L;
  const int nb = static_cast<int>((d.n + G - 1) / G);
  const size_t lds = ((NW + 1) * P + G * 3 * P) * sizeof(R);
  ESP_LAUNCH((k_gather_ik<R, P, NW, false>), dim3(nb), dim3(256), lds, s, KArg<R, false>{d}, f, out7);
  return hipGetLastError();
}

template <typename R, int P>
hipError_t gather_ik_launch(const DevPlan<R>& d, R* f, double* out7, hipStream_t s) {
  ESP_NW_SWITCH(d.nw, gather_ik_nw, d, f, out7, s)
}

template <typename R, int P, int NW>
static hipError_t gather_local_nw(const DevPlan<R>& d, R* w6, double* out7, hipStream_t s) {
  if (d.comp_lane & 2) {
    const size_t base = ((NW + 1) * P + 3) / 4 * 4 * sizeof(R);
    const size_t lds6 = base + 6 * lds_gather_box(d), lds3 = base + 3 * lds_gather_box(d);
    if (lds6 <= kCompLaneOneLaunch) {
      ESP_LAUNCH((k_gather_comp_lane<R, P, NW, 6, false>), dim3(d.ntiles), dim3(256), lds6, s,
                 KArg<R, false>{d}, w6, out7, 0, 6, R(1));
      return hipGetLastError();
    }
    if (lds3 > 65536)
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gather_comp_lane<R, P, NW, 3, false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds3));
    ESP_LAUNCH((k_gather_comp_lane<R, P, NW, 3, false>), dim3(d.ntiles), dim3(256), lds3, s, KArg<R, false>{d},
               w6, out7, 0, 6, R(1));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    ESP_LAUNCH((k_gather_comp_lane<R, P, NW, 3, false>), dim3(d.ntiles), dim3(256), lds3, s, KArg<R, false>{d},
               w6, static_cast<double*>(nullptr), 3, 6, R(1));
    return hipGetLastError();
  }
  constexpr int G = 256 / GatherLanes<P>::L;
  const int nb = static_cast<int>((d.n + G - 1) / G);
  const size_t lds = ((NW + 1) * P + G * 3 * P) * sizeof(R);
  ESP_LAUNCH((k_gather_local<R, P, NW, false>), dim3(nb), dim3(256), lds, s, KArg<R, false>{d}, w6,
                     out7);
  return hipGetLastError();
}

template <typename R, int P>
hipError_t gather_local_launch(const DevPlan<R>& d, R* w6, double* out7, hipStream_t s) {
  ESP_NW_SWITCH(d.nw, gather_local_nw, d, w6, out7, s)
}

template <typename R, int P>
hipError_t spread_launch_batch(const BatchLaunch<R>& b, hipStream_t s) {
  ESP_NW_SWITCH(b.nw, spread_nw_batch, b, s)
}

template <typename R, int P>
hipError_t gather_launch_batch(const BatchLaunch<R>& b, R* f, double* out7, hipStream_t s) {
  ESP_NW_SWITCH(b.nw, gather_nw_batch, b, f, out7, s)
}

template hipError_t spread_launch<float, ESP_P>(const DevPlan<float>&, hipStream_t);
template hipError_t spread_launch<double, ESP_P>(const DevPlan<double>&, hipStream_t);
template hipError_t gather_launch<float, ESP_P>(const DevPlan<float>&, float*, double*, hipStream_t);
template hipError_t gather_launch<double, ESP_P>(const DevPlan<double>&, double*, double*, hipStream_t);
template hipError_t gather_ik_launch<float, ESP_P>(const DevPlan<float>&, float*, double*, hipStream_t);
template hipError_t gather_ik_launch<double, ESP_P>(const DevPlan<double>&, double*, double*, hipStream_t);
template hipError_t gather_local_launch<float, ESP_P>(const DevPlan<float>&, float*, double*, hipStream_t);
template hipError_t gather_local_launch<double, ESP_P>(const DevPlan<double>&, double*, double*, hipStream_t);
template hipError_t spread_launch_batch<float, ESP_P>(const BatchLaunch<float>&, hipStream_t);
template hipError_t spread_launch_batch<double, ESP_P>(const BatchLaunch<double>&, hipStream_t);
template hipError_t gather_launch_batch<float, ESP_P>(const BatchLaunch<float>&, float*, double*, hipStream_t);
template hipError_t gather_launch_batch<double, ESP_P>(const BatchLaunch<double>&, double*, double*,
                                                       hipStream_t);

}  // namespace espx
