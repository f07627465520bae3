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

#include "esp_common.h"

namespace espx {

// ------------------------------------------------------------------- sort
// Inclusive scan of an int over the 64 lanes of a wave with DPP moves: row
// shifts by 1, 2, 4 and 8 scan each row of 16 lanes (lanes without a source
// add 0), then the row broadcasts of lanes 15 and 31 carry the earlier rows.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp_int(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWMASK, 0xf, false);
}
__device__ __forceinline__ int wave_inclusive_scan(int v) {
  v += dpp_int<0x111, 0xf>(v);      // row_shr:1
  v += dpp_int<0x112, 0xf>(v);      // row_shr:2
  v += dpp_int<0x114, 0xf>(v);      // row_shr:4
  v += dpp_int<0x118, 0xf>(v);      // row_shr:8
  v += dpp_int<0x142, 0xa>(v);      // row_bcast:15 into rows 1 and 3
  v += dpp_int<0x143, 0xc>(v);      // row_bcast:31 into rows 2 and 3
  return v;
}

// Exclusive scan of counts[0..n) into offs[0..n] (LDS) by one workgroup
// (integer sums: exact).  Each thread sums a contiguous chunk; the chunk sums
// are scanned within each wave by DPP, the wave totals (at most 16) go
// through LDS with one barrier.  part: LDS scratch of at least 16 ints.
__device__ void block_scan(const int* __restrict__ counts, int* offs, int n, int* part) {
  const int nth = blockDim.x;
  const int chunk = (n + nth - 1) / nth;
  const int b0 = min(n, static_cast<int>(threadIdx.x) * chunk);
  const int b1 = min(n, b0 + chunk);
  int s = 0;
  for (int k = b0; k < b1; ++k) s += counts[k];
  const int incl = wave_inclusive_scan(s);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 63) part[wid] = incl;
  __syncthreads();
  int wpre = 0, total = 0;
#pragma unroll
  for (int w = 0; w < 16; ++w) {
    const int t = w < (nth >> 6) ? part[w] : 0;
    wpre += w < wid ? t : 0;
    total += t;
  }
  int run = wpre + incl - s;
  for (int k = b0; k < b1; ++k) {
    offs[k] = run;
    run += counts[k];
  }
  if (threadIdx.x == nth - 1) offs[n] = total;
  __syncthreads();
}

// Binning: turn the block's tile histogram (LDS) into the first rank of the
// block within each tile, one returning global atomic per occupied tile;
// U atomics per thread are in flight at once.
template <int U>
__device__ __forceinline__ void bin_reserve(int* hist, int* __restrict__ counts, int ntiles, int nth) {
  for (int k0 = threadIdx.x; k0 < ntiles; k0 += U * nth) {
    int c[U], r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u * nth;
      c[u] = k < ntiles ? hist[k] : 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) r[u] = c[u] ? atomicAdd(counts + k0 + u * nth, c[u]) : 0;
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (c[u]) hist[k0 + u * nth] = r[u];
  }
}

// Cell sort, pass 1.  Each particle gets its reduced coordinates (the sorted
// record), its tile key (tile of the stencil base g0) and its rank within the
// tile.  Ranks come from an LDS histogram of the block's keys plus one global
// atomic per occupied tile and block, so no global counter sees more than
// one atomic per block.  Also accumulates sum q, sum q^2 and sum |q| per
// block in FP64.
// A thread takes binppt particles (i0 + u x 256, u < binppt): with many tiles
// the per-block histogram work (clear, read, global atomics) is shared by up
// to 1,024 particles.
template <typename R, bool BATCH, int PPT>
__global__ void __launch_bounds__(kBinThreads) k_bin(KArg<R, BATCH> ka, const R* __restrict__ xyz,
                                                     const R* __restrict__ q) {
  static_assert(PPT == 1 || PPT == kBinMaxPpt, "one particle per thread, or up to kBinMaxPpt");
  extern __shared__ int hist[];            // ntiles entries when d.bin_lds
  __shared__ double red[3 * 16];
  int blk;
  const DevPlan<R>& d = plan_of(ka, blk);
  xyz += 3 * d.pofs;
  q += d.pofs;
  const bool lh = d.bin_lds != 0;
  const int ppt = PPT == 1 ? 1 : d.binppt, nth = blockDim.x;
  const int64_t i0 = static_cast<int64_t>(blk) * nth * ppt + threadIdx.x;
  // inputs fetched first; the histogram is cleared while they arrive
  R x[PPT], y[PPT], z[PPT], qi[PPT];
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    const int64_t i = i0 + static_cast<int64_t>(u) * nth;
    const int64_t ii = i < d.n ? i : 0;
    if (u < ppt) {
      x[u] = xyz[3 * ii];
      y[u] = xyz[3 * ii + 1];
      z[u] = xyz[3 * ii + 2];
      qi[u] = q[ii];
    }
  }
  if (lh)
    for (int k = threadIdx.x; k < d.ntiles; k += nth) hist[k] = 0;
  __syncthreads();
  double v[3] = {0.0, 0.0, 0.0};
  const Divisor dT1(d.T1), dT2(d.T2), dT3(d.T3);   // exact for the grid indices (< 2^24)
  int key[PPT], lr[PPT];
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    key[u] = 0;
    lr[u] = 0;
    const int64_t i = i0 + static_cast<int64_t>(u) * nth;
    if (u < ppt && i < d.n) {
      R xu = x[u], yu = y[u], zu = z[u], qu = qi[u];
      if (!(finite_r(xu) && finite_r(yu) && finite_r(zu) && finite_r(qu))) {
        atomicOr(d.flags, 1);
        xu = yu = zu = qu = R(0);
      }
      Record<R> rec;
      Coord<R>::make(d, xu, yu, zu, qu, rec);
      d.tmp[i] = rec;
      int k;
      if (d.cellsort) {
        k = (Coord<R>::cell(rec, 2, d.cn3) * d.cn2 + Coord<R>::cell(rec, 1, d.cn2)) * d.cn1 +
            Coord<R>::cell(rec, 0, d.cn1);
      } else {
        int g1, g2, g3;
        R t;
        Coord<R>::stencil(rec, 0, d.M1, d.P, g1, t);
        Coord<R>::stencil(rec, 1, d.M2, d.P, g2, t);
        Coord<R>::stencil(rec, 2, d.M3, d.P, g3, t);
        int rm;
        k = (dT3.div(g3, rm) * d.nt2 + dT2.div(g2, rm)) * d.nt1 + dT1.div(g1, rm);
      }
      key[u] = k;
      lr[u] = lh ? atomicAdd(hist + k, 1)
                 : atomicAdd(d.counts + static_cast<size_t>(blk % d.nsub) * d.ntiles + k, 1);
      v[0] += static_cast<double>(qu);
      v[1] += static_cast<double>(qu) * static_cast<double>(qu);
      v[2] += fabs(static_cast<double>(qu));
    }
  }
  __syncthreads();
  int* counts = d.counts + static_cast<size_t>(blk % d.nsub) * d.ntiles;
  if (lh) {
    // a thread issues all of its (returning) atomics before it uses a result,
    // so their round trips overlap instead of adding up: rounds of 16 tiles
    // per thread where tiles are many (10^6 slab, 3,328 tiles: one round trip
    // instead of four), of 4 otherwise
    if (d.ntiles > 4 * nth)
      bin_reserve<16>(hist, counts, d.ntiles, nth);
    else
      bin_reserve<4>(hist, counts, d.ntiles, nth);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    const int64_t i = i0 + static_cast<int64_t>(u) * nth;
    if (u < ppt && i < d.n) {
      d.keys[i] = key[u];
      d.ranks[i] = lh ? hist[key[u]] + lr[u] : lr[u];
    }
  }
  block_sum<3>(v, red);
  if (threadIdx.x == 0) {
    d.qpart[3 * blk] = v[0];
    d.qpart[3 * blk + 1] = v[1];
    d.qpart[3 * blk + 2] = v[2];
  }
}

// FP32 plans with fixed-point spreading add each tile's integer sums into an
// int64 grid at one scale 2^gexp for the call: with B = wmax^3 sum |q| no
// cell exceeds B in magnitude, and gexp = kGridExp - ilogb(B) keeps every
// cell below 2^57 while a tile's own scale (2^58 over its own, smaller bound)
// is at least twice as fine, so a tile's sums reach the grid by a rounding
// right shift.  Integer sums do not depend on the order of the atomics: the
// grid, and everything computed from it, repeats bit for bit.  One block
// (of the pass that ends the cell sort) reduces the binning partials.
template <typename R>
__device__ void publish_gexp(const DevPlan<R>& d, double* red) {
  double v[1] = {0.0};
  for (int b = threadIdx.x; b < d.nbin; b += blockDim.x) v[0] += d.qpart[3 * b + 2];
  block_sum<1>(v, red);
  if (threadIdx.x == 0) {
    const double bound = v[0] * static_cast<double>(d.wmax3);
    d.gexp[0] = max(-100, min(120, kGridExp - ilogb(fmax(bound, 1e-30))));
  }
}

// Tile offsets for nsub > 1 counter copies (large systems, where one counter
// per tile would see hundreds of same-address atomics): one workgroup turns
// the copies into per-copy bases within each tile and the tile offsets, and
// clears the counters for the next call.  Tiles go in rounds of one per
// thread; the nsub counts of kScanTpt rounds are loaded at once (coalesced,
// one round trip), then each round's tile totals are scanned (DPP within
// waves, wave totals through LDS, a carry across rounds) and its bases
// written.
template <typename R, bool BATCH>
__global__ void __launch_bounds__(1024) k_scan_sub(KArg<R, BATCH> ka) {
  static_assert(kScanTpt % 2 == 0, "consecutive rounds alternate the two slot sets");
  __shared__ int part[2][16];
  __shared__ double red[16];
  int blk;
  const DevPlan<R>& d = plan_of(ka, blk);
  if (d.nsub <= 1) return;
  const int nt = d.ntiles, nsub = d.nsub, nth = blockDim.x, tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6, nw = nth >> 6;
  int carry = 0;
  for (int g0 = 0; g0 < nt; g0 += nth * kScanTpt) {
    int v[kScanTpt][kMaxCounterCopies];
#pragma unroll
    for (int j = 0; j < kScanTpt; ++j) {
      const int t = g0 + j * nth + tid;
#pragma unroll
      for (int c = 0; c < kMaxCounterCopies; ++c)
        v[j][c] = (t < nt && c < nsub) ? d.counts[static_cast<size_t>(c) * nt + t] : 0;
    }
#pragma unroll
    for (int j = 0; j < kScanTpt; ++j) {
      const int t = g0 + j * nth + tid;
      int tot = 0;
#pragma unroll
      for (int c = 0; c < kMaxCounterCopies; ++c) tot += v[j][c];
      const int incl = wave_inclusive_scan(tot);
      int* pj = part[j & 1];                  // alternating slots: one barrier per round
      if (lane == 63) pj[wid] = incl;
      __syncthreads();
      int wpre = 0, rtot = 0;
#pragma unroll
      for (int w = 0; w < 16; ++w) {
        const int x = w < nw ? pj[w] : 0;
        wpre += w < wid ? x : 0;
        rtot += x;
      }
      if (t < nt) {
        int run = carry + wpre + incl - tot;
        d.offsets[t] = run;
#pragma unroll
        for (int c = 0; c < kMaxCounterCopies; ++c)
          if (c < nsub) {
            const size_t k = static_cast<size_t>(c) * nt + t;
            d.sbase[k] = run;
            d.counts[k] = 0;
            run += v[j][c];
          }
      }
      carry += rtot;
    }
  }
  if (tid == 0) d.offsets[nt] = carry;
  if (d.grid_fixed) publish_gexp(d, red);
}

// Cell sort, pass 2.  With one counter per tile every block scans the tile
// counts itself (they are few) and scatters its particles to offset[key] +
// rank, and block 0 publishes the offsets for the spreading pass; with
// counter copies the bases come from k_scan_sub.
template <typename R, bool BATCH>
__global__ void __launch_bounds__(1024) k_scatter(KArg<R, BATCH> ka) {
  extern __shared__ int offs[];             // ntiles + 1
  __shared__ int part[1024];
  __shared__ double red[16];
  int blk;
  const DevPlan<R>& d = plan_of(ka, blk);
  const int64_t i = static_cast<int64_t>(blk) * blockDim.x + threadIdx.x;
  if (d.nsub > 1) {
    if (i < d.n) {
      const size_t copy = static_cast<size_t>((i / (static_cast<int64_t>(kBinThreads) * d.binppt)) % d.nsub);  // binning block of i
      const int pos = d.sbase[copy * d.ntiles + d.keys[i]] + d.ranks[i];
      if (pos >= 0 && pos < d.n) {
        d.sorted[pos] = d.tmp[i];
        d.perm[pos] = static_cast<int>(i);
      } else {
        atomicOr(d.flags, 2);
      }
    }
    return;
  }
  // the particle's key, rank and record are fetched before the scan, so
  // their round trip overlaps it
  const int64_t ii = i < d.n ? i : 0;
  const int key = d.keys[ii], rank = d.ranks[ii];
  const Record<R> rec = d.tmp[ii];
  block_scan(d.counts, offs, d.ntiles, part);
  if (i < d.n) {
    const int pos = offs[key] + rank;
    if (pos >= 0 && pos < d.n) {
      d.sorted[pos] = rec;
      d.perm[pos] = static_cast<int>(i);
    } else {
      atomicOr(d.flags, 2);                 // inconsistent tile counts
    }
  }
  if (blk == 0) {
    for (int k = threadIdx.x; k <= d.ntiles; k += blockDim.x) d.offsets[k] = offs[k];
    if (d.grid_fixed) publish_gexp(d, red);
  }
}

template <typename R, bool BATCH>
__global__ void __launch_bounds__(256) k_finalize(KArg<R, BATCH> ka, double* __restrict__ out7) {
  __shared__ double red[kNumSums * 16];
  int blk;
  const DevPlan<R>& d = plan_of(ka, blk);
  finalize_sums(d, out7 + kNumSums * d.rep, red);
}

// ------------------------------------------------------------------ FFT xy
// grid / spec: explicit operands of a single-plan launch, or null for the
// plan's own rho / spec (batched launches); GF: the plan's own grid is the
// int64 fixed-point grid (grid_in null).
template <typename R, bool BATCH, bool GF>
__global__ void __launch_bounds__(1024) k_fft_xy(KArg<R, BATCH> ka, const R* __restrict__ grid_in,
                                                 Cplx<R>* __restrict__ spec_in, int clear) {
  extern __shared__ __align__(16) unsigned char smem[];
  int blk;
  const DevPlan<R>& d = plan_of(ka, blk);
  const R* grid = grid_in ? grid_in : d.rho;
  Cplx<R>* spec = spec_in ? spec_in : d.spec;
  const int M1 = d.M1, M2 = d.M2, H = d.H;
  const int npairs = (M2 + 1) / 2;
  const Divisor dM1(M1), dH(H);
  const int L = max(npairs * M1, M2 * H);
  Cplx<R>* A = reinterpret_cast<Cplx<R>*>(smem);
  Cplx<R>* B = A + L;
  Cplx<R>* tw1 = B + L;
  Cplx<R>* tw2 = tw1 + M1;
  const int nth = blockDim.x, tid = threadIdx.x;
  const size_t zoff = static_cast<size_t>(blk) * M2 * M1;
  const R* plane = grid + zoff;
  R* wplane = const_cast<R*>(grid) + zoff;
  // the plan's own grid in fixed point: int64 at scale 2^gexp
  constexpr bool fx = GF;
  long long* fplane = d.rhofix + (fx ? zoff : 0);
  const double finv = fx ? ldexp(1.0, -d.gexp[0]) : 0.0;
  auto cell = [&](int k) { return fx ? static_cast<R>(static_cast<double>(fplane[k]) * finv) : plane[k]; };
  auto zero = [&](int k) {
    if (fx)
      fplane[k] = 0;
    else
      wplane[k] = R(0);
  };
  // The plane in rounds of U loads per thread, issued before their stores;
  // the first round is straight-line code together with the twiddle loads,
  // so that all of them are in flight at once (indices clamped: no branches).
  constexpr int U = 4;
  auto round = [&](int k0) {
    R re[U], im[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = min(k0 + u * nth, npairs * M1 - 1);
      int x;
      const int p = dM1.div(k, x);
      const int y0 = 2 * p;
      re[u] = cell(y0 * M1 + x);
      im[u] = cell(min(y0 + 1, M2 - 1) * M1 + x);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u * nth;
      if (k < npairs * M1) {
        int x;
        const int p = dM1.div(k, x);
        const int y0 = 2 * p;
        A[k] = {re[u], y0 + 1 < M2 ? im[u] : R(0)};
        if (clear) {
          zero(y0 * M1 + x);
          if (y0 + 1 < M2) zero((y0 + 1) * M1 + x);
        }
      }
    }
  };
  const Cplx<R> tv1 = d.tw[d.f1.tw + min(tid, M1 - 1)];
  const Cplx<R> tv2 = d.tw[d.f2.tw + min(tid, M2 - 1)];
  round(tid);
  for (int k0 = tid + U * nth; k0 < npairs * M1; k0 += U * nth) round(k0);
  if (tid < M1) tw1[tid] = tv1;
  if (tid < M2) tw2[tid] = tv2;
  for (int k = tid + nth; k < M1; k += nth) tw1[k] = d.tw[d.f1.tw + k];
  for (int k = tid + nth; k < M2; k += nth) tw2[k] = d.tw[d.f2.tw + k];
  __syncthreads();
  Cplx<R>* res = fft_lines(A, B, d.f1, npairs, M1, 1, tw1, false, nth);
  Cplx<R>* oth = res == A ? B : A;
  // rows 2p (real part) and 2p+1 (imaginary part) were transformed together:
  // X_a[k] = (Z[k] + conj Z[-k]) / 2,  X_b[k] = (Z[k] - conj Z[-k]) / (2 i)
  for (int k = tid; k < npairs * H; k += nth) {
    int m;
    const int p = dH.div(k, m);
    const Cplx<R> Z = res[p * M1 + m];
    const Cplx<R> Zm = res[p * M1 + (m == 0 ? 0 : M1 - m)];
    oth[(2 * p) * H + m] = {R(0.5) * (Z.x + Zm.x), R(0.5) * (Z.y - Zm.y)};
    if (2 * p + 1 < M2) oth[(2 * p + 1) * H + m] = {R(0.5) * (Z.y + Zm.y), R(0.5) * (Zm.x - Z.x)};
  }
  __syncthreads();
  res = fft_lines(oth, res, d.f2, H, 1, H, tw2, false, nth);
  Cplx<R>* out = spec + static_cast<size_t>(blk) * M2 * H;
  for (int k = tid; k < M2 * H; k += nth) out[k] = res[k];
}

template <typename R, bool BATCH>
__global__ void __launch_bounds__(1024) k_fft_xy_inv(KArg<R, BATCH> ka) {
  extern __shared__ __align__(16) unsigned char smem[];
  int blk;
  const DevPlan<R>& d = plan_of(ka, blk);
  const int M1 = d.M1, M2 = d.M2, H = d.H;
  const int npairs = (M2 + 1) / 2;
  const Divisor dM1(M1);
  const int L = max(npairs * M1, M2 * H);
  Cplx<R>* A = reinterpret_cast<Cplx<R>*>(smem);
  Cplx<R>* B = A + L;
  Cplx<R>* tw1 = B + L;
  Cplx<R>* tw2 = tw1 + M1;
  const int nth = blockDim.x, tid = threadIdx.x;
  const Cplx<R> tv1 = d.tw[d.f1.tw + min(tid, M1 - 1)];
  const Cplx<R> tv2 = d.tw[d.f2.tw + min(tid, M2 - 1)];
  // block = component * M3 + plane
  const int comp = blk / d.M3, zp = blk - comp * d.M3;
  const Cplx<R>* in = d.spec + static_cast<size_t>(comp) * d.M3 * M2 * H + static_cast<size_t>(zp) * M2 * H;
  {
    // as in the forward pass: the first round straight-line with the twiddle loads
    constexpr int U = 4;
    auto round = [&](int k0) {
      Cplx<R> v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = in[min(k0 + u * nth, M2 * H - 1)];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (k0 + u * nth < M2 * H) A[k0 + u * nth] = v[u];
    };
    round(tid);
    for (int k0 = tid + U * nth; k0 < M2 * H; k0 += U * nth) round(k0);
  }
  if (tid < M1) tw1[tid] = tv1;
  if (tid < M2) tw2[tid] = tv2;
  for (int k = tid + nth; k < M1; k += nth) tw1[k] = d.tw[d.f1.tw + k];
  for (int k = tid + nth; k < M2; k += nth) tw2[k] = d.tw[d.f2.tw + k];
  __syncthreads();
  Cplx<R>* res = fft_lines(A, B, d.f2, H, 1, H, tw2, true, nth);
  Cplx<R>* oth = res == A ? B : A;
  // Hermitian rows a (= row 2p) and b (= row 2p+1): Z[x] = X_a[x] + i X_b[x]
  for (int k = tid; k < npairs * M1; k += nth) {
    int x;
    const int p = dM1.div(k, x);
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
  res = fft_lines(oth, res, d.f1, npairs, M1, 1, tw1, true, nth);
  R* plane = d.phi + static_cast<size_t>(comp) * d.M3 * M2 * M1 + static_cast<size_t>(zp) * M2 * M1;
  for (int k = tid; k < npairs * M1; k += nth) {
    int x;
    const int p = dM1.div(k, x);
    plane[(2 * p) * M1 + x] = res[k].x;
    if (2 * p + 1 < M2) plane[(2 * p + 1) * M1 + x] = res[k].y;
  }
}

// ------------------------------------------------- FFT xy, split passes
// For planes that do not fit one workgroup's LDS the x and y transforms run
// as separate passes: the x pass on groups of npb row pairs (two real rows as
// one complex transform, as above), the y pass on groups of ncol adjacent
// half-spectrum columns of one plane, transformed in place.
template <typename R, bool GF>
__global__ void __launch_bounds__(256) k_fft_x(DevPlan<R> d, const R* __restrict__ grid_in,
                                              Cplx<R>* __restrict__ spec_in, int clear, int npb) {
  extern __shared__ __align__(16) unsigned char smem[];
  const R* grid = grid_in ? grid_in : d.rho;
  Cplx<R>* spec = spec_in ? spec_in : d.spec;
  const int M1 = d.M1, M2 = d.M2, H = d.H;
  const int npairs = (M2 + 1) / 2, total = npairs * d.M3;
  const Divisor dM1(M1), dH(H), dnp(npairs);
  const int q0 = xcd_block(blockIdx.x, gridDim.x) * npb, np = min(npb, total - q0);
  Cplx<R>* A = reinterpret_cast<Cplx<R>*>(smem);
  Cplx<R>* B = A + static_cast<size_t>(npb) * M1;
  Cplx<R>* tw1 = B + static_cast<size_t>(npb) * M1;
  const int nth = blockDim.x, tid = threadIdx.x;
  for (int k = tid; k < M1; k += nth) tw1[k] = d.tw[d.f1.tw + k];
  R* wgrid = const_cast<R*>(grid);
  constexpr bool fx = GF;                                 // the plan's int64 grid at scale 2^gexp
  const double finv = fx ? ldexp(1.0, -d.gexp[0]) : 0.0;
  auto cell = [&](size_t k) { return fx ? static_cast<R>(static_cast<double>(d.rhofix[k]) * finv) : grid[k]; };
  auto zero = [&](size_t k) {
    if (fx)
      d.rhofix[k] = 0;
    else
      wgrid[k] = R(0);
  };
  for (int k = tid; k < np * M1; k += nth) {
    int x;
    const int j = dM1.div(k, x);
    int zr;
    const int q = q0 + j, z = dnp.div(q, zr), y0 = 2 * zr;
    const size_t r0 = (static_cast<size_t>(z) * M2 + y0) * M1 + x;
    const R re = cell(r0);
    const R im = y0 + 1 < M2 ? cell(r0 + M1) : R(0);
    A[k] = {re, im};
    if (clear) {
      zero(r0);
      if (y0 + 1 < M2) zero(r0 + M1);
    }
  }
  __syncthreads();
  const Cplx<R>* res = fft_lines(A, B, d.f1, np, M1, 1, tw1, false, nth);
  for (int k = tid; k < np * H; k += nth) {
    int m;
    const int j = dH.div(k, m);
    int zr;
    const int q = q0 + j, z = dnp.div(q, zr), y0 = 2 * zr;
    const Cplx<R> Z = res[j * M1 + m];
    const Cplx<R> Zm = res[j * M1 + (m == 0 ? 0 : M1 - m)];
    Cplx<R>* row = spec + (static_cast<size_t>(z) * M2 + y0) * H;
    row[m] = {R(0.5) * (Z.x + Zm.x), R(0.5) * (Z.y - Zm.y)};
    if (y0 + 1 < M2) row[H + m] = {R(0.5) * (Z.y + Zm.y), R(0.5) * (Zm.x - Z.x)};
  }
}

// block = (component x M3 + plane) x column groups + group
template <typename R>
__global__ void __launch_bounds__(256) k_fft_y(DevPlan<R> d, Cplx<R>* __restrict__ spec_in, int ncol, int inverse) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cplx<R>* spec = spec_in ? spec_in : d.spec;
  const int M2 = d.M2, H = d.H;
  const int ngrp = (H + ncol - 1) / ncol;
  const int bx = xcd_block(blockIdx.x, gridDim.x);
  const int plane = bx / ngrp, grp = bx - plane * ngrp;
  const int m0 = grp * ncol, nc = min(ncol, H - m0);
  const Divisor dnc(nc);
  Cplx<R>* A = reinterpret_cast<Cplx<R>*>(smem);
  Cplx<R>* B = A + static_cast<size_t>(ncol) * M2;
  Cplx<R>* tw2 = B + static_cast<size_t>(ncol) * M2;
  const int nth = blockDim.x, tid = threadIdx.x;
  for (int k = tid; k < M2; k += nth) tw2[k] = d.tw[d.f2.tw + k];
  Cplx<R>* base = spec + static_cast<size_t>(plane) * M2 * H + m0;
  for (int k = tid; k < M2 * nc; k += nth) {
    int c;
    const int y = dnc.div(k, c);
    A[k] = base[static_cast<size_t>(y) * H + c];
  }
  __syncthreads();
  const Cplx<R>* res = fft_lines(A, B, d.f2, nc, 1, nc, tw2, inverse != 0, nth);
  for (int k = tid; k < M2 * nc; k += nth) {
    int c;
    const int y = dnc.div(k, c);
    base[static_cast<size_t>(y) * H + c] = res[k];
  }
}

// inverse x pass (complex-to-real) of component comp = blockIdx.y
template <typename R>
__global__ void __launch_bounds__(256) k_fft_x_inv(DevPlan<R> d, int npb) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int M1 = d.M1, M2 = d.M2, H = d.H;
  const int npairs = (M2 + 1) / 2, total = npairs * d.M3;
  const Divisor dM1(M1), dnp(npairs);
  const int q0 = xcd_block(blockIdx.x, gridDim.x) * npb, np = min(npb, total - q0);
  const int comp = blockIdx.y;
  Cplx<R>* A = reinterpret_cast<Cplx<R>*>(smem);
  Cplx<R>* B = A + static_cast<size_t>(npb) * M1;
  Cplx<R>* tw1 = B + static_cast<size_t>(npb) * M1;
  const int nth = blockDim.x, tid = threadIdx.x;
  for (int k = tid; k < M1; k += nth) tw1[k] = d.tw[d.f1.tw + k];
  const Cplx<R>* spec = d.spec + static_cast<size_t>(comp) * d.M3 * M2 * H;
  R* phi = d.phi + static_cast<size_t>(comp) * d.M3 * M2 * M1;
  // Hermitian rows a (= row y0) and b (= row y0 + 1): Z[x] = X_a[x] + i X_b[x]
  for (int k = tid; k < np * M1; k += nth) {
    int x;
    const int j = dM1.div(k, x);
    int zr;
    const int q = q0 + j, z = dnp.div(q, zr), y0 = 2 * zr;
    const bool lo = x < H;
    const int xs = lo ? x : M1 - x;
    const Cplx<R>* row = spec + (static_cast<size_t>(z) * M2 + y0) * H;
    Cplx<R> a = row[xs];
    Cplx<R> b = y0 + 1 < M2 ? row[H + xs] : Cplx<R>{R(0), R(0)};
    if (!lo) {
      a.y = -a.y;
      b.y = -b.y;
    }
    A[k] = {a.x - b.y, a.y + b.x};
  }
  __syncthreads();
  const Cplx<R>* res = fft_lines(A, B, d.f1, np, M1, 1, tw1, true, nth);
  for (int k = tid; k < np * M1; k += nth) {
    int x;
    const int j = dM1.div(k, x);
    int zr;
    const int q = q0 + j, z = dnp.div(q, zr), y0 = 2 * zr;
    const size_t r0 = (static_cast<size_t>(z) * M2 + y0) * M1 + x;
    phi[r0] = res[k].x;
    if (y0 + 1 < M2) phi[r0 + M1] = res[k].y;
  }
}

// ------------------------------------------------------------------- FFT z
// Both kernel series at z by Clenshaw's recurrence: c holds (f_k, g_k)
// pairs, zero-padded to degree n (a multiple of 4), so the loop takes four
// degrees per trip and the two recurrences run as independent chains (one
// series at a time, in a loop of one degree per trip, spent most of the z
// pass's VALU issue).
template <typename R>
__device__ __forceinline__ void clenshaw2(const Cplx<R>* __restrict__ c, int n, R z, R& f, R& g) {
  const R z2 = z + z;
  R b1 = R(0), b2 = R(0), e1 = R(0), e2 = R(0);
  for (int k = n; k > 0; k -= 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const Cplx<R> ck = c[k - u];
      const R b0 = z2 * b1 - b2 + ck.x;
      const R e0 = z2 * e1 - e2 + ck.y;
      b2 = b1;
      b1 = b0;
      e2 = e1;
      e1 = e0;
    }
  }
  f = z * b1 - b2 + c[0].x;
  g = z * e1 - e2 + c[0].y;
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

template <typename R, bool BATCH>
__global__ void __launch_bounds__(256) k_fft_z(KArg<R, BATCH> ka, int mode) {
  extern __shared__ __align__(16) unsigned char smem[];
  int blk;
  const DevPlan<R>& d = plan_of(ka, blk);
  const int M1 = d.M1, M2 = d.M2, M3 = d.M3, H = d.H, cz = d.cz;
  const int ngrp = (H + cz - 1) / cz;
  const int y = blk / ngrp;
  const int k0 = (blk - y * ngrp) * cz;
  const int nc = min(cz, H - k0);
  const Divisor dnc(nc);
  double* red = reinterpret_cast<double*>(smem);                   // kNumSums x 16
  Cplx<R>* A = reinterpret_cast<Cplx<R>*>(red + kNumSums * 16);
  Cplx<R>* B = A + cz * M3;
  Cplx<R>* C = B + cz * M3;                                        // component buffer (Z_IK, Z_LOCAL)
  Cplx<R>* tw3 = C + (mode >= Z_IK ? cz * M3 : 0);
  Cplx<R>* kc = tw3 + M3;                                          // kernel coefficient pairs
  R* fw = reinterpret_cast<R*>(kc + d.nker + 1);                   // Z_LOCAL: F_hat / (2 V W_hat^2)
  R* bw = fw + (mode == Z_LOCAL ? cz * M3 : 0);                    //          beta / (2 V W_hat^2)
  const int nth = blockDim.x, tid = threadIdx.x;
  const size_t colstride = static_cast<size_t>(M2) * H;
  Cplx<R>* col = d.spec + static_cast<size_t>(y) * H + k0;
  // prologue: the column, twiddle and kernel-table loads are all issued
  // before the first LDS store, so their round trips overlap
  // (indices are clamped so that the loads need no branches)
  constexpr int U = 4;
  Cplx<R> cv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = min(tid + u * nth, nc * M3 - 1);
    int c;
    const int z = dnc.div(k, c);
    cv[u] = col[z * colstride + c];
  }
  const Cplx<R> twv = d.tw[d.f3.tw + min(tid, M3 - 1)];
  const Cplx<R> kcv = d.kerfg[min(tid, d.nker)];
  // the 1 / W_hat^2 factors of the scaling, fetched with the column
  R iw1p[U], iw3p[U];
  const R iwy = d.iw2[y];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int k = min(tid + u * nth, nc * M3 - 1);
    int c;
    const int z = dnc.div(k, c);
    iw1p[u] = d.iw1[k0 + c];
    iw3p[u] = d.iw3[z];
  }
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (tid + u * nth < nc * M3) A[tid + u * nth] = cv[u];
  if (tid < M3) tw3[tid] = twv;
  if (tid <= d.nker) kc[tid] = kcv;
  for (int k = tid + nth; k < M3; k += nth) tw3[k] = d.tw[d.f3.tw + k];
  for (int k = tid + nth; k <= d.nker; k += nth) kc[k] = d.kerfg[k];
  for (int k = tid + U * nth; k < nc * M3; k += nth) {
    int c;
    const int z = dnc.div(k, c);
    A[k] = col[z * colstride + c];
  }
  __syncthreads();
  Cplx<R>* res = fft_lines(A, B, d.f3, nc, 1, nc, tw3, false, nth);
  if (mode == Z_FFT_ONLY) {
    for (int k = tid; k < nc * M3; k += nth) {
      int c;
      const int z = dnc.div(k, c);
      col[z * colstride + c] = res[k];
    }
    return;
  }
  Acc<R> acc[kNumSums];
  const int m2 = y <= (M2 - 1) / 2 ? y : y - M2;
  // element k of the block; iw = 1 / W_hat^2 of its mode
  auto scale_one = [&](int k, R iw) {
    int c;
    const int z = dnc.div(k, c);
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
    R g = R(0), fl = R(0), bl = R(0);
    if (inside) {
      const R zc = R(2) * kk * d.ysc - R(1);
      R f, xg;
      clenshaw2(kc, d.nker, zc, f, xg);
      const R ik = R(1) / kk;
      const R Fh = d.A * f * ik;
      const R beta = (d.A * xg * ik - R(2) * Fh) * ik;
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
      fl = R(0.5) * g;
      bl = R(0.5) * beta * iw * d.inv_vol;
    }
    if (mode == Z_POTENTIAL || mode == Z_IK) res[k] = cscale(v, g);
    if (mode == Z_LOCAL) {
      fw[k] = fl;
      bw[k] = bl;
    }
  };
#pragma unroll
  for (int u = 0; u < U; ++u)
    if (tid + u * nth < nc * M3) scale_one(tid + u * nth, iw1p[u] * iwy * iw3p[u]);
  for (int k = tid + U * nth; k < nc * M3; k += nth) {
    int c;
    const int z = dnc.div(k, c);
    scale_one(k, d.iw1[k0 + c] * iwy * d.iw3[z]);
  }
  // block sums: wave sums by DPP, one LDS slot per wave, and the barrier that
  // also orders the scaled column before the inverse transform; thread k then
  // adds the wave slots of sum k (in wave order, as block_sum does)
#pragma unroll
  for (int k = 0; k < kNumSums; ++k) {
    const double w = wave_sum_to_last(acc[k].value());
    if ((tid & 63) == 63) red[k * 16 + (tid >> 6)] = w;
  }
  __syncthreads();
  if (tid < kNumSums) {
    const int nw = nth >> 6;
    double s = 0;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
      const double t = red[tid * 16 + w];
      s += w < nw ? t : 0.0;
    }
    d.zpart[static_cast<size_t>(blk) * kNumSums + tid] = s;
  }
  if (mode == Z_ENERGY) return;
  Cplx<R>* oth = res == A ? B : A;
  if (mode == Z_POTENTIAL) {
    res = fft_lines(res, oth, d.f3, nc, 1, nc, tw3, true, nth);
    for (int k = tid; k < nc * M3; k += nth) {
      int c;
      const int z = dnc.div(k, c);
      col[z * colstride + c] = res[k];
    }
    return;
  }
  // Z_IK: the three components i k_a G rho_hat of the field (App. C,
  // eq. rhodiagforce), each inverse-transformed along z into its own half
  // spectrum.  Nyquist modes of even grids have no -m partner and are dropped.
  // Z_LOCAL: the six components P_hat_ab rho_hat / (2 V W_hat^2) (Sec. 4.4,
  // eq. rhodiag), P_hat = F_hat I + beta k k^T.
  const size_t S = static_cast<size_t>(H) * M2 * M3;
  const bool nyq2 = (M2 % 2 == 0) && 2 * y == M2;
  const int ncomp = mode == Z_IK ? 3 : 6;
  for (int a = 0; a < ncomp; ++a) {
    for (int k = tid; k < nc * M3; k += nth) {
      int c;
      const int z = dnc.div(k, c);
      const int i1 = k0 + c;
      const int m1 = i1 <= (M1 - 1) / 2 ? i1 : i1 - M1;
      const int m3 = z <= (M3 - 1) / 2 ? z : z - M3;
      const bool nyq = nyq2 || ((M1 % 2 == 0) && 2 * i1 == M1) || ((M3 % 2 == 0) && 2 * z == M3);
      const R fm1 = R(m1), fm2 = R(m2), fm3 = R(m3);
      const Cplx<R> v = res[k];
      if (mode == Z_IK) {
        const R ka = d.B[3 * a] * fm1 + d.B[3 * a + 1] * fm2 + d.B[3 * a + 2] * fm3;
        C[k] = nyq ? Cplx<R>{R(0), R(0)} : Cplx<R>{-ka * v.y, ka * v.x};   // i k_a (G rho_hat)
      } else {
        // component a -> (i, j): xx yy zz xy xz yz
        const int ci = a < 3 ? a : (a == 5 ? 1 : 0);
        const int cj = a < 3 ? a : (a == 3 ? 1 : 2);
        const R ki = d.B[3 * ci] * fm1 + d.B[3 * ci + 1] * fm2 + d.B[3 * ci + 2] * fm3;
        const R kj = d.B[3 * cj] * fm1 + d.B[3 * cj + 1] * fm2 + d.B[3 * cj + 2] * fm3;
        C[k] = cscale(v, (ci == cj ? fw[k] : R(0)) + bw[k] * ki * kj);
      }
    }
    __syncthreads();
    Cplx<R>* out = fft_lines(C, oth, d.f3, nc, 1, nc, tw3, true, nth);
    Cplx<R>* dst = col + a * S;
    for (int k = tid; k < nc * M3; k += nth) {
      int c;
      const int z = dnc.div(k, c);
      dst[z * colstride + c] = out[k];
    }
    __syncthreads();
  }
}

template <typename R>
__global__ void k_grid_out(DevPlan<R> d, R* __restrict__ out, size_t count) {
  const double inv = ldexp(1.0, -d.gexp[0]);
  for (size_t k = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < count;
       k += static_cast<size_t>(gridDim.x) * blockDim.x) {
    out[k] = static_cast<R>(static_cast<double>(d.rhofix[k]) * inv);
    d.rhofix[k] = 0;
  }
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, size_t count) {
  for (size_t k = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; k < count;
       k += static_cast<size_t>(gridDim.x) * blockDim.x)
    p[k] = T(0);
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
  const size_t col = static_cast<size_t>(d.cz) * d.M3;
  return ((d.ncomp > 1 ? 3 : 2) * col + d.M3) * sizeof(Cplx<R>) +
         (2 * (d.nker + 1) + 2 + (d.local ? 2 * col : 0)) * sizeof(R) + kNumSums * 16 * sizeof(double) + 16;
}

template <typename R>
size_t lds_spread(const DevPlan<R>& d) {
  const size_t cells = ((static_cast<size_t>(d.T1 + d.P - 1) * (d.T2 + d.P - 1)) | 1) * (d.T3 + d.P - 1);
  return cells * sizeof(double) + (kSpreadWaves * kWaveChunk * 3 * d.P + d.P * (d.nw + 1)) * sizeof(R) +
         kSpreadWaves * kWaveChunk * 4 * sizeof(int) + 16;
}

// Raise the dynamic-LDS limit of a kernel when a launch needs more than 64 KiB.
inline void allow_lds(const void* fn, size_t lds) {
  if (lds > 65536)
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
}

template <typename R>
inline KArg<R, true> karg(const BatchLaunch<R>& b) {
  return KArg<R, true>{b.plans, b.boff, b.nrep};
}

template <typename R>
size_t lds_gather_box(const DevPlan<R>& d) {
  const size_t E1 = std::min(d.T1, d.M1) + d.P - 1, E2 = std::min(d.T2, d.M2) + d.P - 1,
               E3 = std::min(d.T3, d.M3) + d.P - 1;
  return E1 * E2 * E3 * sizeof(R);
}

template <typename R>
hipError_t launch_bin(const DevPlan<R>& d, const R* xyz, const R* q, hipStream_t s) {
  const size_t lds = d.bin_lds ? static_cast<size_t>(d.ntiles) * sizeof(int) : 0;
  if (d.binppt > 1)
    ESP_LAUNCH((k_bin<R, false, kBinMaxPpt>), dim3(d.nbin), dim3(kBinThreads), lds, s, KArg<R, false>{d}, xyz, q);
  else
    ESP_LAUNCH((k_bin<R, false, 1>), dim3(d.nbin), dim3(kBinThreads), lds, s, KArg<R, false>{d}, xyz, q);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_scatter(const DevPlan<R>& d, hipStream_t s) {
  const int nb = static_cast<int>((d.n + 1023) / 1024);
  const size_t lds = (static_cast<size_t>(d.ntiles) + 1) * sizeof(int);
  allow_lds(reinterpret_cast<const void*>(&k_scatter<R, false>), lds);
  ESP_LAUNCH((k_scatter<R, false>), dim3(nb), dim3(1024), lds, s, KArg<R, false>{d});
  return hipGetLastError();
}

template <typename R>
hipError_t launch_scan_sub(const DevPlan<R>& d, hipStream_t s) {
  ESP_LAUNCH((k_scan_sub<R, false>), dim3(1), dim3(1024), 0, s, KArg<R, false>{d});
  return hipGetLastError();
}

template <typename R>
hipError_t launch_finalize(const DevPlan<R>& d, double* out7, hipStream_t s) {
  ESP_LAUNCH((k_finalize<R, false>), dim3(1), dim3(256), 0, s, KArg<R, false>{d}, out7);
  return hipGetLastError();
}

#define ESP_P_SWITCH(PV, FN, ...)             \
  switch (PV) {                               \
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
  ESP_P_SWITCH(d.P, spread_launch, d, s)
}

template <typename R>
hipError_t launch_gather_local(const DevPlan<R>& d, R* w6, double* out7, hipStream_t s) {
  ESP_P_SWITCH(d.P, gather_local_launch, d, w6, out7, s)
}

template <typename R>
hipError_t launch_gather(const DevPlan<R>& d, R* f, double* out7, hipStream_t s) {
  if (d.ik) {
    ESP_P_SWITCH(d.P, gather_ik_launch, d, f, out7, s)
  }
  ESP_P_SWITCH(d.P, gather_launch, d, f, out7, s)
}

template <typename R>
size_t lds_fft_x(const DevPlan<R>& d, int npb) {
  return (2 * static_cast<size_t>(npb) + 1) * d.M1 * sizeof(Cplx<R>);
}

template <typename R>
size_t lds_fft_y(const DevPlan<R>& d, int ncol) {
  return (2 * static_cast<size_t>(ncol) + 1) * d.M2 * sizeof(Cplx<R>);
}

template <typename R>
hipError_t launch_fft_xy(const DevPlan<R>& d, const R* grid, Cplx<R>* spec, bool clear_input,
                         hipStream_t s) {
  const bool gf = sizeof(R) == 4 && grid == nullptr && d.grid_fixed;
  if (d.xy_split) {
    const int total = (d.M2 + 1) / 2 * d.M3;
    size_t lds = lds_fft_x(d, d.xpairs);
    const dim3 nb((total + d.xpairs - 1) / d.xpairs);
    if (gf) {
      allow_lds(reinterpret_cast<const void*>(&k_fft_x<R, true>), lds);
      ESP_LAUNCH((k_fft_x<R, true>), nb, dim3(256), lds, s, d, grid, spec, clear_input ? 1 : 0, d.xpairs);
    } else {
      allow_lds(reinterpret_cast<const void*>(&k_fft_x<R, false>), lds);
      ESP_LAUNCH((k_fft_x<R, false>), nb, dim3(256), lds, s, d, grid, spec, clear_input ? 1 : 0, d.xpairs);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    lds = lds_fft_y(d, d.ycols);
    allow_lds(reinterpret_cast<const void*>(&k_fft_y<R>), lds);
    ESP_LAUNCH(k_fft_y<R>, dim3(d.M3 * ((d.H + d.ycols - 1) / d.ycols)), dim3(256), lds, s, d, spec,
                       d.ycols, 0);
    return hipGetLastError();
  }
  const size_t lds = lds_fft_xy(d);
  const int nth = fft_threads(d.M1 * d.M2);
  if (gf) {
    allow_lds(reinterpret_cast<const void*>(&k_fft_xy<R, false, true>), lds);
    ESP_LAUNCH((k_fft_xy<R, false, true>), dim3(d.M3), dim3(nth), lds, s, KArg<R, false>{d}, grid, spec,
               clear_input ? 1 : 0);
  } else {
    allow_lds(reinterpret_cast<const void*>(&k_fft_xy<R, false, false>), lds);
    ESP_LAUNCH((k_fft_xy<R, false, false>), dim3(d.M3), dim3(nth), lds, s, KArg<R, false>{d}, grid, spec,
               clear_input ? 1 : 0);
  }
  return hipGetLastError();
}

template <typename R>
hipError_t launch_fft_xy_inv(const DevPlan<R>& d, int ncomp, hipStream_t s) {
  if (d.xy_split) {
    size_t lds = lds_fft_y(d, d.ycols);
    allow_lds(reinterpret_cast<const void*>(&k_fft_y<R>), lds);
    ESP_LAUNCH(k_fft_y<R>, dim3(ncomp * d.M3 * ((d.H + d.ycols - 1) / d.ycols)), dim3(256), lds, s, d,
                       static_cast<Cplx<R>*>(nullptr), d.ycols, 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int total = (d.M2 + 1) / 2 * d.M3;
    lds = lds_fft_x(d, d.xpairs);
    allow_lds(reinterpret_cast<const void*>(&k_fft_x_inv<R>), lds);
    ESP_LAUNCH(k_fft_x_inv<R>, dim3((total + d.xpairs - 1) / d.xpairs, ncomp), dim3(256), lds, s, d,
                       d.xpairs);
    return hipGetLastError();
  }
  const size_t lds = lds_fft_xy(d);
  allow_lds(reinterpret_cast<const void*>(&k_fft_xy_inv<R, false>), lds);
  const int nth = fft_threads(d.M1 * d.M2);
  ESP_LAUNCH((k_fft_xy_inv<R, false>), dim3(d.M3 * ncomp), dim3(nth), lds, s, KArg<R, false>{d});
  return hipGetLastError();
}

template <typename R>
hipError_t launch_fft_z(const DevPlan<R>& d, ZMode mode, hipStream_t s) {
  const size_t lds = lds_fft_z(d);
  allow_lds(reinterpret_cast<const void*>(&k_fft_z<R, false>), lds);
  ESP_LAUNCH((k_fft_z<R, false>), dim3(d.nzblk), dim3(256), lds, s, KArg<R, false>{d},
                     static_cast<int>(mode));
  return hipGetLastError();
}

// ------------------------------------------------------- batched launchers
template <typename R>
hipError_t launch_bin_batch(const BatchLaunch<R>& b, const R* xyz, const R* q, hipStream_t s) {
  if (b.ppt > 1) {
    allow_lds(reinterpret_cast<const void*>(&k_bin<R, true, kBinMaxPpt>), b.lds);
    ESP_LAUNCH((k_bin<R, true, kBinMaxPpt>), dim3(b.nblk), dim3(b.nth), b.lds, s, karg(b), xyz, q);
  } else {
    allow_lds(reinterpret_cast<const void*>(&k_bin<R, true, 1>), b.lds);
    ESP_LAUNCH((k_bin<R, true, 1>), dim3(b.nblk), dim3(b.nth), b.lds, s, karg(b), xyz, q);
  }
  return hipGetLastError();
}

template <typename R>
hipError_t launch_scatter_batch(const BatchLaunch<R>& b, hipStream_t s) {
  allow_lds(reinterpret_cast<const void*>(&k_scatter<R, true>), b.lds);
  ESP_LAUNCH((k_scatter<R, true>), dim3(b.nblk), dim3(b.nth), b.lds, s, karg(b));
  return hipGetLastError();
}

template <typename R>
hipError_t launch_scan_sub_batch(const BatchLaunch<R>& b, hipStream_t s) {
  ESP_LAUNCH((k_scan_sub<R, true>), dim3(b.nblk), dim3(1024), 0, s, karg(b));
  return hipGetLastError();
}

template <typename R>
hipError_t launch_spread_batch(const BatchLaunch<R>& b, hipStream_t s) {
  ESP_P_SWITCH(b.P, spread_launch_batch, b, s)
}

template <typename R>
hipError_t launch_gather_batch(const BatchLaunch<R>& b, R* f, double* out7, hipStream_t s) {
  ESP_P_SWITCH(b.P, gather_launch_batch, b, f, out7, s)
}

template <typename R>
hipError_t launch_fft_xy_batch(const BatchLaunch<R>& b, hipStream_t s) {
  // deterministic FP32 batches read their replicas' int64 grids
  if (sizeof(R) == 4 && b.grid_fixed) {
    allow_lds(reinterpret_cast<const void*>(&k_fft_xy<R, true, true>), b.lds);
    ESP_LAUNCH((k_fft_xy<R, true, true>), dim3(b.nblk), dim3(b.nth), b.lds, s, karg(b),
               static_cast<const R*>(nullptr), static_cast<Cplx<R>*>(nullptr), 1);
  } else {
    allow_lds(reinterpret_cast<const void*>(&k_fft_xy<R, true, false>), b.lds);
    ESP_LAUNCH((k_fft_xy<R, true, false>), dim3(b.nblk), dim3(b.nth), b.lds, s, karg(b),
               static_cast<const R*>(nullptr), static_cast<Cplx<R>*>(nullptr), 1);
  }
  return hipGetLastError();
}

template <typename R>
hipError_t launch_fft_xy_inv_batch(const BatchLaunch<R>& b, hipStream_t s) {
  allow_lds(reinterpret_cast<const void*>(&k_fft_xy_inv<R, true>), b.lds);
  ESP_LAUNCH((k_fft_xy_inv<R, true>), dim3(b.nblk), dim3(b.nth), b.lds, s, karg(b));
  return hipGetLastError();
}

template <typename R>
hipError_t launch_fft_z_batch(const BatchLaunch<R>& b, ZMode mode, hipStream_t s) {
  allow_lds(reinterpret_cast<const void*>(&k_fft_z<R, true>), b.lds);
  ESP_LAUNCH((k_fft_z<R, true>), dim3(b.nblk), dim3(b.nth), b.lds, s, karg(b), static_cast<int>(mode));
  return hipGetLastError();
}

template <typename R>
hipError_t launch_finalize_batch(const BatchLaunch<R>& b, double* out7, hipStream_t s) {
  ESP_LAUNCH((k_finalize<R, true>), dim3(b.nblk), dim3(256), 0, s, karg(b), out7);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T* p, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const int nb = static_cast<int>(std::min<size_t>((count + 255) / 256, 4096));
  ESP_LAUNCH(k_fill<T>, dim3(nb), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_grid_out(const DevPlan<R>& d, R* out, hipStream_t s) {
  const size_t count = static_cast<size_t>(d.M1) * d.M2 * d.M3;
  const int nb = static_cast<int>(std::min<size_t>((count + 255) / 256, 4096));
  ESP_LAUNCH(k_grid_out<R>, dim3(nb), dim3(256), 0, s, d, out, count);
  return hipGetLastError();
}

#define ESP_INSTANTIATE(R)                                                                    \
  template hipError_t launch_bin<R>(const DevPlan<R>&, const R*, const R*, hipStream_t);      \
  template hipError_t launch_scatter<R>(const DevPlan<R>&, hipStream_t);                      \
  template hipError_t launch_scan_sub<R>(const DevPlan<R>&, hipStream_t);                     \
  template hipError_t launch_scan_sub_batch<R>(const BatchLaunch<R>&, hipStream_t);           \
  template hipError_t launch_finalize<R>(const DevPlan<R>&, double*, hipStream_t);            \
  template hipError_t launch_spread<R>(const DevPlan<R>&, hipStream_t);                       \
  template hipError_t launch_fft_xy<R>(const DevPlan<R>&, const R*, Cplx<R>*, bool, hipStream_t); \
  template hipError_t launch_fft_z<R>(const DevPlan<R>&, ZMode, hipStream_t);                 \
  template hipError_t launch_fft_xy_inv<R>(const DevPlan<R>&, int, hipStream_t);              \
  template hipError_t launch_gather_local<R>(const DevPlan<R>&, R*, double*, hipStream_t);    \
  template hipError_t launch_gather<R>(const DevPlan<R>&, R*, double*, hipStream_t);          \
  template hipError_t launch_bin_batch<R>(const BatchLaunch<R>&, const R*, const R*, hipStream_t); \
  template hipError_t launch_scatter_batch<R>(const BatchLaunch<R>&, hipStream_t);            \
  template hipError_t launch_spread_batch<R>(const BatchLaunch<R>&, hipStream_t);             \
  template hipError_t launch_fft_xy_batch<R>(const BatchLaunch<R>&, hipStream_t);             \
  template hipError_t launch_fft_z_batch<R>(const BatchLaunch<R>&, ZMode, hipStream_t);       \
  template hipError_t launch_fft_xy_inv_batch<R>(const BatchLaunch<R>&, hipStream_t);         \
  template hipError_t launch_gather_batch<R>(const BatchLaunch<R>&, R*, double*, hipStream_t); \
  template hipError_t launch_finalize_batch<R>(const BatchLaunch<R>&, double*, hipStream_t);  \
  template hipError_t launch_fill<R>(R*, size_t, hipStream_t);                                \
  template hipError_t launch_grid_out<R>(const DevPlan<R>&, R*, hipStream_t);                 \
  template size_t lds_fft_xy<R>(const DevPlan<R>&);                                           \
  template size_t lds_fft_x<R>(const DevPlan<R>&, int);                                       \
  template size_t lds_fft_y<R>(const DevPlan<R>&, int);                                       \
  template size_t lds_fft_z<R>(const DevPlan<R>&);                                            \
  template size_t lds_spread<R>(const DevPlan<R>&);                                           \
  template size_t lds_gather_box<R>(const DevPlan<R>&);

ESP_INSTANTIATE(float)
ESP_INSTANTIATE(double)
template hipError_t launch_fill<int>(int*, size_t, hipStream_t);
template hipError_t launch_fill<long long>(long long*, size_t, hipStream_t);

}  // namespace espx
