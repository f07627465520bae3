// Real-space (near) part of the PSWF kernel split (paper Sec. 3.1, eq. UN,
// eq. PinsN, eq. Fc with eq. mathFN): energy, virial and forces of the pairs
// closer than rc, after a cell sort with cells of perpendicular width >= rc
// along the cell vectors.  Every pair within rc then lies in adjacent cells
// and, with rc below half the smallest width, its separation is the minimum
// image in reduced coordinates.
//
// Each unordered pair within rc is evaluated once (Newton's third law): the
// cell with the lower index handles a pair of neighbouring cells, and within
// a cell a particle pairs with the ones sorted after it.  Workgroups of 256
// threads, rsplit per home cell, each take an equal share of the cell's
// candidate list (the particles of the neighbouring cells kept for it, the
// home cell included), so that small systems still fill the chip.
// Candidates are staged through LDS in chunks; thread t tests home particle
// t % HC against every (256 / HC)-th candidate (a residue class that differs
// between the lanes of a group), HC in {16, 32, 64} chosen per cell to waste
// the fewest lanes.  Pairs within rc go to a per-wave queue and
// are evaluated 64 at a time on full waves.  The force on the home particle
// accumulates in LDS per thread and is summed over its thread group into a
// per-share array that a second kernel adds in a fixed order; the reaction
// on the candidate accumulates in LDS per staged record and is added to an
// FP64 array with one atomic per record and chunk.  The split functions of
// x = r / rc, 1 - phi0(x) (N^c = that / r) and
// F_N(x) = 1 - phi0(x) + x psi(x) / C0 (pair force q_i q_j F_N d / r^3), are
// piecewise polynomials on nseg equal segments of [0, 1].
#include <hip/hip_runtime.h>

#include "esp_common.h"

namespace espx {

constexpr int kRealThreads = 256;
constexpr int kRealStage = 256;      // candidate records staged per round

// 1 / sqrt(x): the hardware reciprocal square root (1 ulp) in FP32, the
// correctly rounded quotient in FP64.
__device__ __forceinline__ float inv_sqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double inv_sqrt(double x) { return 1.0 / sqrt(x); }

template <typename R, int NC>
__device__ __forceinline__ R horner(const R* __restrict__ c, R t) {
  R v = c[NC - 1];
#pragma unroll
  for (int k = NC - 2; k >= 0; --k) v = v * t + c[k];
  return v;
}

template <typename R>
__global__ void __launch_bounds__(kRealThreads) __attribute__((amdgpu_waves_per_eu(6))) k_real_pairs(DevPlan<R> d) {
  constexpr int NC = kRealDeg<R> + 1;
  __shared__ Record<R> stage[kRealStage];
  __shared__ Record<R> home[kRealThreads];       // each thread's home particle
  __shared__ double fsh[3 * kRealThreads];       // each thread's home-particle force (FP64: the
                                                 // LDS float add is slow on this chip)
  __shared__ double jf[3 * kRealStage];          // reaction forces on the staged candidates
  __shared__ int sidx[kRealStage];               // sorted index of each staged candidate
  __shared__ int wqueue[3 * kRealThreads];       // per wave: pairs within rc awaiting evaluation
  __shared__ double red[kNumSums * 16];
  __shared__ int nstart[27], ncnt[27], ncum[28];
  extern __shared__ __align__(16) unsigned char smem[];
  R* tab = reinterpret_cast<R*>(smem);          // nseg x {N, F} x NC coefficients
  const int ncells = d.cn1 * d.cn2 * d.cn3;
  const int cell = blockIdx.x % ncells, ks = blockIdx.x / ncells, tid = threadIdx.x;
  const int nseg = d.nrs;
  for (int k = tid; k < nseg * 2 * NC; k += kRealThreads) tab[k] = d.rsN[k];
  {
    // neighbour cell at offset (o1, o2, o3) in {-1, 0, 1}^3; along a dimension
    // with only 2 cells the offsets -1 and +1 name the same cell, so -1 is
    // left out.  Each unordered pair of cells is handled once, by the lower
    // cell index (slot 13, the cell itself, holds the pairs within it).
    // Empty slots stay in the list with no particles.
    if (tid < 27) {
      const int o1 = tid % 3 - 1, o2 = (tid / 3) % 3 - 1, o3 = tid / 9 - 1;
      const bool ok = (d.cn1 > 2 || o1 >= 0) && (d.cn2 > 2 || o2 >= 0) && (d.cn3 > 2 || o3 >= 0);
      int st = 0, en = 0;
      if (ok) {
        const int c1 = (cell % d.cn1 + o1 + d.cn1) % d.cn1;
        const int c2 = ((cell / d.cn1) % d.cn2 + o2 + d.cn2) % d.cn2;
        const int c3 = (cell / (d.cn1 * d.cn2) + o3 + d.cn3) % d.cn3;
        const int nc = (c3 * d.cn2 + c2) * d.cn1 + c1;
        if (nc >= cell) {
          st = d.offsets[nc];
          en = d.offsets[nc + 1];
        }
      }
      nstart[tid] = st;
      ncnt[tid] = en - st;
    }
    __syncthreads();
    if (tid == 0) {
      int run = 0;
      for (int m = 0; m < 27; ++m) {
        ncum[m] = run;
        run += ncnt[m];
      }
      ncum[27] = run;
      if (ks == 0) d.counts[cell] = 0;          // ready for the next binning pass
    }
  }
  __syncthreads();
  const int hs = d.offsets[cell], he = d.offsets[cell + 1], nh = he - hs;
  // this block's share of the candidate list
  const int total = ncum[27];
  const int clo = static_cast<int>(static_cast<int64_t>(total) * ks / d.rsplit);
  const int chi = static_cast<int>(static_cast<int64_t>(total) * (ks + 1) / d.rsplit);
  // home-particle group size with the fewest idle lanes (ties: the larger)
  int HC = 64;
  {
    int best = ((nh + 63) / 64) * 64;
    for (int c = 32; c >= 16; c >>= 1) {
      const int w = ((nh + c - 1) / c) * c;
      if (w < best) {
        best = w;
        HC = c;
      }
    }
  }
  const int G = kRealThreads / HC, hi = tid % HC, g = tid / HC;
  const R nsegr = static_cast<R>(nseg);
  R* fpart = d.fpart + static_cast<size_t>(ks) * d.n * 3;
  const int self0 = ncum[13], self1 = ncum[14];   // candidates of the home cell itself
  const int lane = tid & 63, wbase = tid & ~63;
  int* queue = wqueue + 3 * wbase;              // this wave's 192 entries
  double part[kNumSums];
#pragma unroll
  for (int k = 0; k < kNumSums; ++k) part[k] = 0.0;
  // energy and virial of the pairs this lane evaluates, folded into FP64 per chunk
  R u = R(0), w0 = R(0), w1 = R(0), w2 = R(0), w3 = R(0), w4 = R(0), w5 = R(0);
  // Evaluate queue entries [0, cnt) of this wave, one per lane (cnt <= 64):
  // entry = (lane of the home particle << 16) | candidate slot.
  auto evaluate = [&](int cnt) {
    if (lane < cnt) {
      const int e = queue[lane];
      const int src = wbase + (e >> 16);
      const Record<R> ri = home[src];
      const Record<R> rj = stage[e & 0xffff];
      R ds[3];
      Coord<R>::disp(ri, rj, ds);
      const R dx = d.hmat[0] * ds[0] + d.hmat[1] * ds[1] + d.hmat[2] * ds[2];
      const R dy = d.hmat[3] * ds[0] + d.hmat[4] * ds[1] + d.hmat[5] * ds[2];
      const R dz = d.hmat[6] * ds[0] + d.hmat[7] * ds[1] + d.hmat[8] * ds[2];
      const R r2 = dx * dx + dy * dy + dz * dz;
      const R ir = inv_sqrt(r2);
      const R xs = r2 * ir * d.inv_rc * nsegr;
      const int sg = min(nseg - 1, static_cast<int>(xs));
      const R t = xs - static_cast<R>(sg) - R(0.5);
      const R* cf = tab + sg * 2 * NC;
      const R qq = ri.q * rj.q;
      const R gn = horner<R, NC>(cf, t), gf = horner<R, NC>(cf + NC, t);
      const R fw = qq * gf * ir * ir * ir;
      const R wx = fw * dx, wy = fw * dy, wz = fw * dz;
      const int js = e & 0xffff;
      atomicAdd(fsh + 3 * src + 0, static_cast<double>(wx));
      atomicAdd(fsh + 3 * src + 1, static_cast<double>(wy));
      atomicAdd(fsh + 3 * src + 2, static_cast<double>(wz));
      atomicAdd(jf + 3 * js + 0, -static_cast<double>(wx));
      atomicAdd(jf + 3 * js + 1, -static_cast<double>(wy));
      atomicAdd(jf + 3 * js + 2, -static_cast<double>(wz));
      u += qq * gn * ir;
      w0 += wx * dx;
      w1 += wy * dy;
      w2 += wz * dz;
      w3 += wx * dy;
      w4 += wx * dz;
      w5 += wy * dz;
    }
  };
  // stage candidates [c0, c0 + nc) with their sorted indices and cleared reactions
  auto stage_chunk = [&](int c0, int nc) {
    for (int k = tid; k < nc; k += kRealThreads) {
      const int cand = c0 + k;
      int lo = 0, hi2 = 26;                     // slot m with ncum[m] <= cand < ncum[m + 1]
      while (lo < hi2) {
        const int mid = (lo + hi2 + 1) >> 1;
        if (ncum[mid] <= cand) lo = mid; else hi2 = mid - 1;
      }
      const int idx = nstart[lo] + cand - ncum[lo];
      stage[k] = d.sorted[idx];
      sidx[k] = idx;
      jf[3 * k + 0] = 0.0;
      jf[3 * k + 1] = 0.0;
      jf[3 * k + 2] = 0.0;
    }
  };
  // add the staged reactions to the FP64 force array (after a barrier)
  auto flush_reactions = [&](int nc) {
    for (int k = tid; k < nc; k += kRealThreads) {
      double* dst = d.facc + 3 * static_cast<size_t>(sidx[k]);
      const double a = jf[3 * k + 0], b = jf[3 * k + 1], c = jf[3 * k + 2];
      if (a != 0.0 || b != 0.0 || c != 0.0) {
        atomicAdd(dst + 0, a);
        atomicAdd(dst + 1, b);
        atomicAdd(dst + 2, c);
      }
    }
  };
  // a share that fits in one chunk is staged once for all home passes
  const bool once = chi - clo <= kRealStage;
  if (once) stage_chunk(clo, chi - clo);
  for (int h0 = hs; h0 < he; h0 += HC) {
    const int i = h0 + hi;
    const bool own = i < he;
    const Record<R> ri = d.sorted[own ? i : hs];
    home[tid] = ri;
    fsh[3 * tid + 0] = 0.0;
    fsh[3 * tid + 1] = 0.0;
    fsh[3 * tid + 2] = 0.0;
    for (int c0 = clo; c0 < chi; c0 += kRealStage) {
      const int nc = min(kRealStage, chi - c0);
      __syncthreads();                          // previous chunk consumed; home and fsh set
      if (!once) {
        stage_chunk(c0, nc);
        __syncthreads();
      }
      // test phase: every lane takes the same number of steps, so the wave
      // stays converged; pairs within rc are appended to the wave's queue and
      // evaluated 64 at a time
      int count = 0;
      // is candidate jj within rc of this lane's home particle (and, within
      // the home cell, sorted after it)?
      auto test = [&](int jj) {
        bool hit = false;
        if (own && jj < nc) {
          const Record<R> rj = stage[jj];
          R n[3];
          Coord<R>::disp_raw(ri, rj, n);
          // r^2 from the metric h^T h (the evaluation recomputes d itself)
          const R t0 = d.gmet[0] * n[0] + d.gmet[3] * n[1] + d.gmet[4] * n[2];
          const R t1 = d.gmet[1] * n[1] + d.gmet[5] * n[2];
          const R r2 = n[0] * t0 + n[1] * t1 + n[2] * (d.gmet[2] * n[2]);
          const int cand = c0 + jj;
          hit = r2 < d.rc2 && r2 > R(0) && (cand < self0 || cand >= self1 || cand - self0 > i - hs);
        }
        return hit;
      };
      auto append = [&](bool hit, int jj) {
        const unsigned long long mask = __ballot(hit);
        if (hit) {
          const int below = __builtin_amdgcn_mbcnt_hi(static_cast<unsigned>(mask >> 32),
                                                      __builtin_amdgcn_mbcnt_lo(static_cast<unsigned>(mask), 0u));
          queue[count + below] = (lane << 16) | jj;
        }
        count += __popcll(mask);
      };
      // Lane (g, hi) takes the candidates of residue class (g + hi) mod G, so
      // a home particle still meets every candidate once over its G lanes
      // while the lanes of one group read (and react on) different records.
      // Two candidates per step; every lane takes the same number of steps,
      // so the wave stays converged.
      const int rcls = (g + hi) % G;
      const int steps = (nc + 2 * G - 1) / (2 * G);
      for (int st = 0; st < steps; ++st) {
        const int ja = rcls + 2 * st * G, jb = ja + G;
        const bool ha = test(ja), hb = test(jb);
        append(ha, ja);
        append(hb, jb);
        while (count >= 64) {
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          evaluate(64);
          count -= 64;
          // move the remaining entries (at most 127) to the front: read all, then write
          const int r0 = lane < count ? queue[64 + lane] : 0;
          const int r1 = lane + 64 < count ? queue[128 + lane] : 0;
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          if (lane < count) queue[lane] = r0;
          if (lane + 64 < count) queue[64 + lane] = r1;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      evaluate(count);                          // the chunk's remaining pairs
      if (!once) {
        __syncthreads();                        // every reaction force of the chunk is in jf
        flush_reactions(nc);
      }
      part[0] += static_cast<double>(u);
      part[1] += static_cast<double>(w0);
      part[2] += static_cast<double>(w1);
      part[3] += static_cast<double>(w2);
      part[4] += static_cast<double>(w3);
      part[5] += static_cast<double>(w4);
      part[6] += static_cast<double>(w5);
      u = w0 = w1 = w2 = w3 = w4 = w5 = R(0);
    }
    // sum each home particle's forces over its thread group
    __syncthreads();
    if (tid < HC && h0 + tid < he) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
      for (int k = 0; k < G; ++k) {
        const int t = k * HC + tid;
        s0 += fsh[3 * t + 0];
        s1 += fsh[3 * t + 1];
        s2 += fsh[3 * t + 2];
      }
      const size_t o = static_cast<size_t>(h0 + tid) * 3;
      fpart[o + 0] = static_cast<R>(s0);
      fpart[o + 1] = static_cast<R>(s1);
      fpart[o + 2] = static_cast<R>(s2);
    }
    __syncthreads();                            // fsh read before it is cleared again
  }
  __syncthreads();
  if (once) flush_reactions(chi - clo);
  block_sum<kNumSums>(part, red);
  if (tid == 0)
#pragma unroll
    for (int k = 0; k < kNumSums; ++k) d.rpart[static_cast<size_t>(blockIdx.x) * kNumSums + k] = part[k];
}

// Near forces in input order: the candidate shares summed, times coulomb_k,
// written to f or added to it.
template <typename R>
__global__ void __launch_bounds__(256) k_real_forces(DevPlan<R> d, R* __restrict__ f, int accumulate) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  double s[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    s[a] = d.facc[3 * i + a];
    d.facc[3 * i + a] = 0.0;                    // zero again for the next call
  }
  for (int k = 0; k < d.rsplit; ++k)
#pragma unroll
    for (int a = 0; a < 3; ++a) s[a] += static_cast<double>(d.fpart[(static_cast<size_t>(k) * d.n + i) * 3 + a]);
  const int64_t j = d.perm[i];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const R v = static_cast<R>(d.fin.coulomb_k * s[a]);
    f[3 * j + a] = accumulate ? f[3 * j + a] + v : v;
  }
}

template <typename R>
__global__ void __launch_bounds__(256) k_real_finalize(DevPlan<R> d, double* __restrict__ out7, int add) {
  __shared__ double red[kNumSums * 16];
  const int nblk = d.cn1 * d.cn2 * d.cn3 * d.rsplit;
  double v[kNumSums];
#pragma unroll
  for (int k = 0; k < kNumSums; ++k) v[k] = 0.0;
  for (int c = threadIdx.x; c < nblk; c += blockDim.x)
#pragma unroll
    for (int k = 0; k < kNumSums; ++k) v[k] += d.rpart[static_cast<size_t>(c) * kNumSums + k];
  block_sum<kNumSums>(v, red);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < kNumSums; ++k) out7[k] = (add ? out7[k] : 0.0) + d.fin.coulomb_k * v[k];   // each pair once
}

template <typename R>
size_t lds_real(const DevPlan<R>& d) {
  return static_cast<size_t>(d.nrs) * 2 * (kRealDeg<R> + 1) * sizeof(R);
}

template <typename R>
hipError_t launch_real_pairs(const DevPlan<R>& d, hipStream_t s) {
  const size_t lds = lds_real(d);     // at most 40 KiB (segment count capped on the host)
  const int nblk = d.cn1 * d.cn2 * d.cn3 * d.rsplit;
  ESP_LAUNCH(k_real_pairs<R>, dim3(nblk), dim3(kRealThreads), lds, s, d);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_real_forces(const DevPlan<R>& d, R* f, int accumulate, hipStream_t s) {
  ESP_LAUNCH(k_real_forces<R>, dim3(static_cast<unsigned>((d.n + 255) / 256)), dim3(256), 0, s, d, f,
                     accumulate);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_real_finalize(const DevPlan<R>& d, double* out7, int add, hipStream_t s) {
  ESP_LAUNCH(k_real_finalize<R>, dim3(1), dim3(256), 0, s, d, out7, add);
  return hipGetLastError();
}

template size_t lds_real<float>(const DevPlan<float>&);
template size_t lds_real<double>(const DevPlan<double>&);
template hipError_t launch_real_pairs<float>(const DevPlan<float>&, hipStream_t);
template hipError_t launch_real_pairs<double>(const DevPlan<double>&, hipStream_t);
template hipError_t launch_real_forces<float>(const DevPlan<float>&, float*, int, hipStream_t);
template hipError_t launch_real_forces<double>(const DevPlan<double>&, double*, int, hipStream_t);
template hipError_t launch_real_finalize<float>(const DevPlan<float>&, double*, int, hipStream_t);
template hipError_t launch_real_finalize<double>(const DevPlan<double>&, double*, int, hipStream_t);

}  // namespace espx
