// Real-space (near) part of the PSWF kernel split (paper Sec. 3.1, eq. UN,
// eq. PinsN, eq. Fc with eq. mathFN): energy, virial and forces of the pairs
// closer than rc, after a cell sort with cells of perpendicular width >= rc
// along the cell vectors.  Every pair within rc then lies in adjacent cells
// and, with rc below half the smallest width, its separation is the minimum
// image in reduced coordinates.
//
// One workgroup of 256 threads per home cell.  The candidates (the particles
// of the distinct neighbouring cells, the home cell included) are staged
// through LDS in chunks; thread t works on home particle t % HC against every
// (256 / HC)-th candidate, HC in {16, 32, 64} chosen per cell to waste the
// fewest lanes, and the partial forces of a home particle are summed over its
// thread group in LDS.  Every ordered pair is visited once, so the forces need
// no atomics; energy and virial take the factor 1/2 at the end.  The split
// functions of x = r / rc, 1 - phi0(x) (N^c = that / r) and
// F_N(x) = 1 - phi0(x) + x psi(x) / C0 (pair force q_i q_j F_N d / r^3), are
// piecewise polynomials on nseg equal segments of [0, 1].
#include <hip/hip_runtime.h>

#include "esp_common.h"

namespace espx {

constexpr int kRealThreads = 256;
constexpr int kRealStage = 1024;     // candidate records staged per round

template <typename R, int NC>
__device__ __forceinline__ R horner(const R* __restrict__ c, R t) {
  R v = c[NC - 1];
#pragma unroll
  for (int k = NC - 2; k >= 0; --k) v = v * t + c[k];
  return v;
}

template <typename R>
__global__ void __launch_bounds__(kRealThreads) k_real_pairs(DevPlan<R> d, R* __restrict__ f, int accumulate) {
  constexpr int NC = kRealDeg<R> + 1;
  __shared__ Record<R> stage[kRealStage];
  __shared__ R fred[3 * kRealThreads];
  __shared__ double red[kNumSums * 16];
  __shared__ int nstart[27], ncum[28], nnb;
  extern __shared__ __align__(16) unsigned char smem[];
  R* tab = reinterpret_cast<R*>(smem);          // nseg x {N, F} x NC coefficients
  const int cell = blockIdx.x, tid = threadIdx.x;
  const int nseg = d.nrs;
  for (int k = tid; k < nseg * 2 * NC; k += kRealThreads) tab[k] = d.rsN[k];
  if (tid == 0) {
    // distinct neighbour cells (27, fewer along dimensions with 2 cells)
    const int n[3] = {d.cn1, d.cn2, d.cn3};
    const int c[3] = {cell % d.cn1, (cell / d.cn1) % d.cn2, cell / (d.cn1 * d.cn2)};
    int nb[3][3], cnt[3];
    for (int a = 0; a < 3; ++a) {
      cnt[a] = 0;
      for (int o = -1; o <= 1; ++o) {
        const int v = (c[a] + o + n[a]) % n[a];
        bool seen = false;
        for (int j = 0; j < cnt[a]; ++j) seen = seen || nb[a][j] == v;
        if (!seen) nb[a][cnt[a]++] = v;
      }
    }
    int m = 0, run = 0;
    for (int z = 0; z < cnt[2]; ++z)
      for (int y = 0; y < cnt[1]; ++y)
        for (int x = 0; x < cnt[0]; ++x) {
          const int nc = (nb[2][z] * d.cn2 + nb[1][y]) * d.cn1 + nb[0][x];
          const int s = d.offsets[nc], e = d.offsets[nc + 1];
          nstart[m] = s;
          ncum[m] = run;
          run += e - s;
          ++m;
        }
    ncum[m] = run;
    nnb = m;
    d.counts[cell] = 0;                         // ready for the next binning pass
  }
  __syncthreads();
  const int hs = d.offsets[cell], he = d.offsets[cell + 1], nh = he - hs;
  const int total = ncum[nnb];
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
  double part[kNumSums];
#pragma unroll
  for (int k = 0; k < kNumSums; ++k) part[k] = 0.0;
  for (int h0 = hs; h0 < he; h0 += HC) {
    const int i = h0 + hi;
    const bool own = i < he;
    const Record<R> ri = d.sorted[own ? i : hs];
    R fx = R(0), fy = R(0), fz = R(0);
    for (int c0 = 0; c0 < total; c0 += kRealStage) {
      const int nc = min(kRealStage, total - c0);
      __syncthreads();                          // previous chunk consumed
      for (int k = tid; k < nc; k += kRealThreads) {
        const int cand = c0 + k;
        int m = 0;
        while (ncum[m + 1] <= cand) ++m;
        stage[k] = d.sorted[nstart[m] + cand - ncum[m]];
      }
      __syncthreads();
      if (own) {
        for (int jj = g; jj < nc; jj += G) {
          const Record<R> rj = stage[jj];
          R ds[3];
          Coord<R>::disp(ri, rj, ds);
          const R dx = d.hmat[0] * ds[0] + d.hmat[1] * ds[1] + d.hmat[2] * ds[2];
          const R dy = d.hmat[3] * ds[0] + d.hmat[4] * ds[1] + d.hmat[5] * ds[2];
          const R dz = d.hmat[6] * ds[0] + d.hmat[7] * ds[1] + d.hmat[8] * ds[2];
          const R r2 = dx * dx + dy * dy + dz * dz;
          if (r2 < d.rc2 && r2 > R(0)) {
            const R r = sqrt(r2);
            const R ir = R(1) / r;
            const R xs = r * d.inv_rc * nsegr;
            const int sg = min(nseg - 1, static_cast<int>(xs));
            const R t = xs - static_cast<R>(sg) - R(0.5);
            const R* cf = tab + sg * 2 * NC;
            const R qq = ri.q * rj.q;
            const R gn = horner<R, NC>(cf, t), gf = horner<R, NC>(cf + NC, t);
            const R fw = qq * gf * ir * ir * ir;
            const R wx = fw * dx, wy = fw * dy, wz = fw * dz;
            fx += wx;
            fy += wy;
            fz += wz;
            part[0] += static_cast<double>(qq * gn * ir);
            part[1] += static_cast<double>(wx * dx);
            part[2] += static_cast<double>(wy * dy);
            part[3] += static_cast<double>(wz * dz);
            part[4] += static_cast<double>(wx * dy);
            part[5] += static_cast<double>(wx * dz);
            part[6] += static_cast<double>(wy * dz);
          }
        }
      }
    }
    // sum each home particle's forces over its thread group
    fred[3 * tid + 0] = fx;
    fred[3 * tid + 1] = fy;
    fred[3 * tid + 2] = fz;
    __syncthreads();
    if (tid < HC && h0 + tid < he) {
      R s0 = R(0), s1 = R(0), s2 = R(0);
      for (int k = 0; k < G; ++k) {
        const int t = k * HC + tid;
        s0 += fred[3 * t + 0];
        s1 += fred[3 * t + 1];
        s2 += fred[3 * t + 2];
      }
      const int64_t j = d.perm[h0 + tid];
      const R kc = d.coulomb_k;
      if (accumulate) {
        f[3 * j + 0] += kc * s0;
        f[3 * j + 1] += kc * s1;
        f[3 * j + 2] += kc * s2;
      } else {
        f[3 * j + 0] = kc * s0;
        f[3 * j + 1] = kc * s1;
        f[3 * j + 2] = kc * s2;
      }
    }
  }
  block_sum<kNumSums>(part, red);
  if (tid == 0)
#pragma unroll
    for (int k = 0; k < kNumSums; ++k) d.rpart[static_cast<size_t>(cell) * kNumSums + k] = part[k];
}

template <typename R>
__global__ void __launch_bounds__(256) k_real_finalize(DevPlan<R> d, double* __restrict__ out7) {
  __shared__ double red[kNumSums * 16];
  const int ncell = d.cn1 * d.cn2 * d.cn3;
  double v[kNumSums];
#pragma unroll
  for (int k = 0; k < kNumSums; ++k) v[k] = 0.0;
  for (int c = threadIdx.x; c < ncell; c += blockDim.x)
#pragma unroll
    for (int k = 0; k < kNumSums; ++k) v[k] += d.rpart[static_cast<size_t>(c) * kNumSums + k];
  block_sum<kNumSums>(v, red);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < kNumSums; ++k) out7[k] = 0.5 * d.fin.coulomb_k * v[k];
}

template <typename R>
size_t lds_real(const DevPlan<R>& d) {
  return static_cast<size_t>(d.nrs) * 2 * (kRealDeg<R> + 1) * sizeof(R);
}

template <typename R>
hipError_t launch_real_pairs(const DevPlan<R>& d, R* f, int accumulate, hipStream_t s) {
  const size_t lds = lds_real(d);     // at most 40 KiB (segment count capped on the host)
  hipLaunchKernelGGL(k_real_pairs<R>, dim3(d.cn1 * d.cn2 * d.cn3), dim3(kRealThreads), lds, s, d, f, accumulate);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_real_finalize(const DevPlan<R>& d, double* out7, hipStream_t s) {
  hipLaunchKernelGGL(k_real_finalize<R>, dim3(1), dim3(256), 0, s, d, out7);
  return hipGetLastError();
}

template size_t lds_real<float>(const DevPlan<float>&);
template size_t lds_real<double>(const DevPlan<double>&);
template hipError_t launch_real_pairs<float>(const DevPlan<float>&, float*, int, hipStream_t);
template hipError_t launch_real_pairs<double>(const DevPlan<double>&, double*, int, hipStream_t);
template hipError_t launch_real_finalize<float>(const DevPlan<float>&, double*, hipStream_t);
template hipError_t launch_real_finalize<double>(const DevPlan<double>&, double*, hipStream_t);

}  // namespace espx
