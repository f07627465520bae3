// Device-side data layout shared by the kernels and the host plan.
//
// Precision policy: R = float is the production path (spreading, FFT and
// gather in FP32, FP32 Kahan-compensated per-thread mode sums, FP64 block
// partials and final sums); R = double is the plain FP64 path built from the
// same kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace espx {

constexpr int kMaxP = 12;          // largest window support per dimension
constexpr double kFp32TolFloor = 1e-6;  // FP32 plans with a smaller tol get ESP_WARN_PRECISION
constexpr int kMaxWinDeg = 16;     // largest degree of the window polynomials (classes 8, 12, 16)
constexpr int kMaxKerDeg = 48;     // largest Chebyshev degree of the kernel fits
constexpr int kMaxRadix = 8;
constexpr int kMaxStages = 16;
constexpr int kNumSums = 7;        // energy + 6 virial components
constexpr int kNumXcd = 8;        // XCDs of the MI355X, each with its own L2
constexpr int kXcdRun = 16;       // consecutive block numbers one XCD takes (see xcd_block)
constexpr int kSpreadWaves = 4;   // waves of a spreading workgroup (256 threads)
constexpr int kWaveChunk = 21;    // particles a spreading wave stages at a time (3 weight tasks each)
constexpr int kSpreadFixedMin = 128;  // automatic fixed-point spreading of FP64 plans: mean particles
constexpr int kSpreadFixedMinTiles = 512;  // per tile, and tiles (two per CU), at least
constexpr size_t kCompLaneOneLaunch = 48 * 1024;  // virial gather: six boxes in one launch up to this LDS
constexpr int kCompLaneMin = 8;      // mean particles per tile from which the ik / virial gathers stage boxes
constexpr int kTiledGatherMin = 96;  // mean particles per tile above which the gather is tile-staged
constexpr int kBinContention = 64;   // target same-address atomics per tile counter in binning
constexpr int kMaxCounterCopies = 16;
constexpr int kBinThreads = 256;     // threads of a binning workgroup
constexpr int kBinMaxPpt = 4;        // particles per binning thread, at most
constexpr int kGridExp = 56;        // FP32 fixed-point grid scale 2^gexp, gexp = kGridExp - ilogb(wmax^3 sum |q|)
constexpr int kScanTpt = 4;          // rounds of tiles the counter-copy scan loads at once

template <typename R>
struct Cplx {
  R x, y;
};

// Sorted particle record.  FP32: reduced coordinates as 32-bit fixed point
// (s = S / 2^32), so binning and stencil placement are exact integer
// operations; FP64: reduced coordinates in [0, 1).
template <typename R>
struct Record;
template <>
struct alignas(16) Record<float> {
  uint32_t S[3];
  float q;
};
template <>
struct alignas(32) Record<double> {
  double s[3];
  double q;
};

struct FftLen {
  int n;                 // transform length
  int nstage;
  int rad[kMaxStages];   // radices, applied in order
  int tw;                // offset of exp(-2 pi i k / n), k < n, in the twiddle table
};

// Constants of the final sums (self energy, background, units).
struct FinalConsts {
  double inv2V;        // 1 / (2 V)
  double self_coef;    // psi(0) / (2 C0 rc)
  double bg_coef;      // 2 pi Ic / V  (U_corr = -bg_coef Q^2)
  double coulomb_k;
};

template <typename R>
struct DevPlan {
  // sizes
  int64_t n;
  int M1, M2, M3, H;               // grid; H = M1 / 2 + 1 half-spectrum columns
  int P, nw, nker;                 // window support, padded window degree (8/12/16), kernel degree
                                   // padded to a multiple of 4
  int T1, T2, T3, nt1, nt2, nt3, ntiles;
  int cz;                          // columns per block in the z-pass
  int nbin;                        // blocks of the binning kernel
  int binppt;                      // particles per binning thread: block b takes particles
                                   // [b, b + 1) x kBinThreads x binppt
  int nzblk;                       // blocks of the z-pass
  // cell (updated by esp_set_box)
  float hinv_hi[9], hinv_lo[9];    // h^-1 as float-float (FP32 path), row major
  double hinv[9];                  // h^-1 (FP64 path), row major
  R B[9];                          // 2 pi h^-T, row major: k = B m
  R G[9];                          // -h^-T diag(M): force = q G grad_u
  R kcut2;                         // (c_split / rc)^2
  R ysc;                           // (rc / c_split)^2: y = |k|^2 ysc = x^2
  R A;                             // 2 pi lam0 / C0 of the splitting PSWF
  R inv_vol;                       // 1 / V
  R coulomb_k;
  float wmax, wmax3;               // bound of |window value| and its cube (fixed-point spreading scales)
  int spread_fixed;                // spreading tile in 64-bit fixed point (else FP64)
  // tables (device)
  const R* win;                    // (nw + 1) x P monomial coefficients in tau, coefficient-major
  const Cplx<R>* kerfg;            // (nker + 1) pairs of Chebyshev coefficients in z = 2y - 1:
                                   // (psi(sqrt y), x psi'(x) at x = sqrt y), zero past the fit
  const R* iw1;                    // 1 / w_hat(2 pi m / M1)^2, DFT index order
  const R* iw2;
  const R* iw3;
  const Cplx<R>* tw;               // twiddles for the three lengths
  FftLen f1, f2, f3;
  // buffers
  int* counts;                     // nsub x ntiles
  int* offsets;                    // ntiles + 1
  int* keys;                       // n
  int* ranks;                      // n
  int* perm;                       // n: sorted position -> particle
  Record<R>* tmp;                  // n: records in input order
  Record<R>* sorted;               // n
  R* rho;                          // M1 M2 M3 real grid (kept zero between calls), unless grid_fixed
  long long* rhofix;               // grid_fixed: the grid as int64 at scale 2^gexp (kept zero)
  int* gexp;                       // grid_fixed: that exponent for the current call (set by the sort)
  int grid_fixed;                  // FP32 with fixed-point spreading: tiles add integers into rhofix
  Cplx<R>* spec;                   // ncomp x H M2 M3 half spectra
  R* phi;                          // ncomp x M1 M2 M3 real grids (potential, ik field or Pi)
  double* zpart;                   // nzblk x 7 partial mode sums of the z-pass
  double* qpart;                   // nbin x 3 partial sums (sum q, sum q^2, sum |q|)
  int* flags;                      // bit 0: non-finite input; bit 1: inconsistent tile counts
  int bin_lds;                     // tile histogram of the binning pass fits in LDS
  int gather_tiled;                // gather stages each tile's potential box in LDS
  int gather_lane;                 // tile-staged gather with one particle per lane
  int comp_lane;                   // bit 0 / 1: the ik / virial gathers stage three component
                                   // boxes per tile (one particle per lane)
  int ik;                          // forces by ik-differentiation (3 field components)
  int local;                       // per-particle virial enabled (6 field components)
  int ncomp;                       // spectra / real grids allocated (1, 3 or 6)
  int nsub;                        // tile counters per tile: binning block b uses copy b % nsub
  int cellsort;                    // binning keys are real-space cells (cn1 x cn2 x cn3), not tiles
  int xy_split;                    // xy transforms as separate x and y passes (plane beyond LDS)
  int xpairs, ycols;               // split passes: row pairs / half-spectrum columns per workgroup
  int* sbase;                      // nsub > 1: nsub x ntiles first rank of each copy in its tile
  FinalConsts fin;                 // final-sum constants (updated by esp_set_box)
  // real-space (near) part: cells of perpendicular width >= rc along the cell vectors
  int cn1, cn2, cn3;               // cells per dimension (current box)
  int nrs;                         // segments of the near-kernel polynomials on x = r / rc in [0, 1]
  const R* rsN;                    // nrs x 2 x (kRealDeg + 1) monomial coefficients in the segment's
                                   // local t = nrs x - s - 1/2: first 1 - phi0(x), then
                                   // F_N(x) = 1 - phi0(x) + x psi(x) / C0 (eq. mathFN)
  R hmat[9];                       // h, row major: d = h ds
  R gmet[6];                       // metric h^T h as (g00, g11, g22, 2 g01, 2 g02, 2 g12), scaled
                                   // by 2^-64 for the FP32 path (raw fixed-point displacements)
  R rc2, inv_rc;
  int rsplit;                      // workgroups per cell, each with a share of the candidates
  R* fpart;                        // rsplit x n x 3 near-force shares (sorted order)
  double* facc;                    // n x 3 reaction forces (sorted order; kept zero between calls)
  double* rpart;                   // cells x rsplit x 7 partial sums of the near energy and virial
  // cell-sort buffers of the real-space part, apart from the Fourier part's
  // so that the two can run at once on two streams
  int* nr_counts;                  // kMaxCells
  int* nr_offsets;                 // kMaxCells + 1
  int* nr_keys;                    // n
  int* nr_ranks;                   // n
  int* nr_perm;                    // n
  Record<R>* nr_tmp;               // n
  Record<R>* nr_sorted;            // n
  double* nr_qpart;                // nbin x 3
  int64_t pofs;                    // batched launches: first particle of this plan in the
  int rep;                         // concatenated inputs, and its index (0 for single plans)
};

// Degree of the near-kernel segment polynomials (FP32 / FP64 path).
template <typename R>
inline constexpr int kRealDeg = sizeof(R) == 8 ? 9 : 5;
constexpr int kMaxCells = 32768;   // real-space cells (the scatter pass keeps their offsets in LDS)
constexpr int kMaxRealSplit = 8;   // workgroups per real-space cell
constexpr int kRealBlocks = 3072;  // target workgroups of the pair kernel (rsplit up to kMaxRealSplit)

// Lanes per particle of the gather kernel (a power of two >= P).
constexpr int gather_lanes(int P) { return P <= 4 ? 4 : (P <= 8 ? 8 : 16); }

// Kernel argument: one plan by value, or, for a batched launch, a device array
// of plans and the first block of each plan's block range (nrep + 1 entries).
template <typename R, bool BATCH>
struct KArg;
template <typename R>
struct KArg<R, false> {
  DevPlan<R> d;
};
template <typename R>
struct KArg<R, true> {
  const DevPlan<R>* plans;
  const int* boff;
  int nrep;
};

// Geometry of one batched launch (blocks, threads, dynamic LDS) over a range
// of plans; P and nw select the spreading / gather instantiation.
template <typename R>
struct BatchLaunch {
  const DevPlan<R>* plans;
  const int* boff;
  int nrep, nblk, nth;
  size_t lds;
  int P, nw;
  int ppt;                         // binning stage: largest particles per thread of its plans
  int grid_fixed;                  // xy stage: the plans keep int64 grids (deterministic FP32)
  int lane;                        // gather stage: tile-staged, one particle per lane
};

// Per-stage kernel timing.  While the host plan times a stage it sets the two
// events here; every kernel of that stage is then launched with
// hipExtLaunchKernelGGL, the first recording `start` at its own start and
// each recording `stop` at its end (the last one counts), so the timed span
// is the stage's kernels alone, without the dispatch latency before them.
// One per host thread (defined in esp_plan.cpp).
struct LaunchTiming {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};
LaunchTiming& launch_timing();

// Launchers (defined in esp_kernels.hip, instantiated for float and double).
template <typename R>
hipError_t launch_bin(const DevPlan<R>& d, const R* xyz, const R* q, hipStream_t s);
template <typename R>
hipError_t launch_scatter(const DevPlan<R>& d, hipStream_t s);
// nsub > 1 only: tile offsets and per-copy bases from the counter copies
// (one workgroup), which also clears the counters.
template <typename R>
hipError_t launch_scan_sub(const DevPlan<R>& d, hipStream_t s);
// Final sums into out7 (one workgroup) after a z-pass in energy mode.
template <typename R>
hipError_t launch_finalize(const DevPlan<R>& d, double* out7, hipStream_t s);
template <typename R>
hipError_t launch_spread(const DevPlan<R>& d, hipStream_t s);
// grid: an R grid, or null for the plan's own grid (rhofix when grid_fixed).
template <typename R>
hipError_t launch_fft_xy(const DevPlan<R>& d, const R* grid, Cplx<R>* spec, bool clear_input,
                         hipStream_t s);
// grid_fixed plans: the int64 grid as R values into out, and cleared.
template <typename R>
hipError_t launch_grid_out(const DevPlan<R>& d, R* out, hipStream_t s);
// Z_POTENTIAL: G rho_hat, inverse z; Z_IK: the three components i k_a G rho_hat,
// each inverse z into its own half spectrum (spec + a * H M2 M3); Z_LOCAL: the
// six components of P_hat rho_hat / (2 V W_hat^2) (xx, yy, zz, xy, xz, yz).
enum ZMode { Z_FFT_ONLY = 0, Z_ENERGY = 1, Z_POTENTIAL = 2, Z_IK = 3, Z_LOCAL = 4 };
// z-pass; unless mode is Z_FFT_ONLY it writes nzblk x 7 partial mode sums.
template <typename R>
hipError_t launch_fft_z(const DevPlan<R>& d, ZMode mode, hipStream_t s);
// Inverse xy pass of the first ncomp half spectra into the real grids.
template <typename R>
hipError_t launch_fft_xy_inv(const DevPlan<R>& d, int ncomp, hipStream_t s);
// Per-particle virial from the six Pi grids: w6[6 j + c], input order.
template <typename R>
hipError_t launch_gather_local(const DevPlan<R>& d, R* w6, double* out7, hipStream_t s);
// Gather; when out7 is non-null its block 0 also writes the final sums.
template <typename R>
hipError_t launch_gather(const DevPlan<R>& d, R* f, double* out7, hipStream_t s);

// Batched launches: one launch per stage covers every plan of the range
// (xyz, q, f are the concatenated arrays, out7 holds 7 values per plan;
// fft_xy works on each plan's own rho / spec).
template <typename R>
hipError_t launch_bin_batch(const BatchLaunch<R>& b, const R* xyz, const R* q, hipStream_t s);
template <typename R>
hipError_t launch_scatter_batch(const BatchLaunch<R>& b, hipStream_t s);
template <typename R>
hipError_t launch_scan_sub_batch(const BatchLaunch<R>& b, hipStream_t s);
template <typename R>
hipError_t launch_spread_batch(const BatchLaunch<R>& b, hipStream_t s);
template <typename R>
hipError_t launch_fft_xy_batch(const BatchLaunch<R>& b, hipStream_t s);
template <typename R>
hipError_t launch_fft_z_batch(const BatchLaunch<R>& b, ZMode mode, hipStream_t s);
template <typename R>
hipError_t launch_fft_xy_inv_batch(const BatchLaunch<R>& b, hipStream_t s);
template <typename R>
hipError_t launch_gather_batch(const BatchLaunch<R>& b, R* f, double* out7, hipStream_t s);
template <typename R>
hipError_t launch_finalize_batch(const BatchLaunch<R>& b, double* out7, hipStream_t s);
template <typename T>
hipError_t launch_fill(T* p, size_t count, hipStream_t s);

// Real-space part (one workgroup share per cell, after a cell sort with
// cellsort set): launch_real_pairs leaves the force shares in fpart / facc and
// the partial sums in rpart; launch_real_forces writes (accumulate: adds) the
// near forces to f in input order; launch_real_finalize writes (add: adds)
// out7 = {U_N, W_N}.
template <typename R>
hipError_t launch_real_pairs(const DevPlan<R>& d, hipStream_t s);
template <typename R>
hipError_t launch_real_forces(const DevPlan<R>& d, R* f, int accumulate, hipStream_t s);
template <typename R>
hipError_t launch_real_finalize(const DevPlan<R>& d, double* out7, int add, hipStream_t s);
template <typename R>
size_t lds_real(const DevPlan<R>& d);

// LDS bytes the kernels need for a plan (the host checks them against the
// device limit before any launch).
template <typename R>
size_t lds_fft_xy(const DevPlan<R>& d);
template <typename R>
size_t lds_fft_z(const DevPlan<R>& d);
// Split xy passes: x pass with npb row pairs, y pass with ncol columns per workgroup.
template <typename R>
size_t lds_fft_x(const DevPlan<R>& d, int npb);
template <typename R>
size_t lds_fft_y(const DevPlan<R>& d, int ncol);
template <typename R>
size_t lds_spread(const DevPlan<R>& d);
// Potential box of the tile-staged gather: (T_d + P - 1) cells per dimension.
template <typename R>
size_t lds_gather_box(const DevPlan<R>& d);
int fft_threads(int lines_x_len);

}  // namespace espx
