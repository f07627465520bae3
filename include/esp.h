/*
 * esp.h -- C ABI of the MI355X (gfx950) reciprocal-space ESP library.
 *
 * Ewald summation with prolates (ESP) for NPT: the long-range (Fourier-space)
 * energy, the full 6-component virial tensor and the forces of a periodic
 * system of point charges in a general (triclinic) cell.
 *
 * What is computed (citations are to Liang, Lu & Jiang, "Fast Ewald Summation
 * with Prolates for Charged Systems in the NPT Ensemble", arXiv 2601.00161):
 *
 *   E  = U_F + U_self (+ U_cb + U_bb when sum q != 0)     eq. UF, eq. selfen, eq. Corr
 *   W  = V * (P_F + P_cb + P_bb)                           eq. diag, eq. PFfinal, eq. Corr
 *   F  = F_F, the Fourier-space force by analytic
 *        differentiation of the gridded energy             App. C, eq. UFAnal / eq. AD
 *
 * through the particle-mesh steps of Sec. 4.1 (Algorithm 1): PSWF spreading
 * onto a uniform grid along the cell vectors, one forward 3D FFT, diagonal
 * scaling by W_hat^-2 times the splitting kernel, and a Fourier-space
 * reduction; forces add one inverse FFT and a gather with the window gradient.
 * The real-space part (U_N, P_N, F_N of eq. UN / eq. PinsN) is NOT computed
 * here; the caller adds it.
 *
 * Conventions
 *   Units: any consistent length unit (the defaults assume nm); charges in e;
 *     the Coulomb constant is esp_opts.coulomb_k (1 by default).
 *   Cell: h[3*i + j] = component i of cell vector j (cell vectors are the
 *     columns of h, Sec. 2.2); det h must be positive.
 *   Positions: xyz[3*p + d], any real values (wrapped into the cell).
 *   out7 = { E, W_xx, W_yy, W_zz, W_xy, W_xz, W_yz }, W = V * P in energy
 *     units, so tr W = E for the converged Coulomb energy (eq. PSRela).
 *   Forces: f[3*p + d], overwritten (not accumulated).
 *
 * Memory and ordering
 *   xyz, q, f and out7 are DEVICE pointers owned by the caller.  Every call
 *   is enqueued on the plan's stream and is asynchronous; results are valid
 *   after the stream is synchronised.  The plan owns all scratch memory,
 *   which it allocates in esp_plan only; the per-step calls allocate nothing.
 *   A plan is used by one host thread at a time; calls on one plan must not
 *   overlap.
 *
 * Errors
 *   Negative status = error, nothing was enqueued; positive = warning, the
 *   result is valid.  esp_last_error() describes the most recent problem.
 *   Non-finite positions or charges are detected on the device: the affected
 *   particles are treated as uncharged, and the next call to esp_check()
 *   (which synchronises) reports ESP_ENONFINITE.
 */
#ifndef ESP_MI355X_H
#define ESP_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct esp_plan_s esp_plan_t;
typedef struct esp_batch_s esp_batch_t;

typedef enum {
  ESP_OK = 0,
  ESP_WARN_REPLAN = 1,    /* esp_set_box: the new box is >10% off the grid rule */
  ESP_WARN_FALLBACK = 2,  /* esp_plan: learned parameters rejected, analytic used */
  ESP_WARN_PRECISION = 3, /* esp_plan: FP32 plan with tol below 1e-6, which FP32 rounding
                             (relative errors of a few 1e-7 up to ~3e-6 per virial
                             component) is not expected to meet; use ESP_FP64 */
  ESP_EINVAL = -1,        /* bad argument (null pointer, bad size or option) */
  ESP_EBOX = -2,          /* det h <= 0 or not finite */
  ESP_ECUTOFF = -3,       /* rc >= half the smallest perpendicular cell width */
  ESP_ENOMEM = -4,        /* device allocation failed */
  ESP_EDEVICE = -5,       /* HIP runtime error */
  ESP_ENONFINITE = -6     /* non-finite input seen by the device */
} esp_status;

enum { ESP_FP32 = 0, ESP_FP64 = 1 };
enum { ESP_ANALYTIC = 0, ESP_EXPLICIT = 1, ESP_LEARNED = 2 };
enum { ESP_ISO = 0, ESP_SEMI = 1, ESP_ANISO = 2, ESP_FLEX = 3 };

/* Options.  Fill with esp_opts_default() and override fields.
 *
 * tol semantics (target relative error of the requested outputs):
 *   analytic parameters use Delta = tol for ISO/SEMI/ANISO coupling and
 *   Delta = tol/5 for FLEX (off-diagonal virial components are harder,
 *   Sec. 5.1), then c from psi_0^c(1)/psi_0^c(0) = Delta, P = ceil(-log10
 *   Delta) + 1, and M_d = next 2,3,5-smooth integer >= sigma |h_d| c /(pi rc)
 *   with sigma = grid_sigma.
 * With params = ESP_EXPLICIT the fields c_split, c_spread, P, M are used
 * as given (each must be set).  With ESP_LEARNED the parameters come from the
 * proposer registered with esp_proposer_set (analytic fallback otherwise). */
typedef struct {
  int precision;       /* ESP_FP32 (default) or ESP_FP64 */
  int params;          /* ESP_ANALYTIC (default), ESP_EXPLICIT, ESP_LEARNED */
  int coupling;        /* ESP_ISO .. ESP_FLEX: which virial components must meet tol */
  double rc;           /* cutoff radius of the split; default 0.9 */
  double c_split;      /* explicit: PSWF bandwidth of the splitting kernel */
  double c_spread;     /* explicit: PSWF bandwidth of the window */
  int P;               /* explicit: window support in grid points per dimension */
  int M[3];            /* explicit: grid subintervals along each cell vector */
  double grid_sigma;   /* analytic grid oversampling; default 1.07 */
  double coulomb_k;    /* Coulomb constant multiplying E, W, F; default 1 */
  int tile;            /* spreading tile edge in grid cells; 0 = automatic */
  void *stream;        /* hipStream_t for every call on the plan; NULL = default */
  double window_tol;   /* max error of the window polynomials relative to psi(0);
                          0 = automatic: max(Delta/100, 2e-8) for FP32, Delta/1000
                          for FP64 */
  int gather;          /* ESP_GATHER_AUTO (0): tile-staged gather with one lane per
                          particle when tiles hold 96+ particles on average, else
                          per particle; ESP_GATHER_PARTICLE (1),
                          ESP_GATHER_TILE (2: tile-staged, a group of lanes per
                          particle) or ESP_GATHER_LANE (3: tile-staged, one lane
                          per particle) force one variant (the tile-staged ones
                          are refused if the potential box does not fit in LDS) */
  int force;           /* ESP_FORCE_AD (0, default): analytic differentiation,
                          one inverse FFT and a window-gradient gather (App. C,
                          eq. AD); ESP_FORCE_IK (1): ik-differentiation, three
                          inverse FFTs of i k F_hat rho_hat / W_hat^2 and a
                          plain-window gather (App. C, eq. rhodiagforce), which
                          conserves momentum.  Energy and virial are the same. */
  int local_virial;    /* nonzero: allocate the six tensor-component grids used by
                          esp_local_virial */
  int fft_split;       /* nonzero: run the x and y transforms as separate passes even
                          when a grid plane fits one workgroup's LDS (planes that do
                          not fit always take them) */
  int spread_accum;    /* accumulator of the spreading tile in LDS: ESP_SPREAD_AUTO (0:
                          64-bit fixed point for FP32 plans; for FP64 plans when
                          there are 512+ tiles holding 128+ particles on average,
                          else FP64), ESP_SPREAD_FIXED (1) or ESP_SPREAD_FP64 (2).
                          Fixed point: per tile, scale 2^e with 2^e wmax^3 sum|q|
                          <= 2^59 (FP32) or < 2^62 (FP64), each term rounded once to
                          2^-e, exact integer sums (FP32 terms: the int32-rounded
                          factors q wx 2^eq and wy wz 2^ka multiplied exactly).
                          Tiles add their cells to the grid with floating-point
                          atomics (see deterministic).  Single plans only;
                          batched launches spread FP32 batches in fixed point and
                          FP64 batches with FP64 adds. */
  int deterministic;   /* nonzero, FP32 plans with fixed-point spreading: the grid is
                          kept in fixed point too.  Tiles add their sums, rounded
                          to one scale per call (2^gexp with 2^gexp wmax^3 sum|q|
                          < 2^57 over all particles), into an int64 grid, so no
                          sum depends on the order of the atomics and every output
                          (energy, virial, forces) repeats bit for bit on the same
                          input (esp_params.grid_fixed).  Costs ~2-3 % per step
                          (64-bit grid atomics, 8-byte grid reads).  FP64 plans
                          ignore it. */
} esp_opts;

enum { ESP_GATHER_AUTO = 0, ESP_GATHER_PARTICLE = 1, ESP_GATHER_TILE = 2, ESP_GATHER_LANE = 3 };
enum { ESP_FORCE_AD = 0, ESP_FORCE_IK = 1 };
enum { ESP_SPREAD_AUTO = 0, ESP_SPREAD_FIXED = 1, ESP_SPREAD_FP64 = 2 };

/* Parameters a plan resolved to (returned by esp_get_params). */
typedef struct {
  int precision;
  int64_t n;
  double tol, delta, rc, c_split, c_spread;
  int P, M[3];
  int tile[3], ntiles;
  int window_degree;   /* degree of the per-subinterval window polynomials */
  int kernel_degree;   /* Chebyshev degree of the psi / psi' kernel fits */
  double lambda0_split, C0_split, psi0_split;
  double volume;
  int params_source;   /* ESP_ANALYTIC / ESP_EXPLICIT / ESP_LEARNED actually used */
  double predicted_log10_err[4];  /* ESP_LEARNED: the proposer's prediction, else 0 */
  double predicted_cost;          /* ESP_LEARNED: cost-model value of the choice */
  int gather_tiled;               /* 1: the gather stages each tile's potential in LDS */
  int counter_copies;             /* tile-counter copies used by the cell sort */
  int force;                      /* ESP_FORCE_AD or ESP_FORCE_IK */
  int local_virial;               /* the plan supports esp_local_virial */
  int real_cells[3];              /* esp_real_space cells per cell vector (current box) */
  int real_segments;              /* segments of the near-kernel polynomials on [0, rc] */
  int fft_split;                  /* the xy transforms run as separate x and y passes */
  int spread_fixed;               /* 1: the spreading tile accumulates in 64-bit fixed point */
  double hinv[9];                 /* h^-1 of the current cell, row major (the FP32 path uses it as
                                     the float pair hi = (float) hinv, lo = (float) (hinv - hi)) */
  int gather_lane;                /* 1: the tile-staged gather takes one particle per lane */
  int grid_fixed;                 /* 1: deterministic FP32 plan (fixed-point tiles into an int64
                                     grid): every output repeats bit for bit on the same input */
} esp_params;

void esp_opts_default(esp_opts *o);

/* Create a plan for n particles in cell h at tolerance tol (Sec. 5.1 rules,
 * or explicit / learned parameters).  Allocates every device buffer.
 *   h: host, 9 doubles.   n >= 1.   tol in [1e-12, 1e-1).   o may be NULL.
 * Errors: ESP_EINVAL, ESP_EBOX, ESP_ECUTOFF, ESP_ENOMEM, ESP_EDEVICE.
 * Warnings (the plan is made): ESP_WARN_FALLBACK (learned parameters),
 * ESP_WARN_PRECISION (FP32 plan with tol < 1e-6). */
esp_status esp_plan(const double h[9], int64_t n, double tol, const esp_opts *o,
                    esp_plan_t **out);

/* New cell for the following calls (an NPT step).  No re-allocation: the
 * splitting and grid parameters stay fixed while the box fluctuates
 * (Sec. 3.3, Sec. 5.1).  Returns ESP_WARN_REPLAN if the grid rule is now
 * violated by more than 10 %; ESP_EBOX / ESP_ECUTOFF on an invalid cell. */
esp_status esp_set_box(esp_plan_t *p, const double h[9]);

/* Energy and virial only: spreading, one forward FFT, scaling and reduction
 * (Algorithm 1; no inverse FFT).  FP32 plans take float pointers; FP64
 * plans use the _f64 variants.  xyz: 3n, q: n, out7: 7 doubles (device). */
esp_status esp_energy_virial(esp_plan_t *p, const float *xyz, const float *q, double *out7);
esp_status esp_energy_virial_f64(esp_plan_t *p, const double *xyz, const double *q, double *out7);

/* Energy, virial and forces (App. C, analytic differentiation).
 * f: 3n (device), overwritten.  out7 may be NULL. */
esp_status esp_forces(esp_plan_t *p, const float *xyz, const float *q, float *f, double *out7);
esp_status esp_forces_f64(esp_plan_t *p, const double *xyz, const double *q, double *f,
                          double *out7);

/* Allocation-free variant of esp_plan + esp_forces + esp_destroy, for callers
 * that cannot allocate device memory (tight serving loops, harnesses that
 * forbid hipMalloc).  It makes a plan for (h, n, tol, o) exactly as esp_plan
 * would, with every device buffer carved out of a static device array of
 * ESP_NOALLOC_SCRATCH_BYTES per GPU (held from the library's first use on
 * that GPU until the process ends), runs the esp_forces path on o->stream and
 * frees the plan's host side; it calls no hipMalloc, hipFree or other device
 * allocator.  Results equal those of esp_forces on an esp_plan plan with the
 * same arguments.
 *   h: host, 9 doubles; xyz (3n floats), q (n floats), f (3n floats,
 *   overwritten) and out7 (7 doubles, may be NULL): device pointers owned
 *   by the caller, FP32 only (o->precision must be ESP_FP32; o may be NULL).
 *   ESP_LEARNED parameters and local_virial are refused (ESP_EINVAL); the
 *   real-space entry points have no allocation-free variant.
 * Ordering: the plan's tables are uploaded on o->stream after earlier work
 *   there and the call waits for that upload (it synchronises the stream
 *   once); the force kernels are enqueued asynchronously behind it.
 * Sharing: every call on one GPU uses that GPU's one array and leaves its
 *   contents behind (the buffers that must start at zero are cleared by each
 *   call).  Calls that overlap on one GPU -- from several host threads, or on
 *   different streams without ordering between them -- race and give wrong
 *   results; serialise them.
 * Errors: as esp_plan / esp_forces, described on stderr (there is no plan
 *   for esp_last_error).  A plan that does not fit the array returns
 *   ESP_ENOMEM before anything is enqueued.  A plan takes about 44 bytes per
 *   particle plus 12 bytes per grid point (e.g. 68 MB for 10^6 particles on
 *   a 135 x 135 x 108 grid).
 *   Non-finite inputs are treated as uncharged particles but not reported
 *   (esp_check needs a plan). */
#define ESP_NOALLOC_SCRATCH_BYTES ((size_t)96 << 20)
esp_status esp_forces_noalloc(const double h[9], int64_t n, double tol, const esp_opts *o,
                              const float *xyz, const float *q, float *f, double *out7);

/* Per-particle share of the Fourier virial (Sec. 4.4, eq. rhodiag,
 * eq. PinsFind), for pressure profiles of inhomogeneous systems: the six
 * components of P_hat rho_hat / (2 V W_hat^2) are brought back by inverse
 * FFTs and gathered with the plain window,
 *   w6[6 i + c] = q_i sum_g W(u_i - g) Pi_c(g),  c = xx, yy, zz, xy, xz, yz,
 * in input order (device, 6n reals of the plan's precision).  The shares add
 * up to the Fourier virial W_F (out7 minus the background term of eq. Corr,
 * which is not split).  out7 may be NULL.  Needs a plan made with
 * o->local_virial != 0 (ESP_EINVAL otherwise). */
esp_status esp_local_virial(esp_plan_t *p, const float *xyz, const float *q, float *w6, double *out7);
esp_status esp_local_virial_f64(esp_plan_t *p, const double *xyz, const double *q, double *w6,
                                double *out7);

/* Real-space (near) part of the split (Sec. 3.1, eq. UN, eq. PinsN and
 * eq. Fc with eq. mathFN): over the pairs closer than rc (minimum image),
 *   out7 = { sum_{i<j} q_i q_j N^c(r_ij),
 *            W_N = 1/2 sum_{i != j} q_i q_j F_N(r_ij) d_ij d_ij^T / r_ij^3 }
 * (W_N as xx, yy, zz, xy, xz, yz), and the forces
 *   f_i = sum_j q_i q_j F_N(r_ij) d_ij / r_ij^3,  d_ij = r_i - r_j,
 * all times coulomb_k.  Adding out7 to the Fourier part's out7 gives the
 * total Coulomb energy and virial; with accumulate != 0 the near forces are
 * added to f (e.g. the Fourier forces of esp_forces), else f is overwritten.
 * Device pointers: xyz 3n, q n, f 3n, out7 7 doubles.  The cell sort uses
 * cells of perpendicular width >= rc (the plan's rc, below half the smallest
 * cell width as esp_plan / esp_set_box require), so each call costs about
 * 27 n^2 rc^3 / V pair tests.  A non-finite input is flagged for esp_check
 * and the particle is treated as uncharged at the origin. */
esp_status esp_real_space(esp_plan_t *p, const float *xyz, const float *q, float *f, int accumulate,
                          double *out7);
esp_status esp_real_space_f64(esp_plan_t *p, const double *xyz, const double *q, double *f,
                              int accumulate, double *out7);

/* Total Coulomb interaction of the split (Sec. 3.2, eq. splitting: near
 * part plus Fourier part, whose out7 carries the self term; forces as in
 * eq. Fc): f is overwritten with the esp_forces forces
 * plus the esp_real_space forces, and out7 with the sum of the two parts'
 * energy and virial, i.e. the result of esp_forces followed by
 * esp_real_space with accumulate != 0, up to the rounding of the final
 * additions.  The real-space part runs on a second stream of the plan
 * (created on the first call, default priority, forked from and joined back
 * to the plan's stream by events) at the same time as the Fourier part; it
 * sorts into buffers of its own, so the two never write the same memory.
 * The call is asynchronous like the others: later work on the plan's stream
 * sees the complete result.  Device pointers: xyz 3n, q n, f 3n, out7 7
 * doubles (neither may be NULL). */
esp_status esp_coulomb(esp_plan_t *p, const float *xyz, const float *q, float *f, double *out7);
esp_status esp_coulomb_f64(esp_plan_t *p, const double *xyz, const double *q, double *f, double *out7);

/* Synchronise the plan's stream and report device-side errors
 * (ESP_ENONFINITE) seen since the last check; clears the flag. */
esp_status esp_check(esp_plan_t *p);

esp_status esp_get_params(const esp_plan_t *p, esp_params *out);
const char *esp_last_error(const esp_plan_t *p);
void esp_destroy(esp_plan_t *p);

/* ---- stage hooks (for testing each step of the path in isolation) ------
 * esp_stage_spread: cell sort + spreading only; copies the real grid
 *   (M1*M2*M3 reals, index (g3*M2 + g2)*M1 + g1, i.e. g1 fastest; a
 *   fixed-point grid converted to the plan's precision) to grid_out
 *   (device) and leaves the plan's grid cleared.
 * esp_stage_fft: forward real-to-complex 3D FFT of grid_in (device, layout
 *   as above, unnormalised, sign exp(-2 pi i m.g/M)) into spec_out (device,
 *   (M1/2+1)*M2*M3 complex numbers as interleaved re,im; index
 *   (m3*M2 + m2)*(M1/2+1) + m1).
 * esp_stage_potential: the full force path up to the potential grid phi
 *   (unnormalised inverse FFT of F_hat rho_hat / (V W_hat^2)), copied to
 *   phi_out (device, real grid layout).
 * esp_stage_sort: cell sort only; copies the permutation (int32, sorted
 *   position -> particle index, n entries) and the tile offsets (int32,
 *   ntiles + 1 entries) to perm_out / offsets_out (device).
 * Precision of the real/complex buffers follows the plan. */
esp_status esp_stage_sort(esp_plan_t *p, const void *xyz, const void *q, int32_t *perm_out,
                          int32_t *offsets_out);
esp_status esp_stage_spread(esp_plan_t *p, const void *xyz, const void *q, void *grid_out);
esp_status esp_stage_fft(esp_plan_t *p, const void *grid_in, void *spec_out);
esp_status esp_stage_potential(esp_plan_t *p, const void *xyz, const void *q, void *phi_out);

/* Stream used by every subsequent call on the plan (hipStream_t; NULL =
 * the default stream). */
esp_status esp_set_stream(esp_plan_t *p, void *stream);

/* ---- host-only helpers (no device needed) -------------------------------
 * esp_resolve_params: the parameters esp_plan would choose for (h, n, tol,
 *   o), with the same validation and error codes, without touching the
 *   device.
 * esp_pswf_eval: psi_0^c (unit L2 norm, psi(0) > 0) and its derivative at
 *   m points x (any real x; beyond |x| = 1 the eigen-equation continuation),
 *   plus int_0^x psi for |x| <= 1 (NaN outside); the constants
 *   {psi(0), C0 = int_0^1 psi, lambda0} are written to consts3 if non-NULL.
 *   All pointers are host pointers.  Useful for the caller's real-space
 *   kernel N^c(r) = (1 - int_0^{r/rc} psi / C0) / r (Sec. 3.1).
 * esp_c_from_delta: the bandwidth c with psi_0^c(1) / psi_0^c(0) = delta. */
esp_status esp_resolve_params(const double h[9], int64_t n, double tol, const esp_opts *o,
                              esp_params *out);
esp_status esp_pswf_eval(double c, int64_t m, const double *x, double *psi, double *dpsi,
                         double *ipsi, double *consts3);
double esp_c_from_delta(double delta);

/* ---- per-stage timing ----------------------------------------------------
 * Stages, in launch order: 0 bin (with the tile-offset scan), 1 scatter (the
 * two make up the cell sort), 2 spread, 3 fft_xy, 4 fft_z (z transform +
 * scaling/reduction + final FP64 sums [+ G and inverse z]), 5 fft_xy_inv,
 * 6 gather.
 * esp_profile_enable: record a HIP event pair on the plan's stream around
 *   every stride-th launch (stride >= 1) of the stages in stage_mask (bit s =
 *   stage s), for up to max_launches timed launches per stage; mask 0 turns
 *   profiling off.  Synchronises.
 * esp_profile_read: synchronise and return, per stage (ESP_NUM_STAGES
 *   entries, host arrays), the accumulated milliseconds and launch counts
 *   since profiling was enabled. */
#define ESP_NUM_STAGES 8
esp_status esp_profile_enable(esp_plan_t *p, unsigned stage_mask, int max_launches, int stride);
esp_status esp_profile_read(esp_plan_t *p, double *total_ms, int64_t *launches);
const char *esp_stage_name(int stage);

/* ---- learned parameter proposer ------------------------------------------
 * A small MLP (tanh hidden layers, linear output), trained and evaluated on
 * the GPU by the library's own kernels (FP32).  Parameters are one flat
 * array, layer by layer: W (dims[l+1] x dims[l], row-major) then b.
 * All x / t / mask / y / grad / loss pointers are device pointers; B rows.
 * esp_mlp_gradient: forward + backward of the masked mean squared error
 *   sum mask (y - t)^2 / sum mask; writes the gradient (num_params floats)
 *   and the loss (one float) when the pointers are non-NULL.
 * esp_mlp_train_step: the same, then one Adam step (beta 0.9 / 0.999). */
typedef struct esp_mlp_s esp_mlp_t;
esp_status esp_mlp_create(int nlayer, const int *dims, uint64_t seed, esp_mlp_t **out);
int64_t esp_mlp_num_params(const esp_mlp_t *m);
esp_status esp_mlp_set_params(esp_mlp_t *m, const float *host, int64_t n);
esp_status esp_mlp_get_params(const esp_mlp_t *m, float *host, int64_t n);
esp_status esp_mlp_set_stream(esp_mlp_t *m, void *stream);
esp_status esp_mlp_forward(esp_mlp_t *m, const float *x, int64_t B, float *y);
esp_status esp_mlp_gradient(esp_mlp_t *m, const float *x, const float *t, const float *mask, int64_t B,
                            float *grad, float *loss);
esp_status esp_mlp_train_step(esp_mlp_t *m, const float *x, const float *t, const float *mask,
                              int64_t B, float lr, float *loss);
void esp_mlp_destroy(esp_mlp_t *m);

/* Registration of a trained MLP as the ESP_LEARNED proposer.  The network
 * maps the features (log10 Delta, P, sigma, log10 of the charge density
 * n/V), each normalised as (f - in_mean) / in_std, to normalised log10
 * relative errors of {energy, diagonal pressure, off-diagonal pressure, RMS
 * force} (de-normalised with out_mean / out_std).  The cell shape enters
 * through the grid rule, which sizes M_d per cell vector.  esp_plan with
 * ESP_LEARNED scores a grid of candidates (Delta from 1e-2 to 1e-7 in
 * quarter decades, P from ceil(-log10 Delta) - 1 (at least 3) to + 2, sigma
 * from 0.85 to 1.3, plus the analytic rule's own choice) on the GPU, keeps
 * those whose predicted errors of the components the coupling needs
 * (energy, diagonal pressure and force; plus off-diagonal for ESP_FLEX) are
 * below log10(tol) - margin[component], and picks the cheapest by the cost
 * model t = cost[0] + cost[1] N P^3 + cost[2] G log2 G + cost[3] N
 * + cost[4] G (G = M1 M2 M3).  If none qualifies it takes the candidate
 * with the smallest predicted excess and returns ESP_WARN_FALLBACK; without
 * a registered network ESP_LEARNED uses the analytic rule and returns
 * ESP_WARN_FALLBACK.  The MLP is borrowed and must outlive the
 * registration; NULL clears it. */
#define ESP_PROPOSER_FEATURES 4
typedef struct {
  const esp_mlp_t *mlp;
  double in_mean[ESP_PROPOSER_FEATURES], in_std[ESP_PROPOSER_FEATURES];
  double out_mean[4], out_std[4];
  double margin[4];
  double cost[5];
} esp_proposer;
esp_status esp_proposer_set(const esp_proposer *p);

/* ---- batches of independent systems ------------------------------------
 * Many replicas (each its own cell, particle count and tolerance) evaluated
 * together: every stage is ONE launch over all replicas (spreading and
 * gather: one launch per distinct window support P and window degree), so
 * the launch count per step does not grow with the number of replicas.
 *   esp_batch_plan: nrep replicas; h: 9*nrep doubles (host), n, tol: nrep
 *     entries (host); o applies to every replica (o->precision, coupling,
 *     rc, params ...); tiles (host, may be NULL) overrides the spreading tile
 *     edge per replica (0 = the plan's rule).
 *   xyz, q, f: the replicas' arrays concatenated in replica order (3*sum n,
 *     sum n, 3*sum n; device); out7: 7*nrep doubles (device), replica r at
 *     out7 + 7*r.  out7 may be NULL for esp_batch_forces.
 *   esp_batch_set_box: new cell of replica r (host, 9 doubles); the update
 *     is enqueued on the batch stream.
 *   esp_batch_set_graph: with enable != 0 each call records its launches
 *     once into a HIP graph (re-recorded when the pointers or the kind of
 *     call change) and replays it; the graph holds no memset nodes.
 *   esp_batch_check: synchronise and report device-side errors of any
 *     replica (as esp_check).
 * Batched forces use analytic differentiation (o->force must be ESP_FORCE_AD).
 * Errors and warnings of a replica's planning are returned by
 * esp_batch_plan with the replica index in the error text. */
esp_status esp_batch_plan(int nrep, const double *h, const int64_t *n, const double *tol,
                          const esp_opts *o, const int *tiles, esp_batch_t **out);
esp_status esp_batch_energy_virial(esp_batch_t *b, const float *xyz, const float *q, double *out7);
esp_status esp_batch_forces(esp_batch_t *b, const float *xyz, const float *q, float *f,
                            double *out7);
esp_status esp_batch_energy_virial_f64(esp_batch_t *b, const double *xyz, const double *q,
                                       double *out7);
esp_status esp_batch_forces_f64(esp_batch_t *b, const double *xyz, const double *q, double *f,
                                double *out7);
esp_status esp_batch_set_box(esp_batch_t *b, int r, const double h[9]);
esp_status esp_batch_set_stream(esp_batch_t *b, void *stream);
esp_status esp_batch_set_graph(esp_batch_t *b, int enable);
esp_status esp_batch_check(esp_batch_t *b);
esp_status esp_batch_get_params(const esp_batch_t *b, int r, esp_params *out);
int esp_batch_num_launches(const esp_batch_t *b, int forces);
const char *esp_batch_last_error(const esp_batch_t *b);
void esp_batch_destroy(esp_batch_t *b);

/* Library version string. */
const char *esp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ESP_MI355X_H */
