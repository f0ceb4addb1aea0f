/*
 * fe.h - C ABI of an FFT-based elasticity homogenization solver for AMD
 * MI355X (gfx950).
 *
 * The solver runs the Lippmann-Schwinger fixed-point iteration of
 * F. Willot, "Fourier-based schemes for computing the mechanical response
 * of composites with accurate local fields" (arXiv 1412.8398), on a
 * periodic voxel grid:
 *
 *   tau = (C - C0) : eps                       polarization, eq. (6)
 *   e   = eps_bar - G' * tau                   Green operator, eqs. (6), (24)
 *   DS: eps <- e                               direct scheme, eq. (9)
 *   AS: eps <- eps + 2 (C + C0)^-1 C0 : (e - eps)   accelerated scheme, eq. (16)
 *
 * until the equilibrium norm eta of eq. (43) falls below a tolerance.  G' is
 * one of the continuous Moulinec-Suquet operator (eq. (8) with the Nyquist
 * rule of eq. (14)), the Willot-Pellegrini operator (k of eq. (21)), or the
 * rotated-grid operator (k of eq. (36), zeroed where eq. (41) says).
 *
 * Conventions shared by every entry point
 *   - grid: nx, ny, nz voxels; device fields are C-ordered [z][y][x], x fastest.
 *   - tensor fields are structure-of-arrays with 6 planes of N = nx*ny*nz
 *     values in tensor Voigt order (11, 22, 33, 23, 13, 12); shear planes
 *     hold the tensor component eps_ij, not the engineering strain 2 eps_ij.
 *   - macroscopic strains are 6 doubles in the same order.
 *   - phase maps are uint8, one label per voxel, labels < n_phases.
 *   - every device pointer is caller-owned memory on the device the plan was
 *     created on; the library keeps no pointer after a call returns.
 *   - functions return a status; negative values are errors for which nothing
 *     was written to the outputs; fe_last_error() gives a thread-local message.
 *   - argument checks happen before any device work.
 */
#ifndef FE_H_
#define FE_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FE_OK = 0,               /* converged: eta <= tol                           */
  FE_NOT_CONVERGED = 1,    /* iteration cap reached; outputs hold the last iterate */
  FE_DIVERGED = 2,         /* eta non-finite or growing; outputs hold the last iterate */
  FE_ERR_INVALID_ARG = -1, /* a bad argument; nothing was run                 */
  FE_ERR_UNSUPPORTED = -2, /* valid but not supported (e.g. a grid size)      */
  FE_ERR_OOM = -3,         /* device allocation failed                        */
  FE_ERR_DEVICE = -4       /* a HIP runtime error                             */
} fe_status;

/* Discrete Green operator (§3, §4 of the paper). */
typedef enum {
  FE_GREEN_MS = 0,      /* continuous operator, k = i q, eqs. (8), (14)       */
  FE_GREEN_WP = 1,      /* Willot-Pellegrini, k = exp(i q) - 1, eq. (21)       */
  FE_GREEN_ROT = 2,     /* rotated grid, k of eq. (36), special modes eq. (41)  */
  FE_GREEN_CENTERED = 3, /* centered differences, k = i sin q (§4.2); zero where
                           every q_i is 0 or pi, eq. (29).  Six-component form
                           like FE_GREEN_MS.                                 */
  FE_GREEN_MS_SYMMETRIZED = 4 /* continuous operator with the symmetrised
                           Nyquist rule of eq. (15) instead of eq. (14): at a
                           mode with some q_i = pi, the mean of eq. (8) at q
                           and at its grid partner (-q with the Nyquist
                           components kept at +pi), a real operator equal at
                           the two; eta (eq. (43)) is summed over the other
                           modes, where equilibrium is imposed.  The fixed
                           point depends on C0 (eq. (14)'s does not).       */
} fe_discretization;

typedef enum {
  FE_DIRECT = 0,              /* eq. (9)                                            */
  FE_ACCELERATED = 1,         /* eq. (16)                                           */
  FE_CONJUGATE_GRADIENT = 2   /* conjugate gradients on the discrete problem of
                                 eq. (19), the use of the modified operators that
                                 §1 and §7 name; reference medium of eq. (17)
                                 (FE_REF_PAPER), start eps_bar only (strain_init
                                 must be NULL); not with FE_GREEN_MS_SYMMETRIZED
                                 (FE_ERR_UNSUPPORTED at plan creation).
                                 WP and ROT (corner displacement, preconditioned
                                 by the reference medium's operator): the true
                                 residual is recomputed when the recursive one
                                 reaches tol or stalls, and the iteration
                                 restarts from it on drift.  Float32 plans with
                                 refine (the default) keep the displacement in
                                 float64 and form every true residual in
                                 float64; the float32 strain returned must
                                 verify <= tol (else FE_NOT_CONVERGED).  Without
                                 refine a restart gaining less than a factor 2
                                 ends the run (FE_NOT_CONVERGED, float32 floor).
                                 MS and CENTERED (six-component form): CG on the
                                 strain in the inner product sum a:C0:b, eta of
                                 the iterate every iteration; float32 plans run
                                 in float32 (no 5% gain in eta over 100
                                 iterations: FE_NOT_CONVERGED).               */
} fe_scheme;

/* Arithmetic of the fields, FFTs and Green operator.  Reductions (eta, mean
 * stress), reference-medium constants and the verification residual are
 * always float64. */
typedef enum { FE_FP64 = 0, FE_FP32 = 1 } fe_precision;

/* Reference medium C0 (isotropic). */
typedef enum {
  FE_REF_PAPER = 0,    /* AS: kappa0 = sqrt(kmin kmax), mu0 = sqrt(mumin mumax), eq. (17);
                          DS: kappa0 = beta (kmin + kmax), mu0 = beta (mumin + mumax), eq. (18) */
  FE_REF_EXPLICIT = 1  /* Young's modulus E0 and Poisson ratio nu0 given (§6.1) */
} fe_ref_rule;

typedef struct {
  int32_t nx, ny, nz;
} fe_grid;

typedef struct {
  uint32_t struct_size;   /* sizeof(fe_plan_options)                             */
  fe_precision precision; /* default FE_FP32                                      */
  int32_t max_iter;       /* iteration cap, default 1000                          */
  int32_t ref_rule;       /* fe_ref_rule, default FE_REF_PAPER                     */
  double ds_beta;         /* beta of eq. (18), default 0.5                         */
  double E0, nu0;         /* used when ref_rule == FE_REF_EXPLICIT                 */
  int32_t check_every;    /* evaluate eta every m iterations (default 1); the
                             iteration count is then a multiple of m            */
  int32_t diverge_window; /* report FE_DIVERGED after this many consecutive
                             increases of eta (default 50; 0 disables)          */
  int32_t timing;         /* nonzero: time every pass with HIP events on the plan's
                             stream and report it in fe_result.pass_seconds     */
  int32_t refine;         /* FP32 plans: when the float32 iteration stalls (or
                             reaches tol while the float64 check does not),
                             re-anchor in float64 and iterate in float32 on the
                             correction (default 1; 0 = plain float32)         */
  void* hip_stream;       /* hipStream_t to run on; NULL = the null stream        */
  int32_t batch_launch;   /* fe_solve_batched, float32: fe_batch_launch, default
                             FE_BATCH_PER_PASS                                  */
} fe_plan_options;

/* How fe_solve_batched runs the float32 iteration of a batch. */
typedef enum {
  FE_BATCH_PER_PASS = 0,   /* one launch per pass per iteration over the active
                              samples of each grid, eta read back per iteration */
  FE_BATCH_PERSISTENT = 1  /* one cooperative persistent launch for all passes of
                              all iterations, eta and retirement on the device;
                              grid lengths 16, 24, 32, 48, 64, 96, 128 and at
                              most 8 distinct grids (else the per-pass launch) */
} fe_batch_launch;

/* Passes of one iteration, indices of fe_result.pass_seconds / pass_launches. */
enum {
  FE_PASS_POINTWISE = 0, /* divergence stencil (WP, ROT) or polarization (MS)  */
  FE_PASS_ZFWD = 1,      /* real-to-complex transform along z                   */
  FE_PASS_YFWD = 2,      /* complex transform along y                           */
  FE_PASS_XGREEN = 3,    /* transform along x, Green operator, inverse along x  */
  FE_PASS_YINV = 4,      /* inverse transform along y                           */
  FE_PASS_ZINV = 5,      /* complex-to-real transform along z                   */
  FE_PASS_UPDATE = 6,    /* strain update (gradient stencil or pointwise)       */
  FE_PASS_ETA = 7,       /* reductions and the extra transforms of eta (MS)     */
  FE_NUM_PASSES = 8
};

typedef struct fe_plan fe_plan;

/* Fill *opt with the defaults above. */
void fe_plan_options_default(fe_plan_options* opt);

/*
 * Create a plan: validates the grid (each of nx, ny, nz of the form 2^a or
 * 3*2^a, between 4 and 1024; nz may also be 1: a one-plane cell, the 2D
 * problem in plane strain, where every operator takes its 2D form, q3 = 0),
 * allocates the device workspace and builds the FP64 twiddle and
 * wave-vector tables.  opt may be NULL (defaults).
 * Errors: FE_ERR_INVALID_ARG (bad enum/size), FE_ERR_UNSUPPORTED (size outside
 * the supported set), FE_ERR_OOM, FE_ERR_DEVICE.
 */
fe_status fe_plan_create(fe_grid grid, fe_discretization disc, fe_scheme scheme,
                         const fe_plan_options* opt, fe_plan** out);

/* Release a plan and its workspace (NULL is ignored). */
void fe_plan_destroy(fe_plan* plan);

/* Device bytes held by the plan's workspace. */
size_t fe_plan_workspace_bytes(const fe_plan* plan);

/* Per-phase isotropic moduli, host memory, float64: E > 0, -1 < nu < 0.5. */
typedef struct {
  int32_t n_phases; /* 1..256 */
  const double* E;
  const double* nu;
} fe_materials;

typedef struct {
  /* inputs (may be NULL) */
  void* strain;            /* device, 6*N of the plan precision: receives eps^n       */
  void* stress;            /* device, 6*N of the plan precision: receives C:eps^n     */
  double* eta_history;     /* host, receives eta^k for k = 0..min(n, capacity-1)      */
  int32_t history_capacity;
  /* outputs */
  double mean_stress[6];   /* <sigma^n>, float64 volume average (eq. (5))             */
  double eta;              /* eta^n, eq. (43), float64 reduction                      */
  double eta_verify_fp64;  /* eta^n recomputed with float64 arithmetic from eps^n
                              (equals eta for FE_FP64 plans)                           */
  int32_t iterations;      /* n: first k with eta^k <= tol, or the cap                */
  double seconds;          /* wall time of the iteration loop on the device stream    */
  double pass_seconds[8];  /* with fe_plan_options.timing: summed device time per pass */
  int32_t pass_launches[8];/* with fe_plan_options.timing: launches per pass          */
  int32_t refinements;     /* float64 re-anchors performed (fe_plan_options.refine)   */
  /* input (may be NULL): host, receives <sigma^k> (6 values per k, tensor Voigt
     order, float64) for k = 0..min(n, history_capacity-1), the volume averages
     that eta^k is normalised by; the sequence of effective-moduli estimates
     of §6.2 */
  double* mean_stress_history;
} fe_result;

/*
 * Solve one load case.
 *   phase        device, N uint8 labels (checked on the device; a label
 *                >= n_phases gives FE_ERR_INVALID_ARG after the check kernel)
 *   materials    host table of per-phase (E, nu)
 *   macro_strain host, 6 doubles, tensor Voigt order (eq. (4): <eps> = eps_bar)
 *   tol          > 0; iteration stops at the first k with eta^k <= tol
 *   strain_init  device, 6*N of the plan precision, or NULL for eps^0 = eps_bar
 *                (must be NULL for FE_CONJUGATE_GRADIENT: FE_ERR_UNSUPPORTED)
 *                (eq. (9)); its mean need not equal eps_bar
 *   out          result; out->strain may be NULL (the plan then keeps the
 *                iterate in its own workspace)
 * Returns FE_OK, FE_NOT_CONVERGED or FE_DIVERGED with out filled, or an error.
 */
fe_status fe_solve(fe_plan* plan, const uint8_t* phase, fe_materials materials,
                   const double macro_strain[6], double tol, const void* strain_init,
                   fe_result* out);

/*
 * Effective stiffness (eq. (5)) from the six unit macroscopic strains:
 * C_voigt[6*I + J] is <sigma_I> for a normal load J (eps_bar_JJ = 1) and
 * <sigma_I>/2 for a shear load J (eps_bar_ab = eps_bar_ba = 1).
 * iterations[J] receives the iteration count of load J (may be NULL).
 * Returns the worst status over the six solves.
 */
fe_status fe_effective_stiffness(fe_plan* plan, const uint8_t* phase, fe_materials materials,
                                 double tol, double C_voigt[36], int32_t iterations[6]);

/*
 * Batched solves of many independent microstructures (possibly of different
 * grid sizes) with one operator and scheme, e.g. to generate training data.
 * Supported: FE_GREEN_WP and FE_GREEN_ROT (displacement form), FE_DIRECT and
 * FE_ACCELERATED.  Every sample follows the iteration of a single-sample
 * fe_solve with refine = 0 (same kernels, constants and fixed-order
 * reductions): a sample retires as soon as its own eta^k <= tol, its
 * iteration cap is reached, eta rises for diverge_window checks
 * (FE_DIVERGED), or eta has not fallen by 5% over 100 iterations (the
 * float32 storage floor: FE_NOT_CONVERGED).
 *   Float32: the iteration runs as opt->batch_launch says (fe_batch_launch);
 *   then every returned strain is verified in float64, and with opt->refine
 *   (the default) a sample whose float32 strain does not verify to tol
 *   continues with float64 fields from it (one launch per pass per iteration
 *   over those samples only); its strain is returned rounded to float32,
 *   verified again, and FE_OK only if that verification meets tol (a sample
 *   that reached tol in float64 but misses it after the rounding continues
 *   again with tol halved, at most four times, while its verified eta keeps
 *   falling); iterations counts every phase.
 *   Float64: one launch per pass per iteration (FE_BATCH_PERSISTENT gives
 *   FE_ERR_UNSUPPORTED).
 *   desc->phase[i]   device, N_i uint8 labels of sample i
 *   desc->strain[i]  device, 6*N_i of the requested precision, receives eps of
 *                    sample i (NULL: not returned)
 *   results          host, n_samples entries
 *   seconds          host, may be NULL: device time of the iterations
 * Returns FE_OK if every sample converged, FE_NOT_CONVERGED / FE_DIVERGED if
 * some did not (see results[i].status), or an error (nothing written).
 */
typedef struct {
  int32_t n_samples;
  const fe_grid* grids;          /* host, n_samples                              */
  const uint8_t* const* phase;   /* host array of n_samples device pointers      */
  const fe_materials* materials; /* host, n_samples                              */
  const double* macro_strain;    /* host, 6*n_samples, tensor Voigt order       */
  void* const* strain;           /* host array of n_samples device pointers or NULL */
} fe_batch_desc;

typedef struct {
  int32_t status;          /* fe_status of this sample                           */
  int32_t iterations;
  double eta;              /* eta at the returned iterate, float64 reduction    */
  double eta_verify_fp64;  /* eta recomputed with float64 arithmetic            */
  double mean_stress[6];
} fe_batch_result;

fe_status fe_solve_batched(fe_discretization disc, fe_scheme scheme, const fe_plan_options* opt,
                           const fe_batch_desc* desc, double tol, fe_batch_result* results,
                           double* seconds);

/*
 * fe_solve without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the plan's workspace (transform buffers, second iterate,
 * partial sums, phase constants, twiddle and wave tables) is carved from a
 * static device array of FE_STATIC_SCRATCH_BYTES that the library holds on
 * every device it runs on until the process ends; no plan, no events, no
 * pinned buffer.  Same kernels and results as fe_plan_create + fe_solve with
 * the same options, restricted to:
 *   - disc FE_GREEN_WP or FE_GREEN_ROT, scheme FE_DIRECT or FE_ACCELERATED
 *     (FE_ERR_UNSUPPORTED otherwise);
 *   - grids whose workspace fits the array: about 60 bytes per voxel in
 *     float32 (96^3 fits), 120 in float64 (64^3 fits); larger grids give
 *     FE_ERR_UNSUPPORTED before any device work;
 *   - float32 plans iterate in float32 only (opt->refine is not used) and
 *     report eta_verify_fp64 of the returned strain;
 *   - opt->timing must be 0; the convergence check is not overlapped with
 *     the next iteration; out->seconds is host time around the loop;
 *   - out->strain must be a device buffer of 6*N plan-precision values.
 * Runs on the current device and opt->hip_stream.  Calls that overlap on one
 * device share the array and race: serialize them (one stream, or wait for
 * a call to return before the next starts).  Arguments and errors as fe_solve.
 */
#define FE_STATIC_SCRATCH_BYTES (64u << 20)
fe_status fe_solve_static(fe_grid grid, fe_discretization disc, fe_scheme scheme, const fe_plan_options* opt,
                          const uint8_t* phase, fe_materials materials, const double macro_strain[6], double tol,
                          const void* strain_init, fe_result* out);

/*
 * Measurement reference: copy `bytes` (a multiple of 16) from src to dst,
 * both device memory, 16-byte aligned, with the library's streaming copy
 * kernel (16-byte vectors, all loads of a thread in flight before its
 * stores; nontemporal != 0 marks loads and stores as streaming).  dst == src
 * rewrites the buffer in place (each vector read and written back: the
 * access pattern of the solver's in-place passes); other overlaps are
 * errors.  Asynchronous on hip_stream (NULL: the null stream).  The solver's
 * passes are compared with the bandwidth this kernel reaches.
 * Errors: FE_ERR_INVALID_ARG (NULL, size or alignment, partial overlap).
 */
fe_status fe_stream_copy(void* dst, const void* src, size_t bytes, int32_t nontemporal, void* hip_stream);

/* Human-readable name of a status code (static string). */
const char* fe_status_string(fe_status s);

/* Message of the last error raised on the calling thread ("" if none). */
const char* fe_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FE_H_ */
