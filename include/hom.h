/*
 * hom.h -- C ABI of the MI355X FFT homogenization library (libhom.so).
 *
 * The library solves the thermomechanical cell problem of first-order
 * homogenization with a microscopically homogeneous temperature (paper
 * Sec. 2, equation "micro cell problem"): for a prescribed macro strain E and
 * macro temperature theta, find the periodic strain field with mean E whose
 * stress is divergence free, for a voxel microstructure whose phases follow
 * the laws of Sec. 4 (isotropic linear thermoelasticity; the PA66
 * thermo-viscoelastic / viscoplastic law). The internal variables are
 * integrated by implicit Euler (Sec. 3.3, condensed incremental potential).
 * It returns the effective quantities of Sec. 2: stress <sigma>, heat flux
 * <q> = -<kappa grad theta> for a prescribed macro temperature gradient (the
 * effective-conductivity problem of Sec. 6), dissipation <D_diss>, coupling
 * term <D> and heat capacity <c0>.
 *
 * Discretization: trigonometric collocation on voxel centres (Moulinec-
 * Suquet, cited in Sec. 5.2/5.4); for even grid sizes the Nyquist frequency
 * of an axis gets a zero wave number.
 *
 * Conventions
 *   - Strain / stress tensors cross the ABI as 6 components in the order
 *     (11, 22, 33, 23, 13, 12) with tensorial (not engineering) shear.
 *   - Units: MPa, s, K, m. Heat capacity c0 in MPa/K, conductivity in
 *     W/(m K), temperature gradient in K/m, heat flux in W/m^2,
 *     dissipation and coupling term in MPa/s.
 *   - Voxel arrays are x-fastest: index = x + nx (y + ny z).
 *   - Phase ids are uint8; phase id i follows laws[i].
 *
 * Ownership: the caller owns every array passed in or out. Setup copies the
 * phases and law parameters to the device; a context owns its device memory
 * until it is destroyed. Calls on one context are not thread safe.
 *
 * Errors: every int-returning call returns HOM_OK (0) or a negative code and
 * keeps a message retrievable with hom_last_error / hom_batch_last_error.
 * A failed increment does not commit: internal variables and the last
 * converged strain field are left as they were.
 */
#ifndef HOM_H
#define HOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HOM_OK 0
#define HOM_E_ARG (-1)           /* invalid argument (sizes, ids, parameters) */
#define HOM_E_OOM (-2)           /* device allocation failed */
#define HOM_E_NOT_CONVERGED (-3) /* iteration limit reached before the tolerance */
#define HOM_E_NAN (-4)           /* non-finite residual or breakdown */
#define HOM_E_DEVICE (-5)        /* HIP runtime error */
#define HOM_E_UNSUPPORTED (-6)   /* grid size or law combination not supported */

#define HOM_MAX_MAXWELL 16
#define HOM_MAX_LAWS 8

typedef enum { HOM_LAW_THERMOELASTIC = 1, HOM_LAW_PA66 = 2 } hom_law_kind;

/* Grid: n[0] = nx (fastest), n[1] = ny, n[2] = nz; len = cell edge lengths
 * (only their ratios matter). Each n must be one of 16, 24, 32, 48, 64, 96,
 * 128, 256. */
typedef struct {
  int32_t n[3];
  double len[3];
} hom_grid;

/* Constitutive law of one phase (paper Sec. 4).
 * Thermoelastic: E, nu, alpha0, kappa0, c0, theta0 (stress-free temperature).
 * PA66: additionally n_maxwell branches (E_i, log10 of tau_i in s), WLF
 * constants C1, C2 [K], theta_ref, yield stress sigma_y0, hardening
 * H = Gamma(theta, beta1) k_h eps_p^n_h, viscosity eta0 and exponent m (>= 1),
 * softening exponents beta1, beta2. At most one PA66 law per setup. */
typedef struct {
  int32_t kind;
  double E, nu, alpha0, kappa0, c0, theta0;
  int32_t n_maxwell;
  double E_i[HOM_MAX_MAXWELL];
  double log10_tau_i[HOM_MAX_MAXWELL];
  double C1, C2, theta_ref, sigma_y0, k_h, n_h, eta0, m, beta1, beta2;
} hom_law;

#define HOM_SCHEME_BASIC 0     /* Moulinec-Suquet fixed point, isotropic reference medium */
#define HOM_SCHEME_NEWTON_CG 1 /* inexact Newton with CG on the projected tangent system */
#define HOM_FP64 0             /* all fields in FP64 */
#define HOM_FP32 1             /* FP32 fields; FP64 reductions, CG scalars, return mapping and state */
#define HOM_DISC_COLLOCATION 0 /* Moulinec-Suquet trigonometric collocation (Sec. 5.4) */
#define HOM_DISC_ROTATED 1     /* rotated finite differences: the projector with modified wave vectors
                                  k_j = (e_j - 1) / h_j prod_{l != j} (1 + e_l) / 2, e_j = exp(i 2 pi k_j / n_j),
                                  the discretization the paper cites for its stiffness samples (Sec. 5.2,
                                  "staggered grid"); Newton-CG only */

typedef struct {
  int32_t scheme;      /* HOM_SCHEME_* */
  int32_t precision;   /* HOM_FP64 / HOM_FP32 */
  double tol;          /* relative residual tolerance (mechanics) */
  double thermal_tol;  /* relative tolerance of the conduction problem; 0 => tol */
  int32_t max_iter;    /* basic: iterations; Newton: residual evaluations; 0 => default */
  int32_t max_krylov;  /* CG iterations per Newton step; 0 => default */
  int32_t chunk;       /* solver iterations launched between host checks; 0 => default (4 from 2^22
                          voxels in a group, else 16) */
  int32_t use_graph;   /* 1: replay chunks as captured hipGraphs */
  int32_t profile;     /* 1: time every kernel launch with HIP events */
  int32_t autotune;    /* 1: time the tile choices of the y/z passes at setup */
  void* stream;        /* hipStream_t to run on; NULL => a stream owned by the context */
  int32_t tangent;     /* 1: keep the per-voxel partials of each converged increment that the
                          temperature and coupling tangents need (hom_algorithmic_tangent,
                          what = 1); costs 13 field components of memory and one pass of
                          14 PA66 point evaluations per increment */
  int32_t discretization; /* HOM_DISC_*; default collocation */
  int32_t predictor;   /* 1: start the mechanical solve of an increment from the committed strain
                          plus the macro increment plus s times the strain fluctuation that the
                          last committed increment added, s = dE . dE_last / |dE_last|^2 clamped
                          to [0, 2] (Mandel, strain-controlled components; s = 0 after hom_set_state or
                          hom_set_laws); costs 6 field components of memory and one more write
                          stream in the commit. It also starts each linearized solve of
                          hom_algorithmic_tangent from the same column's solution of the previous
                          call (up to 42 more field components, allocated on the first call).
                          0: the uniform start eps^n + dE (default) */
} hom_options;

/* Macroscopic temperature input: theta [K] and its gradient [K/m]. */
typedef struct {
  double theta;
  double grad[3];
} hom_macro_temp;

typedef struct {
  double stress[6];      /* <sigma>, components (11,22,33,23,13,12) */
  double heat_flux[3];   /* <q> = -<kappa g> */
  double dissipation;    /* <D_diss> */
  double coupling;       /* <D> */
  double heat_capacity;  /* <c0> */
  double residual;       /* final relative residual (mechanics) */
  int32_t newton_iters;  /* residual evaluations (Newton) or iterations (basic) */
  int32_t krylov_iters;  /* CG iterations (mechanics) */
  int32_t thermal_iters; /* iterations of the conduction problem */
  int32_t status;        /* HOM_OK or the error code of this problem */
  double pipelines;      /* FFT pipeline applications (mechanics) */
  double thermal_pipelines;
  double strain[6];      /* <eps> of the increment, components (equals the prescribed strain
                            where it is strain-controlled) */
  double theta;          /* temperature the increment was solved at (theta^{n+1}) */
  int32_t stagger_iters; /* mechanical solves of the adiabatic staggering (1 otherwise) */
  int32_t reserved;
} hom_result;

/* One load increment of a single-point virtual experiment.
 * Mixed boundary conditions (the paper's stress-free lateral directions,
 * Sec. 5.4 and the appendix): bit c of stress_mask set => component c (order
 * 11,22,33,23,13,12) is stress-controlled with <sigma>_c = stress[c];
 * otherwise <eps>_c = strain[c]. The stress-controlled strain components are
 * unknowns of the same Newton-CG iteration: the zero-frequency block of the
 * projector keeps them instead of removing them. Needs the Newton-CG scheme.
 * adiabatic = 1: temp.theta is theta^n and theta^{n+1} solves the macroscopic
 * heat equation of Sec. 2 at one point without source or flux divergence,
 * <c0> (theta^{n+1} - theta^n) / dt = <D>, by implicit staggering (mechanics
 * at fixed theta, then theta from the heat equation, until theta is
 * stationary to tol times its change). */
typedef struct {
  double strain[6];
  double stress[6];
  uint32_t stress_mask;  /* bits 0..5 */
  int32_t adiabatic;
  hom_macro_temp temp;
  double dt;
  int32_t trial;         /* 1: solve, return the outputs and keep the tangent, but commit
                            nothing (internal variables, converged strain field and macro
                            strain stay at step n), as a macroscopic Newton iteration needs;
                            the same for every problem of a batch */
  int32_t reserved;
} hom_load;

typedef struct hom_ctx hom_ctx;
typedef struct hom_batch hom_batch;

/* Fill opts with defaults: Newton-CG, FP32, tol 1e-6, graphs on. */
void hom_default_options(hom_options* opts);

/* Create a context for one microstructure. phases: nx*ny*nz ids (host).
 * Returns HOM_OK and *out, or an error code (then *out is NULL). */
int hom_setup(const hom_grid* grid, const uint8_t* phases, const hom_law* laws, int32_t n_laws,
              const hom_options* opts, hom_ctx** out);

/* Solve one load increment to (E, theta, grad theta) over dt > 0 and, on
 * success, commit the internal variables. macro_strain: 6 components. */
int hom_solve_increment(hom_ctx* ctx, const double macro_strain[6], const hom_macro_temp* temp, double dt,
                        hom_result* out);

/* Replace the parameters of the phase laws for later increments: n_laws must
 * equal the setup's, every law keeps its kind and a PA66 law its number of
 * Maxwell branches; the committed fields and internal variables stay, the
 * algorithmic tangent of the last increment is no longer available. One
 * context (or batch) then serves many material samples of one
 * microstructure, as the DMN's training data needs (Sec. 3.2). */
int hom_set_laws(hom_ctx* ctx, const hom_law* laws, int32_t n_laws);
int hom_batch_set_laws(hom_batch* b, const hom_law* laws, int32_t n_laws);

/* hom_solve_increment with mixed boundary conditions and / or the adiabatic
 * heat balance (hom_load). hom_solve_increment(E, temp, dt) equals a load
 * with stress_mask 0 and adiabatic 0. */
int hom_solve_load(hom_ctx* ctx, const hom_load* load, hom_result* out);

/* Checkpoint of the committed state (internal variables, last converged
 * strain and gradient fields, macro history). hom_state_size gives the byte
 * count; get writes it into host_buf, set restores it. */
size_t hom_state_size(const hom_ctx* ctx);
int hom_get_state(hom_ctx* ctx, void* host_buf, size_t bytes);
int hom_set_state(hom_ctx* ctx, const void* host_buf, size_t bytes);

/* Copy a field of the last increment to the host as FP64, voxel arrays of
 * 6 (Mandel) or 3 components, component-major:
 *   0 strain (Mandel), 1 stress of the last evaluation (Mandel),
 *   2 temperature gradient, 3 PA66 internal variables (1 + 6 + 6 n_maxwell). */
#define HOM_FIELD_STRAIN 0
#define HOM_FIELD_STRESS 1
#define HOM_FIELD_GRADIENT 2
#define HOM_FIELD_STATE 3
int hom_get_field(hom_ctx* ctx, int32_t which, double* host_buf, size_t count);

/* Per-kernel timing collected with profile = 1: names, launch counts and
 * accumulated milliseconds. Returns the number of kernel kinds (<= cap). */
int hom_kernel_stats(const hom_ctx* ctx, const char** names, int64_t* launches, double* ms, int32_t cap);

/* Switch per-kernel event timing on (1) or off (0) for later increments; the
 * accumulated statistics are reset. While on, chunks run eagerly (no graph). */
int hom_set_profiling(hom_ctx* ctx, int32_t on);

/* Effective algorithmic tangents of the last converged increment: the
 * derivatives of the effective stress and coupling term with respect to the
 * macro strain and temperature that a macroscopic Newton method needs
 * (Sec. 3.3, computed after Newton's method has converged). The derivatives
 * of the paper's strain jumps become the fluctuation fields of the cell
 * problem linearized at the converged strain with the algorithmic tangent of
 * the local laws: one linear CG solve through the FFT pipeline per unit macro
 * strain, and one with mean zero driven by d sigma / d theta. Point partials
 * that the paper leaves to the law (d sigma / d theta, dD / d eps,
 * dD / d theta) are closed-form for thermoelastic phases and FP64 central
 * differences of the PA66 update (steps 1e-6 in Mandel strain, 1e-3 K).
 *
 * Strain derivatives are taken with respect to the 6 strain components that
 * hom_solve_increment takes (tensorial shear: the component eps_23 moves
 * eps_23 and eps_32 together), stress components as in hom_result.
 * what = 0: dsde only (6 solves), the other fields are set to NaN;
 * what = 1: all four (7 solves); needs a setup with opts.tangent = 1.
 * Needs the Newton-CG scheme and a converged last increment (for a batch:
 * every problem's), else HOM_E_UNSUPPORTED / HOM_E_ARG. The strain and stress
 * fields of the increment are left as they were; the calls may be repeated. */
typedef struct {
  double dsde[36];       /* d<sigma>_I / dE_J, row-major [I][J] */
  double dsdt[6];        /* d<sigma>_I / dtheta [MPa/K] */
  double dDde[6];        /* d<D> / dE_J [MPa/s] */
  double dDdt;           /* d<D> / dtheta [MPa/(s K)] */
  int32_t solves;        /* linearized cell solves */
  int32_t krylov_iters;  /* CG iterations over the solves */
  double pipelines;      /* FFT pipeline applications over the solves */
  int32_t status;        /* HOM_OK */
} hom_tangent;
int hom_algorithmic_tangent(hom_ctx* ctx, int32_t what, hom_tangent* out);

/* Bytes of device memory held by the context. */
size_t hom_device_bytes(const hom_ctx* ctx);

const char* hom_last_error(const hom_ctx* ctx);
void hom_destroy(hom_ctx* ctx);

/* ---- batched microproblems ------------------------------------------------
 * n_prob independent problems, each with its own grid and phases but a shared
 * law table and options. Problems with equal grids are solved together: one
 * launch of every kernel covers all of them, with per-problem solver state on
 * the device. strain: n_prob x 6; temp, dt, out: n_prob entries. */
int hom_batch_setup(int32_t n_prob, const hom_grid* grids, const uint8_t* const* phases, const hom_law* laws,
                    int32_t n_laws, const hom_options* opts, hom_batch** out);
int hom_batch_solve_increment(hom_batch* b, const double* strain, const hom_macro_temp* temp, const double* dt,
                              hom_result* out);
/* hom_solve_load for every problem of a batch; loads, out: n_prob entries. */
int hom_batch_solve_load(hom_batch* b, const hom_load* loads, hom_result* out);
int hom_batch_kernel_stats(const hom_batch* b, const char** names, int64_t* launches, double* ms, int32_t cap);
/* Schedules the autotuner chose (project-written, autotune = 1): per group of
 * problems with one grid, 7 values: nx, ny, nz, then the schedule of the y
 * pass and of the z pass of the mechanics, then of the conduction, each a
 * tile width (kx columns per work-group: 2, 4 or 8) + 16 x FFT plan variant
 * (0 or 1). Writes at most cap groups into out (7 cap values); returns the
 * number of groups, or a negative error code. hom_schedules: the same for a
 * single-problem context. */
int hom_batch_schedules(const hom_batch* b, int32_t* out, int32_t cap);
int hom_schedules(const hom_ctx* ctx, int32_t* out, int32_t cap);
/* hom_algorithmic_tangent for every problem of a batch; out: n_prob entries. */
int hom_batch_algorithmic_tangent(hom_batch* b, int32_t what, hom_tangent* out);
const char* hom_batch_last_error(const hom_batch* b);
void hom_batch_destroy(hom_batch* b);

/* ---- learned surrogate ------------------------------------------------------
 * A fully connected network n_in (<= 32) -> 4 x 256 (GELU) -> n_out (<= 16)
 * mapping the macroscopic inputs of an increment (strain, temperature, dt and
 * a summary of the macroscopic history) to the effective outputs. It plays
 * the role the paper gives its learned surrogate (Sec. 3: a fixed
 * microstructure, macroscopic inputs, effective stress and heat outputs),
 * with the FFT solver as fallback and reference. Weights are bf16 on the matrix
 * cores with FP32 accumulation; inputs and outputs are FP32.
 *
 * Parameters cross the ABI in layer order, each layer its weight matrix
 * [out][in] row-major followed by its bias. Scaling: inputs are normalized as
 * (x - x_mean) / x_std, outputs as (y - y_mean) / y_std; the training loss is
 * the loss_weight-weighted mean squared error of the normalized outputs. */
typedef struct hom_mlp hom_mlp;
int hom_mlp_create(int32_t n_in, int32_t n_out, uint64_t seed, hom_mlp** out);
size_t hom_mlp_param_count(const hom_mlp* net);
int hom_mlp_set_scaling(hom_mlp* net, const float* x_mean, const float* x_std, const float* y_mean,
                        const float* y_std, const float* loss_weight);
/* Fixed gated-polynomial skip added to the outputs (default zero), on the
 * normalized inputs xhat: y_j += c_j + sum_g s_g sum_k G[j][g][k] xhat_k with
 * the 10 gate functions s = (1, v0, v0^2, v0^3, v1, .., v2^3), v_i = xhat at
 * input index gates[i]. G is [n_out][10][n_in] row-major, c [n_out]. The
 * network learns the remainder. */
int hom_mlp_set_skip(hom_mlp* net, const int32_t gates[3], const float* G, const float* c);
/* Fit the skip to host rows (x [n][n_in], y [n][n_out]) by least squares
 * (FP64 normal equations, rows weighted by row_weight [n], NULL: all 1) and
 * set the input scaling from x and the output scaling from the residual
 * y - skip(x); loss_weight [n_out] may be NULL (all 1). hom_mlp_train then
 * trains the network on that residual. */
int hom_mlp_fit_skip(hom_mlp* net, const float* x, const float* y, int64_t n, const int32_t gates[3],
                     const float* loss_weight, const float* row_weight);
int hom_mlp_get_params(const hom_mlp* net, float* host, size_t count);
int hom_mlp_set_params(hom_mlp* net, const float* host, size_t count);
/* Train on n rows (host arrays x [n][n_in], y [n][n_out]) with Adam, minibatch
 * `batch`, peak learning rate lr (cosine decay), seeded shuffling; each row's
 * squared error is weighted by row_weight [n] (NULL: all 1, e.g. the inverse
 * square of the row's error normalization); writes the mean loss of every
 * epoch into epoch_loss (epochs entries) if non-null. */
int hom_mlp_train(hom_mlp* net, const float* x, const float* y, int64_t n, int32_t epochs, int32_t batch,
                  double lr, uint64_t seed, const float* row_weight, float* epoch_loss);
/* Inference on device arrays x_dev [n][n_in] -> y_dev [n][n_out] on `stream`.
 * precise = 1 splits the weights into two bf16 parts (FP32-equivalent).
 * Rows are independent (any n, a ragged last tile included); n = 0 returns
 * HOM_OK without touching the arrays. */
int hom_mlp_forward(hom_mlp* net, const float* x_dev, float* y_dev, int64_t n, int32_t precise, void* stream);
/* Loss and its gradient w.r.t. all parameters for host rows (x, y); grad has
 * hom_mlp_param_count entries. */
int hom_mlp_loss_grad(hom_mlp* net, const float* x, const float* y, int64_t n, int32_t precise, double* loss,
                      float* grad);
/* Ensemble inference with acceptance for 2 .. HOM_ENSEMBLE_MAX_NETS networks
 * of the same shape: y = mean of the networks; spread = RMS pairwise distance
 * of the stress outputs (the first six), sqrt(2 / (M - 1) sum_m |s_m - s|^2)
 * with s their mean, over max(|s|, floor_scale); accept = spread <= threshold.
 * For two networks the spread is |s_a - s_b| / max(|s|, floor_scale). All
 * arrays on the device; n = 0 returns HOM_OK without touching them. The first
 * network keeps a device scratch of n * count * n_out floats between calls
 * (grown on demand), so calls that share a first network must not overlap. */
#define HOM_ENSEMBLE_MAX_NETS 16
int hom_mlp_ensemble_infer(hom_mlp* const* nets, int32_t count, const float* x_dev, float* y_dev, float* spread_dev,
                           uint8_t* accept_dev, int64_t n, double threshold, double floor_scale, void* stream);
/* For callers that cannot allocate device memory (work under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): hom_mlp_ensemble_infer
 * with the same arguments and results, whose per-network outputs go to a
 * static device array of HOM_STATIC_SCRATCH_FLOATS floats (32 MiB) that each
 * GPU the library runs on holds until the process ends, instead of a buffer
 * the library grows. n * count * n_out above that limit returns HOM_E_ARG
 * before anything is launched (65,536 rows of 8 networks with 16 outputs
 * fit). Nothing is allocated or freed on the device. Every call on one GPU
 * shares that GPU's array, which keeps the last call's contents (each call
 * writes the part it reads first): calls that overlap in time on one GPU race,
 * whichever networks and streams they use. */
#define HOM_STATIC_SCRATCH_FLOATS 8388608
int hom_mlp_ensemble_infer_static(hom_mlp* const* nets, int32_t count, const float* x_dev, float* y_dev,
                                  float* spread_dev, uint8_t* accept_dev, int64_t n, double threshold,
                                  double floor_scale, void* stream);
const char* hom_mlp_last_error(const hom_mlp* net);
void hom_mlp_destroy(hom_mlp* net);

/* ---- surrogate with FFT fallback --------------------------------------------
 * The learned part for one fixed microstructure (the role the paper gives its
 * surrogate, Sec. 3: trained per microstructure, evaluated at Gauss points
 * from macroscopic inputs; the FFT solver generates its data, judges its
 * error and answers where it is not trusted). An ensemble of networks
 * (hom_mlp, 32 -> 4 x 256 GELU -> 10) maps one increment's macroscopic
 * inputs to its effective outputs:
 *   inputs  x[0:6]  E^{n+1} (Mandel), x[6] theta^{n+1}, x[7] log10 dt,
 *           x[8:14] E^n, x[14:20] <sigma>^n (Mandel), x[20:26] E^{n-1},
 *           x[26] theta^n, x[27] <D_diss>^n, x[28] time integral of <D_diss>
 *           up to step n, x[29:32] grad theta of the increment;
 *   outputs y[0:6] <sigma>^{n+1} (Mandel), y[6:9] <q>, y[9] <D_diss>^{n+1}.
 * Every input is macroscopic, so a caller rolls the summary forward from the
 * surrogate's own answers. Before the first increment E^n = E^{n-1} = 0,
 * <sigma>^n = 0, <D_diss>^n = 0, theta^n = theta_init. Rows the library
 * builds from rolled summaries (point sets, calibration, training rounds)
 * have their summary inputs x[8:29] clamped to the range of the training
 * rows.
 * The ensemble mean is the answer; the RMS pairwise spread of the stress
 * outputs over max(|mean stress|, floor_scale) decides acceptance against a
 * threshold calibrated on held-out histories: the largest threshold under
 * which at least `quantile` of the accepted held-out rows meet `target` in the
 * paper's error measure |<sigma>_net - <sigma>_FFT| / max_t |<sigma>_FFT|
 * over the history (Sec. 5.4), with the held-out histories rolled forward
 * from the networks' own answers (no FFT value enters their summaries).
 *
 * Point sets (hom_surrogate_points_*): many Gauss points advanced increment by
 * increment. The library keeps each point's summary and macroscopic history.
 * A point whose ensemble answer is rejected is handed to the FFT solver for
 * the rest of its history: a batched solve replays its macroscopic history on
 * a fresh cell (the cell state at step n exists nowhere else), answers the
 * increment, and the cell stays resident in device memory and is advanced
 * with the point's later increments (up to max_resident cells; beyond that a
 * rejected point's cell is replayed, answers and is dropped, and the point
 * returns to the ensemble with a summary taken from the FFT answer).
 * Histories: strain [count][steps][6] (components), theta [count][steps],
 * grad [count][steps][3], dt [count][steps]; host arrays, all histories in
 * lockstep. */
typedef struct hom_surrogate hom_surrogate;
typedef struct hom_surrogate_points hom_surrogate_points;
#define HOM_SURROGATE_IN 32
#define HOM_SURROGATE_OUT 10
typedef struct {
  int32_t n_nets;       /* ensemble size, 2 .. HOM_ENSEMBLE_MAX_NETS (default 8) */
  int32_t epochs;       /* training epochs per network (default 100) */
  int32_t batch;        /* minibatch rows (default 4096) */
  double lr;            /* peak Adam learning rate, cosine decay (default 8e-3) */
  uint64_t seed;        /* initialization, shuffling and the hold-out split (default 0) */
  double target;        /* relative effective-stress error to meet (default 1e-3) */
  double quantile;      /* share of accepted held-out rows that must meet it (default 1: all) */
  double holdout;       /* share of the training histories held out for calibration (default 0.1) */
  double floor_scale;   /* MPa: stress magnitude below which the spread is absolute (default 0.01) */
  double theta_init;    /* temperature before the first increment, K (default 293.15) */
  int32_t chunk;        /* problems per batched FFT solve, data and fallback (default 1024) */
  int32_t max_resident; /* FFT cells kept resident for rejected points of a point set (default 2048) */
} hom_surrogate_config;
typedef struct {
  int64_t train_rows, holdout_rows;
  double threshold;                  /* calibrated spread threshold */
  double holdout_accepted;           /* share of held-out rows (network rollout) accepted */
  double holdout_accepted_max_error; /* largest error of those rows */
  double holdout_accepted_p99_error;
  double holdout_median_error;        /* all held-out rows, network rollout */
  double holdout_median_error_forced; /* the same rows with the FFT history as summary */
  double skip_median_error;           /* the fixed skip alone (no network), FFT history as summary */
  double fit_seconds;                 /* skip fits and network training, all networks */
  double final_loss[HOM_ENSEMBLE_MAX_NETS]; /* last epoch's mean loss of each network */
} hom_surrogate_report;
typedef struct {
  int32_t network_points;      /* points answered by the ensemble */
  int32_t rejected_points;     /* points whose ensemble answer this call rejected */
  int32_t resident_points;     /* points answered by a resident FFT cell kept from an earlier call */
  int32_t replayed_increments; /* FFT increments solved to bring new cells up to this increment */
  double network_ms;           /* wall time of feature build, ensemble and acceptance */
  double fallback_ms;          /* wall time of the FFT fallback (cell setup, replay, solves) */
} hom_surrogate_step_info;
void hom_surrogate_default_config(hom_surrogate_config* cfg);
/* The microstructure, laws and solver options of the FFT side (data and
 * fallback; opts->stream must be NULL), and the ensemble configuration. */
int hom_surrogate_create(const hom_grid* grid, const uint8_t* phases, const hom_law* laws, int32_t n_laws,
                         const hom_options* opts, const hom_surrogate_config* cfg, hom_surrogate** out);
/* The batched FFT solver over `count` histories (chunks of cfg.chunk
 * problems): out [count][steps]. seconds (may be NULL): [0] wall time of the
 * increments, [1] of the cell setups. */
int hom_surrogate_solve_histories(hom_surrogate* s, int32_t count, int32_t steps, const double* strain,
                                  const double* theta, const double* grad, const double* dt, hom_result* out,
                                  double* seconds);
/* Input rows of histories whose summaries come from the given FFT answers
 * (host, no device): X [count * steps][32], Y [count * steps][10] (targets),
 * denom [count * steps] = max_t |<sigma>_FFT| of the row's history (Mandel
 * norm); Y and denom may be NULL. */
int hom_surrogate_features(int32_t count, int32_t steps, const double* strain, const double* theta,
                           const double* grad, const double* dt, const hom_result* fft, double theta_init, float* X,
                           float* Y, double* denom);
/* Trains the ensemble on histories and their FFT answers (fft NULL: the
 * library solves them first): the fixed skip and scaling fitted by least
 * squares, every network trained on the remainder from its own host thread
 * and stream; then calibrates the threshold on the held-out histories. */
int hom_surrogate_train(hom_surrogate* s, int32_t count, int32_t steps, const double* strain, const double* theta,
                        const double* grad, const double* dt, const hom_result* fft, hom_surrogate_report* rep);
/* Re-calibrates the threshold for another target / quantile on the given
 * histories (network rollout, as in training). rep may be NULL. */
int hom_surrogate_calibrate(hom_surrogate* s, int32_t count, int32_t steps, const double* strain,
                            const double* theta, const double* grad, const double* dt, const hom_result* fft,
                            double target, double quantile, hom_surrogate_report* rep);
int hom_surrogate_set_threshold(hom_surrogate* s, double threshold);
double hom_surrogate_threshold(const hom_surrogate* s);
/* Stateless rows: x_dev [n][32] -> y_dev [n][10] (ensemble mean) and
 * accepted_dev [n] (1 when the spread is within the threshold; no fallback:
 * the caller owns the history). Device arrays, on `stream`; n = 0 is a no-op. */
int hom_surrogate_infer(hom_surrogate* s, const float* x_dev, float* y_dev, uint8_t* accepted_dev, int64_t n,
                        void* stream);
int hom_surrogate_points_create(hom_surrogate* s, int32_t n_points, hom_surrogate_points** out);
/* Advances every point by one increment (strain [n][6], theta [n], grad
 * [n][3], dt [n]): out [n] gets stress (components), heat_flux, dissipation,
 * status and, for FFT answers, coupling, iteration counts and pipelines
 * (coupling NaN for ensemble answers: the network does not predict it);
 * accepted [n] = 1 for an ensemble answer, 0 for an FFT answer. info may be
 * NULL. Returns the worst per-point status. */
int hom_surrogate_points_step(hom_surrogate_points* p, const double* strain, const double* theta, const double* grad,
                              const double* dt, hom_result* out, uint8_t* accepted, hom_surrogate_step_info* info);
const char* hom_surrogate_points_last_error(const hom_surrogate_points* p);
void hom_surrogate_points_destroy(hom_surrogate_points* p);
const char* hom_surrogate_last_error(const hom_surrogate* s);
void hom_surrogate_destroy(hom_surrogate* s);

/* ---- direct deep material network (Sec. 3) ---------------------------------
 * A two-phase direct DMN of depth K (1..10): a perfect binary tree of 2^K - 1
 * laminates with free directions of lamination m (2^K - 1 three-vectors,
 * normalized inside, ordered level K first and the root last) and 2^K leaf
 * weights v (w = max(v, 0)); leaves alternate between phase 1 (the 1st, 3rd,
 * ... leaf) and phase 2. Stiffnesses cross the ABI as 6 x 6 row-major
 * matrices in normalized Voigt-Mandel notation, host FP64.
 *
 * Offline (Sec. 3.2): hom_dmn_homogenize is the linear homogenization
 * function of n stiffness pairs; hom_dmn_loss_grad the loss
 * J = (1/n) (sum_s e_s^q)^(1/q) + penalty (sum w - 1)^2, with
 * e_s = |C_eff,s - DMN_s|_1 / |C_eff,s|_1 over the components, and its
 * gradients for all n samples as one batch; hom_dmn_train runs epochs of
 * random mini-batches (incomplete batches dropped) with AMSGrad and the
 * paper's learning-rate modulation
 * lr(epoch) = decay^epoch (lr_min + (lr_max - lr_min) (1 + cos(pi epoch / M)) / 2),
 * writing the mean batch loss of each epoch to epoch_loss (epochs entries,
 * or NULL). FP64 kernels, one work-group per sample.
 *
 * Online (Sec. 3.3, the online algorithm): n_points macroscopic points, each
 * with its own internal variables and jumps; hom_dmn_online_step solves the
 * balance of the jumps by Newton's method with the paper's backtracking
 * (steps 1, 1/2, 1/4, ..., at most 8 cuts) and residual, at tolerance tol and
 * at most maxit Newton steps, then commits (status HOM_OK) or not
 * (HOM_E_NOT_CONVERGED); trial = 1 never commits (a macroscopic Newton
 * iteration), the jumps are kept as the next start. what = 0 returns d<sigma>/dE of the four
 * algorithmic tangents of Sec. 3.3, what = 1 all four (the point partials of
 * the PA66 leaves by central differences, as for hom_algorithmic_tangent).
 * Phase laws: laws[0] for phase 1, laws[1] for phase
 * 2 (at most one PA66). strain [n_points][6] (components), theta and dt
 * [n_points] each, host arrays; points may differ in theta and dt. Depth up
 * to 8 (one wave per point: each lane holds up to four leaves, the levels
 * above are combined across the lanes). */
typedef struct hom_dmn hom_dmn;
typedef struct hom_dmn_online hom_dmn_online;
typedef struct {
  double lr_max, lr_min; /* paper: 1.5e-2, 1.5e-3 */
  int32_t half_period;   /* M; paper: 50 */
  double decay;          /* paper: 0.999 */
  double q, penalty;     /* paper: 10, 1e3 */
} hom_dmn_train_opts;
typedef struct {
  double stress[6];      /* <sigma> = sum_i w_i sigma_i, components */
  double coupling;       /* sum_i w_i D_i */
  double dissipation;    /* sum_i w_i D_diss,i */
  double dsde[36];       /* d<sigma>_I / dE_J, row-major, as hom_tangent.dsde */
  double dsdt[6];        /* d<sigma>_I / dtheta (what = 1, else NaN) */
  double dDde[6];        /* d<D> / dE_J (what = 1, else NaN) */
  double dDdt;           /* d<D> / dtheta (what = 1, else NaN) */
  double residual;
  int32_t newton_iters;
  int32_t status;
} hom_dmn_result;
void hom_dmn_default_train_opts(hom_dmn_train_opts* opts);
int hom_dmn_create(int32_t K, uint64_t seed, hom_dmn** out);
int hom_dmn_get_params(const hom_dmn* net, double* m, double* v);
int hom_dmn_set_params(hom_dmn* net, const double* m, const double* v);
int hom_dmn_homogenize(hom_dmn* net, int64_t n, const double* C1, const double* C2, double* C_out);
int hom_dmn_loss_grad(hom_dmn* net, int64_t n, const double* C1, const double* C2, const double* C_eff,
                      const hom_dmn_train_opts* opts, double* loss, double* grad_m, double* grad_v);
int hom_dmn_train(hom_dmn* net, int64_t n, const double* C1, const double* C2, const double* C_eff, int32_t epochs,
                  int32_t batch, uint64_t seed, const hom_dmn_train_opts* opts, double* epoch_loss);
const char* hom_dmn_last_error(const hom_dmn* net);
void hom_dmn_destroy(hom_dmn* net);
int hom_dmn_online_create(const hom_dmn* net, const hom_law laws[2], int32_t n_points, double tol, int32_t maxit,
                          hom_dmn_online** out);
int hom_dmn_online_step(hom_dmn_online* o, const double* strain, const double* theta, const double* dt,
                        int32_t what, int32_t trial, hom_dmn_result* out);
/* on = 1: start each point's Newton iteration from its committed jumps plus
 * s times their change over the point's last committed increment, s = the
 * projection dE . dE_last / |dE_last|^2 of the macro increments (Mandel),
 * clamped to [0, 2]; no shift after a trial or unconverged call (the jumps
 * then start where that call left them). Takes effect from the second
 * committed call after it is switched on; switching it on again forgets
 * what an earlier on-period recorded. on = 0 (default): start from the
 * current jumps. Same solutions within the tolerance, fewer Newton steps on
 * smooth histories. HOM_E_ARG for other values. */
int hom_dmn_online_set_predictor(hom_dmn_online* o, int32_t on);
const char* hom_dmn_online_last_error(const hom_dmn_online* o);
void hom_dmn_online_destroy(hom_dmn_online* o);

/* ---- kernel-level entry points (used by the parity tests) ------------------
 * hom_apply_operator: out = IFFT(Op(n) FFT(in)) on one grid, in/out host FP64
 * arrays of ncomp x nvox (component-major). ncomp = 6 (Mandel) with op 0 =
 * projector P(n) of the laminate equation (Sec. 3.2) or op 1 = isotropic
 * reference Green operator (p0 = lambda0, p1 = mu0); ncomp = 3 with op 2 =
 * n (n . q) or op 3 = n (n . q) / p0; op 4 (ncomp 6) and op 5 (ncomp 3): the
 * projectors of the rotated discretization (HOM_DISC_ROTATED). precision:
 * HOM_FP64 / HOM_FP32. */
int hom_apply_operator(const hom_grid* grid, int32_t ncomp, int32_t op, double p0, double p1,
                       int32_t precision, const double* in, double* out);
/* The same with a given schedule of the y and z passes: tile width (kx
 * columns per work-group, 2, 4 or 8) + 16 x FFT plan variant (0 or 1; the
 * solver's autotuner picks among these). hom_apply_operator uses width 4,
 * plan 0. HOM_E_ARG for other values; HOM_E_UNSUPPORTED if the schedule does
 * not fit the work-group limits on this grid. */
int hom_apply_operator_schedule(const hom_grid* grid, int32_t ncomp, int32_t op, double p0, double p1,
                                int32_t precision, int32_t schedule, const double* in, double* out);

/* hom_eval_law: evaluate the law of phase 0 of `law` on count points with
 * strains eps (6 x count Mandel, host FP64), previous strains eps_n, and (PA66)
 * internal variables state (nstate x count, nstate = 7 + 6 n_maxwell), at
 * temperature theta over dt. Writes sigma (6 x count), tangent factors
 * ab (2 x count), direction nd (6 x count), and if commit != 0 also
 * state_out, dissipation and coupling (count each). FP64 on the device. */
int hom_eval_law(const hom_law* law, int64_t count, const double* eps, const double* eps_n,
                 const double* state, double theta, double dt, int32_t commit, double* sigma, double* ab,
                 double* nd, double* state_out, double* dissipation, double* coupling);

#ifdef __cplusplus
}
#endif
#endif /* HOM_H */
