/*
 * mrhweno.h -- C ABI of the MI355X (gfx950) moment-based multi-resolution
 * HWENO library.
 *
 * The library advances the zeroth and first moments of hyperbolic
 * conservation laws u_t + div f(u) = 0 on uniform 1D and 2D meshes with the
 * moment-based multi-resolution HWENO scheme of Li, Shu and Qiu (arXiv
 * 2201.12193):
 *   - the state of each cell is its cell average and its first moments,
 *     eq. (1D-moment) / (2D-moment), in the cell's reference coordinates;
 *   - the semi-discrete scheme is eq. (1D-equ-int-approximation) /
 *     (2D-equ-int-approximation) with the four-point Gauss-Lobatto
 *     quadratures of eqs. (F), (integral1)-(integral3);
 *   - point values come from the reconstruction algorithm (Step 1: nested
 *     stencils q1..q4, smoothness indicators, WENO-Z nonlinear weights;
 *     Step 2: KXRCF troubled-cell indicator, modification of the first
 *     moments by the quartic of eq. (p0)/(vi), re-reconstruction);
 *   - fluxes are HLLC for the Euler equations (eqs. f_HLLC, COEF, uLR_) and
 *     Lax-Friedrichs for scalar Burgers;
 *   - time stepping is the third-order TVD Runge-Kutta method (eq.
 *     Runge-Kutta) at a CFL number (0.6 in the paper).
 *
 * Memory: every pointer documented as "device" is device memory owned by the
 * caller; the library never allocates device memory (the only device memory
 * of its own is the static scratch array of mrhweno_residual_noalloc, part
 * of its code object) and never copies between host and device inside a
 * step.  Host pointers are read during the call
 * only.  All entry points are asynchronous on the stream given at creation
 * except mrhweno_sync, mrhweno_last_dt and mrhweno_create.
 *
 * Moment layout (FP64, structure of arrays, x fastest):
 *   1D: U[comp][m][nx],       m = 0 (cell average), 1 (first moment)
 *   2D: U[comp][m][ny][nx],   m = 0 (cell average), 1 (x moment), 2 (y moment)
 * Components: Burgers (u); 1D Euler (rho, rho*mu, E); 2D Euler
 * (rho, rho*mu, rho*nu, E).
 *
 * Errors: a negative status is returned for invalid arguments or a failing
 * device call; mrhweno_last_error describes the most recent one.  A
 * non-physical state met on the device (rho <= 0, p <= 0 or non-finite
 * values in a cell average) is latched per instance: later steps of that
 * instance do nothing, the state is rolled back to the last good step, and
 * the next mrhweno_sync returns MRHWENO_ERR_NONPHYSICAL.
 */
#ifndef MRHWENO_H
#define MRHWENO_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mrhweno_ctx mrhweno_ctx;

typedef enum {
  MRHWENO_OK = 0,
  MRHWENO_ERR_INVALID_ARG = -1,
  MRHWENO_ERR_UNSUPPORTED = -2,
  MRHWENO_ERR_DEVICE = -3,
  MRHWENO_ERR_NONPHYSICAL = -4,
  MRHWENO_ERR_NOT_READY = -5    /* learned indicator used before its weights are set */
} mrhweno_status;

typedef enum { MRHWENO_BURGERS_LF = 0, MRHWENO_EULER_HLLC = 1 } mrhweno_flux;
/* Boundary conditions per axis (both ends).  TRANSMISSIVE ghosts copy the
 * boundary cell's averages with zero first moments; REFLECTIVE (Euler only)
 * ghosts are the mirror images of the interior cells across the wall: the
 * wall-normal momentum and the first moment along the normal change sign
 * (a moment flips when exactly one of the two applies); at a wall face the
 * two traces carry opposite normal velocities, so the KXRCF test never
 * counts it as an inflow face.  SIDES: each end of the axis takes its own
 * data from mrhweno_problem.side (not with the learned indicator). */
typedef enum {
  MRHWENO_BC_PERIODIC = 0,
  MRHWENO_BC_TRANSMISSIVE = 1,
  MRHWENO_BC_REFLECTIVE = 2,
  MRHWENO_BC_SIDES = 3
} mrhweno_bc;
/* Kind of one end of an axis whose bc is SIDES.  INFLOW ghosts hold a
 * prescribed constant state: average = state, first moments zero (e.g. the
 * post-shock inflow of the double Mach reflection, Example 3.9). */
typedef enum {
  MRHWENO_SIDE_TRANSMISSIVE = 1,
  MRHWENO_SIDE_REFLECTIVE = 2,
  MRHWENO_SIDE_INFLOW = 3
} mrhweno_side_kind;
/* Boundary data of one side: side[0] left, [1] right, [2] bottom, [3] top.
 * On the bottom and top sides a front may split the ghost cells: with
 * front = 1, the part x < split[0] + split[1] t + split[2] y holds `pre`
 * (a straight front moving at constant speed; t = t^n, t^n + dt,
 * t^n + dt/2 in the three SSP-RK3 stages).  On an INFLOW side the ghosts
 * hold the exact moments of the two-state field (a cut cell: area fraction
 * and first moments of its part before the front) -- e.g. the exact motion
 * of the Mach 10 shock along the top of the double Mach reflection; before
 * a transmissive or reflective side a ghost holds `pre` if its centre lies
 * before the front, else follows `kind` -- e.g. the post-shock part of
 * that problem's bottom.  A ghost outside in both directions takes
 * the bottom/top side's prescribed state if that side prescribes one
 * there, else the left/right side's, else folds in both directions.  A
 * reflective side's face is a wall only where the ghost across it holds no
 * prescribed state. */
typedef struct {
  int kind;                /* mrhweno_side_kind                                  */
  int front;               /* 1: the front applies (bottom and top sides only)  */
  double state[4];         /* INFLOW: conserved state (first ncomp entries)      */
  double pre[4];           /* state of the ghosts before the front               */
  double split[3];         /* front: s0, st, sn                                  */
} mrhweno_side;
/* Step 2 variants named as in the paper's Sec. 3: HWENO6 (no
 * modification), HWENO6-M5-I (KXRCF-flagged cells), HWENO6-M5-NI (every
 * cell).  LEARNED (2D Euler only; not part of the paper) takes the
 * troubled-cell decision of Step 2.1 from a small network trained on KXRCF
 * flags (mrhweno_set_indicator) and falls back to KXRCF for cells whose
 * score lies in an uncertainty band.  TVB uses the minmod-based TVB limiter
 * as the indicator, one of the alternatives of Remark 2: on the indicator
 * variable (density; u for Burgers) a cell is troubled when the modified
 * minmod m~(a, d+, d-) = (|a| <= M h^2 ? a : minmod(a, d+, d-)) changes a
 * face deviation a (face value minus average, or average minus face value;
 * 2D: Gauss-Lobatto face averages, per direction), with d+- the differences
 * of the neighbouring cell averages, h = dx and M = tvb_m. */
typedef enum {
  MRHWENO_TC_NONE = 0,
  MRHWENO_TC_KXRCF = 1,
  MRHWENO_TC_ALL = 2,
  MRHWENO_TC_LEARNED = 3,
  MRHWENO_TC_TVB = 4
} mrhweno_tc;
/* Smoothness indicators of eq. (beta)/(2D-beta) taken on q_l (default; the
 * reading under which Remark 1's expansion holds) or on p_l as printed. */
typedef enum { MRHWENO_BETA_ON_Q = 0, MRHWENO_BETA_ON_P = 1 } mrhweno_beta;
/* Where the modified first moments of Step 2.2 go besides the troubled
 * cells' re-reconstruction (Steps 2.2, 2.3; the paper does not say):
 * PERSIST (default) - they replace those of every stage input in the SSP-RK3
 *                     combination, U^n included (with this reading the
 *                     modify-everywhere variant reproduces Tables 1 and 3);
 * INTERNAL          - nowhere: the combination uses the stored moments;
 * STAGE             - they replace those of the stage input, not of U^n. */
typedef enum { MRHWENO_MOD_PERSIST = 0, MRHWENO_MOD_INTERNAL = 1, MRHWENO_MOD_STAGE = 2 } mrhweno_mod;

/* A problem posed as the paper poses it (Secs. 2.1, 2.2, 3). */
typedef struct {
  int dim;                 /* 1 or 2                                              */
  int nx, ny;              /* cells (ny ignored in 1D); each >= 8; 1D: nx below
                              2^30; 2D: nx*ny below 2^30/13 (82,595,524 cells,
                              e.g. 9088 x 9088); larger grids are rejected     */
  double x0, x1, y0, y1;   /* domain; 2D requires square cells (dx == dy)        */
  int bc_x, bc_y;          /* mrhweno_bc                                         */
  int flux;                /* mrhweno_flux; ncomp = 1 (Burgers), 3 (1D Euler),
                              4 (2D Euler)                                        */
  double gamma_gas;        /* ratio of specific heats (Euler)                    */
  double cfl;              /* CFL number, > 0                                     */
  double t_final;          /* final time (may be +inf for a fixed step count)    */
  double gamma_bar[4];     /* positive linear weights (paper: 1, 10, 100, 1000)  */
  double eps;              /* epsilon of the nonlinear weights (paper: 1e-10)    */
  int tc_mode;             /* mrhweno_tc                                         */
  int beta_on;             /* mrhweno_beta                                       */
  int modification;        /* mrhweno_mod                                        */
  double tvb_m;            /* M of the TVB indicator (>= 0; other modes ignore it) */
  int charwise;            /* Euler only: 1 = Step 1 on the characteristic
                              fields of the flux Jacobian at the target cell's
                              average (left eigenvectors project the stencil
                              moments, right ones map the values back); in 2D
                              one set of values per direction (the x set for
                              the x faces and the volume integral of f, the
                              y set for the y faces and that of g; KXRCF
                              takes each face's set and the norm over both;
                              with the KXRCF, all-cells or no troubled-cell
                              mode); 0 = component by component, as the paper
                              does                                           */
  mrhweno_side side[4];    /* per-side data of an axis whose bc is SIDES       */
  int step_i, step_j;      /* 2D Euler: a solid step, the cells i >= step_i,
                              j < step_j (the forward step of Example 3.10;
                              step_j = 0: none; 0 < step_j <= step_i < nx,
                              2 step_j <= ny).  Its cells carry no state (the
                              steps write zeros there); read as ghosts they
                              are mirror images of fluid cells across the
                              step's nearest face (across the vertical face
                              when fewer columns into the step than rows
                              below its top, across the top in the opposite
                              case, through the corner when equal), with the
                              flips of a reflective wall; its faces are
                              walls.  KXRCF, all-cells or no troubled cells. */
  int wall_flux;           /* 2D Euler: 0 = the printed HLLC on the mirror
                              state at wall faces; 1 = the Godunov flux of
                              the mirror-image Riemann problem (star state
                              at rest: mass and energy flux 0, normal
                              momentum flux the exact star pressure of the
                              reflected shock or rarefaction).  The printed
                              HLLC lets a stream of normal Mach number above
                              about 2 through a wall (its linearised star
                              pressure puts s_L > 0).                     */
} mrhweno_problem;

/* Device workspace needed for n instances (bytes, 256-byte aligned pieces).
 * Returns 0 if a problem is invalid. */
size_t mrhweno_workspace_bytes(const mrhweno_problem* probs, int n_instances);

/* Create a context for n instances that are advanced together.
 *   probs        host array of n problems;
 *   moments_dev  host array of n device pointers, one FP64 moment array per
 *                instance (layout above); in/out: the current state is
 *                returned there by mrhweno_sync;
 *   workspace    device buffer of mrhweno_workspace_bytes(probs, n) bytes;
 *   hip_stream   hipStream_t the library launches on (NULL = default);
 *   out          receives the context (host object owned by the library).
 * The initial time of every instance is 0. */
mrhweno_status mrhweno_create(const mrhweno_problem* probs, int n_instances,
                              void* const* moments_dev, void* workspace_dev,
                              void* hip_stream, mrhweno_ctx** out);

/* Enqueue nsteps SSP-RK3 steps of every instance (asynchronous).  Each step
 * takes dt from the CFL condition on U^n, clipped at t_final; an instance at
 * t_final (or with a latched error) does not change. */
mrhweno_status mrhweno_step(mrhweno_ctx* ctx, int nsteps);

/* Wait for the stream, bring every instance's current state back into its
 * moments_dev array, and report per-instance time (t_out, n doubles) and
 * step count (steps_out, n longs); either may be NULL.  Returns
 * MRHWENO_ERR_NONPHYSICAL if any instance latched a non-physical state. */
mrhweno_status mrhweno_sync(mrhweno_ctx* ctx, double* t_out, long* steps_out);

/* Set time and step counter of one instance (resume from a checkpoint). */
mrhweno_status mrhweno_set_time(mrhweno_ctx* ctx, int instance, double t, long steps);

/* dt of the most recent step of every instance (synchronises; n doubles). */
mrhweno_status mrhweno_last_dt(mrhweno_ctx* ctx, double* dt_out);

/* Steps 1-2 of the reconstruction algorithm once on a given state of
 * instance `instance`:
 *   moments_dev  device, the state (layout above), read only;
 *   gl_dev       device, final Gauss-Lobatto values after Step 2:
 *                1D [comp][4][nx], 2D [comp][16][ny][nx] with point
 *                k + 4 l at (xi_k, eta_l), xi, eta in
 *                {-1/2, -sqrt(5)/10, sqrt(5)/10, 1/2} (2D
 *                characteristic-wise: the x direction's set);
 *   flags_dev    device uint8 [ny][nx] troubled-cell map, or NULL. */
mrhweno_status mrhweno_reconstruct(mrhweno_ctx* ctx, int instance, const void* moments_dev,
                                   void* gl_dev, void* flags_dev);

/* Step 2.1 (troubled-cell indicator) once on a given state:
 *   flags_dev  device uint8 [ny][nx];
 *   aleph_dev  device FP64 [ny][nx][2]: numerator |J| and denominator
 *              h^2 |dI^-| ||u|| of the KXRCF ratio (1D: h^2 ||u||), or NULL;
 *              KXRCF instances only (UNSUPPORTED otherwise). */
mrhweno_status mrhweno_flag(mrhweno_ctx* ctx, int instance, const void* moments_dev,
                            void* flags_dev, void* aleph_dev);

/* The semi-discrete operator L(U) once on a given state (same layout as the
 * state), with the troubled-cell map of that evaluation in flags_dev (or
 * NULL). */
mrhweno_status mrhweno_residual(mrhweno_ctx* ctx, int instance, const void* moments_dev,
                                void* residual_dev, void* flags_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * operator L(U) of mrhweno_residual for one problem without a context and
 * without any allocation.
 *   prob        host problem (not the learned indicator: UNSUPPORTED);
 *   moments_dev device FP64 state (layout above), read only;
 *   residual_dev device FP64 output, same layout;
 *   flags_dev   device uint8 troubled-cell map [ny][nx], or NULL;
 *   hip_stream  hipStream_t to launch on (NULL = default stream).
 * Its descriptor, work lists, troubled-cell plane and 1D face summaries
 * live in a static device array of MRHWENO_NOALLOC_SCRATCH_BYTES that the
 * library holds on every GPU it runs on until the process ends; a problem
 * that needs more returns MRHWENO_ERR_INVALID_ARG with the size it needs
 * (2D: about (nx+4)(ny+4) bytes plus the work lists; 1D KXRCF/TVB: about
 * 40 (nx+6) bytes more).  Calls on one GPU share that array: two calls
 * that overlap in time on the same GPU (different streams or threads)
 * race and give undefined results.  Synchronises the stream. */
#define MRHWENO_NOALLOC_SCRATCH_BYTES (32u << 20)
mrhweno_status mrhweno_residual_noalloc(const mrhweno_problem* prob, const void* moments_dev,
                                        void* residual_dev, void* flags_dev, void* hip_stream);

/* Rows per work item of the 2D stage kernel and grid size (0 = one work
 * group per work item) -- the launch shape the autotuner chooses. */
mrhweno_status mrhweno_set_launch(mrhweno_ctx* ctx, int rows_2d, int grid_2d);

/* Autotuner: time the 2D stage kernel (in its residual-only mode, which
 * leaves the state untouched) on the instances' current states for every
 * candidate launch shape -- rows per work item in rows_cand (n_rows
 * entries, each in [8, 4096]) and grid sizes in grid_cand (n_grid entries,
 * 0 = one work group per work item) -- with `reps` timed launches each, and
 * apply the fastest.  best_rows/best_grid/best_ms (host, may be NULL)
 * receive the choice and its mean launch time.  Synchronises. */
mrhweno_status mrhweno_autotune(mrhweno_ctx* ctx, const int* rows_cand, int n_rows,
                                const int* grid_cand, int n_grid, int reps,
                                int* best_rows, int* best_grid, float* best_ms);

/* Flag rows per work item of the 2D KXRCF pass (eq. (KXRCF_), Step 2.1):
 * 0 = the height chosen per problem from its size (the default), else a
 * value in [8, 256]; each work item covers 62 flag columns.  The flags do
 * not depend on it.  Synchronises the context's stream. */
mrhweno_status mrhweno_set_indicator_launch(mrhweno_ctx* ctx, int rows);

/* Autotuner of the 2D KXRCF pass: time the pass alone (one-off
 * evaluations that rewrite the first flag plane only, which every step
 * recomputes before it reads it; the state is untouched) for every
 * candidate height in rows_cand (n_rows entries, each 0 -- the height
 * chosen per problem -- or in [8, 256]) with
 * `reps` timed launches each, and apply the fastest.  Instances without a
 * KXRCF pass make it a no-op that keeps the current setting.
 * best_rows/best_ms (host, may be NULL) receive the choice and its mean
 * launch time.  Synchronises. */
mrhweno_status mrhweno_autotune_indicator(mrhweno_ctx* ctx, const int* rows_cand, int n_rows, int reps,
                                          int* best_rows, float* best_ms);

/* Run nsteps steps launched one kernel at a time (no graph) with HIP events
 * recorded on the context's stream between kernel classes, then
 * synchronise.  ms_out (host, 4 floats) receives the summed device time of
 * [0] wave-speed reductions and dt, [1] KXRCF face summaries and
 * learned-indicator inference, [2] KXRCF flags and the band fallback,
 * [3] stage kernels (reconstruction, fluxes, residual, RK combination);
 * launches_out (host, 4 ints, or NULL) the number of launches of each.
 * The state advances exactly as with mrhweno_step. */
mrhweno_status mrhweno_profile(mrhweno_ctx* ctx, int nsteps, float* ms_out, int* launches_out);

/* ------------------------------------------------------------------------
 * Learned troubled-cell indicator (2D Euler; an addition to the paper's
 * method, which uses KXRCF, eq. (KXRCF_), in Step 2.1).
 *
 * Features of a cell (MRHWENO_MLP_FEATURES = 320 BF16 values): the cell
 * average and first moments of rho, rho u, rho v, E on the 5 x 5 window of
 * cells around it, each minus (averages only) the cell's own average and
 * divided by the cell's rho, rho c (momenta; c = sound speed of the cell
 * average) or E; then log2(h)/16; then zeros.  Index f = 32 kb + 8 g + j
 * with slot s = 8 kb + j: s < 60 -> component s/15, moment (s/5)%3, window
 * offset (s%5 - 2, g - 2); 60 <= s < 75 -> component g, moment (s-60)/5,
 * offset ((s-60)%5 - 2, 2); s = 75 with g = 0 -> log2(h)/16.
 *
 * Network: z = W3 . relu(W2 relu(W1 x + b1) + b2) + b3, score sigmoid(z);
 * BF16 weights and activations, FP32 accumulation.  Parameter vector of
 * MRHWENO_MLP_PARAMS entries: W1 [64][320], b1 [64], W2 [64][64], b2 [64],
 * W3 [64], b3, 7 zeros (BF16 for inference, FP32 for the master copy and
 * the gradients).  The troubled-cell decision: score > band_hi flagged,
 * score < band_lo not flagged, otherwise KXRCF.
 * ------------------------------------------------------------------------ */
#define MRHWENO_MLP_FEATURES 320
#define MRHWENO_MLP_PARAMS 24776

/* Set the network of every LEARNED instance: params_dev is a device BF16
 * parameter vector (read before the call returns; the library keeps its own
 * copy), 0 <= band_lo <= band_hi <= 1 (0.2 and 0.8 by default).
 * Synchronises.  Steps and probes of LEARNED instances return
 * MRHWENO_ERR_NOT_READY until this has been called. */
mrhweno_status mrhweno_set_indicator(mrhweno_ctx* ctx, const void* params_dev,
                                     double band_lo, double band_hi);

/* The learned indicator once on a given state of a LEARNED instance:
 *   decision_dev  device uint8 [ny][nx]: 1 flagged, 0 not flagged, 2 left to
 *                 KXRCF (band), or NULL;
 *   flags_dev     device uint8 [ny][nx]: the final troubled-cell map, or NULL.
 * Synchronises. */
mrhweno_status mrhweno_indicator(mrhweno_ctx* ctx, int instance, const void* moments_dev,
                                 void* decision_dev, void* flags_dev);

/* Features of n cells of a 2D Euler instance from a given state:
 *   cells_dev  device int32 [n], interior cell indices j*nx + i;
 *   out_dev    device BF16 [n][MRHWENO_MLP_FEATURES].  Synchronises. */
mrhweno_status mrhweno_features(mrhweno_ctx* ctx, int instance, const void* moments_dev,
                                const int* cells_dev, int n, void* out_dev);

/* Training kernels (no context; asynchronous on the given hipStream_t).
 * All buffers are device memory owned by the caller. */
int mrhweno_mlp_param_count(void);     /* MRHWENO_MLP_PARAMS   */
int mrhweno_mlp_feature_count(void);   /* MRHWENO_MLP_FEATURES */
/* bytes of the activation cache of a batch of `batch` samples */
size_t mrhweno_mlp_cache_bytes(int batch);

/* C[m][n] = sum_k A[m][k] B[k][n] (M x N x K), BF16 A and B, FP32 C, each
 * addressed through its own row and column strides (in elements), on the
 * matrix cores with FP32 accumulation. */
mrhweno_status mrhweno_mlp_gemm(void* hip_stream, int M, int N, int K,
                                const void* A, long long sAm, long long sAk,
                                const void* B, long long sBk, long long sBn,
                                void* C, long long sCm, long long sCn);

/* Forward pass of a batch: x BF16 [batch][320], params BF16, cache of
 * mrhweno_mlp_cache_bytes(batch) bytes (holds the activations for the
 * backward pass), z FP32 [batch] logits. */
mrhweno_status mrhweno_mlp_forward(void* hip_stream, const void* x, const void* params,
                                   void* cache, void* z, int batch);

/* Backward pass of the mean binary cross-entropy of the logits of the last
 * forward pass on the same cache: labels FP32 [batch] in {0, 1}; grads FP32
 * [MRHWENO_MLP_PARAMS] (overwritten); loss FP32 [batch] per-sample loss. */
mrhweno_status mrhweno_mlp_backward(void* hip_stream, const void* x, const void* params,
                                    void* cache, const void* labels, void* grads,
                                    void* loss, int batch);

/* One Adam step (step >= 1) on the FP32 master parameters, m and v
 * moments (FP32), refreshing the BF16 copy params. */
mrhweno_status mrhweno_mlp_adam(void* hip_stream, void* master, void* params, const void* grads,
                                void* m, void* v, int step, float lr, float beta1,
                                float beta2, float eps);

/* Most recent error message (thread-local when ctx is NULL). */
const char* mrhweno_last_error(const mrhweno_ctx* ctx);

/* Release the context (does not free caller memory). */
void mrhweno_destroy(mrhweno_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* MRHWENO_H */
