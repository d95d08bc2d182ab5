/*
 * spff.h -- C ABI of the spectral phase-field fracture library for MI355X
 * (gfx950).
 *
 * The library solves the staggered quasi-static phase-field fracture problem
 * of Andrews & Pastewka, "Crack-path selection in phase-field models for
 * brittle fracture" (arXiv:2203.16467) on 2-D periodic grids:
 *   - mechanics: Fourier-Galerkin equilibrium with the strain as unknown,
 *     eps = eps_bar + eps*, Newton on eps* with conjugate gradients on the
 *     compatibility-projected tangent problem (Sec. 3.1.1);
 *   - phase field: Fourier-collocation Laplacian, bound-constrained
 *     conjugate gradients (Sec. 3.1.2, Algorithm 1);
 *   - one load step = alternating minimisation at a prescribed macroscopic
 *     strain until ||phi_n+1 - phi_n||_1 < Tol_AM (Sec. 3.2.1, Algorithm 2).
 * Constitutive choices: isotropic energy with h(phi) = (1-phi)^2, or the
 * strain-spectral split (Sec. 2.1); AT1 or AT2 local fracture energy;
 * crack-set or damage irreversibility (Sec. 2.1, constraint field).
 *
 * Conventions shared by every entry point
 *   - Grid: ny rows by nx columns, unit spacing, row-major [y][x] arrays.
 *     nx and ny are powers of two, 8 <= n <= 2048.
 *   - Tensors are stored as three planes (xx, yy, xy) of tensor components
 *     (the shear plane holds eps_xy, not the engineering strain).
 *   - "real" is float for precision SPFF_FP32 (fields stored and transformed
 *     in FP32, every dot product, norm and energy sum accumulated in FP64)
 *     and double for SPFF_FP64.  All device arrays passed in or out use the
 *     problem's real type.
 *   - Device pointers are HIP device addresses on the current device; the
 *     caller owns all of them.  The library never allocates device memory:
 *     every persistent and scratch array lives in the caller's workspace.
 *     It allocates small host-side handles and pinned host status buffers.
 *   - The stream argument is a hipStream_t passed as void* (NULL = the
 *     default stream).  All device work of a handle is enqueued on it; calls
 *     that return results synchronise that stream.
 *   - Return value: 0 = OK, > 0 = warning (results valid), < 0 = error;
 *     after an error the state of the handle is unchanged unless stated.
 *     spff_last_error() returns a thread-local message for the last non-OK
 *     status.
 *   - A handle is not thread-safe; use it from one thread at a time.
 */
#ifndef SPFF_H
#define SPFF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SPFF_OK = 0,
  SPFF_WARN_NOT_CONVERGED = 1, /* an iteration cap was hit; fields valid */
  SPFF_E_INVALID = -1,         /* bad argument / configuration / input field */
  SPFF_E_NOMEM = -2,           /* workspace too small */
  SPFF_E_DEVICE = -3,          /* HIP runtime error */
  SPFF_E_NONFINITE = -4,       /* a reduction produced NaN or Inf */
  SPFF_E_BUSY = -5             /* request still pending / no free slot */
} spff_status;

enum { SPFF_AT1 = 1, SPFF_AT2 = 2 };
/* Energy models (Sec. 2.1): isotropic, strain-spectral split, volumetric-
 * deviatoric split (plane strain: K = lambda + 2 mu/3, three-dimensional
 * deviator with zero out-of-plane strain, so every model is isotropic at
 * phi = 0).  `split` selects the crack driving force psi0+, `contact` the
 * stress; equal (or contact = SPFF_CONTACT_SAME) gives the variational
 * model, different values the non-variational pairings of Sec. 4.2.1 (e.g.
 * strain-spectral driving force with the stress-free isotropic contact). */
enum { SPFF_SPLIT_NONE = 0, SPFF_SPLIT_SPECTRAL = 1, SPFF_SPLIT_VOLDEV = 2 };
enum { SPFF_CONTACT_SAME = -1 };
/* Evolution method of a load step (Sec. 3.2): alternating minimisation
 * (Algorithm 2), one iteration of the time-discretized evolution
 * (Algorithm 3) or one iteration of the near-equilibrium evolution
 * (Algorithm 4). */
enum { SPFF_EVOL_AM = 0, SPFF_EVOL_TIME = 1, SPFF_EVOL_NEAR_EQ = 2 };
enum { SPFF_IRR_CRACK_SET = 0, SPFF_IRR_DAMAGE = 1 };
/* Nyquist modes of the strain fluctuation on even grids (the paper uses odd
 * grids, which have none).  ZERO: the gradient component along a Nyquist
 * direction is zero, so those strain components are absent.  FREE: modes
 * with a Nyquist index are unconstrained by the projection (G^ = identity
 * there): laminates are exact again and a pixel-wide crack can open, as on
 * an odd grid. */
enum { SPFF_NYQ_ZERO = 0, SPFF_NYQ_FREE = 1 };
enum { SPFF_FP32 = 0, SPFF_FP64 = 1 };

/* Field selection bits for spff_get_fields, in output order. */
enum {
  SPFF_FIELD_PHI = 1u << 0,      /* phase field phi, 1 plane */
  SPFF_FIELD_PHI_REF = 1u << 1,  /* irreversibility reference: phi at the start
                                    of the last load step, 1 plane */
  SPFF_FIELD_STRAIN = 1u << 2,   /* total strain eps_bar + eps*, 3 planes */
  SPFF_FIELD_STRESS = 1u << 3,   /* stress sigma(eps, phi), 3 planes */
  SPFF_FIELD_PSI_PLUS = 1u << 4, /* crack driving energy psi0+(eps), 1 plane */
  SPFF_FIELD_EPS_STAR = 1u << 5, /* strain fluctuation eps*, 3 planes */
  SPFF_FIELD_DISP = 1u << 6      /* periodic displacement fluctuation u*, 2 planes (x, y): the
                                    zero-mean field with sym(grad u*) = eps* (Sec. 3.1.1 solves
                                    for the strain; u* is recovered mode by mode, and is zero on
                                    modes whose gradient wavevector vanishes); the total
                                    displacement is eps_bar . x + u* */
};

/* Problem configuration (Sec. 2.1, 3.1, 3.2.1; defaults from
 * spff_default_config). */
typedef struct spff_config {
  int32_t nx, ny;          /* grid, powers of two in [8, 2048] */
  int32_t at;              /* SPFF_AT1 (w = phi, c_w = 8/3) or SPFF_AT2 (w = phi^2, c_w = 2) */
  int32_t split;           /* crack driving force model: SPFF_SPLIT_NONE (isotropic), _SPECTRAL, _VOLDEV */
  int32_t irreversibility; /* SPFF_IRR_CRACK_SET or SPFF_IRR_DAMAGE */
  int32_t precision;       /* SPFF_FP32 or SPFF_FP64 */
  double nu;               /* Poisson ratio, -1 < nu < 0.5 (plane strain) */
  double ell;              /* regularisation length in pixels, > 0 */
  double gc;               /* critical energy release rate, > 0 */
  double crack_set_threshold; /* crack-set constraint: phi_ref >= threshold (0.9) */
  double k_res;            /* residual stiffness added to h(phi); 0 in the paper */
  double eta_over_dt;      /* viscous term eta/dt; 0 = alternating minimisation */
  double tol_mech, tol_abs_mech; /* mechanics: ||G[sigma]|| <= tol*max(||sigma_hom||,||R0||) + tol_abs */
  double tol_pf, tol_abs_pf;     /* phase field: ||r|| <= tol*max(||b||,||r0||) + tol_abs */
  double tol_am;           /* AM stop: sum |phi_n+1 - phi_n| < tol_am (pixel units); <0: 1e-3 ell^2 */
  int32_t max_cg, max_newton, max_bccg, max_am; /* iteration caps */
  int32_t ticks_per_sync;  /* solver ticks enqueued between host status checks (>= 1) */
  int32_t use_graph;       /* 1: replay the tick block as a captured HIP graph */
  /* Attainable-accuracy floor (not in the paper): a residual evaluated in the
   * working precision u carries rounding noise of about u sqrt(log2(nx ny))
   * times the norm of the terms it is computed from, so a sub-solve also
   * stops when ||residual|| <= floor_factor u sqrt(log2(nx ny)) *
   * (||sigma|| for mechanics; ||d phi|| + kappa <|2 pi q|^2> ||phi|| + ||b||
   * for the phase field, <.> the mean over the grid's modes).  0 disables it.
   * Irrelevant in FP64 at the default tolerances; what lets FP32 solves
   * terminate instead of iterating on rounding noise. */
  double floor_factor;
  int32_t stall_iters;     /* BCCG stops when its residual has not improved for this many iterations (0: off) */
  /* Launch-plan overrides for every bucket of active problems (0 = the
   * built-in heuristic; set by the autotuner): rows per row-FFT work-group,
   * columns per column-FFT work-group (powers of two), threads per
   * work-group (64, 128 or 256; threads * 8 >= max(nx/2, ny)). */
  int32_t plan_rows, plan_cols, plan_threads;
  int32_t contact;         /* stress (contact) model: SPFF_SPLIT_* or SPFF_CONTACT_SAME (default: = split) */
  /* Evolution (Sec. 3.2).  SPFF_EVOL_AM: a load step is Algorithm 2 at
   * eta_over_dt.  SPFF_EVOL_TIME: a load step is one iteration n of
   * Algorithm 3 at the given eps_bar: elasticity at phi_n, then the phase
   * field with the viscous term eta/dt and phi_con(phi_n), dt halved until
   * ||phi_n+1 - phi_n||_1 < dphi_max or dt <= dt_min and doubled (up to
   * dt_max) after a change below dphi_max/2; dt persists between steps
   * (initially dt_max).  The step's stats report dt and whether Algorithm 3
   * increments the load (dphi < dphi_min and dt >= dt_max); the caller adds
   * the strain increment then. */
  int32_t evolution;       /* SPFF_EVOL_AM, SPFF_EVOL_TIME or SPFF_EVOL_NEAR_EQ */
  double eta;              /* viscosity eta >= 0 (SPFF_EVOL_TIME) */
  double dt_max, dt_min;   /* 0 < dt_min <= dt_max */
  double dphi_max, dphi_min; /* bounds on ||phi_n+1 - phi_n||_1 (pixel units) */
  /* SPFF_EVOL_NEAR_EQ (Sec. 3.2.2, Algorithm 4): a load step is one
   * iteration n at the given eps_bar: elasticity at phi_n; if
   * max(-F_phi(phi_n, eps_n)) > fphi_max and the trigger flag is set (set
   * once max(-h'(phi_n) psi0+) > drive_threshold together with the first
   * condition, kept afterwards), eps* and eps_bar are scaled by
   * g = sqrt((fphi_max - [-F_phi + h' psi0+](x*)) / (-h' psi0+)(x*)) at the
   * first maximiser x* of -F_phi (row-major), g <= 1 + deps_max /
   * max|eps_bar|; then the phase field with phi_con(phi_n) and the viscous
   * term eta/dt_max.  Stats report g, the largest -F_phi before scaling, the
   * scaled eps_bar, the flag and advance = ||phi_n+1 - phi_n||_1 <
   * dphi_min (the caller then adds its increment to the returned eps_bar).
   * Uses eta, dt_max and dphi_min above. */
  double fphi_max;         /* bound on -F_phi, > 0 */
  double drive_threshold;  /* trigger threshold on -h'(phi) psi0+, >= 0 */
  double deps_max;         /* max |component| of the load increment, >= 0 */
  int32_t nyquist;         /* SPFF_NYQ_ZERO (default) or SPFF_NYQ_FREE (even grids) */
} spff_config;

/* Per-problem result of one load step (Sec. 3.2.1 quantities). */
typedef struct spff_step_stats {
  int32_t status;          /* spff_status of this problem's step */
  int32_t am_iters;        /* alternating-minimisation iterations */
  int32_t newton_iters;    /* mechanics Newton steps (sum over AM iterations) */
  int32_t cg_iters;        /* mechanics CG iterations (sum) */
  int32_t bccg_iters;      /* phase-field BCCG iterations (sum) */
  int32_t ticks;           /* solver ticks the step took */
  double dphi_l1;          /* last ||phi_n+1 - phi_n||_1 */
  double mech_residual;    /* last ||G[sigma]||_2 */
  double pf_residual;      /* last BCCG ||r||_2 */
  double F_e, F_f;         /* elastic and fracture energy (pixel area 1) */
  double sigma_bar[3];     /* mean stress (xx, yy, xy) */
  double C_bar;            /* sigma_bar_ij / eps_bar_ij at the largest |eps_bar_ij| */
  double phi_max, phi_mean;
  int64_t crack_px;        /* pixels with phi > 0.9 */
  double wall_ms;          /* host wall time from enqueueing the step to observing its end */
  double dt;               /* SPFF_EVOL_TIME: dt for the next step */
  int32_t halvings;        /* SPFF_EVOL_TIME: dt halvings in this step */
  int32_t advance;         /* SPFF_EVOL_TIME / _NEAR_EQ: 1 if the algorithm increments the load now */
  double gamma;            /* SPFF_EVOL_NEAR_EQ: strain scaling factor of the step (1: none) */
  double fphi_max;         /* SPFF_EVOL_NEAR_EQ: largest -F_phi(phi_n, eps_n) before scaling */
  double eps_bar[3];       /* macroscopic strain at the end of the step (xx, yy, xy) */
  int32_t ne_flag;         /* SPFF_EVOL_NEAR_EQ: trigger flag after the step */
  int32_t reserved;
} spff_step_stats;

typedef struct spff_problem spff_problem; /* opaque: a batch of 1..B problems */

/* Fill *cfg with defaults: 64x64, AT1, spectral split, crack-set (0.9),
 * FP32, nu 0.2, ell 2, gc 1, tolerances 1e-6, tol_am -1 (1e-3 ell^2),
 * caps cg 20000 / newton 50 / bccg 20000 / am 1000, ticks_per_sync 1,
 * use_graph 0, floor_factor 2, stall_iters 200. */
void spff_default_config(spff_config* cfg);

/* Workspace bytes for a batch of nbatch problems with this configuration
 * (resident state + solver scratch + FFT tables + control blocks). */
spff_status spff_workspace_bytes(const spff_config* cfg, int32_t nbatch, size_t* bytes);

/* Create a batch of nbatch independent problems sharing cfg.
 *   E_dev:        device, real[nbatch][ny][nx], Young's modulus (> 0, finite);
 *                 copied into the workspace (the caller may free it after).
 *   phi_init_dev: device, real[nbatch][ny][nx] in [0,1] or NULL (phi = 0).
 *                 If given, the phase field is first solved at zero strain
 *                 with phi_con(phi_init) (Algorithm 2, first two lines).
 *   workspace:    device, >= spff_workspace_bytes bytes, 256-byte aligned,
 *                 owned by the caller and kept alive until destroy.
 * Errors: SPFF_E_INVALID (config or E/phi_init values), SPFF_E_NOMEM
 * (workspace too small), SPFF_E_DEVICE. */
spff_status spff_create_batch(const spff_config* cfg, int32_t nbatch, const void* E_dev,
                              const void* phi_init_dev, void* workspace, size_t workspace_bytes,
                              void* stream, spff_problem** out);

/* spff_create_batch with nbatch = 1. */
spff_status spff_create_problem(const spff_config* cfg, const void* E_dev, const void* phi_init_dev,
                                void* workspace, size_t workspace_bytes, void* stream,
                                spff_problem** out);

/* One load step (Algorithm 2 at macroscopic strain eps_bar) for every
 * problem of the batch.
 *   eps_bar: host, double[nbatch][3] (xx, yy, xy).
 *   stats:   host, spff_step_stats[nbatch] or NULL.
 * Returns the worst per-problem status (errors before warnings).  Blocks
 * until the step has finished on the device. */
spff_status spff_load_step_batch(spff_problem* p, const double* eps_bar, spff_step_stats* stats);

/* Independent load-step sequences: problem b runs its own nsteps steps at
 * eps_bar[b][0..nsteps-1][3] (host, double[nbatch][nsteps][3]); a problem
 * that finishes a step starts its next one at the following status check
 * without waiting for the others (problems never synchronise with each
 * other).  stats: host spff_step_stats[nbatch][nsteps] or NULL.  Returns the
 * worst status over all steps; blocks until every sequence is done. */
spff_status spff_run_sequence(spff_problem* p, int32_t nsteps, const double* eps_bar, spff_step_stats* stats);

/* Time-discretized or near-equilibrium evolution (Sec. 3.2.2, Algorithms 3
 * and 4) driven on the device: problem b runs nsteps iterations; iteration
 * j runs at eps_bar_j = eps_bar_{j-1} + advance_{j-1} deps[b][j], where
 * eps_bar_{j-1} is the previous iteration's final macroscopic strain (scaled
 * by the near-equilibrium rescaling) and advance_{j-1} its advance flag
 * (the problem's last step before this call; 0 strain and advance = 1 for a
 * fresh or reset problem).  deps: host, double[nbatch][nsteps][3], the load
 * increment of each iteration (constant Delta eps_bar in the paper).
 * stats: host spff_step_stats[nbatch][nsteps] or NULL.  Errors:
 * SPFF_E_INVALID if cfg.evolution is SPFF_EVOL_AM (use spff_run_sequence)
 * or an increment is not finite; otherwise as spff_run_sequence. */
spff_status spff_run_evolution(spff_problem* p, int32_t nsteps, const double* deps, spff_step_stats* stats);

/* spff_load_step_batch for a problem created with nbatch = 1. */
spff_status spff_load_step(spff_problem* p, const double eps_bar[3], spff_step_stats* stats);

/* Copy fields of problem `index` (0..nbatch-1), or of all problems when
 * index = -1 (then each output is real[nbatch][planes][ny][nx]), into caller
 * device buffers: dst[i] receives the i-th field selected by mask, in the
 * bit order of the SPFF_FIELD_* enum.  Synchronises the stream. */
spff_status spff_get_fields(spff_problem* p, int32_t index, uint32_t mask, void* const* dst);

/* State = (eps*[3], phi, phi_ref) planes: real[nbatch][5][ny][nx] on the
 * device, plus the macroscopic strain of the last step (host double[nbatch][3],
 * may be NULL).  get copies out, set copies in; set checks that every value
 * (and eps_bar) is finite and fails with SPFF_E_INVALID, state unchanged,
 * otherwise (no other validation of values is made). */
size_t spff_state_bytes(const spff_problem* p);
spff_status spff_get_state(spff_problem* p, void* dst_dev, double* eps_bar_host);
spff_status spff_set_state(spff_problem* p, const void* src_dev, const double* eps_bar_host);

/* Spectral operators of the solver applied to caller fields of every problem
 * of the batch, with the solver's own FFT kernels and the handle's scratch
 * (not while a step runs):
 *   SPFF_OP_PROJECT       out = G[in]: the compatibility projection of
 *                         Sec. 3.1.1 (orthogonal projector onto compatible,
 *                         zero-mean strain fields); in/out
 *                         real[nbatch][3][ny][nx] (xx, yy, xy planes)
 *   SPFF_OP_NEG_LAPLACIAN out = -lap_N in, the collocation Laplacian of
 *                         Sec. 3.1.2 (true |2 pi q|^2 at Nyquist); in/out
 *                         real[nbatch][ny][nx]
 *   SPFF_OP_DISPLACEMENT  out = u*: the zero-mean periodic displacement
 *                         whose symmetric gradient is the compatible part of
 *                         in (the displacement of SPFF_FIELD_DISP); in
 *                         real[nbatch][3][ny][nx] (xx, yy, xy), out
 *                         real[nbatch][2][ny][nx] (x, y)
 * in and out are device buffers owned by the caller and may alias.
 * Synchronises the stream.  Errors: SPFF_E_INVALID (unknown op, NULL
 * buffers), SPFF_E_BUSY (a step is running), SPFF_E_DEVICE. */
enum { SPFF_OP_PROJECT = 0, SPFF_OP_NEG_LAPLACIAN = 1, SPFF_OP_DISPLACEMENT = 2 };
spff_status spff_apply_operator(spff_problem* p, int32_t op, const void* in_dev, void* out_dev);

/* Kernel profiling.  A tick is three kernels: row-forward FFT (which first
 * runs the controller step of the previous tick), column FFT and
 * row-inverse FFT; a block of ticks ends with a closing controller kernel.
 * While enabled, every work-group of the three FFT kernels stamps its first
 * and last device wall-clock reading, and an extra work-group of the next
 * tick's column kernel (the closing kernel, for a block's last tick)
 * accumulates per FFT kernel
 *   kernel_ms       its activity: first work-group start to last end;
 *   kernel_span_ms  its span: first start to the first start of the next
 *                   kernel (activity plus the dead time of its drain,
 *                   end-of-kernel write-back and the next dispatch);
 * a profiler's kernel trace, which also counts dispatch and write-back,
 * falls between the two.  Works inside captured graphs, without host
 * events; index 3 stays zero.  The controller step also accumulates each
 * kernel's algorithmic HBM bytes for the phase every problem executed
 * (inputs read once, outputs written once, half spectra round-tripped).
 * Enabling resets the totals. */
typedef struct spff_profile {
  double kernel_ms[4];       /* summed activity per kernel */
  int64_t launches[4];       /* launches per kernel */
  double alg_bytes[4];       /* summed algorithmic bytes per kernel */
  int64_t ticks;
  double kernel_span_ms[4];  /* summed span per kernel */
} spff_profile;
spff_status spff_profile_enable(spff_problem* p, int32_t enable);
spff_status spff_profile_read(spff_problem* p, spff_profile* out);

/* Launch plans of the three FFT kernels, one per bucket of active problems
 * (the launch covers a power-of-two number of problem slots: bucket i has
 * min(2^i, nbatch) slots).  The handle starts with a built-in heuristic
 * plan per bucket; an autotuner may time alternatives and install the
 * fastest.  Plans change launch shapes and the grouping of the FP64 partial
 * sums (so results by rounding only), never the arithmetic.
 *   row_kind / col_kind: SPFF_FFT_LDS -- Stockham radix-4/2 passes through
 *     LDS, one point pair per thread (any size); SPFF_FFT_REG -- radix-8
 *     Stockham on registers, 8 points per lane (16 for 2048-point rows,
 *     and for 1024- and 2048-point columns a plan may ask for 16 -- see
 *     col_threads), wavefront-local LDS exchanges (a column of more than 64
 *     lanes spans the wavefronts of its work-group) (FP32 only; rows:
 *     128 <= nx <= 2048, columns: ny in {128, 256, 512, 1024, 2048});
 *     SPFF_FFT_REG4 (rows only) -- 4 points per lane and radix-4 passes
 *     (twice the lanes per row, for launches with few problems;
 *     128 <= nx <= 512).
 *   rows / cols: rows per row work-group, columns per column work-group
 *     (powers of two).
 *   row_threads / col_threads: threads per work-group for the LDS kind
 *     (64, 128 or 256, times 8 covering the transform); for the register
 *     kinds derived as rows * (lanes per row: nx/16, nx/32 for nx = 2048,
 *     nx/8 for SPFF_FFT_REG4) and cols * (lanes per column), which must be
 *     a power of two in [64, 256] -- filled in on return.  Lanes per
 *     column: ny/8; for ny = 1024 or 2048 that holds only with cols = 1
 *     and col_threads = ny/8 as given (the built-in plans), any other
 *     plan takes ny/16 (16 points per lane; cols = 1 for ny = 2048). */
enum { SPFF_FFT_LDS = 1, SPFF_FFT_REG = 2, SPFF_FFT_REG4 = 3 };
typedef struct spff_plan {
  int32_t row_kind, rows, row_threads;
  int32_t col_kind, cols, col_threads;
} spff_plan;
/* Number of buckets and their slot counts (sizes may be NULL). */
spff_status spff_plan_buckets(const spff_problem* p, int32_t* count, int32_t* sizes);
/* The plan in use for bucket `bucket`. */
spff_status spff_get_plan(const spff_problem* p, int32_t bucket, spff_plan* out);
/* Install a plan for bucket `bucket` (NULL restores the heuristic).  The
 * plan is validated (SPFF_E_INVALID on a bad plan, state unchanged) and the
 * bucket's captured graph is dropped.  Synchronises the stream. */
spff_status spff_set_plan(spff_problem* p, int32_t bucket, spff_plan* plan);

/* Number of problems, grid and precision of a handle. */
spff_status spff_problem_info(const spff_problem* p, int32_t* nbatch, int32_t* nx, int32_t* ny,
                              int32_t* precision);

/* Release the host handle (the caller frees the workspace). */
spff_status spff_destroy_problem(spff_problem* p);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of load-step requests over resident problems.
 *
 * A server owns a caller-provided device arena.  Each registered problem keeps
 * its resident state there (E, phi, phi_ref, eps*: 6 planes) for the life of
 * the server.  Problems are grouped in size classes (nx, ny, precision); each
 * class has one solver engine with a fixed number of scratch slots (12 planes
 * each: CG/BCCG vectors and half spectra) on its own stream, so classes run
 * concurrently on the device.  The scratch budget sets the slot counts
 * (admission by HBM footprint).  A request is one load step (Algorithm 2) of
 * one problem; requests of one problem run in submission order, one at a time.
 * spff_server_progress admits queued requests into free slots between tick
 * blocks, so requests that arrive while others run join the batch as slots
 * free up (their work overlaps on the device).  A problem's result does not
 * depend on what else runs (fixed-order reductions); with fixed launch-plan
 * overrides it is bitwise identical to running the problem alone.
 * ------------------------------------------------------------------------- */
typedef struct spff_server spff_server;

/* arena_dev: device memory owned by the caller (256-byte aligned), used for
 * resident state and class engines.  scratch_budget_bytes: upper bound on
 * engine scratch over all classes (0 = no bound beyond the arena).
 * ticks_per_sync / use_graph as in spff_config.  Each size class creates
 * its own non-blocking stream of default priority. */
spff_status spff_server_create(void* arena_dev, size_t arena_bytes, size_t scratch_budget_bytes,
                               int32_t ticks_per_sync, int32_t use_graph, spff_server** out);

/* Register a problem (copies E, real[ny][nx] on the device, into the arena;
 * phi = eps* = 0).  cfg->nx, ny, precision pick the class; the physical,
 * solver and evolution fields are per problem (a request is one load step
 * of cfg->evolution; the time step of Algorithm 3 and the trigger flag of
 * Algorithm 4 are kept per problem between its requests, whatever slot
 * serves them).  Fails with SPFF_E_NOMEM when the arena is full.  Problems
 * may be registered while others run. */
spff_status spff_server_register(spff_server* sv, const spff_config* cfg, const void* E_dev, int32_t* id);

/* Queue one load step of problem id at eps_bar (host double[3]). */
spff_status spff_server_submit(spff_server* sv, int32_t id, const double eps_bar[3], uint64_t* ticket);

/* Drive the device: up to max_rounds rounds of (admit, launch one tick block
 * per busy class, collect finished requests).  *completed receives the number
 * of requests finished during the call, *pending the number still queued or
 * running. */
spff_status spff_server_progress(spff_server* sv, int32_t max_rounds, int32_t* completed, int32_t* pending);

/* Result of a request: SPFF_OK and *out filled when done (wall_ms = submit to
 * completion), SPFF_E_BUSY while pending, SPFF_E_INVALID for an unknown or
 * already collected ticket. */
spff_status spff_server_poll(spff_server* sv, uint64_t ticket, spff_step_stats* out);

/* Resident fields of a problem (mask of SPFF_FIELD_PHI, SPFF_FIELD_PHI_REF,
 * SPFF_FIELD_EPS_STAR) into caller device buffers; only between requests of
 * that problem (SPFF_E_BUSY otherwise). */
spff_status spff_server_get_fields(spff_server* sv, int32_t id, uint32_t mask, void* const* dst);

/* Scratch slots per class and bytes used in the arena. */
spff_status spff_server_info(const spff_server* sv, int32_t* nclasses, int32_t* total_slots, size_t* arena_used);

spff_status spff_server_destroy(spff_server* sv);

/* ---------------------------------------------------------------------------
 * Allocation-free load step, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * allocation).  One load step (Algorithm 2 at macroscopic strain eps_bar,
 * as spff_load_step) of one problem whose state lives in caller buffers;
 * every solver scratch array (control block, parameters, FFT twiddles,
 * partial sums, CG / BCCG vectors, half spectra) lives in a static device
 * array of SPFF_STATIC_SCRATCH_BYTES owned by the library: one per device,
 * allocated with the library's code on that device and held until the
 * process ends.  The call allocates no device or pinned memory and builds
 * no graph (use_graph is ignored); it launches kernels, copies and a memset
 * on `stream` and synchronises it.
 *   cfg:       as spff_create_problem; evolution must be SPFF_EVOL_AM.  The
 *              scratch a grid needs is about 12 real planes plus partial
 *              sums: FP32 up to 1024 x 1024, FP64 up to 1024 x 512 fit.
 *   E_dev:     device, real[ny][nx], Young's modulus (> 0, finite).
 *   state_dev: device, real[5][ny][nx] = (eps*[3], phi, phi_ref), the
 *              layout of spff_get_state for one problem; read as the state
 *              before the step and overwritten with the state after it.
 *              phi and phi_ref must lie in [0, 1].
 *   eps_bar:   host, double[3] (xx, yy, xy).
 *   stats:     host, one spff_step_stats, or NULL.
 * Errors: SPFF_E_INVALID (configuration, NULL pointers, E or phi out of
 * range, a grid whose scratch exceeds SPFF_STATIC_SCRATCH_BYTES -- checked
 * before any device work), SPFF_E_DEVICE.  The scratch keeps the last
 * call's contents; every value a step reads is written first in that step.
 * All calls on one device share its scratch: calls that overlap on one
 * device (other threads, other streams) race and must be serialised by the
 * caller. */
#define SPFF_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
spff_status spff_load_step_static(const spff_config* cfg, const void* E_dev, void* state_dev,
                                  const double eps_bar[3], spff_step_stats* stats, void* stream);

/* Thread-local message for the last non-OK status ("" if none). */
const char* spff_last_error(void);

/* Library version string. */
const char* spff_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SPFF_H */
