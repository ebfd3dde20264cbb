/*
 * nn4mg — multigrid pressure solve on MI355X (gfx950).
 *
 * The operation is the implicit pressure step of Chen et al., arXiv 2401.06755:
 * the discretised pressure-Poisson residual of Eq. (ph_disc) / Eq. (ph_disc2)
 * (Sec. 2.4, Stages 1 and 3) is driven to zero by a sawtooth multigrid cycle
 * laid out as a U-Net (Fig. multi-grid): restriction of the residual on the
 * way down, an exact solve at the bottom, trilinear prolongation and weighted
 * Jacobi smoothing on the way up, with the boundary conditions applied at every
 * level (Sec. 2.3.3).  The operator is the linear-element (Q1) Laplacian filter
 * w_lap (27 points: centre 8h/3, faces 0, edges -h/6, corners -h/12), either
 * with a constant coefficient or with a nodal coefficient k (= 1/rho) through
 * the identity of Eq. (k-T), Sec. 2.2.4.
 *
 * Conventions shared by every entry point:
 *  - Fields are device arrays of nx*ny*nz values, x fastest:
 *    idx = i + nx*(j + ny*k).  Cells are centred at ((i+1/2)h, (j+1/2)h, (k+1/2)h).
 *  - Right-hand sides are volume-integrated, as the filter weights are: b is
 *    used as given, and the relative residual ||b - A x||_2 / ||b||_2 is
 *    scale-free.
 *  - All device work is enqueued on the HIP stream given at setup.  Calls that
 *    return host values synchronise that stream before returning.
 *  - Every function returns NN4MG_OK (0) or a negative status; nothing throws
 *    across this boundary.  nn4mg_last_error() gives a message for the last
 *    failure on the calling thread.
 *  - The caller owns every pointer it passes; the library owns the hierarchy
 *    (coarse levels, reduced-precision copies, workspaces, coarsest inverse).
 */
#ifndef NN4MG_H
#define NN4MG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nn4mg_hier *nn4mg_t;

enum nn4mg_status {
    NN4MG_OK = 0,
    NN4MG_EINVAL = -1,     /* bad configuration or argument */
    NN4MG_ENOMEM = -2,     /* device or host allocation failed */
    NN4MG_EDEVICE = -3,    /* a HIP call failed */
    NN4MG_ENOTCONV = -4,   /* max_cycles reached before rtol; x is valid */
    NN4MG_EBREAKDOWN = -5, /* non-finite residual, residual above 1e3 x the first (divergence), or
                              p.Ap <= 0 in flexible CG; x holds the last iterate */
    NN4MG_EBUSY = -6       /* server: request not admissible now */
};

/* Homogeneous boundary rules applied through the one-cell halo (Sec. 2.3.3):
 * DIRICHLET0 halo = -mirror (zero value on the cell face), NEUMANN0 halo =
 * +mirror (zero normal derivative), PERIODIC halo = wrap.  The coefficient k is
 * always continued by +mirror (wrap for periodic). */
enum { NN4MG_BC_DIRICHLET0 = 0, NN4MG_BC_NEUMANN0 = 1, NN4MG_BC_PERIODIC = 2 };

/* CONST: A = f(.; w_lap).  NODAL: A x = 1/2 [f(k.x) + k.f(x) - x.f(k)], Eq. (k-T). */
enum { NN4MG_COEF_CONST = 0, NN4MG_COEF_NODAL = 1 };

/* FP64: every step in double.
 * FP32_SMOOTH: FP64 residual (FP64 k), FP64 coarsest solve and FP64 update
 *   x += e; the V-cycle on the correction runs in FP32 with an FP32 copy of k.
 * FP16_COEF: as FP32_SMOOTH but the smoothing coefficient copy is stored in
 *   FP16 (arithmetic still FP32). */
enum { NN4MG_PREC_FP64 = 0, NN4MG_PREC_FP32_SMOOTH = 1, NN4MG_PREC_FP16_COEF = 2 };

/* Outer iteration: STATIONARY repeats the cycle (x <- x + V(b - A x));
 * FCG runs flexible conjugate gradients (FCG(1)) in FP64 with one cycle from
 * zero as the preconditioner; it needs at least two levels (EINVAL otherwise)
 * and four extra FP64 fields of the finest size.  With FCG, info->cycles
 * counts CG iterations (one preconditioning cycle each, plus one at the start). */
enum { NN4MG_OUTER_STATIONARY = 0, NN4MG_OUTER_FCG = 1 };

typedef struct {
    int nx, ny, nz;   /* interior cells of the finest level, each >= 1 */
    double h;         /* uniform spacing (> 0) */
    int bc[6];        /* x-lo, x-hi, y-lo, y-hi, z-lo, z-hi */
    int coef_mode;    /* NN4MG_COEF_* */
    int precision;    /* NN4MG_PREC_* */
    int nu_post;      /* Jacobi sweeps after each prolongation (default 2, >= 1) */
    double omega;     /* Jacobi weight (default 2/3) */
    int min_coarse;   /* coarsen while every dim is even and the smallest > min_coarse (default 4) */
    int outer;        /* NN4MG_OUTER_* (default STATIONARY) */
    int coarse_avg;   /* 0: coarse k = mean of the 8 children; 1: harmonic mean */
    int reserved[7];  /* must be zero */
} nn4mg_config;

#define NN4MG_HIST_MAX 512

typedef struct {
    int cycles;        /* cycles (outer iterations) performed */
    int status;        /* same as the return value of nn4mg_solve */
    double relres0;    /* ||b - A x0|| / ||b|| */
    double relres;     /* final relative residual (FP64 operator) */
    int hist_len;      /* min(cycles + 1, NN4MG_HIST_MAX) */
    double hist[NN4MG_HIST_MAX]; /* relative residual before each cycle, then the final one */
    double solve_ms;   /* wall time of the call (host clock) */
} nn4mg_info;

/* Fill cfg with the defaults above for an nx x ny x nz grid of spacing h, all
 * walls Dirichlet-zero, constant coefficient, FP64. */
void nn4mg_config_default(nn4mg_config *cfg, int nx, int ny, int nz, double h);

/* Device bytes nn4mg_setup will allocate for cfg (0 if cfg is invalid). */
size_t nn4mg_bytes_required(const nn4mg_config *cfg);

/* Build the level hierarchy (Fig. multi-grid; boundary rules at every level,
 * Sec. 2.3.3).  Levels: halve while all dims are even and the smallest exceeds
 * cfg->min_coarse.  Coarse operators are the same filter at h_l = 2^l h with k
 * averaged over the 8 children.  The coarsest matrix (<= 512 unknowns) is
 * assembled, factorised and inverted on the host in FP64.
 *   k_dev: nx*ny*nz device doubles, > 0, required iff coef_mode == NODAL; it
 *          is copied, so the caller may free it after the call returns.
 *   hip_stream: a hipStream_t (NULL = the null stream).
 * Errors: EINVAL (dims < 1, h <= 0, bad enum, coarsest level too large, NULL
 * k for NODAL or non-positive k), ENOMEM, EDEVICE. */
int nn4mg_setup(const nn4mg_config *cfg, const double *k_dev, void *hip_stream, nn4mg_t *out);

/* Replace the coefficient (same shape) and rebuild the coarse levels and the
 * coarsest inverse, as each time step of the paper's scheme changes rho
 * (Eq. rho).  Errors: EINVAL (CONST handle, NULL, non-positive k), EDEVICE. */
int nn4mg_update_coef(nn4mg_t h, const double *k_dev);

/* r = b - A x on the finest level, in FP64 (the residual of Eq. ph_disc).
 *   x_dev, b_dev: nx*ny*nz device doubles.
 *   r_dev: nx*ny*nz device doubles, or NULL (not written).
 *   norm2_out: host double receiving ||r||_2, or NULL (then no sync).
 * b is used as given (no projection, even for singular problems). */
int nn4mg_residual(nn4mg_t h, const double *x_dev, const double *b_dev, double *r_dev, double *norm2_out);

/* nn4mg_residual without a hierarchy and without any device allocation, for
 * callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same kernel and launch shape as
 * nn4mg_residual on a hierarchy set up from cfg, so r and the norm are the same.
 *   cfg: as for nn4mg_setup (validated the same way).
 *   k_dev: nx*ny*nz device doubles (> 0, not checked) iff coef_mode == NODAL;
 *          read in place (not copied); ignored for CONST.
 *   x_dev, b_dev, r_dev, norm2_out: as for nn4mg_residual.
 *   hip_stream: the hipStream_t to enqueue on (NULL = the null stream); with
 *          norm2_out the call synchronises it.
 * The per-workgroup norm partials live in a static device array of 2 MiB that
 * each GPU holds until the process ends (at most 262144 residual workgroups,
 * about 8.6e9 cells at the default launch shape; larger grids get EINVAL when
 * a norm is asked for).  Calls on one GPU share that array: calls that overlap
 * on one GPU (several host threads or streams) race on it.
 * Errors: EINVAL (bad cfg, NULL x/b, NULL k for NODAL, too many workgroups),
 * EDEVICE. */
int nn4mg_residual_noalloc(const nn4mg_config *cfg, const double *k_dev, const double *x_dev, const double *b_dev,
                           double *r_dev, double *norm2_out, void *hip_stream);


/* One outer iteration on x: FP64 precision: x <- V(x, b), one sawtooth
 * V(0, nu_post) cycle; reduced precisions: x <- x + V32(0, b - A x).  b is used
 * as given.  No norm, no projection; for parity checks of a single cycle. */
int nn4mg_vcycle(nn4mg_t h, const double *b_dev, double *x_dev);

/* Solve A x = b.  x_dev holds the initial guess and receives the solution.
 * Before each cycle the relative residual ||b - A x|| / ||b|| is taken in
 * FP64; the solve stops when it is <= rtol (fixed_cycles == 0) or after
 * max_cycles cycles (fixed_cycles == 1 runs exactly max_cycles, the paper's
 * fixed count of 20 per pressure solve, Sec. 2.4).  Singular problems (no
 * Dirichlet face): b is projected to zero mean for the solve and x is
 * returned with zero mean.  If ||b|| == 0, x is set to 0.
 * Returns OK, ENOTCONV (x valid), EBREAKDOWN, EINVAL (max_cycles < 0), EDEVICE.
 * info (may be NULL) receives the history. */
int nn4mg_solve(nn4mg_t h, const double *b_dev, double *x_dev, double rtol, int max_cycles, int fixed_cycles,
                nn4mg_info *info);

/* Number of levels and their dims (dims must hold 3*max_levels ints, x,y,z per level). */
int nn4mg_levels(nn4mg_t h, int *levels, int *dims, int max_levels);

/* Device bytes held by the handle. */
size_t nn4mg_bytes_held(nn4mg_t h);

/* Kernel timing for benchmarks: while enabled, every launch of the finest-level
 * kernels below is bracketed by a pair of HIP events on the handle's stream;
 * launches that exit early (after the stopping rule fired) are discarded.
 * enable = 1 resets and starts recording, 0 stops.  Recording is capped at
 * 4096 launches per class. */
enum { NN4MG_KCLASS_FINE_RESID = 0,        /* residual + restriction + norm partials */
       NN4MG_KCLASS_FINE_SWEEP_PROLONG = 1, /* first sweep after the prolongation, reads P e of the level
                                               below; with nu_post == 2 both sweeps run in this one pass */
       NN4MG_KCLASS_FINE_SWEEP = 2,         /* later sweeps (nu_post != 2 only) */
       NN4MG_KCLASS_COUNT = 3 };
int nn4mg_profile(nn4mg_t h, int enable);
/* Launch count and summed duration (ms) of one class at the finest level
 * since the last enable. */
int nn4mg_profile_read(nn4mg_t h, int kclass, int *launches, double *total_ms);
/* Same for any level (level 0 = finest); coarse levels have the two sweep
 * classes only. */
int nn4mg_profile_read_level(nn4mg_t h, int level, int kclass, int *launches, double *total_ms);

/* Launch shape of one stencil kernel class (NN4MG_KCLASS_*; -1 = all classes
 * for set) of one level: tile width tx (64, 32 or 16 cells along x), ry cell
 * rows per thread (1, 2 or 4; 2 or 1 when tx == 16; 2 or 4 for the residual
 * class; the tile is tx x ry*256/tx cells in x-y) and the number of z-planes
 * zc (even, >= 2) each workgroup marches.  With the default two post-sweeps
 * the first-sweep class also accepts (8, 8, 8): both sweeps of the level run
 * as independent 8^3 blocks (one round of loads per block instead of a march
 * over z; for small levels); any other shape of that class switches it back.
 * Any shape gives the same results up to rounding; only the speed differs.
 * EINVAL for a bad level, class or shape, or (8, 8, 8) on a level without the
 * two-sweep kernel (nu_post != 2, or a dimension below 4). */
int nn4mg_set_tiles(nn4mg_t h, int level, int kclass, int tx, int ry, int zc);
int nn4mg_get_tiles(nn4mg_t h, int level, int kclass, int *tx, int *ry, int *zc);

/* Autotuner: time the candidate launch shapes (tile width, rows per thread,
 * z-chunk, and the 8^3 block form of the two sweeps) on a few cycles with
 * b_dev and x_dev as input (x_dev is overwritten), keep the fastest shape per
 * level and kernel class, and return them in tiles_out (9 ints per level: tx,
 * ry, zc for each of the 3 classes; (8, 8, 8) for the block form; may be
 * NULL).  Synchronous. */
int nn4mg_autotune(nn4mg_t h, const double *b_dev, double *x_dev, int *tiles_out, int max_levels);

/* ---- Continuous-batching solve server ------------------------------------
 * Serves the pressure solves of a time-stepping or ensemble workload, each with
 * its own grid size, coefficient and right-hand side (the paper's solver runs
 * one pressure solve per stage and per time step, Sec. 2.4).  A worker thread
 * admits queued requests while fewer than max_slots run and the device memory
 * fits (the budget counts every resident hierarchy).  Requests of one
 * configuration are batched: they run as copies of one group (up to 16
 * identical hierarchies at a fixed stride in one allocation), and each kernel
 * of a cycle is one launch over the group's running copies, from a captured
 * hipGraph; a request joins a free copy while the group runs (its coefficient
 * and vectors are set up on a side stream) and leaves when its own stopping
 * rule has fired, checked on the device and read back asynchronously.  Groups
 * of different configurations run on their own streams and overlap; idle
 * groups stay resident for later requests and are evicted, least recently
 * used first, when memory is short.  Configurations with no batched form
 * (flexible CG outer iteration, other than two post-sweeps, no one-workgroup
 * coarse end) run one request per stream.  Results do not depend on which
 * other requests run or on the group's size: every workgroup reads only its
 * own request's data, launch shapes are fixed per configuration, and
 * reductions have a fixed order. */
typedef struct nn4mg_server *nn4mg_srv_t;

typedef struct {
    unsigned long long tag;   /* the caller's tag */
    nn4mg_info info;          /* as from nn4mg_solve; info.status carries the request's status */
    double t_submit_ms;       /* host clock, ms since the server was created */
    double t_start_ms;        /* admitted (to a group copy or a slot) */
    double t_done_ms;         /* x written back and the request completed */
    size_t bytes;             /* device bytes of the request's hierarchy (its share of a group) and work buffers */
} nn4mg_result;

/* hbm_budget_bytes: device memory the server may hold for hierarchies and
 * work buffers; max_slots: requests in flight at once (1..64).  The server uses
 * the current device of the calling thread.  Errors: EINVAL, EDEVICE. */
int nn4mg_server_create(size_t hbm_budget_bytes, int max_slots, nn4mg_srv_t *out);
/* Queue one solve of A x = b to rtol (at most max_cycles cycles; stationary
 * outer iteration).  k_dev (NODAL only), b_dev and x_dev (initial guess in,
 * solution out) are device arrays the caller keeps alive, and does not touch,
 * until nn4mg_server_poll returns the tag; their contents must be ready on the
 * device when this call is made.  Errors: EINVAL (bad config or pointers),
 * EBUSY (the request alone needs more than the whole budget). */
int nn4mg_server_submit(nn4mg_srv_t s, const nn4mg_config *cfg, const double *k_dev, const double *b_dev,
                        double *x_dev, double rtol, int max_cycles, unsigned long long tag);
/* Non-blocking: move up to cap finished requests into out, *n_done of them. */
int nn4mg_server_poll(nn4mg_srv_t s, nn4mg_result *out, int cap, int *n_done);
/* Block until every submitted request has finished (timeout_ms < 0: no limit);
 * EBUSY on timeout. */
int nn4mg_server_drain(nn4mg_srv_t s, double timeout_ms);
/* Device bytes held now and at peak, requests running and queued. */
int nn4mg_server_stats(nn4mg_srv_t s, size_t *bytes_in_use, size_t *peak_bytes, int *active, int *queued);
/* Stop the worker after the requests in flight finish (queued ones are
 * dropped), and free every resident hierarchy. */
int nn4mg_server_destroy(nn4mg_srv_t s);

/* ---- One two-phase time step (Sec. 2.4, Stages 1-4) -----------------------
 * The explicit momentum and compressive volume-of-fluid stencils around the
 * three pressure solves of one step, with linear (p = 1) filters on a uniform
 * grid: Stage 1 the hydrostatic + surface-tension pressure (Eq. ph_disc),
 * Stage 2 n_vel_iter Petrov-Galerkin velocity predictor iterations
 * (Eqs. Petrov, k_Psi-n, velocity-1), Stage 3 n_corr non-hydrostatic
 * corrections (Eqs. ph_disc2, vel-cor), Stage 4 the volume fraction update
 * (Eqs. Petrov-C, transport-indicator-1) with the compressive coefficients of
 * Sec. 2.3.5.  Boundaries are those of the paper's tank (Sec. 3.1): free-slip
 * walls on the sides and the bottom, an outlet on top with zero pressure;
 * C and rho zero-normal-derivative; hydrostatic pressure gradient -rho g at
 * the bottom.  Each pressure solve runs a fixed number of cycles (Sec. 2.4). */
typedef struct nn4mg_stepper *nn4mg_step_t;

typedef struct {
    double rho_l, rho_g;  /* densities of fluid (C = 1) and gas (C = 0) */
    double mu_l, mu_g;    /* dynamic viscosities */
    double g;             /* gravity, acting in -z */
    double sigma_t;       /* surface tension coefficient */
    double dt;            /* time step */
    int mg_cycles;        /* cycles per pressure solve (paper: 20) */
    int n_corr;           /* pressure-velocity corrections (paper: 2) */
    int n_vel_iter;       /* velocity predictor iterations (paper: 2) */
    int mg_cycles_nh;     /* cycles of each correction solve (the j of the paper's i-j strategies,
                             Sec. 3.2, with i = n_corr); 0: mg_cycles */
    int order;            /* 0 or 1: linear filters (3x3x3) throughout.  2: quadratic ConvFEM filters
                             (5x5x5, two-cell halos; Sec. 2.2.3, Sec. 2.3.3) for the momentum terms, the
                             interface geometry (gradients, normals, curvature) and the volume-fraction
                             advection, with linear filters for the volume-fraction diffusion (Table
                             disc_combinations, "linear/quadratic") and for both pressure equations and
                             the velocity correction, whose Poisson operator is this library's linear one */
    int reserved[3];      /* zero */
} nn4mg_step_params;

typedef struct {
    int solves;           /* pressure solves run (1 + n_corr) */
    double relres[8];     /* final relative residual of each */
    double ms_total;      /* device time of the step (HIP events) */
    double ms_mg;         /* device time inside the pressure solves */
    double volume;        /* sum over cells of C^{n+1} h^3 after the step: the integral of the volume
                             fraction whose ratio to the initial one, C(t)/C0, is the mass-conservation
                             measure of Sec. 3.2 (Fig. Multigrid_iteration) */
} nn4mg_step_info;

/* Water/air defaults: rho 1000/1, mu 1e-3/1.8e-5, g 9.81, sigma 0.07, dt 1e-4,
 * 20 cycles, 2 corrections, 2 predictor iterations. */
void nn4mg_step_params_default(nn4mg_step_params *p);
/* Workspace for an nx x ny x nz grid of spacing h (each dim >= 4, even and
 * coarsenable like nn4mg_setup's grids, fewer than 2^31 cells).  The launch shapes of its pressure
 * hierarchy are autotuned once here (a few cycles on zeroed work fields,
 * synchronous on hip_stream).  Errors: EINVAL, ENOMEM, EDEVICE. */
int nn4mg_step_create(int nx, int ny, int nz, double h, const nn4mg_step_params *p, void *hip_stream,
                      nn4mg_step_t *out);
/* Advance the caller's device fields (nx*ny*nz doubles each, updated in
 * place) by one step: C volume fraction, u v w velocity, p_hs hydrostatic and
 * surface-tension pressure (also the initial guess of its solve), p_nh
 * non-hydrostatic pressure.  Synchronous. */
int nn4mg_step(nn4mg_step_t s, double *C, double *u, double *v, double *w, double *p_hs, double *p_nh,
               nn4mg_step_info *info);
/* nsteps successive steps on the same fields (the time loop of Sec. 2.4, as
 * in the mass-conservation study of Sec. 3.2).
 *   volume: host array of nsteps + 1 doubles, or NULL; volume[0] = sum C h^3
 *           before the first step, volume[n] after step n.
 *   steps_done: host int (may be NULL), the steps completed.
 *   info: host record of the last step run (may be NULL).
 * Stops at the first failing step and returns its status: EBREAKDOWN when the
 * volume fraction becomes non-finite (the printed scheme's corrections can
 * amplify interface velocities by about (rho_l - rho_g) / (2 rho_g) per
 * correction at a sharp interface); the fields then hold that step's output.
 * Synchronous. */
int nn4mg_step_run(nn4mg_step_t s, int nsteps, double *C, double *u, double *v, double *w, double *p_hs,
                   double *p_nh, double *volume, int *steps_done, nn4mg_step_info *info);
int nn4mg_step_destroy(nn4mg_step_t s);

/* Release the hierarchy (synchronises its stream first).  NULL is accepted. */
int nn4mg_destroy(nn4mg_t h);

/* Message for the last failing call on this thread ("" if none). */
const char *nn4mg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NN4MG_H */
