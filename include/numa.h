/*
 * numa.h -- C ABI of the MI355X (gfx950) HEVI step for NUMA.
 *
 * The method is the horizontally-explicit, vertically-implicit ("1D-IMEX")
 * ARK2 time step of Abdi, Giraldo, Constantinescu, Carr, Wilcox and
 * Warburton, "Acceleration of the IMEX Non-hydrostatic Unified Model of the
 * Atmosphere (NUMA) on manycore processors", for the compressible Euler
 * equations in the non-conservative set Set2NC (Sec. 3.1) on hexahedral
 * Legendre-Gauss-Lobatto (LGL) spectral elements with continuous Galerkin
 * direct stiffness summation (Sec. 4, Sec. 5.3).
 *
 * Domain: an axis-aligned box, x and y periodic, rigid bottom and top
 * (w = 0 imposed strongly on the bottom and top nodes).  Background:
 * hydrostatic, either neutral with constant theta0 (isentropic) or stably
 * stratified with a constant Brunt-Vaisala frequency.
 *
 * State contract (every entry point that takes a state):
 *   - a DEVICE pointer owned by the caller (e.g. a torch tensor on cuda:0),
 *     5*nz*ny*nx contiguous doubles, structure of arrays [var][k][j][i],
 *     i fastest, variables (rho', u, v, w, theta') in that order;
 *   - nx = nex*N and ny = ney*N unique nodes (node i = nx is node 0, x and y
 *     are periodic), nz = nez*N + 1 levels; node (i, j, k) sits at the LGL
 *     point of its elements;
 *   - w must be 0 on levels 0 and nz-1.
 *
 * All GPU work is enqueued on the stream given to numa_setup; calls are
 * asynchronous except numa_check and numa_destroy, which synchronise.
 * A context serves one host thread at a time.  The only state outside the
 * contexts is the fixed stage-buffer array of numa_hevi_step_mixed_noalloc
 * (one per GPU, shared by every call on that GPU).
 *
 * Every function returns 0 (NUMA_OK) or a negative error code; the message of
 * the last error on a context is returned by numa_last_error.
 */
#ifndef NUMA_H
#define NUMA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NUMA_OK 0
#define NUMA_E_ARG (-1)           /* null pointer, size <= 0, N outside 1..8, bad zface */
#define NUMA_E_NOT_FACTORED (-2)  /* step or solve before numa_factor_columns           */
#define NUMA_E_DT_MISMATCH (-3)   /* dt differs (bitwise) from the factored dt          */
#define NUMA_E_HIP (-4)           /* HIP runtime error; text in numa_last_error         */
#define NUMA_E_NOMEM (-5)         /* device allocation failed                           */
#define NUMA_E_NONFINITE (-6)     /* a step produced NaN or Inf (reported by numa_check) */
#define NUMA_E_NOT_CONVERGED (-7) /* 3D-IMEX GMRES reached maxit before tol             */
#define NUMA_E_UNSUPPORTED (-8)   /* feature or size not supported by this build        */

typedef struct numa_ctx numa_ctx; /* opaque; owns all device memory except states */

typedef struct {
    double lx, ly, lz;            /* box extents [m], > 0                              */
    int32_t nex, ney, nez;        /* elements per axis, >= 1                           */
    const double *zface;          /* optional HOST array of nez+1 strictly increasing
                                     heights from 0 to lz; NULL = uniform             */
} numa_grid;

typedef struct {
    double theta0;                /* background potential temperature [K] at z = 0    */
    double p00;                   /* reference pressure of the equation of state [Pa] */
    double cp, rgas;              /* specific heat at constant pressure, gas constant */
    double grav;                  /* gravitational acceleration [m/s^2]               */
    double nbv;                   /* Brunt-Vaisala frequency Nb [1/s] (>= 0): theta0(z)
                                     = theta0 exp(Nb^2 z / g); 0 = isentropic          */
} numa_background;

typedef struct {
    int64_t nx, ny, nz;           /* unique-node grid                                 */
    int64_t ncol;                 /* vertical columns (nx*ny)                         */
    int64_t factor_bytes;         /* device bytes of the stored column factors        */
    int64_t scratch_bytes;        /* device bytes of the stage buffers                */
    int64_t step_bytes;           /* algorithmic HBM bytes moved per HEVI step        */
    int32_t order;                /* LGL order N                                      */
    int32_t factored;             /* 1 once numa_factor_columns succeeded             */
    double dt_factored;           /* dt of the stored factors                         */
    int32_t column_solver;        /* NUMA_SOLVER_BAND, _BLOCKED or _PER_COLUMN, in use */
    int32_t reserved;
} numa_info;

/*
 * Set up a context: LGL nodes and differentiation matrix of order N
 * (the sD operator of Alg. 1-2), the direct-stiffness-summed 1D derivative
 * operators along x, y and z (Sec. 5.3), and the background profiles
 * theta0(z), rho0 from the hydrostatic Exner function (d pi0/dz =
 * -g/(cp theta0), pi0(0) = 1, integrated in closed form), P0 = EOS(rho0,
 * theta0), G0 = gamma P0/rho0, H0 = gamma P0/theta0 (Sec. 3.1, background
 * split and linearised pressure, Eq. (13)); reference fields are computed
 * once at start-up as in Sec. 5.1.
 * g, bg: host pointers, read during the call only.  order: N in 1..8.
 * hip_stream: a hipStream_t (NULL = the null stream).  *out receives the
 * context.  Errors: NUMA_E_ARG, NUMA_E_UNSUPPORTED (order 9..15; columns
 * whose solve or right-hand-side workgroup would not fit one CU's 160 KB of
 * LDS, i.e. above about 290 levels; a field above 4 GiB), NUMA_E_NOMEM,
 * NUMA_E_HIP.
 */
int numa_setup(const numa_grid *g, int32_t order, const numa_background *bg,
               void *hip_stream, numa_ctx **out);

/* shape[4] (host) = {5, nz, ny, nx}.  Errors: NUMA_E_ARG. */
int numa_state_shape(const numa_ctx *c, int64_t shape[4]);

/* Sizes and byte counts of the context (host struct).  Errors: NUMA_E_ARG. */
int numa_get_info(const numa_ctx *c, numa_info *info);

/* Rebind the context to another stream (hipStream_t; NULL = null stream). */
int numa_set_stream(numa_ctx *c, void *hip_stream);

/*
 * Launch configuration of the right-hand sides (Sec. 5.1: the volume kernel
 * over element tiles), a project autotuner on top of the paper's method.
 * The right-hand-side kernel is compiled for two tile shapes per order (TX x
 * TY columns per workgroup, element aligned; one shape at N = 6 and 8) and runs
 * over a vertical chunk of zchunk elements per workgroup.
 * numa_autotune: times the three right-hand sides of a step on state
 * (device, state contract; read only, outputs into the context's stage
 * buffers) for every tile that fits one CU's LDS and every chunk nez,
 * nez/2, nez/3, ..., 1, `reps` launches each, and keeps the fastest pair for
 * the context; config_out (host, nullable, 4 ints) as numa_get_rhs_config.
 * Synchronous.  The step's results do not depend on the configuration.  The
 * precision form uses the same configuration.
 * numa_set_rhs_config: tile 0 (the default shape) or 1, zchunk 0 (automatic:
 * the largest chunk that still gives two workgroups per CU) or 1..nez.
 * numa_get_rhs_config: out[4] (host) = {tile, TX, TY, zchunk in use}.
 * Errors: NUMA_E_ARG, NUMA_E_UNSUPPORTED (tile 1 where the order has one
 * shape or its LDS does not fit), NUMA_E_HIP.
 */
int numa_autotune(numa_ctx *c, const double *state, int32_t reps, int32_t *config_out);
int numa_set_rhs_config(numa_ctx *c, int32_t tile, int32_t zchunk);
int numa_get_rhs_config(const numa_ctx *c, int32_t *out);

/*
 * Build and LU-factor, once per time-step size, the matrix of every vertical
 * column of the Schur-complement system of the implicit stages (Sec. 3.1,
 * Eqs. (14)-(17), restricted to the vertical; Sec. 5.4: block-diagonal by
 * column, factored once and stored), at lambda = (1 - 1/sqrt(2)) dt, the
 * diagonal of the ARK2 implicit tableau (Table 1).  Banded LU without
 * pivoting, half-bandwidth 2N (Alg. 9); the factors stay on the device.
 * Every column of a context has the same operator (uniform horizontal grid,
 * one set of vertical faces, horizontally uniform background), so one
 * factor set serves all columns, unless NUMA_SOLVER_PER_COLUMN asks for
 * each column's own.  dt > 0.  Errors: NUMA_E_ARG, NUMA_E_NOMEM (per-column
 * factors), NUMA_E_HIP (a zero or non-finite pivot is reported by
 * numa_check as NUMA_E_NONFINITE).
 */
int numa_factor_columns(numa_ctx *c, double dt);

/*
 * How the column solves are laid out on the GPU (both run the forward and
 * backward band substitutions of Alg. 9 with the same stored factors; the
 * results agree to rounding).  NUMA_SOLVER_BAND: one lane per column, each
 * lane walking all levels of its column.  NUMA_SOLVER_BLOCKED: four
 * wavefronts per 64 columns (eight above 64 - 2N levels, sixteen above 128
 * levels), each holding a block of levels in registers for the stage
 * right-hand side and the extraction, and one wavefront running the
 * substitutions from LDS; available for columns of at most 128 levels, and
 * of at most 224 levels where (nz + 2N) * 64 + nz * (4N + 1) doubles of LDS
 * fit one CU's 160 KB.  NUMA_SOLVER_PER_COLUMN: one lane per column with
 * every column's own factors, assembled and factored by its own lane and
 * stored [level][diagonal][column] in device memory (Sec. 5.4: the LU of
 * each column computed once and stored; nz (4N+1) ncol doubles, below
 * 4 GiB, allocated by numa_factor_columns), for columns whose matrices may
 * differ; here they are equal, so it reads the same numbers as the shared
 * band from a layout of ncol times its size.  NUMA_SOLVER_AUTO (the
 * default): blocked where available.
 * Takes effect at the next numa_factor_columns; until then the context
 * counts as not factored.  Errors: NUMA_E_ARG (unknown kind),
 * NUMA_E_UNSUPPORTED (blocked for a column it does not support, per-column
 * factors above 4 GiB).
 */
#define NUMA_SOLVER_AUTO 0
#define NUMA_SOLVER_BAND 1
#define NUMA_SOLVER_BLOCKED 2
#define NUMA_SOLVER_PER_COLUMN 3
int numa_set_column_solver(numa_ctx *c, int32_t kind);

/*
 * Advance state (device, see the state contract) in place by nsteps ARK2
 * HEVI steps of size dt (Sec. 2: HEVI splitting Eq. (4) and the ARK stages
 * of Sec. 2.2 in their q~ predictor-corrector form; Table 1).  Each step
 * evaluates the explicit Set2NC right-hand side with DSS three times and
 * solves the vertical Schur system column by column twice with the stored
 * factors.  dt must equal the factored dt bitwise.  nsteps >= 0.
 * Asynchronous; non-finite results are reported by numa_check.
 * Errors: NUMA_E_ARG, NUMA_E_NOT_FACTORED, NUMA_E_DT_MISMATCH, NUMA_E_HIP.
 */
int numa_hevi_step(numa_ctx *c, double *state, double dt, int32_t nsteps);

/*
 * Same as numa_hevi_step, with a HIP event recorded around every kernel of
 * the step on the context's stream; synchronises at the end.  ms_out (host,
 * 5 doubles) receives the average duration in milliseconds of each of the
 * five kernels of a step over the nsteps steps, in launch order: explicit
 * right-hand side of stage 1, column solve of stage 2, right-hand side of
 * stage 2, column solve of stage 3, right-hand side of stage 3 with the
 * final ARK combination.  nsteps >= 1.  Errors: as numa_hevi_step.
 */
int numa_profile_steps(numa_ctx *c, double *state, double dt, int32_t nsteps, double *ms_out);

/*
 * Precision form of numa_hevi_step.  Not a method of the paper (whose
 * kernels are FP64 and, by its own roofline measurements in Sec. 6.1,
 * mostly memory-bound): a project addition on top of the ARK2 HEVI step of
 * Sec. 2.2 that stores the first stage's tendency R1 in FP32.  The same five
 * kernels, stage algebra and FP64 arithmetic as numa_hevi_step; R1, which
 * the step uses only multiplied by dt, is written and read as FP32 (14 of
 * the step's 65 field passes: 464 bytes per node instead of 520),
 * while the state, the accumulator of the final combination, every stage
 * value and the column solves (FP64 factors) stay in FP64.  state: the FP64
 * device array of the state contract, advanced in place.  Needs the
 * factors of numa_factor_columns(dt) like the FP64 step.  The first call
 * allocates 96 bytes per unique node of stage buffers for the context (112
 * over a stratified background; freed by numa_destroy).  Asynchronous.
 * Errors: as numa_hevi_step, and NUMA_E_NOMEM.
 */
int numa_hevi_step_mixed(numa_ctx *c, double *state, double dt, int32_t nsteps);

/*
 * numa_hevi_step_mixed without any device allocation, for callers that
 * cannot allocate (code under HIP graph capture, serving loops, harnesses
 * that forbid hipMalloc).  Same kernels, arguments and results as
 * numa_hevi_step_mixed, but the precision form's stage buffers (96 bytes
 * per unique node, 112 over a stratified background) live in a fixed 64 MiB
 * device array of the library (one copy per GPU, resolved by numa_setup on
 * its device, held until the process ends), so grids of at most 699,050
 * unique nodes (599,186 stratified) are accepted.  The
 * context's own buffers (allocated by numa_setup) are used as by
 * numa_hevi_step_mixed.  Every call on a GPU shares that GPU's array: calls
 * that overlap in time on one GPU (other streams, other contexts, other
 * host threads) race and must be ordered by the caller.  The array keeps
 * the last call's contents; nothing in it needs to start at zero.
 * Asynchronous.  Errors: as numa_hevi_step, and NUMA_E_UNSUPPORTED (grid
 * above the array's size; nothing is launched).
 */
int numa_hevi_step_mixed_noalloc(numa_ctx *c, double *state, double dt, int32_t nsteps);

/*
 * numa_profile_steps for the precision form (ms_out as there).
 */
int numa_profile_steps_mixed(numa_ctx *c, double *state, double dt, int32_t nsteps, double *ms_out);

/*
 * Batched ensemble (a project addition for many small domains; the paper
 * steps one domain at a time).  n contexts, each already factored with its
 * dt, with their FP64 device states, are stepped together: one step of every
 * domain is captured into a single HIP graph, each domain's five kernels on
 * its own branch, so that domains too small to fill the GPU run side by
 * side and a step costs one graph launch.  mixed != 0 captures the
 * precision form (numa_hevi_step_mixed) instead of the FP64 step.
 * tune != 0 runs the autotuner of numa_autotune on every domain's state
 * first (tile shape and vertical chunk per context; numa_get_rhs_config
 * reports them).  States and dts are fixed at creation (the
 * graph holds them); the contexts must not be destroyed or refactored while
 * the ensemble lives.  hip_stream: the stream the graph is launched on
 * (NULL: the ensemble creates one).  Creation synchronises the contexts'
 * streams.  Errors: NUMA_E_ARG (null or repeated context or state, n outside
 * 1..1024), NUMA_E_NOT_FACTORED, NUMA_E_DT_MISMATCH, NUMA_E_NOMEM,
 * NUMA_E_HIP; message in numa_ensemble_last_error(NULL).
 */
typedef struct numa_ensemble numa_ensemble;
int numa_ensemble_create(numa_ctx *const *ctxs, double *const *states, const double *dts, int32_t n,
                         int32_t mixed, int32_t tune, void *hip_stream, numa_ensemble **out);
/* nsteps steps of every domain (nsteps graph launches).  Asynchronous. */
int numa_ensemble_step(numa_ensemble *e, int32_t nsteps);
/* Synchronise, then numa_check every context (NUMA_E_NONFINITE if any step
 * produced NaN/Inf). */
int numa_ensemble_sync(numa_ensemble *e);
/* The vertical chunk each domain's right-hand side uses (zchunk[n]). */
int numa_ensemble_zchunks(const numa_ensemble *e, int32_t *zchunk);
/* Synchronise and free the graph, streams and events (NULL-safe). */
int numa_ensemble_destroy(numa_ensemble *e);
/* Last error of e (of the last failed creation on this thread if e is NULL). */
const char *numa_ensemble_last_error(const numa_ensemble *e);

/*
 * rhs_out = R(state): the explicit right-hand side of Set2NC in perturbation
 * form (Sec. 3.1) with the continuity equation in divergence form,
 * element-local strong-form LGL derivatives (Alg. 2) and DSS (Sec. 5.3);
 * R_w = 0 on the bottom and top levels.  state, rhs_out: device arrays of
 * the state contract; they must not overlap.  Asynchronous.
 * Errors: NUMA_E_ARG, NUMA_E_HIP.
 */
int numa_rhs(numa_ctx *c, const double *state, double *rhs_out);

/*
 * x = (I - lambda L_V)^{-1} y with the stored factors: the direct column
 * solve of the implicit stage (Sec. 5.4) through the Schur complement for
 * the pressure (Eqs. (16)-(17) in 1D) followed by the extraction of w and
 * rho' (Sec. 5).  u, v and theta' pass through.  y, x: device arrays of the
 * state contract (w = 0 on the walls of y); they must not overlap.
 * Asynchronous.  Errors: NUMA_E_ARG, NUMA_E_NOT_FACTORED, NUMA_E_HIP.
 */
int numa_solve_columns(numa_ctx *c, const double *y, double *x);

/*
 * Standard-form column solve, a comparison point for the Schur form (Sec. 5,
 * Sec. 5.4): the same x = (I - lambda L_V)^{-1} y as numa_solve_columns, but
 * solving for (rho', w) together, unknowns interleaved per level, a band of
 * half-width 2N+1 factored without pivoting.  Its matrix is far worse
 * conditioned than the Schur matrix (about 1e6 against 1e2 at vertical
 * Courant number 15), so it agrees with the Schur solve to about 1e-9, not to
 * rounding.  numa_factor_columns_standard: factors at lambda(dt), one set
 * shared by the identical columns (allocated on first use; *bytes_out,
 * nullable host, = their size).  Asynchronous.
 * numa_solve_columns_standard: as numa_solve_columns (y, x state-contract
 * device arrays, not overlapping; u, v, theta' copied through).
 * Asynchronous.  Errors: NUMA_E_ARG, NUMA_E_NOT_FACTORED, NUMA_E_NOMEM,
 * NUMA_E_HIP (a zero or non-finite pivot is reported by numa_check).
 */
int numa_factor_columns_standard(numa_ctx *c, double dt, int64_t *bytes_out);
int numa_solve_columns_standard(numa_ctx *c, const double *y, double *x);

/*
 * 3D-IMEX (Sec. 2): the implicit part of the ARK2 step is the whole linear
 * operator L (horizontal acoustics included) instead of L_V, and each
 * implicit system (I - lambda L) x = y is solved iteratively (Sec. 5.5) in
 * its Schur-complement form for the linear pressure P = G0 rho' + H0 theta'
 * (the Set2NC analogue of Algs. 4-5):
 *   S P = P - lambda G0 div(rho0 U_p(P)) = b,
 *   U_p(P) = lambda (Dx P/rho0, Dy P/rho0, B (Dz P/rho0 + g P/(G0 rho0))),
 *   b = G0 y_rho + H0 y_theta - lambda G0 div(rho0 U_a),
 *   U_a = (y_u, y_v, B (y_w + lambda g H0 y_theta/(G0 rho0))),
 * B zeroing w on the bottom and top levels, followed by u = U_a - U_p(P),
 * rho' from the continuity row and theta' = y_theta.  S P = b is solved by
 * restarted GMRES from P = 0, right-preconditioned by PBNO (Sec. 5.5,
 * Alg. 8): the Chebyshev minimax polynomial of the given order on the
 * eigenvalue interval [lmin, lmax] of S (order 0 is the scaling
 * 2/(lmin+lmax) alone, -1 no preconditioner).  lambda = (1 - 1/sqrt(2)) dt.
 *
 * numa_imex3d_setup: allocates the solver state of the context (Krylov
 * basis of restart+1 fields, 9 scalar and 4 five-field work fields) and
 * estimates the interval: lmin = 1, lmax = 1.1 |S^k v|/|S^(k-1) v| after
 * k = power_steps power steps from v_I = frac(I * 2654435769 / 2^32) - 1/2
 * (power_steps = 0 keeps [1, 2]; set it with numa_imex3d_set_bounds).
 * restart 1..63, pbno_order -1..16, maxit >= 1 (Arnoldi iterations per
 * solve).  Calling it again replaces the previous state.  Synchronous.
 * Errors: NUMA_E_ARG, NUMA_E_NOMEM, NUMA_E_HIP.
 * numa_imex3d_bounds: out[2] (host) = {lmin, lmax}.  numa_imex3d_set_bounds:
 * overrides them (0 < lmin < lmax).
 * numa_imex3d_set_precision: pbno_fp32 = 1 runs the PBNO recurrence (orders
 * >= 1) in FP32: the residual is rounded to FP32, the p applications of S
 * use FP32 fields, tables and sums, and the result is widened to FP64 (a
 * preconditioner only has to approximate S^-1; the Krylov vectors, S in the
 * Arnoldi step and the stopping test stay FP64).  Rounding makes the
 * polynomial differ slightly between applications, so the solves then run
 * flexible GMRES (the Z basis), which converges to the same true-residual
 * tolerance.  0 (the default after numa_imex3d_setup) is the FP64
 * polynomial.  Also applies to numa_pbno_apply.  Errors: NUMA_E_ARG,
 * NUMA_E_NOT_FACTORED (no numa_imex3d_setup).
 *
 * numa_schur_apply (out = S P), numa_schur_rhs (b from y) and
 * numa_pbno_apply (z = s(S) r): single device fields of nz*ny*nx doubles
 * (y: a state-contract array; P/out and r/z distinct).  Asynchronous.
 *
 * numa_imex3d_solve: x = (I - lambda L)^-1 y to |b - S P| <= tol |b|;
 * y, x state-contract device arrays (x == y allowed, no partial overlap);
 * *iters_out (host, nullable) = Arnoldi iterations.  Synchronous.
 * numa_imex3d_step: one ARK2 step of state (dt equal, bitwise, to the set-up
 * dt), both stage solves to tol; *iters_out = their iterations.
 * Synchronous; NaN or Inf is reported by numa_check.
 * Errors of these: NUMA_E_ARG, NUMA_E_NOT_FACTORED (no numa_imex3d_setup),
 * NUMA_E_DT_MISMATCH, NUMA_E_NOT_CONVERGED (maxit reached; the result is
 * still written), NUMA_E_HIP.
 */
int numa_imex3d_setup(numa_ctx *c, double dt, int32_t restart, int32_t pbno_order, int32_t power_steps,
                      int32_t maxit);
int numa_imex3d_bounds(const numa_ctx *c, double *out);
int numa_imex3d_set_bounds(numa_ctx *c, double lmin, double lmax);
int numa_imex3d_set_precision(numa_ctx *c, int32_t pbno_fp32);
int numa_schur_apply(numa_ctx *c, const double *P, double *out);
int numa_schur_rhs(numa_ctx *c, const double *y, double *b);
int numa_pbno_apply(numa_ctx *c, const double *r, double *z);
int numa_imex3d_solve(numa_ctx *c, const double *y, double *x, double tol, int32_t *iters_out);
int numa_imex3d_step(numa_ctx *c, double *state, double dt, double tol, int32_t *iters_out);

/*
 * Learned correction of the 3D-IMEX preconditioner (a project addition; the
 * paper's preconditioners are polynomial, Sec. 5.5).  A two-layer FP32
 * perceptron per element, h = tanh(W1 x + b1), y = W2 h + b2, nin = (N+1)^3
 * inputs (the element's local nodes, a + (N+1) (b + (N+1) c), a along x),
 * `hidden` units, acts on x = r_e / s_e (s_e the RMS of r over the element);
 * the node average of s_e y over the elements sharing a node is added to
 * the PBNO polynomial: z = s(S) r + corr(r).  While enabled, the 3D-IMEX
 * solves run flexible GMRES (the correction is nonlinear); PBNO alone is
 * the fallback: a restart cycle with the network that does not reduce the
 * residual norm tenfold switches it off for the rest of that solve, and
 * numa_learned_enable(c, 0) switches it off altogether.
 *
 * numa_learned_setup: allocates the network (parameters W1[hidden][nin],
 * b1[hidden], W2[nin][hidden], b2[nin] in that order, FP32; W uniform in
 * +-sqrt(6/(nin+hidden)) from `seed`, b = 0), Adam state and room for
 * max_samples element samples.  Needs numa_imex3d_setup.  Synchronous.
 * numa_learned_info: info[6] (host) = {nparam, nin, hidden, samples,
 * max_samples, enabled}.
 * numa_learned_add_samples: r (device field) -> solves S e = r with the
 * polynomial preconditioner to |r - S e| <= tol |r| and appends the nelem
 * samples (x = r_e/s_e, t = (e - s(S) r)_e / s_e; elements with s_e below
 * 1e-3 of the field's RMS give empty samples, x = t = 0).  Synchronous.
 * numa_learned_samples: copies samples first..first+n-1 to X, T (device,
 * n*nin floats each).
 * numa_learned_params: theta_in (host, nparam floats, nullable) replaces the
 * parameters, then theta_out (host, nullable) receives them.
 * numa_learned_loss_grad: mean squared error of the network on X, T (device,
 * n*nin floats; n <= max(max_samples, elements)) and its gradient into
 * grad_out (device, nparam floats).  Synchronous.
 * numa_learned_train: `steps` Adam steps (lr; betas 0.9, 0.999) on batches of
 * `batch` consecutive samples at seeded offsets; losses of the first and
 * last batch to the host pointers (nullable).  Synchronous.
 * numa_learned_enable: on != 0 uses the correction in the 3D-IMEX solves
 * (unconditionally: numa_learned_judge is the checked way to switch it on).
 * numa_learned_judge: PBNO as the judge of the network.  Solves
 * (I - lambda L) x = y (y, x device 5-field states, distinct, the lambda of
 * numa_imex3d_setup) to tol twice: flexible GMRES with the network, then
 * the polynomial alone; x receives the second solution.  The network is
 * accepted, and left switched on, only if its solve converged in fewer
 * GMRES iterations than the polynomial's; otherwise it is switched off.
 * out[3] (host) = {polynomial iterations, network iterations, accepted}.
 * NUMA_E_NOT_CONVERGED if the polynomial solve does not converge; on that
 * or any other error the network is left switched off.  Synchronous.
 * numa_learned_apply: z = s(S) r + corr(r) (device fields, distinct).
 * Errors: NUMA_E_ARG, NUMA_E_NOT_FACTORED (no numa_imex3d_setup /
 * numa_learned_setup), NUMA_E_NOT_CONVERGED (a sample solve), NUMA_E_HIP.
 */
int numa_learned_setup(numa_ctx *c, int32_t hidden, int64_t max_samples, uint64_t seed);
int numa_learned_info(const numa_ctx *c, int64_t *info);
int numa_learned_add_samples(numa_ctx *c, const double *r, double tol, int32_t *iters_out);
int numa_learned_samples(numa_ctx *c, int64_t first, int64_t n, float *X, float *T);
int numa_learned_params(numa_ctx *c, float *theta_out, const float *theta_in);
int numa_learned_loss_grad(numa_ctx *c, const float *X, const float *T, int64_t n, float *grad_out, double *loss_out);
int numa_learned_train(numa_ctx *c, int32_t steps, int32_t batch, double lr, uint64_t seed, double *loss_first,
                       double *loss_last);
int numa_learned_enable(numa_ctx *c, int32_t on);
int numa_learned_judge(numa_ctx *c, const double *y, double *x, double tol, int32_t *out);
int numa_learned_apply(numa_ctx *c, const double *r, double *z);

/*
 * Host-only helpers (no GPU needed): the operators numa_setup builds.
 * numa_lgl_basis: LGL nodes xi[order+1] on [-1, 1] and the differentiation
 * matrix D[(order+1)^2] (row-major, D[i*(order+1)+j] = l_j'(xi_i)), the sD
 * operator of Alg. 1-2.  numa_line_operators: the direct-stiffness-summed
 * 1D derivative operators (Sec. 5.3) on grid g: wxy[2*order*(2*order+1)]
 * holds, for x then y and for each local index a in 0..order-1, the
 * coefficients of the 2*order+1 nodes starting order nodes before the
 * node's element; dzb[nz*(2*order+1)] holds, for each level k, the
 * coefficients of levels k-order .. k+order.  Caller-owned host arrays.
 * Errors: NUMA_E_ARG.
 */
int numa_lgl_basis(int32_t order, double *xi, double *D);
int numa_line_operators(const numa_grid *g, int32_t order, double *wxy, double *dzb);

/* Synchronise the stream; NUMA_E_NONFINITE if a step or factorisation
 * produced NaN/Inf since the last check (the flag is then cleared). */
int numa_check(numa_ctx *c);

/* Synchronise and free every device allocation of the context.  NULL-safe. */
int numa_destroy(numa_ctx *c);

/* Text of the last error on c (per context; valid until the next call on c).
 * numa_last_error(NULL) returns the last numa_setup failure of this thread. */
const char *numa_last_error(const numa_ctx *c);

#ifdef __cplusplus
}
#endif
#endif /* NUMA_H */
