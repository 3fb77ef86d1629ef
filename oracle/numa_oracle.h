/*
 * numa_oracle.h -- plain FP64 CPU oracle for the 1D-IMEX (HEVI) ARK2 step of
 * NUMA (Abdi, Giraldo, Constantinescu, Carr, Wilcox, Warburton, "Acceleration
 * of the IMEX Non-hydrostatic Unified Model of the Atmosphere (NUMA) on
 * manycore processors").
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against the paper.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product path never does.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Everything is FP64.  Loops follow the paper's statement of the method in
 * its own order and notation: element-local strong-form derivatives on
 * Legendre-Gauss-Lobatto (LGL) nodes (Sec. 5.1, Alg. 1-2), direct stiffness
 * summation (Sec. 5.3), column Jacobians built by probing (Sec. 5.4, Alg. 7)
 * and the ARK2 stages in their direct form (Sec. 2.2, Table 1).
 *
 * State layout (same contract as the GPU library, so the two can be compared
 * element by element): 5 fields (rho', u, v, w, theta'), each a unique-node
 * array [k][j][i], i fastest; nx = nex*N, ny = ney*N (x and y periodic),
 * nz = nez*N + 1 (rigid bottom and top).
 *
 * Return codes: 0 ok, -1 bad argument, -2 not factored / lambda mismatch,
 * -3 precondition violated (w != 0 on a wall), -4 singular column matrix,
 * -5 out of memory, -6 iterative solve did not converge, -7 not available
 * over a stratified background (the 3D-IMEX Schur form assumes theta0
 * constant).
 */
#ifndef NUMA_ORACLE_H
#define NUMA_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_ctx orc_ctx;

/* LGL nodes xi[0..N] (ascending, xi[0] = -1, xi[N] = 1) and weights w[0..N]. */
void orc_lgl(int N, double *xi, double *w);
/* LGL differentiation matrix D[i*(N+1)+j] = d l_j / d xi at xi_i. */
void orc_dmat(int N, const double *xi, double *D);

/* zface: NULL (uniform) or nez+1 increasing heights from 0 to lz.  nbv: the
 * background's Brunt-Vaisala frequency [1/s]; 0 gives the isentropic
 * background (theta0 constant), nbv > 0 theta0(z) = theta0 exp(nbv^2 z / g)
 * (Sec. 3.1: background in hydrostatic balance). */
orc_ctx *orc_setup(double lx, double ly, double lz, int nex, int ney, int nez,
                   const double *zface, int N, double theta0, double p00,
                   double cp, double rgas, double grav, double nbv);
void orc_free(orc_ctx *c);
void orc_set_threads(int n);
int orc_get_threads(void);

/* Sizes: out[0..3] = nx, ny, nz, nelem. */
void orc_sizes(const orc_ctx *c, long *out);
/* Node coordinates: x[nx], y[ny], z[nz]. */
void orc_coords(const orc_ctx *c, double *x, double *y, double *z);
/* Assembled (lumped) mass M_I at every unique node, [k][j][i]. */
void orc_mass(const orc_ctx *c, double *M);
/* Background per level k: rho0, P0, G0 = gamma P0/rho0, H0 = gamma P0/theta0. */
void orc_background(const orc_ctx *c, double *rho0, double *P0, double *G0, double *H0);
/* theta0(z) and its vertical derivative per level. */
void orc_background_theta(const orc_ctx *c, double *th0, double *th0z);

/* Perturbation pressure P' = EOS(rho, theta) - P0 at every unique node
 * (evaluated without cancelling the background pressure). */
int orc_pressure_perturbation(orc_ctx *c, const double *q, double *Pp);
/* Explicit right-hand side R(q) of Set2NC (Sec. 3.1) with DSS. */
int orc_rhs(orc_ctx *c, const double *q, double *R);
/* Vertical linear operator L_V(q) (Sec. 2, HEVI splitting; Sec. 3.1 operator L). */
int orc_lv(orc_ctx *c, const double *q, double *L);
/* Full 3D linear operator L(q) (Sec. 3.1). */
int orc_lfull(orc_ctx *c, const double *q, double *L);
/* Build (by probing, Alg. 7) and LU-factor the column matrices of I - lambda*L_V. */
int orc_factor(orc_ctx *c, double lambda);
/* x = (I - lambda L_V)^{-1} y using the stored factors.  y and x may alias. */
int orc_solve(orc_ctx *c, const double *y, double *x);
/* The dense column matrix (nv M x nv M, row-major, unknowns (rho'_0..M-1,
 * w_0..M-1) and, over a stratified background (nv = 3), theta'_0..M-1) of
 * I - lambda L_V for column (i, j), before factorisation. */
int orc_column_matrix(orc_ctx *c, double lambda, int i, int j, double *A);
/* nsteps ARK2 steps of size dt, in place.  linear != 0 replaces R by the full
 * linear operator L (used by the time-order test).  The factors must have been
 * built with lambda = (1 - 1/sqrt 2) dt. */
int orc_step(orc_ctx *c, double *q, double dt, int nsteps, int linear);
/* ARK2 tableau as used by orc_step: a[3][3], at[3][3], b[3] (Table 1). */
void orc_ark2_tableau(double *a, double *at, double *b);
/* 3D-IMEX (Sec. 2, Sec. 5.5).  Schur-complement pressure operator
 * S P = P - lambda G0 div(rho0 U_p(P)) and its right-hand side b from a
 * 5-field y (Set2NC analogue of Algs. 4-5). */
int orc_schur_apply(orc_ctx *c, const double *P, double *out, double lambda);
int orc_schur_rhs(orc_ctx *c, const double *y, double *b, double lambda);
/* PBNO preconditioner z = s(S) r of the given order (Chebyshev polynomial on
 * [lmin, lmax]) and the interval estimate out = {1, 1.1 x k-step power method}. */
int orc_pbno_apply(orc_ctx *c, const double *r, double *z, double lambda, int order, double lmin, double lmax);
int orc_schur_bounds(orc_ctx *c, double lambda, int k, double *out);
/* x = (I - lambda L)^{-1} y: Schur form, restarted GMRES(restart) from P = 0
 * until |b - S P| <= tol |b|, PBNO of the given order on bounds[0..1]
 * (order < 0: unpreconditioned, bounds unused).  *iters: Arnoldi iterations.
 * Returns -6 (x still written) if maxit iterations did not reach tol. */
int orc_solve3d(orc_ctx *c, const double *y, double *x, double lambda, double tol, int restart, int maxit,
                int order, const double *bounds, int *iters);
/* The same system in its unreduced 5-field form, unpreconditioned GMRES. */
int orc_solve3d_standard(orc_ctx *c, const double *y, double *x, double lambda, double tol, int restart, int maxit,
                         int *iters);
/* Learned correction of the preconditioner (project addition): a two-layer
 * perceptron per element, h = tanh(W1 x + b1), y = W2 h + b2, with
 * W1[nh][nin], W2[nin][nh], nin = (N+1)^3 (the element's local nodes).
 * orc_mlp_loss_grad: mean squared error over B samples X[B][nin] against
 * T[B][nin] and its gradient.  orc_element_features: X[nelem][nin] = r_e/s_e,
 * s_e the RMS of r over element e.  orc_mlp_correction: node average of
 * s_e MLP(r_e/s_e).  orc_learned_apply: z = PBNO(r) + that correction.
 * orc_solve3d_learned: orc_solve3d through flexible GMRES with it; a
 * restart cycle that does not reduce the residual norm tenfold switches the
 * network off for the rest of the solve (the polynomial is the fallback);
 * *net_cycles (nullable): the restart cycles that ran with the network. */
typedef struct {
    int nin, nh;
    const double *W1, *b1, *W2, *b2;
} orc_mlp;
void orc_mlp_forward(const orc_mlp *m, const double *x, double *h, double *y);
double orc_mlp_loss_grad(const orc_mlp *m, int B, const double *X, const double *T, double *gW1, double *gb1,
                         double *gW2, double *gb2);
int orc_element_features(orc_ctx *c, const double *r, double *X, double *scale);
int orc_mlp_correction(orc_ctx *c, const orc_mlp *m, const double *r, double *corr);
int orc_learned_apply(orc_ctx *c, const double *r, double *z, double lambda, int order, const double *bounds,
                      const orc_mlp *mlp);
int orc_solve3d_learned(orc_ctx *c, const double *y, double *x, double lambda, double tol, int restart, int maxit,
                        int order, const double *bounds, const orc_mlp *mlp, int *iters, int *net_cycles);
/* orc_learned_judge: the polynomial as the judge of the network: solves
 * the same system to tol with the network (orc_solve3d_learned) and with
 * the polynomial alone (orc_solve3d); out[3] = {polynomial iterations,
 * network iterations, accepted}, accepted only if the network's solve
 * converged in fewer iterations.  -6 if the polynomial solve does not. */
int orc_learned_judge(orc_ctx *c, const double *y, double lambda, double tol, int restart, int maxit, int order,
                      const double *bounds, const orc_mlp *mlp, int *out);
/* nsteps 3D-IMEX ARK2 steps (orc_step with L in place of L_V and the Schur
 * GMRES solve to tol; linear as in orc_step).  *iters: GMRES iterations in
 * total. */
int orc_step3d(orc_ctx *c, double *q, double dt, int nsteps, int linear, double tol, int order,
               const double *bounds, int *iters);

#ifdef __cplusplus
}
#endif
#endif
