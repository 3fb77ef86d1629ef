/*
 * numa_oracle.c -- plain FP64 CPU oracle of the HEVI (1D-IMEX) ARK2 step, and
 * of the 3D-IMEX step whose implicit systems are solved by GMRES.
 *
 * TEST INFRASTRUCTURE ONLY (see numa_oracle.h).  Written for reading, not for
 * speed: element-local loops, explicit gather/scatter direct stiffness
 * summation, dense column matrices built by probing and solved with partial
 * pivoting, and the ARK2 stages in their direct form.
 *
 * Readings of the paper that this file adopts (the paper is silent or garbled
 * on them; each is listed with its reason in the design notes):
 *  - continuity in divergence form, d rho'/dt = -div((rho0 + rho') u);
 *  - DSS = mass-weighted average of element-local strong-form values;
 *  - x, y periodic; w = 0 imposed strongly at the bottom and top nodes;
 *  - background in hydrostatic balance: isentropic (theta0 constant,
 *    pi0 = 1 - g z/(cp theta0)) or, with a Brunt-Vaisala frequency Nb > 0,
 *    stratified: theta0(z) = theta0 exp(S z), S = Nb^2/g, and the Exner
 *    function integrated in closed form, pi0 = 1 + g (exp(-S z) - 1)/(cp
 *    theta0 S); in both rho0 = p00 pi0^(cv/R)/(R theta0(z)), P0 =
 *    EOS(rho0, theta0(z));
 *  - ARK2 tableau with the signs restored by the order conditions.
 */
#include "numa_oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

struct orc_ctx {
    int N, nq, nex, ney, nez;
    int nx, ny, nz;
    long nelem, nq3, np;
    double lx, ly, lz, hx, hy;
    double *zf; /* nez+1 element faces */
    double *hz; /* nez element heights */
    double *xi, *wq, *D;
    long *gmap;    /* element-local node -> unique node */
    double *mloc;  /* element-local mass weight m_e */
    double *mass;  /* assembled mass M_I */
    double theta0, p00, cp, R, cv, gamma, g;
    double nbv;                       /* Brunt-Vaisala frequency (0: isentropic) */
    double *zk, *rho0, *P0, *G0, *H0; /* per level */
    double *th0, *th0z;               /* theta0(z) and d theta0/dz per level */
    /* column factors of I - lambda L_V; unknowns per level: rho', w, and
     * theta' when the background is stratified (nvar = 3) */
    int nvar;
    int factored;
    double lambda;
    double *A; /* per column (nvar M)^2, LU in place */
    int *piv;  /* per column nvar M */
};

/* ------------------------------------------------------------------------ */
/* LGL basis (the sD operator of Alg. 1-2).                                  */
/* ------------------------------------------------------------------------ */

/* Legendre P_N(x) and P_N'(x) by the three-term recurrence. */
static void legendre(int N, double x, double *P, double *dP)
{
    double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
    if (N == 0) { *P = 1.0; *dP = 0.0; return; }
    for (int k = 1; k < N; ++k) {
        double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        double d2 = d0 + (2.0 * k + 1.0) * p1; /* P'_{k+1} = P'_{k-1} + (2k+1) P_k */
        p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    *P = p1; *dP = d1;
}

void orc_lgl(int N, double *xi, double *w)
{
    /* Interior nodes are the roots of P_N'; Newton from Chebyshev-Lobatto
     * guesses, with P_N'' from Legendre's equation. */
    xi[0] = -1.0; xi[N] = 1.0;
    for (int i = 1; i < N; ++i) {
        double x = -cos(3.14159265358979323846 * i / N);
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(N, x, &P, &dP);
            double d2P = (2.0 * x * dP - N * (N + 1.0) * P) / (1.0 - x * x);
            double dx = dP / d2P;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        xi[i] = x;
    }
    for (int i = 0; i <= N; ++i) {
        double P, dP;
        legendre(N, xi[i], &P, &dP);
        w[i] = 2.0 / (N * (N + 1.0) * P * P);
    }
}

void orc_dmat(int N, const double *xi, double *D)
{
    int nq = N + 1;
    for (int i = 0; i < nq; ++i) {
        double Pi, dPi;
        legendre(N, xi[i], &Pi, &dPi);
        for (int j = 0; j < nq; ++j) {
            if (i == j) {
                double v = 0.0;
                if (i == 0) v = -N * (N + 1.0) / 4.0;
                if (i == N) v = N * (N + 1.0) / 4.0;
                D[i * nq + j] = v;
            } else {
                double Pj, dPj;
                legendre(N, xi[j], &Pj, &dPj);
                D[i * nq + j] = Pi / (Pj * (xi[i] - xi[j]));
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Set-up: grid, mass, background (Sec. 3.1 background split).              */
/* ------------------------------------------------------------------------ */

static long lidx(const orc_ctx *c, int a, int b, int cc) { return a + c->nq * (b + (long)c->nq * cc); }

orc_ctx *orc_setup(double lx, double ly, double lz, int nex, int ney, int nez,
                   const double *zface, int N, double theta0, double p00,
                   double cp, double rgas, double grav, double nbv)
{
    if (N < 1 || N > 15 || nex < 1 || ney < 1 || nez < 1) return NULL;
    if (!(lx > 0) || !(ly > 0) || !(lz > 0)) return NULL;
    if (!(nbv >= 0.0) || (nbv > 0.0 && !(grav > 0.0))) return NULL;
    if (zface) {
        if (zface[0] != 0.0 || zface[nez] != lz) return NULL;
        for (int e = 0; e < nez; ++e) if (!(zface[e + 1] > zface[e])) return NULL;
    }
    orc_ctx *c = (orc_ctx *)calloc(1, sizeof(orc_ctx));
    if (!c) return NULL;
    c->N = N; c->nq = N + 1; c->nex = nex; c->ney = ney; c->nez = nez;
    c->nx = nex * N; c->ny = ney * N; c->nz = nez * N + 1;
    c->nelem = (long)nex * ney * nez;
    c->nq3 = (long)c->nq * c->nq * c->nq;
    c->np = (long)c->nx * c->ny * c->nz;
    c->lx = lx; c->ly = ly; c->lz = lz;
    c->hx = lx / nex; c->hy = ly / ney;
    c->theta0 = theta0; c->p00 = p00; c->cp = cp; c->R = rgas;
    c->cv = cp - rgas; c->gamma = cp / c->cv; c->g = grav;
    c->nbv = nbv;
    c->nvar = nbv > 0.0 ? 3 : 2;

    c->zf = (double *)malloc(sizeof(double) * (nez + 1));
    c->hz = (double *)malloc(sizeof(double) * nez);
    for (int e = 0; e <= nez; ++e) c->zf[e] = zface ? zface[e] : lz * e / nez;
    c->zf[nez] = lz;
    for (int e = 0; e < nez; ++e) c->hz[e] = c->zf[e + 1] - c->zf[e];

    c->xi = (double *)malloc(sizeof(double) * c->nq);
    c->wq = (double *)malloc(sizeof(double) * c->nq);
    c->D = (double *)malloc(sizeof(double) * c->nq * c->nq);
    orc_lgl(N, c->xi, c->wq);
    orc_dmat(N, c->xi, c->D);

    long nl = c->nelem * c->nq3;
    c->gmap = (long *)malloc(sizeof(long) * nl);
    c->mloc = (double *)malloc(sizeof(double) * nl);
    c->mass = (double *)calloc(c->np, sizeof(double));
    if (!c->gmap || !c->mloc || !c->mass) { orc_free(c); return NULL; }
    for (int ez = 0; ez < nez; ++ez)
        for (int ey = 0; ey < ney; ++ey)
            for (int ex = 0; ex < nex; ++ex) {
                long e = ex + (long)nex * (ey + (long)ney * ez);
                for (int cc = 0; cc <= N; ++cc)
                    for (int b = 0; b <= N; ++b)
                        for (int a = 0; a <= N; ++a) {
                            long l = e * c->nq3 + lidx(c, a, b, cc);
                            long i = (ex * N + a) % c->nx;
                            long j = (ey * N + b) % c->ny;
                            long k = ez * N + cc;
                            c->gmap[l] = i + c->nx * (j + (long)c->ny * k);
                            c->mloc[l] = c->wq[a] * c->wq[b] * c->wq[cc] * c->hx * c->hy * c->hz[ez] / 8.0;
                        }
            }
    for (long l = 0; l < nl; ++l) c->mass[c->gmap[l]] += c->mloc[l];

    c->zk = (double *)malloc(sizeof(double) * c->nz);
    c->rho0 = (double *)malloc(sizeof(double) * c->nz);
    c->P0 = (double *)malloc(sizeof(double) * c->nz);
    c->G0 = (double *)malloc(sizeof(double) * c->nz);
    c->H0 = (double *)malloc(sizeof(double) * c->nz);
    c->th0 = (double *)malloc(sizeof(double) * c->nz);
    c->th0z = (double *)malloc(sizeof(double) * c->nz);
    for (int ez = 0; ez < nez; ++ez)
        for (int cc = 0; cc <= N; ++cc)
            c->zk[ez * N + cc] = c->zf[ez] + (c->xi[cc] + 1.0) * c->hz[ez] / 2.0;
    for (int k = 0; k < c->nz; ++k) {
        /* hydrostatic background: d pi0/dz = -g/(cp theta0(z)), pi0(0) = 1 */
        double z = c->zk[k], th, thz, pi0;
        if (nbv > 0.0) { /* constant Brunt-Vaisala frequency: (g/theta0) d theta0/dz = Nb^2 */
            double S = nbv * nbv / grav;
            th = theta0 * exp(S * z);
            thz = S * th;
            pi0 = 1.0 + grav * (exp(-S * z) - 1.0) / (cp * theta0 * S);
        } else { /* neutral: theta0 constant */
            th = theta0;
            thz = 0.0;
            pi0 = 1.0 - grav * z / (cp * theta0);
        }
        if (!(pi0 > 0.0)) { orc_free(c); return NULL; }
        double rho0 = p00 * pow(pi0, c->cv / rgas) / (rgas * th);
        double P0 = p00 * pow(rho0 * rgas * th / p00, c->gamma); /* EOS, Eq. (10) */
        c->th0[k] = th;
        c->th0z[k] = thz;
        c->rho0[k] = rho0;
        c->P0[k] = P0;
        c->G0[k] = c->gamma * P0 / rho0;   /* Eq. (13) */
        c->H0[k] = c->gamma * P0 / th;
    }
    return c;
}

void orc_free(orc_ctx *c)
{
    if (!c) return;
    free(c->zf); free(c->hz); free(c->xi); free(c->wq); free(c->D);
    free(c->gmap); free(c->mloc); free(c->mass);
    free(c->zk); free(c->rho0); free(c->P0); free(c->G0); free(c->H0);
    free(c->th0); free(c->th0z);
    free(c->A); free(c->piv);
    free(c);
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_sizes(const orc_ctx *c, long *out)
{
    out[0] = c->nx; out[1] = c->ny; out[2] = c->nz; out[3] = c->nelem;
}

void orc_coords(const orc_ctx *c, double *x, double *y, double *z)
{
    for (int ex = 0; ex < c->nex; ++ex)
        for (int a = 0; a < c->N; ++a) x[ex * c->N + a] = ex * c->hx + (c->xi[a] + 1.0) * c->hx / 2.0;
    for (int ey = 0; ey < c->ney; ++ey)
        for (int b = 0; b < c->N; ++b) y[ey * c->N + b] = ey * c->hy + (c->xi[b] + 1.0) * c->hy / 2.0;
    for (int k = 0; k < c->nz; ++k) z[k] = c->zk[k];
}

void orc_mass(const orc_ctx *c, double *M) { memcpy(M, c->mass, sizeof(double) * c->np); }

void orc_background(const orc_ctx *c, double *rho0, double *P0, double *G0, double *H0)
{
    for (int k = 0; k < c->nz; ++k) {
        if (rho0) rho0[k] = c->rho0[k];
        if (P0) P0[k] = c->P0[k];
        if (G0) G0[k] = c->G0[k];
        if (H0) H0[k] = c->H0[k];
    }
}

void orc_background_theta(const orc_ctx *c, double *th0, double *th0z)
{
    memcpy(th0, c->th0, sizeof(double) * c->nz);
    memcpy(th0z, c->th0z, sizeof(double) * c->nz);
}

/* ------------------------------------------------------------------------ */
/* Element-local derivative (Alg. 2 with the box metric 2/h).               */
/* ------------------------------------------------------------------------ */

/* d/dxi along direction dir (0: a, 1: b, 2: c) of an element-local field g at
 * local node (a, b, cc), before the metric factor. */
static double dref(const orc_ctx *c, const double *g, int a, int b, int cc, int dir)
{
    int nq = c->nq;
    double s = 0.0;
    for (int n = 0; n < nq; ++n) {
        if (dir == 0) s += c->D[a * nq + n] * g[lidx(c, n, b, cc)];
        else if (dir == 1) s += c->D[b * nq + n] * g[lidx(c, a, n, cc)];
        else s += c->D[cc * nq + n] * g[lidx(c, a, b, n)];
    }
    return s;
}

/* DSS (Sec. 5.3): R_I = sum_e m_e r_e(I) / M_I over the elements containing I,
 * then w = 0 on the bottom and top levels.  r is element-local [5][nelem*nq3]. */
static void dss(const orc_ctx *c, const double *r, double *R)
{
    long nl = c->nelem * c->nq3;
    memset(R, 0, sizeof(double) * 5 * c->np);
    for (int f = 0; f < 5; ++f)
        for (long l = 0; l < nl; ++l) R[f * c->np + c->gmap[l]] += c->mloc[l] * r[f * nl + l];
    for (int f = 0; f < 5; ++f)
        for (long I = 0; I < c->np; ++I) R[f * c->np + I] /= c->mass[I];
    long plane = (long)c->nx * c->ny;
    for (long I = 0; I < plane; ++I) {
        R[3 * c->np + I] = 0.0;
        R[3 * c->np + (long)(c->nz - 1) * plane + I] = 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Explicit RHS of Set2NC in perturbation form (Sec. 3.1), continuity in    */
/* divergence form.                                                         */
/* ------------------------------------------------------------------------ */

/* P' = EOS(rho0 + rho', theta0 + theta') - P0(z), Eq. (10) with the
 * background split of Sec. 3.1.  Since P0 = EOS(rho0, theta0), the same
 * quantity is P0 [((rho theta)/(rho0 theta0))^gamma - 1]; it is evaluated in
 * that form, with rho theta - rho0 theta0 = rho0 theta' + theta0 rho' +
 * rho' theta', so that two ~1e5 Pa pressures are never subtracted (the
 * subtraction would leave P' with an absolute rounding error of about 1e-11
 * Pa, the whole of P' in a balanced state).  Accuracy: a few ulp of P'. */
static double pressure_perturbation(const orc_ctx *c, int k, double rp, double th)
{
    double r0 = c->rho0[k], t0 = c->th0[k];
    /* rho0 theta', theta0 rho' and rho' theta' nearly cancel in a
     * hydrostatically balanced state; the rounding error of each product is
     * recovered exactly with fma, so that their small sum keeps its relative
     * precision (the partial sums of nearly opposite terms are exact) */
    double p1 = r0 * th, p2 = t0 * rp, p3 = rp * th;
    double e1 = fma(r0, th, -p1), e2 = fma(t0, rp, -p2), e3 = fma(rp, th, -p3);
    double d = ((p1 + p2) + p3) + ((e1 + e2) + e3);
    return c->P0[k] * expm1(c->gamma * log1p(d / (r0 * t0)));
}

int orc_pressure_perturbation(orc_ctx *c, const double *q, double *Pp)
{
    if (!c || !q || !Pp) return -1;
    long plane = (long)c->nx * c->ny;
    for (long I = 0; I < c->np; ++I) {
        int k = (int)(I / plane);
        Pp[I] = pressure_perturbation(c, k, q[0 * c->np + I], q[4 * c->np + I]);
    }
    return 0;
}

int orc_rhs(orc_ctx *c, const double *q, double *R)
{
    if (!c || !q || !R) return -1;
    long nl = c->nelem * c->nq3, nq3 = c->nq3, np = c->np;
    double *r = (double *)malloc(sizeof(double) * 5 * nl);
    if (!r) return -5;
    int ok = 1;
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * 11 * nq3);
        if (!buf) ok = 0;
        if (buf) {
            double *rp = buf, *u = buf + nq3, *v = buf + 2 * nq3, *w = buf + 3 * nq3;
            double *th = buf + 4 * nq3, *rho = buf + 5 * nq3, *Pp = buf + 6 * nq3;
            double *Fx = buf + 7 * nq3, *Fy = buf + 8 * nq3, *Fz = buf + 9 * nq3;
            double *tz0 = buf + 10 * nq3; /* d theta0/dz at the node */
#pragma omp for schedule(static)
            for (long e = 0; e < c->nelem; ++e) {
                int ez = (int)(e / ((long)c->nex * c->ney));
                double sx = 2.0 / c->hx, sy = 2.0 / c->hy, sz = 2.0 / c->hz[ez];
                for (long l = 0; l < nq3; ++l) {
                    long I = c->gmap[e * nq3 + l];
                    int k = (int)(I / ((long)c->nx * c->ny));
                    rp[l] = q[0 * np + I]; u[l] = q[1 * np + I]; v[l] = q[2 * np + I];
                    w[l] = q[3 * np + I]; th[l] = q[4 * np + I];
                    rho[l] = c->rho0[k] + rp[l];
                    Pp[l] = pressure_perturbation(c, k, rp[l], th[l]);
                    Fx[l] = rho[l] * u[l]; Fy[l] = rho[l] * v[l]; Fz[l] = rho[l] * w[l];
                    tz0[l] = c->th0z[k];
                }
                for (int cc = 0; cc < c->nq; ++cc)
                    for (int b = 0; b < c->nq; ++b)
                        for (int a = 0; a < c->nq; ++a) {
                            long l = lidx(c, a, b, cc);
                            double dFx = sx * dref(c, Fx, a, b, cc, 0);
                            double dFy = sy * dref(c, Fy, a, b, cc, 1);
                            double dFz = sz * dref(c, Fz, a, b, cc, 2);
                            double ux = sx * dref(c, u, a, b, cc, 0), uy = sy * dref(c, u, a, b, cc, 1), uz = sz * dref(c, u, a, b, cc, 2);
                            double vx = sx * dref(c, v, a, b, cc, 0), vy = sy * dref(c, v, a, b, cc, 1), vz = sz * dref(c, v, a, b, cc, 2);
                            double wx = sx * dref(c, w, a, b, cc, 0), wy = sy * dref(c, w, a, b, cc, 1), wz = sz * dref(c, w, a, b, cc, 2);
                            double tx = sx * dref(c, th, a, b, cc, 0), ty = sy * dref(c, th, a, b, cc, 1), tz = sz * dref(c, th, a, b, cc, 2);
                            double px = sx * dref(c, Pp, a, b, cc, 0), py = sy * dref(c, Pp, a, b, cc, 1), pz = sz * dref(c, Pp, a, b, cc, 2);
                            double U = u[l], V = v[l], W = w[l], rh = rho[l];
                            long o = e * nq3 + l;
                            r[0 * nl + o] = -(dFx + dFy + dFz);
                            r[1 * nl + o] = -(U * ux + V * uy + W * uz + px / rh);
                            r[2 * nl + o] = -(U * vx + V * vy + W * vz + py / rh);
                            r[3 * nl + o] = -(U * wx + V * wy + W * wz + pz / rh + c->g * rp[l] / rh);
                            /* u . grad theta0 = w d theta0/dz (theta0 depends on z only) */
                            r[4 * nl + o] = -(U * tx + V * ty + W * tz + W * tz0[l]);
                        }
            }
            free(buf);
        }
    }
    if (!ok) { free(r); return -5; }
    dss(c, r, R);
    free(r);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Linear operators (Sec. 3.1): P'_lin = G0 rho' + H0 theta' (Eq. (13)).     */
/* full = 0: vertical part L_V only (Eq. (4)); full = 1: the whole L.        */
/* ------------------------------------------------------------------------ */

static int linop(orc_ctx *c, const double *q, double *L, int full)
{
    if (!c || !q || !L) return -1;
    long nl = c->nelem * c->nq3, nq3 = c->nq3, np = c->np;
    double *r = (double *)malloc(sizeof(double) * 5 * nl);
    if (!r) return -5;
    int ok = 1;
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * 7 * nq3);
        if (!buf) ok = 0;
        if (buf) {
            double *rp = buf, *mu = buf + nq3, *mv = buf + 2 * nq3, *mw = buf + 3 * nq3;
            double *pl = buf + 4 * nq3, *r0 = buf + 5 * nq3, *wt = buf + 6 * nq3;
#pragma omp for schedule(static)
            for (long e = 0; e < c->nelem; ++e) {
                int ez = (int)(e / ((long)c->nex * c->ney));
                double sx = 2.0 / c->hx, sy = 2.0 / c->hy, sz = 2.0 / c->hz[ez];
                for (long l = 0; l < nq3; ++l) {
                    long I = c->gmap[e * nq3 + l];
                    int k = (int)(I / ((long)c->nx * c->ny));
                    r0[l] = c->rho0[k];
                    rp[l] = q[0 * np + I];
                    mu[l] = c->rho0[k] * q[1 * np + I];
                    mv[l] = c->rho0[k] * q[2 * np + I];
                    mw[l] = c->rho0[k] * q[3 * np + I];
                    pl[l] = c->G0[k] * q[0 * np + I] + c->H0[k] * q[4 * np + I];
                    wt[l] = q[3 * np + I] * c->th0z[k];
                }
                for (int cc = 0; cc < c->nq; ++cc)
                    for (int b = 0; b < c->nq; ++b)
                        for (int a = 0; a < c->nq; ++a) {
                            long l = lidx(c, a, b, cc), o = e * nq3 + l;
                            double div = sz * dref(c, mw, a, b, cc, 2);
                            if (full) div += sx * dref(c, mu, a, b, cc, 0) + sy * dref(c, mv, a, b, cc, 1);
                            r[0 * nl + o] = -div;
                            r[1 * nl + o] = full ? -(sx * dref(c, pl, a, b, cc, 0) / r0[l]) : 0.0;
                            r[2 * nl + o] = full ? -(sy * dref(c, pl, a, b, cc, 1) / r0[l]) : 0.0;
                            r[3 * nl + o] = -(sz * dref(c, pl, a, b, cc, 2) / r0[l] + c->g * rp[l] / r0[l]);
                            r[4 * nl + o] = -wt[l]; /* -u . grad theta0 = -w d theta0/dz */
                        }
            }
            free(buf);
        }
    }
    if (!ok) { free(r); return -5; }
    dss(c, r, L);
    free(r);
    return 0;
}

int orc_lv(orc_ctx *c, const double *q, double *L) { return linop(c, q, L, 0); }
int orc_lfull(orc_ctx *c, const double *q, double *L) { return linop(c, q, L, 1); }

/* ------------------------------------------------------------------------ */
/* Column matrices of I - lambda L_V (Sec. 5.4): built by probing (Alg. 7),  */
/* unknowns (rho'_k, w_k) per column, and theta'_k when the background is    */
/* stratified, solved by Gaussian elimination with partial pivoting.  u, v  */
/* pass through unchanged because L_V has no rows for them; so does theta'  */
/* over a neutral background, where its row -w d theta0/dz vanishes.       */
/* ------------------------------------------------------------------------ */

/* field of column unknown block gv: rho', w, theta' */
static int unknown_field(int gv) { return gv == 0 ? 0 : (gv == 1 ? 3 : 4); }

static int build_columns(orc_ctx *c, double lambda, double *A)
{
    int M = c->nz, nv = c->nvar, n2 = nv * M;
    long plane = (long)c->nx * c->ny, np = c->np;
    double *P = (double *)calloc(5 * np, sizeof(double));
    double *L = (double *)malloc(sizeof(double) * 5 * np);
    if (!P || !L) { free(P); free(L); return -5; }
    for (int gvar = 0; gvar < nv; ++gvar) {
        int f = unknown_field(gvar);
        for (int m = 0; m < M; ++m) {
            /* unit value of dof (gvar, m) in every column at once */
            for (long I = 0; I < plane; ++I) P[f * np + (long)m * plane + I] = 1.0;
            int rc = orc_lv(c, P, L);
            for (long I = 0; I < plane; ++I) P[f * np + (long)m * plane + I] = 0.0;
            if (rc) { free(P); free(L); return rc; }
            int col = gvar * M + m;
            for (long I = 0; I < plane; ++I) {
                double *Ac = A + I * (long)n2 * n2;
                for (int rv = 0; rv < nv; ++rv)
                    for (int k = 0; k < M; ++k) {
                        int row = rv * M + k;
                        Ac[(long)row * n2 + col] =
                            (col == row ? 1.0 : 0.0) - lambda * L[unknown_field(rv) * np + (long)k * plane + I];
                    }
            }
        }
    }
    free(P); free(L);
    /* w = 0 is imposed strongly on the bottom and top nodes: those two w
     * values are not unknowns.  Their rows are already identity rows (L_V has
     * no w tendency there); clearing their columns as well decouples them, so
     * the solve returns them as exactly y_w = 0. */
    for (long I = 0; I < plane; ++I) {
        double *Ac = A + I * (long)n2 * n2;
        int wall[2] = {M, 2 * M - 1};
        for (int t = 0; t < 2; ++t)
            for (int r = 0; r < n2; ++r)
                if (r != wall[t]) Ac[(long)r * n2 + wall[t]] = 0.0;
    }
    return 0;
}

int orc_column_matrix(orc_ctx *c, double lambda, int i, int j, double *Aout)
{
    if (!c || !Aout || i < 0 || j < 0 || i >= c->nx || j >= c->ny) return -1;
    int n2 = c->nvar * c->nz;
    long plane = (long)c->nx * c->ny;
    double *A = (double *)malloc(sizeof(double) * plane * n2 * n2);
    if (!A) return -5;
    int rc = build_columns(c, lambda, A);
    if (!rc) memcpy(Aout, A + ((long)i + (long)c->nx * j) * n2 * n2, sizeof(double) * n2 * n2);
    free(A);
    return rc;
}

/* In-place LU with partial pivoting of an n x n row-major matrix. */
static int lu_pp(double *A, int *piv, int n)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = fabs(A[k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (fabs(A[i * n + k]) > best) { best = fabs(A[i * n + k]); p = i; }
        piv[k] = p;
        if (best == 0.0) return -4;
        if (p != k)
            for (int j = 0; j < n; ++j) { double t = A[k * n + j]; A[k * n + j] = A[p * n + j]; A[p * n + j] = t; }
        for (int i = k + 1; i < n; ++i) {
            A[i * n + k] /= A[k * n + k];
            double m = A[i * n + k];
            for (int j = k + 1; j < n; ++j) A[i * n + j] -= m * A[k * n + j];
        }
    }
    return 0;
}

static void lu_solve(const double *A, const int *piv, int n, double *x)
{
    for (int k = 0; k < n; ++k)
        if (piv[k] != k) { double t = x[k]; x[k] = x[piv[k]]; x[piv[k]] = t; }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) x[i] -= A[i * n + j] * x[j];
    for (int i = n - 1; i >= 0; --i) {
        for (int j = i + 1; j < n; ++j) x[i] -= A[i * n + j] * x[j];
        x[i] /= A[i * n + i];
    }
}

int orc_factor(orc_ctx *c, double lambda)
{
    if (!c) return -1;
    int n2 = c->nvar * c->nz;
    long plane = (long)c->nx * c->ny;
    free(c->A); free(c->piv);
    c->factored = 0;
    c->A = (double *)malloc(sizeof(double) * plane * n2 * n2);
    c->piv = (int *)malloc(sizeof(int) * plane * n2);
    if (!c->A || !c->piv) return -5;
    int rc = build_columns(c, lambda, c->A);
    if (rc) return rc;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long I = 0; I < plane; ++I)
        if (lu_pp(c->A + I * (long)n2 * n2, c->piv + I * n2, n2)) bad = 1;
    if (bad) return -4;
    c->factored = 1;
    c->lambda = lambda;
    return 0;
}

int orc_solve(orc_ctx *c, const double *y, double *x)
{
    if (!c || !y || !x) return -1;
    if (!c->factored) return -2;
    int M = c->nz, nv = c->nvar, n2 = nv * M;
    long plane = (long)c->nx * c->ny, np = c->np;
    for (long I = 0; I < plane; ++I)
        if (y[3 * np + I] != 0.0 || y[3 * np + (long)(M - 1) * plane + I] != 0.0) return -3;
    /* Over a neutral background theta' is known (x_theta = y_theta): its L_V
     * contribution moves to the right-hand side and the (rho', w) system is
     * solved column by column; over a stratified one theta' is an unknown. */
    double *t = (double *)calloc(5 * np, sizeof(double));
    double *Lt = (double *)calloc(5 * np, sizeof(double));
    if (!t || !Lt) { free(t); free(Lt); return -5; }
    if (nv == 2) {
        memcpy(t + 4 * np, y + 4 * np, sizeof(double) * np);
        int rc = orc_lv(c, t, Lt);
        if (rc) { free(t); free(Lt); return rc; }
    }
    double lam = c->lambda;
#pragma omp parallel
    {
        double *b = (double *)malloc(sizeof(double) * n2);
#pragma omp for schedule(static)
        for (long I = 0; I < plane; ++I) {
            for (int gv = 0; gv < nv; ++gv)
                for (int k = 0; k < M; ++k) {
                    long o = unknown_field(gv) * np + (long)k * plane + I;
                    b[gv * M + k] = y[o] + lam * Lt[o];
                }
            lu_solve(c->A + I * (long)n2 * n2, c->piv + I * n2, n2, b);
            for (int gv = 0; gv < nv; ++gv)
                for (int k = 0; k < M; ++k) t[unknown_field(gv) * np + (long)k * plane + I] = b[gv * M + k];
        }
        free(b);
    }
    for (long I = 0; I < np; ++I) {
        x[0 * np + I] = t[0 * np + I];
        x[1 * np + I] = y[1 * np + I];
        x[2 * np + I] = y[2 * np + I];
        x[3 * np + I] = t[3 * np + I];
        x[4 * np + I] = nv == 3 ? t[4 * np + I] : y[4 * np + I];
    }
    free(t); free(Lt);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* ARK2 (Sec. 2.2, Table 1), direct stage form:                             */
/*   Q_i = q^n + dt sum_{j<i} [a_ij R_j + (at_ij - a_ij) L_j] + at_ii dt L(Q_i) */
/*   q^{n+1} = q^n + dt sum_i b_i R_i          (b = bt)                     */
/* ------------------------------------------------------------------------ */

void orc_ark2_tableau(double *a, double *at, double *b)
{
    double s2 = sqrt(2.0);
    double alpha = (3.0 + 2.0 * s2) / 6.0;
    double d = 1.0 - 1.0 / s2;
    memset(a, 0, sizeof(double) * 9);
    memset(at, 0, sizeof(double) * 9);
    a[1 * 3 + 0] = 2.0 - s2;
    a[2 * 3 + 0] = 1.0 - alpha;
    a[2 * 3 + 1] = alpha;
    at[1 * 3 + 0] = d; at[1 * 3 + 1] = d;
    at[2 * 3 + 0] = 1.0 / (2.0 * s2); at[2 * 3 + 1] = 1.0 / (2.0 * s2); at[2 * 3 + 2] = d;
    b[0] = 1.0 / (2.0 * s2); b[1] = 1.0 / (2.0 * s2); b[2] = d;
}

int orc_step(orc_ctx *c, double *q, double dt, int nsteps, int linear)
{
    if (!c || !q || nsteps < 0) return -1;
    double a[9], at[9], b[3];
    orc_ark2_tableau(a, at, b);
    double lam = at[1 * 3 + 1] * dt;
    if (!c->factored || c->lambda != lam) return -2;
    long n5 = 5 * c->np;
    double *Rs[3], *Ls[2], *Y = (double *)malloc(sizeof(double) * n5);
    double *Q = (double *)malloc(sizeof(double) * n5);
    for (int s = 0; s < 3; ++s) Rs[s] = (double *)malloc(sizeof(double) * n5);
    for (int s = 0; s < 2; ++s) Ls[s] = (double *)malloc(sizeof(double) * n5);
    int rc = (Y && Q && Rs[0] && Rs[1] && Rs[2] && Ls[0] && Ls[1]) ? 0 : -5;
    for (int n = 0; n < nsteps && !rc; ++n) {
        for (int i = 0; i < 3 && !rc; ++i) {
            if (i == 0) {
                memcpy(Q, q, sizeof(double) * n5);
            } else {
                for (long I = 0; I < n5; ++I) {
                    double y = q[I];
                    for (int j = 0; j < i; ++j)
                        y += dt * (a[i * 3 + j] * Rs[j][I] + (at[i * 3 + j] - a[i * 3 + j]) * Ls[j][I]);
                    Y[I] = y;
                }
                rc = orc_solve(c, Y, Q);
                if (rc) break;
            }
            rc = linear ? orc_lfull(c, Q, Rs[i]) : orc_rhs(c, Q, Rs[i]);
            if (!rc && i < 2) rc = orc_lv(c, Q, Ls[i]);
        }
        if (rc) break;
        for (long I = 0; I < n5; ++I) q[I] += dt * (b[0] * Rs[0][I] + b[1] * Rs[1][I] + b[2] * Rs[2][I]);
    }
    free(Y); free(Q);
    for (int s = 0; s < 3; ++s) free(Rs[s]);
    for (int s = 0; s < 2; ++s) free(Ls[s]);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* 3D-IMEX (Sec. 2): the implicit part is the whole linear operator L of    */
/* Sec. 3.1 instead of its vertical part L_V, and the implicit systems are  */
/* solved iteratively (Sec. 5.5).                                           */
/* ------------------------------------------------------------------------ */

static double dot_n(const double *a, const double *b, long n)
{
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* An operator on vectors of length n, and restarted right-preconditioned
 * GMRES(m) for it: textbook Arnoldi with modified Gram-Schmidt, Givens
 * rotations of the Hessenberg matrix, x0 = 0.  Inside a cycle the rotated
 * right-hand side gives the residual norm; a cycle ends when that estimate
 * reaches tol |b| or after m iterations, and the solve ends when the true
 * residual |b - A x| reaches tol |b|.  *iters counts Arnoldi iterations. */
typedef int (*orc_op_fn)(orc_ctx *c, const void *arg, const double *in, double *out);

/* guard (flexible only, may be NULL): called with the residual norms before
 * and after each restart cycle; it may change what M does from then on */
typedef void (*orc_guard_fn)(const void *marg, double before, double after);

static int gmres_impl(orc_ctx *c, long n, orc_op_fn A, const void *aarg, orc_op_fn M, const void *marg,
                      const double *b, double *x, double tol, int m, int maxit, int flexible, orc_guard_fn guard,
                      int *iters)
{
    double prev = -1.0;
    int total = 0, rc = 0, converged = 0;
    /* flexible: keep z_j = M v_j and update x with them (M may change with
     * its argument, as a nonlinear preconditioner does) */
    double *Z = flexible ? (double *)malloc(sizeof(double) * (size_t)m * n) : NULL;
    double *V = (double *)malloc(sizeof(double) * (size_t)(m + 1) * n);
    double *w = (double *)malloc(sizeof(double) * n), *z = (double *)malloc(sizeof(double) * n);
    double *H = (double *)calloc((size_t)(m + 1) * m, sizeof(double));
    double *cs = (double *)malloc(sizeof(double) * m), *sn = (double *)malloc(sizeof(double) * m);
    double *g = (double *)malloc(sizeof(double) * (m + 1)), *yv = (double *)malloc(sizeof(double) * m);
    if (!V || !w || !z || !H || !cs || !sn || !g || !yv || (flexible && !Z)) rc = -5;
    double bnorm = rc ? 0.0 : sqrt(dot_n(b, b, n));
    if (!rc) memset(x, 0, sizeof(double) * n);
    while (!rc) {
        /* true residual r = b - A x */
        rc = A(c, aarg, x, w);
        if (rc) break;
        for (long i = 0; i < n; ++i) w[i] = b[i] - w[i];
        double beta = sqrt(dot_n(w, w, n));
        if (guard && prev >= 0.0) guard(marg, prev, beta);
        prev = beta;
        if (beta <= tol * bnorm) { converged = 1; break; }
        if (total >= maxit) break;
        for (long i = 0; i < n; ++i) V[i] = w[i] / beta;
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        int j = 0;
        while (j < m && total < maxit) {
            double *vj = V + (size_t)j * n, *vn = V + (size_t)(j + 1) * n;
            double *zj = flexible ? Z + (size_t)j * n : z;
            if (M) { rc = M(c, marg, vj, zj); if (rc) break; }
            rc = A(c, aarg, M ? zj : vj, w);
            if (rc) break;
            for (int i = 0; i <= j; ++i) {
                double *vi = V + (size_t)i * n;
                double h = dot_n(w, vi, n);
                H[i * m + j] = h;
                for (long l = 0; l < n; ++l) w[l] -= h * vi[l];
            }
            double hn = sqrt(dot_n(w, w, n));
            H[(j + 1) * m + j] = hn;
            for (long l = 0; l < n; ++l) vn[l] = hn > 0.0 ? w[l] / hn : 0.0;
            for (int i = 0; i < j; ++i) {
                double a = H[i * m + j], bb = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * bb;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
            }
            double a = H[j * m + j], bb = H[(j + 1) * m + j], r = hypot(a, bb);
            cs[j] = r > 0.0 ? a / r : 1.0;
            sn[j] = r > 0.0 ? bb / r : 0.0;
            H[j * m + j] = r;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++total;
            ++j;
            if (fabs(g[j]) <= tol * bnorm) break;
        }
        if (rc) break;
        /* x += M V y with H[0:j,0:j] y = g[0:j] */
        for (int i = j - 1; i >= 0; --i) {
            double t = g[i];
            for (int k = i + 1; k < j; ++k) t -= H[i * m + k] * yv[k];
            yv[i] = t / H[i * m + i];
        }
        if (flexible) { /* x += Z y */
            for (int i = 0; i < j; ++i) {
                double *zi = Z + (size_t)i * n;
                for (long l = 0; l < n; ++l) x[l] += yv[i] * zi[l];
            }
            continue;
        }
        memset(w, 0, sizeof(double) * n);
        for (int i = 0; i < j; ++i) {
            double *vi = V + (size_t)i * n;
            for (long l = 0; l < n; ++l) w[l] += yv[i] * vi[l];
        }
        if (M) { rc = M(c, marg, w, z); if (rc) break; }
        const double *dx = M ? z : w;
        for (long l = 0; l < n; ++l) x[l] += dx[l];
    }
    if (iters) *iters = total;
    free(Z); free(V); free(w); free(z); free(H); free(cs); free(sn); free(g); free(yv);
    if (rc) return rc;
    return converged ? 0 : -6;
}

static int gmres(orc_ctx *c, long n, orc_op_fn A, const void *aarg, orc_op_fn M, const void *marg,
                 const double *b, double *x, double tol, int m, int maxit, int *iters)
{
    return gmres_impl(c, n, A, aarg, M, marg, b, x, tol, m, maxit, 0, NULL, iters);
}

/* Standard (unreduced) form: (I - lambda L) x = y on all five fields. */
static int op_standard(orc_ctx *c, const void *arg, const double *v, double *w)
{
    double lambda = *(const double *)arg;
    int rc = orc_lfull(c, v, w);
    if (rc) return rc;
    for (long i = 0; i < 5 * c->np; ++i) w[i] = v[i] - lambda * w[i];
    return 0;
}

int orc_solve3d_standard(orc_ctx *c, const double *y, double *x, double lambda, double tol, int restart, int maxit,
                         int *iters)
{
    if (!c || !y || !x || restart < 1 || maxit < 1 || !(tol > 0.0)) return -1;
    return gmres(c, 5 * c->np, op_standard, &lambda, NULL, NULL, y, x, tol, restart, maxit, iters);
}

/* Schur-complement form (the Set2NC analogue of the pressure system of
 * Algs. 4-5).  With theta' = y_theta fixed (L has no theta' tendency for a
 * constant theta0) and the linear pressure P = G0 rho' + H0 theta', the
 * velocity rows of (I - lambda L) x = y give
 *     u = U_a - U_p(P),  U_a = (y_u, y_v, B (y_w + lambda g H0 y_theta/(G0 rho0))),
 *     U_p(P) = lambda (Dx P/rho0, Dy P/rho0, B (Dz P/rho0 + g P/(G0 rho0))),
 * B zeroing w on the bottom and top.  U_p is -lambda times the velocity
 * tendencies of L applied to the state (rho' = P/G0, u = 0, theta' = 0).
 * The continuity row times G0, plus H0 y_theta, then reads
 *     S P = P - lambda G0 div(rho0 U_p(P)) = G0 y_rho + H0 y_theta - lambda G0 div(rho0 U_a),
 * where -div(rho0 U) is the rho' tendency of L applied to (0, U, 0). */
typedef struct {
    double lambda;
    double *s, *l; /* 5-field scratch states */
} schur_arg;

/* U_p(P) into the velocity fields of l (rho', theta' of l are cleared) */
static int schur_up(orc_ctx *c, const schur_arg *a, const double *P, double *out_u)
{
    long np = c->np, plane = (long)c->nx * c->ny;
    memset(a->s, 0, sizeof(double) * 5 * np);
    for (long I = 0; I < np; ++I) a->s[I] = P[I] / c->G0[I / plane];
    int rc = orc_lfull(c, a->s, a->l);
    if (rc) return rc;
    for (long I = 0; I < 3 * np; ++I) out_u[I] = -a->lambda * a->l[np + I];
    return 0;
}

/* -div(rho0 U) for a velocity field U (3 fields) */
static int schur_div(orc_ctx *c, const schur_arg *a, const double *U, double *out)
{
    long np = c->np;
    memset(a->s, 0, sizeof(double) * 5 * np);
    memcpy(a->s + np, U, sizeof(double) * 3 * np);
    int rc = orc_lfull(c, a->s, a->l);
    if (rc) return rc;
    memcpy(out, a->l, sizeof(double) * np);
    return 0;
}

static int op_schur(orc_ctx *c, const void *arg, const double *P, double *out)
{
    const schur_arg *a = (const schur_arg *)arg;
    long np = c->np, plane = (long)c->nx * c->ny;
    double *U = (double *)malloc(sizeof(double) * 3 * np);
    if (!U) return -5;
    int rc = schur_up(c, a, P, U);
    if (!rc) rc = schur_div(c, a, U, out); /* out = -div(rho0 U_p) */
    if (!rc)
        for (long I = 0; I < np; ++I) out[I] = P[I] + a->lambda * c->G0[I / plane] * out[I];
    free(U);
    return rc;
}

/* U_a and the Schur right-hand side b */
static int schur_rhs(orc_ctx *c, const schur_arg *a, const double *y, double *Ua, double *b)
{
    long np = c->np, plane = (long)c->nx * c->ny;
    for (long I = 0; I < np; ++I) {
        int k = (int)(I / plane);
        Ua[I] = y[np + I];
        Ua[np + I] = y[2 * np + I];
        Ua[2 * np + I] = (k == 0 || k == c->nz - 1) ? 0.0
                         : y[3 * np + I] + a->lambda * c->g * c->H0[k] * y[4 * np + I] / (c->G0[k] * c->rho0[k]);
    }
    int rc = schur_div(c, a, Ua, b);
    if (rc) return rc;
    for (long I = 0; I < np; ++I) {
        int k = (int)(I / plane);
        b[I] = c->G0[k] * y[I] + c->H0[k] * y[4 * np + I] + a->lambda * c->G0[k] * b[I];
    }
    return 0;
}

int orc_schur_apply(orc_ctx *c, const double *P, double *out, double lambda)
{
    if (!c || !P || !out) return -1;
    if (c->nbv > 0.0) return -7;
    schur_arg a = {lambda, (double *)malloc(sizeof(double) * 5 * c->np), (double *)malloc(sizeof(double) * 5 * c->np)};
    int rc = (a.s && a.l) ? op_schur(c, &a, P, out) : -5;
    free(a.s); free(a.l);
    return rc;
}

int orc_schur_rhs(orc_ctx *c, const double *y, double *b, double lambda)
{
    if (!c || !y || !b) return -1;
    if (c->nbv > 0.0) return -7;
    long np = c->np;
    schur_arg a = {lambda, (double *)malloc(sizeof(double) * 5 * np), (double *)malloc(sizeof(double) * 5 * np)};
    double *Ua = (double *)malloc(sizeof(double) * 3 * np);
    int rc = (a.s && a.l && Ua) ? schur_rhs(c, &a, y, Ua, b) : -5;
    free(a.s); free(a.l); free(Ua);
    return rc;
}

/* PBNO preconditioner (Sec. 5.5): a polynomial s(S) that approximates S^-1
 * on the eigenvalue interval [lmin, lmax].  Its coefficients are those of
 * Chebyshev acceleration (the polynomial of degree p for which 1 - x s(x) is
 * the scaled and shifted Chebyshev polynomial T_{p+1}, minimax on the
 * interval), applied by the three-term recurrence of the Chebyshev
 * iteration for S z = r from z = 0: p applications of S.  For p = 0 it is
 * the scaling 2/(lmin + lmax) alone. */
typedef struct {
    schur_arg *s;
    int p;
    double lmin, lmax;
} pbno_arg;

static int op_pbno(orc_ctx *c, const void *arg, const double *r, double *z)
{
    const pbno_arg *a = (const pbno_arg *)arg;
    long n = c->np;
    double theta = 0.5 * (a->lmax + a->lmin), delta = 0.5 * (a->lmax - a->lmin);
    double sigma = theta / delta, rho = 1.0 / sigma;
    double *res = (double *)malloc(sizeof(double) * n), *d = (double *)malloc(sizeof(double) * n);
    double *Sd = (double *)malloc(sizeof(double) * n);
    int rc = (res && d && Sd) ? 0 : -5;
    if (!rc) {
        for (long i = 0; i < n; ++i) {
            res[i] = r[i];
            d[i] = r[i] / theta;
            z[i] = 0.0;
        }
        for (int k = 0; k <= a->p; ++k) {
            for (long i = 0; i < n; ++i) z[i] += d[i];
            if (k == a->p) break;
            rc = op_schur(c, a->s, d, Sd);
            if (rc) break;
            double rho_n = 1.0 / (2.0 * sigma - rho);
            for (long i = 0; i < n; ++i) {
                res[i] -= Sd[i];
                d[i] = rho_n * rho * d[i] + (2.0 * rho_n / delta) * res[i];
            }
            rho = rho_n;
        }
    }
    free(res); free(d); free(Sd);
    return rc;
}

int orc_pbno_apply(orc_ctx *c, const double *r, double *z, double lambda, int order, double lmin, double lmax)
{
    if (!c || !r || !z || order < 0 || !(lmax > lmin) || !(lmin > 0.0)) return -1;
    if (c->nbv > 0.0) return -7;
    schur_arg s = {lambda, (double *)malloc(sizeof(double) * 5 * c->np), (double *)malloc(sizeof(double) * 5 * c->np)};
    pbno_arg a = {&s, order, lmin, lmax};
    int rc = (s.s && s.l) ? op_pbno(c, &a, r, z) : -5;
    free(s.s); free(s.l);
    return rc;
}

/* Eigenvalue interval of S for the preconditioner: lmin = 1 (S is the
 * identity plus lambda^2 times an operator with a non-negative spectrum up
 * to the small buoyancy coupling), lmax = 1.1 |S^k v| / |S^(k-1) v| after k
 * power-method steps from v_I = frac(I phi) - 1/2, phi the golden-ratio
 * fraction taken as 2654435769 / 2^32 (integer arithmetic, so both
 * implementations start from the same vector). */
int orc_schur_bounds(orc_ctx *c, double lambda, int k, double *out)
{
    if (!c || !out || k < 1) return -1;
    if (c->nbv > 0.0) return -7;
    long n = c->np;
    double *v = (double *)malloc(sizeof(double) * n), *w = (double *)malloc(sizeof(double) * n);
    schur_arg a = {lambda, (double *)malloc(sizeof(double) * 5 * n), (double *)malloc(sizeof(double) * 5 * n)};
    int rc = (v && w && a.s && a.l) ? 0 : -5;
    double est = 0.0;
    if (!rc) {
        for (long i = 0; i < n; ++i) {
            uint32_t h = (uint32_t)((uint64_t)i * 2654435769u);
            v[i] = (double)h / 4294967296.0 - 0.5;
        }
        double nv = sqrt(dot_n(v, v, n));
        for (long i = 0; i < n; ++i) v[i] /= nv;
        for (int it = 0; it < k && !rc; ++it) {
            rc = op_schur(c, &a, v, w);
            if (rc) break;
            est = sqrt(dot_n(w, w, n));
            for (long i = 0; i < n; ++i) v[i] = w[i] / est;
        }
    }
    out[0] = 1.0;
    out[1] = 1.1 * est;
    free(v); free(w); free(a.s); free(a.l);
    return rc;
}

/* x = (I - lambda L)^-1 y through the Schur form: b, GMRES on S P = b with
 * PBNO of the given order (order < 0: none) on the interval bounds, then
 * u = U_a - U_p(P), rho' = y_rho - lambda div(rho0 u), theta' = y_theta. */
int orc_solve3d(orc_ctx *c, const double *y, double *x, double lambda, double tol, int restart, int maxit,
                int order, const double *bounds, int *iters)
{
    if (!c || !y || !x || restart < 1 || maxit < 1 || !(tol > 0.0)) return -1;
    if (c->nbv > 0.0) return -7;
    if (order >= 0 && (!bounds || !(bounds[1] > bounds[0]) || !(bounds[0] > 0.0))) return -1;
    long np = c->np;
    schur_arg a = {lambda, (double *)malloc(sizeof(double) * 5 * np), (double *)malloc(sizeof(double) * 5 * np)};
    double *Ua = (double *)malloc(sizeof(double) * 3 * np), *Up = (double *)malloc(sizeof(double) * 3 * np);
    double *b = (double *)malloc(sizeof(double) * np), *P = (double *)malloc(sizeof(double) * np);
    int rc = (a.s && a.l && Ua && Up && b && P) ? 0 : -5, it = 0, grc = 0;
    pbno_arg pa = {&a, order, bounds ? bounds[0] : 0.0, bounds ? bounds[1] : 0.0};
    if (!rc) rc = schur_rhs(c, &a, y, Ua, b);
    if (!rc) {
        grc = gmres(c, np, op_schur, &a, order >= 0 ? op_pbno : NULL, &pa, b, P, tol, restart, maxit, &it);
        if (grc && grc != -6) rc = grc;
    }
    if (!rc) rc = schur_up(c, &a, P, Up);
    if (!rc) {
        for (long I = 0; I < 3 * np; ++I) x[np + I] = Ua[I] - Up[I];
        rc = schur_div(c, &a, x + np, x); /* x_rho = -div(rho0 u) */
    }
    if (!rc)
        for (long I = 0; I < np; ++I) {
            x[I] = y[I] + lambda * x[I];
            x[4 * np + I] = y[4 * np + I];
        }
    if (iters) *iters = it;
    free(a.s); free(a.l); free(Ua); free(Up); free(b); free(P);
    return rc ? rc : grc;
}

/* ------------------------------------------------------------------------ */
/* Learned correction to the PBNO preconditioner (a project addition; the   */
/* paper's preconditioners are polynomial).  A two-layer perceptron acts on */
/* each element's residual: x = r_e / s_e with s_e the RMS of r_e over the  */
/* element's (N+1)^3 nodes (local order a + nq (b + nq c)), h = tanh(W1 x + */
/* b1), y = W2 h + b2, correction s_e y; the corrections of the elements    */
/* sharing a node are averaged.  The preconditioner is z = s(S) r + that    */
/* average, nonlinear in r, hence flexible GMRES.                           */
/* ------------------------------------------------------------------------ */

void orc_mlp_forward(const orc_mlp *m, const double *x, double *h, double *y)
{
    for (int k = 0; k < m->nh; ++k) {
        double t = m->b1[k];
        for (int i = 0; i < m->nin; ++i) t += m->W1[(long)k * m->nin + i] * x[i];
        h[k] = tanh(t);
    }
    for (int o = 0; o < m->nin; ++o) {
        double t = m->b2[o];
        for (int k = 0; k < m->nh; ++k) t += m->W2[(long)o * m->nh + k] * h[k];
        y[o] = t;
    }
}

/* Loss = mean over the B samples and nin outputs of (y - t)^2, and its
 * gradient with respect to W1, b1, W2, b2 by the chain rule. */
double orc_mlp_loss_grad(const orc_mlp *m, int B, const double *X, const double *T, double *gW1, double *gb1,
                         double *gW2, double *gb2)
{
    int ni = m->nin, nh = m->nh;
    memset(gW1, 0, sizeof(double) * nh * ni);
    memset(gb1, 0, sizeof(double) * nh);
    memset(gW2, 0, sizeof(double) * ni * nh);
    memset(gb2, 0, sizeof(double) * ni);
    double *h = (double *)malloc(sizeof(double) * nh), *y = (double *)malloc(sizeof(double) * ni);
    double *dy = (double *)malloc(sizeof(double) * ni), *dh = (double *)malloc(sizeof(double) * nh);
    double loss = 0.0, scale = 1.0 / ((double)B * ni);
    for (int s = 0; s < B; ++s) {
        const double *x = X + (long)s * ni, *t = T + (long)s * ni;
        orc_mlp_forward(m, x, h, y);
        for (int o = 0; o < ni; ++o) {
            double d = y[o] - t[o];
            loss += d * d * scale;
            dy[o] = 2.0 * d * scale;
            gb2[o] += dy[o];
            for (int k = 0; k < nh; ++k) gW2[(long)o * nh + k] += dy[o] * h[k];
        }
        for (int k = 0; k < nh; ++k) {
            double t2 = 0.0;
            for (int o = 0; o < ni; ++o) t2 += m->W2[(long)o * nh + k] * dy[o];
            dh[k] = t2 * (1.0 - h[k] * h[k]);
            gb1[k] += dh[k];
            for (int i = 0; i < ni; ++i) gW1[(long)k * ni + i] += dh[k] * x[i];
        }
    }
    free(h); free(y); free(dy); free(dh);
    return loss;
}

/* element features of a field: X[e][nq3] = r_e / s_e, scale[e] = s_e */
int orc_element_features(orc_ctx *c, const double *r, double *X, double *scale)
{
    if (!c || !r || !X || !scale) return -1;
    long nq3 = c->nq3;
    for (long e = 0; e < c->nelem; ++e) {
        double ss = 0.0;
        for (long l = 0; l < nq3; ++l) {
            double v = r[c->gmap[e * nq3 + l]];
            ss += v * v;
        }
        double s_e = sqrt(ss / (double)nq3);
        scale[e] = s_e;
        for (long l = 0; l < nq3; ++l) X[e * nq3 + l] = s_e > 0.0 ? r[c->gmap[e * nq3 + l]] / s_e : 0.0;
    }
    return 0;
}

/* corr = node average of the element corrections s_e MLP(r_e / s_e) */
int orc_mlp_correction(orc_ctx *c, const orc_mlp *m, const double *r, double *corr)
{
    if (!c || !m || !r || !corr || m->nin != c->nq3) return -1;
    long nq3 = c->nq3, np = c->np;
    double *X = (double *)malloc(sizeof(double) * c->nelem * nq3), *sc = (double *)malloc(sizeof(double) * c->nelem);
    double *h = (double *)malloc(sizeof(double) * m->nh), *y = (double *)malloc(sizeof(double) * nq3);
    double *cnt = (double *)calloc(np, sizeof(double));
    if (!X || !sc || !h || !y || !cnt) { free(X); free(sc); free(h); free(y); free(cnt); return -5; }
    orc_element_features(c, r, X, sc);
    memset(corr, 0, sizeof(double) * np);
    for (long e = 0; e < c->nelem; ++e) {
        orc_mlp_forward(m, X + e * nq3, h, y);
        for (long l = 0; l < nq3; ++l) {
            long I = c->gmap[e * nq3 + l];
            corr[I] += sc[e] * y[l];
            cnt[I] += 1.0;
        }
    }
    for (long I = 0; I < np; ++I) corr[I] /= cnt[I];
    free(X); free(sc); free(h); free(y); free(cnt);
    return 0;
}

typedef struct {
    pbno_arg *p;
    const orc_mlp *mlp;
    int net_cycles; /* restart cycles that ran with the network */
} learned_arg;

/* The polynomial is the fallback: a restart cycle with the network that
 * does not reduce the residual norm tenfold switches the network off for
 * the rest of the solve. */
static void learned_guard(const void *marg, double before, double after)
{
    learned_arg *a = (learned_arg *)marg;
    if (!a->mlp) return;
    a->net_cycles++;
    if (after > 0.1 * before) a->mlp = NULL;
}

static int op_learned(orc_ctx *c, const void *arg, const double *r, double *z)
{
    const learned_arg *a = (const learned_arg *)arg;
    long n = c->np;
    int rc = 0;
    if (a->p->p >= 0) rc = op_pbno(c, a->p, r, z);
    else memcpy(z, r, sizeof(double) * n);
    if (rc || !a->mlp) return rc;
    double *corr = (double *)malloc(sizeof(double) * n);
    if (!corr) return -5;
    rc = orc_mlp_correction(c, a->mlp, r, corr);
    if (!rc)
        for (long i = 0; i < n; ++i) z[i] += corr[i];
    free(corr);
    return rc;
}

int orc_learned_apply(orc_ctx *c, const double *r, double *z, double lambda, int order, const double *bounds,
                      const orc_mlp *mlp)
{
    if (!c || !r || !z || (order >= 0 && !bounds)) return -1;
    if (c->nbv > 0.0) return -7;
    schur_arg s = {lambda, (double *)malloc(sizeof(double) * 5 * c->np), (double *)malloc(sizeof(double) * 5 * c->np)};
    pbno_arg pa = {&s, order, bounds ? bounds[0] : 0.0, bounds ? bounds[1] : 0.0};
    learned_arg la = {&pa, mlp, 0};
    int rc = (s.s && s.l) ? op_learned(c, &la, r, z) : -5;
    free(s.s); free(s.l);
    return rc;
}

/* orc_solve3d with flexible GMRES and the learned preconditioner (PBNO of
 * the given order, order < 0 none, plus the MLP correction; mlp NULL: the
 * polynomial alone, still through flexible GMRES), with the fallback of
 * learned_guard. */
int orc_solve3d_learned(orc_ctx *c, const double *y, double *x, double lambda, double tol, int restart, int maxit,
                        int order, const double *bounds, const orc_mlp *mlp, int *iters, int *net_cycles)
{
    if (!c || !y || !x || restart < 1 || maxit < 1 || !(tol > 0.0)) return -1;
    if (c->nbv > 0.0) return -7;
    if (order >= 0 && (!bounds || !(bounds[1] > bounds[0]) || !(bounds[0] > 0.0))) return -1;
    long np = c->np;
    schur_arg a = {lambda, (double *)malloc(sizeof(double) * 5 * np), (double *)malloc(sizeof(double) * 5 * np)};
    double *Ua = (double *)malloc(sizeof(double) * 3 * np), *Up = (double *)malloc(sizeof(double) * 3 * np);
    double *b = (double *)malloc(sizeof(double) * np), *P = (double *)malloc(sizeof(double) * np);
    int rc = (a.s && a.l && Ua && Up && b && P) ? 0 : -5, it = 0, grc = 0;
    pbno_arg pa = {&a, order, bounds ? bounds[0] : 0.0, bounds ? bounds[1] : 0.0};
    learned_arg la = {&pa, mlp, 0};
    if (!rc) rc = schur_rhs(c, &a, y, Ua, b);
    if (!rc) {
        grc = gmres_impl(c, np, op_schur, &a, op_learned, &la, b, P, tol, restart, maxit, 1, learned_guard, &it);
        if (grc && grc != -6) rc = grc;
    }
    if (!rc) rc = schur_up(c, &a, P, Up);
    if (!rc) {
        for (long I = 0; I < 3 * np; ++I) x[np + I] = Ua[I] - Up[I];
        rc = schur_div(c, &a, x + np, x);
    }
    if (!rc)
        for (long I = 0; I < np; ++I) {
            x[I] = y[I] + lambda * x[I];
            x[4 * np + I] = y[4 * np + I];
        }
    if (iters) *iters = it;
    if (net_cycles) *net_cycles = la.net_cycles;
    free(a.s); free(a.l); free(Ua); free(Up); free(b); free(P);
    return rc ? rc : grc;
}

/* The polynomial judges the network: the same system solved to tol with
 * the network (flexible GMRES, its fallback included) and with the
 * polynomial alone; the network is accepted only if its solve converged in
 * fewer GMRES iterations.  out = {polynomial iterations, network
 * iterations, accepted}.  -6 if the polynomial solve does not converge. */
int orc_learned_judge(orc_ctx *c, const double *y, double lambda, double tol, int restart, int maxit, int order,
                      const double *bounds, const orc_mlp *mlp, int *out)
{
    if (!c || !y || !mlp || !out) return -1;
    double *x = (double *)malloc(sizeof(double) * 5 * c->np);
    if (!x) return -5;
    int it_net = 0, it_pb = 0;
    int rn = orc_solve3d_learned(c, y, x, lambda, tol, restart, maxit, order, bounds, mlp, &it_net, NULL);
    int rp = (rn == 0 || rn == -6) ? orc_solve3d(c, y, x, lambda, tol, restart, maxit, order, bounds, &it_pb) : rn;
    free(x);
    if (rp) return rp;
    out[0] = it_pb;
    out[1] = it_net;
    out[2] = rn == 0 && it_net < it_pb;
    return 0;
}

/* nsteps 3D-IMEX ARK2 steps: orc_step with L in place of L_V and the Schur
 * GMRES solve (PBNO order and interval as orc_solve3d; restart 30); linear
 * != 0: R := L.  *iters: GMRES iterations of all solves. */
int orc_step3d(orc_ctx *c, double *q, double dt, int nsteps, int linear, double tol, int order,
               const double *bounds, int *iters)
{
    if (!c || !q || nsteps < 0 || !(dt > 0.0)) return -1;
    if (c->nbv > 0.0) return -7;
    double a[9], at[9], b[3];
    orc_ark2_tableau(a, at, b);
    double lam = at[1 * 3 + 1] * dt;
    long n5 = 5 * c->np;
    double *Rs[3], *Ls[2], *Y = (double *)malloc(sizeof(double) * n5);
    double *Q = (double *)malloc(sizeof(double) * n5);
    for (int s = 0; s < 3; ++s) Rs[s] = (double *)malloc(sizeof(double) * n5);
    for (int s = 0; s < 2; ++s) Ls[s] = (double *)malloc(sizeof(double) * n5);
    int rc = (Y && Q && Rs[0] && Rs[1] && Rs[2] && Ls[0] && Ls[1]) ? 0 : -5, total = 0;
    for (int n = 0; n < nsteps && !rc; ++n) {
        for (int i = 0; i < 3 && !rc; ++i) {
            if (i == 0) {
                memcpy(Q, q, sizeof(double) * n5);
            } else {
                for (long I = 0; I < n5; ++I) {
                    double y = q[I];
                    for (int j = 0; j < i; ++j)
                        y += dt * (a[i * 3 + j] * Rs[j][I] + (at[i * 3 + j] - a[i * 3 + j]) * Ls[j][I]);
                    Y[I] = y;
                }
                int it = 0;
                rc = orc_solve3d(c, Y, Q, lam, tol, 30, 100000, order, bounds, &it);
                total += it;
                if (rc) break;
            }
            rc = linear ? orc_lfull(c, Q, Rs[i]) : orc_rhs(c, Q, Rs[i]);
            if (!rc && i < 2) rc = orc_lfull(c, Q, Ls[i]);
        }
        if (rc) break;
        for (long I = 0; I < n5; ++I) q[I] += dt * (b[0] * Rs[0][I] + b[1] * Rs[1][I] + b[2] * Rs[2][I]);
    }
    if (iters) *iters = total;
    free(Y); free(Q);
    for (int s = 0; s < 3; ++s) free(Rs[s]);
    for (int s = 0; s < 2; ++s) free(Ls[s]);
    return rc;
}
