/* Exercises the oracle's C library under AddressSanitizer and
 * UndefinedBehaviorSanitizer: every public routine on small grids (orders 1
 * to 8, uniform and stretched vertical faces, isentropic and stratified
 * backgrounds) and the argument checks.  Prints one checksum line; any
 * sanitizer report aborts with a non-zero status. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "numa_oracle.h"

static unsigned long long lcg = 12345u;
static double urand(void)
{
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) / 9007199254740992.0 - 0.5;
}

static double sum_abs(const double *a, long n)
{
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += fabs(a[i]);
    return s;
}

#define CHECK(x)                                                   \
    do {                                                           \
        if (!(x)) {                                                \
            fprintf(stderr, "check failed: %s (line %d)\n", #x, __LINE__); \
            exit(3);                                               \
        }                                                          \
    } while (0)

int main(void)
{
    double acc = 0.0;
    orc_set_threads(2);
    for (int N = 1; N <= 15; ++N) {
        double xi[16], w[16], D[256];
        orc_lgl(N, xi, w);
        orc_dmat(N, xi, D);
        acc += sum_abs(D, (N + 1) * (N + 1)) * 1e-6;
    }
    CHECK(orc_setup(1.0, 1.0, 1.0, 0, 1, 1, NULL, 4, 300.0, 1e5, 1004.67, 287.17, 9.80616, 0.0) == NULL);
    for (int N = 1; N <= 8; ++N) {
        const int nex = 2, ney = 1 + N % 2, nez = 2;
        double zf[3] = {0.0, 3500.0, 8000.0};
        for (int strat = 0; strat < 2; ++strat) {
            orc_ctx *c = orc_setup(9000.0 * nex, 7000.0 * ney, 8000.0, nex, ney, nez, (N & 1) ? zf : NULL, N, 300.0,
                                   1e5, 1004.67, 287.17, 9.80616, strat ? 0.01 : 0.0);
            CHECK(c != NULL);
            long sz[4];
            orc_sizes(c, sz);
            const long np = sz[0] * sz[1] * sz[2];
            double *q = malloc(sizeof(double) * 5 * np), *R = malloc(sizeof(double) * 5 * np);
            double *x = malloc(sizeof(double) * 5 * np), *M = malloc(sizeof(double) * np);
            double *P = malloc(sizeof(double) * np), *S = malloc(sizeof(double) * np);
            double *cx = malloc(sizeof(double) * sz[0]), *cy = malloc(sizeof(double) * sz[1]);
            double *cz = malloc(sizeof(double) * sz[2]), *bg = malloc(sizeof(double) * 6 * sz[2]);
            CHECK(q && R && x && M && P && S && cx && cy && cz && bg);
            for (long i = 0; i < 5 * np; ++i) q[i] = 0.01 * urand();
            const long plane = sz[0] * sz[1];
            for (long I = 0; I < plane; ++I) q[3 * np + I] = q[3 * np + (sz[2] - 1) * plane + I] = 0.0;  /* w = 0 */
            for (long i = 0; i < np; ++i) P[i] = urand();
            orc_coords(c, cx, cy, cz);
            orc_mass(c, M);
            orc_background(c, bg, bg + sz[2], bg + 2 * sz[2], bg + 3 * sz[2]);
            orc_background_theta(c, bg + 4 * sz[2], bg + 5 * sz[2]);
            CHECK(orc_pressure_perturbation(c, q, S) == 0);
            CHECK(orc_rhs(c, q, R) == 0);
            acc += sum_abs(R, 5 * np) * 1e-9;
            CHECK(orc_lv(c, q, R) == 0);
            CHECK(orc_lfull(c, q, R) == 0);
            CHECK(orc_factor(c, (1.0 - 1.0 / sqrt(2.0)) * 1.5) == 0);
            CHECK(orc_solve(c, q, x) == 0);
            acc += sum_abs(x, 5 * np) * 1e-9;
            double *A = malloc(sizeof(double) * 9 * sz[2] * sz[2]);
            CHECK(A && orc_column_matrix(c, 3.0, 0, 0, A) == 0);
            free(A);
            CHECK(orc_step(c, q, 1.5, 2, 0) == 0);
            if (!strat) {
                double bd[2];
                int it = 0, out[3];
                CHECK(orc_schur_apply(c, P, S, 2.0) == 0);
                CHECK(orc_schur_bounds(c, 2.0, 10, bd) == 0);
                CHECK(orc_pbno_apply(c, P, S, 2.0, 2, bd[0], bd[1]) == 0);
                CHECK(orc_solve3d(c, q, x, 2.0, 1e-8, 10, 500, 1, bd, &it) == 0);
                CHECK(orc_solve3d(c, q, x, 2.0, 1e-8, 0, 500, 1, bd, &it) == -1);
                CHECK(orc_solve3d_standard(c, q, x, 2.0, 1e-8, 10, 2000, &it) == 0);
                const int nin = (N + 1) * (N + 1) * (N + 1), nh = 3;
                double *th = malloc(sizeof(double) * (2 * nin * nh + nh + nin));
                CHECK(th != NULL);
                for (int i = 0; i < 2 * nin * nh + nh + nin; ++i) th[i] = 0.01 * urand();
                orc_mlp m = {nin, nh, th, th + nin * nh, th + nin * nh + nh, th + 2 * nin * nh + nh};
                const long ne = sz[3];
                double *X = malloc(sizeof(double) * ne * nin), *sc = malloc(sizeof(double) * ne);
                double *g = malloc(sizeof(double) * (2 * nin * nh + nh + nin));
                CHECK(X && sc && g);
                CHECK(orc_element_features(c, P, X, sc) == 0);
                acc += orc_mlp_loss_grad(&m, (int)ne, X, X, g, g + nin * nh, g + nin * nh + nh,
                                         g + 2 * nin * nh + nh) * 1e-6;
                CHECK(orc_mlp_correction(c, &m, P, S) == 0);
                CHECK(orc_learned_apply(c, P, S, 2.0, 1, bd, &m) == 0);
                CHECK(orc_solve3d_learned(c, q, x, 2.0, 1e-8, 10, 500, 1, bd, &m, &it, NULL) == 0);
                CHECK(orc_learned_judge(c, q, 2.0, 1e-8, 10, 500, 1, bd, &m, out) == 0);
                CHECK(orc_step3d(c, q, 1.0, 1, 0, 1e-8, 1, bd, &it) == 0);
                free(th); free(X); free(sc); free(g);
            } else {
                CHECK(orc_schur_apply(c, P, S, 2.0) == -7);
            }
            acc += sum_abs(q, 5 * np) * 1e-6;
            free(q); free(R); free(x); free(M); free(P); free(S); free(cx); free(cy); free(cz); free(bg);
            orc_free(c);
        }
    }
    printf("oracle driver ok %.6e\n", acc);
    return 0;
}
