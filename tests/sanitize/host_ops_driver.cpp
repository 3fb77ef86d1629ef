// Exercises the library's host set-up code (LGL basis, DSS line operators,
// column band, background profiles, binomial table of the equation of state)
// under AddressSanitizer and UndefinedBehaviorSanitizer, for orders 1 to 15
// on uniform and stretched vertical faces over isentropic and stratified
// backgrounds, and checks invariants that hold for any grid: derivative
// matrix rows sum to zero, every stencil row differentiates a constant to
// zero and a linear function to its slope.  Prints one line; a sanitizer
// report or a failed check exits non-zero.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "numa_internal.h"

static void check(bool ok, const char *what, int N)
{
    if (!ok) {
        std::fprintf(stderr, "check failed: %s (N=%d)\n", what, N);
        std::exit(3);
    }
}

int main()
{
    double acc = 0.0;
    for (int N = 1; N <= 15; ++N) {
        std::vector<double> xi, D;
        numa::lgl_nodes(N, xi);
        numa::lgl_dmat(N, xi, D);
        check(int(xi.size()) == N + 1 && int(D.size()) == (N + 1) * (N + 1), "sizes", N);
        for (int i = 0; i <= N; ++i) {
            double s = 0.0, t = 0.0;
            for (int j = 0; j <= N; ++j) {
                s += D[i * (N + 1) + j];
                t += D[i * (N + 1) + j] * xi[j];
            }
            check(std::fabs(s) < 1e-9 * (N + 1) * (N + 1) && std::fabs(t - 1.0) < 1e-9 * (N + 1) * (N + 1), "D", N);
        }
        for (int variant = 0; variant < 4; ++variant) {
            numa_ctx c;
            c.N = N;
            c.nex = 2 + variant % 2;
            c.ney = 1 + variant / 2;
            c.nez = 3;
            c.nx = int64_t(c.nex) * N;
            c.ny = int64_t(c.ney) * N;
            c.nz = int64_t(c.nez) * N + 1;
            c.lx = 9000.0 * c.nex;
            c.ly = 7000.0 * c.ney;
            c.lz = 9000.0;
            c.cp = 1004.67;
            c.nbv = variant >= 2 ? 0.01 : 0.0;
            c.eos = {300.0, 1.0e5, 287.17, 1004.67 / (1004.67 - 287.17), 9.80616, {}};
            numa::set_binomial(c.eos);
            const double zf[4] = {0.0, 2000.0, 4500.0, 9000.0};
            numa::build_ops(&c, (variant & 1) ? zf : nullptr);
            const numa::HostOps &o = c.ops;
            const int ns = 2 * N + 1;
            check(int(o.wxy.size()) == 2 * N * ns && o.dzb.size() == size_t(c.nz) * ns, "op sizes", N);
            // line stencils: a constant to zero, x (a linear field) to 1; the
            // stencil of local index a covers the nodes from the start of
            // the previous element (m = 0..N) through the current one
            for (int d = 0; d < 2; ++d) {
                const double h = d == 0 ? c.lx / c.nex : c.ly / c.ney;
                for (int a = 0; a < N; ++a) {
                    double s = 0.0, t = 0.0, scale = 0.0;
                    for (int m = 0; m < ns; ++m) {
                        const double w = o.wxy[(d * N + a) * ns + m];
                        const double pos = m <= N ? 0.5 * (xi[m] + 1.0) * h - h : 0.5 * (xi[m - N] + 1.0) * h;
                        s += w;
                        t += w * pos;
                        scale += std::fabs(w);
                    }
                    check(std::fabs(s) <= 1e-10 * scale && std::fabs(t - 1.0) <= 1e-9 * scale * h, "stencil", N);
                }
            }
            for (long k = 0; k < c.nz; ++k) {
                double s = 0.0, t = 0.0, scale = 0.0;
                for (int m = 0; m < ns; ++m) {
                    const long kk = k - N + m;
                    const double w = o.dzb[size_t(k) * ns + m];
                    if (w == 0.0) continue;
                    check(kk >= 0 && kk < c.nz, "band inside the column", N);
                    s += w;
                    t += w * o.zk[size_t(kk)];
                    scale += std::fabs(w);
                }
                check(std::fabs(s) <= 1e-10 * scale && std::fabs(t - 1.0) <= 1e-8 * scale * c.lz, "band", N);
            }
            for (long k = 0; k < c.nz; ++k)
                check(o.rho0[size_t(k)] > 0.0 && o.th0[size_t(k)] >= 300.0, "background", N);
            acc += o.rho0[0] + o.th0z[size_t(c.nz - 1)] + numa::exner_at(300.0, 1004.67, 9.80616, c.nbv, 5000.0);
        }
    }
    std::printf("host ops driver ok %.9e\n", acc);
    return 0;
}
