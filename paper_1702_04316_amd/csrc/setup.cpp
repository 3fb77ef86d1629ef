// Host set-up of the HEVI library: LGL basis, the direct-stiffness-summed 1D
// derivative operators, and the background profile.
//
// LGL nodes: the interior nodes are the zeros of P_N', i.e. of the Jacobi
// polynomial P^(1,1)_{N-1}; they are the eigenvalues of its symmetric
// tridiagonal Jacobi matrix (zero diagonal, off-diagonal sqrt(b_n),
// b_n = n(n+2)/((2n+1)(2n+3))), found here by Sturm-sequence bisection.
// Differentiation matrix: barycentric form of the Lagrange basis derivative.
//
// DSS line operators.  In an axis-aligned box every element has a constant
// diagonal metric 2/h, and every Set2NC tendency is a node-local coefficient
// times the first derivative of a continuous nodal field.  The mass-weighted
// direct stiffness summation of the element-local strong derivatives
// (Sec. 5.3) therefore factorises into a 1D operator along each grid line:
// at a node inside an element it is (2/h) D[a][.] over that element; at a node
// shared by a left element (h_L) and a right element (h_R) it is
// 2 (D[N][.] g_L + D[0][.] g_R) / (h_L + h_R) (the LGL end weights are equal,
// and the weights of the other two directions cancel).
#include <cmath>
#include <vector>

#include "numa_internal.h"

namespace numa {

namespace {

// Number of eigenvalues below x of the Jacobi matrix of P^(1,1) of size n.
int sturm_count(const std::vector<double> &off2, int n, double x)
{
    int count = 0;
    double d = -x;  // zero diagonal
    if (d < 0) ++count;
    for (int k = 1; k < n; ++k) {
        if (d == 0.0) d = 1e-300;
        d = -x - off2[k - 1] / d;
        if (d < 0) ++count;
    }
    return count;
}

}  // namespace

void lgl_nodes(int N, std::vector<double> &xi)
{
    xi.assign(N + 1, 0.0);
    xi[0] = -1.0;
    xi[N] = 1.0;
    int n = N - 1;  // interior nodes
    if (n <= 0) return;
    std::vector<double> off2(n > 1 ? n - 1 : 1);
    for (int m = 1; m < n; ++m) off2[m - 1] = double(m) * (m + 2) / ((2.0 * m + 1) * (2.0 * m + 3));
    for (int r = 0; r < n; ++r) {
        // the (r+1)-th smallest eigenvalue lies where the count passes r
        double lo = -1.0, hi = 1.0;
        for (int it = 0; it < 200 && hi - lo > 0.0; ++it) {
            double mid = 0.5 * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            if (sturm_count(off2, n, mid) > r) hi = mid;
            else lo = mid;
        }
        xi[1 + r] = 0.5 * (lo + hi);
    }
    // the node set is symmetric about 0: average the two halves
    for (int i = 0; i <= N / 2; ++i) {
        double s = 0.5 * (xi[N - i] - xi[i]);
        xi[i] = -s;
        xi[N - i] = s;
    }
    if (N % 2 == 0) xi[N / 2] = 0.0;
}

void lgl_dmat(int N, const std::vector<double> &xi, std::vector<double> &D)
{
    int nq = N + 1;
    std::vector<double> bw(nq);
    for (int j = 0; j < nq; ++j) {
        double p = 1.0;
        for (int k = 0; k < nq; ++k)
            if (k != j) p *= (xi[j] - xi[k]);
        bw[j] = 1.0 / p;
    }
    D.assign(nq * nq, 0.0);
    for (int i = 0; i < nq; ++i) {
        double diag = 0.0;
        for (int j = 0; j < nq; ++j) {
            if (j == i) continue;
            double v = (bw[j] / bw[i]) / (xi[i] - xi[j]);
            D[i * nq + j] = v;
            diag -= v;
        }
        D[i * nq + i] = diag;
    }
}

void set_binomial(EOS &e)
{
    double ck = 1.0;
    for (int k = 1; k <= kBinomTerms; ++k) {
        ck *= (e.gamma - (k - 1)) / k;  // C(gamma, k) = C(gamma, k-1) (gamma - k + 1) / k
        e.binom[k - 1] = ck;
    }
}

void build_ops(numa_ctx *c, const double *zface)
{
    HostOps &o = c->ops;
    const int N = c->N, nq = N + 1, ns = 2 * N + 1;
    o.N = N;
    lgl_nodes(N, o.xi);
    lgl_dmat(N, o.xi, o.D);

    // x and y stencils for local index a in [0, N): coefficients of the nodes
    // (element start - N + m), m = 0..2N.
    o.wxy.assign(2 * N * ns, 0.0);
    const double h[2] = {c->lx / c->nex, c->ly / c->ney};
    for (int d = 0; d < 2; ++d) {
        double *w = &o.wxy[d * N * ns];
        for (int a = 0; a < N; ++a) {
            double *s = w + a * ns;
            if (a == 0) {
                // interface node: left element (nodes m = 0..N) and right (m = N..2N)
                for (int n = 0; n < nq; ++n) {
                    s[n] += 2.0 * o.D[N * nq + n] / (2.0 * h[d]);
                    s[N + n] += 2.0 * o.D[0 * nq + n] / (2.0 * h[d]);
                }
            } else {
                for (int n = 0; n < nq; ++n) s[N + n] = (2.0 / h[d]) * o.D[a * nq + n];
            }
        }
    }

    // vertical element heights and factors
    std::vector<double> zf(c->nez + 1), hz(c->nez);
    for (int e = 0; e <= c->nez; ++e) zf[e] = zface ? zface[e] : c->lz * e / c->nez;
    zf[c->nez] = c->lz;
    for (int e = 0; e < c->nez; ++e) hz[e] = zf[e + 1] - zf[e];
    o.zsc.assign(3 * c->nez, 0.0);
    for (int e = 0; e < c->nez; ++e) {
        o.zsc[0 * c->nez + e] = 2.0 / hz[e];
        o.zsc[1 * c->nez + e] = e == 0 ? 2.0 / hz[0] : 2.0 / (hz[e - 1] + hz[e]);
        o.zsc[2 * c->nez + e] = e == c->nez - 1 ? 2.0 / hz[e] : 2.0 / (hz[e] + hz[e + 1]);
    }

    // column operator as a band: row k, coefficient of level k - N + m
    const int nz = int(c->nz);
    o.dzb.assign(size_t(nz) * ns, 0.0);
    for (int k = 0; k < nz; ++k) {
        double *b = &o.dzb[size_t(k) * ns];
        int e = k / N, cc = k % N;
        if (k == nz - 1) {  // top node: the top element only
            e = c->nez - 1;
            for (int n = 0; n < nq; ++n) b[(e * N + n) - k + N] += (2.0 / hz[e]) * o.D[N * nq + n];
        } else if (cc != 0) {
            for (int n = 0; n < nq; ++n) b[(e * N + n) - k + N] += (2.0 / hz[e]) * o.D[cc * nq + n];
        } else if (e == 0) {  // bottom node
            for (int n = 0; n < nq; ++n) b[n - k + N] += (2.0 / hz[0]) * o.D[0 * nq + n];
        } else {  // interface between elements e-1 and e
            double s = 2.0 / (hz[e - 1] + hz[e]);
            for (int n = 0; n < nq; ++n) {
                b[((e - 1) * N + n) - k + N] += s * o.D[N * nq + n];
                b[(e * N + n) - k + N] += s * o.D[0 * nq + n];
            }
        }
    }

    // level heights and the hydrostatic background: theta0(z), its vertical
    // derivative, and rho0 = p00 pi0^(cv/R) / (R theta0) from the Exner
    // function (P0 = EOS(rho0, theta0) follows on the device)
    o.zk.assign(nz, 0.0);
    for (int e = 0; e < c->nez; ++e)
        for (int cc = 0; cc <= N; ++cc) o.zk[e * N + cc] = zf[e] + 0.5 * (o.xi[cc] + 1.0) * hz[e];
    o.rho0.assign(nz, 0.0);
    o.th0.assign(nz, 0.0);
    o.th0z.assign(nz, 0.0);
    const double cv = c->cp - c->eos.rgas;
    const double S = c->nbv > 0.0 ? c->nbv * c->nbv / c->eos.grav : 0.0;  // (1/theta0) d theta0/dz
    for (int k = 0; k < nz; ++k) {
        const double z = o.zk[k];
        const double th = S > 0.0 ? c->eos.theta0 * std::exp(S * z) : c->eos.theta0;
        const double exner = exner_at(c->eos.theta0, c->cp, c->eos.grav, c->nbv, z);
        o.th0[k] = th;
        o.th0z[k] = S * th;
        o.rho0[k] = c->eos.p00 * std::pow(exner, cv / c->eos.rgas) / (c->eos.rgas * th);
    }
}

double exner_at(double theta0, double cp, double grav, double nbv, double z)
{
    if (!(nbv > 0.0)) return 1.0 - grav * z / (cp * theta0);
    // theta0(z) = theta0 exp(S z): pi0 = 1 - g (1 - exp(-S z)) / (cp theta0 S)
    const double S = nbv * nbv / grav;
    return 1.0 + grav * std::expm1(-S * z) / (cp * theta0 * S);
}

}  // namespace numa
