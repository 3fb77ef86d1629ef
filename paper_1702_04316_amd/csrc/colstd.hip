// Standard-form column solve: a comparison point for the Schur-complement
// form (Sec. 5, Sec. 5.4).  The column system (I - lambda L_V) x = y is
// solved for (rho', w) directly, without eliminating w, as the unreduced
// form the paper contrasts with the Schur form:
//   rho'_k + lambda sum_m Dz[k][m] rho0_m w_m                    = y_rho,k
//   w_k + lambda (sum_m Dz[k][m] G0_m rho'_m + g rho'_k) / rho0_k = y_w,k - lambda sum_m Dz[k][m] H0_m y_theta,m / rho0_k
// (interior levels; w is 0 on the bottom and top, which decouples those two
// unknowns).  The unknowns are interleaved per level, (rho'_0, w_0,
// rho'_1, w_1, ...), so the matrix is a band of half-width 2N+1; it is
// factored without pivoting (growth stays near 1 because the diagonal
// blocks are the identity) and solved by band substitution, one column per
// thread.  As for the Schur form, every column has the same matrix, so one
// factor set [row][band offset] serves them all.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "numa_internal.h"

namespace numa {

namespace {

template <int N>
struct StdBand {
    static constexpr int K = 2 * N + 1;   // half-bandwidth
    static constexpr int NB = 2 * K + 1;  // stored band width
};

// Assembly and elimination of the one shared band by one workgroup: the
// threads fill the entries, then for each pivot update the trailing window
// in parallel and scale the pivot column.  The band is worked on in LDS when
// it fits (kStdFactorLds bytes), else in place in global memory.
constexpr int kStdFactorThreads = 256;
constexpr size_t kStdFactorLds = 64 * 1024;

template <int N>
__global__ __launch_bounds__(kStdFactorThreads) void k_factor_std(const double *__restrict__ dzb,
                                                                  const double *__restrict__ rho0,
                                                                  const double *__restrict__ G0, double lambda,
                                                                  double grav, int M, int in_lds, double *fac,
                                                                  int *flag)
{
    extern __shared__ double band_lds[];
    constexpr int NS = 2 * N + 1, K = StdBand<N>::K, NB = StdBand<N>::NB;
    const int tid = threadIdx.x;
    const int n = 2 * M;
    double *A = in_lds ? band_lds : fac;  // entry (r, c) at r*NB + (c - r + K)
    auto dz = [&](int k, int m) -> double {
        const int d = m - k + N;
        return (d >= 0 && d < NS) ? dzb[(long)k * NS + d] : 0.0;
    };
    for (int idx = tid; idx < n * NB; idx += kStdFactorThreads) {
        const int r = idx / NB, c = r + idx % NB - K;
        const int k = r >> 1;
        const bool wrow = r & 1;
        const bool wall = k == 0 || k == M - 1;
        double v = 0.0;
        if (c >= 0 && c < n) {
            const int m = c >> 1;
            if (c == r) {
                v = 1.0;
            } else if (!wrow && (c & 1)) {  // rho' row, w unknown of level m
                if (m >= 1 && m <= M - 2) v = lambda * dz(k, m) * rho0[m];
            } else if (wrow && !(c & 1) && !wall) {  // w row, rho' unknown of level m
                v = lambda * (dz(k, m) * G0[m] + (m == k ? grav : 0.0)) / rho0[k];
            }
        }
        A[idx] = v;
    }
    __syncthreads();
    bool bad = false;
    for (int k = 0; k < n; ++k) {
        const double piv = A[k * NB + K];
        const double rp = 1.0 / piv;
        const int w = min(k + K, n - 1) - k;
        for (int t = tid; t < w * w; t += kStdFactorThreads) {
            const int i = k + 1 + t / w, j = k + 1 + t % w;
            const double l = A[i * NB + (k - i + K)] * rp;
            A[i * NB + (j - i + K)] -= l * A[k * NB + (j - k + K)];
        }
        __syncthreads();  // column k and the pivot are read above, written below
        for (int t = tid; t < w; t += kStdFactorThreads) A[(k + 1 + t) * NB + (-1 - t + K)] *= rp;
        if (tid == 0) {
            bad |= !(fabs(piv) > 0.0) || !isfinite(piv);
            A[k * NB + K] = rp;  // the solve multiplies by the reciprocal pivot
        }
        __syncthreads();
    }
    if (in_lds)
        for (int idx = tid; idx < n * NB; idx += kStdFactorThreads) fac[idx] = band_lds[idx];
    if (bad) *flag = 1;
}

template <int N>
__global__ __launch_bounds__(64) void k_solve_std(const double *__restrict__ fac, const double *__restrict__ dzb,
                                                  const double *__restrict__ rho0, const double *__restrict__ H0,
                                                  double lambda, int M, long ncol, const double *yr, const double *yw,
                                                  const double *yt, double *xr, double *xw)
{
    constexpr int NS = 2 * N + 1, K = StdBand<N>::K, NB = StdBand<N>::NB;
    const long col = (long)blockIdx.x * 64 + threadIdx.x;
    if (col >= ncol) return;
    const int n = 2 * M;
    // the shared factor band (all columns alike), d = c - r + K
    auto F = [&](int r, int d) { return fac[(long)r * NB + d]; };
    auto at = [&](int k) { return (long)k * ncol + col; };
    // forward (unit lower): z_r = b_r - sum_d L(r, r-d) z_{r-d}; the last K
    // values in a shift register (win[K-1] is z_{r-1})
    double win[K];
#pragma unroll
    for (int t = 0; t < K; ++t) win[t] = 0.0;
    for (int r = 0; r < n; ++r) {
        const int k = r >> 1;
        double b;
        if (!(r & 1)) {
            b = yr[at(k)];
        } else if (k == 0 || k == M - 1) {
            b = yw[at(k)];
        } else {
            double s = 0.0;
            for (int m = max(k - N, 0); m <= min(k + N, M - 1); ++m)
                s += dzb[(long)k * NS + (m - k + N)] * H0[m] * yt[at(m)];
            b = yw[at(k)] - lambda * s / rho0[k];
        }
#pragma unroll
        for (int d = 1; d <= K; ++d)
            if (r - d >= 0) b -= F(r, K - d) * win[K - d];
#pragma unroll
        for (int t = 0; t < K - 1; ++t) win[t] = win[t + 1];
        win[K - 1] = b;
        if (!(r & 1)) xr[at(k)] = b;
        else xw[at(k)] = b;
    }
    // backward: x_r = (z_r - sum_d U(r, r+d) x_{r+d}) / U(r, r); win[d-1] is x_{r+d}
#pragma unroll
    for (int t = 0; t < K; ++t) win[t] = 0.0;
    for (int r = n - 1; r >= 0; --r) {
        const int k = r >> 1;
        double z = (r & 1) ? xw[at(k)] : xr[at(k)];
#pragma unroll
        for (int d = 1; d <= K; ++d)
            if (r + d < n) z -= F(r, K + d) * win[d - 1];
        z *= F(r, K);
#pragma unroll
        for (int t = K - 1; t > 0; --t) win[t] = win[t - 1];
        win[0] = z;
        if (!(r & 1)) xr[at(k)] = z;
        else xw[at(k)] = z;
    }
}

template <typename F>
hipError_t dispatch_std(int N, F &&f)
{
    switch (N) {
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 3: return f(std::integral_constant<int, 3>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 5: return f(std::integral_constant<int, 5>{});
    case 6: return f(std::integral_constant<int, 6>{});
    case 7: return f(std::integral_constant<int, 7>{});
    case 8: return f(std::integral_constant<int, 8>{});
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

// one factor set shared by all columns (their matrices are identical)
size_t std_factor_bytes(const numa_ctx *c)
{
    return size_t(2 * c->nz) * size_t(2 * (2 * c->N + 1) + 1) * sizeof(double);
}

hipError_t launch_factor_std(numa_ctx *c, double lambda)
{
    if (!c->fac_std) {
        hipError_t e = hipMalloc(&c->fac_std, std_factor_bytes(c));
        if (e != hipSuccess) {
            c->fac_std = nullptr;
            return e;
        }
    }
    return dispatch_std(c->N, [&](auto n) {
        constexpr int NN = decltype(n)::value;
        const size_t bytes = std_factor_bytes(c);
        const bool lds = bytes <= kStdFactorLds;
        hipLaunchKernelGGL((k_factor_std<NN>), dim3(1), dim3(kStdFactorThreads), lds ? bytes : 0, c->stream,
                           c->lev.dzb, c->lev.rho0, c->lev.G0, lambda, c->eos.grav, int(c->nz), int(lds), c->fac_std,
                           c->flag);
        return hipGetLastError();
    });
}

hipError_t launch_solve_std(numa_ctx *c, const double *y, double *x)
{
    const long np = c->np;
    for (int f : {1, 2, 4}) {
        hipError_t e = hipMemcpyAsync(x + f * np, y + f * np, sizeof(double) * np, hipMemcpyDeviceToDevice, c->stream);
        if (e != hipSuccess) return e;
    }
    return dispatch_std(c->N, [&](auto n) {
        constexpr int NN = decltype(n)::value;
        hipLaunchKernelGGL((k_solve_std<NN>), dim3(unsigned((c->ncol + 63) / 64)), dim3(64), 0, c->stream, c->fac_std,
                           c->lev.dzb, c->lev.rho0, c->lev.H0, c->lambda_std, int(c->nz), c->ncol, y + 0 * np,
                           y + 3 * np, y + 4 * np, x + 0 * np, x + 3 * np);
        return hipGetLastError();
    });
}

}  // namespace numa
