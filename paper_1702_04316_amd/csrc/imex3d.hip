// 3D-IMEX step (Sec. 2): the implicit part is the whole linear operator L,
// and the implicit systems (I - lambda L) x = y are solved iteratively
// (Sec. 5.5) in their Schur-complement form (the Set2NC analogue of the
// pressure system of Algs. 4-5).
//
// With theta' = y_theta (L has no theta' tendency for a constant theta0) and
// the linear pressure P = G0 rho' + H0 theta', eliminating the velocities
// leaves one scalar field per node:
//     S P = P - lambda^2 (V P + G0 (Dxx P + Dyy P)) = b,
//     b   = G0 y_rho + H0 y_theta - lambda G0 (rho0 (Dx y_u + Dy y_v) + Dz(rho0 w_a)),
//     w_a = B (y_w + lambda g H0 y_theta / (G0 rho0)),
// where Dx, Dy, Dz are the direct-stiffness-summed line derivatives, B zeroes
// w on the bottom and top, Dxx = Dx Dx and Dyy = Dy Dy (rho0 depends on z
// only, so it cancels in the horizontal terms), and
//     V = G0 Dz B (Dz + g / G0)
// is the vertical part (rho0 cancels there too), a band of half-width 2N per
// column.  The solution is
// then u = y_u - lambda Dx P / rho0, v = y_v - lambda Dy P / rho0,
// w = w_a - lambda B (Dz P / rho0 + g P / (G0 rho0)), and, with r = b - S P,
// rho' = (P - H0 y_theta + r) / G0 (the continuity row written through S).
//
// Kernels (one thread per node; node I = i + nx (j + ny k), i fastest):
//   k_schur_apply   S applied to a field in one pass (composed x and y line
//                   stencils of width 4N+1, the vertical band; x-z slabs
//                   staged in LDS), with an
//                   epilogue for residuals, the Chebyshev (PBNO) recurrence
//                   and fused partial dot products against Krylov vectors
//   k_schur_rhs     b from the 5-field y
//   k_schur_extract the 5-field solution (plus optional stage shifts)
//   k_dots, k_finish, k_cgs_update, k_normalize, k_givens, k_combine:
//                   the GMRES vector work; every reduction is two-pass with
//                   a fixed order, so results do not depend on timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <vector>

#include "numa_internal.h"

namespace numa {

namespace {

constexpr int kTB = 256;  // threads per block of every kernel here

inline long nblocks(long n) { return (n + kTB - 1) / kTB; }

// The node kernels run on a 3D grid: blocks of 32 (i) x 8 (j) threads, one
// plane k per blockIdx.z, so no thread divides to find its node.
constexpr int kBX = 32, kBY = 8;

__device__ inline int wrap(int i, int n)
{
    while (i < 0) i += n;
    while (i >= n) i -= n;
    return i;
}

// one wrap is enough when the stencil reach is at most the line length
template <bool ONE>
__device__ inline int wrapx(int i, int n)
{
    if constexpr (ONE) {
        i += i < 0 ? n : 0;
        return i - (i >= n ? n : 0);
    } else {
        return wrap(i, n);
    }
}

struct Node {
    int i, j, k;
    long I;
    bool ok;
};

__device__ inline Node node_of(int nx, int ny)
{
    Node n;
    n.i = blockIdx.x * kBX + threadIdx.x;
    n.j = blockIdx.y * kBY + threadIdx.y;
    n.k = blockIdx.z;
    n.ok = n.i < nx && n.j < ny;
    n.I = (long(n.k) * ny + n.j) * nx + n.i;
    return n;
}

__device__ inline int tid_flat() { return threadIdx.y * kBX + threadIdx.x; }

// Sum over the 256 threads of a block in a fixed order (wave shuffles, then
// the four wave sums); every thread must call it.
__device__ inline double block_sum(double v, double *sh)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int ft = threadIdx.y * blockDim.x + threadIdx.x;
    const int lane = ft & 63, wid = ft >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    const double t = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return t;
}

// Block sums of nv values per thread (nv <= M) in one barrier: wave
// shuffles, then thread v adds the four wave sums of value v in a fixed
// order and stores it at out[v * stride].  Every thread must call it.
template <int M>
__device__ inline void block_sums(const double (&val)[M], int nv, double *sh /* [4][M] */, double *out, long stride)
{
    const int ft = threadIdx.y * blockDim.x + threadIdx.x;
    const int lane = ft & 63, wid = ft >> 6;
#pragma unroll
    for (int v = 0; v < M; ++v) {
        if (v < nv) {
            double x = val[v];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
            if (lane == 0) sh[wid * M + v] = x;
        }
    }
    __syncthreads();
    if (ft < nv) out[long(ft) * stride] = (sh[ft] + sh[M + ft]) + (sh[2 * M + ft] + sh[3 * M + ft]);
}

struct OpTables {
    const double *wxx, *wyy;  // [N][4N+1] composed x, y stencils by local index
    const double *vb;         // [nz][4N+1] vertical band, offsets -2N..2N
    const double *wxy;        // [2][N][2N+1] first-derivative x, y stencils
    const double *dzb;        // [nz][2N+1] first-derivative column band
    const double *rho0, *G0, *H0;
    int nx, ny, nz;
    long np;
};

enum { AP_AXPY = 0, AP_CHEB = 1 };

struct ApplyArgs {
    const double *in;
    double scale;  // the operand is scale * in
    int mode;
    // AP_AXPY: out = alpha * x + beta * S x + gamma * aux   (x = scale * in)
    double *out;
    double alpha, beta, gamma;
    const double *aux;
    // AP_CHEB (one step of the Chebyshev recurrence, d = scale * in):
    // res = res_in - S d; d' = c1 d + c2 res; z = z_in + d'.  Null res_in
    // means res_in = in (unscaled), null z_in means z_in = d.
    const double *res_in, *z_in;
    double *res_out, *d_out, *z_out;
    double c1, c2;
    // fused partial dots of the AP_AXPY output with V_0..V_{nv-1}
    const double *V;
    int nv;
    double *part;
    long nblk;
    const int *stop;
    double lam2;
};

// k_schur_apply: a block owns 32 nodes along x by 8 levels of one y line.
// The x-z slab it needs (the 32 x 8 nodes plus 2N on every side, zero
// below the bottom and above the top) is staged in LDS with the x and
// vertical coefficient rows, so the x and z taps of a node are LDS reads;
// its y taps are coalesced global reads of neighbouring lines of the plane.
constexpr int kAX = 32, kAK = 8;

template <int N>
struct ApplyTile {
    static constexpr int W = 4 * N + 1;
    static constexpr int R = kAK + 4 * N;  // slab rows (levels)
    static constexpr int C = kAX + 4 * N;  // slab columns (x)
};

template <int N, bool ONE>
__global__ __launch_bounds__(kTB) void k_schur_apply(OpTables t, ApplyArgs a)
{
    using G = ApplyTile<N>;
    constexpr int W = G::W;
    __shared__ double slab[G::R * G::C];
    __shared__ double cx[N * W], cz[kAK * W];
    __shared__ double sh[4 * 64];
    if (a.stop && *a.stop) return;
    const int nx = t.nx, ny = t.ny, nz = t.nz;
    const int tx = threadIdx.x, tk = threadIdx.y, tid = tk * kAX + tx;
    // XCD-aware order: workgroup w runs on XCD w mod 8; XCD x takes one
    // contiguous range of logical blocks, ordered x tile, then level tile,
    // then y line, so that the y neighbours and the slab halos a block
    // reads were mostly fetched into the same XCD's L2 by its neighbours.
    const int gx = (nx + kAX - 1) / kAX, gk = (nz + kAK - 1) / kAK;
    const long nb = long(gx) * gk * ny, w = blockIdx.x;
    const long per = nb / 8, rem = nb % 8, xcd = w % 8;
    const long L = xcd * per + min(xcd, rem) + w / 8;
    const int bx = int(L % gx), bk = int((L / gx) % gk), j = int(L / (long(gx) * gk));
    const int i0 = bx * kAX, k0 = bk * kAK;
    const long plane = long(nx) * ny;
    const double *in = a.in;
    for (int e = tid; e < G::R * G::C; e += kTB) {
        const int r = e / G::C, cc = e - r * G::C;
        // the slab is 32 + 4N wide whatever nx is: wrap as often as needed
        const int k = k0 - 2 * N + r, i = wrap(i0 - 2 * N + cc, nx);
        slab[e] = (k >= 0 && k < nz) ? in[long(k) * plane + long(j) * nx + i] : 0.0;
    }
    for (int e = tid; e < N * W; e += kTB) cx[e] = t.wxx[e];
    for (int e = tid; e < kAK * W; e += kTB) {
        const int k = k0 + e / W;
        cz[e] = k < nz ? t.vb[long(k) * W + e % W] : 0.0;
    }
    __syncthreads();
    const int i = i0 + tx, k = k0 + tk;
    const bool ok = i < nx && k < nz;
    const long I = long(k) * plane + long(j) * nx + i;
    double val = 0.0;
    if (ok) {
        const double *wx = cx + (i % N) * W, *wz = cz + tk * W, *wy = t.wyy + (j % N) * W;
        double sx = 0.0, sy = 0.0, sv = 0.0;
#pragma unroll
        for (int m = 0; m < W; ++m) sx += wx[m] * slab[(tk + 2 * N) * G::C + tx + m];
#pragma unroll
        for (int m = 0; m < W; ++m) sv += wz[m] * slab[(tk + m) * G::C + tx + 2 * N];
        const double *rowk = in + long(k) * plane + i;
#pragma unroll
        for (int m = 0; m < W; ++m) sy += wy[m] * rowk[long(wrapx<ONE>(j - 2 * N + m, ny)) * nx];
        const double center = slab[(tk + 2 * N) * G::C + tx + 2 * N];
        const double Sx = a.scale * (center - a.lam2 * (sv + t.G0[k] * (sx + sy)));
        const double x = a.scale * center;
        if (a.mode == AP_AXPY) {
            val = a.beta * Sx;
            if (a.alpha != 0.0) val += a.alpha * x;
            if (a.aux) val += a.gamma * a.aux[I];
            a.out[I] = val;
        } else {
            const double res = (a.res_in ? a.res_in[I] : center) - Sx;
            const double dn = a.c1 * x + a.c2 * res;
            a.z_out[I] = (a.z_in ? a.z_in[I] : x) + dn;
            if (a.res_out) a.res_out[I] = res;
            if (a.d_out) a.d_out[I] = dn;
        }
    }
    // partial dots with the Krylov vectors, 8 per barrier (each group of 8
    // has its own LDS area, so no barrier is needed between groups)
    const long blk = L;
    for (int v0 = 0; v0 < a.nv; v0 += 8) {
        double q[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) q[u] = (ok && v0 + u < a.nv) ? val * a.V[long(v0 + u) * t.np + I] : 0.0;
        block_sums<8>(q, min(8, a.nv - v0), sh + 4 * 8 * ((v0 / 8) & 7), a.part + long(v0) * a.nblk + blk, a.nblk);
    }
}

// One step of the Chebyshev recurrence of the polynomial preconditioner in
// FP32 (the mixed-precision preconditioner): the same one-pass operator and
// tiling as k_schur_apply's AP_CHEB mode, with FP32 fields, slab, tables and
// sums.  res = res_in - S d, d' = c1 d + c2 res, z = z_in + d' with
// d = scale * in (null res_in: res_in = in; null z_in: z_in = d).
struct ChebArgs32 {
    const float *in, *res_in, *z_in;
    float *res_out, *d_out, *z_out;
    float scale, c1, c2, lam2;
    const int *stop;
};

struct OpTables32 {
    const float *wxx, *wyy, *vb, *G0;
    int nx, ny, nz;
};

template <int N, bool ONE>
__global__ __launch_bounds__(kTB) void k_schur_cheb32(OpTables32 t, ChebArgs32 a)
{
    using G = ApplyTile<N>;
    constexpr int W = G::W;
    __shared__ float slab[G::R * G::C];
    __shared__ float cx[N * W], cz[kAK * W];
    if (a.stop && *a.stop) return;
    const int nx = t.nx, ny = t.ny, nz = t.nz;
    const int tx = threadIdx.x, tk = threadIdx.y, tid = tk * kAX + tx;
    // XCD-aware block order, as k_schur_apply
    const int gx = (nx + kAX - 1) / kAX, gk = (nz + kAK - 1) / kAK;
    const long nb = long(gx) * gk * ny, w = blockIdx.x;
    const long per = nb / 8, rem = nb % 8, xcd = w % 8;
    const long L = xcd * per + min(xcd, rem) + w / 8;
    const int bx = int(L % gx), bk = int((L / gx) % gk), j = int(L / (long(gx) * gk));
    const int i0 = bx * kAX, k0 = bk * kAK;
    const long plane = long(nx) * ny;
    const float *in = a.in;
    for (int e = tid; e < G::R * G::C; e += kTB) {
        const int r = e / G::C, cc = e - r * G::C;
        const int k = k0 - 2 * N + r, i = wrap(i0 - 2 * N + cc, nx);
        slab[e] = (k >= 0 && k < nz) ? in[long(k) * plane + long(j) * nx + i] : 0.0f;
    }
    for (int e = tid; e < N * W; e += kTB) cx[e] = t.wxx[e];
    for (int e = tid; e < kAK * W; e += kTB) {
        const int k = k0 + e / W;
        cz[e] = k < nz ? t.vb[long(k) * W + e % W] : 0.0f;
    }
    __syncthreads();
    const int i = i0 + tx, k = k0 + tk;
    if (!(i < nx && k < nz)) return;
    const long I = long(k) * plane + long(j) * nx + i;
    const float *wx = cx + (i % N) * W, *wz = cz + tk * W, *wy = t.wyy + (j % N) * W;
    float sx = 0.0f, sy = 0.0f, sv = 0.0f;
#pragma unroll
    for (int m = 0; m < W; ++m) sx += wx[m] * slab[(tk + 2 * N) * G::C + tx + m];
#pragma unroll
    for (int m = 0; m < W; ++m) sv += wz[m] * slab[(tk + m) * G::C + tx + 2 * N];
    const float *rowk = in + long(k) * plane + i;
#pragma unroll
    for (int m = 0; m < W; ++m) sy += wy[m] * rowk[long(wrapx<ONE>(j - 2 * N + m, ny)) * nx];
    const float center = slab[(tk + 2 * N) * G::C + tx + 2 * N];
    const float Sx = a.scale * (center - a.lam2 * (sv + t.G0[k] * (sx + sy)));
    const float x = a.scale * center;
    const float res = (a.res_in ? a.res_in[I] : center) - Sx;
    const float dn = a.c1 * x + a.c2 * res;
    a.z_out[I] = (a.z_in ? a.z_in[I] : x) + dn;
    if (a.res_out) a.res_out[I] = res;
    if (a.d_out) a.d_out[I] = dn;
}

__global__ __launch_bounds__(kTB) void k_to_f32(float *out, const double *in, long n, const int *stop)
{
    if (stop && *stop) return;
    const long i = long(blockIdx.x) * kTB + threadIdx.x;
    if (i < n) out[i] = float(in[i]);
}

__global__ __launch_bounds__(kTB) void k_to_f64(double *out, const float *in, long n, const int *stop)
{
    if (stop && *stop) return;
    const long i = long(blockIdx.x) * kTB + threadIdx.x;
    if (i < n) out[i] = double(in[i]);
}

// first derivatives along x, y (line stencils) and z (column band) of f at I
template <int N, bool ONE>
__device__ inline double dline(const double *w, const double *f, int i, int n, long base, long stride)
{
    const int a = i % N, e0 = i - a;
    const double *c = w + a * (2 * N + 1);
    double s = 0.0;
#pragma unroll
    for (int m = 0; m <= 2 * N; ++m) s += c[m] * f[base + long(wrapx<ONE>(e0 - N + m, n)) * stride];
    return s;
}

template <int N, bool ONE>
__global__ __launch_bounds__(kTB) void k_schur_rhs(OpTables t, const double *y, double *b, double lam, double g)
{
    const Node n = node_of(t.nx, t.ny);
    if (!n.ok) return;
    const long I = n.I;
    const int i = n.i, j = n.j, k = n.k;
    const long np = t.np, plane = long(t.nx) * t.ny;
    const double *yr = y, *yu = y + np, *yv = y + 2 * np, *yw = y + 3 * np, *yt = y + 4 * np;
    const double dxu = dline<N, ONE>(t.wxy, yu, i, t.nx, long(k) * plane + long(j) * t.nx, 1);
    const double dyv = dline<N, ONE>(t.wxy + N * (2 * N + 1), yv, j, t.ny, long(k) * plane + i, t.nx);
    // Dz(rho0 w_a)
    const double *dz = t.dzb + long(k) * (2 * N + 1);
    const long col = long(j) * t.nx + i;
    double dzw = 0.0;
#pragma unroll
    for (int m = 0; m <= 2 * N; ++m) {
        const int kk = k - N + m;
        if (kk <= 0 || kk >= t.nz - 1) continue;  // outside, or a wall level (w_a = 0)
        const long J = long(kk) * plane + col;
        const double wa = yw[J] + lam * g * t.H0[kk] * yt[J] / (t.G0[kk] * t.rho0[kk]);
        dzw += dz[m] * (t.rho0[kk] * wa);
    }
    const double G0 = t.G0[k];
    b[I] = G0 * yr[I] + t.H0[k] * yt[I] - lam * G0 * (t.rho0[k] * (dxu + dyv) + dzw);
}

struct ExtractArgs {
    const double *y, *P, *r;
    double *out;
    const double *in0, *in1;  // out = X + d0 in0 + d1 in1 (nullable)
    double d0, d1;
    double lam, g;
};

template <int N, bool ONE>
__global__ __launch_bounds__(kTB) void k_schur_extract(OpTables t, ExtractArgs a)
{
    const Node n = node_of(t.nx, t.ny);
    if (!n.ok) return;
    const long I = n.I;
    const int i = n.i, j = n.j, k = n.k;
    const long np = t.np, plane = long(t.nx) * t.ny;
    const double *P = a.P;
    const double dxp = dline<N, ONE>(t.wxy, P, i, t.nx, long(k) * plane + long(j) * t.nx, 1);
    const double dyp = dline<N, ONE>(t.wxy + N * (2 * N + 1), P, j, t.ny, long(k) * plane + i, t.nx);
    const double *dz = t.dzb + long(k) * (2 * N + 1);
    const double *pc = P + long(j) * t.nx + i;
    double dzp = 0.0;
#pragma unroll
    for (int m = 0; m <= 2 * N; ++m) {
        const int kk = k - N + m;
        if (kk >= 0 && kk < t.nz) dzp += dz[m] * pc[long(kk) * plane];
    }
    const double r0 = t.rho0[k], G0 = t.G0[k], H0 = t.H0[k];
    const double yr = a.y[I], yu = a.y[np + I], yv = a.y[2 * np + I], yw = a.y[3 * np + I], yt = a.y[4 * np + I];
    double X[5];
    X[0] = (P[I] - H0 * yt + a.r[I]) / G0;
    X[1] = yu - a.lam * dxp / r0;
    X[2] = yv - a.lam * dyp / r0;
    const bool wall = k == 0 || k == t.nz - 1;
    X[3] = wall ? 0.0 : yw + a.lam * a.g * H0 * yt / (G0 * r0) - a.lam * (dzp / r0 + a.g * P[I] / (G0 * r0));
    X[4] = yt;
    (void)yr;
#pragma unroll
    for (int f = 0; f < 5; ++f) {
        double v = X[f];
        if (a.in0) v += a.d0 * a.in0[f * np + I];
        if (a.in1) v += a.d1 * a.in1[f * np + I];
        a.out[f * np + I] = v;
    }
}

// out = c0 in0 + c1 in1 + c2 in2 over n elements (null inputs skipped)
__global__ __launch_bounds__(kTB) void k_lincomb(double *out, const double *in0, double c0, const double *in1, double c1,
                                                 const double *in2, double c2, long n)
{
    const long I = long(blockIdx.x) * kTB + threadIdx.x;
    if (I >= n) return;
    double v = c0 * in0[I];
    if (in1) v += c1 * in1[I];
    if (in2) v += c2 * in2[I];
    out[I] = v;
}

// partial dots of w with V_0..V_{nv-1} (V == null: of w with itself)
__global__ __launch_bounds__(kTB) void k_dots(const double *w, const double *V, int nv, long n, double *part,
                                              long nblk, const int *stop)
{
    __shared__ double sh[4];
    if (stop && *stop) return;
    const long I = long(blockIdx.x) * kTB + threadIdx.x;
    const bool ok = I < n;
    const double wv = ok ? w[I] : 0.0;
    for (int v = 0; v < nv; ++v) {
        const double o = ok ? (V ? V[long(v) * n + I] : wv) : 0.0;
        const double s = block_sum(wv * o, sh);
        if (threadIdx.x == 0) part[long(v) * nblk + blockIdx.x] = s;
    }
}

// Second pass: block v sums the nblk partials of dot v (fixed order) into
// h[v] (sqrt of it if root); with H, also H[v*m + col] = h[v] (add: +=).
__global__ __launch_bounds__(kTB) void k_finish(const double *part, long nblk, double *h, int root, double *H, int m,
                                                int col, int add, const int *stop)
{
    __shared__ double sh[4];
    if (stop && *stop) return;
    const int v = blockIdx.x;
    // four independent partial sums per thread, so that four loads are in
    // flight at a time; combined in a fixed order (reproducible)
    const double *pv = part + long(v) * nblk;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    long b = threadIdx.x;
    for (; b + 3 * kTB < nblk; b += 4 * kTB) {
        s0 += pv[b];
        s1 += pv[b + kTB];
        s2 += pv[b + 2 * kTB];
        s3 += pv[b + 3 * kTB];
    }
    for (; b < nblk; b += kTB) s0 += pv[b];
    double s = block_sum((s0 + s1) + (s2 + s3), sh);
    if (threadIdx.x == 0) {
        if (root) s = std::sqrt(s);
        h[v] = s;
        if (H) {
            double *e = H + long(v) * m + col;
            *e = add ? *e + s : s;
        }
    }
}

// w -= sum_v h[v] V_v; then partial dots of the new w with V_0..V_{nvd-1}
// (nvd < 0: the partial of |w|^2 alone).  The nv <= M vectors are read once
// into registers for both.
template <int M>
__global__ __launch_bounds__(kTB) void k_cgs_update(double *w, const double *V, int nv, const double *h, long n,
                                                    int nvd, double *part, long nblk, const int *stop)
{
    __shared__ double sh[4 * M];
    if (stop && *stop) return;
    const long I = long(blockIdx.x) * kTB + threadIdx.x;
    const bool ok = I < n;
    double vv[M];
    double wv = 0.0;
    if (ok) {
        wv = w[I];
#pragma unroll
        for (int v = 0; v < M; ++v) {
            vv[v] = v < nv ? V[long(v) * n + I] : 0.0;
            if (v < nv) wv -= h[v] * vv[v];
        }
        w[I] = wv;
    } else {
#pragma unroll
        for (int v = 0; v < M; ++v) vv[v] = 0.0;
    }
    if (nvd < 0) {
        double q[1] = {wv * wv};
        block_sums<1>(q, 1, sh, part + blockIdx.x, nblk);
    } else {
#pragma unroll
        for (int v = 0; v < M; ++v) vv[v] *= wv;
        block_sums<M>(vv, nvd, sh, part + blockIdx.x, nblk);
    }
}

// out = in / s (s on the device; 0 where s is not positive)
__global__ __launch_bounds__(kTB) void k_normalize(double *out, const double *in, const double *s, long n,
                                                   const int *stop)
{
    if (stop && *stop) return;
    const long I = long(blockIdx.x) * kTB + threadIdx.x;
    if (I >= n) return;
    const double d = *s;
    out[I] = d > 0.0 ? in[I] / d : 0.0;
}

// out = c in (host scalar)
__global__ __launch_bounds__(kTB) void k_scale(double *out, const double *in, double c, long n)
{
    const long I = long(blockIdx.x) * kTB + threadIdx.x;
    if (I < n) out[I] = c * in[I];
}

// Givens step of column j of the Hessenberg matrix (row stride m): the
// earlier rotations, a new one that zeroes H[j+1][j], the rotated residual
// vector g; stop[0] = 1 once |g[j+1]| <= tolb; stop[1] counts iterations.
// One wavefront: its lanes load column j of H and the previous rotations
// into LDS together, then lane 0 applies the rotations in order (the same
// arithmetic as a sequential loop over global memory, without its chain of
// dependent global loads).  m <= 63.
__global__ __launch_bounds__(64) void k_givens(double *H, double *cs, double *sn, double *g, int j, int m,
                                               double tolb, int *stop)
{
    __shared__ double col[65], cc[64], ss[64];
    if (stop[0]) return;
    const int t = threadIdx.x;
    for (int i = t; i <= j + 1; i += 64) col[i] = H[i * m + j];
    for (int i = t; i < j; i += 64) {
        cc[i] = cs[i];
        ss[i] = sn[i];
    }
    __syncthreads();
    if (t != 0) return;
    double a = col[0];
    for (int i = 0; i < j; ++i) {
        const double b = col[i + 1];
        H[i * m + j] = cc[i] * a + ss[i] * b;
        a = -ss[i] * a + cc[i] * b;  // the new H[i+1][j]
    }
    const double b = col[j + 1], r = std::hypot(a, b);
    const double c = r > 0.0 ? a / r : 1.0, sv = r > 0.0 ? b / r : 0.0;
    cs[j] = c;
    sn[j] = sv;
    H[j * m + j] = r;
    H[(j + 1) * m + j] = 0.0;
    const double gj = g[j];
    g[j + 1] = -sv * gj;
    g[j] = c * gj;
    stop[1] += 1;
    if (std::fabs(g[j + 1]) <= tolb) stop[0] = 1;
}

// start of a cycle: g = (beta, 0, ...), flags cleared
__global__ void k_cycle_init(double *g, int m, double beta, int *stop)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    g[0] = beta;
    for (int i = 1; i <= m; ++i) g[i] = 0.0;
    stop[0] = 0;
    stop[1] = 0;
}

// out (+)= sum_v c[v] V_v
__global__ __launch_bounds__(kTB) void k_combine(double *out, const double *V, const double *c, int nv, long n,
                                                 int add)
{
    const long I = long(blockIdx.x) * kTB + threadIdx.x;
    if (I >= n) return;
    double s = add ? out[I] : 0.0;
    for (int v = 0; v < nv; ++v) s += c[v] * V[long(v) * n + I];
    out[I] = s;
}

// power-method start vector: frac(I * 2654435769 / 2^32) - 1/2
__global__ __launch_bounds__(kTB) void k_start_vector(double *v, long n)
{
    const long I = long(blockIdx.x) * kTB + threadIdx.x;
    if (I >= n) return;
    const uint32_t h = uint32_t(uint64_t(I) * 2654435769u);
    v[I] = double(h) / 4294967296.0 - 0.5;
}

template <typename F>
hipError_t dispatch3(int N, F &&f)
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

// Device state of the 3D-IMEX solver of one context.
struct Imex3d {
    int restart = 0, order = -1, maxit = 0, power_steps = 0;
    double dt = 0, lambda = 0, lmin = 1, lmax = 2;
    long np = 0, nblk = 0, nblk3 = 0;  // blocks of the 1D vector kernels and of the apply grid
    void *block = nullptr;  // one allocation for everything below
    double *wxx = nullptr, *wyy = nullptr, *vb = nullptr;
    double *V = nullptr;                                   // (restart+1) np
    double *Z = nullptr;                                   // restart np (flexible GMRES)
    double *b = nullptr, *x = nullptr, *r = nullptr, *z = nullptr, *w = nullptr;
    double *cres = nullptr, *d0 = nullptr, *d1 = nullptr;  // Chebyshev recurrence
    double *part = nullptr;                                // (restart+1) nblk
    double *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *hb = nullptr, *yc = nullptr;
    double *R1 = nullptr, *Q2 = nullptr, *E3 = nullptr, *ACC = nullptr;  // 5 np each
    // the FP32 preconditioner: tables and its five work fields
    int pbno32 = 0;
    float *wxx32 = nullptr, *wyy32 = nullptr, *vb32 = nullptr, *G032 = nullptr;
    float *r32 = nullptr, *cres32 = nullptr, *d032 = nullptr, *d132 = nullptr, *z32 = nullptr;
    int *stop = nullptr;
    std::vector<double> hH, hg, hy;
};

namespace {

OpTables op_tables(const numa_ctx *c)
{
    OpTables t{};
    t.wxx = c->imex->wxx;
    t.wyy = c->imex->wyy;
    t.vb = c->imex->vb;
    t.wxy = c->lev.wxy;
    t.dzb = c->lev.dzb;
    t.rho0 = c->lev.rho0;
    t.G0 = c->lev.G0;
    t.H0 = c->lev.H0;
    t.nx = int(c->nx);
    t.ny = int(c->ny);
    t.nz = int(c->nz);
    t.np = c->np;
    return t;
}

// Composed stencil Dxx = Dx Dx of a periodic line of n nodes from the
// first-derivative stencils w [N][2N+1] (node e0 - N + m for local index a,
// e0 the element start): rows a = 0..N-1, offsets -2N..2N; where offsets
// alias on a short line the coefficient is kept at the first of them.
void composed_line(const double *w, int N, int n, std::vector<double> &out)
{
    const int ns = 2 * N + 1, W = 4 * N + 1;
    auto row = [&](int i, std::vector<double> &r) {
        r.assign(n, 0.0);
        const int a = i % N, e0 = i - a;
        for (int m = 0; m < ns; ++m) r[((e0 - N + m) % n + n) % n] += w[a * ns + m];
    };
    out.assign(size_t(N) * W, 0.0);
    std::vector<double> ra, rl, acc;
    for (int a = 0; a < N; ++a) {
        row(a, ra);
        acc.assign(n, 0.0);
        for (int l = 0; l < n; ++l) {
            if (ra[l] == 0.0) continue;
            row(l, rl);
            for (int q = 0; q < n; ++q) acc[q] += ra[l] * rl[q];
        }
        std::vector<char> used(n, 0);
        for (int m = 0; m < W; ++m) {
            const int col = ((a - 2 * N + m) % n + n) % n;
            if (used[col]) continue;
            used[col] = 1;
            out[a * W + m] = acc[col];
        }
    }
}

// Vertical band V = G0 Dz B (Dz + g/G0), [nz][4N+1] (rho0 of the vertical
// momentum flux cancels against the 1/rho0 of the pressure gradient)
void vertical_band(const std::vector<double> &dzb, const std::vector<double> &G0, double grav, int N, int nz,
                   std::vector<double> &out)
{
    const int ns = 2 * N + 1, W = 4 * N + 1;
    auto dz = [&](int k, int l) -> double {
        const int m = l - k + N;
        return (m >= 0 && m < ns) ? dzb[size_t(k) * ns + m] : 0.0;
    };
    out.assign(size_t(nz) * W, 0.0);
    for (int k = 0; k < nz; ++k)
        for (int m = 0; m < W; ++m) {
            const int l = k - 2 * N + m;
            if (l < 0 || l >= nz) continue;
            double s = 0.0;
            for (int q = std::max(1, k - N); q <= std::min(nz - 2, k + N); ++q) {  // B: interior levels only
                double inner = dz(q, l);
                if (q == l) inner += grav / G0[l];
                s += dz(k, q) * inner;
            }
            out[size_t(k) * W + m] = G0[k] * s;
        }
}

dim3 node_grid(const numa_ctx *c)
{
    return dim3(unsigned((c->nx + kBX - 1) / kBX), unsigned((c->ny + kBY - 1) / kBY), unsigned(c->nz));
}

long node_grid_blocks(const numa_ctx *c)
{
    const dim3 g = node_grid(c);
    return long(g.x) * g.y * g.z;
}

// the single-wrap form needs the widest stencil (2N each side) within a line
bool one_wrap(const numa_ctx *c) { return c->nx >= 2 * c->N && c->ny >= 2 * c->N; }

dim3 apply_grid(const numa_ctx *c)
{
    return dim3(unsigned(((c->nx + kAX - 1) / kAX) * c->ny * ((c->nz + kAK - 1) / kAK)));
}

long apply_grid_blocks(const numa_ctx *c)
{
    const dim3 g = apply_grid(c);
    return long(g.x) * g.y * g.z;
}

template <int N>
hipError_t apply_launch(numa_ctx *c, const ApplyArgs &a)
{
    if (one_wrap(c))
        hipLaunchKernelGGL((k_schur_apply<N, true>), apply_grid(c), dim3(kAX, kAK), 0, c->stream, op_tables(c), a);
    else
        hipLaunchKernelGGL((k_schur_apply<N, false>), apply_grid(c), dim3(kAX, kAK), 0, c->stream, op_tables(c), a);
    return hipGetLastError();
}

hipError_t apply(numa_ctx *c, ApplyArgs a)
{
    a.lam2 = c->imex->lambda * c->imex->lambda;
    a.nblk = c->imex->nblk3;
    return dispatch3(c->N, [&](auto n) { return apply_launch<decltype(n)::value>(c, a); });
}

ApplyArgs axpy_args(const double *in, double *out, double alpha, double beta, double gamma, const double *aux)
{
    ApplyArgs a{};
    a.in = in;
    a.scale = 1.0;
    a.mode = AP_AXPY;
    a.out = out;
    a.alpha = alpha;
    a.beta = beta;
    a.gamma = gamma;
    a.aux = aux;
    return a;
}

hipError_t lincomb(numa_ctx *c, double *out, const double *in0, double c0, const double *in1, double c1,
                   const double *in2, double c2, long n)
{
    hipLaunchKernelGGL(k_lincomb, dim3(unsigned(nblocks(n))), dim3(kTB), 0, c->stream, out, in0, c0, in1, c1, in2, c2,
                       n);
    return hipGetLastError();
}

// |v| into h[0] on the device
hipError_t norm_dev(numa_ctx *c, const double *v, double *h)
{
    Imex3d &s = *c->imex;
    hipLaunchKernelGGL(k_dots, dim3(unsigned(s.nblk)), dim3(kTB), 0, c->stream, v, nullptr, 1, s.np, s.part, s.nblk,
                       nullptr);
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kTB), 0, c->stream, s.part, s.nblk, h, 1, nullptr, 0, 0, 0, nullptr);
    return hipGetLastError();
}

hipError_t norm_host(numa_ctx *c, const double *v, double *out)
{
    hipError_t e = norm_dev(c, v, c->imex->hb);
    if (e == hipSuccess) e = hipMemcpyAsync(out, c->imex->hb, sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e;
}

template <int N>
hipError_t cheb32_launch(numa_ctx *c, const ChebArgs32 &a)
{
    const Imex3d &s = *c->imex;
    OpTables32 t{s.wxx32, s.wyy32, s.vb32, s.G032, int(c->nx), int(c->ny), int(c->nz)};
    if (one_wrap(c))
        hipLaunchKernelGGL((k_schur_cheb32<N, true>), apply_grid(c), dim3(kAX, kAK), 0, c->stream, t, a);
    else
        hipLaunchKernelGGL((k_schur_cheb32<N, false>), apply_grid(c), dim3(kAX, kAK), 0, c->stream, t, a);
    return hipGetLastError();
}

// dst = s(S) src with the recurrence in FP32 (order >= 1): src rounded to
// FP32, p FP32 steps, the result widened to FP64
hipError_t precondition32(numa_ctx *c, const double *src, double *dst)
{
    Imex3d &s = *c->imex;
    const double theta = 0.5 * (s.lmax + s.lmin), delta = 0.5 * (s.lmax - s.lmin);
    const double sigma = theta / delta;
    const unsigned nb = unsigned(nblocks(s.np));
    hipLaunchKernelGGL(k_to_f32, dim3(nb), dim3(kTB), 0, c->stream, s.r32, src, s.np, nullptr);
    double rho = 1.0 / sigma;
    const float *din = s.r32;
    float *dbuf[2] = {s.d032, s.d132};
    for (int k = 1; k <= s.order; ++k) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        ChebArgs32 a{};
        a.in = din;
        a.scale = float(k == 1 ? 1.0 / theta : 1.0);
        a.res_in = k == 1 ? nullptr : s.cres32;
        a.z_in = k == 1 ? nullptr : s.z32;
        a.z_out = s.z32;
        a.res_out = k < s.order ? s.cres32 : nullptr;
        a.d_out = k < s.order ? dbuf[k & 1] : nullptr;
        a.c1 = float(rn * rho);
        a.c2 = float(2.0 * rn / delta);
        a.lam2 = float(s.lambda * s.lambda);
        hipError_t e = dispatch3(c->N, [&](auto n) { return cheb32_launch<decltype(n)::value>(c, a); });
        if (e != hipSuccess) return e;
        din = dbuf[k & 1];
        rho = rn;
    }
    hipLaunchKernelGGL(k_to_f64, dim3(nb), dim3(kTB), 0, c->stream, dst, s.z32, s.np, nullptr);
    return hipGetLastError();
}

// dst = s(S) src, the PBNO polynomial (order < 0: dst = src); in FP32 when
// the mixed-precision preconditioner is on
hipError_t precondition(numa_ctx *c, const double *src, double *dst)
{
    Imex3d &s = *c->imex;
    if (s.order < 0) return hipMemcpyAsync(dst, src, sizeof(double) * s.np, hipMemcpyDeviceToDevice, c->stream);
    if (s.pbno32 && s.order >= 1) return precondition32(c, src, dst);
    const double theta = 0.5 * (s.lmax + s.lmin), delta = 0.5 * (s.lmax - s.lmin);
    const double sigma = theta / delta;
    if (s.order == 0) {
        hipLaunchKernelGGL(k_scale, dim3(unsigned(nblocks(s.np))), dim3(kTB), 0, c->stream, dst, src, 1.0 / theta,
                           s.np);
        return hipGetLastError();
    }
    double rho = 1.0 / sigma;
    const double *din = src;
    double *dbuf[2] = {s.d0, s.d1};
    for (int k = 1; k <= s.order; ++k) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        ApplyArgs a{};
        a.mode = AP_CHEB;
        a.in = din;
        a.scale = k == 1 ? 1.0 / theta : 1.0;
        a.res_in = k == 1 ? nullptr : s.cres;
        a.z_in = k == 1 ? nullptr : dst;
        a.z_out = dst;
        a.res_out = k < s.order ? s.cres : nullptr;
        a.d_out = k < s.order ? dbuf[k & 1] : nullptr;
        a.c1 = rn * rho;
        a.c2 = 2.0 * rn / delta;
        hipError_t e = apply(c, a);
        if (e != hipSuccess) return e;
        din = dbuf[k & 1];
        rho = rn;
    }
    return hipSuccess;
}

template <int N>
hipError_t rhs_kernel_launch(numa_ctx *c, const double *y, double *b)
{
    const double lam = c->imex->lambda, g = c->eos.grav;
    if (one_wrap(c))
        hipLaunchKernelGGL((k_schur_rhs<N, true>), node_grid(c), dim3(kBX, kBY), 0, c->stream, op_tables(c), y, b, lam, g);
    else
        hipLaunchKernelGGL((k_schur_rhs<N, false>), node_grid(c), dim3(kBX, kBY), 0, c->stream, op_tables(c), y, b, lam,
                           g);
    return hipGetLastError();
}

template <int N>
hipError_t extract_launch(numa_ctx *c, const ExtractArgs &a)
{
    if (one_wrap(c))
        hipLaunchKernelGGL((k_schur_extract<N, true>), node_grid(c), dim3(kBX, kBY), 0, c->stream, op_tables(c), a);
    else
        hipLaunchKernelGGL((k_schur_extract<N, false>), node_grid(c), dim3(kBX, kBY), 0, c->stream, op_tables(c), a);
    return hipGetLastError();
}

// w -= sum of the nv vectors times hb, with the fused partial dots (nvd)
hipError_t cgs_update(numa_ctx *c, int nv, int nvd)
{
    Imex3d &s = *c->imex;
    const dim3 g(unsigned(s.nblk)), b(kTB);
    if (nv <= 8)
        hipLaunchKernelGGL(k_cgs_update<8>, g, b, 0, c->stream, s.w, s.V, nv, s.hb, s.np, nvd, s.part, s.nblk, s.stop);
    else if (nv <= 16)
        hipLaunchKernelGGL(k_cgs_update<16>, g, b, 0, c->stream, s.w, s.V, nv, s.hb, s.np, nvd, s.part, s.nblk, s.stop);
    else if (nv <= 32)
        hipLaunchKernelGGL(k_cgs_update<32>, g, b, 0, c->stream, s.w, s.V, nv, s.hb, s.np, nvd, s.part, s.nblk, s.stop);
    else
        hipLaunchKernelGGL(k_cgs_update<64>, g, b, 0, c->stream, s.w, s.V, nv, s.hb, s.np, nvd, s.part, s.nblk, s.stop);
    return hipGetLastError();
}

// Back substitution of the rotated Hessenberg system of j columns.
void upper_solve(const std::vector<double> &H, const std::vector<double> &g, int m, int j, std::vector<double> &y)
{
    y.assign(size_t(std::max(j, 1)), 0.0);
    for (int i = j - 1; i >= 0; --i) {
        double t = g[i];
        for (int k = i + 1; k < j; ++k) t -= H[size_t(i) * m + k] * y[k];
        y[i] = t / H[size_t(i) * m + i];
    }
}

}  // namespace

void imex3d_free(numa_ctx *c)
{
    if (!c || !c->imex) return;
    if (c->imex->block) (void)hipFree(c->imex->block);
    delete c->imex;
    c->imex = nullptr;
}

hipError_t imex3d_setup(numa_ctx *c, double dt, int restart, int order, int power_steps, int maxit)
{
    imex3d_free(c);
    Imex3d *s = new Imex3d();
    c->imex = s;
    const int N = c->N, W = 4 * N + 1;
    const long np = c->np, nz = c->nz;
    s->restart = restart;
    s->order = order;
    s->maxit = maxit;
    s->power_steps = power_steps;
    s->dt = dt;
    s->lambda = (1.0 - 1.0 / std::sqrt(2.0)) * dt;
    s->np = np;
    s->nblk = nblocks(np);
    s->nblk3 = apply_grid_blocks(c);
    const long npart = std::max(s->nblk, s->nblk3);
    const int m = restart;
    // sizes in doubles
    const size_t n_tab = size_t(2 * N * W + nz * W);
    const size_t n_vec = size_t(2 * m + 1) * np + 8 * size_t(np) + 20 * size_t(np);
    // FP32 tables and five FP32 work fields, in doubles
    const size_t n_f32 = (size_t(2 * N * W + nz * W + nz) + 5 * size_t(np) + 8) / 2 + 8;
    const size_t n_small = size_t(m + 1) * npart + size_t(m + 1) * m + 4 * size_t(m + 2) + size_t(m + 2);
    const size_t total = n_tab + n_vec + n_small + n_f32 + 64;
    hipError_t e = hipMalloc(&s->block, total * sizeof(double) + 64);
    if (e != hipSuccess) {
        s->block = nullptr;
        return e;
    }
    double *p = static_cast<double *>(s->block);
    s->wxx = p; p += N * W;
    s->wyy = p; p += N * W;
    s->vb = p; p += nz * W;
    s->V = p; p += size_t(m + 1) * np;
    s->Z = p; p += size_t(m) * np;
    s->b = p; p += np;
    s->x = p; p += np;
    s->r = p; p += np;
    s->z = p; p += np;
    s->w = p; p += np;
    s->cres = p; p += np;
    s->d0 = p; p += np;
    s->d1 = p; p += np;
    s->R1 = p; p += 5 * np;
    s->Q2 = p; p += 5 * np;
    s->E3 = p; p += 5 * np;
    s->ACC = p; p += 5 * np;
    s->part = p; p += size_t(m + 1) * npart;
    s->H = p; p += size_t(m + 1) * m;
    s->cs = p; p += m + 2;
    s->sn = p; p += m + 2;
    s->g = p; p += m + 2;
    s->hb = p; p += m + 2;
    s->yc = p; p += m + 2;
    {
        float *f = reinterpret_cast<float *>(p);
        s->wxx32 = f; f += N * W;
        s->wyy32 = f; f += N * W;
        s->vb32 = f; f += nz * W;
        s->G032 = f; f += nz;
        f += (reinterpret_cast<uintptr_t>(f) / sizeof(float)) & 1;  // 8-byte alignment of the fields
        s->r32 = f; f += np;
        s->cres32 = f; f += np;
        s->d032 = f; f += np;
        s->d132 = f; f += np;
        s->z32 = f; f += np;
        p = reinterpret_cast<double *>(f + ((reinterpret_cast<uintptr_t>(f) / sizeof(float)) & 1));
    }
    s->stop = reinterpret_cast<int *>(p);

    // host tables: composed line stencils and the vertical band
    std::vector<double> G0(nz), wxx, wyy, vb;
    e = hipMemcpy(G0.data(), c->lev.G0, sizeof(double) * nz, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    const int ns = 2 * N + 1;
    composed_line(c->ops.wxy.data(), N, int(c->nx), wxx);
    composed_line(c->ops.wxy.data() + N * ns, N, int(c->ny), wyy);
    vertical_band(c->ops.dzb, G0, c->eos.grav, N, int(nz), vb);
    if ((e = hipMemcpy(s->wxx, wxx.data(), sizeof(double) * N * W, hipMemcpyHostToDevice)) != hipSuccess) return e;
    if ((e = hipMemcpy(s->wyy, wyy.data(), sizeof(double) * N * W, hipMemcpyHostToDevice)) != hipSuccess) return e;
    if ((e = hipMemcpy(s->vb, vb.data(), sizeof(double) * nz * W, hipMemcpyHostToDevice)) != hipSuccess) return e;
    {
        std::vector<float> f32;
        auto put = [&](float *dst, const std::vector<double> &v, size_t n) {
            f32.assign(v.begin(), v.begin() + long(n));
            return hipMemcpy(dst, f32.data(), sizeof(float) * n, hipMemcpyHostToDevice);
        };
        if ((e = put(s->wxx32, wxx, size_t(N) * W)) != hipSuccess) return e;
        if ((e = put(s->wyy32, wyy, size_t(N) * W)) != hipSuccess) return e;
        if ((e = put(s->vb32, vb, size_t(nz) * W)) != hipSuccess) return e;
        if ((e = put(s->G032, G0, size_t(nz))) != hipSuccess) return e;
    }
    if ((e = hipMemset(s->stop, 0, 2 * sizeof(int))) != hipSuccess) return e;
    s->hH.assign(size_t(m + 1) * m, 0.0);
    s->hg.assign(size_t(m + 1), 0.0);

    // eigenvalue interval of S: power method from the fixed start vector
    if (power_steps > 0) {
        hipLaunchKernelGGL(k_start_vector, dim3(unsigned(s->nblk)), dim3(kTB), 0, c->stream, s->z, np);
        if ((e = norm_dev(c, s->z, s->hb)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_normalize, dim3(unsigned(s->nblk)), dim3(kTB), 0, c->stream, s->z, s->z, s->hb, np,
                           nullptr);
        for (int it = 0; it < power_steps; ++it) {
            if ((e = apply(c, axpy_args(s->z, s->w, 0.0, 1.0, 0.0, nullptr))) != hipSuccess) return e;
            if ((e = norm_dev(c, s->w, s->hb)) != hipSuccess) return e;
            hipLaunchKernelGGL(k_normalize, dim3(unsigned(s->nblk)), dim3(kTB), 0, c->stream, s->z, s->w, s->hb, np,
                               nullptr);
        }
        double est = 0.0;
        if ((e = hipMemcpyAsync(&est, s->hb, sizeof(double), hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
            return e;
        if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return e;
        s->lmin = 1.0;
        s->lmax = 1.1 * est;
    }
    return hipGetLastError();
}

void imex3d_set_pbno32(numa_ctx *c, int on) { c->imex->pbno32 = on ? 1 : 0; }

void imex3d_set_bounds(numa_ctx *c, double lmin, double lmax)
{
    c->imex->lmin = lmin;
    c->imex->lmax = lmax;
}

hipError_t schur_apply(numa_ctx *c, const double *P, double *out)
{
    return apply(c, axpy_args(P, out, 0.0, 1.0, 0.0, nullptr));
}

hipError_t schur_rhs(numa_ctx *c, const double *y, double *b)
{
    return dispatch3(c->N, [&](auto n) { return rhs_kernel_launch<decltype(n)::value>(c, y, b); });
}

hipError_t pbno_apply(numa_ctx *c, const double *r, double *z) { return precondition(c, r, z); }

// S x = b by restarted GMRES from x = 0 (flexible, with the Z basis, when
// the learned correction is on): the solution in s.x, its residual b - S x
// in s.r.  *iters: Arnoldi iterations; *converged: 0 if maxit was reached.
hipError_t schur_gmres(numa_ctx *c, const double *bvec, int *iters, int *converged, double tol)
{
    Imex3d &s = *c->imex;
    const long np = s.np;
    const int m = s.restart;
    // the learned correction (flexible GMRES) until a restart cycle with it
    // fails to reduce the residual norm tenfold; then the polynomial alone.
    // The FP32 polynomial is not exactly the same linear map at every
    // application, so it always runs in flexible GMRES.
    bool net = learned_enabled(c);
    const bool flex32 = s.pbno32 && s.order >= 1;
    bool flex = net || flex32;
    hipError_t e;
    *iters = 0;
    *converged = 0;
    double bnorm = 0.0;
    if ((e = norm_host(c, bvec, &bnorm)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(s.x, 0, sizeof(double) * np, c->stream)) != hipSuccess) return e;
    const double tolb = tol * bnorm;
    double beta = bnorm;
    const double *rvec = bvec;  // residual of x = 0
    int total = 0;
    const int chunk = 4;
    while (true) {
        if (beta <= tolb) {
            *converged = 1;
            break;
        }
        if (total >= s.maxit) break;
        hipLaunchKernelGGL(k_scale, dim3(unsigned(s.nblk)), dim3(kTB), 0, c->stream, s.V, rvec, 1.0 / beta, np);
        hipLaunchKernelGGL(k_cycle_init, dim3(1), dim3(1), 0, c->stream, s.g, m, beta, s.stop);
        const int jmax = std::min(m, s.maxit - total);
        int jdone = 0;
        for (int j0 = 0; j0 < jmax; j0 += chunk) {
            for (int j = j0; j < std::min(jmax, j0 + chunk); ++j) {
                const double *vj = s.V + size_t(j) * np;
                double *vn = s.V + size_t(j + 1) * np;
                const double *zin = vj;
                if (flex) {
                    double *zj = s.Z + size_t(j) * np;
                    if ((e = precondition(c, vj, zj)) != hipSuccess) return e;
                    if (net && (e = learned_correction_add(c, vj, zj, s.stop)) != hipSuccess) return e;
                    zin = zj;
                } else if (s.order >= 0) {
                    if ((e = precondition(c, vj, s.z)) != hipSuccess) return e;
                    zin = s.z;
                }
                // w = S z and the first Gram-Schmidt dots
                ApplyArgs a = axpy_args(zin, s.w, 0.0, 1.0, 0.0, nullptr);
                a.V = s.V;
                a.nv = j + 1;
                a.part = s.part;
                a.stop = s.stop;
                if ((e = apply(c, a)) != hipSuccess) return e;
                hipLaunchKernelGGL(k_finish, dim3(unsigned(j + 1)), dim3(kTB), 0, c->stream, s.part, s.nblk3, s.hb, 0,
                                   s.H, m, j, 0, s.stop);
                // first update with the second pass dots fused; second update with |w|^2
                if ((e = cgs_update(c, j + 1, j + 1)) != hipSuccess) return e;
                hipLaunchKernelGGL(k_finish, dim3(unsigned(j + 1)), dim3(kTB), 0, c->stream, s.part, s.nblk, s.hb, 0,
                                   s.H, m, j, 1, s.stop);
                if ((e = cgs_update(c, j + 1, -1)) != hipSuccess) return e;
                hipLaunchKernelGGL(k_finish, dim3(1), dim3(kTB), 0, c->stream, s.part, s.nblk, s.hb, 1,
                                   s.H + size_t(j + 1) * m, m, j, 0, s.stop);
                hipLaunchKernelGGL(k_normalize, dim3(unsigned(s.nblk)), dim3(kTB), 0, c->stream, vn, s.w,
                                   s.H + size_t(j + 1) * m + j, np, s.stop);
                hipLaunchKernelGGL(k_givens, dim3(1), dim3(64), 0, c->stream, s.H, s.cs, s.sn, s.g, j, m, tolb, s.stop);
                if ((e = hipGetLastError()) != hipSuccess) return e;
            }
            int flags[2] = {0, 0};
            if ((e = hipMemcpyAsync(flags, s.stop, sizeof(flags), hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
                return e;
            if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return e;
            jdone = flags[1];
            if (flags[0]) break;
        }
        // x += M V y
        if ((e = hipMemcpyAsync(s.hH.data(), s.H, sizeof(double) * s.hH.size(), hipMemcpyDeviceToHost, c->stream)) !=
            hipSuccess)
            return e;
        if ((e = hipMemcpyAsync(s.hg.data(), s.g, sizeof(double) * s.hg.size(), hipMemcpyDeviceToHost, c->stream)) !=
            hipSuccess)
            return e;
        if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return e;
        upper_solve(s.hH, s.hg, m, jdone, s.hy);
        if ((e = hipMemcpyAsync(s.yc, s.hy.data(), sizeof(double) * jdone, hipMemcpyHostToDevice, c->stream)) !=
            hipSuccess)
            return e;
        if (flex) {
            hipLaunchKernelGGL(k_combine, dim3(unsigned(s.nblk)), dim3(kTB), 0, c->stream, s.x, s.Z, s.yc, jdone, np, 1);
        } else if (s.order < 0) {
            hipLaunchKernelGGL(k_combine, dim3(unsigned(s.nblk)), dim3(kTB), 0, c->stream, s.x, s.V, s.yc, jdone, np, 1);
        } else {
            hipLaunchKernelGGL(k_combine, dim3(unsigned(s.nblk)), dim3(kTB), 0, c->stream, s.w, s.V, s.yc, jdone, np, 0);
            if ((e = precondition(c, s.w, s.z)) != hipSuccess) return e;
            if ((e = lincomb(c, s.x, s.x, 1.0, s.z, 1.0, nullptr, 0.0, np)) != hipSuccess) return e;
        }
        total += jdone;
        // true residual
        if ((e = apply(c, axpy_args(s.x, s.r, 0.0, -1.0, 1.0, bvec))) != hipSuccess) return e;
        const double before = beta;
        if ((e = norm_host(c, s.r, &beta)) != hipSuccess) return e;
        if (net && beta > 0.1 * before) {
            net = false;
            flex = flex32;
        }
        rvec = s.r;
    }
    *iters = total;
    if (rvec == bvec)  // x = 0: r = b
        return hipMemcpyAsync(s.r, bvec, sizeof(double) * np, hipMemcpyDeviceToDevice, c->stream);
    return hipSuccess;
}

// S e = r for a field r (device), solution copied to e_out
hipError_t schur_solve_field(numa_ctx *c, const double *r, double *e_out, double tol, int *iters, int *converged)
{
    hipError_t e = schur_gmres(c, r, iters, converged, tol);
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(e_out, c->imex->x, sizeof(double) * c->np, hipMemcpyDeviceToDevice, c->stream);
}

// x = (I - lambda L)^-1 y (5 fields), out = x + d0 in0 + d1 in1.  out may be
// y itself.  *iters: Arnoldi iterations; *converged: 0 if maxit was reached.
hipError_t imex3d_solve(numa_ctx *c, const double *y, double *out, const double *in0, double d0, const double *in1,
                        double d1, double tol, int *iters, int *converged)
{
    Imex3d &s = *c->imex;
    hipError_t e;
    if ((e = schur_rhs(c, y, s.b)) != hipSuccess) return e;
    if ((e = schur_gmres(c, s.b, iters, converged, tol)) != hipSuccess) return e;
    ExtractArgs a{};
    a.y = y;
    a.P = s.x;
    a.r = s.r;
    a.out = out;
    a.in0 = in0;
    a.d0 = d0;
    a.in1 = in1;
    a.d1 = d1;
    a.lam = s.lambda;
    a.g = c->eos.grav;
    return dispatch3(c->N, [&](auto n) { return extract_launch<decltype(n)::value>(c, a); });
}

// One 3D-IMEX ARK2 step in the shifted-stage form of the HEVI step with L in
// place of L_V: Q2 = q + solve(dt a21 R1); Q3 = solve(E3 + c31 q + c32 Q2)
// - c31 q - c32 Q2; q' = ACC + dt b3 R(Q3).
hipError_t imex3d_step(numa_ctx *c, double *q, double dt, double tol, int *iters, int *converged)
{
    Imex3d &s = *c->imex;
    const long n5 = 5 * s.np;
    const double s2 = std::sqrt(2.0), al = (3.0 + 2.0 * s2) / 6.0, ad = 1.0 - 1.0 / s2;
    const double a21 = 2.0 - s2, a31 = 1.0 - al, a32 = al, b1 = 1.0 / (2.0 * s2), b2 = b1, b3 = ad;
    const double c31 = (1.0 / (2.0 * s2) - a31) / ad, c32 = (1.0 / (2.0 * s2) - a32) / ad;
    hipError_t e;
    int it2 = 0, it3 = 0, cv2 = 0, cv3 = 0;
    *iters = 0;
    *converged = 0;
    if ((e = launch_rhs_plain(c, q, s.R1)) != hipSuccess) return e;
    if ((e = lincomb(c, s.Q2, s.R1, dt * a21, nullptr, 0.0, nullptr, 0.0, n5)) != hipSuccess) return e;
    if ((e = imex3d_solve(c, s.Q2, s.Q2, q, 1.0, nullptr, 0.0, tol, &it2, &cv2)) != hipSuccess) return e;
    if ((e = launch_rhs_two(c, s.Q2, q, s.R1, s.E3, s.ACC, dt * a31, dt * a32, dt * b1, dt * b2)) != hipSuccess)
        return e;
    if ((e = lincomb(c, s.E3, s.E3, 1.0, q, c31, s.Q2, c32, n5)) != hipSuccess) return e;
    if ((e = imex3d_solve(c, s.E3, s.E3, q, -c31, s.Q2, -c32, tol, &it3, &cv3)) != hipSuccess) return e;
    if ((e = launch_rhs_final(c, s.E3, s.ACC, q, dt * b3)) != hipSuccess) return e;
    *iters = it2 + it3;
    *converged = cv2 && cv3;
    return hipSuccess;
}

void imex3d_info(const numa_ctx *c, double *dt, double *lmin, double *lmax)
{
    *dt = c->imex->dt;
    *lmin = c->imex->lmin;
    *lmax = c->imex->lmax;
}

}  // namespace numa
