// Learned correction of the 3D-IMEX preconditioner (a project addition on
// top of the polynomial preconditioners of Sec. 5.5).
//
// A two-layer perceptron acts on each element's residual: x = r_e / s_e,
// s_e the RMS of r over the element's (N+1)^3 nodes (local order
// a + nq (b + nq c), a along x), h = tanh(W1 x + b1), y = W2 h + b2; the
// correction s_e y is averaged over the elements sharing a node and added
// to the PBNO polynomial, z = s(S) r + corr(r).  corr is nonlinear, so the
// solver switches to flexible GMRES while it is enabled.
//
// Training (FP32, on the device): samples are element patches of
// (r, S^-1 r - s(S) r) pairs, the solutions coming from the solver itself
// (PBNO GMRES to a tight tolerance); loss = mean squared error of y against
// (S^-1 r - s(S) r)_e / s_e; Adam.  The gradient is computed by
//   k_mlp_forward     h, y per sample (one block per sample)
//   k_mlp_out_grad    dy = 2 (y - t) / (B nin), loss partials
//   k_mlp_hidden_grad dh = (1 - h^2) W2^T dy
//   k_mlp_param_grad  one thread per parameter, a fixed-order sum over the
//                     batch (no atomics, so gradients are reproducible)
//   k_adam            the update.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <random>
#include <vector>

#include "numa_internal.h"

namespace numa {

struct Learned {
    int nin = 0, nh = 0, enabled = 0;
    long nparam = 0, cap = 0, nsamp = 0, nelem = 0;
    long adam_t = 0;
    void *block = nullptr;
    float *theta = nullptr, *grad = nullptr, *am = nullptr, *av = nullptr;  // nparam each
    float *X = nullptr, *T = nullptr;                                       // cap * nin training samples
    float *Xe = nullptr, *Ye = nullptr, *He = nullptr;                      // per element (inference, batches)
    float *dY = nullptr, *dH = nullptr;                                     // batch gradients
    double *se = nullptr;                                                   // element scales
    double *e = nullptr, *pb = nullptr;                                     // solution and PBNO of a sample field
    double *lossp = nullptr;                                                // loss partials
};

namespace {

constexpr int kLB = 256;

// parameter layout in theta: W1[nh][nin], b1[nh], W2[nin][nh], b2[nin]
struct Params {
    const float *W1, *b1, *W2, *b2;
};

__host__ __device__ inline Params params_of(const float *th, int nin, int nh)
{
    Params p;
    p.W1 = th;
    p.b1 = th + long(nh) * nin;
    p.W2 = p.b1 + nh;
    p.b2 = p.W2 + long(nin) * nh;
    return p;
}

__device__ inline double block_reduce(double v, double *sh)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    const double t = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return t;
}

// unique node of local node (a, b, cc) of element e
__device__ inline long elem_node(int e, int a, int b, int cc, int N, int nex, int ney, int nx, int ny)
{
    const int ex = e % nex, ey = (e / nex) % ney, ez = e / (nex * ney);
    const int i = (ex * N + a) % nx, j = (ey * N + b) % ny, k = ez * N + cc;
    return (long(k) * ny + j) * nx + i;
}

// features of field r: X[e][l] = r_e / s_e (FP32), se[e] = s_e.  One block per element.
__global__ __launch_bounds__(kLB) void k_features(const double *r, float *X, double *se, int N, int nex, int ney,
                                                  int nx, int ny)
{
    __shared__ double sh[4];
    const int e = blockIdx.x, nq = N + 1, nin = nq * nq * nq;
    double ss = 0.0;
    for (int l = threadIdx.x; l < nin; l += kLB) {
        const int a = l % nq, b = (l / nq) % nq, cc = l / (nq * nq);
        const double v = r[elem_node(e, a, b, cc, N, nex, ney, nx, ny)];
        ss += v * v;
    }
    const double s = std::sqrt(block_reduce(ss, sh) / nin);
    if (threadIdx.x == 0) se[e] = s;
    for (int l = threadIdx.x; l < nin; l += kLB) {
        const int a = l % nq, b = (l / nq) % nq, cc = l / (nq * nq);
        const double v = r[elem_node(e, a, b, cc, N, nex, ney, nx, ny)];
        X[long(e) * nin + l] = s > 0.0 ? float(v / s) : 0.0f;
    }
}

// targets of a sample field: T[e][l] = (e_field - pb)_e / s_e.  Elements
// whose s_e is below `floor` (where the field is nearly zero, the
// normalised target would be huge) become empty samples (X = T = 0).
__global__ __launch_bounds__(kLB) void k_targets(const double *ef, const double *pb, const double *se, float *X,
                                                 float *T, double floor, int N, int nex, int ney, int nx, int ny)
{
    const int e = blockIdx.x, nq = N + 1, nin = nq * nq * nq;
    const double s = se[e];
    const bool keep = s > floor && s > 0.0;
    for (int l = threadIdx.x; l < nin; l += kLB) {
        const int a = l % nq, b = (l / nq) % nq, cc = l / (nq * nq);
        const long I = elem_node(e, a, b, cc, N, nex, ney, nx, ny);
        T[long(e) * nin + l] = keep ? float((ef[I] - pb[I]) / s) : 0.0f;
        if (!keep) X[long(e) * nin + l] = 0.0f;
    }
}

// h, y of samples X[n][nin]; one block per sample
__global__ __launch_bounds__(kLB) void k_mlp_forward(const float *X, const float *theta, int nin, int nh, float *H,
                                                     float *Y)
{
    extern __shared__ float lds[];
    float *x = lds, *h = lds + nin;
    const Params p = params_of(theta, nin, nh);
    const long s = blockIdx.x;
    for (int i = threadIdx.x; i < nin; i += kLB) x[i] = X[s * nin + i];
    __syncthreads();
    for (int k = threadIdx.x; k < nh; k += kLB) {
        float t = p.b1[k];
        const float *w = p.W1 + long(k) * nin;
        for (int i = 0; i < nin; ++i) t = fmaf(w[i], x[i], t);
        const float hv = tanhf(t);
        h[k] = hv;
        H[s * nh + k] = hv;
    }
    __syncthreads();
    for (int o = threadIdx.x; o < nin; o += kLB) {
        float t = p.b2[o];
        const float *w = p.W2 + long(o) * nh;
        for (int k = 0; k < nh; ++k) t = fmaf(w[k], h[k], t);
        Y[s * nin + o] = t;
    }
}

// dY = 2 (Y - T) / (n nin); lossp[block] = partial sum of (Y - T)^2 / (n nin)
__global__ __launch_bounds__(kLB) void k_mlp_out_grad(const float *Y, const float *T, long total, float *dY,
                                                      double *lossp)
{
    __shared__ double sh[4];
    const long I = long(blockIdx.x) * kLB + threadIdx.x;
    const double sc = 1.0 / double(total);
    double l = 0.0;
    if (I < total) {
        const double d = double(Y[I]) - double(T[I]);
        dY[I] = float(2.0 * d * sc);
        l = d * d * sc;
    }
    l = block_reduce(l, sh);
    if (threadIdx.x == 0) lossp[blockIdx.x] = l;
}

// dH[s][k] = (1 - h^2) sum_o W2[o][k] dY[s][o]; one block per sample
__global__ __launch_bounds__(kLB) void k_mlp_hidden_grad(const float *dY, const float *H, const float *theta, int nin,
                                                         int nh, float *dH)
{
    const Params p = params_of(theta, nin, nh);
    const long s = blockIdx.x;
    for (int k = threadIdx.x; k < nh; k += kLB) {
        float t = 0.0f;
        for (int o = 0; o < nin; ++o) t = fmaf(p.W2[long(o) * nh + k], dY[s * nin + o], t);
        const float h = H[s * nh + k];
        dH[s * nh + k] = (1.0f - h * h) * t;
    }
}

// gradient of every parameter, a fixed-order sum over the n samples
__global__ __launch_bounds__(kLB) void k_mlp_param_grad(const float *X, const float *H, const float *dY,
                                                        const float *dH, long n, int nin, int nh, float *g)
{
    const long q = long(blockIdx.x) * kLB + threadIdx.x;
    const long nW1 = long(nh) * nin, nP = nW1 + nh + long(nin) * nh + nin;
    if (q >= nP) return;
    float acc = 0.0f;
    if (q < nW1) {  // W1[k][i]
        const int k = int(q / nin), i = int(q % nin);
        for (long s = 0; s < n; ++s) acc = fmaf(dH[s * nh + k], X[s * nin + i], acc);
    } else if (q < nW1 + nh) {  // b1[k]
        const int k = int(q - nW1);
        for (long s = 0; s < n; ++s) acc += dH[s * nh + k];
    } else if (q < nW1 + nh + long(nin) * nh) {  // W2[o][k]
        const long r = q - nW1 - nh;
        const int o = int(r / nh), k = int(r % nh);
        for (long s = 0; s < n; ++s) acc = fmaf(dY[s * nin + o], H[s * nh + k], acc);
    } else {  // b2[o]
        const int o = int(q - nW1 - nh - long(nin) * nh);
        for (long s = 0; s < n; ++s) acc += dY[s * nin + o];
    }
    g[q] = acc;
}

__global__ __launch_bounds__(kLB) void k_adam(float *theta, const float *g, float *m, float *v, long n, float lr,
                                              float b1, float b2, float eps, float c1, float c2)
{
    const long q = long(blockIdx.x) * kLB + threadIdx.x;
    if (q >= n) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.0f - b1) * gq;
    const float vq = b2 * v[q] + (1.0f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    theta[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

// z[I] += average over the elements holding node I of se[e] Y[e][l(I, e)]
__global__ __launch_bounds__(kLB) void k_corr_add(const float *Y, const double *se, double *z, int N, int nex,
                                                  int ney, int nez, int nx, int ny, int nz, const int *stop)
{
    if (stop && *stop) return;
    const long I = long(blockIdx.x) * kLB + threadIdx.x;
    const long np = long(nx) * ny * nz;
    if (I >= np) return;
    const int i = int(I % nx), j = int((I / nx) % ny), k = int(I / (long(nx) * ny));
    const int nq = N + 1, nin = nq * nq * nq;
    // the one or two elements along each axis (local index N in the left one)
    int ex[2], ax[2], ey[2], ay[2], ez[2], az[2], cx = 0, cy = 0, cz = 0;
    ex[cx] = i / N; ax[cx++] = i % N;
    if (i % N == 0) { ex[cx] = (i / N + nex - 1) % nex; ax[cx++] = N; }
    ey[cy] = j / N; ay[cy++] = j % N;
    if (j % N == 0) { ey[cy] = (j / N + ney - 1) % ney; ay[cy++] = N; }
    if (k == nz - 1) { ez[cz] = nez - 1; az[cz++] = N; }
    else {
        ez[cz] = k / N; az[cz++] = k % N;
        if (k % N == 0 && k > 0) { ez[cz] = k / N - 1; az[cz++] = N; }
    }
    double s = 0.0;
    for (int p = 0; p < cz; ++p)
        for (int q = 0; q < cy; ++q)
            for (int r = 0; r < cx; ++r) {
                const long e = ex[r] + long(nex) * (ey[q] + long(ney) * ez[p]);
                const int l = ax[r] + nq * (ay[q] + nq * az[p]);
                s += se[e] * double(Y[e * nin + l]);
            }
    z[I] += s / double(cx * cy * cz);
}

inline unsigned blocks(long n) { return unsigned((n + kLB - 1) / kLB); }

}  // namespace

bool learned_enabled(const numa_ctx *c) { return c->learned && c->learned->enabled; }

LearnedInfo learned_info(const numa_ctx *c)
{
    const Learned &L = *c->learned;
    return LearnedInfo{L.nparam, L.nsamp, L.cap, L.nelem, L.nin, L.nh, L.enabled, L.theta, L.grad, L.X, L.T};
}

void learned_set_enabled(numa_ctx *c, int on) { c->learned->enabled = on ? 1 : 0; }

void learned_free(numa_ctx *c)
{
    if (!c || !c->learned) return;
    if (c->learned->block) (void)hipFree(c->learned->block);
    delete c->learned;
    c->learned = nullptr;
}

hipError_t learned_setup(numa_ctx *c, int nh, long cap, uint64_t seed)
{
    learned_free(c);
    Learned *L = new Learned();
    c->learned = L;
    const int nq = c->N + 1;
    L->nin = nq * nq * nq;
    L->nh = nh;
    L->nparam = long(nh) * L->nin + nh + long(L->nin) * nh + L->nin;
    L->nelem = long(c->nex) * c->ney * c->nez;
    L->cap = cap;
    const long nb = std::max(cap, L->nelem);  // batch / inference rows
    const size_t nf = size_t(4 * L->nparam) + size_t(2 * cap * L->nin) + size_t(nb) * (2 * L->nin + 2 * nh);
    const size_t nd = size_t(L->nelem) + size_t(2 * c->np) + size_t(blocks(nb * L->nin));
    hipError_t e = hipMalloc(&L->block, nf * sizeof(float) + nd * sizeof(double) + 256);
    if (e != hipSuccess) {
        L->block = nullptr;
        return e;
    }
    double *d = static_cast<double *>(L->block);
    L->se = d; d += L->nelem;
    L->e = d; d += c->np;
    L->pb = d; d += c->np;
    L->lossp = d; d += blocks(nb * L->nin);
    float *f = reinterpret_cast<float *>(d);
    L->theta = f; f += L->nparam;
    L->grad = f; f += L->nparam;
    L->am = f; f += L->nparam;
    L->av = f; f += L->nparam;
    L->X = f; f += cap * L->nin;
    L->T = f; f += cap * L->nin;
    L->Xe = nullptr;  // inference reuses the batch rows below
    L->Ye = f; f += nb * L->nin;
    L->dY = f; f += nb * L->nin;
    L->He = f; f += nb * nh;
    L->dH = f; f += nb * nh;
    L->Xe = L->dY;  // features of an inference pass live in the gradient rows (not used at the same time)
    // initial weights: uniform in +-sqrt(6/(fan_in + fan_out)), biases 0
    std::vector<float> th(size_t(L->nparam), 0.0f);
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    const double a1 = std::sqrt(6.0 / (L->nin + nh)), a2 = std::sqrt(6.0 / (nh + L->nin));
    const long nW1 = long(nh) * L->nin;
    for (long q = 0; q < nW1; ++q) th[q] = float(a1 * u(rng));
    for (long q = 0; q < long(L->nin) * nh; ++q) th[nW1 + nh + q] = float(a2 * u(rng));
    if ((e = hipMemcpy(L->theta, th.data(), sizeof(float) * L->nparam, hipMemcpyHostToDevice)) != hipSuccess)
        return e;
    if ((e = hipMemset(L->am, 0, sizeof(float) * 2 * L->nparam)) != hipSuccess) return e;
    return hipSuccess;
}

// z += corr(r) (the network must be set up)
hipError_t learned_correction_add(numa_ctx *c, const double *r, double *z, const int *stop)
{
    Learned &L = *c->learned;
    hipLaunchKernelGGL(k_features, dim3(unsigned(L.nelem)), dim3(kLB), 0, c->stream, r, L.Xe, L.se, c->N, c->nex,
                       c->ney, int(c->nx), int(c->ny));
    hipLaunchKernelGGL(k_mlp_forward, dim3(unsigned(L.nelem)), dim3(kLB), sizeof(float) * (L.nin + L.nh), c->stream,
                       L.Xe, L.theta, L.nin, L.nh, L.He, L.Ye);
    hipLaunchKernelGGL(k_corr_add, dim3(blocks(c->np)), dim3(kLB), 0, c->stream, L.Ye, L.se, z, c->N, c->nex, c->ney,
                       c->nez, int(c->nx), int(c->ny), int(c->nz), stop);
    return hipGetLastError();
}

// one sample field r: solve S e = r (polynomial preconditioner, the network
// off), append its element patches (r_e / s_e, (e - s(S) r)_e / s_e); the
// patches of elements with s_e below 1e-3 of the field's RMS stay empty
hipError_t learned_add_samples(numa_ctx *c, const double *r, double tol, int *iters, int *converged)
{
    Learned &L = *c->learned;
    if (L.nsamp + L.nelem > L.cap) return hipErrorInvalidValue;
    const int keep = L.enabled;
    L.enabled = 0;
    hipError_t e = schur_solve_field(c, r, L.e, tol, iters, converged);
    L.enabled = keep;
    if (e != hipSuccess) return e;
    if ((e = pbno_apply(c, r, L.pb)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_features, dim3(unsigned(L.nelem)), dim3(kLB), 0, c->stream, r, L.X + L.nsamp * L.nin, L.se,
                       c->N, c->nex, c->ney, int(c->nx), int(c->ny));
    // the field's RMS scale from the element scales (host, nelem values)
    std::vector<double> se(size_t(L.nelem));
    if ((e = hipMemcpyAsync(se.data(), L.se, sizeof(double) * se.size(), hipMemcpyDeviceToHost, c->stream)) !=
        hipSuccess)
        return e;
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return e;
    double ms = 0.0;
    for (double v : se) ms += v * v;
    const double floor = 1e-3 * std::sqrt(ms / double(se.size()));
    hipLaunchKernelGGL(k_targets, dim3(unsigned(L.nelem)), dim3(kLB), 0, c->stream, L.e, L.pb, L.se,
                       L.X + L.nsamp * L.nin, L.T + L.nsamp * L.nin, floor, c->N, c->nex, c->ney, int(c->nx),
                       int(c->ny));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    L.nsamp += L.nelem;
    return hipSuccess;
}

// loss and gradient (into L.grad) of n samples X, T (device, FP32)
hipError_t learned_loss_grad(numa_ctx *c, const float *X, const float *T, long n, double *loss)
{
    Learned &L = *c->learned;
    const long tot = n * L.nin;
    hipLaunchKernelGGL(k_mlp_forward, dim3(unsigned(n)), dim3(kLB), sizeof(float) * (L.nin + L.nh), c->stream, X,
                       L.theta, L.nin, L.nh, L.He, L.Ye);
    hipLaunchKernelGGL(k_mlp_out_grad, dim3(blocks(tot)), dim3(kLB), 0, c->stream, L.Ye, T, tot, L.dY, L.lossp);
    hipLaunchKernelGGL(k_mlp_hidden_grad, dim3(unsigned(n)), dim3(kLB), 0, c->stream, L.dY, L.He, L.theta, L.nin, L.nh,
                       L.dH);
    hipLaunchKernelGGL(k_mlp_param_grad, dim3(blocks(L.nparam)), dim3(kLB), 0, c->stream, X, L.He, L.dY, L.dH, n,
                       L.nin, L.nh, L.grad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !loss) return e;
    std::vector<double> lp(blocks(tot));
    if ((e = hipMemcpyAsync(lp.data(), L.lossp, sizeof(double) * lp.size(), hipMemcpyDeviceToHost, c->stream)) !=
        hipSuccess)
        return e;
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return e;
    double s = 0.0;
    for (double v : lp) s += v;
    *loss = s;
    return hipSuccess;
}

// Adam over minibatches of the stored samples: batches are consecutive
// windows of a fixed pseudo-random order of the samples (seeded)
hipError_t learned_train(numa_ctx *c, int steps, int batch, double lr, uint64_t seed, double *loss_first,
                         double *loss_last)
{
    Learned &L = *c->learned;
    if (L.nsamp < 1 || batch < 1) return hipErrorInvalidValue;
    batch = int(std::min<long>(batch, L.nsamp));
    // order of samples: a permutation applied by gathering windows into the
    // batch rows is avoided; instead batches start at seeded offsets
    std::mt19937_64 rng(seed);
    std::uniform_int_distribution<long> start(0, L.nsamp - batch);
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    hipError_t e = hipSuccess;
    for (int t = 0; t < steps; ++t) {
        const long s0 = start(rng);
        double *lp = (t == 0 || t == steps - 1) ? (t == 0 ? loss_first : loss_last) : nullptr;
        if ((e = learned_loss_grad(c, L.X + s0 * L.nin, L.T + s0 * L.nin, batch, lp)) != hipSuccess) return e;
        ++L.adam_t;
        const float c1 = float(1.0 - std::pow(double(b1), double(L.adam_t)));
        const float c2 = float(1.0 - std::pow(double(b2), double(L.adam_t)));
        hipLaunchKernelGGL(k_adam, dim3(blocks(L.nparam)), dim3(kLB), 0, c->stream, L.theta, L.grad, L.am, L.av,
                           L.nparam, float(lr), b1, b2, eps, c1, c2);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipStreamSynchronize(c->stream);
}

}  // namespace numa
