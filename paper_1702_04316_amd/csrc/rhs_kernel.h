// The right-hand-side kernel of the HEVI step and its launcher, templated on
// the order N and the tile variant V; shared by kernels.hip (variant 0, and
// everything else of the step) and rhs_alt.hip (variant 1), which compile in
// parallel.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "numa_internal.h"

namespace numa {

// ---------------------------------------------------------------------------
// Right-hand-side kernel.  A workgroup owns a TX x TY tile of columns
// (element aligned) and marches upwards through a chunk of vertical
// elements.  For element ez its TX*TY*N threads compute the N owned levels
// ez*N + c (c = 0..N-1, c slowest in the thread index, so a wavefront shares
// c).  The N+1 levels of the element sit in an LDS ring of planes (level k in
// slot k mod (N+1)); each plane holds the tile plus the halo the DSS line
// operators need (N nodes below, 1 node above, in x and in y).
// ---------------------------------------------------------------------------
// Tile<N, V>: the tile of variant V (0, the default, or 1) for order N; the
// autotuner times both on a context and keeps the faster.  Tiles are element
// aligned (multiples of N) and a workgroup's ring must fit one CU's LDS.
template <int N, int V>
struct Tile;
template <> struct Tile<1, 0> { static constexpr int TX = 32, TY = 16; };
template <> struct Tile<2, 0> { static constexpr int TX = 32, TY = 8; };
template <> struct Tile<3, 0> { static constexpr int TX = 24, TY = 6; };
template <> struct Tile<4, 0> { static constexpr int TX = 16, TY = 8; };
template <> struct Tile<5, 0> { static constexpr int TX = 15, TY = 5; };
template <> struct Tile<6, 0> { static constexpr int TX = 12, TY = 6; };
template <> struct Tile<7, 0> { static constexpr int TX = 14, TY = 7; };
template <> struct Tile<8, 0> { static constexpr int TX = 8, TY = 8; };
template <> struct Tile<1, 1> { static constexpr int TX = 16, TY = 16; };
template <> struct Tile<2, 1> { static constexpr int TX = 16, TY = 8; };
template <> struct Tile<3, 1> { static constexpr int TX = 12, TY = 6; };
template <> struct Tile<4, 1> { static constexpr int TX = 16, TY = 4; };
template <> struct Tile<5, 1> { static constexpr int TX = 20, TY = 5; };
// N = 6 has one shape: the 18 x 6 tile (648 threads) returned wrong values
// in its stage-2 kernel, in the precision form with this ring layout and in
// the FP64 step with a per-node interleaved one, while 12 x 6 and every
// other order's shapes agree; the cause was not found
template <> struct Tile<6, 1> { static constexpr int TX = 12, TY = 6; };
template <> struct Tile<7, 1> { static constexpr int TX = 7, TY = 14; };
template <> struct Tile<8, 1> { static constexpr int TX = 8, TY = 8; };  // no other shape fits: same as 0

template <int N, int V = 0>  // V: tile variant
struct RhsGeom {
    static constexpr int TX = Tile<N, V>::TX, TY = Tile<N, V>::TY;
    static constexpr int NT = TX * TY * N;          // threads
    static constexpr int LX = TX + N + 1;           // plane incl. halo
    static constexpr int LY = TY + N + 1;
    static constexpr int FS = LX * LY;              // one field of one plane
    // a plane: rho', u, v, w, theta', P' (FP64 each)
    static constexpr int POFF = 5 * FS * 8;         // byte offset of P'
    static constexpr int PB = POFF + 8 * FS;        // bytes of a plane
    static constexpr int NS = 2 * N + 1;            // x/y stencil width
    // cross-shaped part of a plane that is loaded: tile rows with the x halo,
    // plus the y-halo rows of the tile columns
    static constexpr int NCROSS = TY * LX + TX * (N + 1);
    static constexpr int NITEM = (N * NCROSS + NT - 1) / NT;  // plane loads per thread
    static constexpr size_t LDS = size_t(N + 1) * PB;
    // waves per SIMD to compile for: two workgroups per CU where LDS allows
    static constexpr int MINW = (NT <= 512 && 2 * LDS <= 150 * 1024) ? 2 * (NT / 256) : 1;
};

// device equation of state: P = p00 (rho R theta / p00)^gamma (Eq. (10))
__device__ __forceinline__ double eos_pressure(double rho, double theta, const EOS &e)
{
    return e.p00 * pow(rho * e.rgas * theta / e.p00, e.gamma);
}

// P' = EOS(rho0 + rho', theta0 + theta') - P0 evaluated as
// P0 [((rho theta)/(rho0 theta0))^gamma - 1]: with rho theta - rho0 theta0 =
// rho0 theta' + theta0 rho' + rho' theta' no two ~1e5 Pa numbers are
// subtracted, so P' keeps its own relative precision.
// rho0 theta', theta0 rho' and rho' theta' nearly cancel in a balanced state:
// each product is split into rounded value + exact error (fma), so their
// small sum keeps its relative precision (no contraction may touch this).
// With x = (rho theta - rho0 theta0)/(rho0 theta0), P' = P0 ((1 + x)^gamma - 1):
// a 10-term binomial series for |x| <= 1/32 (every state of a weather
// perturbation; the first omitted term is below 1e-18 relative), log1p/expm1
// beyond.
// (1 + x)^gamma - 1 for |x| beyond the series range.  Out of line: inlined,
// the compiler keeps the constants of log1p and expm1 in vector registers
// across the stencil loops, for a path that weather states do not take.
__device__ __noinline__ double binom_power_m1(double x, double gamma) { return expm1(gamma * log1p(x)); }

// r0, t0, P0: rho0, theta0, P0 of the level; irt = 1/(rho0 theta0).
__device__ __forceinline__ double pressure_perturbation(double rp, double th, double r0, double P0, double irt,
                                                        double t0, const EOS &e)
{
#pragma clang fp contract(off)
    const double p1 = r0 * th, p2 = t0 * rp, p3 = rp * th;
    const double e1 = __builtin_fma(r0, th, -p1), e2 = __builtin_fma(t0, rp, -p2), e3 = __builtin_fma(rp, th, -p3);
    const double d = ((p1 + p2) + p3) + ((e1 + e2) + e3);
    const double x = d * irt;
    if (fabs(x) > kBinomMaxX) return P0 * binom_power_m1(x, e.gamma);
    // (1 + x)^gamma - 1 by its binomial series, Horner form
    double s = e.binom[kBinomTerms - 1];
#pragma unroll
    for (int k = kBinomTerms - 2; k >= 0; --k) s = __builtin_fma(s, x, e.binom[k]);
    return P0 * (s * x);
}

// Global access as (uniform 64-bit base) + (32-bit per-lane byte offset):
// compiles to global_load/store with a scalar base address, so a field needs
// two scalar registers whatever the number of lanes and levels.  NT: the
// FP64 store is non-temporal, chosen for large fields (nontemporal_stores).
// It is a template argument: a runtime choice between two otherwise equal
// stores is merged by the compiler, which drops the hint.
__device__ __forceinline__ double gload(const double *base, unsigned off)
{
    return *reinterpret_cast<const double *>(reinterpret_cast<const char *>(base) + off);
}
template <bool NT = false>
__device__ __forceinline__ void gstore(double *base, unsigned off, double v)
{
    double *a = reinterpret_cast<double *>(reinterpret_cast<char *>(base) + off);
    if constexpr (NT) __builtin_nontemporal_store(v, a);
    else *a = v;
}

// The same for a field of element type T, with off the offset an FP64 field
// would have (an FP32 field is addressed at off / 2).
template <class T>
__device__ __forceinline__ double tload(const void *base, unsigned off)
{
    if constexpr (sizeof(T) == 8) return gload(static_cast<const double *>(base), off);
    else return double(*reinterpret_cast<const float *>(static_cast<const char *>(base) + (off >> 1)));
}
template <class T, bool NT = false>
__device__ __forceinline__ void tstore(void *base, unsigned off, double v)
{
    if constexpr (sizeof(T) == 8) gstore<NT>(static_cast<double *>(base), off, v);
    else *reinterpret_cast<float *>(static_cast<char *>(base) + (off >> 1)) = float(v);  // (non-temporal was slower)
}
// field f of a five-field buffer of element type T, field stride fs elements
template <class T>
__device__ __forceinline__ const void *field(const void *base, int f, long fs)
{
    return static_cast<const T *>(base) + f * fs;
}
template <class T>
__device__ __forceinline__ void *field(void *base, int f, long fs)
{
    return static_cast<T *>(base) + f * fs;
}

struct RhsParams {
    // input fields (rho', u, v, w, theta'); with HASB, u, v, theta' of the
    // input are e0 + cb * e1 (a[1], a[2], a[4] unused), except theta' when
    // theta_in is set (a[4]: the stage value the column solve wrote over a
    // stratified background)
    const void *a[5];
    double cb;
    int theta_in;
    // five-field buffers (field f at + f * fs): out0 = e0 + k01 e1 + k02 R,
    // out1 = e0 + k11 e1 + k12 R
    void *out0, *out1;
    const void *e0, *e1;
    long fs;
    double k01, k02, k11, k12;
    const double *rho0, *P0, *zsc, *wxy, *D;
    const double *th0, *th0z;  // theta0 and d theta0/dz per level
    EOS eos;
    int nx, ny, nz, nez, zchunk, nchunk, ntx, nty;
    int *flag;
};

enum { EPI_R = 0, EPI_TWO = 1, EPI_FINAL = 2 };

// Layout of a five-field stage buffer of np nodes: all FP64, or (M) the
// precision form's first-stage tendency R1 with all five fields in FP32.
// R1 is a tendency: the step uses it only multiplied by dt (Sec. 2.2), so
// its FP32 rounding is relative to the change over a step, not to the
// state.  Byte offsets of the fields per node: 8 f (FP64) or 4 f (M).
// Offsets passed in are those an FP64 field would have.
template <bool M>
struct FiveField {
    static __device__ __forceinline__ bool f32(int) { return M; }
    static __device__ __forceinline__ size_t ofs(int f, long np) { return size_t(np) * (M ? 4 : 8) * size_t(f); }
    // field f stored alone at p
    static __device__ __forceinline__ double load1(const void *p, int f, unsigned off)
    {
        return f32(f) ? tload<float>(p, off) : tload<double>(p, off);
    }
    static __device__ __forceinline__ double load(const void *buf, int f, long np, unsigned off)
    {
        return load1(static_cast<const char *>(buf) + ofs(f, np), f, off);
    }
    template <bool NT>
    static __device__ __forceinline__ void store(void *buf, int f, long np, unsigned off, double v)
    {
        void *p = static_cast<char *>(buf) + ofs(f, np);
        if (f32(f)) tstore<float>(p, off, v);
        else tstore<double, NT>(p, off, v);
    }
};

// Buffers of one right-hand-side launch.  The FP64 step keeps every field
// in FP64.  The precision form (MIX) stores R1 in FP32 (written by the first
// launch, read by the second); its arithmetic, the LDS ring and every other
// buffer are the FP64 step's.  Stage values (Q2, Q3, E3, ACC) stay FP64: the
// next right-hand side differentiates them, which multiplies their rounding
// by the stencil's sum of |coefficients| (about N^2 / h).
template <int EPI, bool MIX>
struct RhsTypes {
    using A = FiveField<false>;                     // inputs a[]
    using E1 = FiveField<MIX>;                      // e1 (R1)
    using O0 = FiveField<MIX && EPI == EPI_R>;      // out0 (R1 in the first launch)
    using D = FiveField<false>;                     // e0, out1
};

// Map the launch index to a tile so that each of the 8 XCDs (which receive
// workgroups round-robin) works on a contiguous band of tiles and shares the
// halo rows in its own L2.
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    int q = nb >> 3, r = nb & 7;
    int x = b & 7, s = b >> 3;
    return x < r ? x * (q + 1) + s : r * (q + 1) + (x - r) * q + s;
}

// Stage input of field f at offset off.
template <bool HASB, class TA, class TE1>
__device__ __forceinline__ double stage_input(const RhsParams &p, int f, unsigned off)
{
    if constexpr (HASB) {
        if (f == 1 || f == 2 || (f == 4 && !p.theta_in))
            return FiveField<false>::load(p.e0, f, p.fs, off) + p.cb * TE1::load(p.e1, f, p.fs, off);
    }
    return TA::load1(p.a[f], f, off);
}

template <int N, int EPI, bool HASB, bool MIX, bool NT = false, int V = 0>
__global__ __launch_bounds__((RhsGeom<N, V>::NT), (RhsGeom<N, V>::MINW)) void k_rhs(RhsParams p)
{
    using TT = RhsTypes<EPI, MIX>;
    using TA = typename TT::A;
    using TE1 = typename TT::E1;
    using TO0 = typename TT::O0;
    using G = RhsGeom<N, V>;
    constexpr int NQ = N + 1, NS = G::NS, TX = G::TX, TY = G::TY, LX = G::LX, FS = G::FS;
    // dynamic LDS: ring of N+1 planes [rho', u, v, w, theta', P'] of
    // [LY][LX], then per-level tables rho0, P0, 1/(rho0 theta0), theta0,
    // d theta0/dz for the
    // levels this chunk touches, zsc [3][nez], and the interface shares
    // [2][6][TX*TY] (FP64)
    extern __shared__ double lds_block[];
    char *const ringb = reinterpret_cast<char *>(lds_block);
    auto cfield = [&](int slot) { return reinterpret_cast<double *>(ringb + slot * G::PB); };
    auto pfield = [&](int slot) { return reinterpret_cast<double *>(ringb + slot * G::PB + G::POFF); };
    // line stencils and the differentiation matrix
    __shared__ double sw[2][N][NS];
    __shared__ double sD[NQ * NQ];
    const double *const swd = &sw[0][0][0];

    const int tid = threadIdx.x;
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int ntile = p.ntx * p.nty;
    const int chunk = lb / ntile;
    const int tt = lb - chunk * ntile;
    const int tyb = tt / p.ntx, txb = tt - tyb * p.ntx;
    const int x0 = txb * TX, y0 = tyb * TY;
    const int nx = p.nx, ny = p.ny;
    const unsigned pbytes = unsigned(nx) * unsigned(ny) * 8u;
    const int ez0 = chunk * p.zchunk;
    const int ez1 = min(p.nez, ez0 + p.zchunk);
    const int kb = max(ez0 - 1, 0) * N;          // lowest level in the tables
    const int nlev = ez1 * N + 1 - kb;
    double *sR0 = lds_block + G::LDS / sizeof(double);
    double *sP0 = sR0 + nlev;
    double *sIRT = sP0 + nlev;
    double *sT0 = sIRT + nlev;
    double *sTZ = sT0 + nlev;
    double *zs = sTZ + nlev;  // [0,nez): 2/h ; [nez,2nez): bottom factor ; [2nez,3nez): top factor
    // the lower element's share of the six z-derivatives at the interface
    // node of each column, double-buffered by element parity: [2][6][TX*TY]
    double *zp = zs + 3 * p.nez;
    const EOS eos = p.eos;

    for (int s = tid; s < 2 * N * NS; s += G::NT) {
        (&sw[0][0][0])[s] = p.wxy[s];
    }
    for (int s = tid; s < NQ * NQ; s += G::NT) sD[s] = p.D[s];
    for (int s = tid; s < nlev; s += G::NT) {
        const double r0 = p.rho0[kb + s];
        const double t0 = p.th0[kb + s];
        sR0[s] = r0;
        sP0[s] = p.P0[kb + s];
        sIRT[s] = 1.0 / (r0 * t0);
        sT0[s] = t0;
        sTZ[s] = p.th0z[kb + s];
    }
    for (int s = tid; s < 3 * p.nez; s += G::NT) zs[s] = p.zsc[s];
    // plane loads of this thread: which of the N new planes (1..N, 0 = none),
    // LDS offset in the plane, byte offset in a level plane
    int it_p[G::NITEM], it_l[G::NITEM];
    unsigned it_o[G::NITEM];
#pragma unroll
    for (int s = 0; s < G::NITEM; ++s) {
        const int item = tid + s * G::NT;
        const int pl = item / G::NCROSS, q = item - pl * G::NCROSS;
        int lx, ly;
        if (q < TY * LX) {
            ly = N + q / LX;
            lx = q % LX;
        } else {
            const int r = q - TY * LX, hy = r / TX;
            lx = N + r % TX;
            ly = hy < N ? hy : TY + N;
        }
        int gi = (x0 - N + lx) % nx;
        if (gi < 0) gi += nx;
        int gj = (y0 - N + ly) % ny;
        if (gj < 0) gj += ny;
        // an item past the N planes reads level + 0 and writes a plane corner
        // (lx, ly < N), which no stencil reads
        const bool valid = item < N * G::NCROSS;
        it_p[s] = valid ? pl + 1 : 0;
        it_l[s] = valid ? ly * LX + lx : 0;
        it_o[s] = unsigned(gj * nx + gi) * 8u;
    }

    const int c = tid / (TX * TY);
    const int txy = tid - c * (TX * TY);
    const int ty = txy / TX, tx = txy - ty * TX;
    const int i = x0 + tx, j = y0 + ty;
    const bool owner = (i < nx) && (j < ny);
    const unsigned own = unsigned((j % ny) * nx + (i % nx)) * 8u;
    const int ax = tx % N, ay = ty % N;
    const int l_own = (ty + N) * LX + (tx + N);
    const int l_x = (ty + N) * LX + (tx - ax);
    const int l_y = (ty - ay) * LX + (tx + N);
    const double *cwxd = swd + ax * NS;
    const double *cwyd = swd + (N + ay) * NS;

    // the N new planes above level kbase into their ring slots, in two parts:
    // issue (every global load of every item, into registers, no item
    // branches) and commit (P' and the LDS stores)
    constexpr int NV = HASB ? 8 : 5;
    auto issue_planes = [&](int kbase, double (*v)[NV]) {
#pragma unroll
        for (int s = 0; s < G::NITEM; ++s) {
            const unsigned off = unsigned(kbase + it_p[s]) * pbytes + it_o[s];
#pragma unroll
            for (int f = 0; f < 4; ++f)
                v[s][f] = HASB && (f == 1 || f == 2) ? FiveField<false>::load(p.e0, f, p.fs, off)
                                                     : TA::load1(p.a[f], f, off);
            v[s][4] = HASB && !p.theta_in ? FiveField<false>::load(p.e0, 4, p.fs, off) : TA::load1(p.a[4], 4, off);
            if constexpr (HASB) {
                v[s][5 % NV] = TE1::load(p.e1, 1, p.fs, off);
                v[s][6 % NV] = TE1::load(p.e1, 2, p.fs, off);
                v[s][7 % NV] = p.theta_in ? 0.0 : TE1::load(p.e1, 4, p.fs, off);
            }
        }
    };
    auto commit_planes = [&](int kbase, double (*v)[NV]) {
        if constexpr (HASB) {
#pragma unroll
            for (int s = 0; s < G::NITEM; ++s) {
                v[s][1] += p.cb * v[s][5 % NV];
                v[s][2] += p.cb * v[s][6 % NV];
                if (!p.theta_in) v[s][4] += p.cb * v[s][7 % NV];
            }
        }
#pragma unroll
        for (int s = 0; s < G::NITEM; ++s) {
            const int k = kbase + it_p[s], kl = k - kb;
            const double Pp = pressure_perturbation(v[s][0], v[s][4], sR0[kl], sP0[kl], sIRT[kl], sT0[kl], eos);
            double *d = cfield(k % NQ) + it_l[s];
#pragma unroll
            for (int f = 0; f < 5; ++f) d[f * FS] = v[s][f];
            pfield(k % NQ)[it_l[s]] = Pp;
        }
    };
    // The first right-hand side (no epilogue inputs, fewest live registers)
    // issues the next element's plane loads before computing the current
    // element, so that they are in flight during its stencils; the others
    // would spill the registers that needs.
    constexpr bool PREFETCH = EPI == EPI_R;

    // sum_n D[r][n] g(level ez*N + n) over the own column for the six
    // z-differentiated quantities rho w, u, v, w, theta' (out) and P' (outp)
    // (not unrolled: unrolled, all 6*(N+1) LDS reads would be in flight at once)
    auto zsum = [&](int ez, int r, double *out, double &outp, double &outr, double &outw) {
#pragma unroll
        for (int f = 0; f < 5; ++f) out[f] = 0.0;
        outp = 0.0;
        outr = 0.0;
        outw = 0.0;
        int k = ez * N, slot = k % NQ;
#pragma unroll 1
        for (int n = 0; n < NQ; ++n) {
            const double *q = cfield(slot) + l_own;
            const double d = sD[r * NQ + n];
            outr += d * ((sR0[k - kb] + q[0]) * q[3 * FS]);
            outw += d * q[3 * FS];
            out[1] += d * q[1 * FS];
            out[2] += d * q[2 * FS];
            out[4] += d * q[4 * FS];
            outp += d * pfield(slot)[l_own];
            ++k;
            slot = (slot + 1 == NQ) ? 0 : slot + 1;
        }
    };

    // epilogue inputs of a node at byte offset off (issued before the node's
    // z sums and stencils, so that they arrive while those run)
    constexpr int NEPI = EPI == EPI_TWO ? 10 : (EPI == EPI_FINAL ? 5 : 1);
    auto epi_load = [&](unsigned off, double *ev) {
        if constexpr (EPI == EPI_TWO) {
#pragma unroll
            for (int f = 0; f < 5; ++f) {
                ev[f] = FiveField<false>::load(p.e0, f, p.fs, off);
                ev[5 + f] = TE1::load(p.e1, f, p.fs, off);
            }
        } else if constexpr (EPI == EPI_FINAL) {
#pragma unroll
            for (int f = 0; f < 5; ++f) ev[f] = FiveField<false>::load(p.e0, f, p.fs, off);
        }
    };

    // tendencies at level k (Set2NC, Sec. 3.1) from the x/y line derivatives
    // of the plane in the ring and the scaled vertical derivatives dz; then
    // the stage epilogue with its inputs ev
    auto node = [&](int k, const double *dz, double dzp, double dz0, double dzw, const double *ev) {
        const double *q = cfield(k % NQ);
        const double *qp = pfield(k % NQ);
        const double r0 = sR0[k - kb];
        const double rp = q[l_own], w = q[3 * FS + l_own];
        const double u = q[FS + l_own], v = q[2 * FS + l_own];
        const double ir = 1.0 / (r0 + rp);
        // the vertical terms first, so that only the tendencies stay live
        // across the x and y stencils (with few live registers the stencil
        // loads can be in flight together)
        double R[5];
        R[0] = dz0;
        R[1] = w * dz[1];
        R[2] = w * dz[2];
        // w: the nearly balanced vertical pressure gradient and buoyancy
        R[3] = w * dzw + dzp * ir + eos.grav * rp * ir;
        // theta': advection of theta' and of the background, w d theta0/dz
        R[4] = w * dz[4] + w * sTZ[k - kb];
        // line derivative of the six quantities along x (dir 0) or y (dir 1)
        // (not unrolled: unrolled, the scheduler hoists all its LDS reads)
        auto line = [&](int dir, double *d5, double &dp, double &dfl, double &dwl) {
            const double *cwd = dir == 0 ? cwxd : cwyd;
            const int base = dir == 0 ? l_x : l_y, step = dir == 0 ? 1 : LX;
            const int fv = dir == 0 ? FS : 2 * FS;  // the velocity in rho u or rho v
#pragma unroll
            for (int f = 0; f < 5; ++f) d5[f] = 0.0;
            dp = 0.0;
            dfl = 0.0;
            dwl = 0.0;
#pragma unroll 1
            for (int m = 0; m < NS; ++m) {
                const double cm = cwd[m];
                const double *qm = q + base + m * step;
                dfl += cm * ((r0 + qm[0]) * qm[fv]);
                d5[1] += cm * qm[1 * FS];
                d5[2] += cm * qm[2 * FS];
                dwl += cm * qm[3 * FS];
                d5[4] += cm * qm[4 * FS];
                dp += cm * qp[base + m * step];
            }
        };
        double d5[5];
        double dp, dfl, dwl;
        line(0, d5, dp, dfl, dwl);
        R[0] += dfl;
        R[1] += u * d5[1] + dp * ir;
        R[2] += u * d5[2];
        R[3] += u * dwl;
        R[4] += u * d5[4];
        line(1, d5, dp, dfl, dwl);
        R[0] = -(R[0] + dfl);
        R[1] = -(R[1] + v * d5[1]);
        R[2] = -(R[2] + v * d5[2] + dp * ir);
        R[3] = -(R[3] + v * dwl);
        R[4] = -(R[4] + v * d5[4]);
        if (k == 0 || k == p.nz - 1) R[3] = 0.0;
        if (!owner) return;
        auto Rv = [&](int f) -> double { return R[f]; };
        const unsigned off = unsigned(k) * pbytes + own;
        if constexpr (EPI == EPI_R) {
#pragma unroll
            for (int f = 0; f < 5; ++f) TO0::template store<NT>(p.out0, f, p.fs, off, Rv(f));
        } else if constexpr (EPI == EPI_TWO) {
#pragma unroll
            for (int f = 0; f < 5; ++f) {
                const double e0 = ev[f], e1 = ev[5 + f], r = Rv(f);
                TO0::template store<NT>(p.out0, f, p.fs, off, e0 + p.k01 * e1 + p.k02 * r);
                FiveField<false>::store<NT>(p.out1, f, p.fs, off, e0 + p.k11 * e1 + p.k12 * r);
            }
        } else {
            bool bad = false;
#pragma unroll
            for (int f = 0; f < 5; ++f) {
                const double v2 = ev[f] + p.k02 * Rv(f);
                bad |= !isfinite(v2);
                TO0::template store<NT>(p.out0, f, p.fs, off, v2);
            }
            if (bad) *p.flag = 1;
        }
    };

    __syncthreads();  // tables are in LDS

    // prologue: level ez0*N into the ring (the items of the first new plane
    // cover one whole plane); the c = 0 threads take the contribution of the
    // element below to the interface at ez0*N from their own column
#pragma unroll
    for (int s = 0; s < G::NITEM; ++s) {
        if (it_p[s] != 1) continue;
        const int k = ez0 * N, kl = k - kb;
        const unsigned off = unsigned(k) * pbytes + it_o[s];
        const double rp = stage_input<HASB, TA, TE1>(p, 0, off), u = stage_input<HASB, TA, TE1>(p, 1, off);
        const double v = stage_input<HASB, TA, TE1>(p, 2, off), w = stage_input<HASB, TA, TE1>(p, 3, off);
        const double th = stage_input<HASB, TA, TE1>(p, 4, off);
        const double Pp = pressure_perturbation(rp, th, sR0[kl], sP0[kl], sIRT[kl], sT0[kl], eos);
        double *d = cfield(k % NQ) + it_l[s];
        d[0 * FS] = rp;
        d[1 * FS] = u;
        d[2 * FS] = v;
        d[3 * FS] = w;
        d[4 * FS] = th;
        pfield(k % NQ)[it_l[s]] = Pp;
    }
    if (c == 0 && ez0 > 0) {
        const int eb = ez0 - 1;
        double acc[6] = {0, 0, 0, 0, 0, 0};
        for (int n = 0; n < NQ; ++n) {
            const int k = eb * N + n, kl = k - kb;
            const unsigned off = unsigned(k) * pbytes + own;
            const double rp = stage_input<HASB, TA, TE1>(p, 0, off);
            const double u = stage_input<HASB, TA, TE1>(p, 1, off);
            const double v = stage_input<HASB, TA, TE1>(p, 2, off);
            const double w = stage_input<HASB, TA, TE1>(p, 3, off);
            const double th = stage_input<HASB, TA, TE1>(p, 4, off);
            const double rho = sR0[kl] + rp;
            const double Pp = pressure_perturbation(rp, th, sR0[kl], sP0[kl], sIRT[kl], sT0[kl], eos);
            const double d = sD[N * NQ + n];
            acc[0] += d * (rho * w);
            acc[1] += d * u;
            acc[2] += d * v;
            acc[3] += d * w;
            acc[4] += d * th;
            acc[5] += d * Pp;
        }
        const double st = zs[2 * p.nez + eb];
        double *zb = zp + (ez0 & 1) * 6 * (TX * TY) + txy;
#pragma unroll
        for (int f = 0; f < 6; ++f) zb[f * (TX * TY)] = st * acc[f];
    }

    double vpre[G::NITEM][NV];
    if constexpr (PREFETCH) issue_planes(ez0 * N, vpre);
    for (int ez = ez0; ez < ez1; ++ez) {
        __syncthreads();  // the slots about to be overwritten are no longer read
        if constexpr (PREFETCH) {
            commit_planes(ez * N, vpre);
        } else {
            double v[G::NITEM][NV];
            issue_planes(ez * N, v);
            commit_planes(ez * N, v);
        }
        __syncthreads();
        if constexpr (PREFETCH) {
            if (ez + 1 < ez1) issue_planes((ez + 1) * N, vpre);
        }
        double ev[NEPI];
        epi_load(unsigned(ez * N + c) * pbytes + own, ev);
        double dz[5], sum[5];
        double sump, sumr, sumw;
        zsum(ez, c, sum, sump, sumr, sumw);
        const double sc = (c == 0) ? zs[p.nez + ez] : zs[ez];
        const double *zb = zp + (ez & 1) * 6 * (TX * TY) + txy;
        const bool below = c == 0 && ez > 0;  // a lower element shares the node
#pragma unroll
        for (int f = 0; f < 5; ++f) dz[f] = (below ? zb[f * (TX * TY)] : 0.0) + sc * sum[f];
        const double dzp = (below ? zb[5 * (TX * TY)] : 0.0) + sc * sump;
        const double dz0 = (below ? zb[0] : 0.0) + sc * sumr;
        const double dzw = (below ? zb[3 * (TX * TY)] : 0.0) + sc * sumw;
        node(ez * N + c, dz, dzp, dz0, dzw, ev);
        // this element's share of the interface (or top node) above
        const double st = zs[2 * p.nez + ez];
        double *zn = zp + ((ez + 1) & 1) * 6 * (TX * TY) + txy;
        if (c == 0) {
            double s5[5];
            double s5p, s5r, s5w;
            zsum(ez, N, s5, s5p, s5r, s5w);
#pragma unroll
            for (int f = 0; f < 5; ++f) zn[f * (TX * TY)] = f == 0 ? st * s5r : (f == 3 ? st * s5w : st * s5[f]);
            zn[5 * (TX * TY)] = st * s5p;
        }
    }
    // top node of the column: one-sided from the top element
    __syncthreads();  // the shares of the top element are in LDS
    if (ez1 == p.nez && c == 0) {
        const double *zb = zp + (ez1 & 1) * 6 * (TX * TY) + txy;
        double dz[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) dz[f] = zb[f * (TX * TY)];
        const double dzp = zb[5 * (TX * TY)];
        double ev[NEPI];
        epi_load(unsigned(p.nez * N) * pbytes + own, ev);
        node(p.nez * N, dz, dzp, zb[0], zb[3 * (TX * TY)], ev);
    }
}

// ---------------------------------------------------------------------------
// Launchers of k_rhs
// ---------------------------------------------------------------------------
// dynamic LDS of k_rhs: the ring, three per-level tables of the chunk's
// levels (zchunk + 1 elements), the element factors, the interface shares
template <int N, int V = 0>
size_t rhs_lds_bytes(int zchunk, int nez)
{
    using G = RhsGeom<N, V>;
    return G::LDS + sizeof(double) * (5 * ((zchunk + 1) * N + 1) + 3 * nez + 2 * 6 * G::TX * G::TY);
}

template <int N, int V = 0>
int rhs_zchunk_auto(const numa_ctx *c)
{
    if (c->rhs_zchunk > 0) return c->rhs_zchunk;
    using G = RhsGeom<N, V>;
    long tiles = ((c->nx + G::TX - 1) / G::TX) * ((c->ny + G::TY - 1) / G::TY);
    // enough workgroups for every CU (256) to hold two
    int zc = c->nez;
    while (zc > 1 && tiles * ((c->nez + zc - 1) / zc) < 512) zc = (zc + 1) / 2;
    return zc;
}

// Opt the kernel into lds bytes of dynamic LDS (needed above 64 KB); done
// once per size, before the first launch (and before any stream capture).
template <int N, int EPI, bool HASB, bool MIX, bool NT = false, int V = 0>
hipError_t rhs_prepare(size_t lds)
{
    static size_t attr_set = 0;
    if (attr_set < lds) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rhs<N, EPI, HASB, MIX, NT, V>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
        attr_set = lds;
    }
    return hipSuccess;
}

// Non-temporal FP64 stores for fields of at least 12 MB at order N <= 4: the
// largest kernel of such a step touches about 22 fields, more than the
// 256 MB last-level cache, so the next kernel reads its inputs from HBM
// whatever the store does.  Below that size the fields a kernel writes can
// still be in cache when the next kernel reads them.  Measured: on the
// 2.7M-node N = 4 benchmark grid they cut the stage-2 right-hand side from
// 132 to 124 us; on the ensemble, whose large domains are N = 5 and 7, they
// made the step 5 % slower, so higher orders keep ordinary stores.
constexpr size_t kNontemporalFieldBytes = size_t(12) << 20;
inline bool nontemporal_stores(const numa_ctx *c)
{
    return c->N <= 4 && size_t(c->np) * sizeof(double) >= kNontemporalFieldBytes;
}

// Launch k_rhs with tile variant V (numa_ctx::rhs_tile selects it).
template <int N, int V, int EPI, bool HASB, bool MIX>
hipError_t rhs_launch_t(numa_ctx *c, RhsParams p)
{
    using G = RhsGeom<N, V>;
    p.rho0 = c->lev.rho0;
    p.P0 = c->lev.P0;
    p.zsc = c->lev.zsc;
    p.wxy = c->lev.wxy;
    p.D = c->lev.D;
    p.th0 = c->lev.th0;
    p.th0z = c->lev.th0z;
    p.eos = c->eos;
    p.nx = int(c->nx);
    p.ny = int(c->ny);
    p.nz = int(c->nz);
    p.nez = c->nez;
    p.zchunk = rhs_zchunk_auto<N, V>(c);
    p.nchunk = (c->nez + p.zchunk - 1) / p.zchunk;
    p.ntx = int((c->nx + G::TX - 1) / G::TX);
    p.nty = int((c->ny + G::TY - 1) / G::TY);
    p.flag = c->flag;
    const size_t lds = rhs_lds_bytes<N, V>(p.zchunk, p.nez);
    dim3 grid(unsigned(p.ntx * p.nty * p.nchunk));
    if (nontemporal_stores(c)) {
        hipError_t e = rhs_prepare<N, EPI, HASB, MIX, true, V>(lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_rhs<N, EPI, HASB, MIX, true, V>), grid, dim3(G::NT), lds, c->stream, p);
    } else {
        hipError_t e = rhs_prepare<N, EPI, HASB, MIX, false, V>(lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_rhs<N, EPI, HASB, MIX, false, V>), grid, dim3(G::NT), lds, c->stream, p);
    }
    return hipGetLastError();
}

// The LDS opt-ins of the three right-hand sides of a step with tile V and
// vertical chunk zc (before any stream capture); MIX: the precision form,
// whose last right-hand side is the FP64 step's.
template <int N, int V, bool MIX>
hipError_t rhs_prepare_step(const numa_ctx *c, int zc)
{
    const size_t lds = rhs_lds_bytes<N, V>(zc, c->nez);
    auto three = [&](auto nt) -> hipError_t {
        constexpr bool NTS = decltype(nt)::value;
        hipError_t e = rhs_prepare<N, EPI_R, false, MIX, NTS, V>(lds);
        if (e == hipSuccess) e = rhs_prepare<N, EPI_TWO, true, MIX, NTS, V>(lds);
        if (e == hipSuccess) e = rhs_prepare<N, EPI_FINAL, false, false, NTS, V>(lds);
        return e;
    };
    return nontemporal_stores(c) ? three(std::true_type{}) : three(std::false_type{});
}

// The second tile variant (rhs_alt.hip): the step's three right-hand sides
// (EPI_R, EPI_TWO with the stage-2 inputs, EPI_FINAL), of the FP64 step or
// (mixed) of the precision form.
hipError_t rhs_launch_alt(numa_ctx *c, const RhsParams &p, int epi, bool mixed);
hipError_t rhs_prepare_alt(const numa_ctx *c, int zc, bool mixed);
// dynamic LDS of the variant's launch with vertical chunk zc
size_t rhs_lds_alt(int N, int zc, int nez);
// whether variant 1 differs from variant 0 for order N
bool rhs_alt_differs(int N);


}  // namespace numa
