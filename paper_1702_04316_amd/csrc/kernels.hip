// HIP kernels of the HEVI (1D-IMEX) ARK2 step for gfx950 (MI355X).
//
//  k_rhs      explicit Set2NC right-hand side with DSS, fused with the ARK
//             stage combinations (one pass over the state per evaluation)
//  k_colsolve_blocked  Schur-complement column solve with the stored band LU
//             factors, fused with the stage right-hand side and the
//             extraction; four wavefronts per 64 columns (short columns)
//  k_colsolve the same, one lane per column (tall columns)
//  k_factor   assembly and unpivoted band LU of the column Schur matrix (one
//             band shared by all columns, factored by one workgroup)
//  k_background  P0, G0, H0 per level with the device equation of state
//
// Layout: fields are FP64 structure of arrays [var][k][j][i], i fastest, on
// the unique nodes (x, y periodic).  The column factors are one band
// [k][m] that every column shares (all columns have the same matrix).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>
#include <vector>

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
template <int N>
struct Tile;
//                     TX  TY      threads   LDS (ring of N+1 planes, 6 fields)
template <> struct Tile<1> { static constexpr int TX = 32, TY = 16; };
template <> struct Tile<2> { static constexpr int TX = 32, TY = 8; };
template <> struct Tile<3> { static constexpr int TX = 24, TY = 6; };
template <> struct Tile<4> { static constexpr int TX = 16, TY = 8; };
template <> struct Tile<5> { static constexpr int TX = 15, TY = 5; };
template <> struct Tile<6> { static constexpr int TX = 12, TY = 6; };
template <> struct Tile<7> { static constexpr int TX = 14, TY = 7; };
template <> struct Tile<8> { static constexpr int TX = 8, TY = 8; };

template <int N, int ES = 8>  // ES: bytes of an LDS ring element (8 FP64, 4 FP32)
struct RhsGeom {
    static constexpr int TX = Tile<N>::TX, TY = Tile<N>::TY;
    static constexpr int NT = TX * TY * N;          // threads
    static constexpr int LX = TX + N + 1;           // plane incl. halo
    static constexpr int LY = TY + N + 1;
    static constexpr int FS = LX * LY;              // one field of one plane
    // a plane: rho', u, v, w, theta' (ES bytes each), then P' in FP64 (the
    // pressure and its derivatives stay FP64 in every form), and with FP32
    // fields FP64 copies of rho' and w for the buoyancy, the mass flux and
    // w's tendency
    static constexpr int POFF = (5 * FS * ES + 7) / 8 * 8;  // byte offset of P'
    static constexpr int ROFF = POFF + 8 * FS;               // byte offset of the FP64 rho' (ES = 4)
    static constexpr int WOFF = ROFF + 8 * FS;               // byte offset of the FP64 w (ES = 4)
    static constexpr int PB = ES == 8 ? ROFF : WOFF + 8 * FS; // bytes of a plane
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
// precision form's R1 with u and v in FP32 and rho', w, theta' in FP64.  The
// pressure perturbation P0 ((1+x)^gamma - 1) scales the relative rounding of
// rho' and theta' by P0, so their stage values stay FP64; w's tendency holds
// the stiff vertical pressure gradient and buoyancy, whose FP32 rounding,
// multiplied by the vertical Courant number, reached 2e-6 relative in w
// after 100 steps, so w stays FP64 too.  Byte offsets of the fields per
// node: 0, 8, 16, 24, 32 (FP64) or 0, 8, 12, 16, 24 (M).
// Offsets passed in are those an FP64 field would have.
template <bool M>
struct FiveField {
    static __device__ __forceinline__ bool f32(int f) { return M && (f == 1 || f == 2); }
    static __device__ __forceinline__ size_t ofs(int f, long np)
    {
        return M ? size_t(np) * size_t(f == 0 ? 0 : (f == 1 ? 8 : (f == 2 ? 12 : 8 * f - 8))) : size_t(np) * 8 * size_t(f);
    }
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
// in FP64.  The precision form (MIX) keeps the state q and the accumulator
// ACC (e0 of the last two launches, out1) in FP64, its other stage buffers
// in the mixed layout, and the LDS ring (except P' and FP64 copies of rho'
// and w) and the stencil arithmetic in FP32.  FP64 in that form: P' and its
// derivatives, w with its derivatives and tendency, and the mass flux
// (rho0 + rho') u_i with its divergence.  The flux divergence is a small
// difference of large terms at the finest LGL spacing, and its FP32
// rounding, carried through rho' into the buoyancy, left 2.5e-6 relative
// error in w after 100 steps at N = 7; FP32 derivatives of w under a strong
// wind left 2e-6 after 50 steps at N = 3.
template <int EPI, bool MIX>
struct RhsTypes {
    using A = FiveField<false>;                     // inputs a[]
    using E1 = FiveField<MIX>;                      // e1 (R1)
    using O0 = FiveField<MIX && EPI == EPI_R>;      // out0 (R1 in the first launch)
    using D = FiveField<false>;                     // e0, out1
    using C = std::conditional_t<MIX, float, double>;
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

template <int N, int EPI, bool HASB, bool MIX, bool NT = false>
__global__ __launch_bounds__((RhsGeom<N, MIX ? 4 : 8>::NT), (RhsGeom<N, MIX ? 4 : 8>::MINW)) void k_rhs(RhsParams p)
{
    using TT = RhsTypes<EPI, MIX>;
    using TA = typename TT::A;
    using TE1 = typename TT::E1;
    using TO0 = typename TT::O0;
    using C = typename TT::C;
    using G = RhsGeom<N, sizeof(C)>;
    constexpr int NQ = N + 1, NS = G::NS, TX = G::TX, TY = G::TY, LX = G::LX, FS = G::FS;
    // dynamic LDS: ring of N+1 planes [rho', u, v, w, theta' (C)][P' (FP64)]
    // of [LY][LX], then per-level tables rho0, P0, 1/(rho0 theta0), theta0,
    // d theta0/dz for the
    // levels this chunk touches, zsc [3][nez], and the interface shares
    // [2][6][TX*TY] (FP64)
    extern __shared__ double lds_block[];
    char *const ringb = reinterpret_cast<char *>(lds_block);
    auto cfield = [&](int slot) { return reinterpret_cast<C *>(ringb + slot * G::PB); };
    auto pfield = [&](int slot) { return reinterpret_cast<double *>(ringb + slot * G::PB + G::POFF); };
    auto rfield = [&](int slot) { return reinterpret_cast<double *>(ringb + slot * G::PB + G::ROFF); };
    auto wfield = [&](int slot) { return reinterpret_cast<double *>(ringb + slot * G::PB + G::WOFF); };
    __shared__ C sw[2][N][NS];
    __shared__ C sD[NQ * NQ];
    // FP64 copies of the tables for the mass flux of the precision form (the
    // FP64 form reads sw and sD themselves)
    __shared__ double swd_m[MIX ? 2 * N * NS : 1];
    __shared__ double sDd_m[MIX ? NQ * NQ : 1];
    const double *const swd = [&]() -> const double * {
        if constexpr (MIX) return swd_m;
        else return &sw[0][0][0];
    }();
    const double *const sDd = [&]() -> const double * {
        if constexpr (MIX) return sDd_m;
        else return sD;
    }();

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
        (&sw[0][0][0])[s] = C(p.wxy[s]);
        if constexpr (MIX) swd_m[s] = p.wxy[s];
    }
    for (int s = tid; s < NQ * NQ; s += G::NT) {
        sD[s] = C(p.D[s]);
        if constexpr (MIX) sDd_m[s] = p.D[s];
    }
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
    // Precision form: the ring holds u - uref and v - vref in FP32, with the
    // workgroup's reference velocities uref, vref (FP64) taken at the first
    // node of its tile.  A wind far larger than its variation (a uniform
    // wind) then keeps its variation's relative precision in the FP32
    // derivatives, which annihilate the constants; u and v themselves are
    // uref + (u - uref).  The FP64 form stores u and v as they are.
    double uref = 0.0, vref = 0.0;
    if constexpr (MIX) {
        const unsigned oref = unsigned(ez0 * N) * pbytes + unsigned(y0 * nx + x0) * 8u;
        uref = stage_input<HASB, TA, TE1>(p, 1, oref);
        vref = stage_input<HASB, TA, TE1>(p, 2, oref);
    }

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
    const C *cwx = &sw[0][0][0] + ax * NS;
    const C *cwy = &sw[1][0][0] + ay * NS;
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
            C *d = cfield(k % NQ) + it_l[s];
            d[0 * FS] = C(v[s][0]);
            d[1 * FS] = C(v[s][1] - uref);
            d[2 * FS] = C(v[s][2] - vref);
            d[3 * FS] = C(v[s][3]);
            d[4 * FS] = C(v[s][4]);
            pfield(k % NQ)[it_l[s]] = Pp;
            if constexpr (MIX) {
                rfield(k % NQ)[it_l[s]] = v[s][0];
                wfield(k % NQ)[it_l[s]] = v[s][3];
            }
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
    auto zsum = [&](int ez, int r, C *out, double &outp, double &outr, double &outw) {
#pragma unroll
        for (int f = 0; f < 5; ++f) out[f] = C(0);
        outp = 0.0;
        outr = 0.0;
        outw = 0.0;
        int k = ez * N, slot = k % NQ;
#pragma unroll 1
        for (int n = 0; n < NQ; ++n) {
            const C *q = cfield(slot) + l_own;
            const C d = sD[r * NQ + n];
            if constexpr (MIX) {
                const double wv = wfield(slot)[l_own], dd = sDd[r * NQ + n];
                outr += dd * ((sR0[k - kb] + rfield(slot)[l_own]) * wv);
                outw += dd * wv;
            } else {
                outr += double(d) * ((C(sR0[k - kb]) + q[0]) * q[3 * FS]);
                outw += double(d) * q[3 * FS];
            }
            out[1] += d * q[1 * FS];
            out[2] += d * q[2 * FS];
            out[4] += d * q[4 * FS];
            outp += double(d) * pfield(slot)[l_own];
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
    auto node = [&](int k, const C *dz, double dzp, double dz0, double dzw, const double *ev) {
        const C *q = cfield(k % NQ);
        const double *qp = pfield(k % NQ);
        const C r0 = C(sR0[k - kb]);
        const C rp = q[l_own], w = q[3 * FS + l_own];
        C u = q[FS + l_own], v = q[2 * FS + l_own];
        if constexpr (MIX) {
            u = C(uref + double(u));
            v = C(vref + double(v));
        }
        const C ir = C(1) / (r0 + rp);
        // rho' and 1/rho for the pressure and buoyancy terms: FP64 in every form
        const double rpd = MIX ? rfield(k % NQ)[l_own] : double(rp);
        const double irp = MIX ? 1.0 / (sR0[k - kb] + rpd) : double(ir);
        // the vertical terms first, so that only the tendencies stay live
        // across the x and y stencils (with few live registers the stencil
        // loads can be in flight together)
        C R[5];
        double R0 = dz0;
        R[1] = w * dz[1];
        R[2] = w * dz[2];
        // w's tendency accumulates in FP64 in every form: it holds the nearly
        // balanced vertical pressure gradient and buoyancy (in the precision
        // form only its advection products are FP32)
        double R3;
        if constexpr (MIX)
            R3 = wfield(k % NQ)[l_own] * dzw + (dzp * irp + eos.grav * rpd * irp);
        else
            R3 = w * dzw + dzp * ir + eos.grav * rp * ir;
        // theta': advection of theta' and of the background, w d theta0/dz
        R[4] = w * dz[4] + w * C(sTZ[k - kb]);
        // line derivative of the six quantities along x (dir 0) or y (dir 1)
        // (not unrolled: unrolled, the scheduler hoists all its LDS reads)
        auto line = [&](int dir, C *d5, double &dp, double &dfl, double &dwl) {
            const C *cw = dir == 0 ? cwx : cwy;
            const double *cwd = dir == 0 ? cwxd : cwyd;
            const double *rq = rfield(k % NQ);
            const double *wq = wfield(k % NQ);
            const int base = dir == 0 ? l_x : l_y, step = dir == 0 ? 1 : LX;
            const int fv = dir == 0 ? FS : 2 * FS;  // the velocity in rho u or rho v
            const double vr = dir == 0 ? uref : vref;
#pragma unroll
            for (int f = 0; f < 5; ++f) d5[f] = C(0);
            dp = 0.0;
            dfl = 0.0;
            dwl = 0.0;
#pragma unroll 1
            for (int m = 0; m < NS; ++m) {
                const C cm = cw[m];
                const C *qm = q + base + m * step;
                if constexpr (MIX) dfl += cwd[m] * ((sR0[k - kb] + rq[base + m * step]) * (vr + double(qm[fv])));
                else dfl += double(cm) * ((r0 + qm[0]) * qm[fv]);
                d5[1] += cm * qm[1 * FS];
                d5[2] += cm * qm[2 * FS];
                if constexpr (MIX) dwl += cwd[m] * wq[base + m * step];
                else dwl += double(cm) * qm[3 * FS];
                d5[4] += cm * qm[4 * FS];
                dp += double(cm) * qp[base + m * step];
            }
        };
        C d5[5];
        double dp, dfl, dwl;
        line(0, d5, dp, dfl, dwl);
        R0 += dfl;
        R[1] += u * d5[1] + C(dp * irp);
        R[2] += u * d5[2];
        R3 += double(u) * dwl;
        R[4] += u * d5[4];
        line(1, d5, dp, dfl, dwl);
        R0 = -(R0 + dfl);
        R[1] = -(R[1] + v * d5[1]);
        R[2] = -(R[2] + v * d5[2] + C(dp * irp));
        R3 = -(R3 + double(v) * dwl);
        R[4] = -(R[4] + v * d5[4]);
        if (k == 0 || k == p.nz - 1) R3 = 0.0;
        if (!owner) return;
        auto Rv = [&](int f) -> double { return f == 3 ? R3 : (f == 0 ? R0 : double(R[f])); };
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
        C *d = cfield(k % NQ) + it_l[s];
        d[0 * FS] = C(rp);
        d[1 * FS] = C(u - uref);
        d[2 * FS] = C(v - vref);
        d[3 * FS] = C(w);
        d[4 * FS] = C(th);
        pfield(k % NQ)[it_l[s]] = Pp;
        if constexpr (MIX) {
            rfield(k % NQ)[it_l[s]] = rp;
            wfield(k % NQ)[it_l[s]] = w;
        }
    }
    if (c == 0 && ez0 > 0) {
        const int eb = ez0 - 1;
        double acc[6] = {0, 0, 0, 0, 0, 0};
        for (int n = 0; n < NQ; ++n) {
            const int k = eb * N + n, kl = k - kb;
            const unsigned off = unsigned(k) * pbytes + own;
            // rounded to the ring's type first, as the layer loop sees them
            const double rp = C(stage_input<HASB, TA, TE1>(p, 0, off));
            const double u = C(stage_input<HASB, TA, TE1>(p, 1, off) - uref);
            const double v = C(stage_input<HASB, TA, TE1>(p, 2, off) - vref);
            const double w = stage_input<HASB, TA, TE1>(p, 3, off);  // FP64 in both forms
            const double th0 = stage_input<HASB, TA, TE1>(p, 4, off), th = C(th0);
            const double rho = MIX ? sR0[kl] + stage_input<HASB, TA, TE1>(p, 0, off) : double(C(sR0[kl])) + rp;
            const double Pp = pressure_perturbation(stage_input<HASB, TA, TE1>(p, 0, off), th0, sR0[kl], sP0[kl],
                                                    sIRT[kl], sT0[kl], eos);
            const double d = double(sD[N * NQ + n]);
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
        for (int f = 0; f < 5; ++f) zb[f * (TX * TY)] = (f == 0 || f == 3) ? st * acc[f] : double(C(st * acc[f]));
        zb[5 * (TX * TY)] = st * acc[5];
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
        C dz[5], sum[5];
        double sump, sumr, sumw;
        zsum(ez, c, sum, sump, sumr, sumw);
        const double scd = (c == 0) ? zs[p.nez + ez] : zs[ez];
        const C sc = C(scd);
        const double *zb = zp + (ez & 1) * 6 * (TX * TY) + txy;
        const bool below = c == 0 && ez > 0;  // a lower element shares the node
#pragma unroll
        for (int f = 0; f < 5; ++f) dz[f] = (below ? C(zb[f * (TX * TY)]) : C(0)) + sc * sum[f];
        const double dzp = (below ? zb[5 * (TX * TY)] : 0.0) + scd * sump;
        const double dz0 = (below ? zb[0] : 0.0) + scd * sumr;
        const double dzw = (below ? zb[3 * (TX * TY)] : 0.0) + scd * sumw;
        node(ez * N + c, dz, dzp, dz0, dzw, ev);
        // this element's share of the interface (or top node) above
        const double st = zs[2 * p.nez + ez];
        double *zn = zp + ((ez + 1) & 1) * 6 * (TX * TY) + txy;
        if (c == 0) {
            C s5[5];
            double s5p, s5r, s5w;
            zsum(ez, N, s5, s5p, s5r, s5w);
#pragma unroll
            for (int f = 0; f < 5; ++f)
                zn[f * (TX * TY)] = f == 0 ? st * s5r : (f == 3 ? st * s5w : double(C(st) * s5[f]));
            zn[5 * (TX * TY)] = st * s5p;
        }
    }
    // top node of the column: one-sided from the top element
    __syncthreads();  // the shares of the top element are in LDS
    if (ez1 == p.nez && c == 0) {
        const double *zb = zp + (ez1 & 1) * 6 * (TX * TY) + txy;
        C dz[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) dz[f] = C(zb[f * (TX * TY)]);
        const double dzp = zb[5 * (TX * TY)];
        double ev[NEPI];
        epi_load(unsigned(p.nez * N) * pbytes + own, ev);
        node(p.nez * N, dz, dzp, zb[0], zb[3 * (TX * TY)], ev);
    }
}

// ---------------------------------------------------------------------------
// Column solve.  One lane per column, 64 columns per workgroup (one
// wavefront, so one wavefront per SIMD on the benchmark grid).  The column's
// pressure P and rho0*w live in LDS as [level][lane] (conflict free), padded
// so the band operators need no bounds tests.  Every pass walks the levels
// once and streams its per-level global loads a fixed number of levels ahead
// of their use (slots in registers, rotated by unrolling), keeping up to ~56
// loads in flight per wavefront: with one wavefront per SIMD there is no
// other wavefront to hide the memory latency.
// ---------------------------------------------------------------------------
// Per-level tables are read through the constant address space: their loads
// are uniform and become scalar loads.
typedef const __attribute__((address_space(4))) double cdouble;
__device__ __forceinline__ cdouble *as_const(const double *p) { return (cdouble *)(p); }


struct SolveParams {
    // q~_e for rho', w, theta': sum_t c_t * ptr_t
    const void *er[3], *ew[3], *et[3];
    double cr[3], cw[3], ct[3];
    // outputs: rho' = sum_t cbr_t br_t - lambda Dz(rho0 w~);  w = w~ + sum_t cbw_t bw_t;
    // over a stratified background (out_t set) also theta' = sum_t cbt_t bt_t - TZ w~
    const void *br[2], *bw[2], *bt[2];
    double cbr[2], cbw[2], cbt[2];
    void *out_r, *out_w, *out_t;
    // FP64 field where the forward pass parks w_a for the extraction (out_w
    // itself when that is FP64): w~ = w_a - lambda (...) cancels strongly at
    // large vertical Courant numbers, so w_a must keep FP64 precision
    double *park;
    const double *fac;
    const double *scf, *dzb;
    double lambda;
    int nz;
    long ncol;
};

// term counts of the stage variants: (NR, NW, NT) explicit-estimate terms,
// (NBR, NBW) output terms; F32: which fields are FP32 (bit 0+t er[t], 3+t
// ew[t], 6+t et[t], 9+t br[t], 11+t bw[t], 13 out_w, 14 out_r), the rest FP64
template <int NR_, int NW_, int NT_, int NBR_, int NBW_, int NBT_, unsigned F32_ = 0>
struct SolveShape {
    static constexpr int NR = NR_, NW = NW_, NT = NT_, NBR = NBR_, NBW = NBW_, NBT = NBT_;
    static constexpr unsigned F32 = F32_;
};
using ShapePlain = SolveShape<1, 1, 1, 1, 0, 1>;
using ShapeStage2 = SolveShape<1, 1, 1, 2, 1, 2>;
using ShapeStage3 = SolveShape<3, 3, 3, 1, 2, 1>;
// element type of field bit b of a shape
template <class SH, int B>
using SolveT = std::conditional_t<((SH::F32 >> B) & 1u) != 0, float, double>;

template <int N, class SH>
struct SolveGeom {
    static constexpr int HB = 2 * N;   // half-bandwidth of S
    static constexpr int NE = SH::NR + SH::NW + SH::NT;
    static constexpr int depth(int per_level) { return 56 / per_level < 1 ? 1 : (56 / per_level > 8 ? 8 : 56 / per_level); }
    static constexpr int DF = depth(NE);                        // forward: the estimates
    static constexpr int DX = depth(1 + SH::NBW + SH::NBR);     // extraction
    // ring of rho0*w levels (>= 2N+1 for the band window, >= HB for the
    // reads of P below level 0)
    static constexpr int R = (2 * N + 1) <= 16 ? 16 : 32;
    static size_t lds_bytes(int M) { return size_t(R + M + HB) * 64 * sizeof(double); }
    // the shared factor band is staged in LDS too when the total fits a CU
    static size_t fac_bytes(int M) { return size_t(M) * (4 * N + 1) * sizeof(double); }
    static bool fac_in_lds(int M) { return lds_bytes(M) + fac_bytes(M) <= kLdsPerCU; }
    static size_t lds_total(int M) { return lds_bytes(M) + (fac_in_lds(M) ? fac_bytes(M) : 0); }
};

template <int N, class SH, bool FL>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_colsolve(SolveParams p)
{
    using G = SolveGeom<N, SH>;
    extern __shared__ double smem[];
    constexpr int NS = 2 * N + 1, NB = 4 * N + 1, HB = G::HB, R = G::R, NE = G::NE;
    constexpr int DF = G::DF, DX = G::DX, NXL = 1 + SH::NBW + SH::NBR;
    const int lane = threadIdx.x;
    const long col = (long)blockIdx.x * 64 + lane;
    const bool act = col < p.ncol;
    const unsigned cbyte = unsigned(act ? col : 0) * 8u;
    const int M = p.nz;
    const unsigned lbytes = unsigned(p.ncol) * 8u;  // one level of a field
    cdouble *scf = as_const(p.scf);
    cdouble *dzb = as_const(p.dzb);
    // LDS: [ring of rho0*w: R levels][P: M levels][HB zero levels].  The
    // substitutions and band sums read up to HB levels outside [0, M); there
    // the factor or band coefficient is exactly 0 and the LDS holds finite
    // values (ring or zero levels), so those terms vanish.
    double *W = smem + lane;                   // W[(k & (R-1)) * 64]
    double *P = smem + R * 64 + lane;          // P[k * 64], k in [-R, M + HB)
    for (int k = 0; k < R; ++k) W[k * 64] = 0.0;
    for (int k = 0; k < HB; ++k) P[(M + k) * 64] = 0.0;
    // row d of the factor band of level k
    // the factor band, one set shared by all columns: [k][d].  FL: staged in
    // LDS after P (broadcast reads); otherwise read through the constant
    // address space (scalar loads)
    double *facl = smem + (R + M + HB) * 64;
    if constexpr (FL) {
        for (int e = lane; e < M * NB; e += 64) facl[e] = p.fac[e];
        __syncthreads();
    }
    auto fac = [&](int idx) -> double {
        if constexpr (FL) return facl[idx];
        else return as_const(p.fac)[idx];
    };

    // ---- forward.  Step s: P_e and rho0 w_a of level s into LDS (w_a also
    //      parked in p.park for the extraction), then the substitution of
    //      level s - N, whose Dz(rho0 w_a) band is complete:
    //      y_k = P_e,k - lambda G0 Dz(rho0 w_a)_k - sum_d L_kd y_{k-d}
    {
        double es[DF][NE];
        auto load = [&](double *e, int s) {
            const unsigned off = unsigned(min(s, M - 1)) * lbytes + cbyte;
            // (t = 0..2 spelled out: the element type is a template argument)
            if constexpr (SH::NR > 0) e[0] = tload<SolveT<SH, 0>>(p.er[0], off);
            if constexpr (SH::NR > 1) e[1] = tload<SolveT<SH, 1>>(p.er[1], off);
            if constexpr (SH::NR > 2) e[2] = tload<SolveT<SH, 2>>(p.er[2], off);
            if constexpr (SH::NW > 0) e[SH::NR + 0] = tload<SolveT<SH, 3>>(p.ew[0], off);
            if constexpr (SH::NW > 1) e[SH::NR + 1] = tload<SolveT<SH, 4>>(p.ew[1], off);
            if constexpr (SH::NW > 2) e[SH::NR + 2] = tload<SolveT<SH, 5>>(p.ew[2], off);
            if constexpr (SH::NT > 0) e[SH::NR + SH::NW + 0] = tload<SolveT<SH, 6>>(p.et[0], off);
            if constexpr (SH::NT > 1) e[SH::NR + SH::NW + 1] = tload<SolveT<SH, 7>>(p.et[1], off);
            if constexpr (SH::NT > 2) e[SH::NR + SH::NW + 2] = tload<SolveT<SH, 8>>(p.et[2], off);
        };
#pragma unroll
        for (int b = 0; b < DF; ++b) load(es[b], b);
        for (int s0 = 0; s0 < M + N; s0 += DF) {
#pragma unroll
            for (int b = 0; b < DF; ++b) {
                const int s = s0 + b;
                if (s < M) {
                    double re = 0.0, we = 0.0, te = 0.0;
#pragma unroll
                    for (int t = 0; t < SH::NR; ++t) re += p.cr[t] * es[b][t];
#pragma unroll
                    for (int t = 0; t < SH::NW; ++t) we += p.cw[t] * es[b][SH::NR + t];
#pragma unroll
                    for (int t = 0; t < SH::NT; ++t) te += p.ct[t] * es[b][SH::NR + SH::NW + t];
                    cdouble *cf = scf + s * SC_N;
                    // w_a = B A^-1 (w_e + lambda g H0 theta_e / (G0 rho0))  (Eq. (16))
                    const double wa = (s == 0 || s == M - 1) ? 0.0 : cf[SC_AI] * we + cf[SC_WA] * te;
                    P[s * 64] = cf[SC_G0] * re + cf[SC_H0] * te;
                    W[(s & (R - 1)) * 64] = cf[SC_RHO0] * wa;
                    if (act) gstore(p.park, unsigned(s) * lbytes + cbyte, wa);
                }
                const int k = s - N;
                if (k >= 0 && k < M) {
                    cdouble *bz = dzb + k * NS;
                    double d = 0.0;
#pragma unroll
                    for (int m = 0; m < NS; ++m) d += bz[m] * W[((k - N + m) & (R - 1)) * 64];
                    cdouble *ck = scf + k * SC_N;
                    double y = P[k * 64] - ck[SC_LG] * d - ck[SC_HZ] * (W[(k & (R - 1)) * 64] / ck[SC_RHO0]);
#pragma unroll
                    for (int dd = 0; dd < HB; ++dd) y -= fac(k * NB + dd) * P[(k - HB + dd) * 64];  // column k - HB + dd
                    P[k * 64] = y;
                }
                load(es[b], s + DF);
            }
        }
    }
    // ---- backward substitution (U; the reciprocal pivot is stored)
    {
        for (int k = M - 1; k >= 0; --k) {
            const int u = k * NB + HB;  // U row of level k: reciprocal pivot, then columns k + 1 .. k + HB
            double x = P[k * 64];
#pragma unroll
            for (int dd = 1; dd <= HB; ++dd) x -= fac(u + dd) * P[(k + dd) * 64];
            P[k * 64] = x * fac(u);
        }
    }
    // ---- extraction.  Step s: w~_s = B (w_a - lambda (Dz P / rho0 + g P /
    //      (G0 rho0))), w out = w~ + shifts, rho0 w~ into the ring; then
    //      rho'_k = q_e,rho - lambda Dz(rho0 w~) of level k = s - N, whose
    //      band is complete
    {
        double xs[DX][NXL];
        auto load = [&](double *x, int s) {
            const unsigned off = unsigned(min(s, M - 1)) * lbytes + cbyte;
            x[0] = gload(p.park, off);  // w_a parked by the forward pass
            if constexpr (SH::NBW > 0) x[1] = tload<SolveT<SH, 11>>(p.bw[0], off);
            if constexpr (SH::NBW > 1) x[2] = tload<SolveT<SH, 12>>(p.bw[1], off);
            const unsigned offr = unsigned(min(max(s - N, 0), M - 1)) * lbytes + cbyte;
            if constexpr (SH::NBR > 0) x[1 + SH::NBW] = tload<SolveT<SH, 9>>(p.br[0], offr);
            if constexpr (SH::NBR > 1) x[2 + SH::NBW] = tload<SolveT<SH, 10>>(p.br[1], offr);
        };
#pragma unroll
        for (int b = 0; b < DX; ++b) load(xs[b], b);
        for (int s0 = 0; s0 < M + N; s0 += DX) {
#pragma unroll
            for (int b = 0; b < DX; ++b) {
                const int s = s0 + b;
                if (s < M) {
                    cdouble *cf = scf + s * SC_N;
                    cdouble *bz = dzb + s * NS;
                    double d = 0.0;
#pragma unroll
                    for (int m = 0; m < NS; ++m) d += bz[m] * P[(s - N + m) * 64];
                    const double wt =
                        (s == 0 || s == M - 1) ? 0.0 : xs[b][0] - (cf[SC_X1] * d + cf[SC_X2] * P[s * 64]);
                    double sh = 0.0;
#pragma unroll
                    for (int t = 0; t < SH::NBW; ++t) sh += p.cbw[t] * xs[b][1 + t];
                    W[(s & (R - 1)) * 64] = cf[SC_RHO0] * wt;
                    if (act) tstore<SolveT<SH, 13>>(p.out_w, unsigned(s) * lbytes + cbyte, wt + sh);
                    if (p.out_t && act) {  // theta' over a stratified background
                        const unsigned off = unsigned(s) * lbytes + cbyte;
                        double th = 0.0;
#pragma unroll
                        for (int t = 0; t < SH::NBT; ++t) th += p.cbt[t] * gload(static_cast<const double *>(p.bt[t]), off);
                        gstore(static_cast<double *>(p.out_t), off, th - cf[SC_TZ] * wt);
                    }
                }
                const int k = s - N;
                if (k >= 0 && k < M) {
                    cdouble *bz = dzb + k * NS;
                    double d = 0.0;
#pragma unroll
                    for (int m = 0; m < NS; ++m) d += bz[m] * W[((k - N + m) & (R - 1)) * 64];
                    double qr = 0.0;
#pragma unroll
                    for (int t = 0; t < SH::NBR; ++t) qr += p.cbr[t] * xs[b][1 + SH::NBW + t];
                    if (act) tstore<SolveT<SH, 14>>(p.out_r, unsigned(k) * lbytes + cbyte, qr - p.lambda * d);
                }
                load(xs[b], s + DX);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Level-blocked column solve (columns of at most 224 levels).  A workgroup
// of W wavefronts owns 64 columns (one per lane): W = 4 for columns of at
// most 64 - 2N levels, 8 up to 128 levels, 16 (the largest workgroup) up to
// 224 levels where the LDS below fits one CU.  Wavefront g owns the level
// block [g KL, (g+1) KL), KL = ceil(nz/W) <= blocked_kl(W), and
// keeps its levels' values in registers.  One LDS array V, [N pad][M
// levels][N pad] x 64 lanes, exchanges the one field a phase needs from
// other levels, and the shared LU band sits in LDS beside it:
//  1. the estimates: P_e and w_a in registers, V = rho0 w_a;
//  2. b = P_e - lambda G0 Dz(rho0 w_a), then V = b;
//  3. the forward and backward band substitutions (Alg. 9) in place in V,
//     by wavefront 0 for all 64 columns: the only level-by-level
//     recurrence, with every operand in LDS or registers;
//  4. w~ = B (w_a - lambda (Dz x / rho0 + g x / (G0 rho0))), w out, then
//     V = rho0 w~;
//  5. rho' = q_e,rho - lambda Dz(rho0 w~).
// w_a never leaves the registers, so nothing is parked in HBM, and the
// global loads of phases 1, 4 and 5 come from four wavefronts per 64
// columns.  The pads hold zeros and meet only zero band coefficients.
// ---------------------------------------------------------------------------
constexpr int kBlockedKL = 16;
// levels per wavefront: 16 with 4 or 8 wavefronts; 14 with 16 wavefronts,
// whose four wavefronts per SIMD leave 128 registers per lane
constexpr int blocked_kl(int W) { return W == 16 ? 14 : kBlockedKL; }
constexpr int kBlockedMaxLevels = 16 * 14;

// levels whose global loads are issued together
constexpr int blocked_chunk(int per_level, int W) { return W == 16 ? (per_level >= 6 ? 2 : 4) : (per_level >= 6 ? 4 : 8); }

template <int N, class SH, bool NT, int W>
__global__ __launch_bounds__(64 * W)
__attribute__((amdgpu_waves_per_eu(W == 16 ? 4 : (W == 8 ? 2 : (N <= 6 ? 4 : 3)))))
void k_colsolve_blocked(SolveParams p)
{
    extern __shared__ double smem[];
    constexpr int NS = 2 * N + 1, KX = blocked_kl(W), NE = SolveGeom<N, SH>::NE;
    constexpr int CF = blocked_chunk(NE, W), CX = blocked_chunk(1 + SH::NBW + SH::NBR, W);
    const int lane = threadIdx.x & 63;
    const int g = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const long col = (long)blockIdx.x * 64 + lane;
    const bool act = col < p.ncol;
    const unsigned cbyte = unsigned(act ? col : 0) * 8u;
    const int M = p.nz, KL = (M + W - 1) / W, k0 = g * KL;
    const int nk = max(0, min(KL, M - k0));  // levels of this wavefront
    const unsigned lbytes = unsigned(p.ncol) * 8u;
    cdouble *scf = as_const(p.scf);
    cdouble *dzb = as_const(p.dzb);
    double *V = smem + N * 64 + lane;  // V[k * 64], k in [-N, M + N)
    constexpr int HB = 2 * N, NB = 4 * N + 1;
    double *F = smem + (M + 2 * N) * 64;  // the shared LU band, [k][NB]
    for (int t = threadIdx.x; t < N * 64; t += 64 * W) {
        smem[t] = 0.0;
        smem[(M + N) * 64 + t] = 0.0;
    }
    for (int e = threadIdx.x; e < M * NB; e += 64 * W) F[e] = p.fac[e];
    // Dz of the field in V at level s (band of half-width N)
    auto dz_of_v = [&](int s) {
        cdouble *bz = dzb + s * NS;
        double d = 0.0;
#pragma unroll
        for (int m = 0; m < NS; ++m) d += bz[m] * V[(s - N + m) * 64];
        return d;
    };
    double wa[KX], r[KX];  // w_a; then P_e, b, x, rho0 w~ in turn
    // ---- 1. estimates, CF levels at a time (loads first, then the algebra)
#pragma unroll
    for (int i0 = 0; i0 < KX; i0 += CF) {
        if (i0 < nk) {
            double e[CF][NE];
#pragma unroll
            for (int b = 0; b < CF; ++b) {
                const unsigned off = unsigned(k0 + min(i0 + b, nk - 1)) * lbytes + cbyte;
                if constexpr (SH::NR > 0) e[b][0] = tload<SolveT<SH, 0>>(p.er[0], off);
                if constexpr (SH::NR > 1) e[b][1] = tload<SolveT<SH, 1>>(p.er[1], off);
                if constexpr (SH::NR > 2) e[b][2] = tload<SolveT<SH, 2>>(p.er[2], off);
                if constexpr (SH::NW > 0) e[b][SH::NR + 0] = tload<SolveT<SH, 3>>(p.ew[0], off);
                if constexpr (SH::NW > 1) e[b][SH::NR + 1] = tload<SolveT<SH, 4>>(p.ew[1], off);
                if constexpr (SH::NW > 2) e[b][SH::NR + 2] = tload<SolveT<SH, 5>>(p.ew[2], off);
                if constexpr (SH::NT > 0) e[b][SH::NR + SH::NW + 0] = tload<SolveT<SH, 6>>(p.et[0], off);
                if constexpr (SH::NT > 1) e[b][SH::NR + SH::NW + 1] = tload<SolveT<SH, 7>>(p.et[1], off);
                if constexpr (SH::NT > 2) e[b][SH::NR + SH::NW + 2] = tload<SolveT<SH, 8>>(p.et[2], off);
            }
#pragma unroll
            for (int b = 0; b < CF; ++b) {
                const int i = i0 + b, s = k0 + i;
                if (i < nk) {
                    double re = 0.0, we = 0.0, te = 0.0;
#pragma unroll
                    for (int t = 0; t < SH::NR; ++t) re += p.cr[t] * e[b][t];
#pragma unroll
                    for (int t = 0; t < SH::NW; ++t) we += p.cw[t] * e[b][SH::NR + t];
#pragma unroll
                    for (int t = 0; t < SH::NT; ++t) te += p.ct[t] * e[b][SH::NR + SH::NW + t];
                    cdouble *cf = scf + s * SC_N;
                    // w_a = B A^-1 (w_e + lambda g H0 theta_e / (G0 rho0))  (Eq. (16))
                    wa[i] = (s == 0 || s == M - 1) ? 0.0 : cf[SC_AI] * we + cf[SC_WA] * te;
                    r[i] = cf[SC_G0] * re + cf[SC_H0] * te;
                    V[s * 64] = cf[SC_RHO0] * wa[i];
                }
            }
        }
    }
    __syncthreads();
    // ---- 2. b = P_e - lambda G0 Dz(rho0 w_a) - lambda H0 (d theta0/dz) w_a
#pragma unroll
    for (int i = 0; i < KX; ++i)
        if (i < nk) r[i] -= scf[(k0 + i) * SC_N + SC_LG] * dz_of_v(k0 + i) + scf[(k0 + i) * SC_N + SC_HZ] * wa[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < KX; ++i)
        if (i < nk) V[(k0 + i) * 64] = r[i];
    __syncthreads();
    // ---- 3. x = S^-1 b by the band substitutions of the LU factors, one
    //      wavefront for the 64 columns.  The newest value enters each sum
    //      last, so the recurrence is one multiply-add per level; b and (for
    //      N <= 4, where the registers allow) the factor row are read one
    //      level ahead
    if (g == 0) {
        constexpr bool PF = N <= 4;
        constexpr int PR = PF ? HB + 1 : 1;  // prefetched row entries
        double win[HB];
#pragma unroll
        for (int t = 0; t < HB; ++t) win[t] = 0.0;
        double bn = V[0], ln[PR];
        if constexpr (PF) {
#pragma unroll
            for (int dd = 0; dd < HB; ++dd) ln[dd] = F[dd];
        }
        for (int k = 0; k < M; ++k) {
            double y = bn, l[PR];
            if constexpr (PF) {
#pragma unroll
                for (int dd = 0; dd < HB; ++dd) l[dd] = ln[dd];
            }
            if (k + 1 < M) {
                bn = V[(k + 1) * 64];
                if constexpr (PF) {
#pragma unroll
                    for (int dd = 0; dd < HB; ++dd) ln[dd] = F[(k + 1) * NB + dd];
                }
            }
#pragma unroll
            for (int dd = 0; dd < HB; ++dd) y -= (PF ? l[dd] : F[k * NB + dd]) * win[dd];
#pragma unroll
            for (int t = 0; t < HB - 1; ++t) win[t] = win[t + 1];
            win[HB - 1] = y;
            V[k * 64] = y;
        }
#pragma unroll
        for (int t = 0; t < HB; ++t) win[t] = 0.0;
        double xn = V[(M - 1) * 64], un[PR];
        if constexpr (PF) {
#pragma unroll
            for (int dd = 0; dd <= HB; ++dd) un[dd] = F[(M - 1) * NB + HB + dd];
        }
        for (int k = M - 1; k >= 0; --k) {
            double x = xn, u[PR];
            if constexpr (PF) {
#pragma unroll
                for (int dd = 0; dd <= HB; ++dd) u[dd] = un[dd];
            }
            if (k > 0) {
                xn = V[(k - 1) * 64];
                if constexpr (PF) {
#pragma unroll
                    for (int dd = 0; dd <= HB; ++dd) un[dd] = F[(k - 1) * NB + HB + dd];
                }
            }
#pragma unroll
            for (int dd = HB; dd >= 1; --dd) x -= (PF ? u[dd] : F[k * NB + HB + dd]) * win[dd - 1];
            x *= PF ? u[0] : F[k * NB + HB];
#pragma unroll
            for (int t = HB - 1; t > 0; --t) win[t] = win[t - 1];
            win[0] = x;
            V[k * 64] = x;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < KX; ++i)
        if (i < nk) r[i] = V[(k0 + i) * 64];
    // ---- 4. w~ and the w output (and theta' over a stratified background)
    const bool strat = p.out_t != nullptr;
#pragma unroll
    for (int i0 = 0; i0 < KX; i0 += CX) {
        if (i0 < nk) {
            double xb[CX][2], xt[CX][2];
#pragma unroll
            for (int b = 0; b < CX; ++b) {
                const unsigned off = unsigned(k0 + min(i0 + b, nk - 1)) * lbytes + cbyte;
                if constexpr (SH::NBW > 0) xb[b][0] = tload<SolveT<SH, 11>>(p.bw[0], off);
                if constexpr (SH::NBW > 1) xb[b][1] = tload<SolveT<SH, 12>>(p.bw[1], off);
                if (strat) {
#pragma unroll
                    for (int t = 0; t < SH::NBT; ++t) xt[b][t] = gload(static_cast<const double *>(p.bt[t]), off);
                }
            }
#pragma unroll
            for (int b = 0; b < CX; ++b) {
                const int i = i0 + b, s = k0 + i;
                if (i < nk) {
                    cdouble *cf = scf + s * SC_N;
                    const double wt =
                        (s == 0 || s == M - 1) ? 0.0 : wa[i] - (cf[SC_X1] * dz_of_v(s) + cf[SC_X2] * r[i]);
                    double sh = 0.0;
#pragma unroll
                    for (int t = 0; t < SH::NBW; ++t) sh += p.cbw[t] * xb[b][t];
                    r[i] = cf[SC_RHO0] * wt;
                    if (act) tstore<SolveT<SH, 13>, NT>(p.out_w, unsigned(s) * lbytes + cbyte, wt + sh);
                    if (strat && act) {
                        double th = 0.0;
#pragma unroll
                        for (int t = 0; t < SH::NBT; ++t) th += p.cbt[t] * xt[b][t];
                        gstore<NT>(static_cast<double *>(p.out_t), unsigned(s) * lbytes + cbyte, th - cf[SC_TZ] * wt);
                    }
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < KX; ++i)
        if (i < nk) V[(k0 + i) * 64] = r[i];
    __syncthreads();
    // ---- 5. rho' = q_e,rho - lambda Dz(rho0 w~)
#pragma unroll
    for (int i0 = 0; i0 < KX; i0 += CX) {
        if (i0 < nk) {
            double xr[CX][2];
#pragma unroll
            for (int b = 0; b < CX; ++b) {
                const unsigned off = unsigned(k0 + min(i0 + b, nk - 1)) * lbytes + cbyte;
                if constexpr (SH::NBR > 0) xr[b][0] = tload<SolveT<SH, 9>>(p.br[0], off);
                if constexpr (SH::NBR > 1) xr[b][1] = tload<SolveT<SH, 10>>(p.br[1], off);
            }
#pragma unroll
            for (int b = 0; b < CX; ++b) {
                const int i = i0 + b, k = k0 + i;
                if (i < nk) {
                    double qr = 0.0;
#pragma unroll
                    for (int t = 0; t < SH::NBR; ++t) qr += p.cbr[t] * xr[b][t];
                    if (act)
                        tstore<SolveT<SH, 14>, NT>(p.out_r, unsigned(k) * lbytes + cbyte, qr - p.lambda * dz_of_v(k));
                }
            }
        }
    }
}

// Per-level coefficients of the column solve at lambda (Eqs. (14)-(17) in
// 1D): with the vertical part of A = I + lambda^2 (g/theta0) grad(theta0)^T,
// a = 1 + lambda^2 g (d theta0/dz)/theta0 (1 over a neutral background), and
// F0 . u = G0 w d rho0/dz + H0 w d theta0/dz, whose G0 part the divergence
// form G0 Dz(rho0 w) holds:
//   w_a = B (w_e + lambda g H0 theta_e/(G0 rho0)) / a = AI w_e + WA theta_e,
//   w_p = B (X1 Dz P + X2 P), X1 = lambda/(a rho0), X2 = lambda g/(a G0 rho0),
//   S P = P - LG Dz(rho0 w_p) - HZ w_p, LG = lambda G0, HZ = lambda H0 d theta0/dz,
//   theta' = theta_e - TZ w~, TZ = lambda d theta0/dz.
__global__ void k_solve_coefs(const double *rho0, const double *G0, const double *H0, const double *th0,
                              const double *th0z, double lambda, double grav, int nz, double *scf)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nz) return;
    const double r0 = rho0[k], g0 = G0[k], h0 = H0[k], tz = th0z[k];
    const double ai = 1.0 / (1.0 + lambda * lambda * grav * tz / th0[k]);
    double *o = scf + SC_N * k;
    o[SC_G0] = g0;
    o[SC_H0] = h0;
    o[SC_RHO0] = r0;
    o[SC_WA] = ai * (lambda * grav * h0 / (g0 * r0));
    o[SC_LG] = lambda * g0;
    o[SC_X1] = (lambda * ai) / r0;
    o[SC_X2] = (lambda * ai) * grav / (g0 * r0);
    o[SC_AI] = ai;
    o[SC_HZ] = lambda * h0 * tz;
    o[SC_TZ] = lambda * tz;
    for (int t = SC_TZ + 1; t < SC_N; ++t) o[t] = 0.0;
}

// ---------------------------------------------------------------------------
// Column factorisation: S = I - LG Dz rho0 B (X1 Dz + X2) - HZ B (X1 Dz + X2)
// (the Schur matrix of the coefficients above; over a neutral background
// I - lambda^2 G0 Dz B (Dz + g/G0)), assembled as a band of half-width 2N,
// then Doolittle LU without pivoting (Alg. 9).  Every column has the same
// matrix, so one workgroup factors the single shared band [row][offset]:
// its threads assemble the entries, then for each pivot k update the
// (2N x 2N) trailing window in parallel and scale column k.  Each entry sees
// the same updates in the same order as a sequential elimination.  The band
// is worked on in LDS when it fits (kFactorLds bytes), else in place in
// global memory; both through one generic pointer.
// ---------------------------------------------------------------------------
constexpr int kFactorThreads = 256;
constexpr size_t kFactorLds = 64 * 1024;

template <int N>
__global__ __launch_bounds__(kFactorThreads) void k_factor(const double *__restrict__ dzb,
                                                           const double *__restrict__ scf, int M, int in_lds,
                                                           double *fac, int *flag)
{
    extern __shared__ double band_lds[];
    constexpr int NS = 2 * N + 1, NB = 4 * N + 1, HB = 2 * N;
    const int tid = threadIdx.x;
    double *A = in_lds ? band_lds : fac;  // entry (r, c) at r*NB + (c - r + HB)
    for (int idx = tid; idx < M * NB; idx += kFactorThreads) {
        const int r = idx / NB, cidx = r + idx % NB - HB;
        double v = 0.0;
        if (cidx >= 0 && cidx < M) {
            // rows of the interior levels m (B zeroes the walls)
            double s = 0.0;
            const int mlo = max(max(r, cidx) - N, 1), mhi = min(min(r, cidx) + N, M - 2);
            for (int m = mlo; m <= mhi; ++m) {
                const double drm = dzb[(long)r * NS + (m - r + N)];
                const double dmc = dzb[(long)m * NS + (cidx - m + N)];
                const double *cm = scf + (long)m * SC_N;
                s += drm * cm[SC_RHO0] * (cm[SC_X1] * dmc + (m == cidx ? cm[SC_X2] : 0.0));
            }
            const double *cr = scf + (long)r * SC_N;
            v = (r == cidx ? 1.0 : 0.0) - cr[SC_LG] * s;
            if (r >= 1 && r <= M - 2 && cidx >= r - N && cidx <= r + N)
                v -= cr[SC_HZ] * (cr[SC_X1] * dzb[(long)r * NS + (cidx - r + N)] + (r == cidx ? cr[SC_X2] : 0.0));
        }
        A[idx] = v;
    }
    __syncthreads();
    bool bad = false;
    for (int k = 0; k < M; ++k) {
        const double piv = A[k * NB + HB];
        const double rp = 1.0 / piv;
        const int w = min(k + HB, M - 1) - k;  // rows below / columns right of the pivot
        for (int t = tid; t < w * w; t += kFactorThreads) {
            const int i = k + 1 + t / w, jj = k + 1 + t % w;
            const double l = A[i * NB + (k - i + HB)] * rp;
            A[i * NB + (jj - i + HB)] -= l * A[k * NB + (jj - k + HB)];
        }
        __syncthreads();  // column k and the pivot are read above, written below
        for (int t = tid; t < w; t += kFactorThreads) A[(k + 1 + t) * NB + (-1 - t + HB)] *= rp;
        if (tid == 0) {
            bad |= !(fabs(piv) > 0.0) || !isfinite(piv);
            A[k * NB + HB] = rp;  // the solve multiplies by the reciprocal pivot
        }
        __syncthreads();
    }
    if (in_lds)
        for (int idx = tid; idx < M * NB; idx += kFactorThreads) fac[idx] = band_lds[idx];
    if (bad) *flag = 1;
}

// P0 = EOS(rho0, theta0), G0 = gamma P0 / rho0, H0 = gamma P0 / theta0 per level
__global__ void k_background(const double *rho0, const double *th0, double *P0, double *G0, double *H0, int nz,
                             EOS e)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nz) return;
    double P = eos_pressure(rho0[k], th0[k], e);
    P0[k] = P;
    G0[k] = e.gamma * P / rho0[k];
    H0[k] = e.gamma * P / th0[k];
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
namespace {

// dynamic LDS of k_rhs: the ring, three per-level tables of the chunk's
// levels (zchunk + 1 elements), the element factors, the interface shares
template <int N, bool MIX = false>
size_t rhs_lds_bytes(int zchunk, int nez)
{
    constexpr int ES = MIX ? 4 : 8;
    return RhsGeom<N, ES>::LDS +
           sizeof(double) * (5 * ((zchunk + 1) * N + 1) + 3 * nez + 2 * 6 * RhsGeom<N>::TX * RhsGeom<N>::TY);
}

template <int N>
int rhs_zchunk_auto(const numa_ctx *c)
{
    if (c->rhs_zchunk > 0) return c->rhs_zchunk;
    using G = RhsGeom<N>;
    long tiles = ((c->nx + G::TX - 1) / G::TX) * ((c->ny + G::TY - 1) / G::TY);
    // enough workgroups for every CU (256) to hold two
    int zc = c->nez;
    while (zc > 1 && tiles * ((c->nez + zc - 1) / zc) < 512) zc = (zc + 1) / 2;
    return zc;
}

// Opt the kernel into lds bytes of dynamic LDS (needed above 64 KB); done
// once per size, before the first launch (and before any stream capture).
template <int N, int EPI, bool HASB, bool MIX, bool NT = false>
hipError_t rhs_prepare(size_t lds)
{
    static size_t attr_set = 0;
    if (attr_set < lds) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rhs<N, EPI, HASB, MIX, NT>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
        attr_set = lds;
    }
    return hipSuccess;
}

template <int N, class SH, bool FL>
hipError_t solve_prepare_fl(size_t shm)
{
    static size_t attr_set = 0;  // tall columns need LDS above 64 KB
    if (shm > 65536 && attr_set < shm) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_colsolve<N, SH, FL>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));
        if (e != hipSuccess) return e;
        attr_set = shm;
    }
    return hipSuccess;
}

// the LDS opt-in of the column-solve variant used for M levels
template <int N, class SH>
hipError_t solve_prepare(int M)
{
    using G = SolveGeom<N, SH>;
    return G::fac_in_lds(M) ? solve_prepare_fl<N, SH, true>(G::lds_total(M))
                            : solve_prepare_fl<N, SH, false>(G::lds_total(M));
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
bool nontemporal_stores(const numa_ctx *c)
{
    return c->N <= 4 && size_t(c->np) * sizeof(double) >= kNontemporalFieldBytes;
}

template <int N, int EPI, bool HASB, bool MIX = false>
hipError_t rhs_launch(numa_ctx *c, RhsParams p)
{
    using G = RhsGeom<N>;
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
    p.zchunk = rhs_zchunk_auto<N>(c);
    p.nchunk = (c->nez + p.zchunk - 1) / p.zchunk;
    p.ntx = int((c->nx + G::TX - 1) / G::TX);
    p.nty = int((c->ny + G::TY - 1) / G::TY);
    p.flag = c->flag;
    const size_t lds = rhs_lds_bytes<N, MIX>(p.zchunk, p.nez);
    dim3 grid(unsigned(p.ntx * p.nty * p.nchunk));
    if (!MIX && nontemporal_stores(c)) {
        hipError_t e = rhs_prepare<N, EPI, HASB, MIX, true>(lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_rhs<N, EPI, HASB, MIX, true>), grid, dim3(G::NT), lds, c->stream, p);
    } else {
        hipError_t e = rhs_prepare<N, EPI, HASB, MIX>(lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_rhs<N, EPI, HASB, MIX>), grid, dim3(G::NT), lds, c->stream, p);
    }
    return hipGetLastError();
}

// The eight- and sixteen-wavefront blocked solves of columns above 64 - 2N
// levels: their LDS, (nz + 2N) x 64 doubles plus the band, can exceed the
// default 64 KB (at most 108 KB at 128 levels, 160 KB above)
template <int N, class SH, int W>
hipError_t blocked_prepare(size_t lds)
{
    static size_t attr_set = 65536;
    if (lds > attr_set) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_colsolve_blocked<N, SH, false, W>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
        attr_set = lds;
    }
    return hipSuccess;
}

size_t blocked_lds_bytes(int N, int M) { return (size_t(M + 2 * N) * 64 + size_t(M) * (4 * N + 1)) * sizeof(double); }

template <int N, class SH>
hipError_t solve_launch(numa_ctx *c, SolveParams p)
{
    if (!p.park) p.park = static_cast<double *>(p.out_w);  // FP64 output: park in place
    p.fac = c->fac;
    p.scf = c->lev.scf;
    p.dzb = c->lev.dzb;
    p.lambda = c->lambda;
    p.nz = int(c->nz);
    p.ncol = c->ncol;
    using G = SolveGeom<N, SH>;
    const int M = int(c->nz);
    if (blocked_solve_used(c)) {
        const size_t lds = blocked_lds_bytes(N, M);
        const dim3 grid(unsigned((c->ncol + 63) / 64));
        if (M > 8 * kBlockedKL) {
            hipError_t e = blocked_prepare<N, SH, 16>(lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((k_colsolve_blocked<N, SH, false, 16>), grid, dim3(1024), lds, c->stream, p);
        } else if (M + 2 * N > 64) {
            hipError_t e = blocked_prepare<N, SH, 8>(lds);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((k_colsolve_blocked<N, SH, false, 8>), grid, dim3(512), lds, c->stream, p);
        } else if (nontemporal_stores(c)) {
            hipLaunchKernelGGL((k_colsolve_blocked<N, SH, true, 4>), grid, dim3(256), lds, c->stream, p);
        } else {
            hipLaunchKernelGGL((k_colsolve_blocked<N, SH, false, 4>), grid, dim3(256), lds, c->stream, p);
        }
        return hipGetLastError();
    }
    const size_t shm = G::lds_total(M);
    hipError_t e = solve_prepare<N, SH>(M);
    if (e != hipSuccess) return e;
    dim3 grid(unsigned((c->ncol + 63) / 64));
    if (G::fac_in_lds(M))
        hipLaunchKernelGGL((k_colsolve<N, SH, true>), grid, dim3(64), shm, c->stream, p);
    else
        hipLaunchKernelGGL((k_colsolve<N, SH, false>), grid, dim3(64), shm, c->stream, p);
    return hipGetLastError();
}

template <int N>
hipError_t factor_launch(numa_ctx *c, double lambda)
{
    // one factor set, shared by all columns (their matrices are identical)
    const size_t bytes = size_t(c->nz) * (4 * N + 1) * sizeof(double);
    const bool lds = bytes <= kFactorLds;
    hipLaunchKernelGGL((k_factor<N>), dim3(1), dim3(kFactorThreads), lds ? bytes : 0, c->stream, c->lev.dzb,
                       c->lev.scf, int(c->nz), int(lds), c->fac, c->flag);
    return hipGetLastError();
}

}  // namespace

// the blocked solve holds at most 16 levels per wavefront in registers with
// up to 8 wavefronts (128 levels, LDS at most 108 KB), 14 with 16 (224
// levels, where its LDS fits one CU)
bool blocked_solve_ok(int N, int64_t nz)
{
    if (N < 1 || nz < 2) return false;
    if (nz <= 8 * kBlockedKL) return true;
    return nz <= kBlockedMaxLevels && blocked_lds_bytes(N, int(nz)) <= kLdsPerCU;
}

bool blocked_solve_used(const numa_ctx *c)
{
    if (c->column_solver == NUMA_SOLVER_BAND) return false;
    return c->column_solver == NUMA_SOLVER_BLOCKED || blocked_solve_ok(c->N, c->nz);
}

namespace {

// Run f(std::integral_constant<int, N>) for the context's order N.
template <typename F>
hipError_t dispatch(int N, F &&f)
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

void set_fields(const void *arr[5], const double *base, long np)
{
    for (int f = 0; f < 5; ++f) arr[f] = base ? base + f * np : nullptr;
}

// ARK2 tableau (Table 1, signs restored by the order conditions)
struct Ark2 {
    double a21, a31, a32, ad, b1, b2, b3, c31, c32;
    Ark2()
    {
        const double s2 = std::sqrt(2.0);
        const double al = (3.0 + 2.0 * s2) / 6.0;
        a21 = 2.0 - s2;
        a31 = 1.0 - al;
        a32 = al;
        ad = 1.0 - 1.0 / s2;                 // implicit diagonal
        const double at31 = 1.0 / (2.0 * s2), at32 = 1.0 / (2.0 * s2);
        b1 = b2 = 1.0 / (2.0 * s2);
        b3 = ad;
        c31 = (at31 - a31) / ad;             // q~ shifts (Sec. 2.2)
        c32 = (at32 - a32) / ad;             // (c21 = -1 exactly)
    }
};

}  // namespace

// LDS one workgroup of each kernel needs on this grid (the right-hand side
// at its largest vertical chunk), static arrays included.
size_t lds_needed(int N, int nez, int nz)
{
    size_t need = 0;
    auto f = [&](auto n) -> hipError_t {
        constexpr int NN = decltype(n)::value;
        const size_t stat = sizeof(double) * (2 * NN * (2 * NN + 1) + (NN + 1) * (NN + 1));
        need = std::max(rhs_lds_bytes<NN>(nez, nez) + stat, SolveGeom<NN, ShapeStage3>::lds_bytes(nz));
        return hipSuccess;
    };
    (void)dispatch(N, f);
    return need;
}

StageBuffers stage_buffers(numa_ctx *c)
{
    const long np = c->np;
    StageBuffers s;
    s.R1 = c->work;
    s.E3 = c->work + 5 * np;
    s.ACC = c->work + 10 * np;
    s.Q2r = c->work + 15 * np;
    s.Q2w = c->work + 16 * np;
    s.Q3r = c->work + 17 * np;
    s.Q3w = c->work + 18 * np;
    s.Q2t = c->work + 19 * np;
    s.Q3t = c->work + 20 * np;
    return s;
}

hipError_t launch_background(numa_ctx *c)
{
    hipLaunchKernelGGL(k_background, dim3(unsigned((c->nz + 63) / 64)), dim3(64), 0, c->stream, c->lev.rho0,
                       c->lev.th0, c->lev.P0, c->lev.G0, c->lev.H0, int(c->nz), c->eos);
    return hipGetLastError();
}

hipError_t launch_factor(numa_ctx *c, double lambda)
{
    hipLaunchKernelGGL(k_solve_coefs, dim3(unsigned((c->nz + 63) / 64)), dim3(64), 0, c->stream, c->lev.rho0,
                       c->lev.G0, c->lev.H0, c->lev.th0, c->lev.th0z, lambda, c->eos.grav, int(c->nz), c->lev.scf);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return dispatch(c->N, [&](auto n) { return factor_launch<decltype(n)::value>(c, lambda); });
}

hipError_t launch_rhs_plain(numa_ctx *c, const double *q, double *R)
{
    RhsParams p{};
    set_fields(p.a, q, c->np);
    p.out0 = R;
    p.fs = c->np;
    return dispatch(c->N, [&](auto n) { return rhs_launch<decltype(n)::value, EPI_R, false>(c, p); });
}

// R(Q) with the stage epilogue out0 = e0 + k01 e1 + k02 R, out1 = e0 + k11 e1 + k12 R
// (all five fields of Q given)
hipError_t launch_rhs_two(numa_ctx *c, const double *Q, const double *e0, const double *e1, double *out0,
                          double *out1, double k01, double k02, double k11, double k12)
{
    RhsParams p{};
    set_fields(p.a, Q, c->np);
    p.out0 = out0;
    p.out1 = out1;
    p.e0 = e0;
    p.e1 = e1;
    p.fs = c->np;
    p.k01 = k01; p.k02 = k02;
    p.k11 = k11; p.k12 = k12;
    return dispatch(c->N, [&](auto n) { return rhs_launch<decltype(n)::value, EPI_TWO, false>(c, p); });
}

// out = e0 + k R(Q), non-finite values flagged
hipError_t launch_rhs_final(numa_ctx *c, const double *Q, const double *e0, double *out, double k)
{
    RhsParams p{};
    set_fields(p.a, Q, c->np);
    p.out0 = out;
    p.e0 = e0;
    p.fs = c->np;
    p.k02 = k;
    return dispatch(c->N, [&](auto n) { return rhs_launch<decltype(n)::value, EPI_FINAL, false>(c, p); });
}

hipError_t launch_solve_plain(numa_ctx *c, const double *y, double *x)
{
    const long np = c->np;
    SolveParams p{};
    p.er[0] = y + 0 * np; p.cr[0] = 1.0;
    p.ew[0] = y + 3 * np; p.cw[0] = 1.0;
    p.et[0] = y + 4 * np; p.ct[0] = 1.0;
    p.br[0] = y + 0 * np; p.cbr[0] = 1.0;
    p.out_r = x + 0 * np;
    p.out_w = x + 3 * np;
    if (stratified(c)) {  // theta' = y_theta - lambda (d theta0/dz) w
        p.bt[0] = y + 4 * np; p.cbt[0] = 1.0;
        p.out_t = x + 4 * np;
    }
    hipError_t e;
    for (int f : {1, 2, 4}) {
        if (f == 4 && stratified(c)) continue;
        e = hipMemcpyAsync(x + f * np, y + f * np, sizeof(double) * np, hipMemcpyDeviceToDevice, c->stream);
        if (e != hipSuccess) return e;
    }
    return dispatch(c->N, [&](auto n) { return solve_launch<decltype(n)::value, ShapePlain>(c, p); });
}

// One ARK2 step in the q~ form (Sec. 2.2):
//   stage i:  q~ = q~_e + lambda L_V(q~),  q~_e = q_e^(i) + sum_j c_ij Q_j,
//             Q_i = q~ - sum_j c_ij Q_j,   c_ij = (at_ij - a_ij)/at_ii,
//   q^{n+1} = q^n + dt sum_i b_i R_i.
// With c21 = -1 and Q1 = q^n, stage 2 needs q~_e = dt a21 R1 only.  Kernels:
//   K1 rhs(q^n)            -> R1
//   K2 colsolve(stage 2)   -> Q2 rho', w  (u, v, theta' of Q2 are q^n + dt a21 R1)
//   K3 rhs(Q2)             -> E3 = q^n + dt(a31 R1 + a32 R2), ACC = q^n + dt b1 (R1 + R2)
//   K4 colsolve(stage 3)   -> Q3 rho', w  (u, v, theta' of Q3 are E3's)
//   K5 rhs(Q3)             -> q^{n+1} = ACC + dt b3 R3 (in place)
hipError_t launch_hevi_step(numa_ctx *c, double *q, double dt, hipEvent_t *ev)
{
    static const Ark2 t;
    const long np = c->np;
    StageBuffers s = stage_buffers(c);
    const double *qr = q + 0 * np, *qw = q + 3 * np, *qt = q + 4 * np;
    const double *R1 = s.R1;
    const bool strat = stratified(c);
    hipError_t e;

    // ev (optional): events ev[0..5] recorded around the 5 kernels
    auto mark = [&](int i) -> hipError_t { return ev ? hipEventRecord(ev[i], c->stream) : hipSuccess; };
    if ((e = mark(0)) != hipSuccess) return e;

    // K1
    e = launch_rhs_plain(c, q, s.R1);
    if (e != hipSuccess) return e;
    if ((e = mark(1)) != hipSuccess) return e;

    // K2: q~_e = dt a21 R1 ; Q2 rho' = q^n + dt a21 R1 - lambda Dz(rho0 w~) ; Q2 w = w~ + q^n w
    {
        SolveParams p{};
        const double f = dt * t.a21;
        p.er[0] = R1 + 0 * np; p.cr[0] = f;
        p.ew[0] = R1 + 3 * np; p.cw[0] = f;
        p.et[0] = R1 + 4 * np; p.ct[0] = f;
        p.br[0] = qr; p.cbr[0] = 1.0; p.br[1] = R1 + 0 * np; p.cbr[1] = f;
        p.bw[0] = qw; p.cbw[0] = 1.0;
        p.out_r = s.Q2r;
        p.out_w = s.Q2w;
        if (strat) {  // Q2 theta' = q^n + dt a21 R1 - lambda (d theta0/dz) w~
            p.bt[0] = qt; p.cbt[0] = 1.0; p.bt[1] = R1 + 4 * np; p.cbt[1] = f;
            p.out_t = s.Q2t;
        }
        e = dispatch(c->N, [&](auto n) { return solve_launch<decltype(n)::value, ShapeStage2>(c, p); });
        if (e != hipSuccess) return e;
        if ((e = mark(2)) != hipSuccess) return e;
    }

    // K3: rhs(Q2), Q2 = (Q2r, qu + f R1u, qv + f R1v, Q2w, qt + f R1t)
    {
        RhsParams p{};
        const double f = dt * t.a21;
        p.a[0] = s.Q2r;
        p.a[3] = s.Q2w;
        p.cb = f;  // u, v, theta' = e0 + f e1 = q^n + f R1
        if (strat) {  // theta' from the solve
            p.theta_in = 1;
            p.a[4] = s.Q2t;
        }
        p.out0 = s.E3;
        p.out1 = s.ACC;
        p.e0 = q;
        p.e1 = R1;
        p.fs = np;
        p.k01 = dt * t.a31; p.k02 = dt * t.a32;
        p.k11 = dt * t.b1;  p.k12 = dt * t.b2;
        e = dispatch(c->N, [&](auto n) { return rhs_launch<decltype(n)::value, EPI_TWO, true>(c, p); });
        if (e != hipSuccess) return e;
        if ((e = mark(3)) != hipSuccess) return e;
    }

    // K4: q~_e = E3 + c31 q^n + c32 Q2 (rho', w, theta');  theta' of Q2 = qt + f R1t
    {
        SolveParams p{};
        const double f = dt * t.a21;
        p.er[0] = s.E3 + 0 * np; p.cr[0] = 1.0; p.er[1] = qr; p.cr[1] = t.c31; p.er[2] = s.Q2r; p.cr[2] = t.c32;
        p.ew[0] = s.E3 + 3 * np; p.cw[0] = 1.0; p.ew[1] = qw; p.cw[1] = t.c31; p.ew[2] = s.Q2w; p.cw[2] = t.c32;
        p.et[0] = s.E3 + 4 * np; p.ct[0] = 1.0; p.et[1] = qt; p.ct[1] = t.c31 + t.c32; p.et[2] = R1 + 4 * np;
        p.ct[2] = t.c32 * f;
        p.br[0] = s.E3 + 0 * np; p.cbr[0] = 1.0;
        p.bw[0] = qw; p.cbw[0] = -t.c31; p.bw[1] = s.Q2w; p.cbw[1] = -t.c32;
        p.out_r = s.Q3r;
        p.out_w = s.Q3w;
        if (strat) {  // Q2 theta' is the solve's; Q3 theta' = E3 - lambda (d theta0/dz) w~
            p.ct[1] = t.c31; p.et[2] = s.Q2t; p.ct[2] = t.c32;
            p.bt[0] = s.E3 + 4 * np; p.cbt[0] = 1.0;
            p.out_t = s.Q3t;
        }
        e = dispatch(c->N, [&](auto n) { return solve_launch<decltype(n)::value, ShapeStage3>(c, p); });
        if (e != hipSuccess) return e;
        if ((e = mark(4)) != hipSuccess) return e;
    }

    // K5: rhs(Q3), Q3 = (Q3r, E3u, E3v, Q3w, E3t);  q^{n+1} = ACC + dt b3 R3
    {
        RhsParams p{};
        p.a[0] = s.Q3r;
        p.a[1] = s.E3 + 1 * np;
        p.a[2] = s.E3 + 2 * np;
        p.a[3] = s.Q3w;
        p.a[4] = strat ? s.Q3t : s.E3 + 4 * np;
        p.out0 = q;
        p.e0 = s.ACC;
        p.fs = np;
        p.k02 = dt * t.b3;
        e = dispatch(c->N, [&](auto n) { return rhs_launch<decltype(n)::value, EPI_FINAL, false>(c, p); });
        if (e != hipSuccess) return e;
        if ((e = mark(5)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// byte offset of field f in the precision form's five-field buffers (the
// device layout of FiveField<true>)
size_t mixed_field_offset(int f, long np)
{
    return size_t(np) * size_t(f == 0 ? 0 : (f == 1 ? 8 : (f == 2 ? 12 : 8 * f - 8)));
}

// The precision form of the step (same stage algebra as launch_hevi_step):
// the right-hand sides evaluate in FP32 (P', its derivatives, w's tendency
// and the mass flux in FP64); the stage buffer R1 holds u, v in FP32 and
// rho', w, theta' in FP64, E3 and Q2, Q3 (rho', w) are FP64 (E3's u and v
// are differentiated by the last right-hand side, and their FP32 rounding
// would be amplified there like any rounding of a stage value); the state
// and the accumulator ACC stay FP64; the column solves read those and run
// in FP64 with the FP64 factors.  mb: mixed_bytes_per_node(c) * np bytes.
hipError_t launch_hevi_step_mixed_in(numa_ctx *c, double *q, double dt, char *mb, hipEvent_t *ev)
{
    static const Ark2 t;
    const long np = c->np;
    // R1 in the mixed five-field layout (32 bytes per node), E3 in FP64 (40),
    // then Q2 and Q3 rho' and w, and over a stratified background theta'
    char *const R1 = mb, *const E3 = mb + 32 * np;
    double *const Q2r = reinterpret_cast<double *>(mb + 72 * np), *const Q3r = reinterpret_cast<double *>(mb + 80 * np);
    double *const Q2w = reinterpret_cast<double *>(mb + 88 * np), *const Q3w = reinterpret_cast<double *>(mb + 96 * np);
    const bool strat = stratified(c);
    double *const Q2t = strat ? reinterpret_cast<double *>(mb + 104 * np) : nullptr;
    double *const Q3t = strat ? reinterpret_cast<double *>(mb + 112 * np) : nullptr;
    auto fld = [&](char *buf, int f) { return buf + (buf == E3 ? size_t(8) * f * np : mixed_field_offset(f, np)); };
    double *const ACC = stage_buffers(c).ACC;
    const double *qr = q + 0 * np, *qw = q + 3 * np, *qt = q + 4 * np;
    const double f = dt * t.a21;
    hipError_t e;
    auto mark = [&](int i) -> hipError_t { return ev ? hipEventRecord(ev[i], c->stream) : hipSuccess; };
    if ((e = mark(0)) != hipSuccess) return e;
    {  // K1: R1 = R(q^n)
        RhsParams p{};
        set_fields(p.a, q, np);
        p.out0 = R1;
        p.fs = np;
        e = dispatch(c->N, [&](auto n) { return rhs_launch<decltype(n)::value, EPI_R, false, true>(c, p); });
        if (e != hipSuccess || (e = mark(1)) != hipSuccess) return e;
    }
    {  // K2
        SolveParams p{};
        p.er[0] = fld(R1, 0); p.cr[0] = f;
        p.ew[0] = fld(R1, 3); p.cw[0] = f;
        p.et[0] = fld(R1, 4); p.ct[0] = f;
        p.br[0] = qr; p.cbr[0] = 1.0; p.br[1] = fld(R1, 0); p.cbr[1] = f;
        p.bw[0] = qw; p.cbw[0] = 1.0;
        p.out_r = Q2r;
        p.out_w = Q2w;
        if (strat) {
            p.bt[0] = qt; p.cbt[0] = 1.0; p.bt[1] = fld(R1, 4); p.cbt[1] = f;
            p.out_t = Q2t;
        }
        e = dispatch(c->N, [&](auto n) { return solve_launch<decltype(n)::value, ShapeStage2>(c, p); });
        if (e != hipSuccess || (e = mark(2)) != hipSuccess) return e;
    }
    {  // K3: rhs(Q2) -> E3 (FP32), ACC (FP64)
        RhsParams p{};
        p.a[0] = Q2r;
        p.a[3] = Q2w;
        p.cb = f;
        if (strat) {
            p.theta_in = 1;
            p.a[4] = Q2t;
        }
        p.out0 = E3;
        p.out1 = ACC;
        p.e0 = q;
        p.e1 = R1;
        p.fs = np;
        p.k01 = dt * t.a31; p.k02 = dt * t.a32;
        p.k11 = dt * t.b1;  p.k12 = dt * t.b2;
        e = dispatch(c->N, [&](auto n) { return rhs_launch<decltype(n)::value, EPI_TWO, true, true>(c, p); });
        if (e != hipSuccess || (e = mark(3)) != hipSuccess) return e;
    }
    {  // K4
        SolveParams p{};
        p.er[0] = fld(E3, 0); p.cr[0] = 1.0; p.er[1] = qr; p.cr[1] = t.c31; p.er[2] = Q2r; p.cr[2] = t.c32;
        p.ew[0] = fld(E3, 3); p.cw[0] = 1.0; p.ew[1] = qw; p.cw[1] = t.c31; p.ew[2] = Q2w; p.cw[2] = t.c32;
        p.et[0] = fld(E3, 4); p.ct[0] = 1.0; p.et[1] = qt; p.ct[1] = t.c31 + t.c32; p.et[2] = fld(R1, 4);
        p.ct[2] = t.c32 * f;
        p.br[0] = fld(E3, 0); p.cbr[0] = 1.0;
        p.bw[0] = qw; p.cbw[0] = -t.c31; p.bw[1] = Q2w; p.cbw[1] = -t.c32;
        p.out_r = Q3r;
        p.out_w = Q3w;
        if (strat) {
            p.ct[1] = t.c31; p.et[2] = Q2t; p.ct[2] = t.c32;
            p.bt[0] = fld(E3, 4); p.cbt[0] = 1.0;
            p.out_t = Q3t;
        }
        e = dispatch(c->N, [&](auto n) { return solve_launch<decltype(n)::value, ShapeStage3>(c, p); });
        if (e != hipSuccess || (e = mark(4)) != hipSuccess) return e;
    }
    {  // K5: q^{n+1} = ACC + dt b3 R(Q3)
        RhsParams p{};
        p.a[0] = Q3r;
        p.a[1] = fld(E3, 1);
        p.a[2] = fld(E3, 2);
        p.a[3] = Q3w;
        p.a[4] = strat ? static_cast<const void *>(Q3t) : fld(E3, 4);
        p.out0 = q;
        p.e0 = ACC;
        p.fs = np;
        p.k02 = dt * t.b3;
        e = dispatch(c->N, [&](auto n) { return rhs_launch<decltype(n)::value, EPI_FINAL, false, true>(c, p); });
        if (e != hipSuccess || (e = mark(5)) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_hevi_step_mixed(numa_ctx *c, double *q, double dt, hipEvent_t *ev)
{
    return launch_hevi_step_mixed_in(c, q, dt, c->work_mix, ev);
}

// The precision form's stage buffers for callers that cannot allocate: one
// array per GPU in the code object.  Host code never uses the array's name
// as an address (on the host it is only a stand-in for the symbol): each
// device's copy is resolved once, with that device current, and kept here.
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
char *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_init()
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (g_scratch_ptr[dev]) return hipSuccess;
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = static_cast<char *>(ptr);
    return hipSuccess;
}

char *noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    return g_scratch_ptr[device];
}

// Set the LDS attributes of every kernel one step of this context launches,
// so that a step can be captured into a graph (no first-use set-up inside).
hipError_t prepare_step(numa_ctx *c, bool mixed)
{
    return dispatch(c->N, [&](auto n) -> hipError_t {
        constexpr int NN = decltype(n)::value;
        const int zc = c->rhs_zchunk > 0 ? c->rhs_zchunk : rhs_zchunk_auto<NN>(c);
        const int nez = c->nez, nz = int(c->nz);
        hipError_t e = hipSuccess;
        if (!mixed) {
            const size_t lds = rhs_lds_bytes<NN, false>(zc, nez);
            if (nontemporal_stores(c)) {
                if (e == hipSuccess) e = rhs_prepare<NN, EPI_R, false, false, true>(lds);
                if (e == hipSuccess) e = rhs_prepare<NN, EPI_TWO, true, false, true>(lds);
                if (e == hipSuccess) e = rhs_prepare<NN, EPI_FINAL, false, false, true>(lds);
            } else {
                if (e == hipSuccess) e = rhs_prepare<NN, EPI_R, false, false>(lds);
                if (e == hipSuccess) e = rhs_prepare<NN, EPI_TWO, true, false>(lds);
                if (e == hipSuccess) e = rhs_prepare<NN, EPI_FINAL, false, false>(lds);
            }
        } else {
            const size_t lds = rhs_lds_bytes<NN, true>(zc, nez);
            if (e == hipSuccess) e = rhs_prepare<NN, EPI_R, false, true>(lds);
            if (e == hipSuccess) e = rhs_prepare<NN, EPI_TWO, true, true>(lds);
            if (e == hipSuccess) e = rhs_prepare<NN, EPI_FINAL, false, true>(lds);
        }
        // the column solves of both forms are the FP64 ones
        if (e == hipSuccess) e = solve_prepare<NN, ShapeStage2>(nz);
        if (e == hipSuccess) e = solve_prepare<NN, ShapeStage3>(nz);
        if (blocked_solve_used(c) && nz > 8 * kBlockedKL) {
            if (e == hipSuccess) e = blocked_prepare<NN, ShapeStage2, 16>(blocked_lds_bytes(NN, nz));
            if (e == hipSuccess) e = blocked_prepare<NN, ShapeStage3, 16>(blocked_lds_bytes(NN, nz));
        } else if (blocked_solve_used(c) && nz + 2 * NN > 64) {
            if (e == hipSuccess) e = blocked_prepare<NN, ShapeStage2, 8>(blocked_lds_bytes(NN, nz));
            if (e == hipSuccess) e = blocked_prepare<NN, ShapeStage3, 8>(blocked_lds_bytes(NN, nz));
        }
        return e;
    });
}

// Autotuner of the right-hand side's vertical chunk (elements per workgroup,
// i.e. the workgroup's height in the z march): times the plain right-hand
// side of state (written to the context's stage buffer R1; state is only
// read) for chunks nez, nez/2, nez/3, ... 1 and keeps the fastest in
// c->rhs_zchunk.  Synchronises the context's stream.
hipError_t autotune_rhs_zchunk(numa_ctx *c, const double *state, int reps, int *chosen)
{
    std::vector<int> cand;
    for (int d = 1; d <= c->nez; ++d) {
        const int zc = (c->nez + d - 1) / d;
        if (cand.empty() || cand.back() != zc) cand.push_back(zc);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const int keep = c->rhs_zchunk;
    float best = 0.f;
    int best_zc = keep;
    double *R = stage_buffers(c).R1;
    for (size_t i = 0; i < cand.size() && e == hipSuccess; ++i) {
        c->rhs_zchunk = cand[i];
        e = launch_rhs_plain(c, state, R);  // warm-up (and LDS attribute)
        if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_rhs_plain(c, state, R);
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && (i == 0 || ms < best)) {
            best = ms;
            best_zc = cand[i];
        }
    }
    c->rhs_zchunk = e == hipSuccess ? best_zc : keep;
    if (chosen) *chosen = c->rhs_zchunk;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return e;
}

}  // namespace numa
