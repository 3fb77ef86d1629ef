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
#include "rhs_kernel.h"

namespace numa {

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
// (NBR, NBW, NBT) output terms; F32: which fields are FP32 (bit 0+t er[t],
// 3+t ew[t], 6+t et[t], 9+t br[t], 11+t bw[t], 13 out_w, 14 out_r, 15+t
// bt[t]), the rest FP64
template <int NR_, int NW_, int NT_, int NBR_, int NBW_, int NBT_, unsigned F32_ = 0>
struct SolveShape {
    static constexpr int NR = NR_, NW = NW_, NT = NT_, NBR = NBR_, NBW = NBW_, NBT = NBT_;
    static constexpr unsigned F32 = F32_;
};
using ShapePlain = SolveShape<1, 1, 1, 1, 0, 1>;
using ShapeStage2 = SolveShape<1, 1, 1, 2, 1, 2>;
using ShapeStage3 = SolveShape<3, 3, 3, 1, 2, 1>;
// the precision form's solves: R1 (FP32) in er[0], ew[0], et[0], br[1] and
// bt[1] of stage 2, and (over the isentropic background) in et[2] of stage 3
using ShapeStage2R = SolveShape<1, 1, 1, 2, 1, 2, (1u << 0) | (1u << 3) | (1u << 6) | (1u << 10) | (1u << 16)>;
using ShapeStage3R = SolveShape<3, 3, 3, 1, 2, 1, (1u << 8)>;
// element type of field bit b of a shape
template <class SH, int B>
using SolveT = std::conditional_t<((SH::F32 >> B) & 1u) != 0, float, double>;
// term t of the theta' output (t is a constant after unrolling)
template <class SH>
__device__ __forceinline__ double bt_load(const SolveParams &p, int t, unsigned off)
{
    return t == 0 ? tload<SolveT<SH, 15>>(p.bt[0], off) : tload<SolveT<SH, 16>>(p.bt[1], off);
}

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

// FL: where the factor band comes from: 0, the band shared by all columns
// through scalar loads; 1, the shared band staged in LDS; 2, each column's
// own band, [level][diagonal][column] in global memory (the per-column
// layout)
template <int N, class SH, int FL>
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
    if constexpr (FL == 1) {
        for (int e = lane; e < M * NB; e += 64) facl[e] = p.fac[e];
        __syncthreads();
    }
    auto fac = [&](int idx) -> double {
        if constexpr (FL == 1) return facl[idx];
        else if constexpr (FL == 2) return gload(p.fac, unsigned(idx) * lbytes + cbyte);
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
                        for (int t = 0; t < SH::NBT; ++t) th += p.cbt[t] * bt_load<SH>(p, t, off);
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
                    for (int t = 0; t < SH::NBT; ++t) xt[b][t] = bt_load<SH>(p, t, off);
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

// The per-column layout of the factors (Sec. 5.4: every column's LU stored
// for reuse): each lane assembles and factors its own column's band, the
// same matrix and the same elimination as k_factor, in place in
// F[(row * NB + offset) * ncol + col] (consecutive lanes, consecutive
// columns).
template <int N>
__global__ __launch_bounds__(64) void k_factor_cols(const double *__restrict__ dzb, const double *__restrict__ scf,
                                                    int M, long ncol, double *F, int *flag)
{
    constexpr int NS = 2 * N + 1, NB = 4 * N + 1, HB = 2 * N;
    const long col = (long)blockIdx.x * 64 + threadIdx.x;
    if (col >= ncol) return;
    auto A = [&](int r, int cidx) -> double & { return F[(size_t(r) * NB + size_t(cidx - r + HB)) * size_t(ncol) + col]; };
    for (int r = 0; r < M; ++r)
        for (int j = 0; j < NB; ++j) {
            const int cidx = r + j - HB;
            double v = 0.0;
            if (cidx >= 0 && cidx < M) {
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
            F[(size_t(r) * NB + j) * size_t(ncol) + col] = v;
        }
    bool bad = false;
    for (int k = 0; k < M; ++k) {
        const double piv = A(k, k);
        const double rp = 1.0 / piv;
        const int last = min(k + HB, M - 1);
        for (int i = k + 1; i <= last; ++i) {
            const double l = A(i, k) * rp;
            for (int jj = k + 1; jj <= last; ++jj) A(i, jj) -= l * A(k, jj);
            A(i, k) = l;
        }
        bad |= !(fabs(piv) > 0.0) || !isfinite(piv);
        A(k, k) = rp;  // the solve multiplies by the reciprocal pivot
    }
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

template <int N, class SH, int FL>
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
    return G::fac_in_lds(M) ? solve_prepare_fl<N, SH, 1>(G::lds_total(M))
                            : solve_prepare_fl<N, SH, 0>(G::lds_total(M));
}

// k_rhs with the context's tile variant: the second variant serves the
// three right-hand sides of a step; other launches use the first.  MS: a
// launch of the precision-form step, whose first two right-hand sides have
// R1 in FP32 and whose last is the FP64 step's.
template <int N, int EPI, bool HASB, bool MS = false>
hipError_t rhs_launch(numa_ctx *c, RhsParams p)
{
    constexpr bool MIX = MS && EPI != EPI_FINAL;
    const bool step_kernel = (EPI == EPI_TWO) == HASB;
    if (step_kernel && c->rhs_tile == 1) return rhs_launch_alt(c, p, EPI, MIX);
    return rhs_launch_t<N, 0, EPI, HASB, MIX>(c, p);
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
    dim3 grid(unsigned((c->ncol + 63) / 64));
    if (per_column_factors(c)) {  // each column's own band from global memory
        p.fac = c->fac_cols;
        const size_t shm = G::lds_bytes(M);
        hipError_t e = solve_prepare_fl<N, SH, 2>(shm);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_colsolve<N, SH, 2>), grid, dim3(64), shm, c->stream, p);
        return hipGetLastError();
    }
    const size_t shm = G::lds_total(M);
    hipError_t e = solve_prepare<N, SH>(M);
    if (e != hipSuccess) return e;
    if (G::fac_in_lds(M))
        hipLaunchKernelGGL((k_colsolve<N, SH, 1>), grid, dim3(64), shm, c->stream, p);
    else
        hipLaunchKernelGGL((k_colsolve<N, SH, 0>), grid, dim3(64), shm, c->stream, p);
    return hipGetLastError();
}

template <int N>
hipError_t factor_launch(numa_ctx *c, double lambda)
{
    if (per_column_factors(c)) {
        hipLaunchKernelGGL((k_factor_cols<N>), dim3(unsigned((c->ncol + 63) / 64)), dim3(64), 0, c->stream,
                           c->lev.dzb, c->lev.scf, int(c->nz), c->ncol, c->fac_cols, c->flag);
        return hipGetLastError();
    }
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
    if (c->column_solver == NUMA_SOLVER_BAND || c->column_solver == NUMA_SOLVER_PER_COLUMN) return false;
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

// The precision form of the step (same stage algebra and arithmetic as
// launch_hevi_step): the first-stage tendency R1 is stored in FP32, five
// fields of 4 bytes per node, written once and read by the next three
// kernels; every stage value (Q2, Q3, E3), the accumulator ACC and the
// state stay FP64, and so do the right-hand sides' LDS ring and arithmetic
// and the column solves with their factors.  mb: mixed_bytes_per_node(c) *
// np bytes.
hipError_t launch_hevi_step_mixed_in(numa_ctx *c, double *q, double dt, char *mb, hipEvent_t *ev)
{
    static const Ark2 t;
    const long np = c->np;
    // R1 (FP32, 20 bytes per node in a 24-byte slot, so that the FP64
    // buffers after it stay 8-byte aligned), E3 in FP64 (40), then Q2 and Q3
    // rho' and w, and over a stratified background theta'
    char *const R1 = mb, *const E3 = mb + 24 * np;
    double *const Q2r = reinterpret_cast<double *>(mb + 64 * np), *const Q3r = reinterpret_cast<double *>(mb + 72 * np);
    double *const Q2w = reinterpret_cast<double *>(mb + 80 * np), *const Q3w = reinterpret_cast<double *>(mb + 88 * np);
    const bool strat = stratified(c);
    double *const Q2t = strat ? reinterpret_cast<double *>(mb + 96 * np) : nullptr;
    double *const Q3t = strat ? reinterpret_cast<double *>(mb + 104 * np) : nullptr;
    auto fld = [&](char *buf, int f) { return buf + size_t(buf == E3 ? 8 : 4) * f * np; };
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
        e = dispatch(c->N, [&](auto n) { return solve_launch<decltype(n)::value, ShapeStage2R>(c, p); });
        if (e != hipSuccess || (e = mark(2)) != hipSuccess) return e;
    }
    {  // K3: rhs(Q2) -> E3, ACC
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
        // over a stratified background et[2] is Q2's theta' (FP64), else R1's
        e = dispatch(c->N, [&](auto n) {
            return strat ? solve_launch<decltype(n)::value, ShapeStage3>(c, p)
                         : solve_launch<decltype(n)::value, ShapeStage3R>(c, p);
        });
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
        // the FP64 step's last right-hand side
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
        const int nz = int(c->nz);
        hipError_t e;
        if (c->rhs_tile == 1) {
            const int zc = c->rhs_zchunk > 0 ? c->rhs_zchunk : rhs_zchunk_auto<NN, 1>(c);
            e = rhs_prepare_alt(c, zc, mixed);
        } else {
            const int zc = c->rhs_zchunk > 0 ? c->rhs_zchunk : rhs_zchunk_auto<NN, 0>(c);
            e = mixed ? rhs_prepare_step<NN, 0, true>(c, zc) : rhs_prepare_step<NN, 0, false>(c, zc);
        }
        // the column solves: the FP64 step's shapes, or the precision form's
        // (its stage-3 solve over a stratified background is the FP64 one)
        auto solves = [&](auto s2, auto s3) -> hipError_t {
            using S2 = decltype(s2);
            using S3 = decltype(s3);
            hipError_t h = solve_prepare<NN, S2>(nz);
            if (h == hipSuccess) h = solve_prepare<NN, S3>(nz);
            if (per_column_factors(c)) {
                if (h == hipSuccess) h = solve_prepare_fl<NN, S2, 2>(SolveGeom<NN, S2>::lds_bytes(nz));
                if (h == hipSuccess) h = solve_prepare_fl<NN, S3, 2>(SolveGeom<NN, S3>::lds_bytes(nz));
            }
            if (blocked_solve_used(c) && nz > 8 * kBlockedKL) {
                if (h == hipSuccess) h = blocked_prepare<NN, S2, 16>(blocked_lds_bytes(NN, nz));
                if (h == hipSuccess) h = blocked_prepare<NN, S3, 16>(blocked_lds_bytes(NN, nz));
            } else if (blocked_solve_used(c) && nz + 2 * NN > 64) {
                if (h == hipSuccess) h = blocked_prepare<NN, S2, 8>(blocked_lds_bytes(NN, nz));
                if (h == hipSuccess) h = blocked_prepare<NN, S3, 8>(blocked_lds_bytes(NN, nz));
            }
            return h;
        };
        if (e == hipSuccess) {
            if (!mixed) e = solves(ShapeStage2{}, ShapeStage3{});
            else if (stratified(c)) e = solves(ShapeStage2R{}, ShapeStage3{});
            else e = solves(ShapeStage2R{}, ShapeStage3R{});
        }
        return e;
    });
}

int rhs_zchunk_in_use(const numa_ctx *c)
{
    int zc = 0;
    (void)dispatch(c->N, [&](auto n) -> hipError_t {
        constexpr int NN = decltype(n)::value;
        zc = c->rhs_tile == 1 ? rhs_zchunk_auto<NN, 1>(c) : rhs_zchunk_auto<NN, 0>(c);
        return hipSuccess;
    });
    return zc;
}

int rhs_tile_shape(int N, int variant, int *tx)
{
    int ty = 0;
    (void)dispatch(N, [&](auto n) -> hipError_t {
        constexpr int NN = decltype(n)::value;
        *tx = variant == 1 ? Tile<NN, 1>::TX : Tile<NN, 0>::TX;
        ty = variant == 1 ? Tile<NN, 1>::TY : Tile<NN, 0>::TY;
        return hipSuccess;
    });
    return ty;
}

// The three right-hand sides of a step, timed on state without changing it:
// R(state) into R1; the stage-2 form reading state and R1 into E3 and ACC;
// the final form reading state and ACC into E3 (outputs are scratch).
static hipError_t launch_rhs_set(numa_ctx *c, const double *state)
{
    StageBuffers s = stage_buffers(c);
    const long np = c->np;
    hipError_t e = launch_rhs_plain(c, state, s.R1);
    if (e != hipSuccess) return e;
    e = dispatch(c->N, [&](auto n) {
        RhsParams p{};
        p.a[0] = state;
        p.a[3] = state + 3 * np;
        p.cb = 0.5;
        p.out0 = s.E3;
        p.out1 = s.ACC;
        p.e0 = state;
        p.e1 = s.R1;
        p.fs = np;
        p.k01 = p.k02 = p.k11 = p.k12 = 0.5;
        return rhs_launch<decltype(n)::value, EPI_TWO, true>(c, p);
    });
    if (e != hipSuccess) return e;
    return launch_rhs_final(c, state, s.ACC, s.E3, 0.5);
}

// Autotuner of the right-hand sides: for each tile variant that differs
// from the first and fits one CU's LDS, and each vertical chunk (elements
// per workgroup in the z march: nez, nez/2, nez/3, ... 1), times the three
// right-hand sides of a step on state (read only; outputs into the stage
// buffers) and keeps the fastest pair in c->rhs_tile and c->rhs_zchunk.
// Synchronises the context's stream.
hipError_t autotune_rhs(numa_ctx *c, const double *state, int reps, int *zchunk_out, int *tile_out)
{
    std::vector<int> chunks;
    for (int d = 1; d <= c->nez; ++d) {
        const int zc = (c->nez + d - 1) / d;
        if (chunks.empty() || chunks.back() != zc) chunks.push_back(zc);
    }
    std::vector<int> tiles = {0};
    if (rhs_alt_differs(c->N)) tiles.push_back(1);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const int keep_zc = c->rhs_zchunk, keep_tile = c->rhs_tile;
    float best = 0.f;
    int best_zc = keep_zc, best_tile = keep_tile;
    bool any = false;
    for (int tile : tiles) {
        for (size_t i = 0; i < chunks.size() && e == hipSuccess; ++i) {
            if (tile == 1 && rhs_lds_alt(c->N, chunks[i], c->nez) > kLdsPerCU) continue;
            c->rhs_tile = tile;
            c->rhs_zchunk = chunks[i];
            e = launch_rhs_set(c, state);  // warm-up (and LDS attributes)
            if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
            for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_rhs_set(c, state);
            if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && (!any || ms < best)) {
                any = true;
                best = ms;
                best_zc = chunks[i];
                best_tile = tile;
            }
        }
    }
    c->rhs_zchunk = e == hipSuccess ? best_zc : keep_zc;
    c->rhs_tile = e == hipSuccess ? best_tile : keep_tile;
    if (zchunk_out) *zchunk_out = c->rhs_zchunk;
    if (tile_out) *tile_out = c->rhs_tile;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return e;
}

}  // namespace numa
