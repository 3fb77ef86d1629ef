// Internal declarations of the HEVI library: the context, the host set-up
// (LGL basis, DSS line operators, background) and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/numa.h"

namespace numa {

constexpr int kMaxOrder = 8;

// Host-side operators of one context (built by setup.cpp).
struct HostOps {
    int N = 0;
    std::vector<double> xi;     // LGL nodes, N+1
    std::vector<double> D;      // differentiation matrix, (N+1)^2, D[i*(N+1)+j]
    std::vector<double> wxy;    // [2][N][2N+1] x and y DSS stencils, metric included
    std::vector<double> zsc;    // [3][nez]: 2/h_e, bottom-interface and top-interface factors
    std::vector<double> dzb;    // [nz][2N+1] column DSS derivative band (offsets -N..N)
    std::vector<double> zk;     // level heights, nz
    std::vector<double> rho0;   // nz
    std::vector<double> th0;    // theta0 per level, nz
    std::vector<double> th0z;   // d theta0/dz per level, nz
};

// Exner function of the hydrostatic background at height z: d pi0/dz =
// -g/(cp theta0(z)), pi0(0) = 1, with theta0(z) = theta0 exp(nbv^2 z/g)
// (theta0 constant for nbv = 0), in closed form.
double exner_at(double theta0, double cp, double grav, double nbv, double z);

// per-level coefficients of the column solve, [nz][SC_N]: G0, H0, rho0;
// w_a = AI w_e + WA theta_e; LG = lambda G0; w~ = w_a - (X1 Dz P + X2 P);
// the stratified terms HZ = lambda H0 d theta0/dz (Schur right-hand side and
// matrix) and TZ = lambda d theta0/dz (theta' extraction)
enum { SC_G0 = 0, SC_H0, SC_RHO0, SC_WA, SC_LG, SC_X1, SC_X2, SC_AI, SC_HZ, SC_TZ, SC_N = 12 };

// Per-level background on the device (P0, G0, H0 are evaluated on the device
// with the same equation-of-state code as the right-hand side, so that the
// rest state gives P' = 0 exactly).
struct DevLevels {
    double *rho0 = nullptr, *P0 = nullptr, *G0 = nullptr, *H0 = nullptr;
    double *dzb = nullptr, *zsc = nullptr, *wxy = nullptr, *D = nullptr;
    double *scf = nullptr;  // [nz][SC_N] column-solve coefficients at the factored lambda
    double *th0 = nullptr, *th0z = nullptr;  // theta0 and d theta0/dz per level
};

// Binomial series (1 + x)^gamma - 1 = sum_k C(gamma, k) x^k, used for the
// perturbation pressure when |x| <= kBinomMaxX: for gamma of dry air the first
// omitted term is below 1e-18 of the sum.
constexpr int kBinomTerms = 10;
constexpr double kBinomMaxX = 1.0 / 32.0;

struct Imex3d;   // 3D-IMEX solver state (imex3d.hip)
struct Learned;  // learned preconditioner correction (learned.hip)

struct EOS {
    double theta0, p00, rgas, gamma, grav;
    double binom[kBinomTerms];  // C(gamma, k), k = 1..kBinomTerms
};

void set_binomial(EOS &e);

}  // namespace numa

struct numa_ctx {
    int N = 0, nex = 0, ney = 0, nez = 0;
    int64_t nx = 0, ny = 0, nz = 0, ncol = 0, plane = 0, np = 0;
    double lx = 0, ly = 0, lz = 0;
    numa::EOS eos{};
    double cp = 0;
    double nbv = 0;                // background Brunt-Vaisala frequency (0: isentropic)
    hipStream_t stream = nullptr;
    int device = 0;                // the device current at numa_setup
    numa::HostOps ops;
    numa::DevLevels lev;
    void *lev_block = nullptr;     // one allocation holding all of lev
    double *fac = nullptr;         // [nz][4N+1] column LU factors, one set shared by all columns
    double *fac_cols = nullptr;    // per-column layout [nz][4N+1][ncol] (NUMA_SOLVER_PER_COLUMN)
    int column_solver = 0;         // NUMA_SOLVER_*: 0 auto, 1 one lane per column, 2 level-blocked,
                                   // 3 one lane per column with per-column factors
    double *work = nullptr;        // stage buffers (19 fields)
    char *work_mix = nullptr;      // precision form: R1 (FP32), E3, Q2, Q3 rho' and w (FP64)
    int *flag = nullptr;           // device non-finite flag
    int factored = 0;
    double dt_factored = 0, lambda = 0;
    int rhs_zchunk = 0;            // z elements per RHS workgroup (0 = auto)
    int rhs_tile = 0;              // RHS tile variant (0 default, 1 the alternative)
    numa::Imex3d *imex = nullptr;  // 3D-IMEX solver (numa_imex3d_setup)
    numa::Learned *learned = nullptr;  // learned correction (numa_learned_setup)
    double *fac_std = nullptr;     // standard-form column factors [2 nz][4N+3], shared by all columns
    int std_factored = 0;
    double dt_std = 0, lambda_std = 0;
    std::string err;
};

namespace numa {

// setup.cpp
void lgl_nodes(int N, std::vector<double> &xi);
void lgl_dmat(int N, const std::vector<double> &xi, std::vector<double> &D);
void build_ops(numa_ctx *c, const double *zface);

// kernels.hip: launchers return hipSuccess or the launch error.
struct StageBuffers {
    double *R1, *Q2r, *Q2w, *E3, *ACC, *Q3r, *Q3w;  // R1/E3/ACC: 5 fields each
    double *Q2t, *Q3t;                              // theta' of Q2, Q3 (stratified background)
};
constexpr int kStageFields = 21;  // fields of the stage buffers (c->work)

// a background with a buoyancy frequency: the column solves change theta'
inline bool stratified(const numa_ctx *c) { return c->nbv > 0.0; }
// the column solves read every column's own factors (per-column layout)
inline bool per_column_factors(const numa_ctx *c) { return c->column_solver == NUMA_SOLVER_PER_COLUMN; }
// device bytes of the factors the column solves read
inline int64_t factor_bytes(const numa_ctx *c)
{
    const int64_t band = c->nz * (4 * c->N + 1) * int64_t(sizeof(double));
    return per_column_factors(c) ? band * c->ncol : band;
}
StageBuffers stage_buffers(numa_ctx *c);

// LDS per CU on gfx950, and what one workgroup of the kernels needs
constexpr size_t kLdsPerCU = 160 * 1024;
size_t lds_needed(int N, int nez, int nz);

hipError_t launch_background(numa_ctx *c);
hipError_t launch_factor(numa_ctx *c, double lambda);
// the level-blocked column solve: supported for this order and column height
bool blocked_solve_ok(int N, int64_t nz);
// whether the column solves use it (the context's choice, else by height)
bool blocked_solve_used(const numa_ctx *c);
hipError_t launch_rhs_plain(numa_ctx *c, const double *q, double *R);
hipError_t launch_solve_plain(numa_ctx *c, const double *y, double *x);
hipError_t launch_rhs_two(numa_ctx *c, const double *Q, const double *e0, const double *e1, double *out0,
                          double *out1, double k01, double k02, double k11, double k12);
hipError_t launch_rhs_final(numa_ctx *c, const double *Q, const double *e0, double *out, double k);
hipError_t launch_hevi_step(numa_ctx *c, double *q, double dt, hipEvent_t *ev = nullptr);
// the precision form's stage buffers: bytes per unique node (R1 in a 24-byte
// slot, E3 40, Q2 and Q3 rho' and w 32; 16 more over a stratified
// background, for theta' of Q2 and Q3)
constexpr size_t kMixedBytesPerNode = 96;
inline size_t mixed_bytes_per_node(const numa_ctx *c) { return kMixedBytesPerNode + (stratified(c) ? 16 : 0); }
hipError_t launch_hevi_step_mixed(numa_ctx *c, double *q, double dt, hipEvent_t *ev = nullptr);
// the same with the stage buffers at mb (kMixedBytesPerNode * np bytes)
hipError_t launch_hevi_step_mixed_in(numa_ctx *c, double *q, double dt, char *mb, hipEvent_t *ev = nullptr);
// Fixed stage-buffer memory of the precision form for callers that cannot
// allocate: a device array in the library's code object, one copy per GPU,
// kept until the process ends.  noalloc_scratch_init resolves the current
// device's copy (once per device); noalloc_scratch returns it (nullptr if
// that device was never initialised).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
hipError_t noalloc_scratch_init();
char *noalloc_scratch(int device);
hipError_t prepare_step(numa_ctx *c, bool mixed);
// times the step's right-hand sides for every tile variant and vertical
// chunk on state (read only) and keeps the fastest; synchronises
hipError_t autotune_rhs(numa_ctx *c, const double *state, int reps, int *zchunk_out, int *tile_out);
// TX of tile variant (0, 1) of order N into *tx; returns TY
int rhs_tile_shape(int N, int variant, int *tx);
// the vertical chunk the step's right-hand sides use (both forms): the set
// one, else the automatic
int rhs_zchunk_in_use(const numa_ctx *c);
// whether tile variant 1 differs from 0 for order N, and its LDS
bool rhs_alt_differs(int N);
size_t rhs_lds_alt(int N, int zc, int nez);
// abi.cpp: NUMA_OK or the error code (message recorded in the context)
int ensure_mixed_buffers(numa_ctx *c, const char *who);
int step_preconditions(numa_ctx *c, double dt, const char *who);

// imex3d.hip: the 3D-IMEX Schur-complement GMRES solver
hipError_t imex3d_setup(numa_ctx *c, double dt, int restart, int order, int power_steps, int maxit);
void imex3d_free(numa_ctx *c);
void imex3d_set_bounds(numa_ctx *c, double lmin, double lmax);
void imex3d_set_pbno32(numa_ctx *c, int on);
void imex3d_info(const numa_ctx *c, double *dt, double *lmin, double *lmax);
hipError_t schur_apply(numa_ctx *c, const double *P, double *out);
hipError_t schur_rhs(numa_ctx *c, const double *y, double *b);
hipError_t pbno_apply(numa_ctx *c, const double *r, double *z);
hipError_t imex3d_solve(numa_ctx *c, const double *y, double *out, const double *in0, double d0, const double *in1,
                        double d1, double tol, int *iters, int *converged);
hipError_t imex3d_step(numa_ctx *c, double *q, double dt, double tol, int *iters, int *converged);
hipError_t schur_solve_field(numa_ctx *c, const double *r, double *e_out, double tol, int *iters, int *converged);

// colstd.hip: the standard-form column solve (comparison point)
size_t std_factor_bytes(const numa_ctx *c);
hipError_t launch_factor_std(numa_ctx *c, double lambda);
hipError_t launch_solve_std(numa_ctx *c, const double *y, double *x);

// learned.hip: the learned correction of the preconditioner
bool learned_enabled(const numa_ctx *c);
void learned_free(numa_ctx *c);
hipError_t learned_setup(numa_ctx *c, int nh, long cap, uint64_t seed);
hipError_t learned_correction_add(numa_ctx *c, const double *r, double *z, const int *stop);
hipError_t learned_add_samples(numa_ctx *c, const double *r, double tol, int *iters, int *converged);
hipError_t learned_loss_grad(numa_ctx *c, const float *X, const float *T, long n, double *loss);
hipError_t learned_train(numa_ctx *c, int steps, int batch, double lr, uint64_t seed, double *loss_first,
                         double *loss_last);
struct LearnedInfo {
    long nparam, nsamp, cap, nelem;
    int nin, nh, enabled;
    float *theta, *grad, *X, *T;
};
LearnedInfo learned_info(const numa_ctx *c);
void learned_set_enabled(numa_ctx *c, int on);

}  // namespace numa
