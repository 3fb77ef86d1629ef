// C ABI of the HEVI library: argument validation, context lifetime, device
// memory, and the stage schedule (kernels in kernels.hip).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "numa_internal.h"

namespace {

thread_local std::string g_setup_error;

int fail(numa_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    else g_setup_error = msg;
    return code;
}

int hip_fail(numa_ctx *c, hipError_t e, const char *where)
{
    std::string m = std::string(where) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
    return fail(c, e == hipErrorOutOfMemory ? NUMA_E_NOMEM : NUMA_E_HIP, m);
}

void free_ctx(numa_ctx *c)
{
    if (!c) return;
    if (c->lev_block) (void)hipFree(c->lev_block);
    if (c->fac) (void)hipFree(c->fac);
    if (c->fac_cols) (void)hipFree(c->fac_cols);
    if (c->work) (void)hipFree(c->work);
    if (c->work_mix) (void)hipFree(c->work_mix);
    if (c->flag) (void)hipFree(c->flag);
    if (c->fac_std) (void)hipFree(c->fac_std);
    numa::learned_free(c);
    numa::imex3d_free(c);
    delete c;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }


int64_t step_bytes_model(const numa_ctx *c)
{
    // Field passes per step of the fused schedule (reads + writes of whole
    // unique-node fields): K1 5+5, K2 5+2, K3 12+10, K4 9+2, K5 10+5 = 65,
    // plus two reads of the (shared) column factors.  Over a stratified
    // background the solves also write theta' (K2 reads q^n and R1 theta'
    // for it, K3 reads it, K4 reads E3 theta' for it): 6 more.
    const int64_t fields = numa::stratified(c) ? 71 : 65;
    return fields * c->np * int64_t(sizeof(double)) + 2 * numa::factor_bytes(c);
}

}  // namespace

namespace numa {

// The checks shared by the step entry points; NUMA_OK if the step may run.
int step_preconditions(numa_ctx *c, double dt, const char *who)
{
    if (!c->factored) return fail(c, NUMA_E_NOT_FACTORED, std::string(who) + ": call numa_factor_columns first");
    if (std::memcmp(&dt, &c->dt_factored, sizeof(double)) != 0)
        return fail(c, NUMA_E_DT_MISMATCH, std::string(who) + ": dt differs from the factored dt");
    return NUMA_OK;
}

// The precision form's stage buffers, allocated on first use.
int ensure_mixed_buffers(numa_ctx *c, const char *who)
{
    if (c->work_mix) return NUMA_OK;
    hipError_t e = hipMalloc(&c->work_mix, numa::mixed_bytes_per_node(c) * size_t(c->np));
    if (e != hipSuccess) {
        c->work_mix = nullptr;
        return hip_fail(c, e, (std::string(who) + ": hipMalloc(precision-form stage buffers)").c_str());
    }
    return NUMA_OK;
}

}  // namespace numa

using numa::ensure_mixed_buffers;
using numa::step_preconditions;

extern "C" {

int numa_setup(const numa_grid *g, int32_t order, const numa_background *bg, void *hip_stream, numa_ctx **out)
{
    g_setup_error.clear();
    if (!out) return fail(nullptr, NUMA_E_ARG, "numa_setup: out is NULL");
    *out = nullptr;
    if (!g || !bg) return fail(nullptr, NUMA_E_ARG, "numa_setup: grid or background is NULL");
    if (order < 1 || order > 15) return fail(nullptr, NUMA_E_ARG, "numa_setup: order must be in 1..15");
    if (order > numa::kMaxOrder)
        return fail(nullptr, NUMA_E_UNSUPPORTED, "numa_setup: orders above 8 are not built");
    if (!finite_pos(g->lx) || !finite_pos(g->ly) || !finite_pos(g->lz))
        return fail(nullptr, NUMA_E_ARG, "numa_setup: box extents must be finite and > 0");
    if (g->nex < 1 || g->ney < 1 || g->nez < 1)
        return fail(nullptr, NUMA_E_ARG, "numa_setup: element counts must be >= 1");
    const int64_t nx = int64_t(g->nex) * order, ny = int64_t(g->ney) * order, nz = int64_t(g->nez) * order + 1;
    if (nx > (1 << 30) || ny > (1 << 30) || nx * ny > (int64_t(1) << 40))
        return fail(nullptr, NUMA_E_ARG, "numa_setup: grid too large");
    if (g->zface) {
        if (g->zface[0] != 0.0 || !(std::fabs(g->zface[g->nez] - g->lz) <= 1e-12 * g->lz))
            return fail(nullptr, NUMA_E_ARG, "numa_setup: zface must run from 0 to lz");
        for (int e = 0; e < g->nez; ++e)
            if (!(g->zface[e + 1] > g->zface[e]) || !std::isfinite(g->zface[e + 1]))
                return fail(nullptr, NUMA_E_ARG, "numa_setup: zface must be strictly increasing");
    }
    if (!finite_pos(bg->theta0) || !finite_pos(bg->p00) || !finite_pos(bg->rgas) || !finite_pos(bg->cp) ||
        !(bg->cp > bg->rgas) || !std::isfinite(bg->grav) || bg->grav < 0.0 || !std::isfinite(bg->nbv) ||
        bg->nbv < 0.0 || (bg->nbv > 0.0 && !(bg->grav > 0.0)))
        return fail(nullptr, NUMA_E_ARG, "numa_setup: invalid background constants");
    if (!(numa::exner_at(bg->theta0, bg->cp, bg->grav, bg->nbv, g->lz) > 0.0))
        return fail(nullptr, NUMA_E_ARG, "numa_setup: box top above the background atmosphere's top");
    if (numa::lds_needed(order, g->nez, int(nz)) > numa::kLdsPerCU)
        return fail(nullptr, NUMA_E_UNSUPPORTED, "numa_setup: columns too tall for one CU's LDS");
    if (nx * ny * nz * int64_t(sizeof(double)) >= (int64_t(1) << 32))
        return fail(nullptr, NUMA_E_UNSUPPORTED, "numa_setup: a field above 4 GiB is not supported");

    numa_ctx *c = new (std::nothrow) numa_ctx();
    if (!c) return fail(nullptr, NUMA_E_NOMEM, "numa_setup: host allocation failed");
    c->N = order;
    c->nex = g->nex;
    c->ney = g->ney;
    c->nez = g->nez;
    c->nx = nx;
    c->ny = ny;
    c->nz = nz;
    c->ncol = nx * ny;
    c->plane = nx * ny;
    c->np = nx * ny * nz;
    c->lx = g->lx;
    c->ly = g->ly;
    c->lz = g->lz;
    c->cp = bg->cp;
    c->eos.theta0 = bg->theta0;
    c->eos.p00 = bg->p00;
    c->eos.rgas = bg->rgas;
    c->eos.gamma = bg->cp / (bg->cp - bg->rgas);
    c->eos.grav = bg->grav;
    c->nbv = bg->nbv;
    numa::set_binomial(c->eos);
    c->stream = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipGetDevice(&c->device);
    // the fixed stage buffers of numa_hevi_step_mixed_noalloc on this device
    if (e == hipSuccess) e = numa::noalloc_scratch_init();
    if (e != hipSuccess) {
        int rc = hip_fail(nullptr, e, "numa_setup: device");
        delete c;
        return rc;
    }

    numa::build_ops(c, g->zface);

    const int N = order, ns = 2 * N + 1;
    const size_t n_lev =
        size_t(4 * nz + nz * ns + 3 * g->nez + 2 * N * ns + (N + 1) * (N + 1) + numa::SC_N * nz + 2 * nz);
    e = hipMalloc(&c->lev_block, n_lev * sizeof(double));
    if (e != hipSuccess) {
        int rc = hip_fail(nullptr, e, "numa_setup: hipMalloc(levels)");
        free_ctx(c);
        return rc;
    }
    double *p = static_cast<double *>(c->lev_block);
    c->lev.rho0 = p; p += nz;
    c->lev.P0 = p; p += nz;
    c->lev.G0 = p; p += nz;
    c->lev.H0 = p; p += nz;
    c->lev.dzb = p; p += nz * ns;
    c->lev.zsc = p; p += 3 * g->nez;
    c->lev.wxy = p; p += 2 * N * ns;
    c->lev.D = p; p += (N + 1) * (N + 1);
    c->lev.scf = p; p += numa::SC_N * nz;
    c->lev.th0 = p; p += nz;
    c->lev.th0z = p;

    // every column has the same operator (uniform horizontal grid, one set of
    // vertical faces, horizontally uniform background): one factor set
    const size_t fac_n = size_t(nz) * size_t(4 * N + 1);
    const size_t work_n = size_t(numa::kStageFields) * size_t(c->np);
    e = hipMalloc(&c->fac, fac_n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&c->work, work_n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&c->flag, sizeof(int));
    if (e != hipSuccess) {
        int rc = hip_fail(nullptr, e, "numa_setup: hipMalloc(factors/work)");
        free_ctx(c);
        return rc;
    }
    struct Up { double *dst; const std::vector<double> *src; };
    const Up ups[] = {{c->lev.rho0, &c->ops.rho0}, {c->lev.dzb, &c->ops.dzb}, {c->lev.zsc, &c->ops.zsc},
                      {c->lev.wxy, &c->ops.wxy}, {c->lev.D, &c->ops.D}, {c->lev.th0, &c->ops.th0},
                      {c->lev.th0z, &c->ops.th0z}};
    for (const Up &u : ups) {
        e = hipMemcpyAsync(u.dst, u.src->data(), u.src->size() * sizeof(double), hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) break;
    }
    if (e == hipSuccess) e = hipMemsetAsync(c->flag, 0, sizeof(int), c->stream);
    if (e == hipSuccess) e = numa::launch_background(c);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        int rc = hip_fail(nullptr, e, "numa_setup: upload");
        free_ctx(c);
        return rc;
    }
    *out = c;
    return NUMA_OK;
}

int numa_state_shape(const numa_ctx *c, int64_t shape[4])
{
    if (!c || !shape) return NUMA_E_ARG;
    shape[0] = 5;
    shape[1] = c->nz;
    shape[2] = c->ny;
    shape[3] = c->nx;
    return NUMA_OK;
}

int numa_get_info(const numa_ctx *c, numa_info *info)
{
    if (!c || !info) return NUMA_E_ARG;
    info->nx = c->nx;
    info->ny = c->ny;
    info->nz = c->nz;
    info->ncol = c->ncol;
    info->factor_bytes = numa::factor_bytes(c);
    info->scratch_bytes = numa::kStageFields * c->np * int64_t(sizeof(double));
    info->step_bytes = step_bytes_model(c);
    info->order = c->N;
    info->factored = c->factored;
    info->dt_factored = c->dt_factored;
    info->column_solver = numa::per_column_factors(c) ? NUMA_SOLVER_PER_COLUMN
                          : numa::blocked_solve_used(c) ? NUMA_SOLVER_BLOCKED
                                                        : NUMA_SOLVER_BAND;
    info->reserved = 0;
    return NUMA_OK;
}

int numa_set_stream(numa_ctx *c, void *hip_stream)
{
    if (!c) return NUMA_E_ARG;
    c->stream = static_cast<hipStream_t>(hip_stream);
    return NUMA_OK;
}

int numa_set_column_solver(numa_ctx *c, int32_t kind)
{
    if (!c) return NUMA_E_ARG;
    if (kind != NUMA_SOLVER_AUTO && kind != NUMA_SOLVER_BAND && kind != NUMA_SOLVER_BLOCKED &&
        kind != NUMA_SOLVER_PER_COLUMN)
        return fail(c, NUMA_E_ARG, "numa_set_column_solver: unknown kind");
    if (kind == NUMA_SOLVER_PER_COLUMN &&
        c->nz * (4 * c->N + 1) * c->ncol * int64_t(sizeof(double)) >= (int64_t(1) << 32))
        return fail(c, NUMA_E_UNSUPPORTED, "numa_set_column_solver: per-column factors above 4 GiB");
    if (kind == NUMA_SOLVER_BLOCKED && !numa::blocked_solve_ok(c->N, c->nz))
        return fail(c, NUMA_E_UNSUPPORTED, "numa_set_column_solver: the blocked solve needs nz <= 128, or nz <= 224 where its LDS fits one CU");
    c->column_solver = kind;
    c->factored = 0;
    return NUMA_OK;
}

int numa_autotune(numa_ctx *c, const double *state, int32_t reps, int32_t *config_out)
{
    if (!c) return NUMA_E_ARG;
    if (!state || reps < 1 || reps > 1000) return fail(c, NUMA_E_ARG, "numa_autotune: null state or reps outside 1..1000");
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = numa::autotune_rhs(c, state, reps, nullptr, nullptr);
    if (e != hipSuccess) return hip_fail(c, e, "numa_autotune");
    return config_out ? numa_get_rhs_config(c, config_out) : NUMA_OK;
}

int numa_set_rhs_config(numa_ctx *c, int32_t tile, int32_t zchunk)
{
    if (!c) return NUMA_E_ARG;
    if (tile < 0 || tile > 1 || zchunk < 0 || zchunk > c->nez)
        return fail(c, NUMA_E_ARG, "numa_set_rhs_config: tile must be 0 or 1 and zchunk in 0..nez");
    if (tile == 1) {
        const int zc = zchunk > 0 ? zchunk : 1;
        if (!numa::rhs_alt_differs(c->N) || numa::rhs_lds_alt(c->N, zc, c->nez) > numa::kLdsPerCU)
            return fail(c, NUMA_E_UNSUPPORTED, "numa_set_rhs_config: no second tile for this order or column");
    }
    c->rhs_tile = tile;
    c->rhs_zchunk = zchunk;
    return NUMA_OK;
}

int numa_get_rhs_config(const numa_ctx *c, int32_t *out)
{
    if (!c || !out) return NUMA_E_ARG;
    int tx = 0;
    const int ty = numa::rhs_tile_shape(c->N, c->rhs_tile, &tx);
    out[0] = c->rhs_tile;
    out[1] = tx;
    out[2] = ty;
    out[3] = numa::rhs_zchunk_in_use(c);
    return NUMA_OK;
}

int numa_factor_columns(numa_ctx *c, double dt)
{
    if (!c) return NUMA_E_ARG;
    if (!finite_pos(dt)) return fail(c, NUMA_E_ARG, "numa_factor_columns: dt must be finite and > 0");
    const double lambda = (1.0 - 1.0 / std::sqrt(2.0)) * dt;
    c->factored = 0;
    hipError_t e = hipSuccess;
    if (numa::per_column_factors(c) && !c->fac_cols) {
        e = hipMalloc(&c->fac_cols, size_t(numa::factor_bytes(c)));
        if (e != hipSuccess) {
            c->fac_cols = nullptr;
            return hip_fail(c, e, "numa_factor_columns: hipMalloc(per-column factors)");
        }
    }
    e = numa::launch_factor(c, lambda);
    if (e != hipSuccess) return hip_fail(c, e, "numa_factor_columns");
    c->factored = 1;
    c->dt_factored = dt;
    c->lambda = lambda;
    return NUMA_OK;
}

namespace {

using StepFn = hipError_t (*)(numa_ctx *, double *, double, hipEvent_t *);

int run_steps(numa_ctx *c, StepFn step, double *state, double dt, int32_t nsteps, const char *who)
{
    for (int32_t s = 0; s < nsteps; ++s) {
        hipError_t e = step(c, state, dt, nullptr);
        if (e != hipSuccess) return hip_fail(c, e, who);
    }
    return NUMA_OK;
}

int profile_steps(numa_ctx *c, StepFn step, double *state, double dt, int32_t nsteps, double *ms_out, const char *who)
{
    // 6 events per step around its 5 kernels
    std::vector<hipEvent_t> ev(size_t(6) * nsteps, nullptr);
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < ev.size() && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
    for (int32_t s = 0; s < nsteps && e == hipSuccess; ++s) e = step(c, state, dt, &ev[size_t(6) * s]);
    if (e == hipSuccess) e = hipEventSynchronize(ev.back());
    double acc[5] = {0, 0, 0, 0, 0};
    for (int32_t s = 0; s < nsteps && e == hipSuccess; ++s)
        for (int i = 0; i < 5 && e == hipSuccess; ++i) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, ev[size_t(6) * s + i], ev[size_t(6) * s + i + 1]);
            acc[i] += ms;
        }
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    if (e != hipSuccess) return hip_fail(c, e, who);
    for (int i = 0; i < 5; ++i) ms_out[i] = acc[i] / nsteps;
    return NUMA_OK;
}

}  // namespace

int numa_hevi_step(numa_ctx *c, double *state, double dt, int32_t nsteps)
{
    if (!c) return NUMA_E_ARG;
    if (!state || nsteps < 0) return fail(c, NUMA_E_ARG, "numa_hevi_step: null state or nsteps < 0");
    int rc = step_preconditions(c, dt, "numa_hevi_step");
    if (rc != NUMA_OK) return rc;
    return run_steps(c, numa::launch_hevi_step, state, dt, nsteps, "numa_hevi_step");
}

int numa_hevi_step_mixed(numa_ctx *c, double *state, double dt, int32_t nsteps)
{
    if (!c) return NUMA_E_ARG;
    if (!state || nsteps < 0) return fail(c, NUMA_E_ARG, "numa_hevi_step_mixed: null state or nsteps < 0");
    int rc = step_preconditions(c, dt, "numa_hevi_step_mixed");
    if (rc == NUMA_OK) rc = ensure_mixed_buffers(c, "numa_hevi_step_mixed");
    if (rc != NUMA_OK) return rc;
    return run_steps(c, numa::launch_hevi_step_mixed, state, dt, nsteps, "numa_hevi_step_mixed");
}

int numa_hevi_step_mixed_noalloc(numa_ctx *c, double *state, double dt, int32_t nsteps)
{
    if (!c) return NUMA_E_ARG;
    if (!state || nsteps < 0) return fail(c, NUMA_E_ARG, "numa_hevi_step_mixed_noalloc: null state or nsteps < 0");
    int rc = step_preconditions(c, dt, "numa_hevi_step_mixed_noalloc");
    if (rc != NUMA_OK) return rc;
    const size_t per = numa::mixed_bytes_per_node(c), need = per * size_t(c->np);
    if (need > numa::kNoAllocScratchBytes)
        return fail(c, NUMA_E_UNSUPPORTED,
                    "numa_hevi_step_mixed_noalloc: the grid needs " + std::to_string(need) + " bytes of stage buffers (" +
                        std::to_string(per) + " per unique node), above the fixed " +
                        std::to_string(numa::kNoAllocScratchBytes) + " bytes");
    char *mb = numa::noalloc_scratch(c->device);
    if (!mb)
        return fail(c, NUMA_E_HIP, "numa_hevi_step_mixed_noalloc: no fixed stage buffers on the context's device");
    for (int32_t s = 0; s < nsteps; ++s) {
        hipError_t e = numa::launch_hevi_step_mixed_in(c, state, dt, mb);
        if (e != hipSuccess) return hip_fail(c, e, "numa_hevi_step_mixed_noalloc");
    }
    return NUMA_OK;
}

int numa_profile_steps(numa_ctx *c, double *state, double dt, int32_t nsteps, double *ms_out)
{
    if (!c) return NUMA_E_ARG;
    if (!state || nsteps < 1 || nsteps > 100000 || !ms_out)
        return fail(c, NUMA_E_ARG, "numa_profile_steps: bad arguments");
    int rc = step_preconditions(c, dt, "numa_profile_steps");
    if (rc != NUMA_OK) return rc;
    return profile_steps(c, numa::launch_hevi_step, state, dt, nsteps, ms_out, "numa_profile_steps");
}

int numa_profile_steps_mixed(numa_ctx *c, double *state, double dt, int32_t nsteps, double *ms_out)
{
    if (!c) return NUMA_E_ARG;
    if (!state || nsteps < 1 || nsteps > 100000 || !ms_out)
        return fail(c, NUMA_E_ARG, "numa_profile_steps_mixed: bad arguments");
    int rc = step_preconditions(c, dt, "numa_profile_steps_mixed");
    if (rc == NUMA_OK) rc = ensure_mixed_buffers(c, "numa_profile_steps_mixed");
    if (rc != NUMA_OK) return rc;
    return profile_steps(c, numa::launch_hevi_step_mixed, state, dt, nsteps, ms_out, "numa_profile_steps_mixed");
}

int numa_rhs(numa_ctx *c, const double *state, double *rhs_out)
{
    if (!c) return NUMA_E_ARG;
    if (!state || !rhs_out) return fail(c, NUMA_E_ARG, "numa_rhs: null pointer");
    hipError_t e = numa::launch_rhs_plain(c, state, rhs_out);
    if (e != hipSuccess) return hip_fail(c, e, "numa_rhs");
    return NUMA_OK;
}

int numa_solve_columns(numa_ctx *c, const double *y, double *x)
{
    if (!c) return NUMA_E_ARG;
    if (!y || !x) return fail(c, NUMA_E_ARG, "numa_solve_columns: null pointer");
    if (!c->factored) return fail(c, NUMA_E_NOT_FACTORED, "numa_solve_columns: call numa_factor_columns first");
    hipError_t e = numa::launch_solve_plain(c, y, x);
    if (e != hipSuccess) return hip_fail(c, e, "numa_solve_columns");
    return NUMA_OK;
}

int numa_factor_columns_standard(numa_ctx *c, double dt, int64_t *bytes_out)
{
    if (!c) return NUMA_E_ARG;
    if (!finite_pos(dt)) return fail(c, NUMA_E_ARG, "numa_factor_columns_standard: dt must be finite and > 0");
    if (numa::stratified(c))
        return fail(c, NUMA_E_UNSUPPORTED, "numa_factor_columns_standard: built for the isentropic background only");
    const double lambda = (1.0 - 1.0 / std::sqrt(2.0)) * dt;
    c->std_factored = 0;
    hipError_t e = numa::launch_factor_std(c, lambda);
    if (e != hipSuccess) return hip_fail(c, e, "numa_factor_columns_standard");
    c->std_factored = 1;
    c->dt_std = dt;
    c->lambda_std = lambda;
    if (bytes_out) *bytes_out = int64_t(numa::std_factor_bytes(c));
    return NUMA_OK;
}

int numa_solve_columns_standard(numa_ctx *c, const double *y, double *x)
{
    if (!c) return NUMA_E_ARG;
    if (!y || !x) return fail(c, NUMA_E_ARG, "numa_solve_columns_standard: null pointer");
    if (!c->std_factored)
        return fail(c, NUMA_E_NOT_FACTORED, "numa_solve_columns_standard: call numa_factor_columns_standard first");
    hipError_t e = numa::launch_solve_std(c, y, x);
    if (e != hipSuccess) return hip_fail(c, e, "numa_solve_columns_standard");
    return NUMA_OK;
}

int numa_imex3d_setup(numa_ctx *c, double dt, int32_t restart, int32_t pbno_order, int32_t power_steps,
                      int32_t maxit)
{
    if (!c) return NUMA_E_ARG;
    if (numa::stratified(c))
        return fail(c, NUMA_E_UNSUPPORTED, "numa_imex3d_setup: the 3D Schur form is built for theta0 constant");
    if (!finite_pos(dt) || restart < 1 || restart > 63 || pbno_order < -1 || pbno_order > 16 || power_steps < 0 ||
        power_steps > 1000 || maxit < 1)
        return fail(c, NUMA_E_ARG, "numa_imex3d_setup: bad arguments");
    hipError_t e = numa::imex3d_setup(c, dt, restart, pbno_order, power_steps, maxit);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        numa::imex3d_free(c);
        return hip_fail(c, e, "numa_imex3d_setup");
    }
    return NUMA_OK;
}

int numa_imex3d_bounds(const numa_ctx *c, double *out)
{
    if (!c || !out || !c->imex) return NUMA_E_ARG;
    double dt;
    numa::imex3d_info(c, &dt, &out[0], &out[1]);
    return NUMA_OK;
}

int numa_imex3d_set_bounds(numa_ctx *c, double lmin, double lmax)
{
    if (!c) return NUMA_E_ARG;
    if (!c->imex) return fail(c, NUMA_E_NOT_FACTORED, "numa_imex3d_set_bounds: call numa_imex3d_setup first");
    if (!finite_pos(lmin) || !std::isfinite(lmax) || !(lmax > lmin))
        return fail(c, NUMA_E_ARG, "numa_imex3d_set_bounds: need 0 < lmin < lmax");
    numa::imex3d_set_bounds(c, lmin, lmax);
    return NUMA_OK;
}

int numa_imex3d_set_precision(numa_ctx *c, int32_t pbno_fp32)
{
    if (!c) return NUMA_E_ARG;
    if (!c->imex) return fail(c, NUMA_E_NOT_FACTORED, "numa_imex3d_set_precision: call numa_imex3d_setup first");
    if (pbno_fp32 != 0 && pbno_fp32 != 1) return fail(c, NUMA_E_ARG, "numa_imex3d_set_precision: pbno_fp32 must be 0 or 1");
    numa::imex3d_set_pbno32(c, pbno_fp32);
    return NUMA_OK;
}

namespace {

int imex3d_ready(numa_ctx *c, const char *who)
{
    if (!c->imex) return fail(c, NUMA_E_NOT_FACTORED, std::string(who) + ": call numa_imex3d_setup first");
    return NUMA_OK;
}

}  // namespace

int numa_schur_apply(numa_ctx *c, const double *P, double *out)
{
    if (!c) return NUMA_E_ARG;
    if (!P || !out || P == out) return fail(c, NUMA_E_ARG, "numa_schur_apply: null or identical pointers");
    int rc = imex3d_ready(c, "numa_schur_apply");
    if (rc != NUMA_OK) return rc;
    hipError_t e = numa::schur_apply(c, P, out);
    return e == hipSuccess ? NUMA_OK : hip_fail(c, e, "numa_schur_apply");
}

int numa_schur_rhs(numa_ctx *c, const double *y, double *b)
{
    if (!c) return NUMA_E_ARG;
    if (!y || !b) return fail(c, NUMA_E_ARG, "numa_schur_rhs: null pointer");
    int rc = imex3d_ready(c, "numa_schur_rhs");
    if (rc != NUMA_OK) return rc;
    hipError_t e = numa::schur_rhs(c, y, b);
    return e == hipSuccess ? NUMA_OK : hip_fail(c, e, "numa_schur_rhs");
}

int numa_pbno_apply(numa_ctx *c, const double *r, double *z)
{
    if (!c) return NUMA_E_ARG;
    if (!r || !z || r == z) return fail(c, NUMA_E_ARG, "numa_pbno_apply: null or identical pointers");
    int rc = imex3d_ready(c, "numa_pbno_apply");
    if (rc != NUMA_OK) return rc;
    hipError_t e = numa::pbno_apply(c, r, z);
    return e == hipSuccess ? NUMA_OK : hip_fail(c, e, "numa_pbno_apply");
}

int numa_imex3d_solve(numa_ctx *c, const double *y, double *x, double tol, int32_t *iters_out)
{
    if (iters_out) *iters_out = 0;
    if (!c) return NUMA_E_ARG;
    if (!y || !x || !(tol > 0.0) || !std::isfinite(tol)) return fail(c, NUMA_E_ARG, "numa_imex3d_solve: bad arguments");
    int rc = imex3d_ready(c, "numa_imex3d_solve");
    if (rc != NUMA_OK) return rc;
    int it = 0, conv = 0;
    hipError_t e = numa::imex3d_solve(c, y, x, nullptr, 0.0, nullptr, 0.0, tol, &it, &conv);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (iters_out) *iters_out = it;
    if (e != hipSuccess) return hip_fail(c, e, "numa_imex3d_solve");
    if (!conv) return fail(c, NUMA_E_NOT_CONVERGED, "numa_imex3d_solve: GMRES did not reach tol within maxit");
    return NUMA_OK;
}

int numa_imex3d_step(numa_ctx *c, double *state, double dt, double tol, int32_t *iters_out)
{
    if (iters_out) *iters_out = 0;
    if (!c) return NUMA_E_ARG;
    if (!state || !(tol > 0.0) || !std::isfinite(tol)) return fail(c, NUMA_E_ARG, "numa_imex3d_step: bad arguments");
    int rc = imex3d_ready(c, "numa_imex3d_step");
    if (rc != NUMA_OK) return rc;
    double dts, lmin, lmax;
    numa::imex3d_info(c, &dts, &lmin, &lmax);
    if (dt != dts) return fail(c, NUMA_E_DT_MISMATCH, "numa_imex3d_step: dt differs from the numa_imex3d_setup dt");
    int it = 0, conv = 0;
    hipError_t e = numa::imex3d_step(c, state, dt, tol, &it, &conv);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (iters_out) *iters_out = it;
    if (e != hipSuccess) return hip_fail(c, e, "numa_imex3d_step");
    if (!conv) return fail(c, NUMA_E_NOT_CONVERGED, "numa_imex3d_step: GMRES did not reach tol within maxit");
    return NUMA_OK;
}

namespace {

int learned_ready(numa_ctx *c, const char *who)
{
    if (!c->learned) return fail(c, NUMA_E_NOT_FACTORED, std::string(who) + ": call numa_learned_setup first");
    return NUMA_OK;
}

}  // namespace

int numa_learned_setup(numa_ctx *c, int32_t hidden, int64_t max_samples, uint64_t seed)
{
    if (!c) return NUMA_E_ARG;
    if (hidden < 1 || hidden > 1024 || max_samples < 1) return fail(c, NUMA_E_ARG, "numa_learned_setup: bad arguments");
    int rc = imex3d_ready(c, "numa_learned_setup");
    if (rc != NUMA_OK) return rc;
    hipError_t e = numa::learned_setup(c, hidden, long(max_samples), seed);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        numa::learned_free(c);
        return hip_fail(c, e, "numa_learned_setup");
    }
    return NUMA_OK;
}

int numa_learned_info(const numa_ctx *c, int64_t *info)
{
    if (!c || !info || !c->learned) return NUMA_E_ARG;
    const numa::LearnedInfo L = numa::learned_info(c);
    info[0] = L.nparam;
    info[1] = L.nin;
    info[2] = L.nh;
    info[3] = L.nsamp;
    info[4] = L.cap;
    info[5] = L.enabled;
    return NUMA_OK;
}

int numa_learned_add_samples(numa_ctx *c, const double *r, double tol, int32_t *iters_out)
{
    if (iters_out) *iters_out = 0;
    if (!c) return NUMA_E_ARG;
    if (!r || !(tol > 0.0)) return fail(c, NUMA_E_ARG, "numa_learned_add_samples: bad arguments");
    int rc = learned_ready(c, "numa_learned_add_samples");
    if (rc != NUMA_OK) return rc;
    const numa::LearnedInfo L = numa::learned_info(c);
    if (L.nsamp + L.nelem > L.cap) return fail(c, NUMA_E_ARG, "numa_learned_add_samples: sample capacity reached");
    int it = 0, conv = 0;
    hipError_t e = numa::learned_add_samples(c, r, tol, &it, &conv);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (iters_out) *iters_out = it;
    if (e != hipSuccess) return hip_fail(c, e, "numa_learned_add_samples");
    if (!conv) return fail(c, NUMA_E_NOT_CONVERGED, "numa_learned_add_samples: the sample solve did not converge");
    return NUMA_OK;
}

int numa_learned_samples(numa_ctx *c, int64_t first, int64_t n, float *X, float *T)
{
    if (!c) return NUMA_E_ARG;
    int rc = learned_ready(c, "numa_learned_samples");
    if (rc != NUMA_OK) return rc;
    const numa::LearnedInfo L = numa::learned_info(c);
    if (first < 0 || n < 1 || first + n > L.nsamp || !X || !T)
        return fail(c, NUMA_E_ARG, "numa_learned_samples: bad range or null pointer");
    const size_t bytes = sizeof(float) * size_t(n) * L.nin;
    hipError_t e = hipMemcpyAsync(X, L.X + first * L.nin, bytes, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(T, L.T + first * L.nin, bytes, hipMemcpyDeviceToDevice, c->stream);
    return e == hipSuccess ? NUMA_OK : hip_fail(c, e, "numa_learned_samples");
}

int numa_learned_params(numa_ctx *c, float *theta_out, const float *theta_in)
{
    if (!c) return NUMA_E_ARG;
    int rc = learned_ready(c, "numa_learned_params");
    if (rc != NUMA_OK) return rc;
    const numa::LearnedInfo L = numa::learned_info(c);
    const size_t bytes = sizeof(float) * size_t(L.nparam);
    hipError_t e = hipSuccess;
    if (theta_in) e = hipMemcpyAsync(L.theta, theta_in, bytes, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && theta_out) e = hipMemcpyAsync(theta_out, L.theta, bytes, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? NUMA_OK : hip_fail(c, e, "numa_learned_params");
}

int numa_learned_loss_grad(numa_ctx *c, const float *X, const float *T, int64_t n, float *grad_out, double *loss_out)
{
    if (!c) return NUMA_E_ARG;
    int rc = learned_ready(c, "numa_learned_loss_grad");
    if (rc != NUMA_OK) return rc;
    const numa::LearnedInfo L = numa::learned_info(c);
    if (!X || !T || !grad_out || !loss_out || n < 1 || n > std::max(L.cap, L.nelem))
        return fail(c, NUMA_E_ARG, "numa_learned_loss_grad: bad arguments");
    hipError_t e = numa::learned_loss_grad(c, X, T, long(n), loss_out);
    if (e == hipSuccess)
        e = hipMemcpyAsync(grad_out, L.grad, sizeof(float) * size_t(L.nparam), hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? NUMA_OK : hip_fail(c, e, "numa_learned_loss_grad");
}

int numa_learned_train(numa_ctx *c, int32_t steps, int32_t batch, double lr, uint64_t seed, double *loss_first,
                       double *loss_last)
{
    if (!c) return NUMA_E_ARG;
    if (steps < 1 || batch < 1 || !(lr > 0.0)) return fail(c, NUMA_E_ARG, "numa_learned_train: bad arguments");
    int rc = learned_ready(c, "numa_learned_train");
    if (rc != NUMA_OK) return rc;
    const numa::LearnedInfo L = numa::learned_info(c);
    if (L.nsamp < 1) return fail(c, NUMA_E_ARG, "numa_learned_train: no samples");
    if (batch > std::max(L.cap, L.nelem)) return fail(c, NUMA_E_ARG, "numa_learned_train: batch too large");
    double lf = 0.0, ll = 0.0;
    hipError_t e = numa::learned_train(c, steps, batch, lr, seed, &lf, &ll);
    if (loss_first) *loss_first = lf;
    if (loss_last) *loss_last = steps == 1 ? lf : ll;
    return e == hipSuccess ? NUMA_OK : hip_fail(c, e, "numa_learned_train");
}

int numa_learned_enable(numa_ctx *c, int32_t on)
{
    if (!c) return NUMA_E_ARG;
    int rc = learned_ready(c, "numa_learned_enable");
    if (rc != NUMA_OK) return rc;
    numa::learned_set_enabled(c, on);
    return NUMA_OK;
}

// PBNO judges the network: the flexible solve with it must reach tol in
// fewer GMRES iterations than the polynomial alone on the same system.
int numa_learned_judge(numa_ctx *c, const double *y, double *x, double tol, int32_t *out)
{
    if (!c) return NUMA_E_ARG;
    if (!y || !x || !out || y == x || !(tol > 0.0) || !std::isfinite(tol))
        return fail(c, NUMA_E_ARG, "numa_learned_judge: bad arguments");
    int rc = imex3d_ready(c, "numa_learned_judge");
    if (rc != NUMA_OK) return rc;
    if ((rc = learned_ready(c, "numa_learned_judge")) != NUMA_OK) return rc;
    out[0] = out[1] = out[2] = 0;
    int it_net = 0, conv_net = 0, it_pb = 0, conv_pb = 0;
    numa::learned_set_enabled(c, 1);
    hipError_t e = numa::imex3d_solve(c, y, x, nullptr, 0.0, nullptr, 0.0, tol, &it_net, &conv_net);
    numa::learned_set_enabled(c, 0);
    if (e == hipSuccess) e = numa::imex3d_solve(c, y, x, nullptr, 0.0, nullptr, 0.0, tol, &it_pb, &conv_pb);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "numa_learned_judge");
    if (!conv_pb) return fail(c, NUMA_E_NOT_CONVERGED, "numa_learned_judge: the polynomial solve did not converge");
    const int accepted = conv_net && it_net < it_pb;
    numa::learned_set_enabled(c, accepted);
    out[0] = it_pb;
    out[1] = it_net;
    out[2] = accepted;
    return NUMA_OK;
}

int numa_learned_apply(numa_ctx *c, const double *r, double *z)
{
    if (!c) return NUMA_E_ARG;
    if (!r || !z || r == z) return fail(c, NUMA_E_ARG, "numa_learned_apply: null or identical pointers");
    int rc = learned_ready(c, "numa_learned_apply");
    if (rc != NUMA_OK) return rc;
    hipError_t e = numa::pbno_apply(c, r, z);
    if (e == hipSuccess) e = numa::learned_correction_add(c, r, z, nullptr);
    return e == hipSuccess ? NUMA_OK : hip_fail(c, e, "numa_learned_apply");
}

int numa_lgl_basis(int32_t order, double *xi, double *D)
{
    if (order < 1 || order > 15 || !xi || !D) return NUMA_E_ARG;
    std::vector<double> x, d;
    numa::lgl_nodes(order, x);
    numa::lgl_dmat(order, x, d);
    std::memcpy(xi, x.data(), x.size() * sizeof(double));
    std::memcpy(D, d.data(), d.size() * sizeof(double));
    return NUMA_OK;
}

int numa_line_operators(const numa_grid *g, int32_t order, double *wxy, double *dzb)
{
    if (!g || !wxy || !dzb || order < 1 || order > 15) return NUMA_E_ARG;
    if (!finite_pos(g->lx) || !finite_pos(g->ly) || !finite_pos(g->lz) || g->nex < 1 || g->ney < 1 || g->nez < 1)
        return NUMA_E_ARG;
    if (g->zface) {
        if (g->zface[0] != 0.0 || !(std::fabs(g->zface[g->nez] - g->lz) <= 1e-12 * g->lz)) return NUMA_E_ARG;
        for (int e = 0; e < g->nez; ++e)
            if (!(g->zface[e + 1] > g->zface[e])) return NUMA_E_ARG;
    }
    numa_ctx c;
    c.N = order;
    c.nex = g->nex;
    c.ney = g->ney;
    c.nez = g->nez;
    c.nx = int64_t(g->nex) * order;
    c.ny = int64_t(g->ney) * order;
    c.nz = int64_t(g->nez) * order + 1;
    c.lx = g->lx;
    c.ly = g->ly;
    c.lz = g->lz;
    c.cp = 1004.67;  // background is not used by the operators; any valid constants
    c.eos = {300.0, 1.0e5, 287.17, 1.4, 0.0, {}};
    numa::build_ops(&c, g->zface);
    std::memcpy(wxy, c.ops.wxy.data(), c.ops.wxy.size() * sizeof(double));
    std::memcpy(dzb, c.ops.dzb.data(), c.ops.dzb.size() * sizeof(double));
    return NUMA_OK;
}

int numa_check(numa_ctx *c)
{
    if (!c) return NUMA_E_ARG;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "numa_check: synchronize");
    int flag = 0;
    e = hipMemcpy(&flag, c->flag, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(c, e, "numa_check: read flag");
    if (flag) {
        e = hipMemset(c->flag, 0, sizeof(int));
        if (e != hipSuccess) return hip_fail(c, e, "numa_check: clear flag");
        return fail(c, NUMA_E_NONFINITE, "numa_check: a step or factorisation produced NaN/Inf");
    }
    return NUMA_OK;
}

int numa_destroy(numa_ctx *c)
{
    if (!c) return NUMA_OK;
    (void)hipStreamSynchronize(c->stream);
    free_ctx(c);
    return NUMA_OK;
}

const char *numa_last_error(const numa_ctx *c)
{
    if (!c) return g_setup_error.c_str();
    return c->err.c_str();
}

}  // extern "C"
