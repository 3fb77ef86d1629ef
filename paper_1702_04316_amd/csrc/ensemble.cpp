// Batched ensemble of HEVI domains: one step of every domain captured into a
// single HIP graph, each domain's five-kernel chain on its own branch, so
// that domains too small to fill the GPU run side by side and the step costs
// one graph launch.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "numa_internal.h"

struct numa_ensemble {
    std::vector<numa_ctx *> ctx;
    std::vector<double *> state;
    std::vector<double> dt;
    std::vector<int> zchunk;
    int mixed = 0;
    hipStream_t origin = nullptr;
    std::vector<hipStream_t> branch;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::string err;
};

namespace {

thread_local std::string g_ens_error;

int efail(numa_ensemble *e, int code, const std::string &msg)
{
    (e ? e->err : g_ens_error) = msg;
    return code;
}

int ehip(numa_ensemble *e, hipError_t h, const char *where)
{
    return efail(e, h == hipErrorOutOfMemory ? NUMA_E_NOMEM : NUMA_E_HIP,
                 std::string(where) + ": " + hipGetErrorName(h) + " (" + hipGetErrorString(h) + ")");
}

void release(numa_ensemble *e)
{
    if (!e) return;
    if (e->exec) (void)hipGraphExecDestroy(e->exec);
    if (e->graph) (void)hipGraphDestroy(e->graph);
    for (hipEvent_t x : e->join)
        if (x) (void)hipEventDestroy(x);
    if (e->fork) (void)hipEventDestroy(e->fork);
    for (hipStream_t s : e->branch)
        if (s) (void)hipStreamDestroy(s);
    delete e;
}

// Capture one step of every domain: fork from the origin stream, one branch
// per domain (the context's stream is pointed at its branch meanwhile),
// join back.  No allocation, memset or first-use set-up happens inside.
hipError_t capture(numa_ensemble *e)
{
    hipError_t h = hipStreamBeginCapture(e->origin, hipStreamCaptureModeThreadLocal);
    if (h != hipSuccess) return h;
    hipError_t first = hipEventRecord(e->fork, e->origin);
    for (size_t i = 0; i < e->ctx.size() && first == hipSuccess; ++i) {
        numa_ctx *c = e->ctx[i];
        hipStream_t keep = c->stream;
        c->stream = e->branch[i];
        first = hipStreamWaitEvent(e->branch[i], e->fork, 0);
        if (first == hipSuccess)
            first = e->mixed ? numa::launch_hevi_step_mixed(c, e->state[i], e->dt[i])
                             : numa::launch_hevi_step(c, e->state[i], e->dt[i]);
        if (first == hipSuccess) first = hipEventRecord(e->join[i], e->branch[i]);
        if (first == hipSuccess) first = hipStreamWaitEvent(e->origin, e->join[i], 0);
        c->stream = keep;
    }
    h = hipStreamEndCapture(e->origin, &e->graph);  // always end the capture
    if (first != hipSuccess) return first;
    if (h != hipSuccess) return h;
    return hipGraphInstantiate(&e->exec, e->graph, nullptr, nullptr, 0);
}

}  // namespace

extern "C" {

int numa_ensemble_create(numa_ctx *const *ctxs, double *const *states, const double *dts, int32_t n, int32_t mixed,
                         int32_t tune, void *hip_stream, numa_ensemble **out)
{
    g_ens_error.clear();
    if (!out) return efail(nullptr, NUMA_E_ARG, "numa_ensemble_create: out is NULL");
    *out = nullptr;
    if (!ctxs || !states || !dts || n < 1 || n > 1024)
        return efail(nullptr, NUMA_E_ARG, "numa_ensemble_create: null arrays or n outside 1..1024");
    for (int32_t i = 0; i < n; ++i) {
        if (!ctxs[i] || !states[i]) return efail(nullptr, NUMA_E_ARG, "numa_ensemble_create: null context or state");
        for (int32_t j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i] || states[j] == states[i])
                return efail(nullptr, NUMA_E_ARG, "numa_ensemble_create: contexts and states must be distinct");
        int rc = numa::step_preconditions(ctxs[i], dts[i], "numa_ensemble_create");
        if (rc != NUMA_OK) return efail(nullptr, rc, ctxs[i]->err);
        if (mixed) {
            rc = numa::ensure_mixed_buffers(ctxs[i], "numa_ensemble_create");
            if (rc != NUMA_OK) return efail(nullptr, rc, ctxs[i]->err);
        }
    }
    numa_ensemble *e = new (std::nothrow) numa_ensemble();
    if (!e) return efail(nullptr, NUMA_E_NOMEM, "numa_ensemble_create: host allocation failed");
    e->ctx.assign(ctxs, ctxs + n);
    e->state.assign(states, states + n);
    e->dt.assign(dts, dts + n);
    e->zchunk.assign(size_t(n), 0);
    e->mixed = mixed ? 1 : 0;
    e->origin = static_cast<hipStream_t>(hip_stream);
    e->branch.assign(size_t(n), nullptr);
    e->join.assign(size_t(n), nullptr);
    hipError_t h = hipSuccess;
    // the origin must be a stream that can be captured: make one if none given
    if (!e->origin) {
        h = hipStreamCreateWithFlags(&e->origin, hipStreamNonBlocking);
        if (h == hipSuccess) e->branch.push_back(e->origin);  // destroyed with the branches
    }
    for (int32_t i = 0; i < n && h == hipSuccess; ++i) h = hipStreamCreateWithFlags(&e->branch[i], hipStreamNonBlocking);
    if (h == hipSuccess) h = hipEventCreateWithFlags(&e->fork, hipEventDisableTiming);
    for (int32_t i = 0; i < n && h == hipSuccess; ++i) h = hipEventCreateWithFlags(&e->join[i], hipEventDisableTiming);
    // every domain's pending work (set-up, factors) done before tuning and capture
    for (int32_t i = 0; i < n && h == hipSuccess; ++i) h = hipStreamSynchronize(ctxs[i]->stream);
    for (int32_t i = 0; i < n && h == hipSuccess; ++i) {
        if (tune) h = numa::autotune_rhs(ctxs[i], states[i], 3, &e->zchunk[i], nullptr);
        if (h == hipSuccess) h = numa::prepare_step(ctxs[i], e->mixed != 0);
        if (h == hipSuccess) h = hipStreamSynchronize(ctxs[i]->stream);
        if (!tune) e->zchunk[i] = ctxs[i]->rhs_zchunk;
    }
    if (h == hipSuccess) h = capture(e);
    if (h != hipSuccess) {
        int rc = ehip(nullptr, h, "numa_ensemble_create");
        release(e);
        return rc;
    }
    *out = e;
    return NUMA_OK;
}

int numa_ensemble_step(numa_ensemble *e, int32_t nsteps)
{
    if (!e) return NUMA_E_ARG;
    if (nsteps < 0) return efail(e, NUMA_E_ARG, "numa_ensemble_step: nsteps < 0");
    for (int32_t s = 0; s < nsteps; ++s) {
        hipError_t h = hipGraphLaunch(e->exec, e->origin);
        if (h != hipSuccess) return ehip(e, h, "numa_ensemble_step");
    }
    return NUMA_OK;
}

int numa_ensemble_sync(numa_ensemble *e)
{
    if (!e) return NUMA_E_ARG;
    hipError_t h = hipStreamSynchronize(e->origin);
    if (h != hipSuccess) return ehip(e, h, "numa_ensemble_sync");
    for (numa_ctx *c : e->ctx) {
        int rc = numa_check(c);
        if (rc != NUMA_OK) return efail(e, rc, "numa_ensemble_sync: " + c->err);
    }
    return NUMA_OK;
}

int numa_ensemble_zchunks(const numa_ensemble *e, int32_t *zchunk)
{
    if (!e || !zchunk) return NUMA_E_ARG;
    for (size_t i = 0; i < e->zchunk.size(); ++i) zchunk[i] = e->zchunk[i];
    return NUMA_OK;
}

int numa_ensemble_destroy(numa_ensemble *e)
{
    if (!e) return NUMA_OK;
    (void)hipStreamSynchronize(e->origin);
    release(e);
    return NUMA_OK;
}

const char *numa_ensemble_last_error(const numa_ensemble *e)
{
    return e ? e->err.c_str() : g_ens_error.c_str();
}

}  // extern "C"
