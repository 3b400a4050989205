// C ABI of librbm.so (declared in include/rbm.h): argument checks, workspace
// plan, context bookkeeping and the launch sequence of each call.  No device
// memory is allocated here; every buffer lives in the caller's workspace.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>
#include <string>

#include "../../include/rbm.h"
#include "rbm_plan.hpp"

using rbm::Plan;
using rbm::StepArgs;

static_assert(rbm::RBM_NPH == RBM_NPHASES, "phase count of the kernels and the header differ");

struct rbm_ctx {
    rbm_params prm;
    Plan plan;
    void *ws;
    int64_t m;  // index of the next step
    bool pending;  // stored positions lack the noise of step m - 1
    // per-phase timing (measurement aid)
    hipEvent_t *ev;   // tmax * (RBM_NPHASES + 1) events
    int32_t tmax;     // steps the pool can record
    int32_t trec;     // steps recorded so far
};

namespace {

thread_local std::string g_err;

rbm_status fail(rbm_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
rbm_status fail(rbm_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

rbm_status hip_fail(hipError_t e, const char *what)
{
    return fail(RBM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t align256(size_t x)
{
    return (x + 255) & ~(size_t)255;
}

rbm_status check_params(const rbm_params *prm)
{
    if (!prm) return fail(RBM_ERR_INVALID, "params is NULL");
    if (prm->d < 1 || prm->d > 3) return fail(RBM_ERR_INVALID, "d = %d not in 1..3", prm->d);
    if (prm->kernel < RBM_K_GAUSS || prm->kernel > RBM_K_ATTREP)
        return fail(RBM_ERR_INVALID, "unknown kernel %d", prm->kernel);
    if (prm->n < 2) return fail(RBM_ERR_INVALID, "N = %lld < 2", (long long)prm->n);
    if (prm->n > RBM_MAX_N)
        return fail(RBM_ERR_UNSUPPORTED, "N = %lld above the supported %lld", (long long)prm->n,
                    (long long)RBM_MAX_N);
    if (prm->p < 2 || (int64_t)prm->p > prm->n)
        return fail(RBM_ERR_INVALID, "p = %d not in 2..N", prm->p);
    if (prm->reserved != 0 || prm->reserved2 != 0)
        return fail(RBM_ERR_INVALID, "reserved fields must be 0");
    if (!(prm->dt > 0.0) || !std::isfinite(prm->dt)) return fail(RBM_ERR_INVALID, "dt must be > 0");
    if (!(prm->sigma >= 0.0) || !std::isfinite(prm->sigma))
        return fail(RBM_ERR_INVALID, "sigma must be >= 0");
    if (!(prm->kparam >= 0.0) || !std::isfinite(prm->kparam))
        return fail(RBM_ERR_INVALID, "kparam must be >= 0");
    if (!std::isfinite(prm->beta)) return fail(RBM_ERR_INVALID, "beta must be finite");
    if (prm->n > RBM_SINGLE_CAP && prm->p > RBM_MAX_P_MULTI)
        return fail(RBM_ERR_UNSUPPORTED, "p = %d above %d needs N <= %d", prm->p, RBM_MAX_P_MULTI,
                    RBM_SINGLE_CAP);
    return RBM_OK;
}

Plan make_plan(const rbm_params *prm)
{
    Plan pl{};
    pl.n = (uint32_t)prm->n;
    pl.p = (uint32_t)prm->p;
    pl.nbat = pl.n / pl.p;
    pl.d = prm->d;
    pl.kernel = prm->kernel;
    pl.rec_bytes = (size_t)4 * (prm->d + 1);
    if (pl.n <= RBM_SINGLE_CAP) {
        pl.nbuck = pl.nb1 = 1;
    } else {
        const uint32_t target = (pl.n + RBM_BUCKET_MEAN - 1) / RBM_BUCKET_MEAN;
        const uint32_t per = 1u << RBM_SPLIT_SHIFT;
        if (target <= per) {
            pl.shift = 0;
            pl.nb1 = pl.nbuck = target;
        } else {
            pl.shift = RBM_SPLIT_SHIFT;
            pl.nb1 = (target + per - 1) / per;
            pl.nbuck = pl.nb1 * per;
            // chunks per coarse bucket: room for the mean plus 16 standard deviations
            const double mean = (double)pl.n / pl.nb1;
            pl.jmax = (uint32_t)std::ceil((mean + 16.0 * std::sqrt(mean) + 64.0) / RBM_CHUNK);
        }
        pl.ntiles = (pl.n + RBM_TILE - 1) / RBM_TILE;
        // about 128 key-count tiles, a multiple of 4 slots each
        uint32_t tf = (pl.n + 127) / 128;
        tf = (tf + 4095) & ~4095u;
        pl.tilef = tf < 16384 ? 16384 : tf;
        pl.ntf = (pl.n + pl.tilef - 1) / pl.tilef;
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    const size_t recs = (size_t)pl.n * pl.rec_bytes;
    pl.off_state = take(recs);
    pl.off_scratch = take(recs);
    if (pl.nbuck > 1) {
        pl.off_stage1 = take(recs);
        pl.off_w1 = take((size_t)pl.n * 4);
        if (pl.shift > 0) {
            pl.off_stage2 = take(recs);
            pl.off_w2 = take((size_t)pl.n * 4);
        }
        pl.off_kcnt = take((size_t)pl.ntf * pl.nbuck * 4);
        pl.off_ftot = take((size_t)pl.nbuck * 4);
        pl.off_fstart = take((size_t)(pl.nbuck + 1) * 4);
        pl.off_fcur = take((size_t)pl.nbuck * 4);
        pl.off_cstart = take((size_t)(pl.nb1 + 1) * 4);
        pl.off_ccur = take((size_t)pl.nb1 * 4);
    }
    pl.off_flags = take(256);
    pl.total = off;
    return pl;
}

// pending: the stored positions lack the noise of step m - 1.
StepArgs make_args(const rbm_params *prm, const Plan &pl, uint32_t m, bool pending)
{
    StepArgs s{};
    s.n = pl.n;
    s.p = pl.p;
    s.nbat = pl.nbat;
    s.m = m;
    s.k0 = (uint32_t)(prm->seed & 0xffffffffu);
    s.k1 = (uint32_t)(prm->seed >> 32);
    s.sys = prm->sys;
    s.nbuck = pl.nbuck;
    s.inv_p1 = (float)(1.0 / (double)(pl.p - 1));
    s.inv_last = (float)(1.0 / (double)(pl.p + pl.n % pl.p - 1));
    s.a = (float)prm->kparam;
    s.beta = (float)prm->beta;
    s.dt = (float)prm->dt;
    s.ssd = (float)(prm->sigma * std::sqrt(prm->dt));
    s.pm = m - 1u;
    s.pssd = pending ? s.ssd : 0.0f;
    return s;
}

rbm_status check_ctx(const rbm_ctx *ctx)
{
    if (!ctx) return fail(RBM_ERR_INVALID, "context is NULL");
    return RBM_OK;
}

}  // namespace

extern "C" {

const char *rbm_status_str(rbm_status st)
{
    switch (st) {
    case RBM_OK: return "ok";
    case RBM_ERR_INVALID: return "invalid argument";
    case RBM_ERR_WORKSPACE: return "workspace too small or misaligned";
    case RBM_ERR_HIP: return "HIP runtime error";
    case RBM_ERR_UNSUPPORTED: return "unsupported configuration";
    case RBM_ERR_DEVICE: return "device-side check failed";
    }
    return "unknown status";
}

const char *rbm_last_error(void)
{
    return g_err.c_str();
}

rbm_status rbm_workspace_size(const rbm_params *prm, size_t *bytes)
{
    rbm_status st = check_params(prm);
    if (st != RBM_OK) return st;
    if (!bytes) return fail(RBM_ERR_INVALID, "bytes is NULL");
    *bytes = make_plan(prm).total;
    return RBM_OK;
}

rbm_status rbm_init(const rbm_params *prm, const float *d_x0, const uint32_t *d_slots,
                    int64_t step0, void *d_ws, size_t ws_bytes, void *stream, rbm_ctx **out)
{
    rbm_status st = check_params(prm);
    if (st != RBM_OK) return st;
    if (!d_x0 || !d_ws || !out) return fail(RBM_ERR_INVALID, "NULL pointer argument");
    if (step0 < 0 || step0 > 0xffffffffLL) return fail(RBM_ERR_INVALID, "step0 out of range");
    const Plan pl = make_plan(prm);
    if (ws_bytes < pl.total)
        return fail(RBM_ERR_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, pl.total);
    if (((uintptr_t)d_ws & 255u) != 0) return fail(RBM_ERR_WORKSPACE, "workspace not 256-byte aligned");
    rbm_ctx *ctx = (rbm_ctx *)calloc(1, sizeof(rbm_ctx));
    if (!ctx) return fail(RBM_ERR_INVALID, "out of host memory");
    ctx->prm = *prm;
    ctx->plan = pl;
    ctx->ws = d_ws;
    ctx->m = step0;
    hipError_t e = rbm::launch_init(pl, prm->d, d_x0, d_slots, d_ws, (hipStream_t)stream);
    if (e != hipSuccess) {
        free(ctx);
        return hip_fail(e, "rbm_init launch");
    }
    *out = ctx;
    return RBM_OK;
}

rbm_status rbm_step(rbm_ctx *ctx, void *stream)
{
    return rbm_run(ctx, 1, stream);
}

rbm_status rbm_run(rbm_ctx *ctx, int64_t nsteps, void *stream)
{
    rbm_status st = check_ctx(ctx);
    if (st != RBM_OK) return st;
    if (nsteps < 0) return fail(RBM_ERR_INVALID, "nsteps < 0");
    if (ctx->m + nsteps > 0x100000000LL) return fail(RBM_ERR_INVALID, "step index would pass 2^32");
    const Plan &pl = ctx->plan;
    void *state = (char *)ctx->ws + pl.off_state;
    for (int64_t k = 0; k < nsteps; ++k) {
        const StepArgs s = make_args(&ctx->prm, pl, (uint32_t)ctx->m, ctx->pending);
        hipEvent_t *ev = nullptr;
        if (ctx->trec < ctx->tmax) ev = ctx->ev + (size_t)ctx->trec++ * (RBM_NPHASES + 1);
        hipError_t e = rbm::launch_step(pl, s, pl.d, pl.kernel, ctx->ws, (hipStream_t)stream, state,
                                        nullptr, ev);
        if (e != hipSuccess) return hip_fail(e, "rbm_step launch");
        ctx->m += 1;
        ctx->pending = s.ssd != 0.0f;
    }
    return RBM_OK;
}

rbm_status rbm_positions(rbm_ctx *ctx, float *d_x, void *stream)
{
    rbm_status st = check_ctx(ctx);
    if (st != RBM_OK) return st;
    if (!d_x) return fail(RBM_ERR_INVALID, "d_x is NULL");
    const StepArgs s = make_args(&ctx->prm, ctx->plan, (uint32_t)ctx->m, ctx->pending);
    hipError_t e = rbm::launch_positions(ctx->plan, s, ctx->plan.d, ctx->ws, d_x, nullptr,
                                         (hipStream_t)stream);
    return e == hipSuccess ? RBM_OK : hip_fail(e, "rbm_positions launch");
}

rbm_status rbm_perm(rbm_ctx *ctx, uint32_t *d_ids, void *stream)
{
    rbm_status st = check_ctx(ctx);
    if (st != RBM_OK) return st;
    if (!d_ids) return fail(RBM_ERR_INVALID, "d_ids is NULL");
    const StepArgs s = make_args(&ctx->prm, ctx->plan, (uint32_t)ctx->m, ctx->pending);
    hipError_t e = rbm::launch_positions(ctx->plan, s, ctx->plan.d, ctx->ws, nullptr, d_ids,
                                         (hipStream_t)stream);
    return e == hipSuccess ? RBM_OK : hip_fail(e, "rbm_perm launch");
}

rbm_status rbm_forces(rbm_ctx *ctx, int64_t step, float *d_f, void *stream)
{
    rbm_status st = check_ctx(ctx);
    if (st != RBM_OK) return st;
    if (!d_f) return fail(RBM_ERR_INVALID, "d_f is NULL");
    if (step < 0 || step > 0xffffffffLL) return fail(RBM_ERR_INVALID, "step out of range");
    const Plan &pl = ctx->plan;
    StepArgs s = make_args(&ctx->prm, pl, (uint32_t)step, false);
    s.pm = (uint32_t)(ctx->m - 1);
    s.pssd = ctx->pending ? s.ssd : 0.0f;
    void *scratch = (char *)ctx->ws + pl.off_scratch;
    hipError_t e = rbm::launch_step(pl, s, pl.d, pl.kernel, ctx->ws, (hipStream_t)stream, scratch, d_f,
                                    nullptr);
    return e == hipSuccess ? RBM_OK : hip_fail(e, "rbm_forces launch");
}

rbm_status rbm_step_index(const rbm_ctx *ctx, int64_t *m)
{
    rbm_status st = check_ctx(ctx);
    if (st != RBM_OK) return st;
    if (!m) return fail(RBM_ERR_INVALID, "m is NULL");
    *m = ctx->m;
    return RBM_OK;
}

rbm_status rbm_check(rbm_ctx *ctx, void *stream)
{
    rbm_status st = check_ctx(ctx);
    if (st != RBM_OK) return st;
    uint32_t flags = 0;
    hipError_t e = hipMemcpyAsync(&flags, (char *)ctx->ws + ctx->plan.off_flags, sizeof flags,
                                  hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "rbm_check");
    if (flags & 1u) return fail(RBM_ERR_DEVICE, "a bucket exceeded its capacity");
    if (flags & 2u) return fail(RBM_ERR_DEVICE, "rbm_init: a slot id was >= N");
    return RBM_OK;
}

static void release_events(rbm_ctx *ctx)
{
    for (int64_t i = 0; i < (int64_t)ctx->tmax * (RBM_NPHASES + 1); ++i) (void)hipEventDestroy(ctx->ev[i]);
    free(ctx->ev);
    ctx->ev = nullptr;
    ctx->tmax = ctx->trec = 0;
}

rbm_status rbm_timing(rbm_ctx *ctx, int32_t max_steps)
{
    rbm_status st = check_ctx(ctx);
    if (st != RBM_OK) return st;
    if (max_steps < 0 || max_steps > 100000) return fail(RBM_ERR_INVALID, "max_steps out of range");
    if (ctx->ev) {
        hipError_t e = hipEventSynchronize(ctx->ev[(size_t)ctx->tmax * (RBM_NPHASES + 1) - 1]);
        (void)e;
        (void)hipDeviceSynchronize();
        release_events(ctx);
    }
    if (max_steps == 0) return RBM_OK;
    const size_t nev = (size_t)max_steps * (RBM_NPHASES + 1);
    ctx->ev = (hipEvent_t *)calloc(nev, sizeof(hipEvent_t));
    if (!ctx->ev) return fail(RBM_ERR_INVALID, "out of host memory");
    for (size_t i = 0; i < nev; ++i) {
        hipError_t e = hipEventCreate(&ctx->ev[i]);
        if (e != hipSuccess) {
            ctx->tmax = (int32_t)(i / (RBM_NPHASES + 1));
            for (size_t j = (size_t)ctx->tmax * (RBM_NPHASES + 1); j < i; ++j) (void)hipEventDestroy(ctx->ev[j]);
            release_events(ctx);
            return hip_fail(e, "hipEventCreate");
        }
    }
    ctx->tmax = max_steps;
    ctx->trec = 0;
    return RBM_OK;
}

rbm_status rbm_phase_times(rbm_ctx *ctx, double *ms, int64_t *steps)
{
    rbm_status st = check_ctx(ctx);
    if (st != RBM_OK) return st;
    if (!ms || !steps) return fail(RBM_ERR_INVALID, "NULL pointer argument");
    for (int i = 0; i < RBM_NPHASES; ++i) ms[i] = 0.0;
    *steps = ctx->trec;
    if (ctx->trec == 0) return RBM_OK;
    const int K = RBM_NPHASES + 1;
    hipError_t e = hipEventSynchronize(ctx->ev[(size_t)(ctx->trec - 1) * K + K - 1]);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    for (int32_t s = 0; s < ctx->trec; ++s) {
        for (int i = 0; i < RBM_NPHASES; ++i) {
            float t = 0.0f;
            e = hipEventElapsedTime(&t, ctx->ev[(size_t)s * K + i], ctx->ev[(size_t)s * K + i + 1]);
            if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
            ms[i] += t;
        }
    }
    for (int i = 0; i < RBM_NPHASES; ++i) ms[i] /= (double)ctx->trec;
    ctx->trec = 0;
    return RBM_OK;
}

rbm_status rbm_destroy(rbm_ctx *ctx)
{
    if (!ctx) return RBM_OK;
    if (ctx->ev) release_events(ctx);
    free(ctx);
    return RBM_OK;
}

rbm_status direct_forces(const rbm_params *prm, const float *d_x, const uint32_t *d_ids,
                         int64_t nids, float *d_f, void *stream)
{
    rbm_status st = check_params(prm);
    if (st == RBM_ERR_UNSUPPORTED && prm && prm->n <= RBM_MAX_N) st = RBM_OK;  // p is not used
    if (st != RBM_OK) return st;
    if (!d_x || !d_f) return fail(RBM_ERR_INVALID, "NULL pointer argument");
    if (d_ids == nullptr) nids = prm->n;
    if (nids < 0 || nids > prm->n) return fail(RBM_ERR_INVALID, "nids out of range");
    if (nids == 0) return RBM_OK;
    const Plan pl = make_plan(prm);
    const StepArgs s = make_args(prm, pl, 0, false);
    hipError_t e = rbm::launch_direct(s, prm->d, prm->kernel, d_x, d_ids, (uint32_t)nids, d_f, 0,
                                      (hipStream_t)stream);
    return e == hipSuccess ? RBM_OK : hip_fail(e, "direct_forces launch");
}

rbm_status direct_step(const rbm_params *prm, const float *d_x, float *d_x_out, int64_t step,
                       void *stream)
{
    rbm_status st = check_params(prm);
    if (st == RBM_ERR_UNSUPPORTED && prm && prm->n <= RBM_MAX_N) st = RBM_OK;
    if (st != RBM_OK) return st;
    if (!d_x || !d_x_out) return fail(RBM_ERR_INVALID, "NULL pointer argument");
    if (d_x == d_x_out) return fail(RBM_ERR_INVALID, "d_x_out must not alias d_x");
    if (step < 0 || step > 0xffffffffLL) return fail(RBM_ERR_INVALID, "step out of range");
    const Plan pl = make_plan(prm);
    const StepArgs s = make_args(prm, pl, (uint32_t)step, false);
    hipError_t e = rbm::launch_direct(s, prm->d, prm->kernel, d_x, nullptr, (uint32_t)prm->n,
                                      d_x_out, 1, (hipStream_t)stream);
    return e == hipSuccess ? RBM_OK : hip_fail(e, "direct_step launch");
}

}  // extern "C"
