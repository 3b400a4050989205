// C ABI of librbm.so (declared in include/rbm.h): argument checks, workspace
// plan, context bookkeeping and the launch sequence of each call.  No device
// memory is allocated here; every buffer lives in the caller's workspace.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>
#include <mutex>
#include <string>

#include "../../include/rbm.h"
#include <algorithm>
#include <numeric>
#include <vector>

#include "rbm_cv.hpp"
#include "rbm_ensemble.hpp"
#include "rbm_plan.hpp"
#include "rbm_rbmr.hpp"

using rbm::Plan;
using rbm::StepArgs;

static_assert(rbm::RBM_NPH == RBM_NPHASES, "phase count of the kernels and the header differ");

struct rbm_ctx {
    rbm_params prm;
    Plan plan;
    void *ws;
    int64_t m;  // index of the next step
    bool pending;  // stored positions lack the noise of step m - 1
    int64_t cv_t;  // Adam steps taken (the pair streams count them)
    // per-phase timing (measurement aid)
    hipEvent_t *ev;   // tmax * (RBM_NPHASES + 1) events
    int32_t tmax;     // steps the pool can record
    int32_t trec;     // steps recorded so far
    // fused runs: the key passes of the next group of steps run on a second
    // stream (default priority) while the current group's steps run
    hipStream_t ks;
    hipEvent_t ev_go, ev_keys;
    bool side;
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
    if (prm->kernel < RBM_K_GAUSS || prm->kernel > RBM_K_HAMILTON)
        return fail(RBM_ERR_INVALID, "unknown kernel %d", prm->kernel);
    if (prm->kernel == RBM_K_HAMILTON && (prm->d != 2 || prm->sigma != 0.0 || !(prm->kparam > 0.0)))
        return fail(RBM_ERR_INVALID, "the Hamiltonian system needs d = 2 records (x, u), sigma = 0 and a > 0");
    if (prm->kernel == RBM_K_WEALTH_SPLIT && !(prm->kparam > 0.0))
        return fail(RBM_ERR_INVALID, "the wealth model needs a trading rate kparam > 0");
    if (prm->kernel == RBM_K_COULOMB_SPLIT && prm->kparam != 0.0)
        return fail(RBM_ERR_INVALID, "the split Coulomb kernel has no softening (kparam must be 0)");
    if (prm->n < 2) return fail(RBM_ERR_INVALID, "N = %lld < 2", (long long)prm->n);
    if (prm->n > RBM_MAX_N)
        return fail(RBM_ERR_UNSUPPORTED, "N = %lld above the supported %lld", (long long)prm->n,
                    (long long)RBM_MAX_N);
    if (prm->p < 2 || (int64_t)prm->p > prm->n)
        return fail(RBM_ERR_INVALID, "p = %d not in 2..N", prm->p);
    if (prm->reserved != 0) return fail(RBM_ERR_INVALID, "reserved field must be 0");
    if (prm->cv != 0 && prm->cv != 1) return fail(RBM_ERR_INVALID, "cv must be 0 or 1");
    if (prm->cv && (prm->d != 2 || prm->kernel != RBM_K_GAUSS || prm->p > RBM_MAX_P_CV))
        return fail(RBM_ERR_UNSUPPORTED, "the control variate needs d = 2, the Gaussian kernel and p <= %d",
                    RBM_MAX_P_CV);
    if (!(prm->dt > 0.0) || !std::isfinite(prm->dt)) return fail(RBM_ERR_INVALID, "dt must be > 0");
    if (!(prm->sigma >= 0.0) || !std::isfinite(prm->sigma))
        return fail(RBM_ERR_INVALID, "sigma must be >= 0");
    if (!(prm->kparam >= 0.0) || !std::isfinite(prm->kparam))
        return fail(RBM_ERR_INVALID, "kparam must be >= 0");
    if (!std::isfinite(prm->beta)) return fail(RBM_ERR_INVALID, "beta must be finite");
    if ((prm->kernel == RBM_K_COULOMB_SPLIT || prm->kernel == RBM_K_WEALTH_SPLIT) &&
        (prm->p != 2 || prm->n % 2 != 0))
        return fail(RBM_ERR_UNSUPPORTED, "the exact pair flow needs p = 2 and an even N");
    if (prm->n > RBM_SINGLE_CAP && prm->p > RBM_MAX_P_MULTI)
        return fail(RBM_ERR_UNSUPPORTED, "p = %d above %d needs N <= %d", prm->p, RBM_MAX_P_MULTI,
                    RBM_SINGLE_CAP);
    return RBM_OK;
}

// The force kernel of the kernels: the split Coulomb kernel evaluates its
// forces (rbm_forces, the direct sum) as x/|x|^2, the soft Coulomb kernel
// with a = 0, the wealth model as -a x; their steps differ by
// StepArgs.scheme.
int kern_of(int kernel)
{
    if (kernel == RBM_K_COULOMB_SPLIT) return rbm::K_SOFTCOULOMB;
    if (kernel == RBM_K_WEALTH_SPLIT) return rbm::K_LINEAR;
    if (kernel == RBM_K_HAMILTON) return rbm::K_HAMILTON;
    return kernel;
}

Plan make_plan(const rbm_params *prm)
{
    Plan pl{};
    pl.kb = pl.nsets = 1;
    pl.n = (uint32_t)prm->n;
    pl.p = (uint32_t)prm->p;
    pl.nbat = pl.n / pl.p;
    pl.d = prm->d;
    pl.kernel = kern_of(prm->kernel);
    pl.rec_bytes = (size_t)4 * (prm->d + 1);
    if (pl.n <= RBM_SINGLE_CAP) {
        pl.nbuck = pl.nb1 = 1;
    } else {
        // at most RBM_MAX_FINE fine buckets (the one-workgroup scan of the
        // bucket totals) and so at most RBM_MAX_FINE / 2^shift coarse ones
        const uint32_t target = std::min<uint32_t>((pl.n + RBM_BUCKET_MEAN - 1) / RBM_BUCKET_MEAN, RBM_MAX_FINE);
        // 2^shift fine buckets per coarse one: RBM_SPLIT_SHIFT, or more when
        // the coarse buckets would not fit the digit arrays
        uint32_t shift = RBM_SPLIT_SHIFT;
        while ((target >> shift) >= RBM_MAX_COARSE) ++shift;
        const uint32_t per = 1u << shift;
        if (target <= per) {
            pl.shift = 0;
            pl.nb1 = pl.nbuck = target;
        } else {
            pl.shift = shift;
            pl.nb1 = (target + per - 1) / per;
            pl.nbuck = pl.nb1 * per;
            // chunks per coarse bucket: room for the mean plus 16 standard deviations
            const double mean = (double)pl.n / pl.nb1;
            const double room = mean + 16.0 * std::sqrt(mean) + 64.0;
            pl.chunk = RBM_CHUNK;
            pl.jmax = (uint32_t)std::ceil(room / pl.chunk);
            if (pl.nb1 * pl.jmax < RBM_SPLIT_FEW) {
                pl.chunk = RBM_CHUNK_SMALL;
                pl.jmax = (uint32_t)std::ceil(room / pl.chunk);
            }
        }
        pl.cap = RBM_SORT_CAP;
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
        // fused steps need the split level; the control-variate step keeps
        // its own order of kernels
        const char *env = getenv("RBM_FUSE");
        pl.fuse = pl.shift > 0 && !prm->cv && !(env && env[0] == '0');
        // groups of up to kb steps share the key passes; fused runs hold two
        // banks of key sets, the next group's passes made before the current
        // group's last step
        pl.kb = RBM_KEY_SETS;
        pl.nsets = pl.fuse ? 2 * pl.kb : pl.kb;
        pl.off_kcnt = take((size_t)pl.nsets * pl.ntf * pl.nbuck * 4);
        pl.off_ftot = take((size_t)pl.nsets * pl.nbuck * 4);
        pl.off_fstart = take((size_t)pl.nsets * (pl.nbuck + 1) * 4);
        pl.off_fcur = take((size_t)pl.nsets * pl.nbuck * 4);
        pl.off_cstart = take((size_t)pl.nsets * (pl.nb1 + 1) * 4);
        pl.off_ccur = take((size_t)pl.nsets * pl.nb1 * 4);
        if (pl.fuse) {
            pl.ntx = (pl.nbuck + RBM_CROSS_G - 1) / RBM_CROSS_G;
            pl.off_xrow = take((size_t)pl.nsets * pl.nbuck * pl.nb1 * 2);
            pl.off_xtsum = take((size_t)pl.nsets * pl.ntx * pl.nb1 * 4);
            pl.off_xbase = take((size_t)pl.nsets * pl.ntx * pl.nb1 * 4);
            pl.off_fixpos = take((size_t)pl.n * 4);
            pl.off_xdig = take((size_t)pl.nsets * align256(pl.n));
        }
    }
    pl.cv = prm->cv;
    if (pl.cv) {
        pl.off_sorted = take(recs);
        pl.off_cvc = take((size_t)pl.n * CV_NO * 2);
        pl.off_cvmaster = take((size_t)2 * CV_NP * 4);
        pl.off_cvam = take((size_t)2 * CV_NP * 4);
        pl.off_cvav = take((size_t)2 * CV_NP * 4);
        pl.off_cvwb = take((size_t)2 * CV_NB * 2);
        pl.off_cvspart = take((size_t)CV_SUM_WG * CV_NO * 8);
        pl.off_cvS = take((size_t)CV_NO * 8);
        pl.off_cvgpart = take((size_t)CV_GRAD_WG * 2 * CV_NP * 4);
        pl.off_cvlpart = take((size_t)CV_GRAD_WG * 4);
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
    s.scheme = prm->kernel == RBM_K_COULOMB_SPLIT ? 1u
               : prm->kernel == RBM_K_WEALTH_SPLIT ? 2u
               : prm->kernel == RBM_K_HAMILTON     ? 3u
                                                    : 0u;
    s.flowc = (float)std::exp(-2.0 * prm->kparam * prm->dt);
    return s;
}

rbm_status check_ctx(const rbm_ctx *ctx)
{
    if (!ctx) return fail(RBM_ERR_INVALID, "context is NULL");
    return RBM_OK;
}

}  // namespace

rbm_status check_cv(const rbm_ctx *ctx)
{
    rbm_status st = check_ctx(ctx);
    if (st != RBM_OK) return st;
    if (!ctx->plan.cv) return fail(RBM_ERR_INVALID, "context was created without cv = 1");
    return RBM_OK;
}

template <typename T>
T *wsp(const rbm_ctx *ctx, size_t off)
{
    return reinterpret_cast<T *>((char *)ctx->ws + off);
}

hipError_t zero_words(void *p, size_t nwords, hipStream_t st)
{
    return rbm::launch_fill(reinterpret_cast<uint32_t *>(p), nwords, 0u, st);
}

rbm_status cv_after_weights(rbm_ctx *ctx, hipStream_t st)
{
    const Plan &pl = ctx->plan;
    hipError_t e = zero_words(wsp<float>(ctx, pl.off_cvam), 2 * CV_NP, st);
    if (e == hipSuccess) e = zero_words(wsp<float>(ctx, pl.off_cvav), 2 * CV_NP, st);
    if (e == hipSuccess) e = rbm::cv_launch_prep(wsp<float>(ctx, pl.off_cvmaster), wsp<__bf16>(ctx, pl.off_cvwb), st);
    if (e != hipSuccess) return hip_fail(e, "control-variate set-up");
    ctx->cv_t = 0;
    return RBM_OK;
}


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

// The plan stays within the limits the step kernels are built for: the
// one-workgroup scan of the fine-bucket totals and the staging arrays of the
// coarse digits.
static rbm_status check_plan(const Plan &pl)
{
    if (pl.nbuck > RBM_MAX_FINE || pl.nb1 > RBM_MAX_COARSE)
        return fail(RBM_ERR_UNSUPPORTED, "N = %u needs %u fine buckets (at most %d)", pl.n, pl.nbuck, RBM_MAX_FINE);
    return RBM_OK;
}

rbm_status rbm_workspace_size(const rbm_params *prm, size_t *bytes)
{
    rbm_status st = check_params(prm);
    if (st != RBM_OK) return st;
    if (!bytes) return fail(RBM_ERR_INVALID, "bytes is NULL");
    const Plan pl = make_plan(prm);
    st = check_plan(pl);
    if (st != RBM_OK) return st;
    *bytes = pl.total;
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
    st = check_plan(pl);
    if (st != RBM_OK) return st;
    if (ws_bytes < pl.total)
        return fail(RBM_ERR_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, pl.total);
    if (((uintptr_t)d_ws & 255u) != 0) return fail(RBM_ERR_WORKSPACE, "workspace not 256-byte aligned");
    rbm_ctx *ctx = (rbm_ctx *)calloc(1, sizeof(rbm_ctx));
    if (!ctx) return fail(RBM_ERR_INVALID, "out of host memory");
    ctx->prm = *prm;
    ctx->plan = pl;
    ctx->ws = d_ws;
    ctx->m = step0;
    if (pl.fuse) {
        // the stream and events of the overlapped key passes (no device memory)
        hipError_t e = hipStreamCreateWithFlags(&ctx->ks, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_go, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->ev_keys, hipEventDisableTiming);
        if (e != hipSuccess) {
            if (ctx->ev_go) (void)hipEventDestroy(ctx->ev_go);
            if (ctx->ks) (void)hipStreamDestroy(ctx->ks);
            free(ctx);
            return hip_fail(e, "rbm_init stream");
        }
        ctx->side = true;
    }
    hipError_t e = rbm::launch_init(pl, prm->d, d_x0, d_slots, d_ws, (hipStream_t)stream);
    if (e != hipSuccess) {
        if (ctx->side) {
            (void)hipEventDestroy(ctx->ev_go);
            (void)hipEventDestroy(ctx->ev_keys);
            (void)hipStreamDestroy(ctx->ks);
        }
        free(ctx);
        return hip_fail(e, "rbm_init launch");
    }
    *out = ctx;
    if (pl.cv) return cv_init(ctx, prm->seed, stream);
    return RBM_OK;
}

rbm_status rbm_step(rbm_ctx *ctx, void *stream)
{
    return rbm_run(ctx, 1, stream);
}

// A fused run whose key passes overlap the steps.  Groups of steps share key
// passes as in rbm_run below (banks of key sets alternating); the first
// group is small (its passes are on the critical path), the later ones hold
// up to kb steps.  At the start of group g (all steps of group g - 1
// enqueued before it, so its bank is free) the side stream makes the key
// passes of group g + 1 in that bank, with the transition from group g's last
// step into group g + 1's first; the main stream waits for them before group
// g's last step, whose sort kernel writes the coarse buckets of group g + 1.
// The same kernels on the same data in the same order per stream: the bits
// are those of the serial order.
static rbm_status run_overlapped(rbm_ctx *ctx, int64_t nsteps, hipStream_t hs)
{
    const Plan &pl = ctx->plan;
    void *state = (char *)ctx->ws + pl.off_state;
    constexpr int64_t FIRST = 2;
    int64_t k = 0;
    int64_t gsize = std::min<int64_t>(FIRST, nsteps);
    uint32_t bank = 0;
    {
        const StepArgs s0 = make_args(&ctx->prm, pl, (uint32_t)ctx->m, ctx->pending);
        hipError_t e = rbm::launch_keys(pl, s0, (uint32_t)gsize, ctx->ws, hs, nullptr, 0);
        if (e != hipSuccess) return hip_fail(e, "rbm_run key launch");
    }
    bool prev_out = false;
    while (k < nsteps) {
        const int64_t rest = nsteps - k - gsize;  // steps after this group
        const int64_t next = std::min<int64_t>(pl.kb, rest);
        if (next > 0) {
            hipError_t e = hipEventRecord(ctx->ev_go, hs);
            if (e == hipSuccess) e = hipStreamWaitEvent(ctx->ks, ctx->ev_go, 0);
            if (e != hipSuccess) return hip_fail(e, "rbm_run side stream");
            const StepArgs sn = make_args(&ctx->prm, pl, (uint32_t)(ctx->m + gsize), false);
            e = rbm::launch_keys(pl, sn, (uint32_t)next, ctx->ws, ctx->ks, nullptr, (bank ^ 1u) * pl.kb,
                                 bank * pl.kb + (uint32_t)gsize - 1u);
            if (e == hipSuccess) e = hipEventRecord(ctx->ev_keys, ctx->ks);
            if (e != hipSuccess) return hip_fail(e, "rbm_run key launch");
        }
        for (int64_t i = 0; i < gsize; ++i) {
            const StepArgs s = make_args(&ctx->prm, pl, (uint32_t)ctx->m, ctx->pending);
            const bool out = k + i + 1 < nsteps;
            if (out && i + 1 == gsize) {
                hipError_t e = hipStreamWaitEvent(hs, ctx->ev_keys, 0);
                if (e != hipSuccess) return hip_fail(e, "rbm_run side stream");
            }
            const uint32_t fuse = (prev_out ? 1u : 0u) | (out ? 2u : 0u);
            hipError_t e = rbm::launch_step(pl, s, pl.d, pl.kernel, ctx->ws, hs, state, nullptr, nullptr,
                                            bank * pl.kb + (uint32_t)i, true, fuse);
            if (e != hipSuccess) return hip_fail(e, "rbm_step launch");
            prev_out = out;
            ctx->m += 1;
            ctx->pending = s.ssd != 0.0f;
        }
        k += gsize;
        gsize = next;
        bank ^= 1u;
    }
    return RBM_OK;
}

rbm_status rbm_run(rbm_ctx *ctx, int64_t nsteps, void *stream)
{
    rbm_status st = check_ctx(ctx);
    if (st != RBM_OK) return st;
    if (nsteps < 0) return fail(RBM_ERR_INVALID, "nsteps < 0");
    if (ctx->m + nsteps > 0x100000000LL) return fail(RBM_ERR_INVALID, "step index would pass 2^32");
    const Plan &pl = ctx->plan;
    void *state = (char *)ctx->ws + pl.off_state;
    const hipStream_t hs = (hipStream_t)stream;
    // Key sets: group g of up to kb steps uses sets [bank_g kb, bank_g kb +
    // size_g), the banks alternating when fused (pl.nsets = 2 kb).  Fused, the
    // sort of every step but the call's last writes the next step's coarse
    // buckets, placed by the transitions that launch_keys makes: inside a
    // group, and from a group's last step into the next group (made with that
    // group's key passes, before the step).  Only the call's first step runs
    // the coarse scatter and its last leaves the state in slot order.
    if (ctx->side && ctx->tmax == 0 && nsteps > 1) return run_overlapped(ctx, nsteps, hs);
    uint32_t set = 0, group = 0, bank = 0, next_group = 0;
    bool prev_out = false;
    for (int64_t k = 0; k < nsteps; ++k) {
        const StepArgs s = make_args(&ctx->prm, pl, (uint32_t)ctx->m, ctx->pending);
        hipEvent_t *ev = nullptr;
        if (ctx->trec < ctx->tmax) ev = ctx->ev + (size_t)ctx->trec++ * (RBM_NPHASES + 1);
        bool keys_timed = false;
        if (set == group) {
            set = 0;
            if (next_group) {
                // made before the previous group's last step
                group = next_group;
                bank ^= 1u;
                next_group = 0;
            } else {
                // the key passes of the next group of steps, in one launch each
                group = (uint32_t)std::min<int64_t>(pl.kb, nsteps - k);
                hipError_t e = rbm::launch_keys(pl, s, group, ctx->ws, hs, ev, 0);
                if (e != hipSuccess) return hip_fail(e, "rbm_step key launch");
                keys_timed = true;
            }
        }
        const uint32_t cur = bank * pl.kb + set;
        const bool out = pl.fuse && k + 1 < nsteps;
        if (out && set + 1 == group) {
            // the next group's key passes into the other bank, and the
            // transition from this step into its first step (timed with this step)
            next_group = (uint32_t)std::min<int64_t>(pl.kb, nsteps - k - 1);
            const uint32_t nb = (bank ^ 1u) * pl.kb;
            const StepArgs sn = make_args(&ctx->prm, pl, (uint32_t)ctx->m + 1, s.ssd != 0.0f);
            hipError_t e = rbm::launch_keys(pl, sn, next_group, ctx->ws, hs, keys_timed ? nullptr : ev, nb, cur);
            if (e != hipSuccess) return hip_fail(e, "rbm_step key launch");
            if (!keys_timed && ev) keys_timed = true;
        }
        if (!keys_timed && ev) {
            // this step's share of the key passes was timed with another step
            for (int i = 0; i < 4; ++i) (void)hipEventRecord(ev[i], hs);
        }
        const uint32_t fuse = (prev_out ? 1u : 0u) | (out ? 2u : 0u);
        hipError_t e = rbm::launch_step(pl, s, pl.d, pl.kernel, ctx->ws, hs, state, nullptr, ev, cur, true, fuse);
        if (e != hipSuccess) return hip_fail(e, "rbm_step launch");
        prev_out = out;
        ++set;
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
    if (ctx->side) {
        // work of this context still queued on the side stream ends first
        (void)hipStreamSynchronize(ctx->ks);
        (void)hipEventDestroy(ctx->ev_go);
        (void)hipEventDestroy(ctx->ev_keys);
        (void)hipStreamDestroy(ctx->ks);
    }
    free(ctx);
    return RBM_OK;
}

rbm_status cv_init(rbm_ctx *ctx, uint64_t seed, void *stream)
{
    rbm_status st = check_cv(ctx);
    if (st != RBM_OK) return st;
    hipError_t e = rbm::cv_launch_glorot(wsp<float>(ctx, ctx->plan.off_cvmaster), seed, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "cv_init");
    return cv_after_weights(ctx, (hipStream_t)stream);
}

rbm_status cv_set_weights(rbm_ctx *ctx, const float *d_w, void *stream)
{
    rbm_status st = check_cv(ctx);
    if (st != RBM_OK) return st;
    if (!d_w) return fail(RBM_ERR_INVALID, "d_w is NULL");
    hipError_t e = hipMemcpyAsync(wsp<float>(ctx, ctx->plan.off_cvmaster), d_w, (size_t)2 * CV_NP * 4,
                                  hipMemcpyDeviceToDevice, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "cv_set_weights");
    return cv_after_weights(ctx, (hipStream_t)stream);
}

rbm_status cv_get_weights(rbm_ctx *ctx, float *d_w, void *stream)
{
    rbm_status st = check_cv(ctx);
    if (st != RBM_OK) return st;
    if (!d_w) return fail(RBM_ERR_INVALID, "d_w is NULL");
    hipError_t e = hipMemcpyAsync(d_w, wsp<float>(ctx, ctx->plan.off_cvmaster), (size_t)2 * CV_NP * 4,
                                  hipMemcpyDeviceToDevice, (hipStream_t)stream);
    return e == hipSuccess ? RBM_OK : hip_fail(e, "cv_get_weights");
}

rbm_status cv_features(rbm_ctx *ctx, const float *d_x, int64_t n, float *d_a, float *d_c, void *stream)
{
    rbm_status st = check_cv(ctx);
    if (st != RBM_OK) return st;
    if (!d_x || n < 0 || n > (1LL << 30)) return fail(RBM_ERR_INVALID, "bad points");
    if (n == 0 || (!d_a && !d_c)) return RBM_OK;
    hipError_t e = rbm::cv_launch_features(wsp<float>(ctx, ctx->plan.off_cvmaster), wsp<__bf16>(ctx, ctx->plan.off_cvwb),
                                           d_x, (uint32_t)n, d_a, d_c, (hipStream_t)stream);
    return e == hipSuccess ? RBM_OK : hip_fail(e, "cv_features");
}

rbm_status cv_grads(rbm_ctx *ctx, const float *d_x, const float *d_y, int64_t npairs, float *d_g,
                    float *d_loss, void *stream)
{
    rbm_status st = check_cv(ctx);
    if (st != RBM_OK) return st;
    if (!d_x || !d_y || !d_g || !d_loss) return fail(RBM_ERR_INVALID, "NULL pointer argument");
    if (npairs < 1 || npairs > (1LL << 24)) return fail(RBM_ERR_INVALID, "npairs out of range");
    const Plan &pl = ctx->plan;
    uint32_t nwg = 0;
    hipError_t e = rbm::cv_launch_grad((uint32_t)npairs, (float)ctx->prm.kparam, d_x, d_y, nullptr, 0, 0, 0,
                                       ctx->prm.seed, wsp<float>(ctx, pl.off_cvmaster), wsp<__bf16>(ctx, pl.off_cvwb),
                                       wsp<float>(ctx, pl.off_cvgpart), wsp<float>(ctx, pl.off_cvlpart), &nwg,
                                       (hipStream_t)stream);
    if (e == hipSuccess)
        e = rbm::cv_launch_reduce(nwg, wsp<float>(ctx, pl.off_cvgpart), wsp<float>(ctx, pl.off_cvlpart), d_g, d_loss,
                                  0, 0.0f, 1, nullptr, nullptr, nullptr, (hipStream_t)stream);
    return e == hipSuccess ? RBM_OK : hip_fail(e, "cv_grads");
}

rbm_status cv_train(rbm_ctx *ctx, const float *d_snap, int32_t nsnap, int64_t nsteps, int32_t batch, float lr,
                    float *d_loss, void *stream)
{
    rbm_status st = check_cv(ctx);
    if (st != RBM_OK) return st;
    if (!d_snap || nsnap < 1 || nsteps < 0 || batch < 1 || batch > (1 << 24) || !(lr > 0.0f))
        return fail(RBM_ERR_INVALID, "bad training arguments");
    if (ctx->cv_t + nsteps > 0xffffffffLL) return fail(RBM_ERR_INVALID, "too many Adam steps");
    const Plan &pl = ctx->plan;
    for (int64_t k = 0; k < nsteps; ++k) {
        uint32_t nwg = 0;
        hipError_t e = rbm::cv_launch_grad((uint32_t)batch, (float)ctx->prm.kparam, nullptr, nullptr, d_snap,
                                           (uint32_t)nsnap, pl.n, (uint32_t)ctx->cv_t, ctx->prm.seed,
                                           wsp<float>(ctx, pl.off_cvmaster), wsp<__bf16>(ctx, pl.off_cvwb),
                                           wsp<float>(ctx, pl.off_cvgpart), wsp<float>(ctx, pl.off_cvlpart), &nwg,
                                           (hipStream_t)stream);
        if (e == hipSuccess)
            e = rbm::cv_launch_reduce(nwg, wsp<float>(ctx, pl.off_cvgpart), wsp<float>(ctx, pl.off_cvlpart), nullptr,
                                      d_loss ? d_loss + k : nullptr, 1, lr, (int)(ctx->cv_t + 1),
                                      wsp<float>(ctx, pl.off_cvmaster), wsp<float>(ctx, pl.off_cvam),
                                      wsp<float>(ctx, pl.off_cvav), (hipStream_t)stream);
        if (e == hipSuccess)
            e = rbm::cv_launch_prep(wsp<float>(ctx, pl.off_cvmaster), wsp<__bf16>(ctx, pl.off_cvwb), (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "cv_train");
        ctx->cv_t += 1;
    }
    return RBM_OK;
}

rbm_status rbm_force_sqerr(const float *d_f, int64_t n, const uint32_t *d_ids, int64_t nids, const float *d_fref,
                           int32_t d, double *d_out, void *stream)
{
    if (!d_f || !d_out || (nids > 0 && (!d_ids || !d_fref))) return fail(RBM_ERR_INVALID, "NULL pointer argument");
    if (d < 1 || d > 3 || n < 1 || n > 0x7fffffffLL || nids < 0 || nids > (1LL << 30))
        return fail(RBM_ERR_INVALID, "bad sizes");
    hipError_t e = rbm::launch_sqerr(d_f, (uint32_t)n, d_ids, (uint32_t)nids, d_fref, d, d_out, (hipStream_t)stream);
    return e == hipSuccess ? RBM_OK : hip_fail(e, "rbm_force_sqerr");
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
    hipError_t e = rbm::launch_direct(s, prm->d, kern_of(prm->kernel), d_x, d_ids, (uint32_t)nids, d_f, 0,
                                      (hipStream_t)stream);
    return e == hipSuccess ? RBM_OK : hip_fail(e, "direct_forces launch");
}

rbm_status direct_moments(const rbm_params *prm, const float *d_x, const uint32_t *d_ids, int64_t nids,
                          float *d_f, float *d_m2, void *stream)
{
    rbm_status st = check_params(prm);
    if (st == RBM_ERR_UNSUPPORTED && prm && prm->n <= RBM_MAX_N) st = RBM_OK;  // p is not used
    if (st != RBM_OK) return st;
    if (!d_x || !d_f || !d_m2) return fail(RBM_ERR_INVALID, "NULL pointer argument");
    if (d_ids == nullptr) nids = prm->n;
    if (nids < 0 || nids > prm->n) return fail(RBM_ERR_INVALID, "nids out of range");
    if (nids == 0) return RBM_OK;
    const Plan pl = make_plan(prm);
    const StepArgs s = make_args(prm, pl, 0, false);
    hipError_t e = rbm::launch_direct(s, prm->d, kern_of(prm->kernel), d_x, d_ids, (uint32_t)nids, d_f, 0,
                                      (hipStream_t)stream, d_m2);
    return e == hipSuccess ? RBM_OK : hip_fail(e, "direct_moments launch");
}

rbm_status direct_step(const rbm_params *prm, const float *d_x, float *d_x_out, int64_t step,
                       void *stream)
{
    rbm_status st = check_params(prm);
    if (st == RBM_ERR_UNSUPPORTED && prm && prm->n <= RBM_MAX_N) st = RBM_OK;
    if (st != RBM_OK) return st;
    if (prm->kernel == RBM_K_WEALTH_SPLIT)
        return fail(RBM_ERR_UNSUPPORTED, "direct_step has additive noise; the wealth model's is multiplicative");
    if (!d_x || !d_x_out) return fail(RBM_ERR_INVALID, "NULL pointer argument");
    if (d_x == d_x_out) return fail(RBM_ERR_INVALID, "d_x_out must not alias d_x");
    if (step < 0 || step > 0xffffffffLL) return fail(RBM_ERR_INVALID, "step out of range");
    const Plan pl = make_plan(prm);
    const StepArgs s = make_args(prm, pl, (uint32_t)step, false);
    hipError_t e = rbm::launch_direct(s, prm->d, kern_of(prm->kernel), d_x, nullptr, (uint32_t)prm->n,
                                      d_x_out, 1, (hipStream_t)stream);
    return e == hipSuccess ? RBM_OK : hip_fail(e, "direct_step launch");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched ensemble
// ---------------------------------------------------------------------------

static_assert(RBM_ENS_LDS == 4096 && RBM_ENS_MAXN == 256 * 1024, "ensemble limits of the header and the kernels differ");

namespace {

struct EnsLayout {
    size_t sys, order, items, ctl, state, stage, wst, wst2, total;
    uint64_t nsum;
};

rbm_status ens_check(const rbm_ensemble *e, const int64_t *h_n, EnsLayout *lay)
{
    if (!e || !h_n) return fail(RBM_ERR_INVALID, "NULL pointer argument");
    if (e->d != 2) return fail(RBM_ERR_UNSUPPORTED, "the ensemble kernels implement d = 2 (got %d)", e->d);
    if (e->kernel < RBM_K_GAUSS || e->kernel > RBM_K_ATTREP) return fail(RBM_ERR_INVALID, "unknown kernel %d", e->kernel);
    if (e->reserved != 0) return fail(RBM_ERR_INVALID, "reserved field must be 0");
    if (e->nsys < 1 || e->nsys > (1LL << 24)) return fail(RBM_ERR_INVALID, "nsys = %lld not in 1..2^24", (long long)e->nsys);
    if (e->p < 2 || e->p > RBM_MAX_P_MULTI) return fail(RBM_ERR_INVALID, "p = %d not in 2..%d", e->p, RBM_MAX_P_MULTI);
    if (!(e->dt > 0.0) || !std::isfinite(e->dt)) return fail(RBM_ERR_INVALID, "dt must be > 0");
    if (!(e->sigma >= 0.0) || !std::isfinite(e->sigma)) return fail(RBM_ERR_INVALID, "sigma must be >= 0");
    if (!(e->kparam >= 0.0) || !std::isfinite(e->kparam)) return fail(RBM_ERR_INVALID, "kparam must be >= 0");
    if (!std::isfinite(e->beta)) return fail(RBM_ERR_INVALID, "beta must be finite");
    uint64_t nsum = 0;
    for (int64_t i = 0; i < e->nsys; ++i) {
        if (h_n[i] < e->p || h_n[i] > RBM_ENS_MAXN)
            return fail(RBM_ERR_INVALID, "system %lld: N = %lld not in p..%d", (long long)i, (long long)h_n[i],
                        RBM_ENS_MAXN);
        nsum += (uint64_t)h_n[i];
    }
    if (nsum > 0x7fffffffULL) return fail(RBM_ERR_UNSUPPORTED, "%llu particles in all, above 2^31 - 1", (unsigned long long)nsum);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    lay->nsum = nsum;
    lay->sys = take((size_t)e->nsys * sizeof(rbm::EnsSys));
    lay->order = take((size_t)e->nsys * 4);
    lay->items = take((size_t)e->nsys * 8);
    lay->ctl = take(8);
    lay->state = take(nsum * sizeof(rbm::Rec<2>));
    lay->stage = take(nsum * sizeof(rbm::Rec<2>));
    lay->wst = take(nsum * 4);
    lay->wst2 = take(nsum * 4);
    lay->total = off;
    return RBM_OK;
}

}  // namespace

extern "C" {

rbm_status ensemble_workspace_size(const rbm_ensemble *e, const int64_t *h_n, size_t *bytes)
{
    EnsLayout lay;
    rbm_status st = ens_check(e, h_n, &lay);
    if (st != RBM_OK) return st;
    if (!bytes) return fail(RBM_ERR_INVALID, "NULL pointer argument");
    *bytes = lay.total;
    return RBM_OK;
}

rbm_status ensemble_run(const rbm_ensemble *e, const int64_t *h_n, const uint64_t *h_seed, float *d_x,
                        int64_t step0, int64_t nsteps, const rbm_ensemble_tile *tile, void *d_ws,
                        size_t ws_bytes, int32_t graph, void *stream)
{
    EnsLayout lay;
    rbm_status st = ens_check(e, h_n, &lay);
    if (st != RBM_OK) return st;
    if (!h_seed || !d_x || !d_ws) return fail(RBM_ERR_INVALID, "NULL pointer argument");
    if (ws_bytes < lay.total)
        return fail(RBM_ERR_WORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, lay.total);
    if (((uintptr_t)d_ws & 255) != 0) return fail(RBM_ERR_WORKSPACE, "workspace not 256-byte aligned");
    if (step0 < 0 || nsteps < 0 || step0 + nsteps > 0x100000000LL)
        return fail(RBM_ERR_INVALID, "steps out of range");
    if (graph != 0 && graph != 1) return fail(RBM_ERR_INVALID, "graph must be 0 or 1");
    int lds_max = tile ? tile->lds_max : 0;
    int grid = tile ? tile->grid : 0;
    int team = tile ? tile->team : 0;
    int bucket = tile ? tile->bucket : 0;
    int wg = tile ? tile->wg : 0;
    if (wg == 0) wg = 1024;
    if (wg != 1024 && wg != 512) return fail(RBM_ERR_INVALID, "wg = %d is not 512 or 1024", wg);
    if (lds_max == 0) lds_max = 4 * wg;
    if (team == 0) team = 256;
    if (bucket == 0) bucket = wg;
    if (lds_max < 0 || lds_max > 4 * wg) return fail(RBM_ERR_INVALID, "lds_max = %d not in 0..%d", lds_max, 4 * wg);
    if (grid < 0 || grid > 65536) return fail(RBM_ERR_INVALID, "grid = %d not in 0..65536", grid);
    if (team < 64 || team > wg || (team & (team - 1)) != 0)
        return fail(RBM_ERR_INVALID, "team = %d is not a power of two in 64..%d", team, wg);
    if (bucket < 256 || bucket > 3 * wg) return fail(RBM_ERR_INVALID, "bucket = %d not in 256..%d", bucket, 3 * wg);
    int64_t nmax = 0;
    for (int64_t i = 0; i < e->nsys; ++i) nmax = std::max(nmax, h_n[i]);
    if (nmax > lds_max && (nmax + bucket - 1) / bucket > RBM_ENS_MAXB)
        return fail(RBM_ERR_INVALID, "bucket = %d gives more than %d buckets for N = %lld", bucket, RBM_ENS_MAXB,
                    (long long)nmax);
    if (grid == 0) {
        int dev = 0, cus = 0;
        hipError_t he = hipGetDevice(&dev);
        if (he == hipSuccess) he = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (he != hipSuccess) return hip_fail(he, "compute unit count");
        grid = cus * (wg == 512 ? 2 : 1);
    }
    if (nsteps == 0) return RBM_OK;
    const hipStream_t hs = (hipStream_t)stream;

    // system table and queue order (largest first; ties by index)
    std::vector<rbm::EnsSys> sys((size_t)e->nsys);
    std::vector<uint32_t> order((size_t)e->nsys);
    uint64_t off = 0;
    for (int64_t i = 0; i < e->nsys; ++i) {
        rbm::EnsSys &y = sys[(size_t)i];
        y = rbm::EnsSys{};
        y.off = (uint32_t)off;
        y.n = (uint32_t)h_n[i];
        y.k0 = (uint32_t)(h_seed[i] & 0xffffffffu);
        y.k1 = (uint32_t)(h_seed[i] >> 32);
        y.inv_last = (float)(1.0 / (double)(e->p + y.n % (uint32_t)e->p - 1));
        off += y.n;
    }
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return sys[a].n > sys[b].n; });
    // work items in queue order: every system above 4 team particles alone,
    // then the rest in groups of wg / team consecutive systems
    std::vector<uint32_t> items;  // pairs (first, count)
    const uint32_t g = (uint32_t)wg / (uint32_t)team, cap = 4u * (uint32_t)team;
    for (size_t i = 0; i < order.size();) {
        uint32_t c = 1;
        if (g > 1 && sys[order[i]].n <= cap) c = (uint32_t)std::min<size_t>(g, order.size() - i);
        items.push_back((uint32_t)i);
        items.push_back(c);
        i += c;
    }
    const uint32_t nitems = (uint32_t)(items.size() / 2);
    if ((int64_t)grid > nitems) grid = (int)nitems;

    char *ws = (char *)d_ws;
    hipError_t he = hipMemcpyAsync(ws + lay.sys, sys.data(), sys.size() * sizeof(rbm::EnsSys), hipMemcpyHostToDevice, hs);
    if (he == hipSuccess)
        he = hipMemcpyAsync(ws + lay.order, order.data(), order.size() * 4, hipMemcpyHostToDevice, hs);
    if (he == hipSuccess)
        he = hipMemcpyAsync(ws + lay.items, items.data(), items.size() * 4, hipMemcpyHostToDevice, hs);
    if (he != hipSuccess) return hip_fail(he, "ensemble table upload");

    rbm::EnsLaunch L{};
    L.base.p = (uint32_t)e->p;
    L.base.m = (uint32_t)step0;
    L.base.inv_p1 = (float)(1.0 / (double)(e->p - 1));
    L.base.a = (float)e->kparam;
    L.base.beta = (float)e->beta;
    L.base.dt = (float)e->dt;
    L.base.ssd = (float)(e->sigma * std::sqrt(e->dt));
    L.nsteps = nsteps;
    L.nitems = nitems;
    L.lds_max = (uint32_t)lds_max;
    L.wg = (uint32_t)wg;
    L.team = (uint32_t)team;
    L.bmean = (uint32_t)bucket;
    L.grid = (uint32_t)grid;
    L.sys = ws + lay.sys;
    L.order = (const uint32_t *)(ws + lay.order);
    L.items = (const uint2 *)(ws + lay.items);
    L.next = (uint32_t *)(ws + lay.ctl);
    L.flags = L.next + 1;
    L.x = d_x;
    L.state = ws + lay.state;
    L.stage = ws + lay.stage;
    L.wst = (uint32_t *)(ws + lay.wst);
    L.wst2 = (uint32_t *)(ws + lay.wst2);

    if (!graph) {
        he = rbm::launch_ensemble(L, e->kernel, hs);
        if (he != hipSuccess) return hip_fail(he, "ensemble launch");
    } else {
        // record the launch on a private stream, replay it once, join the caller's stream
        hipStream_t cs = nullptr;
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        he = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (he == hipSuccess) he = hipEventCreateWithFlags(&ev0, hipEventDisableTiming);
        if (he == hipSuccess) he = hipEventCreateWithFlags(&ev1, hipEventDisableTiming);
        if (he == hipSuccess) he = hipEventRecord(ev0, hs);
        if (he == hipSuccess) he = hipStreamWaitEvent(cs, ev0, 0);
        if (he == hipSuccess) he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (he == hipSuccess) {
            hipError_t le = rbm::launch_ensemble(L, e->kernel, cs);
            he = hipStreamEndCapture(cs, &g);
            if (le != hipSuccess) he = le;
        }
        if (he == hipSuccess) he = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        if (he == hipSuccess) he = hipGraphLaunch(ge, cs);
        if (he == hipSuccess) he = hipEventRecord(ev1, cs);
        if (he == hipSuccess) he = hipStreamWaitEvent(hs, ev1, 0);
        // tear-down: the first error, if any, is the one reported
        hipError_t te = hipSuccess;
        auto keep = [&](hipError_t x) { if (te == hipSuccess) te = x; };
        if (cs) keep(hipStreamSynchronize(cs));
        if (ge) keep(hipGraphExecDestroy(ge));
        if (g) keep(hipGraphDestroy(g));
        if (ev0) keep(hipEventDestroy(ev0));
        if (ev1) keep(hipEventDestroy(ev1));
        if (cs) keep(hipStreamDestroy(cs));
        if (he == hipSuccess) he = te;
        if (he != hipSuccess) return hip_fail(he, "ensemble graph");
    }
    uint32_t flags = 0;
    he = hipMemcpyAsync(&flags, L.flags, 4, hipMemcpyDeviceToHost, hs);
    if (he == hipSuccess) he = hipStreamSynchronize(hs);
    if (he != hipSuccess) return hip_fail(he, "ensemble completion");
    if (flags != 0) return fail(RBM_ERR_DEVICE, "a bucket of a streamed system exceeded the LDS capacity");
    return RBM_OK;
}

// ---------------------------------------------------------------------------
// RBM-r
// ---------------------------------------------------------------------------
static_assert(RBMR_MAX_P == RBM_RBMR_MAX_P && RBMR_MAX_WINDOW == RBM_RBMR_MAX_WINDOW &&
                  RBMR_MAX_ROUNDS == RBM_RBMR_MAX_ROUNDS && (uint64_t)RBMR_MAX_NBK * RBMR_MAX_PB >= RBM_MAX_N,
              "RBM-r limits of the header and the kernels differ");

static rbm_status rbmr_plan(const rbm_params *prm, int64_t window, int32_t rounds, rbm::RbmrLayout *lay)
{
    if (!prm) return fail(RBM_ERR_INVALID, "params is NULL");
    if (prm->d < 1 || prm->d > 3) return fail(RBM_ERR_INVALID, "d = %d not in 1..3", prm->d);
    if (prm->kernel < RBM_K_GAUSS || prm->kernel > RBM_K_COULOMB_SPLIT)
        return fail(RBM_ERR_UNSUPPORTED, "RBM-r takes kernels 0..3 (got %d)", prm->kernel);
    if (prm->n < 2 || prm->n > RBM_MAX_N) return fail(RBM_ERR_INVALID, "N = %lld not in 2..2^25", (long long)prm->n);
    if (prm->p < 2 || prm->p > RBMR_MAX_P || (int64_t)prm->p > prm->n)
        return fail(RBM_ERR_UNSUPPORTED, "RBM-r needs 2 <= p <= min(N, %d)", RBMR_MAX_P);
    if (prm->kernel == RBM_K_COULOMB_SPLIT && (prm->p != 2 || prm->kparam != 0.0))
        return fail(RBM_ERR_UNSUPPORTED, "the split Coulomb kernel needs p = 2 and kparam = 0");
    if (prm->cv != 0 || prm->reserved != 0) return fail(RBM_ERR_INVALID, "cv and reserved must be 0");
    if (!(prm->dt > 0.0) || !std::isfinite(prm->dt)) return fail(RBM_ERR_INVALID, "dt must be > 0");
    if (!(prm->sigma >= 0.0) || !std::isfinite(prm->sigma)) return fail(RBM_ERR_INVALID, "sigma must be >= 0");
    if (!(prm->kparam >= 0.0) || !std::isfinite(prm->kparam)) return fail(RBM_ERR_INVALID, "kparam must be >= 0");
    if (!std::isfinite(prm->beta)) return fail(RBM_ERR_INVALID, "beta must be finite");
    const int64_t wdef = std::min<int64_t>(std::max<int64_t>(prm->n / prm->p, 1), RBMR_MAX_WINDOW);
    if (window == 0) window = wdef;
    if (window < 1 || window > RBMR_MAX_WINDOW)
        return fail(RBM_ERR_INVALID, "window %lld not in 1..%u", (long long)window, RBMR_MAX_WINDOW);
    if (rounds == 0) {
        // rounds across the GPU until a few hundred iterations of a window of
        // N/p are left for the finishing workgroup (touches per particle
        // c = window p / N; the depth grows with c and, slowly, with N)
        const int64_t c = (window * prm->p + prm->n - 1) / prm->n;
        const int64_t extra = prm->n > (1 << 22) ? 1 : 0;
        rounds = (int32_t)std::min<int64_t>((4 + 2 * prm->p) * c + extra, RBM_RBMR_MAX_ROUNDS);
    }
    if (rounds < 1 || rounds > RBM_RBMR_MAX_ROUNDS)
        return fail(RBM_ERR_INVALID, "rounds %d not in 1..%d", rounds, RBM_RBMR_MAX_ROUNDS);
    *lay = rbm::rbmr_layout((uint32_t)prm->n, (uint32_t)prm->p, (uint32_t)window, (uint32_t)rounds);
    return RBM_OK;
}

static rbm_status rbmr_run_ws(const rbm_params *prm, float *d_x, int64_t k0, int64_t niter, int64_t window,
                              int32_t rounds, void *d_ws, size_t ws_bytes, void *stream)
{
    rbm::RbmrLayout lay;
    const rbm_status st = rbmr_plan(prm, window, rounds, &lay);
    if (st != RBM_OK) return st;
    if (!d_x || !d_ws) return fail(RBM_ERR_INVALID, "NULL pointer argument");
    if (k0 < 0 || niter < 0 || k0 > (int64_t)1 << 48 || niter > ((int64_t)1 << 48) - k0)
        return fail(RBM_ERR_INVALID, "iterations k0 .. k0 + niter must lie in 0 .. 2^48");
    if (ws_bytes < lay.bytes) return fail(RBM_ERR_WORKSPACE, "workspace %zu bytes < %zu needed", ws_bytes, lay.bytes);
    if (((uintptr_t)d_ws & 255u) != 0) return fail(RBM_ERR_WORKSPACE, "workspace not 256-byte aligned");
    rbm::RbmrArgs a{};
    a.n = (uint32_t)prm->n;
    a.p = (uint32_t)prm->p;
    a.k0 = (uint32_t)(prm->seed & 0xffffffffu);
    a.k1 = (uint32_t)(prm->seed >> 32);
    a.sys = prm->sys;
    a.inv_p1 = (float)(1.0 / (double)(prm->p - 1));
    a.a = (float)prm->kparam;
    a.beta = (float)prm->beta;
    a.dt = (float)prm->dt;
    a.ssd = (float)(prm->sigma * std::sqrt(prm->dt));
    const hipError_t e = rbm::rbmr_launch(a, prm->d, prm->kernel, lay, d_ws, d_x, (uint64_t)k0, (uint64_t)niter,
                                          (hipStream_t)stream);
    return e == hipSuccess ? RBM_OK : hip_fail(e, "rbmr_run launch");
}

// The workspace of rbmr_run_noalloc: one static array per GPU.  In host code
// its name stands for the array but is not its device address; the address
// is resolved once per device (with that device current) by
// hipGetSymbolAddress and only that pointer is handed to kernels.
static __device__ __align__(256) unsigned char scratch[RBM_NOALLOC_SCRATCH_BYTES];

static rbm_status noalloc_scratch(void **out)
{
    constexpr int MAXDEV = 64;
    static std::mutex mu;
    static void *addr[MAXDEV] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "rbmr_run_noalloc: hipGetDevice");
    if (dev < 0 || dev >= MAXDEV) return fail(RBM_ERR_UNSUPPORTED, "device %d above the %d supported", dev, MAXDEV);
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "rbmr_run_noalloc: hipGetSymbolAddress");
        if (!p || ((uintptr_t)p & 255u) != 0) return fail(RBM_ERR_HIP, "rbmr_run_noalloc: bad scratch address");
        addr[dev] = p;
    }
    *out = addr[dev];
    return RBM_OK;
}


rbm_status rbmr_workspace_size(const rbm_params *prm, int64_t window, int32_t rounds, size_t *bytes)
{
    if (!bytes) return fail(RBM_ERR_INVALID, "bytes is NULL");
    rbm::RbmrLayout lay;
    const rbm_status st = rbmr_plan(prm, window, rounds, &lay);
    if (st != RBM_OK) return st;
    *bytes = lay.bytes;
    return RBM_OK;
}

rbm_status rbmr_run(const rbm_params *prm, float *d_x, int64_t k0, int64_t niter, int64_t window, int32_t rounds,
                    void *d_ws, size_t ws_bytes, void *stream)
{
    return rbmr_run_ws(prm, d_x, k0, niter, window, rounds, d_ws, ws_bytes, stream);
}

rbm_status rbmr_run_noalloc(const rbm_params *prm, float *d_x, int64_t k0, int64_t niter, int64_t window,
                            int32_t rounds, void *stream)
{
    rbm::RbmrLayout lay;
    const rbm_status st = rbmr_plan(prm, window, rounds, &lay);
    if (st != RBM_OK) return st;
    if (lay.bytes > RBM_NOALLOC_SCRATCH_BYTES)
        return fail(RBM_ERR_WORKSPACE, "this run needs %zu bytes of workspace, above the %zu of the static buffer",
                    lay.bytes, (size_t)RBM_NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    const rbm_status sst = noalloc_scratch(&ws);
    if (sst != RBM_OK) return sst;
    return rbmr_run_ws(prm, d_x, k0, niter, window, rounds, ws, RBM_NOALLOC_SCRATCH_BYTES, stream);
}

}  // extern "C"
