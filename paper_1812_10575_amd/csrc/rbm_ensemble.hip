// Batched ensemble: many independent RBM-1 systems (Sec. 2.1, Algorithm 1) of
// uneven size in one persistent launch.
//
// System s uses the Philox key seed_s and counter word 3 = s, so each system
// follows exactly the definitions of a standalone run with those values.
// Workgroups take work items from an atomic queue that the host orders by
// decreasing cost (longest first) and run every step of an item before
// taking the next.  An item is either one system, run by the whole
// workgroup, or a group of up to TPB / T small systems, run side by side by
// teams of T threads (each team with its own slice of the LDS arrays; the
// workgroup barriers keep the teams in step).
//
//   * a system of at most 4 T particles (4 TPB for a whole-workgroup item up
//     to lds_max) lives in LDS for all steps: per step the slots draw their
//     PERM words, a counting pass on the top bits of the word plus an exact
//     rank inside the (tiny) sub-buckets orders them by key, the batch forces
//     and the Euler-Maruyama update are applied, and the updated records, in
//     key order, are the next step's slot order.  HBM is touched only to load
//     and store the system.
//   * a larger system goes through its own region of global memory (written
//     and read by one workgroup only, so the workgroup barrier orders it; a
//     device-scope fence would write back and invalidate the L2 of the whole
//     XCD): a word histogram over buckets of about bmean records, a scatter
//     of the records to their buckets, then the buckets in order, each sorted
//     in LDS; a batch cut by the end of a bucket is carried to the next
//     bucket in LDS, so every batch is complete when it is evaluated.
#include "rbm_ensemble.hpp"
#include "rbm_device.hpp"

namespace rbm {
namespace ens {

// Two workgroup shapes: W = 1024 threads with 4096 records of LDS (one
// workgroup per compute unit), or W = 512 with 2048 (two per compute unit).
// In both, a thread owns E = 4 records and 4 sub-bucket counters.
constexpr int E = 4;
constexpr int MAXB = RBM_ENS_MAXB;
#define RBM_ENS_SHAPE                                                                              \
    constexpr int TPB = W;       /* threads */                                                     \
    constexpr int CAP = 4 * W;   /* records in LDS, all teams together */                          \
    constexpr int S = 4 * W;     /* sub-bucket counters */                                         \
    (void)TPB;                                                                                     \
    (void)CAP;                                                                                     \
    (void)S

using Sys = EnsSys;

template <int D, int W>
struct Lds {
    Rec<D> a[4 * W];      // records (slot order / bucket input)
    Rec<D> b[4 * W];      // records in key order
    uint32_t w[4 * W];    // PERM words
    uint16_t tmp[4 * W];  // sub-bucket member lists
    uint32_t cnt[4 * W];  // sub-bucket counts, then starts (team slices of 4 T)
    uint32_t tot[W / 64]; // records per team slice
    uint32_t scan[W / 64];
    uint32_t hist[MAXB + 1];   // bucket starts of the current step
    uint32_t hist2[MAXB + 1];  // ... of the next step
    uint32_t cur[MAXB];        // scatter cursors
    uint32_t item;
    uint32_t ncarry;
};

// A team: threads [tb T, (tb + 1) T) of the workgroup, owning records
// [tb 4T, (tb + 1) 4T) and counters [tb 4T, (tb + 1) 4T).
struct Team {
    uint32_t T;     // threads (a power of two, 64 .. TPB)
    uint32_t lg;    // log2(4 T): sub-bucket bits
    uint32_t tb;    // team index
    uint32_t lt;    // thread index in the team
    uint32_t base;  // first record / counter of the team
};

__device__ __forceinline__ Team make_team(uint32_t T)
{
    Team t;
    t.T = T;
    t.lg = 33u - __clz(T);  // log2(T) + 2
    t.tb = threadIdx.x / T;
    t.lt = threadIdx.x % T;
    t.base = t.tb * 4u * T;
    return t;
}

__device__ __forceinline__ uint32_t wave_inclusive_scan_e(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

// Exclusive scan of every team's counter slice in place (thread tid owns
// counters 4 tid .. 4 tid + 3, which lie in its team's slice); the team's
// total goes to L.tot.  Ends with a barrier.
template <int D, int W>
__device__ void scan_cnt(Lds<D, W> &L, const Team &tm)
{
    const uint32_t tid = threadIdx.x;
    uint32_t v[4], sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = L.cnt[tid * 4 + k];
        sum += v[k];
    }
    const uint32_t inc = wave_inclusive_scan_e(sum);
    if ((tid & 63) == 63) L.scan[tid >> 6] = inc;
    __syncthreads();
    const uint32_t w0 = tm.tb * (tm.T >> 6), w1 = w0 + (tm.T >> 6), me = tid >> 6;
    uint32_t off = 0, total = 0;
    for (uint32_t w = w0; w < w1; ++w) {
        const uint32_t t = L.scan[w];
        if (w < me) off += t;
        total += t;
    }
    uint32_t run = off + inc - sum;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        L.cnt[tid * 4 + k] = run;
        run += v[k];
    }
    if (tm.lt == 0) L.tot[tm.tb] = total;
    __syncthreads();
}

// Order the team's records a[0..cnt) (team-relative) by the key
// (w << 32 | id), writing b[base_b + rank].  sub(w) is the sub-bucket of a
// word, monotone in w, in [0, 4 T).  Ends with a barrier.
template <int D, int W, typename SubFn>
__device__ void sort_into_b(Lds<D, W> &L, const Team &tm, uint32_t cnt, uint32_t base_b, SubFn sub)
{
    RBM_ENS_SHAPE;
    const uint32_t tid = threadIdx.x, R = tm.base;
    for (uint32_t i = tid; i < (uint32_t)S; i += TPB) L.cnt[i] = 0;
    __syncthreads();
    uint32_t msb[E], mpos[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const uint32_t e = tm.lt + k * tm.T;
        if (e < cnt) {
            msb[k] = sub(L.w[R + e]);
            mpos[k] = atomicAdd(&L.cnt[R + msb[k]], 1u);
        }
    }
    __syncthreads();
    scan_cnt<D, W>(L, tm);
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const uint32_t e = tm.lt + k * tm.T;
        if (e < cnt) L.tmp[R + L.cnt[R + msb[k]] + mpos[k]] = (uint16_t)e;
    }
    __syncthreads();
    const uint32_t top = 4u * tm.T - 1u;
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const uint32_t e = tm.lt + k * tm.T;
        if (e < cnt) {
            const uint32_t w = L.w[R + e], id = L.a[R + e].id;
            const uint32_t b0 = L.cnt[R + msb[k]];
            const uint32_t b1 = msb[k] < top ? L.cnt[R + msb[k] + 1] : L.tot[tm.tb];
            uint32_t rank = b0;
            for (uint32_t j = b0; j < b1; ++j) {
                const uint32_t t = L.tmp[R + j];
                const uint32_t wt = L.w[R + t];
                rank += (wt < w || (wt == w && L.a[R + t].id < id)) ? 1u : 0u;
            }
            L.b[R + base_b + rank] = L.a[R + e];
        }
    }
    __syncthreads();
}

// The update of the standalone step, in the same FP32 operations: the drift
// x + dt (-beta x + F), then the noise sigma sqrt(dt) z(id, m).
template <int D>
__device__ __forceinline__ void update(const StepArgs &s, float (&x)[D], const float (&f)[D], uint32_t id)
{
    drift_update<D>(s, x, f);
    StepArgs t = s;
    t.pm = s.m;
    t.pssd = s.ssd;
    add_pending_noise<D>(t, x, id);
}

// Forces and update of the batches of ranks [r0, r1) held in key order at
// src[0..): batches start at multiples of p (r0 is one); the batch of the
// last rank of a system (r1 == n) takes the leftover ranks.  Writes the
// updated record of rank r to out(r).  The team's threads share the batches.
template <int D, int KERN, int P, typename Out>
__device__ void batches(const StepArgs &s, const Team &tm, const Rec<D> *src, uint32_t r0, uint32_t r1,
                        Out out)
{
    const uint32_t p = s.p;
    const uint32_t nq = (r1 - r0) / p;  // the last batch may be longer than p
    for (uint32_t qq = tm.lt; qq < nq; qq += tm.T) {
        const uint32_t bs = r0 + qq * p;
        const bool last = (qq == nq - 1) && (r1 == s.n);
        const uint32_t sz = last ? r1 - bs : p;
        const Rec<D> *b = src + (bs - r0);
        if (P > 0 && sz == (uint32_t)P) {
            float x[P > 0 ? P : 1][D], f[P > 0 ? P : 1][D];
            uint32_t id[P > 0 ? P : 1];
#pragma unroll
            for (int i = 0; i < P; ++i) {
                const Rec<D> r = b[i];
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    x[i][c] = r.x[c];
                    f[i][c] = 0.0f;
                }
                id[i] = r.id;
            }
#pragma unroll
            for (int i = 0; i < P; ++i)
#pragma unroll
                for (int j = i + 1; j < P; ++j) {
                    constexpr int DK = kdim<D, KERN>();
                    float dx[DK], r2 = 0.0f;
#pragma unroll
                    for (int c = 0; c < DK; ++c) {
                        dx[c] = x[i][c] - x[j][c];
                        r2 = fmaf(dx[c], dx[c], r2);
                    }
                    const float sc = pair_scale<KERN>(r2, s.a);
#pragma unroll
                    for (int c = 0; c < DK; ++c) {
                        f[i][c] = fmaf(sc, dx[c], f[i][c]);
                        f[j][c] = fmaf(-sc, dx[c], f[j][c]);
                    }
                }
#pragma unroll
            for (int i = 0; i < P; ++i) {
#pragma unroll
                for (int c = 0; c < D; ++c) f[i][c] *= s.inv_p1;
                update<D>(s, x[i], f[i], id[i]);
                Rec<D> o;
#pragma unroll
                for (int c = 0; c < D; ++c) o.x[c] = x[i][c];
                o.id = id[i];
                out(bs + i, o);
            }
        } else {
            const float inv = (sz == p) ? s.inv_p1 : s.inv_last;
            for (uint32_t i = 0; i < sz; ++i) {
                const Rec<D> me = b[i];
                float xi[D], f[D];
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    xi[c] = me.x[c];
                    f[c] = 0.0f;
                }
                for (uint32_t j = 0; j < sz; ++j)
                    if (j != i) add_pair<D, KERN>(xi, b[j].x, s.a, f);
#pragma unroll
                for (int c = 0; c < D; ++c) f[c] *= inv;
                update<D>(s, xi, f, me.id);
                Rec<D> o;
#pragma unroll
                for (int c = 0; c < D; ++c) o.x[c] = xi[c];
                o.id = me.id;
                out(bs + i, o);
            }
        }
    }
}

// PERM words of 4 consecutive slots k..k+3
__device__ __forceinline__ uint4 words4(const StepArgs &s, uint32_t k)
{
    return philox4x32_10(make_uint4(k >> 2, s.m, STREAM_PERM, s.sys), s.k0, s.k1);
}

// The team's system (n <= 4 T particles, n = 0 for an idle team) in LDS for
// all steps.  Every team of the workgroup runs the same number of steps.
template <int D, int KERN, int P, int W>
__device__ void run_small(Lds<D, W> &L, const Team &tm, StepArgs s, int64_t nsteps, float *__restrict__ x)
{
    const uint32_t n = s.n, R = tm.base;
    for (uint32_t k = tm.lt; k < n; k += tm.T) {
        Rec<D> r;
#pragma unroll
        for (int c = 0; c < D; ++c) r.x[c] = x[(size_t)k * D + c];
        r.id = k;
        L.a[R + k] = r;
    }
    __syncthreads();
    const uint32_t m0 = s.m, sh = 32u - tm.lg;
    for (int64_t t = 0; t < nsteps; ++t) {
        s.m = m0 + (uint32_t)t;
        for (uint32_t k = 4 * tm.lt; k < n; k += 4 * tm.T) {
            const uint4 w = words4(s, k);
            L.w[R + k] = w.x;
            if (k + 1 < n) L.w[R + k + 1] = w.y;
            if (k + 2 < n) L.w[R + k + 2] = w.z;
            if (k + 3 < n) L.w[R + k + 3] = w.w;
        }
        __syncthreads();
        sort_into_b<D, W>(L, tm, n, 0, [sh](uint32_t w) { return w >> sh; });
        // b (key order, old positions) -> a (key order, new positions)
        if (n > 0)
            batches<D, KERN, P>(s, tm, L.b + R, 0, n, [&](uint32_t r, const Rec<D> &o) { L.a[R + r] = o; });
        __syncthreads();
    }
    for (uint32_t k = tm.lt; k < n; k += tm.T) {
        const Rec<D> r = L.a[R + k];
#pragma unroll
        for (int c = 0; c < D; ++c) x[(size_t)r.id * D + c] = r.x[c];
    }
}

// Bucket plan of step m for a streamed system: histogram of its PERM words
// over all slots (no memory read), exclusive scan into starts[0..nbk] and
// the scatter cursors L.cur.  Ends with a barrier.
template <int D, int W>
__device__ void bucket_plan(Lds<D, W> &L, StepArgs s, uint32_t m, uint32_t nbk, uint32_t *starts)
{
    RBM_ENS_SHAPE;
    const uint32_t n = s.n, tid = threadIdx.x;
    s.m = m;
    for (uint32_t i = tid; i <= nbk; i += TPB) starts[i] = 0;
    __syncthreads();
    for (uint32_t k = 4 * tid; k < n; k += 4 * TPB) {
        const uint4 w = words4(s, k);
        atomicAdd(&starts[__umulhi(w.x, nbk)], 1u);
        if (k + 1 < n) atomicAdd(&starts[__umulhi(w.y, nbk)], 1u);
        if (k + 2 < n) atomicAdd(&starts[__umulhi(w.z, nbk)], 1u);
        if (k + 3 < n) atomicAdd(&starts[__umulhi(w.w, nbk)], 1u);
    }
    __syncthreads();
    if (tid < 64) {
        // exclusive scan of nbk <= 256 counts by one wavefront
        uint32_t v[4], sum = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t i = tid * 4 + k;
            v[k] = i < nbk ? starts[i] : 0u;
            sum += v[k];
        }
        const uint32_t inc = wave_inclusive_scan_e(sum);
        uint32_t run = inc - sum;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t i = tid * 4 + k;
            if (i < nbk) {
                starts[i] = run;
                L.cur[i] = run;
            }
            run += v[k];
        }
        if (tid == 0) starts[nbk] = n;
    }
    __syncthreads();
}

// One system streamed through global memory by the whole workgroup (tm is
// the workgroup as one team).  Between steps the records sit in the bucket
// order of the next step's words, in one of two buffers: a step reads its
// buckets in order, sorts each in LDS (the batch cut by a bucket's end is
// carried to the next bucket), evaluates the batches and writes every
// updated record straight into its bucket of the next step (the next word
// of a record depends only on its rank, its next slot), so each step moves
// a record once in and once out.  The last step writes positions by id.
template <int D, int KERN, int P, int W>
__device__ void run_large(Lds<D, W> &L, const Team &tm, StepArgs s, int64_t nsteps, uint32_t bmean,
                          float *__restrict__ x, Rec<D> *__restrict__ bufA, Rec<D> *__restrict__ bufB,
                          uint32_t *__restrict__ wA, uint32_t *__restrict__ wB, uint32_t *__restrict__ flags)
{
    RBM_ENS_SHAPE;
    const uint32_t n = s.n, tid = threadIdx.x;
    const uint32_t nbk = (n + bmean - 1) / bmean;  // <= MAXB by the host's checks
    const uint32_t m0 = s.m;
    uint32_t *starts = L.hist, *next = L.hist2;
    // step m0: slot k holds particle k
    bucket_plan<D, W>(L, s, m0, nbk, starts);
    for (uint32_t k = 4 * tid; k < n; k += 4 * TPB) {
        const uint4 w = words4(s, k);
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) {
            if (k + j < n) {
                const uint32_t wj = word_of(w, j);
                const uint32_t pos = atomicAdd(&L.cur[__umulhi(wj, nbk)], 1u);
                Rec<D> r;
#pragma unroll
                for (int c = 0; c < D; ++c) r.x[c] = x[(size_t)(k + j) * D + c];
                r.id = k + j;
                bufA[pos] = r;
                wA[pos] = wj;
            }
        }
    }
    __syncthreads();
    for (int64_t t = 0; t < nsteps; ++t) {
        s.m = m0 + (uint32_t)t;
        const bool last = t == nsteps - 1;
        if (!last) bucket_plan<D, W>(L, s, s.m + 1, nbk, next);  // cursors of the next step in L.cur
        StepArgs sn = s;
        sn.m = s.m + 1;
        if (tid == 0) L.ncarry = 0;
        __syncthreads();
        for (uint32_t bk = 0; bk < nbk; ++bk) {
            const uint32_t lo = starts[bk], hi = starts[bk + 1], cnt = hi - lo;
            const uint32_t nc = L.ncarry;
            if (nc + cnt > (uint32_t)CAP) {  // far beyond any bucket's spread: flag, give up the step
                if (tid == 0) atomicOr(flags, 1u);
                break;
            }
            for (uint32_t e = tid; e < cnt; e += TPB) {
                L.a[e] = bufA[lo + e];
                L.w[e] = wA[lo + e];
            }
            __syncthreads();
            // sub-bucket: the next log2(4 W) bits of w nbk / 2^32 below the bucket
            const uint32_t sh = 32u - tm.lg;
            sort_into_b<D, W>(L, tm, cnt, nc, [nbk, sh](uint32_t w) { return (w * nbk) >> sh; });
            // L.b[0..nc) carried records (ranks lo - nc ..), then this bucket
            const uint32_t r0 = lo - nc;
            uint32_t r1;  // end of the complete batches
            if (hi == n) {
                r1 = n;
            } else {
                r1 = r0 + ((hi - r0) / s.p) * s.p;
                // the last batch of the system starts at (nbat - 1) p and runs to n
                const uint32_t last_start = (s.nbat - 1) * s.p;
                if (r1 > last_start) r1 = last_start > r0 ? last_start : r0;
            }
            // a thread emits the ranks of a batch in order: one Philox block
            // gives the next words of 4 consecutive ranks
            uint32_t wk = 0xffffffffu;
            uint4 w4 = make_uint4(0u, 0u, 0u, 0u);
            batches<D, KERN, P>(s, tm, L.b, r0, r1, [&](uint32_t r, const Rec<D> &o) {
                if (last) {
                    if (o.id < n) {
#pragma unroll
                        for (int c = 0; c < D; ++c) x[(size_t)o.id * D + c] = o.x[c];
                    }
                } else {
                    if ((r >> 2) != wk) {
                        wk = r >> 2;
                        w4 = words4(sn, r & ~3u);
                    }
                    const uint32_t wr = word_of(w4, r & 3u);
                    const uint32_t pos = atomicAdd(&L.cur[__umulhi(wr, nbk)], 1u);
                    bufB[pos] = o;
                    wB[pos] = wr;
                }
            });
            __syncthreads();
            const uint32_t keep = hi - r1;
            const uint32_t from = r1 - r0;
            Rec<D> mv[E];
#pragma unroll
            for (int k = 0; k < E; ++k) {
                const uint32_t e = tid + k * TPB;
                if (e < keep) mv[k] = L.b[from + e];
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < E; ++k) {
                const uint32_t e = tid + k * TPB;
                if (e < keep) L.b[e] = mv[k];
            }
            if (tid == 0) L.ncarry = keep;
            __syncthreads();
        }
        __syncthreads();
        // the next step reads the buffers just written, with the next starts
        Rec<D> *tb = bufA;
        bufA = bufB;
        bufB = tb;
        uint32_t *tw = wA;
        wA = wB;
        wB = tw;
        uint32_t *ts = starts;
        starts = next;
        next = ts;
    }
}

__device__ __forceinline__ StepArgs args_of(const StepArgs &base, const Sys &sy, uint32_t id)
{
    StepArgs s = base;
    s.n = sy.n;
    s.nbat = sy.n / s.p;
    s.inv_last = sy.inv_last;
    s.k0 = sy.k0;
    s.k1 = sy.k1;
    s.sys = id;
    return s;
}

template <int D, int KERN, int P, int W>
__global__ __launch_bounds__(W, 4) void k_ensemble(EnsLaunch e)
{
    RBM_ENS_SHAPE;
    __shared__ Lds<D, W> L;
    const Sys *__restrict__ sys = (const Sys *)e.sys;
    for (;;) {
        if (threadIdx.x == 0) L.item = atomicAdd(e.next, 1u);
        __syncthreads();
        const uint32_t q = L.item;
        __syncthreads();
        if (q >= e.nitems) break;  // every workgroup leaves once the queue is empty
        const uint2 it = e.items[q];  // systems order[it.x .. it.x + it.y)
        if (it.y == 1) {
            const uint32_t id = e.order[it.x];
            const Sys sy = sys[id];
            const StepArgs s = args_of(e.base, sy, id);
            float *xs = e.x + (size_t)sy.off * D;
            const Team tm = make_team(W);
            if (sy.n <= e.lds_max)
                run_small<D, KERN, P, W>(L, tm, s, e.nsteps, xs);
            else
                run_large<D, KERN, P, W>(L, tm, s, e.nsteps, e.bmean, xs, (Rec<D> *)e.state + sy.off,
                                         (Rec<D> *)e.stage + sy.off, e.wst + sy.off, e.wst2 + sy.off, e.flags);
        } else {
            const Team tm = make_team(e.team);
            // teams beyond the item's systems run an empty system in step
            Sys sy{};
            uint32_t id = 0;
            if (tm.tb < it.y) {
                id = e.order[it.x + tm.tb];
                sy = sys[id];
            }
            const StepArgs s = args_of(e.base, sy, id);
            run_small<D, KERN, P, W>(L, tm, s, e.nsteps, e.x + (size_t)sy.off * D);
        }
        __syncthreads();
    }
}

// queue counter and error flags to zero (a kernel, so that the launch can be
// recorded into a graph)
__global__ void k_zero(uint32_t *p)
{
    if (threadIdx.x < 2) p[threadIdx.x] = 0u;
}

}  // namespace ens

namespace {

template <int D, int KERN, int W>
hipError_t ens_dkw(const EnsLaunch &e, hipStream_t st)
{
    switch (e.base.p) {
    case 2: hipLaunchKernelGGL((ens::k_ensemble<D, KERN, 2, W>), dim3(e.grid), dim3(W), 0, st, e); break;
    case 4: hipLaunchKernelGGL((ens::k_ensemble<D, KERN, 4, W>), dim3(e.grid), dim3(W), 0, st, e); break;
    case 8: hipLaunchKernelGGL((ens::k_ensemble<D, KERN, 8, W>), dim3(e.grid), dim3(W), 0, st, e); break;
    default: hipLaunchKernelGGL((ens::k_ensemble<D, KERN, 0, W>), dim3(e.grid), dim3(W), 0, st, e); break;
    }
    return hipGetLastError();
}

template <int D, int KERN>
hipError_t ens_dk(const EnsLaunch &e, hipStream_t st)
{
    return e.wg == 512 ? ens_dkw<D, KERN, 512>(e, st) : ens_dkw<D, KERN, 1024>(e, st);
}

}  // namespace

hipError_t launch_ensemble(const EnsLaunch &e, int kernel, hipStream_t st)
{
    hipLaunchKernelGGL(ens::k_zero, dim3(1), dim3(64), 0, st, e.next);
    switch (kernel) {
    case K_GAUSS: return ens_dk<2, K_GAUSS>(e, st);
    case K_SOFTCOULOMB: return ens_dk<2, K_SOFTCOULOMB>(e, st);
    default: return ens_dk<2, K_ATTREP>(e, st);
    }
}

}  // namespace rbm
