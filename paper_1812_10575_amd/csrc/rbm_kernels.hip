// Kernels of the RBM-1 step (Sec. 2.1, Algorithm 1) and of the direct sum
// (eq. (1.2)) for gfx950.
//
// One step m, with the particles held as records (x, id) in "slot" order
// (the order left by the previous step):
//
//   1. k_bucket_count   every slot k draws its PERM word w_k (one Philox
//                       block feeds four consecutive slots) and counts, per
//                       tile of slots, how many words fall in each of B
//                       equal ranges of [0, 2^32) ("buckets").  No memory
//                       is read: the words depend only on (seed, m, k).
//   2. k_bucket_colscan for each bucket, exclusive prefix over tiles
//      k_bucket_starts  exclusive prefix of the bucket totals
//   3. k_bucket_scatter records move to their bucket's region (with w);
//                       order inside a bucket is left free.
//   4. k_sort_step      one workgroup per bucket: load the bucket into LDS,
//                       order it by the unique key (w << 32 | id) with a
//                       counting pass on the next bits of w plus a rank
//                       fix inside the (tiny) sub-buckets, then evaluate
//                       the batch forces of eq. (2.3) for every batch that
//                       lies inside the bucket, apply the Euler-Maruyama
//                       update and write the record at its sorted rank,
//                       which is its slot for step m+1.
//   5. k_fixup          the batches cut by a bucket boundary (at most one
//                       per boundary), one workgroup each.
//
// When N fits one workgroup's LDS, steps 1-3 and 5 vanish: a single
// workgroup sorts, steps and writes the whole system in place.
#include "rbm_device.hpp"
#include "rbm_plan.hpp"

namespace rbm {

// ---------------------------------------------------------------------------
// scans
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

// Exclusive scan of a[0..TPB*PER) in LDS, in place; returns the total.
// `tmp` holds TPB/64 words of LDS.  Ends with a barrier.
template <int TPB, int PER>
__device__ uint32_t block_exclusive_scan(uint32_t *a, uint32_t *tmp)
{
    const int tid = threadIdx.x;
    uint32_t v[PER];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        v[k] = a[tid * PER + k];
        sum += v[k];
    }
    const uint32_t inc = wave_inclusive_scan(sum);
    if ((tid & 63) == 63) tmp[tid >> 6] = inc;
    __syncthreads();
    uint32_t wave_off = 0, total = 0;
#pragma unroll
    for (int w = 0; w < TPB / 64; ++w) {
        const uint32_t t = tmp[w];
        if (w < (tid >> 6)) wave_off += t;
        total += t;
    }
    uint32_t run = wave_off + inc - sum;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        a[tid * PER + k] = run;
        run += v[k];
    }
    __syncthreads();
    return total;
}

__device__ __forceinline__ uint32_t bucket_of(uint32_t w, uint32_t nbuck)
{
    return __umulhi(w, nbuck);
}

// ---------------------------------------------------------------------------
// 1. counts of PERM words per (tile, bucket)
// ---------------------------------------------------------------------------
template <int TPB>
__global__ __launch_bounds__(TPB) void k_bucket_count(StepArgs s, uint32_t tile, uint32_t *cnt)
{
    extern __shared__ uint32_t hist[];
    const uint32_t nb = s.nbuck;
    for (uint32_t i = threadIdx.x; i < nb; i += TPB) hist[i] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * tile;
    const uint32_t end = min(base + tile, s.n);
    for (uint32_t k = base + 4 * threadIdx.x; k < end; k += 4 * TPB) {
        const uint4 w = philox4x32_10(make_uint4(k >> 2, s.m, STREAM_PERM, s.sys), s.k0, s.k1);
        atomicAdd(&hist[bucket_of(w.x, nb)], 1u);
        if (k + 1 < end) atomicAdd(&hist[bucket_of(w.y, nb)], 1u);
        if (k + 2 < end) atomicAdd(&hist[bucket_of(w.z, nb)], 1u);
        if (k + 3 < end) atomicAdd(&hist[bucket_of(w.w, nb)], 1u);
    }
    __syncthreads();
    uint32_t *row = cnt + (size_t)blockIdx.x * nb;
    for (uint32_t i = threadIdx.x; i < nb; i += TPB) row[i] = hist[i];
}

// ---------------------------------------------------------------------------
// 2. prefix sums: per bucket over tiles, then over bucket totals
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bucket_colscan(uint32_t ntiles, uint32_t nbuck,
                                                        uint32_t *cnt, uint32_t *tot)
{
    const uint32_t b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nbuck) return;
    uint32_t run = 0;
    uint32_t t = 0;
    for (; t + 4 <= ntiles; t += 4) {
        const uint32_t v0 = cnt[(size_t)(t + 0) * nbuck + b];
        const uint32_t v1 = cnt[(size_t)(t + 1) * nbuck + b];
        const uint32_t v2 = cnt[(size_t)(t + 2) * nbuck + b];
        const uint32_t v3 = cnt[(size_t)(t + 3) * nbuck + b];
        cnt[(size_t)(t + 0) * nbuck + b] = run;
        cnt[(size_t)(t + 1) * nbuck + b] = run + v0;
        cnt[(size_t)(t + 2) * nbuck + b] = run + v0 + v1;
        cnt[(size_t)(t + 3) * nbuck + b] = run + v0 + v1 + v2;
        run += v0 + v1 + v2 + v3;
    }
    for (; t < ntiles; ++t) {
        const uint32_t v = cnt[(size_t)t * nbuck + b];
        cnt[(size_t)t * nbuck + b] = run;
        run += v;
    }
    tot[b] = run;
}

// bstart[b] = sum of tot[0..b), bstart[nbuck] = N; flags bit 0 if a bucket
// exceeds the sort kernel's capacity.  One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_bucket_starts(uint32_t nbuck, uint32_t cap,
                                                        const uint32_t *tot, uint32_t *bstart,
                                                        uint32_t *flags)
{
    constexpr int TPB = 1024, PER = 16;
    __shared__ uint32_t a[TPB * PER];
    __shared__ uint32_t tmp[TPB / 64];
    bool over = false;
    for (int i = threadIdx.x; i < TPB * PER; i += TPB) {
        const uint32_t v = (uint32_t)i < nbuck ? tot[i] : 0u;
        a[i] = v;
        over |= v > cap;
    }
    __syncthreads();
    const uint32_t total = block_exclusive_scan<TPB, PER>(a, tmp);
    for (uint32_t i = threadIdx.x; i < nbuck; i += TPB) bstart[i] = a[i];
    if (threadIdx.x == 0) bstart[nbuck] = total;
    if (over) atomicOr(flags, 1u);
}

// ---------------------------------------------------------------------------
// 3. bucket scatter
// ---------------------------------------------------------------------------
template <int D, int TPB>
__global__ __launch_bounds__(TPB) void k_bucket_scatter(StepArgs s, uint32_t tile,
                                                        const Rec<D> *__restrict__ state,
                                                        Rec<D> *__restrict__ stage,
                                                        uint32_t *__restrict__ wout,
                                                        const uint32_t *__restrict__ cnt,
                                                        const uint32_t *__restrict__ bstart)
{
    extern __shared__ uint32_t cur[];
    const uint32_t nb = s.nbuck;
    const uint32_t *row = cnt + (size_t)blockIdx.x * nb;
    for (uint32_t i = threadIdx.x; i < nb; i += TPB) cur[i] = bstart[i] + row[i];
    __syncthreads();
    const uint32_t base = blockIdx.x * tile;
    const uint32_t end = min(base + tile, s.n);
    auto place = [&](const Rec<D> &r, uint32_t w) {
        const uint32_t pos = atomicAdd(&cur[bucket_of(w, nb)], 1u);
        stage[pos] = r;
        wout[pos] = w;
    };
    for (uint32_t k = base + 4 * threadIdx.x; k < end; k += 4 * TPB) {
        const uint4 w4 = philox4x32_10(make_uint4(k >> 2, s.m, STREAM_PERM, s.sys), s.k0, s.k1);
        if (k + 4 <= end) {
            const Rec<D> r0 = state[k], r1 = state[k + 1], r2 = state[k + 2], r3 = state[k + 3];
            place(r0, w4.x);
            place(r1, w4.y);
            place(r2, w4.z);
            place(r3, w4.w);
        } else {
            for (uint32_t j = 0; k + j < end; ++j) place(state[k + j], word_of(w4, j));
        }
    }
}

// ---------------------------------------------------------------------------
// 4. per-bucket sort + batch force + Euler-Maruyama
// ---------------------------------------------------------------------------
// SINGLE: the whole system is one bucket read from the slot-ordered state;
// the PERM words are drawn here.  fout != nullptr: forces only (written by
// id, state untouched; dst receives only the records the fix-up needs).
template <int D, int KERN, bool SINGLE, int TPB, int CAP, int SBITS>
__global__ __launch_bounds__(TPB) void k_sort_step(StepArgs s, const Rec<D> *src,
                                                   const uint32_t *__restrict__ wsrc,
                                                   const uint32_t *__restrict__ bstart,
                                                   Rec<D> *dst, float *__restrict__ fout,
                                                   uint32_t *__restrict__ flags)
{
    constexpr int S = 1 << SBITS;
    constexpr int E = (CAP + TPB - 1) / TPB;
    static_assert(S % TPB == 0, "sub-bucket count must be a multiple of the block");
    __shared__ Rec<D> rec[CAP];
    __shared__ uint32_t wv[CAP];
    __shared__ uint32_t cnt[S + 1];
    __shared__ uint16_t tmp[CAP];
    __shared__ uint16_t ord[CAP];
    __shared__ uint32_t scan_tmp[TPB / 64];

    const uint32_t tid = threadIdx.x;
    uint32_t lo, hi;
    if constexpr (SINGLE) {
        lo = 0;
        hi = s.n;
    } else {
        lo = bstart[blockIdx.x];
        hi = bstart[blockIdx.x + 1];
    }
    const uint32_t nb = hi - lo;
    if (nb == 0) return;
    if (nb > (uint32_t)CAP) {
        if (tid == 0) atomicOr(flags, 1u);
        return;
    }

    for (uint32_t i = tid; i <= (uint32_t)S; i += TPB) cnt[i] = 0;
    __syncthreads();

    // load, draw/fetch the PERM word, count per sub-bucket
    uint32_t my_sb[E], my_pos[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const uint32_t e = tid + k * TPB;
        if (e < nb) {
            rec[e] = src[lo + e];
            uint32_t w;
            if constexpr (SINGLE) {
                const uint4 b4 = philox4x32_10(make_uint4(e >> 2, s.m, STREAM_PERM, s.sys), s.k0, s.k1);
                w = word_of(b4, e & 3u);
            } else {
                w = wsrc[lo + e];
            }
            wv[e] = w;
            const uint32_t sb = (w * s.nbuck) >> (32 - SBITS);
            my_sb[k] = sb;
            my_pos[k] = atomicAdd(&cnt[sb], 1u);
        }
    }
    __syncthreads();
    const uint32_t total = block_exclusive_scan<TPB, S / TPB>(cnt, scan_tmp);
    if (tid == 0) cnt[S] = total;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const uint32_t e = tid + k * TPB;
        if (e < nb) tmp[cnt[my_sb[k]] + my_pos[k]] = (uint16_t)e;
    }
    __syncthreads();
    // exact rank: position of the sub-bucket plus the members with smaller key
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const uint32_t e = tid + k * TPB;
        if (e < nb) {
            const uint32_t w = wv[e];
            const uint32_t id = rec[e].id;
            const uint32_t b0 = cnt[my_sb[k]], b1 = cnt[my_sb[k] + 1];
            uint32_t rank = b0;
            for (uint32_t j = b0; j < b1; ++j) {
                const uint32_t t = tmp[j];
                const uint32_t wt = wv[t];
                rank += (wt < w || (wt == w && rec[t].id < id)) ? 1u : 0u;
            }
            ord[rank] = (uint16_t)e;
        }
    }
    __syncthreads();

    // batches inside the bucket: force, update, write at the sorted rank
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const uint32_t l = tid + k * TPB;
        if (l < nb) {
            const uint32_t r = lo + l;
            const Rec<D> me = rec[ord[l]];
            uint32_t bs, be;
            batch_of(s, r, bs, be);
            if (bs >= lo && be <= hi) {
                float xi[D], f[D];
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    xi[c] = me.x[c];
                    f[c] = 0.0f;
                }
                for (uint32_t j = bs; j < be; ++j)
                    if (j != r) add_pair<D, KERN>(xi, rec[ord[j - lo]].x, s.a, f);
                const float inv = 1.0f / (float)(be - bs - 1);
#pragma unroll
                for (int c = 0; c < D; ++c) f[c] *= inv;
                if (fout) {
#pragma unroll
                    for (int c = 0; c < D; ++c) fout[(size_t)me.id * D + c] = f[c];
                } else {
                    em_update<D>(s, xi, f, me.id);
                    Rec<D> o;
#pragma unroll
                    for (int c = 0; c < D; ++c) o.x[c] = xi[c];
                    o.id = me.id;
                    dst[r] = o;
                }
            } else {
                dst[r] = me;  // batch cut by a bucket boundary: k_fixup completes it
            }
        }
    }
}

// ---------------------------------------------------------------------------
// 5. batches cut by bucket boundaries
// ---------------------------------------------------------------------------
// Workgroup b-1 looks at the boundary at rank bstart[b].  The batch around it
// is cut if the boundary is not the batch's first rank; of several
// boundaries inside one batch only the first handles it.
template <int D, int KERN>
__global__ __launch_bounds__(128) void k_fixup(StepArgs s, const uint32_t *__restrict__ bstart,
                                               Rec<D> *dst, float *__restrict__ fout)
{
    const uint32_t b = blockIdx.x + 1;
    const uint32_t r = bstart[b];
    if (r == 0 || r >= s.n) return;
    uint32_t bs, be;
    batch_of(s, r, bs, be);
    if (r == bs) return;
    if (bstart[b - 1] > bs) return;
    __shared__ Rec<D> sh[128];
    const uint32_t sz = be - bs;
    const uint32_t tid = threadIdx.x;
    if (tid < sz) sh[tid] = dst[bs + tid];
    __syncthreads();
    if (tid < sz) {
        const Rec<D> me = sh[tid];
        float xi[D], f[D];
#pragma unroll
        for (int c = 0; c < D; ++c) {
            xi[c] = me.x[c];
            f[c] = 0.0f;
        }
        for (uint32_t j = 0; j < sz; ++j)
            if (j != tid) add_pair<D, KERN>(xi, sh[j].x, s.a, f);
        const float inv = 1.0f / (float)(sz - 1);
#pragma unroll
        for (int c = 0; c < D; ++c) f[c] *= inv;
        if (fout) {
#pragma unroll
            for (int c = 0; c < D; ++c) fout[(size_t)me.id * D + c] = f[c];
        } else {
            em_update<D>(s, xi, f, me.id);
            Rec<D> o;
#pragma unroll
            for (int c = 0; c < D; ++c) o.x[c] = xi[c];
            o.id = me.id;
            dst[bs + tid] = o;
        }
    }
}

// ---------------------------------------------------------------------------
// layout conversion
// ---------------------------------------------------------------------------
// flags bit 1: a caller-supplied slot id was >= N (it is replaced by the
// slot index so that nothing outside x0 is read).
template <int D>
__global__ __launch_bounds__(256) void k_init_state(uint32_t n, const float *__restrict__ x0,
                                                    const uint32_t *__restrict__ slots,
                                                    Rec<D> *__restrict__ state,
                                                    uint32_t *__restrict__ flags)
{
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    uint32_t id = slots ? slots[k] : k;
    if (id >= n) {
        atomicOr(flags, 2u);
        id = k;
    }
    Rec<D> r;
#pragma unroll
    for (int c = 0; c < D; ++c) r.x[c] = x0[(size_t)id * D + c];
    r.id = id;
    state[k] = r;
}

template <int D>
__global__ __launch_bounds__(256) void k_positions(uint32_t n, const Rec<D> *__restrict__ state,
                                                   float *__restrict__ x, uint32_t *__restrict__ ids)
{
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const Rec<D> r = state[k];
    if (x) {
#pragma unroll
        for (int c = 0; c < D; ++c) x[(size_t)r.id * D + c] = r.x[c];
    }
    if (ids) ids[k] = r.id;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t n, uint32_t v)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// direct sum: F_i = 1/(N-1) sum_{j != i} K(X_i - X_j), LDS tiles of j, FP32
// pair terms summed per tile, FP64 across tiles.  step: apply the update.
// ---------------------------------------------------------------------------
template <int D, int KERN, int TPB>
__global__ __launch_bounds__(TPB) void k_direct(StepArgs s, const float *__restrict__ x,
                                                const uint32_t *__restrict__ ids, uint32_t nids,
                                                float *__restrict__ out, int step)
{
    __shared__ float tile[TPB * D];
    const uint32_t t = blockIdx.x * TPB + threadIdx.x;
    const bool active = t < nids;
    uint32_t i = active ? (ids ? ids[t] : t) : 0u;
    const bool valid = i < s.n;  // an id >= N yields NaN forces instead of a wild read
    if (!valid) i = 0;
    float xi[D];
#pragma unroll
    for (int c = 0; c < D; ++c) xi[c] = x[(size_t)i * D + c];
    double acc[D];
#pragma unroll
    for (int c = 0; c < D; ++c) acc[c] = 0.0;
    for (uint32_t base = 0; base < s.n; base += TPB) {
        __syncthreads();
        const uint32_t j = base + threadIdx.x;
        if (j < s.n) {
#pragma unroll
            for (int c = 0; c < D; ++c) tile[threadIdx.x * D + c] = x[(size_t)j * D + c];
        }
        __syncthreads();
        const uint32_t cntj = min((uint32_t)TPB, s.n - base);
        float part[D];
#pragma unroll
        for (int c = 0; c < D; ++c) part[c] = 0.0f;
        for (uint32_t jj = 0; jj < cntj; ++jj) {
            float dx[D];
            float r2 = 0.0f;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                dx[c] = xi[c] - tile[jj * D + c];
                r2 = fmaf(dx[c], dx[c], r2);
            }
            float sc = pair_scale<KERN>(r2, s.a);
            sc = (base + jj == i) ? 0.0f : sc;
#pragma unroll
            for (int c = 0; c < D; ++c) part[c] = fmaf(sc, dx[c], part[c]);
        }
#pragma unroll
        for (int c = 0; c < D; ++c) acc[c] += (double)part[c];
    }
    if (!active) return;
    float f[D];
    const double inv = 1.0 / (double)(s.n - 1);
#pragma unroll
    for (int c = 0; c < D; ++c) f[c] = valid ? (float)(acc[c] * inv) : __builtin_nanf("");
    if (!step) {
#pragma unroll
        for (int c = 0; c < D; ++c) out[(size_t)t * D + c] = f[c];
    } else {
        em_update<D>(s, xi, f, i);
#pragma unroll
        for (int c = 0; c < D; ++c) out[(size_t)i * D + c] = xi[c];
    }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
namespace {

constexpr int SORT_TPB = 512;
constexpr int SORT_CAP = RBM_SORT_CAP;
constexpr int SORT_SBITS = 11;
constexpr int COUNT_TPB = 1024;
constexpr int SCATTER_TPB = 1024;
constexpr int DIRECT_TPB = 256;

hipError_t last()
{
    return hipGetLastError();
}

inline void mark(hipEvent_t *ev, int i, hipStream_t st)
{
    if (ev) (void)hipEventRecord(ev[i], st);
}

template <int D, int KERN>
hipError_t step_dk(const Plan &pl, const StepArgs &s, void *ws, hipStream_t st, void *dst_state,
                   float *fout, hipEvent_t *ev)
{
    auto *state = reinterpret_cast<Rec<D> *>((char *)ws + pl.off_state);
    auto *dst = reinterpret_cast<Rec<D> *>(dst_state);
    auto *flags = reinterpret_cast<uint32_t *>((char *)ws + pl.off_flags);
    if (pl.nbuck == 1) {
        for (int i = 0; i <= 4; ++i) mark(ev, i, st);
        hipLaunchKernelGGL((k_sort_step<D, KERN, true, SORT_TPB, SORT_CAP, SORT_SBITS>), dim3(1),
                           dim3(SORT_TPB), 0, st, s, state, nullptr, nullptr, dst, fout, flags);
        mark(ev, 5, st);
        mark(ev, 6, st);
        return last();
    }
    auto *stage = reinterpret_cast<Rec<D> *>((char *)ws + pl.off_stage);
    auto *wbuf = reinterpret_cast<uint32_t *>((char *)ws + pl.off_w);
    auto *cnt = reinterpret_cast<uint32_t *>((char *)ws + pl.off_cnt);
    auto *tot = reinterpret_cast<uint32_t *>((char *)ws + pl.off_tot);
    auto *bstart = reinterpret_cast<uint32_t *>((char *)ws + pl.off_bstart);
    const size_t lds = (size_t)pl.nbuck * sizeof(uint32_t);
    mark(ev, 0, st);
    hipLaunchKernelGGL((k_bucket_count<COUNT_TPB>), dim3(pl.ntiles), dim3(COUNT_TPB), lds, st, s,
                       pl.tile, cnt);
    mark(ev, 1, st);
    hipLaunchKernelGGL(k_bucket_colscan, dim3((pl.nbuck + 255) / 256), dim3(256), 0, st,
                       pl.ntiles, pl.nbuck, cnt, tot);
    mark(ev, 2, st);
    hipLaunchKernelGGL(k_bucket_starts, dim3(1), dim3(1024), 0, st, pl.nbuck, (uint32_t)SORT_CAP,
                       tot, bstart, flags);
    mark(ev, 3, st);
    hipLaunchKernelGGL((k_bucket_scatter<D, SCATTER_TPB>), dim3(pl.ntiles), dim3(SCATTER_TPB), lds,
                       st, s, pl.tile, state, stage, wbuf, cnt, bstart);
    mark(ev, 4, st);
    hipLaunchKernelGGL((k_sort_step<D, KERN, false, SORT_TPB, SORT_CAP, SORT_SBITS>),
                       dim3(pl.nbuck), dim3(SORT_TPB), 0, st, s, stage, wbuf, bstart, dst, fout,
                       flags);
    mark(ev, 5, st);
    hipLaunchKernelGGL((k_fixup<D, KERN>), dim3(pl.nbuck - 1), dim3(128), 0, st, s, bstart, dst,
                       fout);
    mark(ev, 6, st);
    return last();
}

template <int D>
hipError_t step_d(const Plan &pl, const StepArgs &s, int kernel, void *ws, hipStream_t st,
                  void *dst, float *fout, hipEvent_t *ev)
{
    switch (kernel) {
    case K_GAUSS: return step_dk<D, K_GAUSS>(pl, s, ws, st, dst, fout, ev);
    case K_SOFTCOULOMB: return step_dk<D, K_SOFTCOULOMB>(pl, s, ws, st, dst, fout, ev);
    default: return step_dk<D, K_ATTREP>(pl, s, ws, st, dst, fout, ev);
    }
}

template <int D, int KERN>
hipError_t direct_dk(const StepArgs &s, const float *x, const uint32_t *ids, uint32_t nids,
                     float *out, int step, hipStream_t st)
{
    hipLaunchKernelGGL((k_direct<D, KERN, DIRECT_TPB>), dim3((nids + DIRECT_TPB - 1) / DIRECT_TPB),
                       dim3(DIRECT_TPB), 0, st, s, x, ids, nids, out, step);
    return last();
}

template <int D>
hipError_t direct_d(const StepArgs &s, int kernel, const float *x, const uint32_t *ids,
                    uint32_t nids, float *out, int step, hipStream_t st)
{
    switch (kernel) {
    case K_GAUSS: return direct_dk<D, K_GAUSS>(s, x, ids, nids, out, step, st);
    case K_SOFTCOULOMB: return direct_dk<D, K_SOFTCOULOMB>(s, x, ids, nids, out, step, st);
    default: return direct_dk<D, K_ATTREP>(s, x, ids, nids, out, step, st);
    }
}

}  // namespace

hipError_t launch_step(const Plan &pl, const StepArgs &s, int d, int kernel, void *ws,
                       hipStream_t st, void *dst_state, float *fout, hipEvent_t *ev)
{
    switch (d) {
    case 1: return step_d<1>(pl, s, kernel, ws, st, dst_state, fout, ev);
    case 2: return step_d<2>(pl, s, kernel, ws, st, dst_state, fout, ev);
    default: return step_d<3>(pl, s, kernel, ws, st, dst_state, fout, ev);
    }
}

hipError_t launch_init(const Plan &pl, int d, const float *x0, const uint32_t *slots, void *ws,
                       hipStream_t st)
{
    void *state = (char *)ws + pl.off_state;
    auto *flags = reinterpret_cast<uint32_t *>((char *)ws + pl.off_flags);
    const dim3 g((pl.n + 255) / 256);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, flags, 16u, 0u);
    switch (d) {
    case 1: hipLaunchKernelGGL(k_init_state<1>, g, dim3(256), 0, st, pl.n, x0, slots, (Rec<1> *)state, flags); break;
    case 2: hipLaunchKernelGGL(k_init_state<2>, g, dim3(256), 0, st, pl.n, x0, slots, (Rec<2> *)state, flags); break;
    default: hipLaunchKernelGGL(k_init_state<3>, g, dim3(256), 0, st, pl.n, x0, slots, (Rec<3> *)state, flags); break;
    }
    return last();
}

hipError_t launch_positions(const Plan &pl, int d, const void *ws, float *x, uint32_t *ids,
                            hipStream_t st)
{
    const void *state = (const char *)ws + pl.off_state;
    const dim3 g((pl.n + 255) / 256);
    switch (d) {
    case 1: hipLaunchKernelGGL(k_positions<1>, g, dim3(256), 0, st, pl.n, (const Rec<1> *)state, x, ids); break;
    case 2: hipLaunchKernelGGL(k_positions<2>, g, dim3(256), 0, st, pl.n, (const Rec<2> *)state, x, ids); break;
    default: hipLaunchKernelGGL(k_positions<3>, g, dim3(256), 0, st, pl.n, (const Rec<3> *)state, x, ids); break;
    }
    return last();
}

hipError_t launch_direct(const StepArgs &s, int d, int kernel, const float *x, const uint32_t *ids,
                         uint32_t nids, float *out, int step, hipStream_t st)
{
    switch (d) {
    case 1: return direct_d<1>(s, kernel, x, ids, nids, out, step, st);
    case 2: return direct_d<2>(s, kernel, x, ids, nids, out, step, st);
    default: return direct_d<3>(s, kernel, x, ids, nids, out, step, st);
    }
}

}  // namespace rbm
