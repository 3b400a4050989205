// RBM-r (Sec. 2.2, Algorithm RBM-r) on the GPU.
//
// The method is sequential: iteration k moves the p particles of its batch
// C_k, starting from the positions the earlier iterations left.  Iterations
// whose batches are disjoint commute, so a window of W consecutive
// iterations runs in rounds: round L runs the iterations whose longest chain
// of predecessors inside the window (an earlier iteration sharing a
// particle, its own predecessors, ...) has L links.  Each iteration then
// starts from exactly the positions the sequential order gives it, so the
// result depends neither on the window nor on the rounds (bit for bit: an
// iteration's arithmetic is the same wherever it runs).
//
// The schedule of a window comes from one bucket sort of its p W member
// entries (entry j = e p + r: member r of the iteration at offset e), with
// no atomic operation on particle data:
//   k_rbmr_count    draws every batch and counts the entries per bucket of
//                   2^bsh consecutive particles, per workgroup (LDS)
//   k_rbmr_offsets  per bucket, the exclusive scan of those counts over the
//                   workgroups, and the bucket's total
//   k_rbmr_scatter  draws again and writes each entry (j, member) into its
//                   bucket's segment (and the bucket starts)
//   k_rbmr_lists    per bucket, each particle's entries in iteration order:
//                   succ[j] = the particle's next iteration after entry j's
//                   (NONE after its last), and the particle's record gets
//                   its first one as head
//   k_rbmr_round    round L over the pending iterations (all of them for
//                   L = 0, else the queue of round L - 1): an iteration
//                   runs when every member's record names it as head and
//                   was written before round L, and stores each updated
//                   record with head succ; the others queue themselves
//                   (one atomic add per workgroup and pass, on the length
//                   of one of NSEG queue segments chosen by the workgroup:
//                   a single queue counter, taking an add from every
//                   wavefront, made the first round four times as slow:
//                   adds to one address are carried out one at a time)
//   k_rbmr_finish   one workgroup continues the rounds for what is pending
//                   after the last multi-workgroup round (a window of N/2
//                   random pairs has depth 11 to 13, and after 8 rounds
//                   about 0.03 % of its iterations are left), then runs
//                   anything still pending in iteration order
// A particle record is {tag, position} in 16 bytes, tag = (f << 23) | head:
// head is the next iteration of the window that touches the particle (NONE
// = 2^23 - 1 once none is left) and f is 1 + the round that last wrote the
// record (0 before any).  Only the iteration named by head writes a record,
// so the rounds need plain loads and stores.  An iteration whose
// predecessor on a particle runs in the same round L either reads the old
// head (another iteration) or the new record with f = L + 1: it waits for
// the next round either way, so its positions are always those of finished
// rounds.  Batches are drawn again from the counter wherever they are
// needed (a few ALU operations instead of a stored table read at random).
#include <hip/hip_runtime.h>

#include "rbm_rbmr.hpp"

namespace rbm {
namespace {

constexpr int TPB = 256;   // rounds, bucket offsets
constexpr int STPB = 1024; // bucket count, scatter, lists
constexpr int FIN_TPB = 1024;
constexpr uint32_t FIN_BUDGET = 64;  // single-workgroup rounds before the ordered rest
constexpr uint32_t HEAD_BITS = 23;
constexpr uint32_t HEAD_MASK = (1u << HEAD_BITS) - 1u;
constexpr uint32_t NONE = HEAD_MASK;
constexpr uint32_t NSEG = 256;  // queue segments per round
enum : uint32_t { STREAM_RBMR_DRAW = 2u, STREAM_RBMR_NOISE = 3u };

static_assert(RBMR_MAX_WINDOW <= NONE, "iteration offsets must stay below NONE");
static_assert(RBMR_MAX_ROUNDS + FIN_BUDGET + 1u < (1u << (32 - HEAD_BITS)), "round field too narrow");
static_assert(NSEG % 64 == 0, "queue segments per lane");
static_assert(RBMR_MAX_NBK == 8 * STPB && RBMR_MAX_PB == 4 * STPB && RBMR_MAX_NBLK == 4 * 64,
              "per-thread shares of the scans");

__device__ __forceinline__ uint32_t tag_of(uint32_t f, uint32_t head)
{
    return (f << HEAD_BITS) | head;
}

// iteration e may run in round L on this member
__device__ __forceinline__ bool ready_for(uint32_t tag, uint32_t e, uint32_t L)
{
    return (tag & HEAD_MASK) == e && (tag >> HEAD_BITS) <= L;
}

struct alignas(16) RRec {
    uint32_t tag;
    float x[3];
};

__device__ __forceinline__ uint4 rbmr_block(const RbmrArgs &a, uint64_t k, uint32_t sub, uint32_t stream)
{
    return philox4x32_10(make_uint4((uint32_t)k, (uint32_t)(k >> 32) | (sub << 16), stream, a.sys), a.k0, a.k1);
}

// Members of iteration k in draw order: member r takes the 64-bit word
// U_r, v = floor(U_r (N - r) / 2^64), and becomes the v-th smallest
// particle not drawn yet (a uniformly random ordered p-subset).
__device__ __forceinline__ void draw_members(const RbmrArgs &a, uint64_t k, uint32_t (&m)[RBMR_MAX_P])
{
    uint32_t srt[RBMR_MAX_P];
    uint4 w = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
    for (int r = 0; r < RBMR_MAX_P; ++r) {
        if (r < (int)a.p) {
            if ((r & 1) == 0) w = rbmr_block(a, k, (uint32_t)(r >> 1), STREAM_RBMR_DRAW);
            const uint64_t u = (r & 1) == 0 ? ((uint64_t)w.y << 32) | w.x : ((uint64_t)w.w << 32) | w.z;
            uint32_t v = (uint32_t)__umul64hi(u, (uint64_t)(a.n - (uint32_t)r));
#pragma unroll
            for (int q = 0; q < RBMR_MAX_P - 1; ++q)
                if (q < r && srt[q] <= v) ++v;
            m[r] = v;
            uint32_t cur = v;  // insert into the sorted list
#pragma unroll
            for (int q = 0; q < RBMR_MAX_P; ++q) {
                if (q < r) {
                    if (srt[q] > cur) {
                        const uint32_t t = srt[q];
                        srt[q] = cur;
                        cur = t;
                    }
                } else if (q == r) {
                    srt[q] = cur;
                }
            }
        }
    }
}

template <int D>
__device__ __forceinline__ void rbmr_noise(const RbmrArgs &a, uint64_t k, uint32_t r, float (&z)[D])
{
    const uint4 w = rbmr_block(a, k, r, STREAM_RBMR_NOISE);
    float b0, b1;
    box_muller(u24(w.x), u24(w.y), b0, b1);
    z[0] = b0;
    if constexpr (D >= 2) z[1] = b1;
    if constexpr (D >= 3) {
        float c, e;
        box_muller(u24(w.z), u24(w.w), c, e);
        z[2] = c;
    }
}

// Iteration k on its members: forces at the positions it starts from, one
// Euler-Maruyama step of the batch SDE (SPLIT: the exact pair flow of
// K = x/|x|^2, then the field step), then the noise of its slots.  Each
// updated record is stored whole, with the tag (f, nx[r]).
template <int D, int KERN, bool SPLIT>
__device__ __forceinline__ void run_iteration(const RbmrArgs &a, uint64_t k, const uint32_t (&m)[RBMR_MAX_P],
                                              const float (&xs)[RBMR_MAX_P][D], const uint32_t (&nx)[RBMR_MAX_P],
                                              uint32_t f, RRec *rec)
{
    float y[RBMR_MAX_P][D];
    if constexpr (SPLIT) {
        pair_flow<D>(a.dt, xs[0], xs[1], y[0]);
        pair_flow<D>(a.dt, xs[1], xs[0], y[1]);
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int c = 0; c < D; ++c) y[r][c] = fmaf(a.dt, -a.beta * y[r][c], y[r][c]);
    } else {
#pragma unroll
        for (int r = 0; r < RBMR_MAX_P; ++r) {
            if (r < (int)a.p) {
                float fr[D];
#pragma unroll
                for (int c = 0; c < D; ++c) fr[c] = 0.0f;
#pragma unroll
                for (int q = 0; q < RBMR_MAX_P; ++q)
                    if (q < (int)a.p && q != r) add_pair<D, KERN>(xs[r], xs[q], a.a, fr);
#pragma unroll
                for (int c = 0; c < D; ++c) y[r][c] = fmaf(a.dt, fmaf(-a.beta, xs[r][c], fr[c] * a.inv_p1), xs[r][c]);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RBMR_MAX_P; ++r)
        if (r < (int)a.p) {
            if (a.ssd != 0.0f) {
                float z[D];
                rbmr_noise<D>(a, k, (uint32_t)r, z);
#pragma unroll
                for (int c = 0; c < D; ++c) y[r][c] = fmaf(a.ssd, z[c], y[r][c]);
            }
            const uint4 v = make_uint4(tag_of(f, nx[r]), __float_as_uint(y[r][0]),
                                       D >= 2 ? __float_as_uint(y[r][D >= 2 ? 1 : 0]) : 0u,
                                       D >= 3 ? __float_as_uint(y[r][D >= 3 ? 2 : 0]) : 0u);
            *reinterpret_cast<uint4 *>(&rec[m[r]]) = v;
        }
}

// The members' records (tag, position) and the successors of the
// iteration's entries, all loads issued before any is used.
template <int D>
__device__ __forceinline__ void load_iteration(const RbmrArgs &a, uint32_t e, const RRec *rec, const uint32_t *succ,
                                               const uint32_t (&m)[RBMR_MAX_P], uint32_t (&tag)[RBMR_MAX_P],
                                               float (&xs)[RBMR_MAX_P][D], uint32_t (&nx)[RBMR_MAX_P])
{
    uint4 v[RBMR_MAX_P];
#pragma unroll
    for (int r = 0; r < RBMR_MAX_P; ++r)
        if (r < (int)a.p) {
            v[r] = *reinterpret_cast<const uint4 *>(&rec[m[r]]);
            nx[r] = succ[(size_t)e * a.p + (uint32_t)r];
        }
#pragma unroll
    for (int r = 0; r < RBMR_MAX_P; ++r)
        if (r < (int)a.p) {
            tag[r] = v[r].x;
            xs[r][0] = __uint_as_float(v[r].y);
            if constexpr (D >= 2) xs[r][D >= 2 ? 1 : 0] = __uint_as_float(v[r].z);
            if constexpr (D >= 3) xs[r][D >= 3 ? 2 : 0] = __uint_as_float(v[r].w);
        }
}

template <int D>
__global__ __launch_bounds__(TPB) void k_rbmr_pack(uint32_t n, const float *__restrict__ x, RRec *__restrict__ rec)
{
    const uint32_t i = blockIdx.x * TPB + threadIdx.x;
    if (i >= n) return;
    RRec r{};
#pragma unroll
    for (int c = 0; c < D; ++c) r.x[c] = x[(size_t)i * D + c];
    rec[i] = r;
}

template <int D>
__global__ __launch_bounds__(TPB) void k_rbmr_unpack(uint32_t n, const RRec *__restrict__ rec, float *__restrict__ x)
{
    const uint32_t i = blockIdx.x * TPB + threadIdx.x;
    if (i >= n) return;
    const RRec r = rec[i];
#pragma unroll
    for (int c = 0; c < D; ++c) x[(size_t)i * D + c] = r.x[c];
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

// Exclusive scan of v[0 .. nv) (nv <= 8 STPB, 8 consecutive values per
// thread) into out[0 .. nv) (LDS), plus row[i] when row is not NULL.
// Needs STPB threads; ends with a barrier.
__device__ void block_scan8(const uint32_t *__restrict__ v, uint32_t nv, const uint32_t *__restrict__ row,
                            uint32_t *out, uint32_t *wsum)
{
    constexpr int PER = 8;
    const uint32_t t = threadIdx.x, i0 = t * PER;
    uint32_t u[PER], w[PER], s = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        u[q] = i0 + q < nv ? v[i0 + q] : 0u;
        w[q] = row && i0 + q < nv ? row[i0 + q] : 0u;
        s += u[q];
    }
    const uint32_t inc = wave_incl_scan(s);
    if ((t & 63) == 63) wsum[t >> 6] = inc;
    __syncthreads();
    uint32_t run = inc - s;
    for (uint32_t k = 0; k < (t >> 6); ++k) run += wsum[k];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        if (i0 + q < nv) out[i0 + q] = run + w[q];
        run += u[q];
    }
    __syncthreads();
}

// Entries per bucket of the iterations [blk ipb, (blk + 1) ipb) of the
// window: cnt[blk][bucket] (workgroup-major).
__global__ __launch_bounds__(STPB) void k_rbmr_count(RbmrArgs a, uint64_t kbase, uint32_t wcur, uint32_t ipb,
                                                     uint32_t bsh, uint32_t nbk, uint32_t *__restrict__ cnt)
{
    __shared__ uint32_t h[RBMR_MAX_NBK];
    for (uint32_t i = threadIdx.x; i < nbk; i += STPB) h[i] = 0u;
    __syncthreads();
    const uint32_t e0 = blockIdx.x * ipb, e1 = min(e0 + ipb, wcur);
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += STPB) {
        uint32_t m[RBMR_MAX_P];
        draw_members(a, kbase + e, m);
#pragma unroll
        for (int r = 0; r < RBMR_MAX_P; ++r)
            if (r < (int)a.p) atomicAdd(&h[m[r] >> bsh], 1u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nbk; i += STPB) cnt[(size_t)blockIdx.x * nbk + i] = h[i];
}

// One wavefront per bucket: cnt[.][bucket] becomes the exclusive scan over
// the workgroups (each lane takes 4 consecutive ones), tot[bucket] the sum.
__global__ __launch_bounds__(TPB) void k_rbmr_offsets(uint32_t nbk, uint32_t nblk, uint32_t *__restrict__ cnt,
                                                      uint32_t *__restrict__ tot)
{
    constexpr int PER = RBMR_MAX_NBLK / 64;
    const uint32_t bk = blockIdx.x * (TPB / 64) + (threadIdx.x >> 6);
    if (bk >= nbk) return;  // the whole wavefront
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t v[PER], s = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const uint32_t b = lane * PER + q;
        v[q] = b < nblk ? cnt[(size_t)b * nbk + bk] : 0u;
        s += v[q];
    }
    const uint32_t inc = wave_incl_scan(s);
    uint32_t run = inc - s;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const uint32_t b = lane * PER + q;
        if (b < nblk) cnt[(size_t)b * nbk + bk] = run;
        run += v[q];
    }
    if (lane == 63u) tot[bk] = inc;
}

// The entries of the workgroup's iterations into their buckets' segments
// (bucket starts: the scan of the totals, which workgroup 0 also stores to
// bst; the workgroup's place in each bucket: its row of cnt).
__global__ __launch_bounds__(STPB) void k_rbmr_scatter(RbmrArgs a, uint64_t kbase, uint32_t wcur, uint32_t ipb,
                                                       uint32_t bsh, uint32_t nbk, const uint32_t *__restrict__ cnt,
                                                       const uint32_t *__restrict__ tot, uint2 *__restrict__ ent,
                                                       uint32_t *__restrict__ bst)
{
    __shared__ uint32_t pos[RBMR_MAX_NBK];
    __shared__ uint32_t wsum[STPB / 64];
    block_scan8(tot, nbk, cnt + (size_t)blockIdx.x * nbk, pos, wsum);
    if (blockIdx.x == 0)  // its row of cnt is all zeros: pos holds the starts
        for (uint32_t i = threadIdx.x; i < nbk; i += STPB) bst[i] = pos[i];
    const uint32_t e0 = blockIdx.x * ipb, e1 = min(e0 + ipb, wcur);
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += STPB) {
        uint32_t m[RBMR_MAX_P];
        draw_members(a, kbase + e, m);
#pragma unroll
        for (int r = 0; r < RBMR_MAX_P; ++r)
            if (r < (int)a.p) {
                const uint32_t at = atomicAdd(&pos[m[r] >> bsh], 1u);
                ent[at] = make_uint2(e * a.p + (uint32_t)r, m[r]);
            }
    }
}

// The entries of one particle, l[0 .. c), sorted by entry (that is, by
// iteration: a particle is in a batch at most once), the particle's first
// iteration as the head of its record and every entry's successor.
template <typename P>
__device__ __forceinline__ void particle_list(P *l, uint32_t c, uint32_t p, uint32_t *__restrict__ succ,
                                              uint32_t &head)
{
    head = NONE;
    if (c <= 8u) {
        // sorted in registers (odd-even transposition over 8 slots)
        uint32_t v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = (uint32_t)q < c ? l[q] : 0xffffffffu;
#pragma unroll
        for (int pass = 0; pass < 8; ++pass)
#pragma unroll
            for (int q = pass & 1; q + 1 < 8; q += 2)
                if (v[q] > v[q + 1]) {
                    const uint32_t tq = v[q];
                    v[q] = v[q + 1];
                    v[q + 1] = tq;
                }
        if (c > 0u) head = v[0] / p;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if ((uint32_t)q < c) succ[v[q]] = (uint32_t)q + 1u < c ? v[q < 7 ? q + 1 : 7] / p : NONE;
    } else {
        // a long list (deep windows): insertion sort in place
        for (uint32_t k = 1; k < c; ++k) {
            const uint32_t key = l[k];
            uint32_t q = k;
            while (q > 0 && l[q - 1] > key) {
                l[q] = l[q - 1];
                --q;
            }
            l[q] = key;
        }
        head = l[0] / p;
        for (uint32_t k = 0; k < c; ++k) succ[l[k]] = k + 1 < c ? l[k + 1] / p : NONE;
    }
}

// One workgroup per bucket of particles [p0, p0 + pb): each particle's
// entries sorted by iteration, the successors and the first head.  The
// bucket's entries (segment bst[bucket] .. + tot[bucket] of ent) are
// grouped by particle into the same segment of lst, in particle order: in
// LDS first when they fit (LCAP entries), else in place in lst.  The entries
// are read once, into registers (ER per thread; more are read again).
// Workgroup 0 also clears the round queue lengths (nclear words).
constexpr uint32_t LCAP = 4 * STPB;
constexpr int ER = 2;

__global__ __launch_bounds__(STPB) void k_rbmr_lists(uint32_t n, uint32_t p, uint32_t bsh,
                                                     const uint32_t *__restrict__ bst, const uint32_t *__restrict__ tot,
                                                     const uint2 *__restrict__ ent, uint32_t *__restrict__ lst,
                                                     uint32_t *__restrict__ succ, RRec *__restrict__ rec,
                                                     uint32_t *__restrict__ counts, uint32_t nclear)
{
    __shared__ uint32_t cnt_s[RBMR_MAX_PB];
    __shared__ uint32_t cur_s[RBMR_MAX_PB];
    __shared__ uint32_t ll[LCAP];
    __shared__ uint32_t wsum[STPB / 64];
    const uint32_t bk = blockIdx.x, t = threadIdx.x;
    if (bk == 0)
        for (uint32_t i = t; i < nclear; i += STPB) counts[i] = 0u;
    const uint32_t p0 = bk << bsh;
    const uint32_t pb = min(1u << bsh, n - p0);
    const uint32_t seg = bst[bk], ne = tot[bk];
    uint2 u[ER];
#pragma unroll
    for (int q = 0; q < ER; ++q) {
        const uint32_t i = t + (uint32_t)q * STPB;
        u[q] = i < ne ? ent[seg + i] : make_uint2(0u, 0xffffffffu);
    }
    for (uint32_t i = t; i < pb; i += STPB) cnt_s[i] = 0u;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < ER; ++q)
        if (u[q].y != 0xffffffffu) atomicAdd(&cnt_s[u[q].y - p0], 1u);
    for (uint32_t i = t + ER * STPB; i < ne; i += STPB) atomicAdd(&cnt_s[ent[seg + i].y - p0], 1u);
    __syncthreads();
    block_scan8(cnt_s, pb, nullptr, cur_s, wsum);
    const bool in_lds = ne <= LCAP;
    uint32_t *g = lst + seg;
#pragma unroll
    for (int q = 0; q < ER; ++q)
        if (u[q].y != 0xffffffffu) {
            const uint32_t at = atomicAdd(&cur_s[u[q].y - p0], 1u);
            if (in_lds) ll[at] = u[q].x; else g[at] = u[q].x;
        }
    for (uint32_t i = t + ER * STPB; i < ne; i += STPB) {
        const uint2 v = ent[seg + i];
        const uint32_t at = atomicAdd(&cur_s[v.y - p0], 1u);
        if (in_lds) ll[at] = v.x; else g[at] = v.x;
    }
    __syncthreads();
    for (uint32_t ml = t; ml < pb; ml += STPB) {
        const uint32_t c = cnt_s[ml];
        const uint32_t b0 = cur_s[ml] - c;
        uint32_t head;
        if (in_lds)
            particle_list(ll + b0, c, p, succ, head);
        else
            particle_list(g + b0, c, p, succ, head);
        rec[p0 + ml].tag = tag_of(0u, head);
    }
}

// The queue of round L (L >= 1): NSEG segments of segcap entries in lin,
// segment q of length qlen[q]; pre[0 .. NSEG] gets their exclusive scan
// (one wavefront; the caller synchronises).
__device__ __forceinline__ void queue_prefix(const uint32_t *__restrict__ qlen, uint32_t *pre)
{
    constexpr int PER = NSEG / 64;  // segments per lane
    if (threadIdx.x < 64) {
        uint32_t v[PER], sum = 0;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            v[q] = qlen[threadIdx.x * PER + q];
            sum += v[q];
        }
        uint32_t run = wave_incl_scan(sum) - sum;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            run += v[q];
            pre[threadIdx.x * PER + q + 1] = run;
        }
        if (threadIdx.x == 0) pre[0] = 0u;
    }
}

// Entry idx (< pre[NSEG]) of a segmented queue.
__device__ __forceinline__ uint32_t queue_at(const uint32_t *__restrict__ lin, uint32_t segcap, const uint32_t *pre,
                                             uint32_t idx)
{
    uint32_t lo = 0, hi = NSEG;  // pre[lo] <= idx < pre[hi]
    while (hi - lo > 1u) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= idx) lo = mid; else hi = mid;
    }
    return lin[(size_t)lo * segcap + (idx - pre[lo])];
}

// Round L over the pending iterations: L = 0 takes the whole window, later
// rounds the segmented queue lin / qlen[L].  Not-ready iterations go to
// segment blockIdx.x mod NSEG of lout / qlen[L + 1], one atomic add per
// workgroup and pass of its loop.  The grid is a multiple of NSEG or at
// most the window's tiles, so a segment receives at most wcur / NSEG +
// 2 TPB entries.
template <int D, int KERN, bool SPLIT>
__global__ __launch_bounds__(TPB) void k_rbmr_round(RbmrArgs a, uint32_t L, uint64_t kbase, uint32_t wcur, RRec *rec,
                                                    const uint32_t *__restrict__ succ, const uint32_t *__restrict__ lin,
                                                    uint32_t *__restrict__ lout, uint32_t segcap, uint32_t *qlen)
{
    __shared__ uint32_t pre[NSEG + 1];
    __shared__ uint32_t wq[TPB / 64 + 1];  // per-wavefront offsets, then the workgroup's base
    uint32_t nin = wcur;
    if (L > 0) {
        queue_prefix(qlen + (size_t)L * NSEG, pre);
        __syncthreads();
        nin = pre[NSEG];
    }
    const uint32_t seg = blockIdx.x % NSEG;
    uint32_t *out = lout + (size_t)seg * segcap;
    uint32_t *cnt = qlen + (size_t)(L + 1u) * NSEG + seg;
    for (uint32_t base = blockIdx.x * TPB; base < nin; base += gridDim.x * TPB) {
        const uint32_t idx = base + threadIdx.x;
        bool pend = false;
        uint32_t e = 0;
        if (idx < nin) {
            e = L == 0 ? idx : queue_at(lin, segcap, pre, idx);
            uint32_t m[RBMR_MAX_P], tag[RBMR_MAX_P], nx[RBMR_MAX_P];
            float xs[RBMR_MAX_P][D];
            draw_members(a, kbase + e, m);
            load_iteration<D>(a, e, rec, succ, m, tag, xs, nx);
            bool ready = true;
#pragma unroll
            for (int r = 0; r < RBMR_MAX_P; ++r)
                if (r < (int)a.p) ready = ready && ready_for(tag[r], e, L);
            if (ready)
                run_iteration<D, KERN, SPLIT>(a, kbase + e, m, xs, nx, L + 1u, rec);
            else
                pend = true;
        }
        // queue the pending iterations: wavefront counts, their scan, one
        // atomic add for the workgroup
        const uint64_t mask = __ballot(pend);
        const uint32_t lane = __lane_id(), wv = threadIdx.x >> 6;
        if (lane == 0) wq[wv] = (uint32_t)__popcll(mask);
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t run = 0;
#pragma unroll
            for (int k = 0; k < TPB / 64; ++k) {
                const uint32_t c = wq[k];
                wq[k] = run;
                run += c;
            }
            wq[TPB / 64] = run ? atomicAdd(cnt, run) : 0u;
        }
        __syncthreads();
        if (pend) out[wq[TPB / 64] + wq[wv] + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull))] = e;
        __syncthreads();  // wq is rewritten by the next pass
    }
}

// The iterations still pending after the last multi-workgroup round: one
// workgroup continues the rounds on its own for at most `budget` rounds,
// then runs whatever is left in iteration order on one thread.  Only this
// workgroup touches the records meanwhile, so the workgroup barrier between
// its rounds orders every record store of a round before the next round's
// loads.  Every round runs at least the earliest pending iteration, so the
// rounds make progress.
template <int D, int KERN, bool SPLIT>
__global__ __launch_bounds__(FIN_TPB) void k_rbmr_finish(RbmrArgs a, uint32_t rounds, uint32_t budget, uint64_t kbase,
                                                         RRec *rec, const uint32_t *__restrict__ succ,
                                                         const uint32_t *queue, uint32_t segcap,
                                                         const uint32_t *__restrict__ qlen, uint32_t *flat0,
                                                         uint32_t *flat1)
{
    __shared__ uint32_t s_cnt;
    __shared__ uint32_t pre[NSEG + 1];
    __shared__ uint32_t red[FIN_TPB];
    uint32_t *lists[2] = {flat0, flat1};
    // the segmented queue of round `rounds`, compacted into flat0
    queue_prefix(qlen + (size_t)rounds * NSEG, pre);
    __syncthreads();
    uint32_t n = pre[NSEG];
    for (uint32_t idx = threadIdx.x; idx < n; idx += FIN_TPB) flat0[idx] = queue_at(queue, segcap, pre, idx);
    __syncthreads();
    uint32_t L = rounds;
    for (uint32_t it = 0; n > 0 && it < budget; ++it, ++L) {
        const uint32_t *lin = lists[it & 1u];
        uint32_t *lout = lists[(it + 1u) & 1u];
        if (threadIdx.x == 0) s_cnt = 0;
        __syncthreads();
        for (uint32_t idx = threadIdx.x; idx < n; idx += FIN_TPB) {
            const uint32_t e = lin[idx];
            uint32_t m[RBMR_MAX_P], tag[RBMR_MAX_P], nx[RBMR_MAX_P];
            float xs[RBMR_MAX_P][D];
            draw_members(a, kbase + e, m);
            load_iteration<D>(a, e, rec, succ, m, tag, xs, nx);
            bool ready = true;
#pragma unroll
            for (int r = 0; r < RBMR_MAX_P; ++r)
                if (r < (int)a.p) ready = ready && ready_for(tag[r], e, L);
            if (ready)
                run_iteration<D, KERN, SPLIT>(a, kbase + e, m, xs, nx, L + 1u, rec);
            else
                lout[atomicAdd(&s_cnt, 1u)] = e;
        }
        __syncthreads();
        n = s_cnt;
        __syncthreads();
    }
    if (n == 0) return;
    // the rest in iteration order (the workgroup finds the next one)
    const uint32_t *list = lists[(L - rounds) & 1u];
    uint32_t last = 0;
    bool first_pass = true;
    for (uint32_t it = 0; it < n; ++it) {
        uint32_t best = 0xffffffffu;
        for (uint32_t i = threadIdx.x; i < n; i += FIN_TPB) {
            const uint32_t e = list[i];
            if ((first_pass || e > last) && e < best) best = e;
        }
        red[threadIdx.x] = best;
        __syncthreads();
        for (int s2 = FIN_TPB / 2; s2 > 0; s2 >>= 1) {
            if ((int)threadIdx.x < s2) red[threadIdx.x] = min(red[threadIdx.x], red[threadIdx.x + s2]);
            __syncthreads();
        }
        const uint32_t e = red[0];
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t m[RBMR_MAX_P], tag[RBMR_MAX_P], nx[RBMR_MAX_P];
            float xs[RBMR_MAX_P][D];
            draw_members(a, kbase + e, m);
            load_iteration<D>(a, e, rec, succ, m, tag, xs, nx);
            run_iteration<D, KERN, SPLIT>(a, kbase + e, m, xs, nx, L + 1u, rec);
        }
        last = e;
        first_pass = false;
    }
}

template <int D, int KERN, bool SPLIT>
hipError_t launch_dk(const RbmrArgs &a, const RbmrLayout &lay, void *ws, float *x, uint64_t kbase,
                     uint64_t niter, hipStream_t st)
{
    char *w = static_cast<char *>(ws);
    auto *rec = reinterpret_cast<RRec *>(w + lay.off_rec);
    auto *ent = reinterpret_cast<uint2 *>(w + lay.off_ent);
    auto *lst = reinterpret_cast<uint32_t *>(w + lay.off_lst);
    auto *succ = reinterpret_cast<uint32_t *>(w + lay.off_succ);
    auto *cnt = reinterpret_cast<uint32_t *>(w + lay.off_cnt);
    auto *tot = reinterpret_cast<uint32_t *>(w + lay.off_tot);
    auto *bst = reinterpret_cast<uint32_t *>(w + lay.off_bst);
    uint32_t *lists[2] = {reinterpret_cast<uint32_t *>(w + lay.off_list0),
                          reinterpret_cast<uint32_t *>(w + lay.off_list1)};
    auto *qlen = reinterpret_cast<uint32_t *>(w + lay.off_counts);
    const uint32_t R = lay.rounds;
    const dim3 gn((a.n + TPB - 1) / TPB);
    hipLaunchKernelGGL(k_rbmr_pack<D>, gn, dim3(TPB), 0, st, a.n, x, rec);
    for (uint64_t done = 0; done < niter;) {
        const uint32_t wcur = (uint32_t)((niter - done) < lay.window ? (niter - done) : lay.window);
        const uint32_t nblk = (wcur + lay.ipb - 1) / lay.ipb;
        const uint64_t kb = kbase + done;
        hipLaunchKernelGGL(k_rbmr_count, dim3(nblk), dim3(STPB), 0, st, a, kb, wcur, lay.ipb, lay.bsh, lay.nbk, cnt);
        hipLaunchKernelGGL(k_rbmr_offsets, dim3((lay.nbk + TPB / 64 - 1) / (TPB / 64)), dim3(TPB), 0, st, lay.nbk,
                           nblk, cnt, tot);
        hipLaunchKernelGGL(k_rbmr_scatter, dim3(nblk), dim3(STPB), 0, st, a, kb, wcur, lay.ipb, lay.bsh, lay.nbk,
                           (const uint32_t *)cnt, (const uint32_t *)tot, ent, bst);
        hipLaunchKernelGGL(k_rbmr_lists, dim3(lay.nbk), dim3(STPB), 0, st, a.n, a.p, lay.bsh, (const uint32_t *)bst,
                           (const uint32_t *)tot, (const uint2 *)ent, lst, succ, rec, qlen, (R + 2u) * NSEG);
        // round grids: every tile of the window for round 0, then halving,
        // at least NSEG workgroups (or every tile); above NSEG a multiple of
        // NSEG
        const uint32_t g0 = (wcur + TPB - 1) / TPB;
        for (uint32_t L = 0; L < R; ++L) {
            uint32_t grid = g0 >> L;
            if (grid < NSEG) grid = g0 < NSEG ? g0 : NSEG;
            grid = grid <= NSEG ? grid : (grid + NSEG - 1) / NSEG * NSEG;
            hipLaunchKernelGGL((k_rbmr_round<D, KERN, SPLIT>), dim3(grid), dim3(TPB), 0, st, a, L, kb, wcur, rec,
                               (const uint32_t *)succ, (const uint32_t *)lists[L & 1u], lists[(L + 1u) & 1u],
                               lay.segcap, qlen);
        }
        hipLaunchKernelGGL((k_rbmr_finish<D, KERN, SPLIT>), dim3(1), dim3(FIN_TPB), 0, st, a, R, FIN_BUDGET, kb, rec,
                           (const uint32_t *)succ, (const uint32_t *)lists[R & 1u], lay.segcap,
                           (const uint32_t *)qlen, lists[(R + 1u) & 1u], lst);
        done += wcur;
    }
    hipLaunchKernelGGL(k_rbmr_unpack<D>, gn, dim3(TPB), 0, st, a.n, rec, x);
    return hipGetLastError();
}

template <int D>
hipError_t launch_d(const RbmrArgs &a, int kernel, const RbmrLayout &lay, void *ws, float *x, uint64_t kbase,
                    uint64_t niter, hipStream_t st)
{
    switch (kernel) {
    case K_GAUSS: return launch_dk<D, K_GAUSS, false>(a, lay, ws, x, kbase, niter, st);
    case K_SOFTCOULOMB: return launch_dk<D, K_SOFTCOULOMB, false>(a, lay, ws, x, kbase, niter, st);
    case K_ATTREP: return launch_dk<D, K_ATTREP, false>(a, lay, ws, x, kbase, niter, st);
    default: return launch_dk<D, K_SOFTCOULOMB, true>(a, lay, ws, x, kbase, niter, st);
    }
}

size_t al256(size_t v)
{
    return (v + 255) & ~(size_t)255;
}

}  // namespace

RbmrLayout rbmr_layout(uint32_t n, uint32_t p, uint32_t window, uint32_t rounds)
{
    RbmrLayout l{};
    l.window = window;
    l.rounds = rounds;
    // buckets of 2^bsh consecutive particles: about 1024 buckets, at most
    // RBMR_MAX_PB particles each (so at most RBMR_MAX_NBK buckets)
    uint32_t bsh = 0;
    while ((((uint64_t)n + (1u << bsh) - 1u) >> bsh) > 1024u && (1u << bsh) < RBMR_MAX_PB) ++bsh;
    l.bsh = bsh;
    l.nbk = (uint32_t)(((uint64_t)n + (1u << bsh) - 1u) >> bsh);
    // iterations per counting workgroup: at least 4096, at most
    // RBMR_MAX_NBLK workgroups per window
    const uint32_t per = (window + RBMR_MAX_NBLK - 1) / RBMR_MAX_NBLK;
    l.ipb = per > 4096u ? per : 4096u;
    const uint32_t nblk = (window + l.ipb - 1) / l.ipb;
    const size_t nent = (size_t)window * p;
    size_t o = 0;
    l.off_rec = o;
    o = al256(o + (size_t)n * 16u);
    l.off_ent = o;
    o = al256(o + nent * 8u);
    l.off_lst = o;
    o = al256(o + nent * 4u);
    l.off_succ = o;
    o = al256(o + nent * 4u);
    l.off_cnt = o;
    o = al256(o + (size_t)nblk * l.nbk * 4u);
    l.off_tot = o;
    o = al256(o + (size_t)l.nbk * 4u);
    l.off_bst = o;
    o = al256(o + (size_t)l.nbk * 4u);
    // queue segments: a round's grid puts at most window / NSEG + 2 TPB
    // entries into one
    l.segcap = (window + NSEG - 1) / NSEG + 2u * TPB;
    l.off_list0 = o;
    o = al256(o + (size_t)l.segcap * NSEG * 4u);
    l.off_list1 = o;
    o = al256(o + (size_t)l.segcap * NSEG * 4u);
    l.off_counts = o;
    o = al256(o + (size_t)(rounds + 2) * NSEG * 4u);
    l.bytes = o;
    return l;
}

hipError_t rbmr_launch(const RbmrArgs &a, int d, int kernel, const RbmrLayout &lay, void *ws, float *x,
                       uint64_t kbase, uint64_t niter, hipStream_t st)
{
    if (niter == 0) return hipSuccess;
    switch (d) {
    case 1: return launch_d<1>(a, kernel, lay, ws, x, kbase, niter, st);
    case 2: return launch_d<2>(a, kernel, lay, ws, x, kbase, niter, st);
    default: return launch_d<3>(a, kernel, lay, ws, x, kbase, niter, st);
    }
}

}  // namespace rbm
