// Kernels of the RBM-1 step (Sec. 2.1, Algorithm 1) and of the direct sum
// (eq. (1.2)) for gfx950.
//
// One step m, with the particles held as records (x, id) in "slot" order
// (the order left by the previous step).  Slot k draws the PERM word w_k; the
// key (w_k << 32 | id) orders the particles.  The word range is cut into B
// equal "fine buckets", f = floor(w B / 2^32) (about 1700 records each),
// grouped 2^shift at a time into coarse buckets.
//
//   k_key_count      per tile of slots, fine-bucket histogram of the words
//                    (ALU only: the words depend on (seed, m, slot), not on
//                    the state)
//   k_key_colsum     fine-bucket totals
//   k_key_starts     fine and coarse bucket starts, run cursors
//   k_scatter_coarse a tile's 8K records, held in registers, go to their
//                    coarse buckets; each (tile, bucket) run is reserved with
//                    one atomic and written through an LDS reorder so that
//                    lanes store to consecutive addresses
//   k_split          each chunk of a coarse bucket (12K records, or 4K when
//                    that gives too few workgroups) goes to its fine
//                    buckets the same way
//   k_sort_step      one workgroup per fine bucket: order it in LDS by the
//                    unique key, evaluate the batch forces of eq. (2.3) for
//                    every batch inside the bucket, apply the Euler-Maruyama
//                    update, write each record at its sorted rank (its slot
//                    for step m+1)
//   k_fixup          the batches cut by a fine-bucket boundary
//
// Fused steps: the key passes of a group of steps run ahead of them, and the
// rank of a record after step m is its slot at step m+1, so the sort kernel
// knows every record's coarse bucket of the next step.  Inside a group it
// writes the updated records straight into those coarse buckets (k_cross_count
// and k_cross_scan give each bucket its write offsets), and the next step
// starts with the split: one pass over the records fewer per step.
//
// Records land in a run in whatever order the atomics give; the in-LDS sort
// by the unique key makes the result independent of it.  Up to 128 fine
// buckets the split level is skipped (shift = 0); when N fits one
// workgroup's LDS a single workgroup does the whole step in place.
#include "rbm_cv.hpp"
#include "rbm_device.hpp"
#include "rbm_plan.hpp"

namespace rbm {

// ---------------------------------------------------------------------------
// scans
// ---------------------------------------------------------------------------
// Inclusive scan across the 64 lanes of a wavefront (every lane active):
// within each row of 16 lanes by DPP row shifts of 1, 2, 4 and 8 (lanes
// shifted in from outside the row add 0), then each row adds the totals of
// the rows before it, read from lanes 15, 31 and 47.
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
    const uint32_t r0 = __builtin_amdgcn_readlane(v, 15);
    const uint32_t r1 = __builtin_amdgcn_readlane(v, 31);
    const uint32_t r2 = __builtin_amdgcn_readlane(v, 47);
    const uint32_t row = (threadIdx.x & 63u) >> 4;
    return v + (row >= 1u ? r0 : 0u) + (row >= 2u ? r1 : 0u) + (row >= 3u ? r2 : 0u);
}

// Exclusive scan of a[0..TPB*PER) in LDS, in place; returns the total (and
// stores it at a[TPB*PER] if STORE_TOTAL).  `tmp` holds TPB/64 words of LDS.
// Ends with a barrier.
template <int TPB, int PER, bool STORE_TOTAL = false>
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
    if (STORE_TOTAL && tid == 0) a[TPB * PER] = total;
    __syncthreads();
    return total;
}

__device__ __forceinline__ uint32_t bucket_of(uint32_t w, uint32_t nbuck)
{
    return __umulhi(w, nbuck);
}

__device__ __forceinline__ uint32_t fine_of(uint32_t w, uint32_t nbuck)
{
    return __umulhi(w, nbuck);
}

// Exclusive scan of a[0..nb), nb <= 256, by the first wavefront into out;
// returns the total to that wavefront's lanes.
__device__ __forceinline__ uint32_t wave0_exclusive_scan(const uint32_t *a, uint32_t *out, uint32_t nb)
{
    const uint32_t lane = threadIdx.x;
    uint32_t v[4], sum = 0;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        const uint32_t i = lane * 4 + k;
        v[k] = i < nb ? a[i] : 0u;
        sum += v[k];
    }
    const uint32_t inc = wave_inclusive_scan(sum);
    uint32_t run = inc - sum;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        const uint32_t i = lane * 4 + k;
        if (i < nb) out[i] = run;
        run += v[k];
    }
    return __shfl(inc, 63, 64);
}

// ---------------------------------------------------------------------------
// key counts: fine-bucket histogram of the PERM words, per tile of slots
// ---------------------------------------------------------------------------
constexpr uint32_t TILE = RBM_TILE;    // slots per coarse-scatter workgroup
// A staging level: TPB threads holding P records each, LDS rounds of RPT
// records per thread.
template <int TPB_, int P_, int RPT_>
struct Lvl {
    static constexpr int TPB = TPB_, P = P_, RPT = RPT_;
    static_assert(P % 4 == 0 && P % RPT == 0, "staging rounds must divide the records per thread");
};
using LvlScatter = Lvl<RBM_SCATTER_TPB, RBM_SCATTER_P, RBM_LVL_RPT>;
using LvlSplit = Lvl<RBM_SPLIT_TPB, RBM_SPLIT_P, RBM_SPLIT_RPT>;
using LvlSplitSmall = Lvl<RBM_SPLIT_TPB, RBM_SPLIT_SMALL_P, RBM_SPLIT_SMALL_P>;
constexpr int SCATTER_TPB = LvlScatter::TPB;
constexpr int SPLIT_TPB = LvlSplit::TPB;
constexpr int LVL_NB = RBM_MAX_COARSE; // largest digit count of a level
static_assert(LVL_NB <= 256, "coarse digits are stored in one byte");

// dig != nullptr (fused steps): also the coarse digit of every slot, one
// byte each, key set y at dig + y * dstride.
__global__ __launch_bounds__(1024) void k_key_count(StepArgs s, uint32_t tilef, uint32_t *cnt, uint32_t shift,
                                                    uint8_t *dig, size_t dstride)
{
    extern __shared__ uint32_t hist[];
    const uint32_t nb = s.nbuck;
    s.m += blockIdx.y;  // key set y holds step m + y
    cnt += (size_t)blockIdx.y * gridDim.x * nb;
    if (dig) dig += (size_t)blockIdx.y * dstride;
    for (uint32_t i = threadIdx.x; i < nb; i += 1024) hist[i] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * tilef;
    const uint32_t end = min(base + tilef, s.n);
    for (uint32_t k = base + 4 * threadIdx.x; k < end; k += 4 * 1024) {
        const uint4 w = philox4x32_10(make_uint4(k >> 2, s.m, STREAM_PERM, s.sys), s.k0, s.k1);
        const uint32_t f0 = fine_of(w.x, nb), f1 = fine_of(w.y, nb), f2 = fine_of(w.z, nb), f3 = fine_of(w.w, nb);
        atomicAdd(&hist[f0], 1u);
        if (k + 1 < end) atomicAdd(&hist[f1], 1u);
        if (k + 2 < end) atomicAdd(&hist[f2], 1u);
        if (k + 3 < end) atomicAdd(&hist[f3], 1u);
        if (dig) {
            if (k + 3 < end) {
                *reinterpret_cast<uchar4 *>(dig + k) =
                    make_uchar4((uint8_t)(f0 >> shift), (uint8_t)(f1 >> shift), (uint8_t)(f2 >> shift),
                                (uint8_t)(f3 >> shift));
            } else {
                dig[k] = (uint8_t)(f0 >> shift);
                if (k + 1 < end) dig[k + 1] = (uint8_t)(f1 >> shift);
                if (k + 2 < end) dig[k + 2] = (uint8_t)(f2 >> shift);
            }
        }
    }
    __syncthreads();
    uint32_t *row = cnt + (size_t)blockIdx.x * nb;
    for (uint32_t i = threadIdx.x; i < nb; i += 1024) row[i] = hist[i];
}

// ftot[f] = sum over tiles of cnt[t][f]
__global__ __launch_bounds__(256) void k_key_colsum(uint32_t ntf, uint32_t nbuck,
                                                    const uint32_t *__restrict__ cnt,
                                                    uint32_t *__restrict__ ftot)
{
    const uint32_t f = blockIdx.x * 256 + threadIdx.x;
    if (f >= nbuck) return;
    cnt += (size_t)blockIdx.y * ntf * nbuck;  // key set y
    ftot += (size_t)blockIdx.y * nbuck;
    uint32_t sum = 0;
    uint32_t t = 0;
    for (; t + 8 <= ntf; t += 8) {
        uint32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = cnt[(size_t)(t + u) * nbuck + f];
#pragma unroll
        for (int u = 0; u < 8; ++u) sum += v[u];
    }
    for (; t < ntf; ++t) sum += cnt[(size_t)t * nbuck + f];
    ftot[f] = sum;
}

// One workgroup per key set: fine starts (fstart[nbuck] = N), coarse starts
// cstart[c] = fstart[c << shift], and the run cursors of both levels.
// Global memory is read and written in coalesced order through LDS; thread t
// scans the PER consecutive totals it owns (the LDS index is padded by one
// word per 32 so these strided reads hit distinct banks).  flags bit 0: a
// fine bucket above the sort capacity.
__global__ __launch_bounds__(1024) void k_key_starts(uint32_t nbuck, uint32_t nb1, uint32_t shift,
                                                     uint32_t n, uint32_t fcap,
                                                     const uint32_t *__restrict__ ftot,
                                                     uint32_t *__restrict__ fstart,
                                                     uint32_t *__restrict__ fcur,
                                                     uint32_t *__restrict__ cstart,
                                                     uint32_t *__restrict__ ccur,
                                                     uint32_t *__restrict__ flags)
{
    constexpr int TPB = 1024, PER = RBM_MAX_FINE / TPB;
    static_assert(PER == 32, "padding assumes 32 entries per thread");
    __shared__ uint32_t a[RBM_MAX_FINE + RBM_MAX_FINE / 32];
    __shared__ uint32_t part[TPB];
    __shared__ uint32_t tmp[TPB / 64];
    auto pad = [](uint32_t i) { return i + (i >> 5); };
    const uint32_t t = threadIdx.x;
    // workgroup k: key set k
    ftot += (size_t)blockIdx.x * nbuck;
    fstart += (size_t)blockIdx.x * (nbuck + 1);
    fcur += (size_t)blockIdx.x * nbuck;
    cstart += (size_t)blockIdx.x * (nb1 + 1);
    ccur += (size_t)blockIdx.x * nb1;
    bool over = false;
    for (uint32_t i = t; i < (uint32_t)RBM_MAX_FINE; i += TPB) {
        const uint32_t v = i < nbuck ? ftot[i] : 0u;
        a[pad(i)] = v;
        over |= v > fcap;
    }
    __syncthreads();
    uint32_t v[PER], sum = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        v[k] = a[pad(t * PER + k)];
        sum += v[k];
    }
    part[t] = sum;
    __syncthreads();
    block_exclusive_scan<TPB, 1>(part, tmp);
    uint32_t run = part[t];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        a[pad(t * PER + k)] = run;
        run += v[k];
    }
    __syncthreads();
    for (uint32_t i = t; i < nbuck; i += TPB) {
        const uint32_t x = a[pad(i)];
        fstart[i] = x;
        fcur[i] = x;
    }
    for (uint32_t c = t; c < nb1; c += TPB) {
        const uint32_t x = a[pad(c << shift)];
        cstart[c] = x;
        ccur[c] = x;
    }
    if (t == 0) {
        fstart[nbuck] = n;
        cstart[nb1] = n;
    }
    if (over) atomicOr(flags, 1u);
}

// ---------------------------------------------------------------------------
// cross counts of fused transitions: transition t = blockIdx.y goes from the
// key set at fstart + t (step m) to the one at dig + t (step m + 1).  The
// records of step m at ranks [fstart[f], fstart[f + 1]) are the slots of fine
// bucket f; the sort kernel of that bucket writes each of them into its
// coarse bucket of step m + 1, the digit that the key count stored for that
// slot.  Per tile of RBM_CROSS_G fine buckets: xrow[f][c] (records of bucket
// f headed for coarse bucket c) and the tile's column sums xtsum[x][c].
// ---------------------------------------------------------------------------
constexpr uint32_t XG = RBM_CROSS_G;

__global__ __launch_bounds__(256) void k_cross_count(uint32_t nbuck, uint32_t nb1, uint32_t ntx, size_t dstride,
                                                     const uint32_t *__restrict__ fstart,
                                                     const uint8_t *__restrict__ dig,
                                                     uint16_t *__restrict__ xrow,
                                                     uint32_t *__restrict__ xtsum)
{
    __shared__ uint32_t hist[XG * LVL_NB];
    __shared__ uint32_t bnd[XG + 1];
    const uint32_t t = blockIdx.y, x = blockIdx.x, tid = threadIdx.x;
    fstart += (size_t)t * (nbuck + 1);
    dig += (size_t)t * dstride;  // the coarse digits of the transition's next step
    xrow += (size_t)t * nbuck * nb1;
    xtsum += (size_t)t * ntx * nb1;
    const uint32_t f0 = x * XG;
    const uint32_t ng = min(XG, nbuck - f0);
    for (uint32_t i = tid; i < XG * nb1; i += 256) hist[i] = 0;
    if (tid <= ng) bnd[tid] = fstart[f0 + tid];
    __syncthreads();
    // bucket by bucket, four digits per load (aligned words: the digits of a
    // key set are padded to a multiple of 256 bytes; a word that straddles
    // two buckets is read by both)
    for (uint32_t g = 0; g < ng; ++g) {
        const uint32_t b0 = bnd[g], b1 = bnd[g + 1];
        uint32_t *h = hist + g * nb1;
        for (uint32_t q = (b0 >> 2) + tid; b0 < b1 && 4 * q < b1; q += 256) {
            const uint32_t v = reinterpret_cast<const uint32_t *>(dig)[q];
#pragma unroll
            for (uint32_t j = 0; j < 4; ++j) {
                const uint32_t k = 4 * q + j;
                if (k >= b0 && k < b1) atomicAdd(&h[(v >> (8 * j)) & 255u], 1u);
            }
        }
    }
    __syncthreads();
    uint16_t *row = xrow + (size_t)f0 * nb1;
    for (uint32_t i = tid; i < ng * nb1; i += 256) row[i] = (uint16_t)min(hist[i], 65535u);
    for (uint32_t c = tid; c < nb1; c += 256) {
        uint32_t sum = 0;
        for (uint32_t g = 0; g < ng; ++g) sum += hist[g * nb1 + c];
        xtsum[(size_t)x * nb1 + c] = sum;
    }
}

// Coarse write offsets of fused transitions: xbase[x][c] = cstart[c] (the
// coarse starts of the transition's next step) + the records of tiles
// 0 .. x - 1 headed for coarse bucket c.  One workgroup per (c, t).
__global__ __launch_bounds__(256) void k_cross_scan(uint32_t nb1, uint32_t ntx,
                                                    const uint32_t *__restrict__ xtsum,
                                                    const uint32_t *__restrict__ cstart,
                                                    uint32_t *__restrict__ xbase)
{
    constexpr int PER = RBM_MAX_FINE / RBM_CROSS_G / 256;
    __shared__ uint32_t a[256 * PER];
    __shared__ uint32_t tmp[4];
    const uint32_t c = blockIdx.x, t = blockIdx.y;
    xtsum += (size_t)t * ntx * nb1;
    xbase += (size_t)t * ntx * nb1;
    cstart += (size_t)t * (nb1 + 1);
    for (uint32_t i = threadIdx.x; i < 256u * PER; i += 256) a[i] = i < ntx ? xtsum[(size_t)i * nb1 + c] : 0u;
    __syncthreads();
    block_exclusive_scan<256, PER>(a, tmp);
    const uint32_t c0 = cstart[c];
    for (uint32_t i = threadIdx.x; i < ntx; i += 256) xbase[(size_t)i * nb1 + c] = c0 + a[i];
}

// ---------------------------------------------------------------------------
// staged writes: a workgroup's C::P x C::TPB records (in registers) go to
// per-digit runs.  Each digit's run is reserved once with one global
// atomic on the digit's cursor; the records are then ordered by digit in LDS,
// C::RPT x C::TPB at a time, so that consecutive lanes store to consecutive
// addresses.
// ---------------------------------------------------------------------------
template <int D, class C>
struct StageLds {
    Rec<D> rec[C::RPT * C::TPB];
    uint32_t w[C::RPT * C::TPB];
    uint16_t dig[C::RPT * C::TPB];
    uint32_t cnt[LVL_NB];   // round counts / tile counts
    uint32_t start[LVL_NB]; // round starts
    uint32_t gbase[LVL_NB]; // next global position of each digit
};

// digit(w) = (fine_of(w) >> shift) & mask
template <int D, class C>
__device__ void staged_write(StageLds<D, C> &L, const float (&rx)[C::P][D], const uint32_t (&rid)[C::P],
                             const uint32_t (&w)[C::P], uint32_t nact, uint32_t nbuck,
                             uint32_t shift, uint32_t mask, uint32_t ndig, uint32_t *gcur,
                             Rec<D> *__restrict__ out, uint32_t *__restrict__ wout)
{
    const uint32_t tid = threadIdx.x;
    // record k of this thread is active if k < nact (the caller orders them so)
    for (uint32_t d = tid; d < ndig; d += C::TPB) L.cnt[d] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < C::P; ++k)
        if ((uint32_t)k < nact) atomicAdd(&L.cnt[(fine_of(w[k], nbuck) >> shift) & mask], 1u);
    __syncthreads();
    for (uint32_t d = tid; d < ndig; d += C::TPB)
        L.gbase[d] = L.cnt[d] ? atomicAdd(&gcur[d], L.cnt[d]) : 0u;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < C::P / C::RPT; ++r) {
        for (uint32_t d = tid; d < ndig; d += C::TPB) L.cnt[d] = 0;
        __syncthreads();
        uint32_t lr[C::RPT];
#pragma unroll
        for (int q = 0; q < C::RPT; ++q) {
            const int k = C::RPT * r + q;
            lr[q] = (uint32_t)k < nact ? atomicAdd(&L.cnt[(fine_of(w[k], nbuck) >> shift) & mask], 1u) : 0u;
        }
        __syncthreads();
        uint32_t total = 0;
        if (tid < 64) total = wave0_exclusive_scan(L.cnt, L.start, ndig);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < C::RPT; ++q) {
            const int k = C::RPT * r + q;
            if ((uint32_t)k < nact) {
                const uint32_t d = (fine_of(w[k], nbuck) >> shift) & mask;
                const uint32_t slot = L.start[d] + lr[q];
                Rec<D> t;
#pragma unroll
                for (int c = 0; c < D; ++c) t.x[c] = rx[k][c];
                t.id = rid[k];
                L.rec[slot] = t;
                L.w[slot] = w[k];
                L.dig[slot] = (uint16_t)d;
            }
        }
        __syncthreads();
        const uint32_t rt = L.start[ndig - 1] + L.cnt[ndig - 1];
        (void)total;
        for (uint32_t i = tid; i < rt; i += C::TPB) {
            const uint32_t d = L.dig[i];
            const uint32_t g = L.gbase[d] + (i - L.start[d]);
            out[g] = L.rec[i];
            wout[g] = L.w[i];
        }
        __syncthreads();
        for (uint32_t d = tid; d < ndig; d += C::TPB) L.gbase[d] += L.cnt[d];
        __syncthreads();
    }
}

// Coarse scatter: tile of P x TPB slots.  Thread t holds slots
// 4(t + TPB g) + j.
// Records of a partial last tile are packed so that the first nact of each
// thread are the valid ones.
template <int D>
__global__ __launch_bounds__(SCATTER_TPB) void k_scatter_coarse(StepArgs s, uint32_t shift, uint32_t nb1,
                                                            const Rec<D> *__restrict__ state,
                                                            uint32_t *__restrict__ ccur,
                                                            Rec<D> *__restrict__ stage,
                                                            uint32_t *__restrict__ wout)
{
    __shared__ StageLds<D, LvlScatter> L;
    const uint32_t base = blockIdx.x * TILE;
    const uint32_t end = min(base + TILE, s.n);
    float rx[LvlScatter::P][D];
    uint32_t rid[LvlScatter::P], w[LvlScatter::P];
    // all loads first (indices clamped into the tile), then the words and
    // the pending noise
    Rec<D> t[LvlScatter::P];
#pragma unroll
    for (int g = 0; g < LvlScatter::P / 4; ++g) {
        const uint32_t k = base + 4 * (threadIdx.x + g * LvlScatter::TPB);
#pragma unroll
        for (int j = 0; j < 4; ++j) t[4 * g + j] = state[min(k + j, end - 1u)];
    }
    uint32_t nact = 0;
#pragma unroll
    for (int g = 0; g < LvlScatter::P / 4; ++g) {
        const uint32_t k = base + 4 * (threadIdx.x + g * LvlScatter::TPB);
        const uint4 w4 = philox4x32_10(make_uint4(k >> 2, s.m, STREAM_PERM, s.sys), s.k0, s.k1);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (k + j < end) add_pending_noise<D>(s, t[4 * g + j].x, t[4 * g + j].id);
#pragma unroll
            for (int c = 0; c < D; ++c) rx[4 * g + j][c] = t[4 * g + j].x[c];
            rid[4 * g + j] = t[4 * g + j].id;
            w[4 * g + j] = j == 0 ? w4.x : (j == 1 ? w4.y : (j == 2 ? w4.z : w4.w));
        }
        // slots are consecutive per thread and groups ascend, so the valid
        // records are a prefix
        nact += (k < end) ? min(4u, end - k) : 0u;
    }
    staged_write<D, LvlScatter>(L, rx, rid, w, nact, s.nbuck, shift, 0xffffffffu, nb1, ccur, stage, wout);
}

// Split: chunk j of coarse bucket c (workgroup c * jmax + j; C::P x C::TPB
// records) into the 2^shift fine buckets of c, adding the pending noise of s.
template <int D, class C>
__global__ __launch_bounds__(SPLIT_TPB) void k_split(StepArgs s, uint32_t shift, uint32_t jmax, uint32_t nb1,
                                                   const uint32_t *__restrict__ cstart,
                                                   const Rec<D> *__restrict__ in,
                                                   const uint32_t *__restrict__ win,
                                                   uint32_t *__restrict__ fcur,
                                                   Rec<D> *__restrict__ out,
                                                   uint32_t *__restrict__ wout,
                                                   uint32_t *__restrict__ flags)
{
    static_assert(C::TPB == SPLIT_TPB, "one split block size");
    constexpr uint32_t CH = (uint32_t)(C::P * C::TPB);
    __shared__ StageLds<D, C> L;
#ifdef RBM_SPLIT_XCD
    // every chunk of coarse bucket c runs on XCD c mod 8 (workgroups are
    // dealt to the 8 XCDs in turn), so the lines that neighbouring runs of a
    // fine bucket share meet in one L2
    const uint32_t xcd = blockIdx.x & 7u, k = blockIdx.x >> 3;
    const uint32_t c = xcd + 8u * (k / jmax), j = k % jmax;
    if (c >= nb1) return;
#else
    const uint32_t c = blockIdx.x / jmax, j = blockIdx.x % jmax;
#endif
    const uint32_t c0 = cstart[c], c1 = cstart[c + 1];
    // the jmax chunks must cover the coarse bucket (mean + 16 sd of room)
    if (j == 0 && threadIdx.x == 0 && c1 - c0 > jmax * CH) atomicOr(flags, 1u);
    const uint32_t lo = min(c0 + j * CH, c1);
    const uint32_t hi = min(lo + CH, c1);
    if (lo == hi) return;
    float rx[C::P][D];
    uint32_t rid[C::P], w[C::P];
    // thread t holds records lo + t + C::TPB k: the valid ones are a prefix in k.
    // Every load is issued before any is used (indices clamped into the
    // chunk), so a thread has all of its records in flight at once.
    Rec<D> t[C::P];
#pragma unroll
    for (int k = 0; k < C::P; ++k) {
        const uint32_t e = min(lo + threadIdx.x + k * C::TPB, hi - 1u);
        t[k] = in[e];
        w[k] = win[e];
    }
    uint32_t nact = 0;
#pragma unroll
    for (int k = 0; k < C::P; ++k) {
        if (lo + threadIdx.x + k * C::TPB < hi) {
            // records written by a fused sort still lack the previous step's
            // noise (the host clears s.pssd when the coarse scatter added it)
            add_pending_noise<D>(s, t[k].x, t[k].id);
            ++nact;
        }
#pragma unroll
        for (int cc = 0; cc < D; ++cc) rx[k][cc] = t[k].x[cc];
        rid[k] = t[k].id;
    }
    const uint32_t ndig = 1u << shift;
    staged_write<D, C>(L, rx, rid, w, nact, s.nbuck, 0u, ndig - 1u, ndig, fcur + (c << shift), out, wout);
}

// The split of a plan, by its chunk size.
template <int D>
void launch_split(const Plan &pl, hipStream_t st, const StepArgs &s, const uint32_t *cstart, const Rec<D> *in,
                  const uint32_t *win, uint32_t *fcur, Rec<D> *out, uint32_t *wout, uint32_t *flags)
{
#ifdef RBM_SPLIT_XCD
    const uint32_t grid = 8u * ((pl.nb1 + 7u) / 8u) * pl.jmax;
#else
    const uint32_t grid = pl.nb1 * pl.jmax;
#endif
    if (pl.chunk == (uint32_t)RBM_CHUNK_SMALL)
        hipLaunchKernelGGL((k_split<D, LvlSplitSmall>), dim3(grid), dim3(SPLIT_TPB), 0, st, s, pl.shift,
                           pl.jmax, pl.nb1, cstart, in, win, fcur, out, wout, flags);
    else
        hipLaunchKernelGGL((k_split<D, LvlSplit>), dim3(grid), dim3(SPLIT_TPB), 0, st, s, pl.shift,
                           pl.jmax, pl.nb1, cstart, in, win, fcur, out, wout, flags);
}

// ---------------------------------------------------------------------------
// per-bucket sort + batch force + Euler-Maruyama
// ---------------------------------------------------------------------------
// End of one particle's step: in force mode its force is written (by id)
// and the record comes back unchanged; else the record with the
// Euler-Maruyama update applied.
template <int D>
__device__ __forceinline__ Rec<D> finish(const StepArgs &s, float (&x)[D], float (&f)[D], uint32_t id,
                                         float *__restrict__ fout)
{
    if (fout) {
        if (id < s.n) {  // ids are < N unless a flagged overflow left stale data
#pragma unroll
            for (int c = 0; c < D; ++c) fout[(size_t)id * D + c] = f[c];
        }
    } else {
        drift_update<D>(s, x, f);
    }
    Rec<D> o;
#pragma unroll
    for (int c = 0; c < D; ++c) o.x[c] = x[c];
    o.id = id;
    return o;
}

// LDS slot of the record at global rank r in a bucket starting at lo: one
// empty slot after every 8, so that the batches the lanes of a wavefront
// read in the same instruction (each batch's records are contiguous) start
// in different LDS banks.
struct Slot {
    uint32_t lo;
    __device__ __forceinline__ uint32_t operator()(uint32_t r) const
    {
        const uint32_t l = r - lo;
        return l + (l >> 3);
    }
};
// LDS records needed for n sorted records with that spacing
constexpr uint32_t slot_cap(uint32_t n)
{
    return n + n / 8 + 1;
}

// Member r of the batch of ranks [bs, bs + sz) (any size): its force by
// direct summation.
template <int D, int KERN>
__device__ __forceinline__ Rec<D> member_generic(const StepArgs &s, const Rec<D> *srec, Slot pad,
                                                 uint32_t bs, uint32_t sz, uint32_t r, float *__restrict__ fout)
{
    const Rec<D> me = srec[pad(r)];
    float xi[D], f[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
        xi[c] = me.x[c];
        f[c] = 0.0f;
    }
    for (uint32_t j = bs; j < bs + sz; ++j)
        if (j != r) add_pair<D, KERN>(xi, srec[pad(j)].x, s.a, f);
    const float inv = (sz == s.p) ? s.inv_p1 : s.inv_last;
#pragma unroll
    for (int c = 0; c < D; ++c) f[c] *= inv;
    return finish<D>(s, xi, f, me.id, fout);
}

// Member r of a batch of exactly PM members starting at rank bs: its force
// by direct summation over the batch in rank order, with the member loop
// unrolled.  One thread per record keeps the registers per thread low (64 at
// d = 3, six workgroups per CU); a thread per batch evaluating each pair once
// needed 98 and fitted four.  The sum over j is in the same order either way.
template <int D, int KERN, int PM>
__device__ __forceinline__ Rec<D> member_fixed(const StepArgs &s, const Rec<D> *srec, Slot pad, uint32_t bs,
                                               uint32_t r, float *__restrict__ fout)
{
    const Rec<D> me = srec[pad(r)];
    float xi[D], f[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
        xi[c] = me.x[c];
        f[c] = 0.0f;
    }
    if constexpr (PM == 2) {
        if (pair_flow_scheme(s) && !fout) {
            // the pair moves by its exact flow; the partner's thread makes the
            // same operations with the arguments swapped
            const float *xj = srec[pad(bs + (r == bs ? 1u : 0u))].x;
            float y[D];
            if (s.scheme == 1)
                pair_flow<D>(s.dt, xi, xj, y);
            else
                pair_flow_linear<D>(s.flowc, xi, xj, y);
            return finish<D>(s, y, f, me.id, fout);
        }
    }
    // every member is read before any pair is evaluated (the reads are in
    // flight together).  The own term is evaluated too, with its scale
    // replaced by -0: dx = x - x = +0 exactly, so it adds -0 x +0 = -0 and
    // leaves every partial sum as it was, so the sum is the same additions
    // in the same order as skipping it (one select per member, not D)
    constexpr int DK = kdim<D, KERN>();
    float xm[PM][DK];
#pragma unroll
    for (int j = 0; j < PM; ++j) {
        const Rec<D> o = srec[pad(bs + (uint32_t)j)];
#pragma unroll
        for (int c = 0; c < DK; ++c) xm[j][c] = o.x[c];
    }
#pragma unroll
    for (int j = 0; j < PM; ++j) {
        float dx[DK];
        float r2 = 0.0f;
#pragma unroll
        for (int c = 0; c < DK; ++c) {
            dx[c] = xi[c] - xm[j][c];
            r2 = fmaf(dx[c], dx[c], r2);
        }
        const float sc = bs + (uint32_t)j != r ? pair_scale<KERN>(r2, s.a) : -0.0f;
#pragma unroll
        for (int c = 0; c < DK; ++c) f[c] = fmaf(sc, dx[c], f[c]);
    }
#pragma unroll
    for (int c = 0; c < D; ++c) f[c] *= s.inv_p1;
    return finish<D>(s, xi, f, me.id, fout);
}

// The member at rank r (inside the bucket's whole batches): its batch from
// the batch geometry, p == PM with a compile-time divisor when PM > 0.
template <int D, int KERN, int PM>
__device__ __forceinline__ Rec<D> batch_member(const StepArgs &s, const Rec<D> *srec, Slot pad, uint32_t r,
                                               float *__restrict__ fout)
{
    if constexpr (PM > 0) {
        uint32_t q = r / (uint32_t)PM;
        if (q > s.nbat - 1) q = s.nbat - 1;
        const uint32_t bs = q * (uint32_t)PM;
        if (q != s.nbat - 1 || s.n - bs == (uint32_t)PM) return member_fixed<D, KERN, PM>(s, srec, pad, bs, r, fout);
        return member_generic<D, KERN>(s, srec, pad, bs, s.n - bs, r, fout);
    } else {
        uint32_t bs, be;
        batch_of(s, r, bs, be);
        return member_generic<D, KERN>(s, srec, pad, bs, be - bs, r, fout);
    }
}

// Output of a fused step's sort kernel: the coarse buckets of the next step
// (records and their PERM words of that step), placed by the cross counts of
// the transition.
template <int D>
struct FuseOut {
    const uint16_t *xrow;    // [nbuck][nb1] records of fine bucket f headed for coarse bucket c
    const uint32_t *xbase;   // [ntx][nb1] coarse write offset of each cross tile
    uint32_t *fixpos;        // [n] position written for each record of a cut batch, by rank
    Rec<D> *out;             // coarse buckets of the next step
    uint32_t *wout;          // their PERM words
    uint32_t nb1;
    uint32_t shift;
};

// One workgroup per fine bucket [lo, hi) (SINGLE: the whole system, read
// from the slot-ordered state, PERM words drawn here).
//   1. load: records stay in registers; each record is counted in its
//      sub-bucket (the next SBITS bits of the word below the bucket digits)
//   2. exclusive scan of the sub-bucket counts; the 64-bit keys (w, id) are
//      listed in LDS in sub-bucket order
//   3. rank = sub-bucket start + members with a smaller key
//   4. records written to LDS in sorted order (reusing the ordering bytes)
//   5. batches inside the bucket, one thread per record (PM > 0: p = PM,
//      the member loop unrolled).  Records of cut batches go to dst
//      unchanged for k_fixup.
// fout != nullptr: forces only (by id); dst gets only the cut batches.
// SORTONLY: every record is written to dst at its rank, nothing else.
// FUSED: the updated records go to the next step's coarse buckets (fo), not
// to dst; the records of cut batches also go to dst at their ranks, and
// their positions in fo.out to fo.fixpos, for k_fixup.
template <int D, int KERN, bool SINGLE, int TPB, int CAP, int SBITS, bool SORTONLY = false, int PM = 0,
          bool FUSED = false>
__global__ __launch_bounds__(TPB) void k_sort_step(StepArgs s, const Rec<D> *src,
                                                   const uint32_t *__restrict__ wsrc,
                                                   const uint32_t *__restrict__ bstart,
                                                   Rec<D> *dst, float *__restrict__ fout,
                                                   uint32_t *__restrict__ flags, FuseOut<D> fo)
{
    constexpr int S = 1 << SBITS;
    constexpr int E = (CAP + TPB - 1) / TPB;
    static_assert(S % TPB == 0, "sub-bucket count must be a multiple of the block");
    static_assert(!FUSED || (!SINGLE && !SORTONLY), "fused output is for the multi-bucket step");
    constexpr size_t ORDER_BYTES = (size_t)CAP * 8 + (size_t)(S + 1) * 4;
    constexpr size_t REC_BYTES = (size_t)slot_cap(CAP) * sizeof(Rec<D>);
    __shared__ __align__(16) unsigned char lds[ORDER_BYTES > REC_BYTES ? ORDER_BYTES : REC_BYTES];
    // fused output: two per-digit arrays, the Philox words of the bucket's
    // ranks (WT: at most CAP + 6 of them, in blocks of 4), the staging rounds
    constexpr size_t WT = 4 * ((CAP + 6) / 4 + 1);
    static_assert(8 * LVL_NB + WT * 4 + 64 * (sizeof(Rec<D>) + 4) <= sizeof(lds), "fused staging does not fit");
    __shared__ uint32_t scan_tmp[TPB / 64];
    uint64_t *skey = reinterpret_cast<uint64_t *>(lds);  // [CAP] keys in sub-bucket order
    uint32_t *cnt = reinterpret_cast<uint32_t *>(skey + CAP);
    Rec<D> *srec = reinterpret_cast<Rec<D> *>(lds);

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

    // 1. load: every record and word of the thread is requested before any
    //    is used (indices clamped into the bucket), so their latencies overlap
    Rec<D> ld[E];
    uint32_t lw[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const uint32_t e = min(tid + k * TPB, nb - 1u);
        ld[k] = src[lo + e];
        if constexpr (!SINGLE) lw[k] = wsrc[lo + e];
    }
    // fused: thread c < nb1 gathers the write offset of coarse bucket c for
    // this bucket (its tile's base plus the earlier buckets of the tile) and
    // this bucket's own count, to check against the counts made here; the
    // loads are all issued at once and used only in the output stage
    uint32_t fgo = 0, fchk = 0;
    if constexpr (FUSED) {
        if (tid < fo.nb1) {
            const uint32_t f = blockIdx.x, f0 = f - f % XG;
            uint32_t part[XG];
#pragma unroll
            for (uint32_t g = 0; g < XG; ++g) part[g] = f0 + g < f ? fo.xrow[(size_t)(f0 + g) * fo.nb1 + tid] : 0u;
            fgo = fo.xbase[(size_t)(f / XG) * fo.nb1 + tid];
            fchk = fo.xrow[(size_t)f * fo.nb1 + tid];
#pragma unroll
            for (uint32_t g = 0; g < XG; ++g) fgo += part[g];
        }
    }
    for (uint32_t i = tid; i <= (uint32_t)S; i += TPB) cnt[i] = 0;
    __syncthreads();

    float mx[E][D];
    uint32_t mid[E], mw[E], msb[E], mpos[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const uint32_t e = tid + k * TPB;
        if (e < nb) {
            Rec<D> r = ld[k];
            if constexpr (SINGLE) add_pending_noise<D>(s, r.x, r.id);
#pragma unroll
            for (int c = 0; c < D; ++c) mx[k][c] = r.x[c];
            mid[k] = r.id;
            uint32_t w;
            if constexpr (SINGLE) {
                const uint4 b4 = philox4x32_10(make_uint4(e >> 2, s.m, STREAM_PERM, s.sys), s.k0, s.k1);
                w = word_of(b4, e & 3u);
            } else {
                w = lw[k];
            }
            mw[k] = w;
            const uint32_t sb = (w * s.nbuck) >> (32 - SBITS);
            msb[k] = sb;
            mpos[k] = atomicAdd(&cnt[sb], 1u);
        }
    }
    __syncthreads();
    // 2. sub-bucket starts (cnt[S] = total) and the keys listed by sub-bucket
    (void)block_exclusive_scan<TPB, S / TPB, true>(cnt, scan_tmp);
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const uint32_t e = tid + k * TPB;
        if (e < nb) skey[cnt[msb[k]] + mpos[k]] = ((uint64_t)mw[k] << 32) | mid[k];
    }
    __syncthreads();
    // 3. exact ranks
    uint32_t mrank[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const uint32_t e = tid + k * TPB;
        mrank[k] = 0;
        if (e < nb) {
            const uint64_t key = ((uint64_t)mw[k] << 32) | mid[k];
            const uint32_t b0 = cnt[msb[k]], b1 = cnt[msb[k] + 1];
            uint32_t rank = b0;
            for (uint32_t j = b0; j < b1; ++j) rank += skey[j] < key ? 1u : 0u;
            mrank[k] = rank;
        }
    }
    __syncthreads();
    // 4. sorted records
    const Slot pad{lo};
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const uint32_t e = tid + k * TPB;
        if (e < nb) {
            Rec<D> r;
#pragma unroll
            for (int c = 0; c < D; ++c) r.x[c] = mx[k][c];
            r.id = mid[k];
            srec[pad(lo + mrank[k])] = r;
        }
    }
    __syncthreads();

    if constexpr (SORTONLY) {
        // every record at its rank, unchanged (the control-variate path
        // evaluates the batches from this order)
        for (uint32_t l = tid; l < nb; l += TPB) dst[lo + l] = srec[pad(lo + l)];
        return;
    }
    // 5. batches.  The batches [bs, be) with lo <= bs and be <= hi are
    //    q_first..q_last; they cover ranks [ins_lo, ins_hi).  The last batch
    //    (q = nbat - 1) ends at n, so it is inside only if hi == n.
    const uint32_t p = s.p;
    const int64_t q_first = ((int64_t)lo + p - 1) / p;
    const int64_t q_last = (hi == s.n) ? (int64_t)s.nbat - 1
                                       : min((int64_t)s.nbat - 2, (int64_t)(hi / p) - 1);
    const bool any = q_first <= (int64_t)s.nbat - 1 && q_last >= q_first;
    const uint32_t ins_lo = any ? (uint32_t)q_first * p : hi;
    const uint32_t ins_hi = any ? (q_last == (int64_t)s.nbat - 1 ? s.n : (uint32_t)(q_last + 1) * p) : hi;
    if constexpr (!FUSED) {
        for (uint32_t l = tid; l < nb; l += TPB) {
            const uint32_t r = lo + l;
            if (r < ins_lo || r >= ins_hi) dst[r] = srec[pad(r)];
        }
        if (!any) return;
        for (uint32_t r = ins_lo + tid; r < ins_hi; r += TPB) {
            const Rec<D> o = batch_member<D, KERN, PM>(s, srec, pad, r, fout);
            if (!fout) dst[r] = o;
        }
    } else {
        // 5F. the updated records stay in registers (record l = tid + k TPB)
        Rec<D> u[E];
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const uint32_t l = tid + k * TPB;
            if (l < nb) {
                const uint32_t r = lo + l;
                if (r >= ins_lo && r < ins_hi) {
                    u[k] = batch_member<D, KERN, PM>(s, srec, pad, r, nullptr);
                } else {
                    u[k] = srec[pad(r)];
                    dst[r] = u[k];
                }
            }
        }
        __syncthreads();
        // 6F. the PERM words of ranks lo .. hi - 1 at step m + 1 (rank r is
        //     slot r of that step), one Philox block per 4 ranks; they stay
        //     in LDS until the records are written
        uint32_t *goff = reinterpret_cast<uint32_t *>(lds);  // [LVL_NB] write offset - local start
        uint32_t *ccnt = goff + LVL_NB;                       // [LVL_NB] counts, then local starts
        uint32_t *wtmp = ccnt + 256;                          // [WT] words
        const uint32_t q0 = lo >> 2, nq = ((hi - 1) >> 2) - q0 + 1;
        for (uint32_t j = tid; j < nq; j += TPB) {
            reinterpret_cast<uint4 *>(wtmp)[j] =
                philox4x32_10(make_uint4(q0 + j, s.m + 1, STREAM_PERM, s.sys), s.k0, s.k1);
        }
        if (tid < fo.nb1) ccnt[tid] = 0;
        __syncthreads();
        uint32_t key[E];  // coarse digit | local index in it << 8
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const uint32_t l = tid + k * TPB;
            if (l < nb) {
                const uint32_t c = fine_of(wtmp[lo - 4 * q0 + l], s.nbuck) >> fo.shift;
                key[k] = c | (atomicAdd(&ccnt[c], 1u) << 8);
            }
        }
        __syncthreads();
        // the counts made here must be those of the key passes
        if (tid < fo.nb1 && ccnt[tid] != fchk) atomicOr(flags, 1u);
        __syncthreads();
        if (tid < 64) (void)wave0_exclusive_scan(ccnt, ccnt, fo.nb1);
        __syncthreads();
        if (tid < fo.nb1) goff[tid] = fgo - ccnt[tid];
        __syncthreads();
        // key: the record's position in coarse-digit order (its digit's
        // local start plus its index in the digit); the global position is
        // goff[digit] + key
#pragma unroll
        for (int k = 0; k < E; ++k)
            if (tid + k * TPB < nb) key[k] = ccnt[key[k] & 255u] + (key[k] >> 8);
        // 7F. records in coarse-digit order through LDS, R at a time, so that
        //     consecutive lanes store to consecutive addresses
        constexpr uint32_t R = (uint32_t)((sizeof(lds) - 8 * LVL_NB - WT * 4) / (sizeof(Rec<D>) + 4));
        Rec<D> *stg = reinterpret_cast<Rec<D> *>(lds + 8 * LVL_NB + WT * 4);
        uint32_t *stw = reinterpret_cast<uint32_t *>(stg + R);
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const uint32_t l = tid + k * TPB, r = lo + l;
            if (l < nb && (r < ins_lo || r >= ins_hi))
                fo.fixpos[r] = goff[fine_of(wtmp[lo - 4 * q0 + l], s.nbuck) >> fo.shift] + key[k];
        }
        for (uint32_t base = 0; base < nb; base += R) {
#pragma unroll
            for (int k = 0; k < E; ++k) {
                const uint32_t l = tid + k * TPB;
                if (l < nb) {
                    const uint32_t i = key[k] - base;
                    if (i < R) {
                        stg[i] = u[k];
                        stw[i] = wtmp[lo - 4 * q0 + l];
                    }
                }
            }
            __syncthreads();
            const uint32_t cnt_r = min(R, nb - base);
            for (uint32_t i = tid; i < cnt_r; i += TPB) {
                const uint32_t w = stw[i];
                const uint32_t g = goff[fine_of(w, s.nbuck) >> fo.shift] + base + i;
                if (g < s.n) {
                    fo.out[g] = stg[i];
                    fo.wout[g] = w;
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// batches cut by bucket boundaries
// ---------------------------------------------------------------------------
// Teams of T = 2^tsh threads (T >= the largest batch, 2p - 1), 128 / T per
// workgroup: team j of workgroup x looks at the boundary at rank bstart[b],
// b = x 128 / T + j + 1 <= nbound.  The batch around it is cut if the
// boundary is not the batch's first rank; of several boundaries inside one
// batch only the first handles it.
// fixpos != nullptr (fused step): the cut records are read from dst at their
// ranks and the updated ones written to out[fixpos[rank]].
template <int D, int KERN>
__global__ __launch_bounds__(128) void k_fixup(StepArgs s, const uint32_t *__restrict__ bstart, uint32_t nbound,
                                               uint32_t tsh, Rec<D> *dst, float *__restrict__ fout,
                                               const uint32_t *__restrict__ fixpos, Rec<D> *out)
{
    __shared__ Rec<D> shall[128];
    const uint32_t team = threadIdx.x >> tsh, tid = threadIdx.x & ((1u << tsh) - 1u);
    const uint32_t b = blockIdx.x * (128u >> tsh) + team + 1;
    bool act = false;
    uint32_t bs = 0, be = 0;
    if (b <= nbound) {
        const uint32_t r = bstart[b];
        if (r != 0 && r < s.n) {
            batch_of(s, r, bs, be);
            act = r != bs && bstart[b - 1] <= bs;
        }
    }
    Rec<D> *sh = shall + (team << tsh);
    const uint32_t sz = be - bs;
    if (act && tid < sz) sh[tid] = dst[bs + tid];
    __syncthreads();
    if (!act) return;
    if (tid < sz && pair_flow_scheme(s) && !fout && sz == 2) {
        // a pair moves by its exact flow (the same operations as in the sort kernel)
        const Rec<D> me = sh[tid];
        float xi[D], y[D];
        const float zero[D] = {};
#pragma unroll
        for (int c = 0; c < D; ++c) xi[c] = me.x[c];
        if (s.scheme == 1)
            pair_flow<D>(s.dt, xi, sh[1 - tid].x, y);
        else
            pair_flow_linear<D>(s.flowc, xi, sh[1 - tid].x, y);
        drift_update<D>(s, y, zero);
        Rec<D> o;
#pragma unroll
        for (int c = 0; c < D; ++c) o.x[c] = y[c];
        o.id = me.id;
        if (!fixpos)
            dst[bs + tid] = o;
        else if (fixpos[bs + tid] < s.n)  // positions are < N unless a flagged overflow left stale data
            out[fixpos[bs + tid]] = o;
    } else if (tid < sz) {
        const Rec<D> me = sh[tid];
        float xi[D], f[D];
#pragma unroll
        for (int c = 0; c < D; ++c) {
            xi[c] = me.x[c];
            f[c] = 0.0f;
        }
        for (uint32_t j = 0; j < sz; ++j)
            if (j != tid) add_pair<D, KERN>(xi, sh[j].x, s.a, f);
        const float inv = (sz == s.p) ? s.inv_p1 : s.inv_last;
#pragma unroll
        for (int c = 0; c < D; ++c) f[c] *= inv;
        if (fout) {
            if (me.id < s.n) {
#pragma unroll
                for (int c = 0; c < D; ++c) fout[(size_t)me.id * D + c] = f[c];
            }
        } else {
            drift_update<D>(s, xi, f);
            Rec<D> o;
#pragma unroll
            for (int c = 0; c < D; ++c) o.x[c] = xi[c];
            o.id = me.id;
            if (!fixpos)
                dst[bs + tid] = o;
            else if (fixpos[bs + tid] < s.n)
                out[fixpos[bs + tid]] = o;
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
__global__ __launch_bounds__(256) void k_positions(StepArgs s, const Rec<D> *__restrict__ state,
                                                   float *__restrict__ x, uint32_t *__restrict__ ids)
{
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k >= s.n) return;
    Rec<D> r = state[k];
    if (x) add_pending_noise<D>(s, r.x, r.id);
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

// out[0] = sum_t |f[ids[t]] - fref[t]|^2 in FP64: one workgroup, each thread
// a strided FP64 partial, then a fixed-order tree.  An id >= n is not read
// and makes the sum NaN.
__global__ __launch_bounds__(1024) void k_sqerr(const float *__restrict__ f, uint32_t n,
                                                const uint32_t *__restrict__ ids, uint32_t nids,
                                                const float *__restrict__ fref, int d,
                                                double *__restrict__ out)
{
    __shared__ double part[1024];
    double acc = 0.0;
    for (uint32_t t = threadIdx.x; t < nids; t += 1024) {
        const uint32_t i = ids[t];
        if (i >= n) {
            acc = __builtin_nan("");
            continue;
        }
        for (int c = 0; c < d; ++c) {
            const double e = (double)f[(size_t)i * d + c] - (double)fref[(size_t)t * d + c];
            acc += e * e;
        }
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = part[0];
}

// ---------------------------------------------------------------------------
// direct sum: F_i = 1/(N-1) sum_{j != i} K(X_i - X_j), LDS tiles of j, FP32
// pair terms summed per tile, FP64 across tiles.  step: apply the update.
// ---------------------------------------------------------------------------
// SELF: the pair j = i must be masked out (its scale can be infinite, a = 0
// with a singular kernel).  Otherwise its term is exactly zero (dx = 0 and a
// finite scale) and the mask is left out of the loop.
// m2 != nullptr (force mode only): also m2[t] = 1/(N-1) sum_{j != i}
// |K(X_i - X_j)|^2, the second moment behind the variance of Lemma 3.1.
template <int D, int KERN, int TPB, bool SELF>
__global__ __launch_bounds__(TPB) void k_direct(StepArgs s, const float *__restrict__ x,
                                                const uint32_t *__restrict__ ids, uint32_t nids,
                                                float *__restrict__ out, int step,
                                                float *__restrict__ m2)
{
    constexpr int DK = kdim<D, KERN>();
    __shared__ float tile[TPB * D];
    const uint32_t t = blockIdx.x * TPB + threadIdx.x;
    const bool active = t < nids;
    uint32_t i = active ? (ids ? ids[t] : t) : 0u;
    const bool valid = i < s.n;  // an id >= N yields NaN forces instead of a wild read
    if (!valid) i = 0;
    float xi[D];
#pragma unroll
    for (int c = 0; c < D; ++c) xi[c] = x[(size_t)i * D + c];
    double acc[D], acc2 = 0.0;
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
        float part[D], part2 = 0.0f;
#pragma unroll
        for (int c = 0; c < D; ++c) part[c] = 0.0f;
        if (m2) {
            for (uint32_t jj = 0; jj < cntj; ++jj) {
                float dx[DK];
                float r2 = 0.0f;
#pragma unroll
                for (int c = 0; c < DK; ++c) {
                    dx[c] = xi[c] - tile[jj * D + c];
                    r2 = fmaf(dx[c], dx[c], r2);
                }
                float sc = pair_scale<KERN>(r2, s.a);
                if constexpr (SELF) sc = (base + jj == i) ? 0.0f : sc;
#pragma unroll
                for (int c = 0; c < DK; ++c) part[c] = fmaf(sc, dx[c], part[c]);
                part2 = fmaf(sc * sc, r2, part2);
            }
            acc2 += (double)part2;
        } else
        for (uint32_t jj = 0; jj < cntj; ++jj) {
            float dx[DK];
            float r2 = 0.0f;
#pragma unroll
            for (int c = 0; c < DK; ++c) {
                dx[c] = xi[c] - tile[jj * D + c];
                r2 = fmaf(dx[c], dx[c], r2);
            }
            float sc = pair_scale<KERN>(r2, s.a);
            if constexpr (SELF) sc = (base + jj == i) ? 0.0f : sc;
#pragma unroll
            for (int c = 0; c < DK; ++c) part[c] = fmaf(sc, dx[c], part[c]);
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
        if (m2) m2[t] = valid ? (float)(acc2 * inv) : __builtin_nanf("");
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

constexpr int SINGLE_TPB = 512;
constexpr int SINGLE_CAP = RBM_SINGLE_CAP;
constexpr int SINGLE_SBITS = 11;
constexpr int SORT_TPB = RBM_SORT_TPB;
constexpr int SORT_CAP = RBM_SORT_CAP;
constexpr int SORT_SBITS = RBM_SORT_SBITS;
static_assert((RBM_MAX_FINE >> 7) <= LVL_NB && (1 << RBM_SPLIT_SHIFT) <= LVL_NB && RBM_SPLIT_SHIFT <= 7,
              "digits beyond the staging arrays");
constexpr int DIRECT_TPB = 256;

inline void mark(hipEvent_t *ev, int i, hipStream_t st)
{
    if (ev) (void)hipEventRecord(ev[i], st);
}

inline size_t align_up(size_t x, size_t a)
{
    return (x + a - 1) / a * a;
}

template <typename T>
T *at(void *ws, size_t off)
{
    return reinterpret_cast<T *>((char *)ws + off);
}

// Control-variate step (d = 2, Gaussian kernel): S = sum_j c(X_j) in FP64,
// the same division as the plain step with the records written in rank
// order, then the control-variate batch force and the drift update.
// Buffers of key set k.
struct KeySet {
    uint32_t *kcnt, *ftot, *fstart, *fcur, *cstart, *ccur;
};

KeySet key_set(const Plan &pl, void *ws, uint32_t k)
{
    KeySet q;
    q.kcnt = at<uint32_t>(ws, pl.off_kcnt) + (size_t)k * pl.ntf * pl.nbuck;
    q.ftot = at<uint32_t>(ws, pl.off_ftot) + (size_t)k * pl.nbuck;
    q.fstart = at<uint32_t>(ws, pl.off_fstart) + (size_t)k * (pl.nbuck + 1);
    q.fcur = at<uint32_t>(ws, pl.off_fcur) + (size_t)k * pl.nbuck;
    q.cstart = at<uint32_t>(ws, pl.off_cstart) + (size_t)k * (pl.nb1 + 1);
    q.ccur = at<uint32_t>(ws, pl.off_ccur) + (size_t)k * pl.nb1;
    return q;
}

// The cross kernels for `count` transitions, key sets src + t -> dst + t.
void cross_impl(const Plan &pl, uint32_t src, uint32_t dst, uint32_t count, void *ws, hipStream_t st)
{
    const size_t dstride = align_up(pl.n, 256);
    const KeySet a = key_set(pl, ws, src), b = key_set(pl, ws, dst);
    uint16_t *xrow = at<uint16_t>(ws, pl.off_xrow) + (size_t)src * pl.nbuck * pl.nb1;
    uint32_t *xtsum = at<uint32_t>(ws, pl.off_xtsum) + (size_t)src * pl.ntx * pl.nb1;
    uint32_t *xbase = at<uint32_t>(ws, pl.off_xbase) + (size_t)src * pl.ntx * pl.nb1;
    hipLaunchKernelGGL(k_cross_count, dim3(pl.ntx, count), dim3(256), 0, st, pl.nbuck, pl.nb1, pl.ntx, dstride,
                       a.fstart, at<uint8_t>(ws, pl.off_xdig) + (size_t)dst * dstride, xrow, xtsum);
    hipLaunchKernelGGL(k_cross_scan, dim3(pl.nb1, count), dim3(256), 0, st, pl.nb1, pl.ntx, xtsum, b.cstart, xbase);
}

hipError_t keys_impl(const Plan &pl, const StepArgs &s, uint32_t count, void *ws, hipStream_t st,
                     hipEvent_t *ev, uint32_t base = 0, uint32_t xsrc = 0xffffffffu)
{
    mark(ev, 0, st);
    if (pl.nbuck > 1) {
        const KeySet q = key_set(pl, ws, base);
        auto *flags = at<uint32_t>(ws, pl.off_flags);
        const size_t dstride = align_up(pl.n, 256);
        uint8_t *dig = pl.fuse ? at<uint8_t>(ws, pl.off_xdig) + (size_t)base * dstride : nullptr;
        hipLaunchKernelGGL(k_key_count, dim3(pl.ntf, count), dim3(1024), (size_t)pl.nbuck * 4, st, s, pl.tilef,
                           q.kcnt, pl.shift, dig, dstride);
        mark(ev, 1, st);
        hipLaunchKernelGGL(k_key_colsum, dim3((pl.nbuck + 255) / 256, count), dim3(256), 0, st, pl.ntf,
                           pl.nbuck, q.kcnt, q.ftot);
        mark(ev, 2, st);
        hipLaunchKernelGGL(k_key_starts, dim3(count), dim3(1024), 0, st, pl.nbuck, pl.nb1, pl.shift, pl.n,
                           pl.cap, q.ftot, q.fstart, q.fcur, q.cstart, q.ccur, flags);
        // the transitions base -> base + 1, ..., inside the group, and the
        // one into it
        if (pl.fuse && count > 1) cross_impl(pl, base, base + 1, count - 1, ws, st);
        if (pl.fuse && xsrc < pl.nsets) cross_impl(pl, xsrc, base, 1, ws, st);
    } else {
        mark(ev, 1, st);
        mark(ev, 2, st);
    }
    mark(ev, 3, st);
    return hipGetLastError();
}

hipError_t step_cv(const Plan &pl, const StepArgs &s, void *ws, hipStream_t st, void *dst_state,
                   float *fout, hipEvent_t *ev, uint32_t set, bool keys_ready)
{
    auto *state = at<Rec<2>>(ws, pl.off_state);
    auto *sorted = at<Rec<2>>(ws, pl.off_sorted);
    auto *flags = at<uint32_t>(ws, pl.off_flags);
    const float *master = at<float>(ws, pl.off_cvmaster);
    const __bf16 *wb = at<__bf16>(ws, pl.off_cvwb);
    double *S = at<double>(ws, pl.off_cvS);
    if (!keys_ready) {
        hipError_t e = keys_impl(pl, s, 1, ws, st, ev);
        if (e != hipSuccess) return e;
        set = 0;
    }
    hipError_t e = hipSuccess;
    if (pl.nbuck == 1) {
        for (int i = 4; i <= 5; ++i) mark(ev, i, st);
        hipLaunchKernelGGL((k_sort_step<2, K_GAUSS, true, SINGLE_TPB, SINGLE_CAP, SINGLE_SBITS, true>),
                           dim3(1), dim3(SINGLE_TPB), 0, st, s, state, nullptr, nullptr, sorted,
                           nullptr, flags, FuseOut<2>{});
    } else {
        auto *stage1 = at<Rec<2>>(ws, pl.off_stage1);
        auto *w1 = at<uint32_t>(ws, pl.off_w1);
        const KeySet q = key_set(pl, ws, set);
        uint32_t *fstart = q.fstart, *fcur = q.fcur, *cstart = q.cstart, *ccur = q.ccur;
        const Rec<2> *src = stage1;
        const uint32_t *wsrc = w1;
        if (pl.shift > 0) {
            auto *stage2 = at<Rec<2>>(ws, pl.off_stage2);
            auto *w2 = at<uint32_t>(ws, pl.off_w2);
            hipLaunchKernelGGL((k_scatter_coarse<2>), dim3(pl.ntiles), dim3(SCATTER_TPB), 0, st, s,
                               pl.shift, pl.nb1, state, ccur, stage1, w1);
            mark(ev, 4, st);
            StepArgs ss = s;  // the coarse scatter added the pending noise
            ss.pssd = 0.0f;
            launch_split<2>(pl, st, ss, cstart, stage1, w1, fcur, stage2, w2, flags);
            src = stage2;
            wsrc = w2;
        } else {
            hipLaunchKernelGGL((k_scatter_coarse<2>), dim3(pl.ntiles), dim3(SCATTER_TPB), 0, st, s, 0u,
                               pl.nbuck, state, fcur, stage1, w1);
            mark(ev, 4, st);
        }
        mark(ev, 5, st);
        hipLaunchKernelGGL((k_sort_step<2, K_GAUSS, false, SORT_TPB, SORT_CAP, SORT_SBITS, true>),
                           dim3(pl.nbuck), dim3(SORT_TPB), 0, st, s, src, wsrc, fstart, sorted, nullptr, flags,
                           FuseOut<2>{});
    }
    // phase A over the key-ordered records (their noise is in): c of every
    // particle (BF16), kept for phase B, and S; timed with the batch phase
    mark(ev, 6, st);
    StepArgs sa = s;
    sa.pssd = 0.0f;
    __bf16 *cbuf = at<__bf16>(ws, pl.off_cvc);
    e = cv_launch_csum(sa, sorted, master, wb, at<double>(ws, pl.off_cvspart), S, cbuf, st);
    if (e != hipSuccess) return e;
    e = cv_launch_batch(s, K_GAUSS, sorted, cbuf, master, wb, S, dst_state, fout, st);
    mark(ev, 7, st);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

// Fix-up teams: T = 2^fix_shift threads, the smallest power of two that
// holds the largest batch (2p - 1 members, p <= 64); fix_groups workgroups
// of 128 / T teams cover the nbuck - 1 boundaries.
uint32_t fix_shift(const Plan &pl)
{
    uint32_t t = 0;
    while ((1u << t) < 2 * pl.p - 1) ++t;
    return t;
}

uint32_t fix_groups(const Plan &pl)
{
    const uint32_t per = 128u >> fix_shift(pl);
    return (pl.nbuck - 1 + per - 1) / per;
}

// The sort kernel with the batch size fixed at compile time (unrolled member
// loop) for the common sizes; any other p takes the runtime loop.
template <int D, int KERN, bool SINGLE, int TPB, int CAP, int SB, bool FUSED = false>
void launch_sort(uint32_t p, dim3 grid, hipStream_t st, const StepArgs &s, const Rec<D> *src,
                 const uint32_t *wsrc, const uint32_t *bstart, Rec<D> *dst, float *fout,
                 uint32_t *flags, const FuseOut<D> &fo = FuseOut<D>{})
{
#define RBM_SORT(PMM)                                                                                          \
    hipLaunchKernelGGL((k_sort_step<D, KERN, SINGLE, TPB, CAP, SB, false, PMM, FUSED>), grid, dim3(TPB), 0, st, \
                       s, src, wsrc, bstart, dst, fout, flags, fo)
    switch (p) {
    case 2: RBM_SORT(2); break;
    case 4: RBM_SORT(4); break;
    case 8: RBM_SORT(8); break;
    default: RBM_SORT(0); break;
    }
#undef RBM_SORT
}

template <int D, int KERN>
hipError_t step_dk(const Plan &pl, const StepArgs &s, void *ws, hipStream_t st, void *dst_state,
                   float *fout, hipEvent_t *ev, uint32_t set, bool keys_ready, uint32_t fuse)
{
    auto *state = at<Rec<D>>(ws, pl.off_state);
    auto *dst = reinterpret_cast<Rec<D> *>(dst_state);
    auto *flags = at<uint32_t>(ws, pl.off_flags);
    if constexpr (D == 2 && KERN == K_GAUSS) {
        if (pl.cv) return step_cv(pl, s, ws, st, dst_state, fout, ev, set, keys_ready);
    }
    if (!keys_ready) {
        hipError_t e = keys_impl(pl, s, 1, ws, st, ev);
        if (e != hipSuccess) return e;
        set = 0;
        fuse = 0;
    }
    if (!pl.fuse || fout) fuse = 0;
    if (pl.nbuck == 1) {
        for (int i = 4; i <= 5; ++i) mark(ev, i, st);
        launch_sort<D, KERN, true, SINGLE_TPB, SINGLE_CAP, SINGLE_SBITS>(
            pl.p, dim3(1), st, s, state, nullptr, nullptr, dst, fout, flags);
        mark(ev, 6, st);
        mark(ev, 7, st);
        return hipGetLastError();
    }
    auto *stage1 = at<Rec<D>>(ws, pl.off_stage1);
    auto *w1 = at<uint32_t>(ws, pl.off_w1);
    const KeySet q = key_set(pl, ws, set);
    uint32_t *fstart = q.fstart, *fcur = q.fcur, *cstart = q.cstart, *ccur = q.ccur;
    const bool split = pl.shift > 0;
    const Rec<D> *src = stage1;
    const uint32_t *wsrc = w1;
    if (split) {
        auto *stage2 = at<Rec<D>>(ws, pl.off_stage2);
        auto *w2 = at<uint32_t>(ws, pl.off_w2);
        // the pending noise is added by the first kernel that reads the
        // records: the coarse scatter, or the split when the previous step's
        // sort wrote the coarse buckets
        StepArgs ss = s;
        if (!(fuse & 1u)) {
            hipLaunchKernelGGL((k_scatter_coarse<D>), dim3(pl.ntiles), dim3(SCATTER_TPB), 0, st, s, pl.shift,
                               pl.nb1, state, ccur, stage1, w1);
            ss.pssd = 0.0f;
        }
        mark(ev, 4, st);
        launch_split<D>(pl, st, ss, cstart, stage1, w1, fcur, stage2, w2, flags);
        mark(ev, 5, st);
        src = stage2;
        wsrc = w2;
    } else {
        // one level: the coarse buckets are the fine buckets
        hipLaunchKernelGGL((k_scatter_coarse<D>), dim3(pl.ntiles), dim3(SCATTER_TPB), 0, st, s, 0u,
                           pl.nbuck, state, fcur, stage1, w1);
        mark(ev, 4, st);
        mark(ev, 5, st);
    }
    if (fuse & 2u) {
        // the updated records go to the coarse buckets of the next step
        // (key set set + 1), placed by the cross counts of this transition
        FuseOut<D> fo;
        fo.xrow = at<uint16_t>(ws, pl.off_xrow) + (size_t)set * pl.nbuck * pl.nb1;
        fo.xbase = at<uint32_t>(ws, pl.off_xbase) + (size_t)set * pl.ntx * pl.nb1;
        fo.fixpos = at<uint32_t>(ws, pl.off_fixpos);
        fo.out = stage1;
        fo.wout = w1;
        fo.nb1 = pl.nb1;
        fo.shift = pl.shift;
        launch_sort<D, KERN, false, SORT_TPB, SORT_CAP, SORT_SBITS, true>(pl.p, dim3(pl.nbuck), st, s, src, wsrc,
                                                                          fstart, dst, nullptr, flags, fo);
        mark(ev, 6, st);
        hipLaunchKernelGGL((k_fixup<D, KERN>), dim3(fix_groups(pl)), dim3(128), 0, st, s, fstart, pl.nbuck - 1,
                           fix_shift(pl), dst, nullptr, fo.fixpos, stage1);
        mark(ev, 7, st);
        return hipGetLastError();
    }
    launch_sort<D, KERN, false, SORT_TPB, SORT_CAP, SORT_SBITS>(pl.p, dim3(pl.nbuck), st, s, src, wsrc, fstart,
                                                                dst, fout, flags);
    mark(ev, 6, st);
    hipLaunchKernelGGL((k_fixup<D, KERN>), dim3(fix_groups(pl)), dim3(128), 0, st, s, fstart, pl.nbuck - 1,
                       fix_shift(pl), dst, fout, (const uint32_t *)nullptr, (Rec<D> *)nullptr);
    mark(ev, 7, st);
    return hipGetLastError();
}

template <int D>
hipError_t step_d(const Plan &pl, const StepArgs &s, int kernel, void *ws, hipStream_t st,
                  void *dst, float *fout, hipEvent_t *ev, uint32_t set, bool keys_ready, uint32_t fuse)
{
    switch (kernel) {
    case K_GAUSS: return step_dk<D, K_GAUSS>(pl, s, ws, st, dst, fout, ev, set, keys_ready, fuse);
    case K_SOFTCOULOMB: return step_dk<D, K_SOFTCOULOMB>(pl, s, ws, st, dst, fout, ev, set, keys_ready, fuse);
    case K_LINEAR: return step_dk<D, K_LINEAR>(pl, s, ws, st, dst, fout, ev, set, keys_ready, fuse);
    case K_HAMILTON:
        if constexpr (D == 2) return step_dk<D, K_HAMILTON>(pl, s, ws, st, dst, fout, ev, set, keys_ready, fuse);
        return hipErrorInvalidValue;
    default: return step_dk<D, K_ATTREP>(pl, s, ws, st, dst, fout, ev, set, keys_ready, fuse);
    }
}

template <int D, int KERN>
hipError_t direct_dk(const StepArgs &s, const float *x, const uint32_t *ids, uint32_t nids,
                     float *out, int step, float *m2, hipStream_t st)
{
    const dim3 g((nids + DIRECT_TPB - 1) / DIRECT_TPB);
    if (KERN == K_GAUSS || s.a > 0.0f)
        hipLaunchKernelGGL((k_direct<D, KERN, DIRECT_TPB, false>), g, dim3(DIRECT_TPB), 0, st, s, x, ids, nids,
                           out, step, m2);
    else
        hipLaunchKernelGGL((k_direct<D, KERN, DIRECT_TPB, true>), g, dim3(DIRECT_TPB), 0, st, s, x, ids, nids,
                           out, step, m2);
    return hipGetLastError();
}

template <int D>
hipError_t direct_d(const StepArgs &s, int kernel, const float *x, const uint32_t *ids,
                    uint32_t nids, float *out, int step, float *m2, hipStream_t st)
{
    switch (kernel) {
    case K_GAUSS: return direct_dk<D, K_GAUSS>(s, x, ids, nids, out, step, m2, st);
    case K_SOFTCOULOMB: return direct_dk<D, K_SOFTCOULOMB>(s, x, ids, nids, out, step, m2, st);
    case K_LINEAR: return direct_dk<D, K_LINEAR>(s, x, ids, nids, out, step, m2, st);
    case K_HAMILTON:
        if constexpr (D == 2) return direct_dk<D, K_HAMILTON>(s, x, ids, nids, out, step, m2, st);
        return hipErrorInvalidValue;
    default: return direct_dk<D, K_ATTREP>(s, x, ids, nids, out, step, m2, st);
    }
}

}  // namespace

hipError_t launch_keys(const Plan &pl, const StepArgs &s, uint32_t count, void *ws, hipStream_t st,
                       hipEvent_t *ev, uint32_t base, uint32_t xsrc)
{
    if (count < 1 || count > pl.kb || base + count > pl.nsets) return hipErrorInvalidValue;
    if (xsrc != 0xffffffffu && (!pl.fuse || xsrc >= pl.nsets || (xsrc >= base && xsrc < base + count)))
        return hipErrorInvalidValue;
    return keys_impl(pl, s, count, ws, st, ev, base, xsrc);
}

hipError_t launch_step(const Plan &pl, const StepArgs &s, int d, int kernel, void *ws,
                       hipStream_t st, void *dst_state, float *fout, hipEvent_t *ev, uint32_t set,
                       bool keys_ready, uint32_t fuse)
{
    if (keys_ready && set >= pl.nsets) return hipErrorInvalidValue;
    switch (d) {
    case 1: return step_d<1>(pl, s, kernel, ws, st, dst_state, fout, ev, set, keys_ready, fuse);
    case 2: return step_d<2>(pl, s, kernel, ws, st, dst_state, fout, ev, set, keys_ready, fuse);
    default: return step_d<3>(pl, s, kernel, ws, st, dst_state, fout, ev, set, keys_ready, fuse);
    }
}

hipError_t launch_init(const Plan &pl, int d, const float *x0, const uint32_t *slots, void *ws,
                       hipStream_t st)
{
    void *state = at<char>(ws, pl.off_state);
    auto *flags = at<uint32_t>(ws, pl.off_flags);
    const dim3 g((pl.n + 255) / 256);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, flags, 16u, 0u);
    switch (d) {
    case 1: hipLaunchKernelGGL(k_init_state<1>, g, dim3(256), 0, st, pl.n, x0, slots, (Rec<1> *)state, flags); break;
    case 2: hipLaunchKernelGGL(k_init_state<2>, g, dim3(256), 0, st, pl.n, x0, slots, (Rec<2> *)state, flags); break;
    default: hipLaunchKernelGGL(k_init_state<3>, g, dim3(256), 0, st, pl.n, x0, slots, (Rec<3> *)state, flags); break;
    }
    return hipGetLastError();
}

hipError_t launch_positions(const Plan &pl, const StepArgs &s, int d, const void *ws, float *x,
                            uint32_t *ids, hipStream_t st)
{
    const void *state = (const char *)ws + pl.off_state;
    const dim3 g((pl.n + 255) / 256);
    switch (d) {
    case 1: hipLaunchKernelGGL(k_positions<1>, g, dim3(256), 0, st, s, (const Rec<1> *)state, x, ids); break;
    case 2: hipLaunchKernelGGL(k_positions<2>, g, dim3(256), 0, st, s, (const Rec<2> *)state, x, ids); break;
    default: hipLaunchKernelGGL(k_positions<3>, g, dim3(256), 0, st, s, (const Rec<3> *)state, x, ids); break;
    }
    return hipGetLastError();
}

hipError_t launch_fill(uint32_t *p, size_t n, uint32_t v, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, p, (uint32_t)n, v);
    return hipGetLastError();
}

hipError_t launch_sqerr(const float *f, uint32_t n, const uint32_t *ids, uint32_t nids, const float *fref, int d,
                        double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sqerr, dim3(1), dim3(1024), 0, st, f, n, ids, nids, fref, d, out);
    return hipGetLastError();
}

hipError_t launch_direct(const StepArgs &s, int d, int kernel, const float *x, const uint32_t *ids,
                         uint32_t nids, float *out, int step, hipStream_t st, float *m2)
{
    switch (d) {
    case 1: return direct_d<1>(s, kernel, x, ids, nids, out, step, m2, st);
    case 2: return direct_d<2>(s, kernel, x, ids, nids, out, step, m2, st);
    default: return direct_d<3>(s, kernel, x, ids, nids, out, step, m2, st);
    }
}

}  // namespace rbm
