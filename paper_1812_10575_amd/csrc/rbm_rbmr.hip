// RBM-r (Sec. 2.2, Algorithm RBM-r) on the GPU.
//
// The method is sequential: iteration k moves the p particles of its batch
// C_k, starting from the positions the earlier iterations left.  Iterations
// whose batches are disjoint commute, so a window of W consecutive
// iterations runs in rounds: an iteration runs in the first round in which
// it is the earliest pending iteration of every one of its members.  Each
// iteration then starts from exactly the positions the sequential order
// gives it, so the result depends neither on the window nor on the rounds
// (bit for bit: an iteration's arithmetic is the same wherever it runs).
//
// A call packs the positions into per-particle records {two round tags,
// position} (16 bytes for d <= 2, 32 for d = 3), so that a readiness check
// and the update of a member touch one cache line, and unpacks them at the
// end.  One window:
//   k_rbmr_draw   draws every batch and marks each member with the round-0
//                 tag of the iteration (32-bit atomic min)
//   k_rbmr_round  round L: an iteration whose tag is still on all its
//                 members runs; the others mark their members with the next
//                 round's tag in the other tag word and queue themselves
//   k_rbmr_finish one workgroup continues the rounds for what is pending
//                 after the last multi-workgroup round (a window of N/2
//                 random pairs has depth 11 to 13, and after 8 rounds about
//                 0.03 % of its iterations are left), then runs anything
//                 still pending in iteration order
// Batches are drawn again from the counter wherever they are needed (a few
// ALU operations instead of a stored table read at random).  Tag of
// iteration e (its offset in the window, < 2^22) in round g: ((1023 - g)
// << 22) | e, g = 1 .. 1022 over a stretch of windows (each window reserves
// the round numbers of its multi-workgroup rounds and of the finishing
// workgroup's budget; the records are retagged when g would pass 1022).  A
// later round's tags are below every stale one, so the tags need no reset
// between rounds, and within a round the earliest iteration wins.  Round L
// reads tag word L mod 2 and writes the other, so what it reads was settled
// before it started.
#include <hip/hip_runtime.h>

#include "rbm_rbmr.hpp"

namespace rbm {
namespace {

constexpr int TPB = 256;
constexpr int FIN_TPB = 1024;
constexpr uint32_t FIN_BUDGET = 64;  // single-workgroup rounds before the ordered rest
enum : uint32_t { STREAM_RBMR_DRAW = 2u, STREAM_RBMR_NOISE = 3u };

__device__ __forceinline__ uint32_t tag_of(uint32_t g, uint32_t e)
{
    return ((1023u - g) << 22) | e;
}

template <int D>
struct alignas(D <= 2 ? 16 : 32) RRec {
    uint32_t tag[2];
    float x[D <= 2 ? 2 : 6];
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
// K = x/|x|^2, then the field step), then the noise of its slots.  Only the
// position words of the records are written (other threads may be updating
// the tag words of the same records).
template <int D, int KERN, bool SPLIT>
__device__ __forceinline__ void run_iteration(const RbmrArgs &a, uint64_t k, const uint32_t (&m)[RBMR_MAX_P],
                                              const float (&xs)[RBMR_MAX_P][D], RRec<D> *rec)
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
                float f[D];
#pragma unroll
                for (int c = 0; c < D; ++c) f[c] = 0.0f;
#pragma unroll
                for (int q = 0; q < RBMR_MAX_P; ++q)
                    if (q < (int)a.p && q != r) add_pair<D, KERN>(xs[r], xs[q], a.a, f);
#pragma unroll
                for (int c = 0; c < D; ++c) y[r][c] = fmaf(a.dt, fmaf(-a.beta, xs[r][c], f[c] * a.inv_p1), xs[r][c]);
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
            float *dst = rec[m[r]].x;
            if constexpr (D == 2) {
                *reinterpret_cast<float2 *>(dst) = make_float2(y[r][0], y[r][1]);
            } else {
#pragma unroll
                for (int c = 0; c < D; ++c) dst[c] = y[r][c];
            }
        }
}

template <int D>
__device__ __forceinline__ void load_positions(const RbmrArgs &a, const RRec<D> *rec, const uint32_t (&m)[RBMR_MAX_P],
                                               float (&xs)[RBMR_MAX_P][D])
{
#pragma unroll
    for (int r = 0; r < RBMR_MAX_P; ++r)
        if (r < (int)a.p) {
#pragma unroll
            for (int c = 0; c < D; ++c) xs[r][c] = rec[m[r]].x[c];
        }
}

template <int D>
__global__ __launch_bounds__(TPB) void k_rbmr_pack(uint32_t n, const float *__restrict__ x, RRec<D> *__restrict__ rec)
{
    const uint32_t i = blockIdx.x * TPB + threadIdx.x;
    if (i >= n) return;
    RRec<D> r{};
    r.tag[0] = r.tag[1] = 0xffffffffu;
#pragma unroll
    for (int c = 0; c < D; ++c) r.x[c] = x[(size_t)i * D + c];
    rec[i] = r;
}

// Tags back to "untouched" (a new stretch of round numbers).
template <int D>
__global__ __launch_bounds__(TPB) void k_rbmr_retag(uint32_t n, RRec<D> *__restrict__ rec)
{
    const uint32_t i = blockIdx.x * TPB + threadIdx.x;
    if (i < n) *reinterpret_cast<uint2 *>(rec[i].tag) = make_uint2(0xffffffffu, 0xffffffffu);
}

template <int D>
__global__ __launch_bounds__(TPB) void k_rbmr_unpack(uint32_t n, const RRec<D> *__restrict__ rec, float *__restrict__ x)
{
    const uint32_t i = blockIdx.x * TPB + threadIdx.x;
    if (i >= n) return;
    const RRec<D> r = rec[i];
#pragma unroll
    for (int c = 0; c < D; ++c) x[(size_t)i * D + c] = r.x[c];
}

template <int D>
__global__ __launch_bounds__(TPB) void k_rbmr_draw(RbmrArgs a, uint64_t kbase, uint32_t wcur, uint32_t g,
                                                   RRec<D> *rec, uint32_t *__restrict__ counts, uint32_t rounds)
{
    const uint32_t e = blockIdx.x * TPB + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x <= rounds) counts[threadIdx.x] = 0u;
    if (e >= wcur) return;
    uint32_t m[RBMR_MAX_P];
    draw_members(a, kbase + e, m);
    const uint32_t t = tag_of(g, e);
#pragma unroll
    for (int r = 0; r < RBMR_MAX_P; ++r)
        if (r < (int)a.p) atomicMin(&rec[m[r]].tag[0], t);
}

// Round L (tag g): L = 0 takes the whole window, later rounds the queue
// lin[0 .. counts[L]).  Not-ready iterations go to lout / counts[L + 1].
template <int D, int KERN, bool SPLIT>
__global__ __launch_bounds__(TPB) void k_rbmr_round(RbmrArgs a, uint32_t L, uint32_t g, uint64_t kbase, uint32_t wcur,
                                                    RRec<D> *rec, const uint32_t *__restrict__ lin,
                                                    uint32_t *__restrict__ lout, uint32_t *counts)
{
    const uint32_t nin = L == 0 ? wcur : counts[L];
    const uint32_t wi = L & 1u, wo = wi ^ 1u;
    for (uint32_t base = blockIdx.x * TPB; base < nin; base += gridDim.x * TPB) {
        const uint32_t idx = base + threadIdx.x;
        bool pend = false;
        uint32_t e = 0;
        if (idx < nin) {
            e = L == 0 ? idx : lin[idx];
            uint32_t m[RBMR_MAX_P];
            draw_members(a, kbase + e, m);
            const uint32_t t = tag_of(g, e);
            float xs[RBMR_MAX_P][D];
            bool ready = true;
#pragma unroll
            for (int r = 0; r < RBMR_MAX_P; ++r)
                if (r < (int)a.p) {
                    const RRec<D> rr = rec[m[r]];
                    ready = ready && rr.tag[wi] == t;
#pragma unroll
                    for (int c = 0; c < D; ++c) xs[r][c] = rr.x[c];
                }
            if (ready) {
                run_iteration<D, KERN, SPLIT>(a, kbase + e, m, xs, rec);
            } else {
                const uint32_t t1 = tag_of(g + 1u, e);
#pragma unroll
                for (int r = 0; r < RBMR_MAX_P; ++r)
                    if (r < (int)a.p) atomicMin(&rec[m[r]].tag[wo], t1);
                pend = true;
            }
        }
        // queue the pending iterations: one atomic per wavefront
        const uint64_t mask = __ballot(pend);
        if (mask) {
            const uint32_t lane = __lane_id();
            const int leader = __ffsll((unsigned long long)mask) - 1;
            uint32_t q0 = 0;
            if ((int)lane == leader) q0 = atomicAdd(&counts[L + 1], (uint32_t)__popcll(mask));
            q0 = __shfl(q0, leader);
            if (pend) lout[q0 + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull))] = e;
        }
    }
}

// The iterations still pending after the last multi-workgroup round: one
// workgroup continues the rounds on its own for at most `budget` rounds,
// then runs whatever is left in iteration order on one thread.  Between its
// rounds a device-scope release and acquire around the barrier make every
// tag update (an atomic min carried out past the caches) and every position
// of a round visible before the next reads them; the tags are read with
// device-scope atomic loads.  Every round runs at least the earliest pending
// iteration, so the rounds make progress.
template <int D, int KERN, bool SPLIT>
__global__ __launch_bounds__(FIN_TPB) void k_rbmr_finish(RbmrArgs a, uint32_t rounds, uint32_t g, uint32_t budget,
                                                         uint64_t kbase, RRec<D> *rec, uint32_t *list0,
                                                         uint32_t *list1, const uint32_t *__restrict__ counts)
{
    __shared__ uint32_t s_cnt;
    __shared__ uint32_t red[FIN_TPB];
    uint32_t *lists[2] = {list0, list1};
    uint32_t n = counts[rounds];
    uint32_t L = rounds;
    for (uint32_t it = 0; n > 0 && it < budget; ++it, ++L) {
        const uint32_t *lin = lists[L & 1u];
        uint32_t *lout = lists[(L + 1u) & 1u];
        const uint32_t wi = L & 1u, wo = wi ^ 1u;
        if (threadIdx.x == 0) s_cnt = 0;
        __syncthreads();
        for (uint32_t idx = threadIdx.x; idx < n; idx += FIN_TPB) {
            const uint32_t e = lin[idx];
            uint32_t m[RBMR_MAX_P];
            draw_members(a, kbase + e, m);
            const uint32_t t = tag_of(g + L, e);
            // the positions are loaded with the tags (they are used only if
            // the iteration is ready, and then nothing else writes them)
            float xs[RBMR_MAX_P][D];
            load_positions<D>(a, rec, m, xs);
            bool ready = true;
#pragma unroll
            for (int r = 0; r < RBMR_MAX_P; ++r)
                if (r < (int)a.p)
                    ready = ready && __hip_atomic_load(&rec[m[r]].tag[wi], __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT) == t;
            if (ready) {
                run_iteration<D, KERN, SPLIT>(a, kbase + e, m, xs, rec);
            } else {
                const uint32_t t1 = tag_of(g + L + 1u, e);
#pragma unroll
                for (int r = 0; r < RBMR_MAX_P; ++r)
                    if (r < (int)a.p) atomicMin(&rec[m[r]].tag[wo], t1);
                lout[atomicAdd(&s_cnt, 1u)] = e;
            }
        }
        // this round's tag updates and positions are complete before the
        // next round reads them (the finishing workgroup runs alone, so the
        // device-scope fences have little to write back)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        n = s_cnt;
        __syncthreads();
    }
    if (n == 0) return;
    // the rest in iteration order (the workgroup finds the next one)
    const uint32_t *list = lists[L & 1u];
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
            uint32_t m[RBMR_MAX_P];
            draw_members(a, kbase + e, m);
            float xs[RBMR_MAX_P][D];
            load_positions<D>(a, rec, m, xs);
            run_iteration<D, KERN, SPLIT>(a, kbase + e, m, xs, rec);
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
    auto *rec = reinterpret_cast<RRec<D> *>(w + lay.off_rec);
    uint32_t *lists[2] = {reinterpret_cast<uint32_t *>(w + lay.off_list0),
                          reinterpret_cast<uint32_t *>(w + lay.off_list1)};
    auto *counts = reinterpret_cast<uint32_t *>(w + lay.off_counts);
    const uint32_t R = lay.rounds;
    const dim3 gn((a.n + TPB - 1) / TPB);
    hipLaunchKernelGGL(k_rbmr_pack<D>, gn, dim3(TPB), 0, st, a.n, x, rec);
    uint32_t g = 1;
    for (uint64_t done = 0; done < niter;) {
        const uint32_t wcur = (uint32_t)((niter - done) < lay.window ? (niter - done) : lay.window);
        if (g + R + FIN_BUDGET + 1u > 1022u) {
            hipLaunchKernelGGL(k_rbmr_retag<D>, gn, dim3(TPB), 0, st, a.n, rec);
            g = 1;
        }
        const uint32_t g0 = (wcur + TPB - 1) / TPB;
        hipLaunchKernelGGL(k_rbmr_draw<D>, dim3(g0), dim3(TPB), 0, st, a, kbase + done, wcur, g, rec, counts, R);
        for (uint32_t L = 0; L < R; ++L) {
            uint32_t grid = L == 0 ? g0 : g0 >> L;
            if (grid < 64u) grid = g0 < 64u ? g0 : 64u;
            hipLaunchKernelGGL((k_rbmr_round<D, KERN, SPLIT>), dim3(grid), dim3(TPB), 0, st, a, L, g + L, kbase + done,
                               wcur, rec, lists[L & 1u], lists[(L + 1u) & 1u], counts);
        }
        hipLaunchKernelGGL((k_rbmr_finish<D, KERN, SPLIT>), dim3(1), dim3(FIN_TPB), 0, st, a, R, g, FIN_BUDGET,
                           kbase + done, rec, lists[0], lists[1], counts);
        g += R + FIN_BUDGET + 1u;
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

RbmrLayout rbmr_layout(uint32_t n, uint32_t d, uint32_t window, uint32_t rounds)
{
    RbmrLayout l{};
    l.window = window;
    l.rounds = rounds;
    size_t o = 0;
    l.off_rec = o;
    o = al256(o + (size_t)n * (d <= 2 ? 16u : 32u));
    l.off_list0 = o;
    o = al256(o + (size_t)window * sizeof(uint32_t));
    l.off_list1 = o;
    o = al256(o + (size_t)window * sizeof(uint32_t));
    l.off_counts = o;
    o = al256(o + (size_t)(rounds + 1) * sizeof(uint32_t));
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
