// Workspace plan and launcher entry points shared by the C ABI and the
// kernels of the RBM-1 step.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "rbm_device.hpp"

// Capacity of the one-workgroup path (the whole system in LDS, 75 KB at
// d = 3).
#define RBM_SINGLE_CAP 2816
// Fine buckets average at most RBM_BUCKET_MEAN records (1680 at N = 2^24;
// every N up to RBM_MAX_N needs fewer than RBM_MAX_FINE buckets); a sort
// workgroup of 512 threads holds up to RBM_SORT_CAP (8.4 standard deviations
// above the largest mean; a fuller bucket is reported, not dropped) in 32 KB
// of LDS, four records per thread, so four workgroups share a CU and the
// fused sort kernel fits 64 VGPRs (eight waves per SIMD).  Buckets this large
// keep the coarse buckets few (78 at N = 2^24), so the runs that a scatter
// writes per coarse bucket are long.  The sizes below are compile-time
// choices (-D overrides give the same results with other bucket shapes:
// RBM_SORT_CAP / RBM_SORT_TPB records per thread must stay whole, and
// 2^RBM_SORT_SBITS sub-buckets a multiple of RBM_SORT_TPB).
#ifndef RBM_BUCKET_MEAN
#define RBM_BUCKET_MEAN 1700
#endif
#ifndef RBM_SORT_CAP
#define RBM_SORT_CAP 2048
#endif
#ifndef RBM_SORT_TPB
#define RBM_SORT_TPB 512
#endif
#ifndef RBM_SORT_SBITS
#define RBM_SORT_SBITS 11
#endif
#define RBM_KEY_SETS 16
#define RBM_MAX_FINE 32768
// Scatter and split workgroups: threads holding a fixed number of records
// each, staged through LDS a few per thread at a time.  The coarse scatter
// runs 512 threads with 16 records, 4 per round (two workgroups per CU); the
// split 1024 threads with 12, 6 per round, so that each LDS round (6144
// records) writes runs three times as long (fewer partly written lines) with
// one workgroup per CU.
#define RBM_SCATTER_TPB 512
#define RBM_SCATTER_P 16
#define RBM_LVL_RPT 4
#ifndef RBM_SPLIT_TPB
#define RBM_SPLIT_TPB 1024
#endif
#ifndef RBM_SPLIT_P
#define RBM_SPLIT_P 12
#endif
#ifndef RBM_SPLIT_RPT
#define RBM_SPLIT_RPT 6
#endif
#define RBM_TILE (RBM_SCATTER_P * RBM_SCATTER_TPB)
#define RBM_CHUNK (RBM_SPLIT_P * RBM_SPLIT_TPB)
// A plan with fewer than RBM_SPLIT_FEW split chunks of RBM_CHUNK records
// (N below about 2^23) splits chunks of RBM_CHUNK_SMALL instead (4 records
// per thread, one staging round) so that more workgroups share the GPU.
#define RBM_SPLIT_SMALL_P 4
#define RBM_CHUNK_SMALL (RBM_SPLIT_SMALL_P * RBM_SPLIT_TPB)
#define RBM_SPLIT_FEW 512
#ifndef RBM_SPLIT_SHIFT
#define RBM_SPLIT_SHIFT 7
#endif
// Coarse buckets (digits of the scatter level) at most: the per-digit arrays
// of the staging levels and of the fused sort output, and the one-byte
// coarse digits of the key passes.
#define RBM_MAX_COARSE 256
// Fused steps: fine buckets per tile of the cross counts (records of a tile
// of step m's fine buckets counted by their coarse bucket of step m + 1).
#define RBM_CROSS_G 8

namespace rbm {

// Kernel phases of one step (the order of include/rbm.h's RBM_PHASE_*).
constexpr int RBM_NPH = 7;

struct Plan {
    uint32_t n, p, nbat;
    int d, kernel;
    uint32_t nbuck;   // fine buckets (1: the whole system is sorted by one workgroup)
    uint32_t nb1;     // coarse buckets
    uint32_t shift;   // log2(fine buckets per coarse bucket), 0 without a split level
    uint32_t jmax;    // split chunks per coarse bucket
    uint32_t chunk;   // records per split chunk: RBM_CHUNK or RBM_CHUNK_SMALL
    uint32_t ntiles;  // coarse-scatter tiles of RBM_TILE slots
    uint32_t tilef;   // slots per key-count tile
    uint32_t ntf;     // key-count tiles
    uint32_t kb;      // the key passes of up to kb consecutive steps run as one launch
    uint32_t nsets;   // key sets in the workspace: kb, or two banks of kb with fuse
    uint32_t cap;     // records a sort workgroup holds (RBM_SORT_CAP)
    // fused steps (split level present, no control variate): inside a group
    // of steps sharing the key passes, the sort kernel of step m writes its
    // updated records straight into the coarse buckets of step m + 1
    bool fuse;
    uint32_t ntx;     // cross-count tiles of RBM_CROSS_G fine buckets
    size_t rec_bytes;
    size_t off_state, off_scratch, off_stage1, off_w1, off_stage2, off_w2;
    size_t off_kcnt, off_ftot, off_fstart, off_fcur, off_cstart, off_ccur, off_flags;
    size_t off_xrow, off_xtsum, off_xbase, off_fixpos, off_xdig;
    // control variate (cv != 0)
    int cv;
    size_t off_sorted, off_cvc, off_cvmaster, off_cvam, off_cvav, off_cvwb, off_cvspart, off_cvS;
    size_t off_cvgpart, off_cvlpart, off_cvgrad, off_cvloss;
    size_t total;
};

// Key passes (bucket counts, totals, starts and run cursors) of steps s.m ..
// s.m + count - 1 into key sets base .. base + count - 1 (count <= pl.kb,
// base + count <= pl.nsets); with pl.fuse also the coarse digits of every
// slot and the cross counts and coarse write offsets of the transitions
// between consecutive sets of the group, and (xsrc < pl.nsets) of the one
// from key set xsrc (made earlier, the step before s.m) into set base.  ev:
// four phase events (may be null).
hipError_t launch_keys(const Plan &pl, const StepArgs &s, uint32_t count, void *ws, hipStream_t st,
                       hipEvent_t *ev, uint32_t base = 0, uint32_t xsrc = 0xffffffffu);
// One step with the keys of key set `set`; keys_ready == false computes
// them first (into set 0).  fuse (pl.fuse and keys_ready only): bit 0, the
// coarse buckets of this step were written by the previous step's sort
// kernel (no coarse scatter; the split adds the pending noise); bit 1, this
// step's sort kernel writes the coarse buckets of the next step instead of
// the slot-ordered state, placed by the transition stored with key set
// `set` (made by launch_keys).
hipError_t launch_step(const Plan &pl, const StepArgs &s, int d, int kernel, void *ws,
                       hipStream_t st, void *dst_state, float *fout, hipEvent_t *ev, uint32_t set = 0,
                       bool keys_ready = false, uint32_t fuse = 0);
hipError_t launch_init(const Plan &pl, int d, const float *x0, const uint32_t *slots, void *ws,
                       hipStream_t st);
// x != NULL: positions by id, with the pending noise of s added.
hipError_t launch_positions(const Plan &pl, const StepArgs &s, int d, const void *ws, float *x,
                            uint32_t *ids, hipStream_t st);
hipError_t launch_fill(uint32_t *p, size_t n, uint32_t v, hipStream_t st);
hipError_t launch_sqerr(const float *f, uint32_t n, const uint32_t *ids, uint32_t nids, const float *fref, int d,
                        double *out, hipStream_t st);
// m2 (force mode only, may be null): 1/(N-1) sum_j |K(X_i - X_j)|^2 per target
hipError_t launch_direct(const StepArgs &s, int d, int kernel, const float *x,
                         const uint32_t *ids, uint32_t nids, float *out, int step,
                         hipStream_t st, float *m2 = nullptr);

}  // namespace rbm
