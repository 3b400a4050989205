// RBM-r (random batches drawn with replacement, one batch per iteration):
// launch parameters and the host driver.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "rbm_device.hpp"

#define RBMR_MAX_P 8
#define RBMR_MAX_WINDOW (1u << 22)
#define RBMR_MAX_ROUNDS 255u
// schedule sort: particle buckets (count and size) and counting workgroups
#define RBMR_MAX_NBK 8192u
#define RBMR_MAX_PB 4096u
#define RBMR_MAX_NBLK 256u

namespace rbm {

struct RbmrArgs {
    uint32_t n;       // particles
    uint32_t p;       // batch size, 2 .. RBMR_MAX_P
    uint32_t k0, k1;  // Philox key
    uint32_t sys;     // Philox counter word 3
    float inv_p1;     // 1 / (p - 1)
    float a, beta, dt;
    float ssd;        // sigma sqrt(dt)
};

// Workspace: the particle records [n] (16 bytes: tag and position), the
// window's entries (member, iteration) sorted into particle buckets
// [window p] (8 bytes), grouped by particle [window p], their successors
// [window p], the bucket counts per counting workgroup, the bucket totals
// and starts, two round queues (256 segments of window / 256 + 512
// entries) and the queue lengths [rounds + 2][256].
struct RbmrLayout {
    size_t off_rec, off_ent, off_lst, off_succ, off_cnt, off_tot, off_bst, off_list0, off_list1, off_counts, bytes;
    uint32_t window, rounds;
    uint32_t bsh;  // log2 of the particles per bucket
    uint32_t nbk;  // buckets
    uint32_t ipb;  // iterations per counting workgroup
    uint32_t segcap;  // entries per queue segment
};

RbmrLayout rbmr_layout(uint32_t n, uint32_t p, uint32_t window, uint32_t rounds);

// Iterations kbase .. kbase + niter - 1 on the positions x ([n][d], by id).
hipError_t rbmr_launch(const RbmrArgs &a, int d, int kernel, const RbmrLayout &lay, void *ws, float *x,
                       uint64_t kbase, uint64_t niter, hipStream_t st);

}  // namespace rbm
