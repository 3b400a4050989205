// RBM-r (random batches drawn with replacement, one batch per iteration):
// launch parameters and the host driver.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "rbm_device.hpp"

#define RBMR_MAX_P 8
#define RBMR_MAX_WINDOW (1u << 22)

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

// Workspace: the particle records [n] (16 bytes for d <= 2, 32 for d = 3),
// two queues [window] and the round counters [rounds + 1].
struct RbmrLayout {
    size_t off_rec, off_list0, off_list1, off_counts, bytes;
    uint32_t window, rounds;
};

RbmrLayout rbmr_layout(uint32_t n, uint32_t d, uint32_t window, uint32_t rounds);

// Iterations kbase .. kbase + niter - 1 on the positions x ([n][d], by id).
hipError_t rbmr_launch(const RbmrArgs &a, int d, int kernel, const RbmrLayout &lay, void *ws, float *x,
                       uint64_t kbase, uint64_t niter, hipStream_t st);

}  // namespace rbm
