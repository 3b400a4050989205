// Workspace plan and launcher entry points shared by the C ABI and the
// kernels of the RBM-1 step.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "rbm_device.hpp"

// Records one sort workgroup holds in LDS (75 KB at d = 3, so two
// workgroups share a CU's 160 KB).  Buckets average RBM_BUCKET_MEAN records;
// a bucket above the capacity is 17 standard deviations out.
#define RBM_SORT_CAP 2816
#define RBM_BUCKET_MEAN 2048
#define RBM_MAX_BUCKETS 16384

namespace rbm {

struct Plan {
    uint32_t n, p, nbat;
    int d, kernel;
    uint32_t nbuck;   // 1: the whole system is sorted by one workgroup
    uint32_t tile;    // slots per count/scatter workgroup (multiple of 4)
    uint32_t ntiles;
    size_t rec_bytes;
    size_t off_state, off_stage, off_w, off_scratch, off_cnt, off_tot, off_bstart, off_flags;
    size_t total;
};

// ev: NULL, or RBM_NPHASES + 1 events recorded before the first and after
// every phase of the step.
hipError_t launch_step(const Plan &pl, const StepArgs &s, int d, int kernel, void *ws,
                       hipStream_t st, void *dst_state, float *fout, hipEvent_t *ev);
hipError_t launch_init(const Plan &pl, int d, const float *x0, const uint32_t *slots, void *ws,
                       hipStream_t st);
hipError_t launch_positions(const Plan &pl, int d, const void *ws, float *x, uint32_t *ids,
                            hipStream_t st);
hipError_t launch_direct(const StepArgs &s, int d, int kernel, const float *x,
                         const uint32_t *ids, uint32_t nids, float *out, int step,
                         hipStream_t st);

}  // namespace rbm
