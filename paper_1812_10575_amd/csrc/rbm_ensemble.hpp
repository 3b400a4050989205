// Batched ensemble of independent RBM-1 systems: launch parameters.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "rbm_device.hpp"

#define RBM_ENS_LDS 4096     // largest system kept in LDS for all steps (d = 2)
#define RBM_ENS_MAXB 256     // buckets of a streamed system at most
#define RBM_ENS_MAXN (256 * 1024)

namespace rbm {

struct EnsSys {
    uint32_t off;     // first particle of the system in the packed arrays
    uint32_t n;       // particles
    uint32_t k0, k1;  // Philox key (seed)
    float inv_last;   // 1 / (s - 1) of the last batch, s = p + n mod p
    uint32_t pad[3];
};

struct EnsLaunch {
    StepArgs base;      // shared model parameters; step index in base.m
    int64_t nsteps;
    uint32_t nitems;    // work items in the queue
    uint32_t lds_max;   // a whole-workgroup system up to this size stays in LDS
    uint32_t wg;        // threads per workgroup: 1024 (4096 records of LDS) or 512 (2048)
    uint32_t team;      // threads per system of a grouped item (64 .. wg)
    uint32_t bmean;     // mean bucket of a streamed system
    uint32_t grid;      // persistent workgroups
    void *sys;          // per-system table (EnsSys)
    const uint32_t *order;  // systems in queue order
    const uint2 *items;     // item q: systems order[x .. x + y)
    uint32_t *next;     // queue counter; next[1]: error flags
    float *x;           // packed positions, by (system, id), in and out
    void *state, *stage;     // the two record buffers of the streamed systems
    uint32_t *wst, *wst2;    // their PERM words
    uint32_t *flags;    // == next + 1
};

hipError_t launch_ensemble(const EnsLaunch &e, int kernel, hipStream_t st);

}  // namespace rbm
