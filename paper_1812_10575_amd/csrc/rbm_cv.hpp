// Control-variate constants and launchers (kernels in rbm_cv.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rbm_device.hpp"

#define CV_NP 6432     // parameters of one MLP
#define CV_NB 12288    // BF16 copies of one MLP: W2, W2^T, W3, W3^T
#define CV_NO 32       // outputs: [component 2][rank 16]
#define CV_OW1 0
#define CV_OB1 128
#define CV_OW2 192
#define CV_OB2 4288
#define CV_OW3 4352
#define CV_OB3 6400
#define CV_VACC 288    // dW1 (128) + db1 (64) + db2 (64) + db3 (32)
#define CV_MAXR 128    // records per control-variate batch workgroup
#define CV_SUM_WG 1024 // workgroups of the sum of c over the particles
#define CV_GRAD_WG 256 // workgroups of one gradient evaluation
#define CV_MAX_P 64

namespace rbm {

inline uint32_t cv_batches_per_wg(uint32_t p)
{
    const uint32_t q = CV_MAXR / p;
    return q ? q : 1u;
}

hipError_t cv_launch_glorot(float *master, uint64_t seed, hipStream_t st);
hipError_t cv_launch_prep(const float *master, __bf16 *wb, hipStream_t st);
hipError_t cv_launch_features(const float *master, const __bf16 *wb, const float *x, uint32_t n,
                              float *a, float *c, hipStream_t st);
// S = sum of c over the n records of `state` (pending noise of s added), of
// c rounded to BF16; cout (may be null): those rounded c, [n][32] BF16.
hipError_t cv_launch_csum(const StepArgs &s, const void *state, const float *master,
                          const __bf16 *wb, double *part, double *S, __bf16 *cout, hipStream_t st);
// Batch forces over key-ordered records `sorted`, with c of the same records
// in c ([n][32] BF16) and S.
hipError_t cv_launch_batch(const StepArgs &s, int kernel, const void *sorted, const __bf16 *c,
                           const float *master, const __bf16 *wb, const double *S, void *dst, float *fout,
                           hipStream_t st);
hipError_t cv_launch_grad(uint32_t npairs, float ka, const float *xs, const float *ys,
                          const float *snap, uint32_t nsnap, uint32_t n, uint32_t step,
                          uint64_t seed, const float *master, const __bf16 *wb, float *gpart,
                          float *lpart, uint32_t *nwg_out, hipStream_t st);
hipError_t cv_launch_reduce(uint32_t nwg, const float *gpart, const float *lpart, float *grad_out,
                            float *loss_out, int adam, float lr, int t, float *master, float *am,
                            float *av, hipStream_t st);

}  // namespace rbm
