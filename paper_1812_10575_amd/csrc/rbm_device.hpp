// Device building blocks of the RBM-1 step for gfx950: the Philox4x32-10
// counter-based generator, uniform and Gaussian transforms, particle records
// and the pair kernels K of eq. (1.2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rbm {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).  Ten rounds; each
// multiplies counter words 0 and 2 by fixed odd constants, swaps the
// product halves into place and mixes words 1, 3 and the key in by xor.  The
// key advances by the two Weyl constants between rounds.  The key is uniform
// across a wavefront, so its schedule stays in scalar registers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // 32x32 -> 64-bit products: one v_mad_u64_u32 each
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1,
                       (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ uint32_t word_of(const uint4 &v, uint32_t j)
{
    return j == 0 ? v.x : (j == 1 ? v.y : (j == 2 ? v.z : v.w));
}

// Stream words of the counter (word 2 of the counter selects the stream).
enum : uint32_t { STREAM_PERM = 0u, STREAM_NOISE = 1u };

// Uniform on (0,1) with 24 significant bits, so the value is exact in FP32:
// (2 * (w >> 9) + 1) * 2^-24.
__device__ __forceinline__ float u24(uint32_t w)
{
    return (float)(2u * (w >> 9) + 1u) * 0x1p-24f;
}

// Box-Muller: two independent standard normals from two uniforms,
// r = sqrt(-2 ln u0), angle 2 pi u1.  The hardware sine and cosine take
// their argument in revolutions, so sin(2 pi u1) is v_sin_f32(u1); the
// hardware logarithm is base 2 (ln u = log2(u) ln 2).
__device__ __forceinline__ void box_muller(float u0, float u1, float &z0, float &z1)
{
    const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u0));
    z0 = r * __builtin_amdgcn_cosf(u1);
    z1 = r * __builtin_amdgcn_sinf(u1);
}

// D standard normals of particle `id` at step m: NOISE block (id, m, 1, sys),
// pairs (u0,u1) and (u2,u3).  Only the pairs needed for D are evaluated.
template <int D>
__device__ __forceinline__ void noise(uint32_t id, uint32_t m, uint32_t sys, uint32_t k0,
                                      uint32_t k1, float (&z)[D])
{
    const uint4 w = philox4x32_10(make_uint4(id, m, STREAM_NOISE, sys), k0, k1);
    float a, b;
    box_muller(u24(w.x), u24(w.y), a, b);
    z[0] = a;
    if constexpr (D >= 2) z[1] = b;
    if constexpr (D >= 3) {
        float c, e;
        box_muller(u24(w.z), u24(w.w), c, e);
        z[2] = c;
    }
}

// ---------------------------------------------------------------------------
// Particle record: position and id travel together through the permuted
// layouts.  d = 3 is one 16-byte vector.
// ---------------------------------------------------------------------------
template <int D> struct Rec;
template <> struct alignas(8) Rec<1> { float x[1]; uint32_t id; };
template <> struct Rec<2> { float x[2]; uint32_t id; };
template <> struct alignas(16) Rec<3> { float x[3]; uint32_t id; };

// ---------------------------------------------------------------------------
// Pair kernels, written as K(x) = s(|x|^2) x:
//   GAUSS       s = -exp(-r2)
//   SOFTCOULOMB s = 1 / (r2 + a)
//   ATTREP      s = 1 / (r2 + a) - 1
//   LINEAR      s = -a
//   HAMILTON    s = 1 / (r2 + a) on the first component only: records are
//               (x, u) of the second-order system, the force acts between
//               positions (r2 = (xi - xj)^2) and its u-component is zero
// ---------------------------------------------------------------------------
enum : int { K_GAUSS = 0, K_SOFTCOULOMB = 1, K_ATTREP = 2, K_LINEAR = 3, K_HAMILTON = 4 };

// Components of a record that the pair kernel reads and acts on.
template <int D, int KERN>
constexpr int kdim()
{
    return KERN == K_HAMILTON ? 1 : D;
}

template <int KERN>
__device__ __forceinline__ float pair_scale(float r2, float a)
{
    if constexpr (KERN == K_GAUSS) {
        return -__builtin_amdgcn_exp2f(-1.4426950408889634f * r2);  // -e^{-r2}
    } else if constexpr (KERN == K_SOFTCOULOMB || KERN == K_HAMILTON) {
        return __builtin_amdgcn_rcpf(r2 + a);
    } else if constexpr (KERN == K_LINEAR) {
        return -a;  // K(x) = -a x
    } else {
        return __builtin_amdgcn_rcpf(r2 + a) - 1.0f;
    }
}

// acc += K(xi - xj)
template <int D, int KERN>
__device__ __forceinline__ void add_pair(const float (&xi)[D], const float *xj, float a,
                                         float (&acc)[D])
{
    constexpr int DK = kdim<D, KERN>();
    float dx[DK];
    float r2 = 0.0f;
#pragma unroll
    for (int k = 0; k < DK; ++k) {
        dx[k] = xi[k] - xj[k];
        r2 = fmaf(dx[k], dx[k], r2);
    }
    const float s = pair_scale<KERN>(r2, a);
#pragma unroll
    for (int k = 0; k < DK; ++k) acc[k] = fmaf(s, dx[k], acc[k]);
}

// Parameters of one step, passed by value to every kernel of the step.
struct StepArgs {
    uint32_t n;      // particles
    uint32_t p;      // batch size
    uint32_t nbat;   // floor(n / p) batches; the last takes the leftover
    uint32_t m;      // step index (Philox counter word 1)
    uint32_t k0, k1; // Philox key
    uint32_t sys;    // Philox counter word 3
    uint32_t nbuck;  // fine buckets of the key-space partition
    float inv_p1;    // 1 / (p - 1)
    float inv_last;  // 1 / (s - 1) for the last batch, s = p + n mod p
    float a;         // kernel softening
    float beta;      // -grad V = -beta x
    float dt;        // time step
    float ssd;       // sigma * sqrt(dt)
    uint32_t pm;     // step whose noise the stored positions still lack
    float pssd;      // its amplitude (0: none pending)
    uint32_t scheme; // 0: Euler-Maruyama; batches of two move by their exact pair flow,
                     // 1: of K(x) = x/|x|^2 (additive noise), 2: of K(x) = -a x, with
                     //    multiplicative noise x <- x exp(sigma sqrt(dt) z - sigma^2 dt / 2);
                     // 3: Verlet for records (x, u) of the second-order system (no noise)
    float flowc;     // scheme 2: e^{-2 a dt}, the decay of a pair's difference over a step
};

// Exact flow over a step of a batch of two particles under K(x) = -a x (the
// trading interaction of the wealth model, Sec. 5): the pair's mean stays
// and the difference decays by flowc = e^{-2 a dt}; written for one member,
// like pair_flow.
template <int D>
__device__ __forceinline__ void pair_flow_linear(float flowc, const float (&xi)[D], const float *xj, float (&yi)[D])
{
#pragma unroll
    for (int k = 0; k < D; ++k) yi[k] = fmaf(0.5f * flowc, xi[k] - xj[k], 0.5f * (xi[k] + xj[k]));
}

// Exact flow over a time dt of a batch of two particles under
// K(x) = x/|x|^2 (Sec. 2.3 splitting for singular K, the scheme of Sec. 4.2):
// the centre c = (xi + xj)/2 stays, u = xi - xj keeps its direction and
// |u|^2 grows by 4 dt, so yi = c + g u/2 with g = sqrt(1 + 4 dt/|u|^2).
// Written for one member; the partner's call (with the arguments swapped)
// gives c - g u/2 with the same roundings.  u = 0 stays at c.
template <int D>
__device__ __forceinline__ void pair_flow(float dt, const float (&xi)[D], const float *xj, float (&yi)[D])
{
    float c[D], u[D], r2 = 0.0f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        c[k] = 0.5f * (xi[k] + xj[k]);
        u[k] = xi[k] - xj[k];
        r2 = fmaf(u[k], u[k], r2);
    }
    const float h = r2 > 0.0f ? 0.5f * sqrtf(fmaf(4.0f * dt, __builtin_amdgcn_rcpf(r2), 1.0f)) : 0.0f;
#pragma unroll
    for (int k = 0; k < D; ++k) yi[k] = fmaf(h, u[k], c[k]);
}

// Pair-flow schemes: a batch of two moves by the exact flow of its pair.
__device__ __forceinline__ bool pair_flow_scheme(const StepArgs &s)
{
    return s.scheme == 1u || s.scheme == 2u;
}

// Batch [bs, be) of sorted rank r: groups of p, the last also takes the
// n mod p leftover ranks.
__device__ __forceinline__ void batch_of(const StepArgs &s, uint32_t r, uint32_t &bs, uint32_t &be)
{
    uint32_t q = r / s.p;
    if (q > s.nbat - 1) q = s.nbat - 1;
    bs = q * s.p;
    be = (q == s.nbat - 1) ? s.n : bs + s.p;
}

// The drift part of the step, x <- x + dt (-beta x + F).  The noise of the
// same step, sigma sqrt(dt) z(id, m), is added by whichever kernel reads the
// positions next (deferred noise, below), where the ALU is otherwise idle.
// The FMAs are written out so that every kernel rounds the update the same
// way (no contraction left to the compiler).
//
// Scheme 3 (the second-order system x'' = b(x) + F, b = -beta x, Sec. 4.1
// and Appendix A): the record is (x, u), u the Verlet velocity, and
//   u <- u + h (F - beta x),  x <- x + dt u,   h = dt/2 at step 0, else dt,
// which is x_1 = x_0 + dt v_0 + dt^2 F_0 / 2 and, with u = (x_m - x_{m-1})/dt,
// x_{m+1} = 2 x_m - x_{m-1} + dt^2 F_m.
template <int D>
__device__ __forceinline__ void drift_update(const StepArgs &s, float (&x)[D], const float (&f)[D])
{
    if constexpr (D == 2) {
        if (s.scheme == 3u) {
            const float h = s.m == 0u ? 0.5f * s.dt : s.dt;
            x[1] = fmaf(h, fmaf(-s.beta, x[0], f[0]), x[1]);
            x[0] = fmaf(s.dt, x[1], x[0]);
            return;
        }
    }
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = fmaf(s.dt, fmaf(-s.beta, x[k], f[k]), x[k]);
}

// Add the noise the stored positions still lack: sigma sqrt(dt) z(id, pm).
template <int D>
__device__ __forceinline__ void add_pending_noise(const StepArgs &s, float *x, uint32_t id)
{
    if (s.pssd != 0.0f) {
        float z[D];
        noise<D>(id, s.pm, s.sys, s.k0, s.k1, z);
        if (s.scheme == 2) {
            // the exact factor of dY = sigma Y dB over the step
            const float h = -0.5f * s.pssd * s.pssd;
#pragma unroll
            for (int k = 0; k < D; ++k) x[k] = x[k] * expf(fmaf(s.pssd, z[k], h));
        } else {
#pragma unroll
            for (int k = 0; k < D; ++k) x[k] = fmaf(s.pssd, z[k], x[k]);
        }
    }
}

// Forward Euler-Maruyama in one go: x <- x + dt (-beta x + F) + sigma sqrt(dt) z.
template <int D>
__device__ __forceinline__ void em_update(const StepArgs &s, float (&x)[D], const float (&f)[D],
                                          uint32_t id)
{
    if (s.scheme == 3u) {  // Verlet: no noise
        drift_update<D>(s, x, f);
        return;
    }
    float z[D];
    if (s.ssd != 0.0f) {
        noise<D>(id, s.m, s.sys, s.k0, s.k1, z);
    } else {
#pragma unroll
        for (int k = 0; k < D; ++k) z[k] = 0.0f;
    }
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = fmaf(s.ssd, z[k], fmaf(s.dt, fmaf(-s.beta, x[k], f[k]), x[k]));
}

}  // namespace rbm
