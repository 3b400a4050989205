// Learned control variate for the RBM-1 batch force (d = 2), on BF16 matrix
// cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation).
//
// The kernel is split K(x - y) = a(x) . c(y) + K_res(x, y) with two MLPs
// a, c : R^2 -> R^32 (2 -> 64 -> 64 -> 32, GELU after the hidden layers; the
// 32 outputs are [component k = 0, 1][rank r = 0..15]).  The separable part
// is summed exactly through S = sum_j c(X_j) (FP64), the residual by the
// random batch (RBM applies to general kernels K(x, y), Sec. 2.3):
//
//   F_i = a(X_i) . (S - c(X_i)) / (N - 1)
//         + 1/(s - 1) sum_{j in batch, j != i} [K(X_i - X_j) - a(X_i) . c(X_j)]
//
// which is unbiased for any weights (Lemma 3.1 applied to K_res).
//
// Parameter vector of one net (FP32 master copy): W1[64][2], b1[64],
// W2[64][64], b2[64], W3[32][64], b3[32]; BF16 copies of W2, W3 and their
// transposes feed the matrix instructions.
//
// MFMA operand layout (16x16x32, wave64): lane l holds A[m = l % 16][k = 8(l/16)
// + i] and B[k = 8(l/16) + i][n = l % 16] for i < 8, and receives
// C[m = 4(l/16) + i][n = l % 16] for i < 4.
#include "rbm_cv.hpp"
#include "rbm_device.hpp"

namespace rbm {
namespace cvk {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 ld8(const __bf16 *p)
{
    return *reinterpret_cast<const bf16x8 *>(p);
}

// GELU in its tanh form, 0.5 z (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3))),
// written as z sigma(v) with v = 2 sqrt(2/pi) z (1 + 0.044715 z^2): one
// base-2 exponential and one reciprocal on the VALU.  The constants of v and
// of the change of base are folded, so that sigma takes two multiplies, one
// FMA and one add besides the two transcendental instructions:
// exp(-v) = 2^(z (A z^2 + B)), B = -2 sqrt(2/pi) log2(e), A = 0.044715 B.
constexpr float GELU_K = 1.5957691216057308f;  // 2 sqrt(2/pi)
constexpr float GELU_C = 0.044715f;
constexpr float GELU_B = -2.3022082f;          // -2 sqrt(2/pi) / ln 2
constexpr float GELU_A = -0.10294324f;         // 0.044715 GELU_B

__device__ __forceinline__ float gelu_sig(float z)
{
    const float w = z * fmaf(GELU_A, z * z, GELU_B);
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(w));
}

__device__ __forceinline__ float gelu(float z)
{
    return z * gelu_sig(z);
}

// d/dz [z sigma(v)] = sigma + z sigma (1 - sigma) v'(z), v' = K (1 + 3 C z^2)
__device__ __forceinline__ float gelu_grad(float z)
{
    const float sg = gelu_sig(z);
    return fmaf(z * sg * (1.0f - sg), GELU_K * fmaf(3.0f * GELU_C, z * z, 1.0f), sg);
}

struct NetP {
    const float *p;      // master parameters
    const __bf16 *W2;    // [64][64] (out, in)
    const __bf16 *W2T;   // [64][64] (in, out)
    const __bf16 *W3;    // [32][64]
    const __bf16 *W3T;   // [64][32]
};

__device__ __forceinline__ NetP net_of(const float *master, const __bf16 *wb, int net)
{
    NetP n;
    n.p = master + net * CV_NP;
    const __bf16 *b = wb + net * CV_NB;
    n.W2 = b;
    n.W2T = b + 4096;
    n.W3 = b + 8192;
    n.W3T = b + 10240;
    return n;
}

// ---------------------------------------------------------------------------
// Forward of 16 samples per wavefront (all waves of the workgroup call it
// together; each works on its own 16 rows).  X: [16][2] FP32.  H1, H2:
// [16][64] BF16 scratch; Z1, Z2: [16][64] FP32 pre-activations (kept for the
// backward pass when non-null); O: [16][ostride] FP32 outputs.
// ---------------------------------------------------------------------------
__device__ void fwd16(const NetP &n, const float *X, __bf16 *H1, __bf16 *H2, float *Z1, float *Z2,
                      float *O, int ostride)
{
    const int lane = threadIdx.x & 63, g = lane >> 4, col = lane & 15;
    // layer 1 on the vector ALU: lane f computes feature f of all 16 samples
    {
        const float w0 = n.p[CV_OW1 + 2 * lane], w1 = n.p[CV_OW1 + 2 * lane + 1];
        const float b = n.p[CV_OB1 + lane];
#pragma unroll 4
        for (int s = 0; s < 16; ++s) {
            const float z = fmaf(w0, X[2 * s], fmaf(w1, X[2 * s + 1], b));
            if (Z1) Z1[s * 64 + lane] = z;
            H1[s * 64 + lane] = (__bf16)gelu(z);
        }
    }
    __syncthreads();
    // layer 2: Z2 = H1 W2^T + b2 (M = 16 samples, N = 64, K = 64)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
            acc = mfma(ld8(H1 + col * 64 + 32 * ks + 8 * g), ld8(n.W2 + (16 * t + col) * 64 + 32 * ks + 8 * g), acc);
        const int nn = 16 * t + col;
        const float b = n.p[CV_OB2 + nn];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int s = 4 * g + i;
            const float z = acc[i] + b;
            if (Z2) Z2[s * 64 + nn] = z;
            H2[s * 64 + nn] = (__bf16)gelu(z);
        }
    }
    __syncthreads();
    // layer 3: O = H2 W3^T + b3 (N = 32)
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
            acc = mfma(ld8(H2 + col * 64 + 32 * ks + 8 * g), ld8(n.W3 + (16 * t + col) * 64 + 32 * ks + 8 * g), acc);
        const int nn = 16 * t + col;
        const float b = n.p[CV_OB3 + nn];
#pragma unroll
        for (int i = 0; i < 4; ++i) O[(4 * g + i) * ostride + nn] = acc[i] + b;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// parameters: Glorot-uniform initialisation and BF16 copies
// ---------------------------------------------------------------------------
// Weight qw of net `net` (counting the weights of W1, W2, W3 in storage
// order): (2u - 1) sqrt(6 / (fan_in + fan_out)), u the first uniform of
// Philox(ctr = (qw, net, 4, 0)).  Biases 0.
__global__ __launch_bounds__(256) void k_glorot(float *master, uint32_t k0, uint32_t k1)
{
    const uint32_t q = blockIdx.x * 256 + threadIdx.x;
    if (q >= 2 * CV_NP) return;
    const uint32_t net = q / CV_NP, e = q % CV_NP;
    int qw = -1;
    float lim = 0.0f;
    if (e < CV_OB1) {
        qw = e;
        lim = sqrtf(6.0f / 66.0f);
    } else if (e >= CV_OW2 && e < CV_OB2) {
        qw = 128 + (e - CV_OW2);
        lim = sqrtf(6.0f / 128.0f);
    } else if (e >= CV_OW3 && e < CV_OB3) {
        qw = 128 + 4096 + (e - CV_OW3);
        lim = sqrtf(6.0f / 96.0f);
    }
    float v = 0.0f;
    if (qw >= 0) {
        const uint4 w = philox4x32_10(make_uint4((uint32_t)qw, net, 4u, 0u), k0, k1);
        v = (2.0f * u24(w.x) - 1.0f) * lim;
    }
    master[q] = v;
}

__global__ __launch_bounds__(256) void k_prep(const float *__restrict__ master, __bf16 *__restrict__ wb)
{
    const uint32_t q = blockIdx.x * 256 + threadIdx.x;
    if (q >= 2 * 6144) return;
    const uint32_t net = q / 6144, e = q % 6144;
    const float *p = master + net * CV_NP;
    __bf16 *b = wb + net * CV_NB;
    if (e < 4096) {
        const uint32_t o = e / 64, i = e % 64;
        const __bf16 v = (__bf16)p[CV_OW2 + e];
        b[e] = v;                 // W2[o][i]
        b[4096 + i * 64 + o] = v; // W2T[i][o]
    } else {
        const uint32_t f = e - 4096, o = f / 64, i = f % 64;
        const __bf16 v = (__bf16)p[CV_OW3 + f];
        b[8192 + f] = v;               // W3[o][i]
        b[10240 + i * 32 + o] = v;     // W3T[i][o]
    }
}

// ---------------------------------------------------------------------------
// inference
// ---------------------------------------------------------------------------
struct FwdLds {
    float X[64][2];
    __bf16 H1[64][64];
    __bf16 H2[64][64];
    float O[64][CV_NO];
};

// a and c of n points (x [n][2]) -> out_a, out_c [n][32] (either may be null).
__global__ __launch_bounds__(256) void k_features(const float *__restrict__ master,
                                                  const __bf16 *__restrict__ wb,
                                                  const float *__restrict__ x, uint32_t n,
                                                  float *__restrict__ out_a, float *__restrict__ out_c)
{
    __shared__ FwdLds L;
    const int w = threadIdx.x >> 6;
    for (uint32_t base = blockIdx.x * 64; base < n; base += gridDim.x * 64) {
        if (threadIdx.x < 128) {
            const uint32_t s = threadIdx.x >> 1, c = threadIdx.x & 1;
            L.X[s][c] = base + s < n ? x[(size_t)(base + s) * 2 + c] : 0.0f;
        }
        __syncthreads();
        for (int net = 0; net < 2; ++net) {
            float *out = net == 0 ? out_a : out_c;
            if (!out) continue;
            const NetP np = net_of(master, wb, net);
            fwd16(np, &L.X[16 * w][0], &L.H1[16 * w][0], &L.H2[16 * w][0], nullptr, nullptr,
                  &L.O[16 * w][0], CV_NO);
            for (uint32_t e = threadIdx.x; e < 64 * CV_NO; e += 256) {
                const uint32_t s = e / CV_NO;
                if (base + s < n) out[(size_t)(base + s) * CV_NO + e % CV_NO] = L.O[s][e % CV_NO];
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// inference inside the step: the weights of a net are staged in LDS once per
// workgroup (rows padded to WP so that the 16 lanes of a fragment read hit
// different banks) and every wavefront runs 16-sample tiles on its own,
// with no workgroup barrier between the layers.
// ---------------------------------------------------------------------------
constexpr int WP = 72;

struct __align__(16) NetLds {
    __bf16 W2[64][WP];  // [out][in]
    __bf16 W3[32][WP];
    float w1[64][2];
    float b1[64], b2[64], b3[32];
};

__device__ void stage_net(NetLds &N, const float *master, const __bf16 *wb, int net)
{
    const NetP np = net_of(master, wb, net);
    for (int e = threadIdx.x; e < 64 * 8; e += blockDim.x) {
        const int r = e >> 3, c = (e & 7) * 8;
        *reinterpret_cast<bf16x8 *>(&N.W2[r][c]) = ld8(np.W2 + r * 64 + c);
    }
    for (int e = threadIdx.x; e < 32 * 8; e += blockDim.x) {
        const int r = e >> 3, c = (e & 7) * 8;
        *reinterpret_cast<bf16x8 *>(&N.W3[r][c]) = ld8(np.W3 + r * 64 + c);
    }
    for (int e = threadIdx.x; e < 128; e += blockDim.x) N.w1[e >> 1][e & 1] = np.p[CV_OW1 + e];
    for (int e = threadIdx.x; e < 64; e += blockDim.x) {
        N.b1[e] = np.p[CV_OB1 + e];
        N.b2[e] = np.p[CV_OB2 + e];
    }
    for (int e = threadIdx.x; e < 32; e += blockDim.x) N.b3[e] = np.p[CV_OB3 + e];
}

// One wavefront, 16 samples: lane l brings sample l % 16 (x0, x1) and gets
// out[t][i] = O[4 (l / 16) + i][16 t + l % 16] (t < 2, i < 4).  Layer 1 is
// computed straight into the A fragments (lane l: hidden units 32 ks +
// 8 (l / 16) + i of its sample); H2 goes through the wave's own LDS rows to
// change from the accumulator layout to the A layout.  Same operations and
// roundings as fwd16.
__device__ __forceinline__ void fwd_tile(const NetLds &N, float x0, float x1, __bf16 (*H2)[WP],
                                         float (&out)[2][4])
{
    const int lane = threadIdx.x & 63, g = lane >> 4, col = lane & 15;
    bf16x8 a1[2];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = 32 * ks + 8 * g + i;
            const float z = fmaf(N.w1[k][0], x0, fmaf(N.w1[k][1], x1, N.b1[k]));
            a1[ks][i] = (__bf16)gelu(z);
        }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) acc = mfma(a1[ks], ld8(&N.W2[16 * t + col][32 * ks + 8 * g]), acc);
        const float b = N.b2[16 * t + col];
#pragma unroll
        for (int i = 0; i < 4; ++i) H2[4 * g + i][16 * t + col] = (__bf16)gelu(acc[i] + b);
    }
    // the wave's own LDS writes are seen by its later reads (LDS operations of
    // one wavefront complete in order); keep the compiler from moving them
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
            acc = mfma(ld8(&H2[col][32 * ks + 8 * g]), ld8(&N.W3[16 * t + col][32 * ks + 8 * g]), acc);
        const float b = N.b3[16 * t + col];
#pragma unroll
        for (int i = 0; i < 4; ++i) out[t][i] = acc[i] + b;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Partial sums of c(X_j) over the records (pending noise of s added, if
// any): part[wg][32] in FP64, and c itself to cout[j][32] when cout is not
// null.  c is rounded to BF16 where it is produced: the sums add the
// rounded values, so that S and the c that phase B reads are the same
// numbers (the residual force stays exactly unbiased), and phase B reads
// half the bytes.  Workgroup wg takes tiles of 256 records wg, wg + G, ...;
// each lane sums its samples in tile order, then the lanes and waves of the
// workgroup are added in a fixed order.
struct SumLds {
    NetLds net;
    float X[256][2];
    __bf16 H2[4][16][WP];
    double red[4][4][CV_NO];
};

__global__ __launch_bounds__(256) void k_csum(StepArgs s, const Rec<2> *__restrict__ state,
                                              const float *__restrict__ master,
                                              const __bf16 *__restrict__ wb,
                                              double *__restrict__ part, __bf16 *__restrict__ cout)
{
    __shared__ SumLds L;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, col = lane & 15;
    stage_net(L.net, master, wb, 1);
    double acc[2] = {0.0, 0.0};
    for (uint32_t base = blockIdx.x * 256; base < s.n; base += gridDim.x * 256) {
        {
            const uint32_t k = base + tid;
            float xy[2] = {0.0f, 0.0f};
            if (k < s.n) {
                Rec<2> r = state[k];
                add_pending_noise<2>(s, r.x, r.id);
                xy[0] = r.x[0];
                xy[1] = r.x[1];
            }
            L.X[tid][0] = xy[0];
            L.X[tid][1] = xy[1];
        }
        __syncthreads();
#pragma unroll 1
        for (int mt = 0; mt < 4; ++mt) {
            const int m = 64 * w + 16 * mt;
            float out[2][4];
            fwd_tile(L.net, L.X[m + col][0], L.X[m + col][1], L.H2[w], out);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t r = base + m + 4 * g + i;
                if (r < s.n) {
                    const __bf16 c0 = (__bf16)out[0][i], c1 = (__bf16)out[1][i];
                    acc[0] += (double)(float)c0;
                    acc[1] += (double)(float)c1;
                    if (cout) {
                        cout[(size_t)r * CV_NO + col] = c0;
                        cout[(size_t)r * CV_NO + 16 + col] = c1;
                    }
                }
            }
        }
        __syncthreads();
    }
    L.red[w][g][col] = acc[0];
    L.red[w][g][16 + col] = acc[1];
    __syncthreads();
    if (tid < CV_NO) {
        double t = 0.0;
        for (int ww = 0; ww < 4; ++ww)
            for (int gg = 0; gg < 4; ++gg) t += L.red[ww][gg][tid];
        part[blockIdx.x * CV_NO + tid] = t;
    }
}

// Thread (f, c) of the 32 x 32 block sums workgroups c, c + 32, ... in
// order; thread f of the first 32 then sums the 32 chunk sums in order.
__global__ __launch_bounds__(1024) void k_csum_final(uint32_t nwg, const double *__restrict__ part,
                                                     double *__restrict__ S)
{
    __shared__ double chunk[32][CV_NO + 1];
    const uint32_t f = threadIdx.x % CV_NO, c = threadIdx.x / CV_NO;
    double acc = 0.0;
    for (uint32_t g = c; g < nwg; g += 32) acc += part[g * CV_NO + f];
    chunk[c][f] = acc;
    __syncthreads();
    if (threadIdx.x < CV_NO) {
        double t = 0.0;
        for (uint32_t k = 0; k < 32; ++k) t += chunk[k][threadIdx.x];
        S[threadIdx.x] = t;
    }
}

// ---------------------------------------------------------------------------
// control-variate batch force over sorted records
// ---------------------------------------------------------------------------
// Tile b < T-1 holds batches [b qb, min((b+1) qb, nbat-1)); tile T-1 holds
// the last batch (p plus the leftover ranks).  qb = 128 / p, so a tile has at
// most CV_MAXR = 128 records (p <= 64).  Persistent workgroups take tiles b,
// b + G, ... with net a staged in LDS once; c of every record comes from
// k_csum, which ran over the same key-ordered records.
struct BatchLds {
    NetLds net;  // a
    float X[CV_MAXR][2];
    uint32_t id[CV_MAXR];
    float A[CV_MAXR][CV_NO + 1];  // padded rows: one record per lane hits distinct banks
    uint32_t C[CV_MAXR][CV_NO / 2 + 1];  // BF16 pairs (element 2w in the low half of word w), padded
    __bf16 H2[4][16][WP];
    float sn[CV_NO];  // S / (N - 1)
};

// Element e of a BF16 row stored as pairs in 32-bit words.
__device__ __forceinline__ float bf16_at(const uint32_t *row, int e)
{
    const uint32_t w = row[e >> 1];
    return __uint_as_float((e & 1) ? (w & 0xffff0000u) : (w << 16));
}

template <int KERN>
__global__ __launch_bounds__(256, 3) void k_cv_batch(StepArgs s, uint32_t qb, uint32_t ntiles,
                                                  const Rec<2> *__restrict__ sorted,
                                                  const __bf16 *__restrict__ cin,
                                                  const float *__restrict__ master,
                                                  const __bf16 *__restrict__ wb,
                                                  const double *__restrict__ S,
                                                  Rec<2> *__restrict__ dst, float *__restrict__ fout)
{
    __shared__ BatchLds L;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, col = lane & 15;
    stage_net(L.net, master, wb, 0);
    if (tid < CV_NO) L.sn[tid] = (float)(S[tid] / (double)(s.n - 1));
    const float inv_n1 = 1.0f / (float)(s.n - 1);
    for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        uint32_t q0, q1;
        if (tile == ntiles - 1) {
            q0 = s.nbat - 1;
            q1 = s.nbat;
        } else {
            q0 = tile * qb;
            q1 = min(q0 + qb, s.nbat - 1);
        }
        const uint32_t r0 = q0 * s.p;
        const uint32_t r1 = (q1 == s.nbat) ? s.n : q1 * s.p;
        const uint32_t nr = r1 - r0;  // <= CV_MAXR by the tiling
        __syncthreads();              // the previous tile is done with the LDS
        // c of the tile's records (computed with S by k_csum): loaded now,
        // stored to LDS once a is computed, so the loads overlap that work
        // (16 B per load: elements 8 tid + 2048 k .. + 7, whole or absent
        // since a row holds 32)
        uint4 cr[CV_MAXR * CV_NO / 2048];
#pragma unroll
        for (int k = 0; k < CV_MAXR * CV_NO / 2048; ++k) {
            const uint32_t e = 8 * tid + 2048 * k;
            cr[k] = e < nr * CV_NO ? *reinterpret_cast<const uint4 *>(cin + (size_t)r0 * CV_NO + e)
                                   : make_uint4(0u, 0u, 0u, 0u);
        }
        if (tid < CV_MAXR) {
            float xy[2] = {0.0f, 0.0f};
            uint32_t id = 0;
            if ((uint32_t)tid < nr) {
                const Rec<2> r = sorted[r0 + tid];
                xy[0] = r.x[0];
                xy[1] = r.x[1];
                id = r.id;
            }
            L.X[tid][0] = xy[0];
            L.X[tid][1] = xy[1];
            L.id[tid] = id;
        }
        __syncthreads();
        // a of the tile's records: wave w takes rows 32 w .. 32 w + 31
#pragma unroll 1
        for (int mt = 0; mt < 2; ++mt) {
            const int m = 32 * w + 16 * mt;
            float out[2][4];
            fwd_tile(L.net, L.X[m + col][0], L.X[m + col][1], L.H2[w], out);
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) L.A[m + 4 * g + i][16 * t + col] = out[t][i];
        }
#pragma unroll
        for (int k = 0; k < CV_MAXR * CV_NO / 2048; ++k) {
            const uint32_t e = 8 * tid + 2048 * k;
            uint32_t *w = &L.C[e / CV_NO][(e % CV_NO) / 2];
            w[0] = cr[k].x;
            w[1] = cr[k].y;
            w[2] = cr[k].z;
            w[3] = cr[k].w;
        }
        __syncthreads();
        // forces, one thread per record
        if ((uint32_t)tid < nr) {
            const uint32_t l = tid, r = r0 + l;
            uint32_t bs, be;
            batch_of(s, r, bs, be);
            const float *a = L.A[l];
            float f[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                float acc = 0.0f;
#pragma unroll
                for (int rr = 0; rr < 16; ++rr)
                    acc = fmaf(a[16 * k + rr], L.sn[16 * k + rr] - bf16_at(L.C[l], 16 * k + rr) * inv_n1, acc);
                f[k] = acc;
            }
            const float xi[2] = {L.X[l][0], L.X[l][1]};
            float res[2] = {0.0f, 0.0f};
            for (uint32_t j = bs; j < be; ++j) {
                if (j == r) continue;
                const uint32_t lj = j - r0;
                float kv[2] = {0.0f, 0.0f};
                add_pair<2, KERN>(xi, L.X[lj], s.a, kv);
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    float dot = 0.0f;
#pragma unroll
                    for (int rr = 0; rr < 16; ++rr) dot = fmaf(a[16 * k + rr], bf16_at(L.C[lj], 16 * k + rr), dot);
                    res[k] += kv[k] - dot;
                }
            }
            const float inv = (be - bs == s.p) ? s.inv_p1 : s.inv_last;
            float x[2] = {xi[0], xi[1]};
            f[0] = fmaf(res[0], inv, f[0]);
            f[1] = fmaf(res[1], inv, f[1]);
            const uint32_t id = L.id[l];
            if (fout) {
                if (id < s.n) {
                    fout[(size_t)id * 2] = f[0];
                    fout[(size_t)id * 2 + 1] = f[1];
                }
            } else {
                drift_update<2>(s, x, f);
                Rec<2> o;
                o.x[0] = x[0];
                o.x[1] = x[1];
                o.id = id;
                dst[r] = o;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// training: loss gradient on a minibatch of pairs
// ---------------------------------------------------------------------------
struct NetAct {
    float Z1[64][64];    // pre-activations, later delta1
    __bf16 H1[64][64];
    float Z2[64][64];    // pre-activations, later delta2
    __bf16 H2[64][64];   // activations, later delta2 in BF16
    float O[64][CV_NO];  // outputs, later dO
};

struct GradLds {
    float X[64][2];
    float Y[64][2];
    NetAct act[2];
    float vacc[2][CV_VACC];  // per-net VALU-accumulated gradients: dW1, db1, db2, db3
    float loss[128];         // per (sample, component)
};

// offsets inside vacc: dW1[64][2], db1[64], db2[64], db3[32]
constexpr int VA_W1 = 0, VA_B1 = 128, VA_B2 = 192, VA_B3 = 256;

// Backward of one net over the 64 samples of the tile.  act.O holds dO,
// act.Z1/Z2 the pre-activations, act.H1/H2 the BF16 activations, In the
// network input.  Accumulates dW3 (2 tiles per wave) and dW2 (4 tiles per
// wave) in MFMA accumulators, the rest in vacc.
__device__ void bwd64(const NetP &n, NetAct &A, const float (*In)[2], float *vacc, f32x4 (&dw3)[2],
                      f32x4 (&dw2)[4])
{
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, col = lane & 15;
    // dW3[o][i] += sum_s dO[s][o] H2[s][i]: tiles 2w, 2w+1 of the 2 x 4 grid
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int tile = 2 * w + u, to = tile >> 2, ti = tile & 3;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            bf16x8 a, b;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int sm = 32 * ks + 8 * g + j;
                a[j] = (__bf16)A.O[sm][16 * to + col];
                b[j] = A.H2[sm][16 * ti + col];
            }
            dw3[u] = mfma(a, b, dw3[u]);
        }
    }
    // db3
    if (tid < CV_NO) {
        float acc = 0.0f;
        for (int sm = 0; sm < 64; ++sm) acc += A.O[sm][tid];
        vacc[VA_B3 + tid] += acc;
    }
    __syncthreads();
    // dH2[s][i] = sum_o dO[s][o] W3[o][i]  (M = samples 16w.., N = 64, K = 32);
    // delta2 = dH2 gelu'(Z2) -> Z2 (FP32) and H2 (BF16)
    {
        bf16x8 a;
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = (__bf16)A.O[16 * w + col][8 * g + j];
        float d2[4][4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = mfma(a, ld8(n.W3T + (16 * t + col) * 32 + 8 * g), acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) d2[t][i] = acc[i] * gelu_grad(A.Z2[16 * w + 4 * g + i][16 * t + col]);
        }
        __syncthreads();  // all reads of H2 (as activations) are done
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int sm = 16 * w + 4 * g + i, nn = 16 * t + col;
                A.Z2[sm][nn] = d2[t][i];
                A.H2[sm][nn] = (__bf16)d2[t][i];
            }
    }
    __syncthreads();
    // dW2[o][i] += sum_s delta2[s][o] H1[s][i]: tiles (w, u) of the 4 x 4 grid
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            bf16x8 a, b;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int sm = 32 * ks + 8 * g + j;
                a[j] = A.H2[sm][16 * w + col];
                b[j] = A.H1[sm][16 * u + col];
            }
            dw2[u] = mfma(a, b, dw2[u]);
        }
    }
    if (tid < 64) {
        float acc = 0.0f;
        for (int sm = 0; sm < 64; ++sm) acc += A.Z2[sm][tid];
        vacc[VA_B2 + tid] += acc;
    }
    // dH1[s][i] = sum_o delta2[s][o] W2[o][i] (K = 64); delta1 = dH1 gelu'(Z1)
    {
        float d1[4][4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
                acc = mfma(ld8(&A.H2[16 * w + col][32 * ks + 8 * g]), ld8(n.W2T + (16 * t + col) * 64 + 32 * ks + 8 * g), acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) d1[t][i] = acc[i] * gelu_grad(A.Z1[16 * w + 4 * g + i][16 * t + col]);
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) A.Z1[16 * w + 4 * g + i][16 * t + col] = d1[t][i];
    }
    __syncthreads();
    // dW1[f][c] += sum_s delta1[s][f] In[s][c]; db1[f] += sum_s delta1[s][f]
    if (tid < 192) {
        const int f = tid % 64, which = tid / 64;  // 0: dW1[f][0], 1: dW1[f][1], 2: db1[f]
        float acc = 0.0f;
        for (int sm = 0; sm < 64; ++sm) acc += A.Z1[sm][f] * (which < 2 ? In[sm][which] : 1.0f);
        if (which < 2)
            vacc[VA_W1 + 2 * f + which] += acc;
        else
            vacc[VA_B1 + f] += acc;
    }
    __syncthreads();
}

// Workgroup g evaluates tiles of 64 pairs and writes its summed gradient
// (2 x 6432 values) and loss to gpart[g], lpart[g].  Pairs come from
// (xs, ys) if given, else are drawn from the snapshots (stream 3).
template <int KERN>
__global__ __launch_bounds__(256) void k_grad(uint32_t npairs, uint32_t tiles_per_wg, float ka,
                                              const float *__restrict__ xs,
                                              const float *__restrict__ ys,
                                              const float *__restrict__ snap, uint32_t nsnap,
                                              uint32_t n, uint32_t step, uint32_t k0, uint32_t k1,
                                              const float *__restrict__ master,
                                              const __bf16 *__restrict__ wb,
                                              float *__restrict__ gpart, float *__restrict__ lpart)
{
    __shared__ GradLds L;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, g = lane >> 4, col = lane & 15;
    for (int e = tid; e < 2 * CV_VACC; e += 256) (&L.vacc[0][0])[e] = 0.0f;
    if (tid < 128) L.loss[tid] = 0.0f;
    f32x4 dw3[2][2], dw2[2][4];
#pragma unroll
    for (int net = 0; net < 2; ++net) {
#pragma unroll
        for (int u = 0; u < 2; ++u) dw3[net][u] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int u = 0; u < 4; ++u) dw2[net][u] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    const float inv_b = 1.0f / (float)npairs;
    const NetP na = net_of(master, wb, 0), nc = net_of(master, wb, 1);
    for (uint32_t tt = 0; tt < tiles_per_wg; ++tt) {
        const uint32_t base = (blockIdx.x * tiles_per_wg + tt) * 64;
        __syncthreads();
        if (tid < 64) {
            const uint32_t q = base + tid;
            float x0 = 0.f, x1 = 0.f, y0 = 0.f, y1 = 0.f;
            if (q < npairs) {
                if (xs) {
                    x0 = xs[2 * q];
                    x1 = xs[2 * q + 1];
                    y0 = ys[2 * q];
                    y1 = ys[2 * q + 1];
                } else {
                    const uint4 wq = philox4x32_10(make_uint4(q, step, 3u, 0u), k0, k1);
                    const uint32_t t = __umulhi(wq.x, nsnap);
                    const uint32_t i = __umulhi(wq.y, n);
                    uint32_t j = __umulhi(wq.z, n - 1);
                    j += (j >= i) ? 1u : 0u;
                    const float *sp = snap + (size_t)t * n * 2;
                    x0 = sp[2 * i];
                    x1 = sp[2 * i + 1];
                    y0 = sp[2 * j];
                    y1 = sp[2 * j + 1];
                }
            }
            L.X[tid][0] = x0;
            L.X[tid][1] = x1;
            L.Y[tid][0] = y0;
            L.Y[tid][1] = y1;
        }
        __syncthreads();
        fwd16(na, &L.X[16 * w][0], &L.act[0].H1[16 * w][0], &L.act[0].H2[16 * w][0],
              &L.act[0].Z1[16 * w][0], &L.act[0].Z2[16 * w][0], &L.act[0].O[16 * w][0], CV_NO);
        fwd16(nc, &L.Y[16 * w][0], &L.act[1].H1[16 * w][0], &L.act[1].H2[16 * w][0],
              &L.act[1].Z1[16 * w][0], &L.act[1].Z2[16 * w][0], &L.act[1].O[16 * w][0], CV_NO);
        // residuals res_k = K_k(x - y) - a_k . c_k; dO_a = -res c / B, dO_c = -res a / B
        float ga[16], gc[16];
        const int sm = tid >> 1, k = tid & 1;  // 128 threads: (sample, component)
        if (tid < 128) {
            const bool valid = base + sm < npairs;
            float dx[2] = {L.X[sm][0] - L.Y[sm][0], L.X[sm][1] - L.Y[sm][1]};
            const float r2 = dx[0] * dx[0] + dx[1] * dx[1];
            const float kv = pair_scale<KERN>(r2, ka) * dx[k];
            float dot = 0.0f;
#pragma unroll
            for (int r = 0; r < 16; ++r) dot = fmaf(L.act[0].O[sm][16 * k + r], L.act[1].O[sm][16 * k + r], dot);
            const float res = valid ? kv - dot : 0.0f;
            const float d = -res * inv_b;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                ga[r] = d * L.act[1].O[sm][16 * k + r];
                gc[r] = d * L.act[0].O[sm][16 * k + r];
            }
            L.loss[tid] += 0.5f * res * res;
        }
        __syncthreads();
        if (tid < 128) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                L.act[0].O[sm][16 * k + r] = ga[r];
                L.act[1].O[sm][16 * k + r] = gc[r];
            }
        }
        __syncthreads();
        bwd64(na, L.act[0], L.X, L.vacc[0], dw3[0], dw2[0]);
        bwd64(nc, L.act[1], L.Y, L.vacc[1], dw3[1], dw2[1]);
    }
    __syncthreads();
    // write the workgroup's gradient
    float *gp = gpart + (size_t)blockIdx.x * 2 * CV_NP;
#pragma unroll
    for (int net = 0; net < 2; ++net) {
        float *o = gp + net * CV_NP;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int tile = 2 * w + u, to = tile >> 2, ti = tile & 3;
#pragma unroll
            for (int i = 0; i < 4; ++i) o[CV_OW3 + (16 * to + 4 * g + i) * 64 + 16 * ti + col] = dw3[net][u][i];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int i = 0; i < 4; ++i) o[CV_OW2 + (16 * w + 4 * g + i) * 64 + 16 * u + col] = dw2[net][u][i];
        for (int e = tid; e < 128; e += 256) o[CV_OW1 + e] = L.vacc[net][VA_W1 + e];
        if (tid < 64) {
            o[CV_OB1 + tid] = L.vacc[net][VA_B1 + tid];
            o[CV_OB2 + tid] = L.vacc[net][VA_B2 + tid];
        }
        if (tid < 32) o[CV_OB3 + tid] = L.vacc[net][VA_B3 + tid];
    }
    if (tid == 0) {
        float acc = 0.0f;
        for (int i = 0; i < 128; ++i) acc += L.loss[i];
        lpart[blockIdx.x] = acc * inv_b;
    }
}

// g[q] = sum over workgroups of gpart[wg][q] (workgroup order); loss likewise.
// adam != 0: one Adam step on the master weights (t = step count from 1).
__global__ __launch_bounds__(256) void k_reduce_adam(uint32_t nwg, const float *__restrict__ gpart,
                                                     const float *__restrict__ lpart,
                                                     float *__restrict__ grad_out,
                                                     float *__restrict__ loss_out, int adam,
                                                     float lr, float bc1, float bc2,
                                                     float *__restrict__ master,
                                                     float *__restrict__ am, float *__restrict__ av)
{
    const uint32_t q = blockIdx.x * 256 + threadIdx.x;
    if (q == 0 && loss_out) {
        float l = 0.0f;
        for (uint32_t g = 0; g < nwg; ++g) l += lpart[g];
        *loss_out = l;
    }
    if (q >= 2 * CV_NP) return;
    // in workgroup order, 16 loads in flight at a time
    float gs = 0.0f;
    uint32_t g = 0;
    for (; g + 16 <= nwg; g += 16) {
        float v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = gpart[(size_t)(g + k) * 2 * CV_NP + q];
#pragma unroll
        for (int k = 0; k < 16; ++k) gs += v[k];
    }
    for (; g < nwg; ++g) gs += gpart[(size_t)g * 2 * CV_NP + q];
    if (grad_out) grad_out[q] = gs;
    if (adam) {
        const float m = 0.9f * am[q] + 0.1f * gs;
        const float v = 0.999f * av[q] + 0.001f * gs * gs;
        am[q] = m;
        av[q] = v;
        master[q] -= lr * (m / bc1) / (sqrtf(v / bc2) + 1e-8f);
    }
}

}  // namespace cvk

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
hipError_t cv_launch_glorot(float *master, uint64_t seed, hipStream_t st)
{
    hipLaunchKernelGGL(cvk::k_glorot, dim3((2 * CV_NP + 255) / 256), dim3(256), 0, st, master,
                       (uint32_t)seed, (uint32_t)(seed >> 32));
    return hipGetLastError();
}

hipError_t cv_launch_prep(const float *master, __bf16 *wb, hipStream_t st)
{
    hipLaunchKernelGGL(cvk::k_prep, dim3((2 * 6144 + 255) / 256), dim3(256), 0, st, master, wb);
    return hipGetLastError();
}

hipError_t cv_launch_features(const float *master, const __bf16 *wb, const float *x, uint32_t n,
                              float *a, float *c, hipStream_t st)
{
    const uint32_t g = min((n + 63) / 64, 2048u);
    hipLaunchKernelGGL(cvk::k_features, dim3(g), dim3(256), 0, st, master, wb, x, n, a, c);
    return hipGetLastError();
}

hipError_t cv_launch_csum(const StepArgs &s, const void *state, const float *master,
                          const __bf16 *wb, double *part, double *S, __bf16 *cout, hipStream_t st)
{
    const uint32_t g = min((s.n + 255) / 256, (uint32_t)CV_SUM_WG);
    hipLaunchKernelGGL(cvk::k_csum, dim3(g), dim3(256), 0, st, s, (const Rec<2> *)state, master, wb,
                       part, cout);
    hipLaunchKernelGGL(cvk::k_csum_final, dim3(1), dim3(1024), 0, st, g, part, S);
    return hipGetLastError();
}

hipError_t cv_launch_batch(const StepArgs &s, int kernel, const void *sorted, const __bf16 *c,
                           const float *master, const __bf16 *wb, const double *S, void *dst, float *fout,
                           hipStream_t st)
{
    const uint32_t qb = cv_batches_per_wg(s.p);
    const uint32_t ntiles = (s.nbat - 1 + qb - 1) / qb + 1;
    if (kernel != K_GAUSS) return hipErrorInvalidValue;
    static int resident = 0;  // workgroups that fit on the device at once
    if (resident == 0) {
        int dev = 0, cus = 0, per = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, cvk::k_cv_batch<K_GAUSS>, 256, 0);
        if (e != hipSuccess) return e;
        resident = cus * (per > 0 ? per : 1);
    }
    const uint32_t g = min(ntiles, (uint32_t)resident);
    hipLaunchKernelGGL(cvk::k_cv_batch<K_GAUSS>, dim3(g), dim3(256), 0, st, s, qb, ntiles,
                       (const Rec<2> *)sorted, c, master, wb, S, (Rec<2> *)dst, fout);
    return hipGetLastError();
}

hipError_t cv_launch_grad(uint32_t npairs, float ka, const float *xs, const float *ys,
                          const float *snap, uint32_t nsnap, uint32_t n, uint32_t step,
                          uint64_t seed, const float *master, const __bf16 *wb, float *gpart,
                          float *lpart, uint32_t *nwg_out, hipStream_t st)
{
    const uint32_t tiles = (npairs + 63) / 64;
    const uint32_t tpw = (tiles + CV_GRAD_WG - 1) / CV_GRAD_WG;
    const uint32_t nwg = (tiles + tpw - 1) / tpw;
    *nwg_out = nwg;
    hipLaunchKernelGGL(cvk::k_grad<K_GAUSS>, dim3(nwg), dim3(256), 0, st, npairs, tpw, ka, xs, ys,
                       snap, nsnap, n, step, (uint32_t)seed, (uint32_t)(seed >> 32), master, wb,
                       gpart, lpart);
    return hipGetLastError();
}

hipError_t cv_launch_reduce(uint32_t nwg, const float *gpart, const float *lpart, float *grad_out,
                            float *loss_out, int adam, float lr, int t, float *master, float *am,
                            float *av, hipStream_t st)
{
    const float bc1 = 1.0f - powf(0.9f, (float)t), bc2 = 1.0f - powf(0.999f, (float)t);
    hipLaunchKernelGGL(cvk::k_reduce_adam, dim3((2 * CV_NP + 255) / 256), dim3(256), 0, st, nwg,
                       gpart, lpart, grad_out, loss_out, adam, lr, bc1, bc2, master, am, av);
    return hipGetLastError();
}

}  // namespace rbm
