/*
 * rbm_oracle.c -- plain, slow FP64 reference of one RBM-1 time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product
 * path (the HIP library and its Python binding) never calls it, and the two
 * share no source, header, table or helper.
 *
 * What is computed, and where the paper defines it (Jin, Li & Liu, "Random
 * Batch Methods (RBM) for interacting particle systems", arXiv:1812.10575):
 *
 *   - the binary particle system, eq. (1.2):
 *       dX^i = -grad V(X^i) dt + 1/(N-1) sum_{j != i} K(X^i - X^j) dt + sigma dB^i
 *   - RBM-1, Sec. 2.1 / Algorithm 1: at every step divide the particles into
 *     batches of p at random, then evolve each batch with the interaction
 *     restricted to the batch and the prefactor 1/(p-1), eq. (2.3)
 *   - the random division is a uniformly random permutation whose first p
 *     entries form batch 1, the next p batch 2, and so on (Sec. 2.1, the
 *     remark on the cost of the division)
 *   - if p does not divide N the last batch is allowed to differ in size
 *     (Sec. 2.1, the parenthetical on p dividing N; Sec. 2.3, item on
 *     unequal batch sizes).  Reading used here: the N mod p leftover
 *     particles join the last batch, so every batch has at least p >= 2
 *     members and 1/(s-1) is defined for the batch size s.
 *   - forward Euler (Euler-Maruyama when sigma > 0) solves the batch SDE over
 *     one step (Sec. 4.1 uses forward Euler for every step).
 *
 * The paper leaves the random-number source open (it names MATLAB's randperm).
 * This oracle fixes it as follows; the GPU library implements the same
 * definitions independently.
 *
 *   Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 *   easy as 1, 2, 3", SC'11): a 4x32-bit counter c, a 2x32-bit key k; each of
 *   10 rounds multiplies c0 and c2 by two fixed odd constants, recombines the
 *   high and low halves with c1, c3 and the key by xor, and the key is bumped
 *   by two Weyl constants between rounds.
 *
 *   key = (seed mod 2^32, seed div 2^32)
 *   PERM word of slot k at step m : Philox(c = (k >> 2, m, 0, sys))[k & 3]
 *   NOISE of particle id i, step m: Philox(c = (i, m, 1, sys)) -> 4 words
 *   uniform(w)  = (2 * (w >> 9) + 1) * 2^-24   (24 significant bits: the same
 *                 number in FP32 and FP64)
 *   normals     : Box-Muller on (u0,u1) -> (z0,z1), on (u2,u3) -> (z2,z3)
 *
 *   The permutation of step m: the particles sit in "slots" 0..N-1 (the
 *   order left by the previous step; the identity before the first step).
 *   Slot k draws the PERM word w_k and gets the unique 64-bit key
 *   (w_k << 32) | id(k).  Sorting the keys ascending gives the permutation;
 *   it is uniform because the words are i.i.d. and independent of the slot
 *   order (ties on w, probability 2^-32 per pair, resolve by id).  The sorted
 *   order becomes the next step's slot order.
 *
 * Loops over particles (keys, batch forces, updates, direct sums) run in
 * parallel with OpenMP when the library is built with it; each particle's
 * arithmetic is the same written sequence of FP64 operations whatever the
 * thread count, and the keys are unique, so every result is independent of
 * the number of threads (ora_set_threads).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (SC'11)                                                     */
/* ------------------------------------------------------------------------ */

static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0];
    const uint32_t n1 = lo1;
    const uint32_t n2 = hi0 ^ c[3] ^ k[1];
    const uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

static void philox_seeded(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                          uint32_t c3, uint32_t out[4])
{
    const uint32_t ctr[4] = {c0, c1, c2, c3};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    ora_philox4x32_10(ctr, key, out);
}

/* 24-bit uniform in (0,1): exactly representable in FP32 and FP64. */
double ora_uniform(uint32_t w)
{
    return (double)(2u * (w >> 9) + 1u) * (1.0 / 16777216.0);
}

/* PERM word of slot k at step m. */
uint32_t ora_perm_word(uint64_t seed, uint32_t sys, uint32_t m, uint32_t slot)
{
    uint32_t o[4];
    philox_seeded(seed, slot >> 2, m, 0u, sys, o);
    return o[slot & 3u];
}

/* Four standard normals of particle id at step m (Box-Muller on the NOISE
 * block).  The Brownian increment of eq. (1.2) over one step is
 * sqrt(dt) * z. */
void ora_normals(uint64_t seed, uint32_t sys, uint32_t m, uint32_t id, double z[4])
{
    uint32_t o[4];
    philox_seeded(seed, id, m, 1u, sys, o);
    const double two_pi = 6.283185307179586476925286766559;
    for (int h = 0; h < 2; ++h) {
        const double u0 = ora_uniform(o[2 * h]);
        const double u1 = ora_uniform(o[2 * h + 1]);
        const double r = sqrt(-2.0 * log(u0));
        z[2 * h] = r * cos(two_pi * u1);
        z[2 * h + 1] = r * sin(two_pi * u1);
    }
}

/* ------------------------------------------------------------------------ */
/* Model: the pair kernel K and the external field -grad V of eq. (1.2)     */
/* ------------------------------------------------------------------------ */

enum { ORA_K_GAUSS = 0, ORA_K_SOFTCOULOMB = 1, ORA_K_ATTREP = 2, ORA_K_COULOMB_SPLIT = 3,
       ORA_K_WEALTH_SPLIT = 4, ORA_K_HAMILTON = 5 };

typedef struct {
    int32_t d;          /* space dimension, 1..3 */
    int32_t kernel;     /* ORA_K_* */
    double kparam;      /* softening a of the kernels below */
    double beta;        /* V(x) = beta |x|^2 / 2, so -grad V = -beta x */
    double sigma;       /* noise amplitude */
    double dt;          /* time step tau */
    uint64_t seed;
    uint32_t sys;
} ora_params;

/* The interaction kernels used by the workloads:
 *   GAUSS       K(x) = -x exp(-|x|^2)
 *   SOFTCOULOMB K(x) = x / (|x|^2 + a)         (a = eps^2; a = 1 gives the
 *                                               Sec. 4.1 kernel x/(1+x^2))
 *   ATTREP      K(x) = x / (|x|^2 + a) - x
 *   COULOMB_SPLIT K(x) = x / |x|^2, the singular kernel of Sec. 4.2, whose
 *               steps use the splitting with the exact pair flow (below)
 *   WEALTH_SPLIT  K(x) = -a x, the trading interaction phi(y) = y^2/2 of the
 *               wealth model of Sec. 5 (a = kappa), stepped by splitting:
 *               exact pair flow, then exact multiplicative noise (below)
 *   HAMILTON    the second-order system of Sec. 4.1 / Appendix A in one
 *               space dimension: a record is (x, u) (d = 2, u the Verlet
 *               velocity), the force x/(x^2 + a) acts between positions
 *               only (K of a record difference is (K1(x_i - x_j), 0))
 * All are odd: K(-x) = -K(x). */
void ora_pair_kernel(int32_t kernel, int32_t d, double a, const double *x, double *out)
{
    if (kernel == ORA_K_HAMILTON) {
        out[0] = x[0] / (x[0] * x[0] + a);
        for (int k = 1; k < d; ++k) out[k] = 0.0;
        return;
    }
    double r2 = 0.0;
    for (int k = 0; k < d; ++k) r2 += x[k] * x[k];
    double s;
    switch (kernel) {
    case ORA_K_GAUSS:       s = -exp(-r2); break;
    case ORA_K_SOFTCOULOMB: s = 1.0 / (r2 + a); break;
    case ORA_K_ATTREP:      s = 1.0 / (r2 + a) - 1.0; break;
    case ORA_K_COULOMB_SPLIT: s = 1.0 / r2; break;
    case ORA_K_WEALTH_SPLIT: s = -a; break;
    default:                s = 0.0; break;
    }
    for (int k = 0; k < d; ++k) out[k] = s * x[k];
}

/* ------------------------------------------------------------------------ */
/* Random division (Sec. 2.1)                                               */
/* ------------------------------------------------------------------------ */

static int cmp_u64(const void *a, const void *b)
{
    const uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/* Threads of the parallel loops (OpenMP; the arithmetic of every particle
 * is the same whatever the count, so results do not depend on it). */
void ora_set_threads(int32_t nt)
{
#ifdef _OPENMP
    if (nt > 0) omp_set_num_threads(nt);
#else
    (void)nt;
#endif
}

int32_t ora_get_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* Ascending sort of n distinct 64-bit keys: qsort of one run per thread,
 * then rounds of pairwise merges.  The keys are unique, so the order is the
 * one any correct sort gives. */
static void sort_keys(uint64_t *keys, int64_t n)
{
    int64_t runs = ora_get_threads();
    if (runs > n / 4096) runs = n / 4096;
    if (runs < 2) {
        qsort(keys, (size_t)n, sizeof(uint64_t), cmp_u64);
        return;
    }
    int64_t *bnd = (int64_t *)malloc((size_t)(runs + 1) * sizeof(int64_t));
    for (int64_t r = 0; r <= runs; ++r) bnd[r] = n * r / runs;
#pragma omp parallel for schedule(static, 1)
    for (int64_t r = 0; r < runs; ++r)
        qsort(keys + bnd[r], (size_t)(bnd[r + 1] - bnd[r]), sizeof(uint64_t), cmp_u64);
    uint64_t *tmp = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    uint64_t *src = keys, *dst = tmp;
    for (int64_t width = 1; width < runs; width *= 2) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t r = 0; r < runs; r += 2 * width) {
            const int64_t lo = bnd[r];
            const int64_t mid = bnd[r + width < runs ? r + width : runs];
            const int64_t hi = bnd[r + 2 * width < runs ? r + 2 * width : runs];
            int64_t a = lo, b = mid, o = lo;
            while (a < mid && b < hi) dst[o++] = src[a] < src[b] ? src[a++] : src[b++];
            while (a < mid) dst[o++] = src[a++];
            while (b < hi) dst[o++] = src[b++];
        }
        uint64_t *t = src;
        src = dst;
        dst = t;
    }
    if (src != keys) memcpy(keys, src, (size_t)n * sizeof(uint64_t));
    free(tmp);
    free(bnd);
}

/* slots[k] = id of the particle in slot k (input); perm[r] = id at sorted
 * rank r (output; may alias slots). */
void ora_permutation(const ora_params *prm, int64_t n, uint32_t m,
                     const uint32_t *slots, uint32_t *perm)
{
    uint64_t *keys = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        const uint64_t w = ora_perm_word(prm->seed, prm->sys, m, (uint32_t)k);
        keys[k] = (w << 32) | (uint64_t)slots[k];
    }
    sort_keys(keys, n);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) perm[r] = (uint32_t)(keys[r] & 0xffffffffu);
    free(keys);
}

/* Batch of sorted rank r: consecutive groups of p; the last of the
 * floor(N/p) groups also takes the N mod p leftover ranks. */
void ora_batch_of(int64_t n, int32_t p, int64_t r, int64_t *start, int64_t *end)
{
    const int64_t nb = n / p;
    int64_t q = r / p;
    if (q > nb - 1) q = nb - 1;
    *start = q * p;
    *end = (q == nb - 1) ? n : (q + 1) * p;
}

/* ------------------------------------------------------------------------ */
/* Forces                                                                   */
/* ------------------------------------------------------------------------ */

/* RBM-1 batch force of every particle for a given division perm (eq. (2.3)):
 *   F_i = 1/(s-1) sum_{j in C(i), j != i} K(X_i - X_j),  s = |C(i)|.
 * x and f are N x d, indexed by particle id. */
void ora_rbm_forces(const ora_params *prm, int64_t n, int32_t p,
                    const double *x, const uint32_t *perm, double *f)
{
    const int d = prm->d;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
        int64_t b0, b1;
        ora_batch_of(n, p, r, &b0, &b1);
        const uint32_t i = perm[r];
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t t = b0; t < b1; ++t) {
            const uint32_t j = perm[t];
            if (j == i) continue;
            double dx[3], kv[3];
            for (int k = 0; k < d; ++k) dx[k] = x[(int64_t)i * d + k] - x[(int64_t)j * d + k];
            ora_pair_kernel(prm->kernel, d, prm->kparam, dx, kv);
            for (int k = 0; k < d; ++k) acc[k] += kv[k];
        }
        const double inv = 1.0 / (double)(b1 - b0 - 1);
        for (int k = 0; k < d; ++k) f[(int64_t)i * d + k] = acc[k] * inv;
    }
}

/* Exact interaction force of eq. (1.2) for the particles listed in ids:
 *   F_i = 1/(N-1) sum_{j != i} K(X_i - X_j). */
void ora_direct_forces(const ora_params *prm, int64_t n, const double *x,
                       const uint32_t *ids, int64_t nids, double *f)
{
    const int d = prm->d;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nids; ++t) {
        const uint32_t i = ids[t];
        double acc[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == (int64_t)i) continue;
            double dx[3], kv[3];
            for (int k = 0; k < d; ++k) dx[k] = x[(int64_t)i * d + k] - x[j * d + k];
            ora_pair_kernel(prm->kernel, d, prm->kparam, dx, kv);
            for (int k = 0; k < d; ++k) acc[k] += kv[k];
        }
        for (int k = 0; k < d; ++k) f[t * d + k] = acc[k] / (double)(n - 1);
    }
}

/* The same sums plus the second moment m2_i = 1/(N-1) sum_{j != i}
 * |K(X_i - X_j)|^2, from which the variance of Lemma 3.1 follows:
 *   Lambda_i = 1/(N-2) sum_{j != i} |K(X_i - X_j) - F_i|^2
 *            = (N-1)/(N-2) (m2_i - |F_i|^2). */
void ora_direct_moments(const ora_params *prm, int64_t n, const double *x,
                        const uint32_t *ids, int64_t nids, double *f, double *m2)
{
    const int d = prm->d;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nids; ++t) {
        const uint32_t i = ids[t];
        double acc[3] = {0.0, 0.0, 0.0}, acc2 = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == (int64_t)i) continue;
            double dx[3], kv[3];
            for (int k = 0; k < d; ++k) dx[k] = x[(int64_t)i * d + k] - x[j * d + k];
            ora_pair_kernel(prm->kernel, d, prm->kparam, dx, kv);
            for (int k = 0; k < d; ++k) {
                acc[k] += kv[k];
                acc2 += kv[k] * kv[k];
            }
        }
        for (int k = 0; k < d; ++k) f[t * d + k] = acc[k] / (double)(n - 1);
        m2[t] = acc2 / (double)(n - 1);
    }
}

/* ------------------------------------------------------------------------ */
/* Time stepping                                                            */
/* ------------------------------------------------------------------------ */

/* One Euler-Maruyama step of  dX = (-beta X + F) dt + sigma dB  for every
 * particle, all forces taken at the old positions:
 *   X_i <- X_i + dt (-beta X_i + F_i) + sigma sqrt(dt) z_i. */
static void euler_update(const ora_params *prm, int64_t n, uint32_t m,
                         const double *f, double *x)
{
    const int d = prm->d;
    const double sq = sqrt(prm->dt);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double z[4] = {0.0, 0.0, 0.0, 0.0};
        if (prm->sigma != 0.0) ora_normals(prm->seed, prm->sys, m, (uint32_t)i, z);
        for (int k = 0; k < d; ++k) {
            const double xi = x[i * d + k];
            x[i * d + k] = xi + prm->dt * (-prm->beta * xi + f[i * d + k])
                         + prm->sigma * sq * z[k];
        }
    }
}

/* Exact flow over a time t of one batch of two particles under
 * K(x) = x/|x|^2 with prefactor 1/(p-1) = 1 (Sec. 2.3, the splitting for
 * singular K; the scheme of Sec. 4.2).  The centre c = (xi + xj)/2 does not
 * move and u = xi - xj obeys du/dt = 2 u/|u|^2: its direction is kept and
 * |u|^2 = |u0|^2 + 4t.  So yi = c + g u0/2, yj = c - g u0/2 with
 * g = sqrt(1 + 4t/|u0|^2).  (The separation is g |u0|, hence the factor 1/2
 * on the square root that the printed scheme of Sec. 4.2 leaves out.)  Two
 * coincident particles (u0 = 0) stay at c. */
void ora_pair_flow(int32_t d, double t, const double *xi, const double *xj, double *yi, double *yj)
{
    double c[3], u[3], r2 = 0.0;
    for (int k = 0; k < d; ++k) {
        c[k] = 0.5 * (xi[k] + xj[k]);
        u[k] = xi[k] - xj[k];
        r2 += u[k] * u[k];
    }
    const double g = r2 > 0.0 ? sqrt(1.0 + 4.0 * t / r2) : 0.0;
    for (int k = 0; k < d; ++k) {
        yi[k] = c[k] + 0.5 * g * u[k];
        yj[k] = c[k] - 0.5 * g * u[k];
    }
}

/* Exact flow over a time t of a batch of two particles under K(x) = -kappa x
 * (prefactor 1/(p-1) = 1): the pair's mean c stays and u = xi - xj obeys
 * du/dt = -2 kappa u, so yi = c + e^{-2 kappa t} u/2, yj = c - e^{-2 kappa t} u/2
 * (the interaction part of the mean-preserving splitting of Sec. 5). */
void ora_pair_flow_linear(int32_t d, double t, double kappa, const double *xi, const double *xj,
                          double *yi, double *yj)
{
    const double g = exp(-2.0 * kappa * t);
    for (int k = 0; k < d; ++k) {
        const double c = 0.5 * (xi[k] + xj[k]), u = xi[k] - xj[k];
        yi[k] = c + 0.5 * g * u;
        yj[k] = c - 0.5 * g * u;
    }
}

/* The noise part of the wealth model's splitting: dY = sigma Y dB (sigma =
 * sqrt(2D)) solved exactly over dt, Y <- Y exp(sigma sqrt(dt) z - sigma^2
 * dt / 2), after the field step Y <- Y - dt beta Y.  The factor has mean 1,
 * so the mean wealth is kept in expectation (the pair step keeps it
 * exactly). */
static void gbm_update(const ora_params *prm, int64_t n, uint32_t m, double *x)
{
    const int d = prm->d;
    const double sq = sqrt(prm->dt), s = prm->sigma;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double z[4] = {0.0, 0.0, 0.0, 0.0};
        if (s != 0.0) ora_normals(prm->seed, prm->sys, m, (uint32_t)i, z);
        for (int k = 0; k < d; ++k) {
            const double y = x[i * d + k] + prm->dt * (-prm->beta * x[i * d + k]);
            x[i * d + k] = y * exp(s * sq * z[k] - 0.5 * s * s * prm->dt);
        }
    }
}

/* The Verlet scheme of Sec. 4.1 for x'' = F (records (x, u)), in the form
 *   u_{m+1} = u_m + h (F_m - beta x_m),  x_{m+1} = x_m + dt u_{m+1},
 * h = dt for m >= 1 and h = dt/2 at m = 0, where u_0 is the initial
 * velocity: x_1 = x_0 + dt v_0 + dt^2 F_0 / 2 and, with u_m = (x_m -
 * x_{m-1}) / dt, x_{m+1} = 2 x_m - x_{m-1} + dt^2 F_m. */
static void verlet_update(const ora_params *prm, int64_t n, uint32_t m, const double *f, double *x)
{
    const double h = m == 0 ? 0.5 * prm->dt : prm->dt;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double xi = x[i * 2], ui = x[i * 2 + 1];
        const double u1 = ui + h * (f[i * 2] - prm->beta * xi);
        x[i * 2 + 1] = u1;
        x[i * 2] = xi + prm->dt * u1;
    }
}

/* One RBM-1 step m (Algorithm 1): draw the division from the slot order,
 * compute batch forces at the old positions, update.  slots is replaced by
 * the new order (the sorted permutation).  COULOMB_SPLIT (p = 2, N even):
 * each pair moves by its exact flow over dt, then the external field and
 * the noise act by one Euler-Maruyama step from the moved positions
 * (Sec. 2.3 splitting, Sec. 4.2).  WEALTH_SPLIT (p = 2, N even): the pair
 * flow of K = -kappa x, then the exact multiplicative noise (Sec. 5).
 * HAMILTON: the batch forces, then the Verlet update. */
void ora_rbm_step(const ora_params *prm, int64_t n, int32_t p, uint32_t m,
                  double *x, uint32_t *slots)
{
    const int d = prm->d;
    double *f = (double *)malloc((size_t)n * d * sizeof(double));
    ora_permutation(prm, n, m, slots, slots);
    if (prm->kernel == ORA_K_COULOMB_SPLIT) {
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < n - 1; q += 2) {
            const int64_t i = slots[q], j = slots[q + 1];
            double yi[3], yj[3];
            ora_pair_flow(d, prm->dt, x + i * d, x + j * d, yi, yj);
            for (int k = 0; k < d; ++k) {
                x[i * d + k] = yi[k];
                x[j * d + k] = yj[k];
            }
        }
        for (int64_t e = 0; e < n * d; ++e) f[e] = 0.0;
    } else if (prm->kernel == ORA_K_WEALTH_SPLIT) {
#pragma omp parallel for schedule(static)
        for (int64_t q = 0; q < n - 1; q += 2) {
            const int64_t i = slots[q], j = slots[q + 1];
            double yi[3], yj[3];
            ora_pair_flow_linear(d, prm->dt, prm->kparam, x + i * d, x + j * d, yi, yj);
            for (int k = 0; k < d; ++k) {
                x[i * d + k] = yi[k];
                x[j * d + k] = yj[k];
            }
        }
        gbm_update(prm, n, m, x);
        free(f);
        return;
    } else {
        ora_rbm_forces(prm, n, p, x, slots, f);
    }
    if (prm->kernel == ORA_K_HAMILTON)
        verlet_update(prm, n, m, f, x);
    else
        euler_update(prm, n, m, f, x);
    free(f);
}

/* nsteps consecutive RBM-1 steps m0, m0+1, ... */
void ora_rbm_run(const ora_params *prm, int64_t n, int32_t p, uint32_t m0,
                 int64_t nsteps, double *x, uint32_t *slots)
{
    for (int64_t s = 0; s < nsteps; ++s)
        ora_rbm_step(prm, n, p, (uint32_t)(m0 + s), x, slots);
}

/* One step of the fully coupled system with the same update and the same
 * noise as the RBM-1 step m. */
void ora_direct_step(const ora_params *prm, int64_t n, uint32_t m, double *x)
{
    const int d = prm->d;
    double *f = (double *)malloc((size_t)n * d * sizeof(double));
    uint32_t *ids = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    for (int64_t i = 0; i < n; ++i) ids[i] = (uint32_t)i;
    ora_direct_forces(prm, n, x, ids, n, f);
    if (prm->kernel == ORA_K_HAMILTON)
        verlet_update(prm, n, m, f, x);
    else
        euler_update(prm, n, m, f, x);
    free(ids);
    free(f);
}

/* ------------------------------------------------------------------------ */
/* RBM-r: random batches with replacement (Sec. 2.2, Algorithm RBM-r)        */
/* ------------------------------------------------------------------------ */
/*
 * Iteration k (k = 0, 1, ..., below 2^48) picks a set C_k of p distinct
 * particles at random and moves only them, by the batch SDE over a (pseudo-)
 * time dt; the next iteration starts from the positions this one left.
 * N/p iterations stand for one time step dt (RBM-r', the same sequence of
 * batches read as N/p batches per step).  Random numbers of iteration k:
 *
 *   DRAW block b : Philox(c = (k mod 2^32, (k >> 32) | (b << 16), 2, sys))
 *                  64-bit words U_{2b} = (w1 << 32) | w0, U_{2b+1} = (w3 << 32) | w2
 *   member r     : v_r = floor(U_r (N - r) / 2^64), and m_r is the v_r-th
 *                  smallest particle not among m_0 .. m_{r-1} (so C_k is a
 *                  uniformly random ordered p-subset)
 *   NOISE slot r : Philox(c = (k mod 2^32, (k >> 32) | (r << 16), 3, sys)),
 *                  Box-Muller as for RBM-1 -> z_r
 *
 * Update of member r (the batch SDE by one Euler-Maruyama step, forces at the
 * positions the iteration started from):
 *   x_{m_r} += dt (-beta x_{m_r} + 1/(p-1) sum_{q != r} K(x_{m_r} - x_{m_q}))
 *              + sigma sqrt(dt) z_r
 * COULOMB_SPLIT (p = 2): the pair moves by its exact flow over dt, then
 *   y += dt (-beta y) + sigma sqrt(dt) z_r (the splitting used in Sec. 4.2
 *   for RBM-r as for RBM-1).
 */
static void rbmr_counter(uint64_t k, uint32_t sub, uint32_t stream, uint32_t sys,
                         uint64_t seed, uint32_t out[4])
{
    philox_seeded(seed, (uint32_t)k, (uint32_t)(k >> 32) | (sub << 16), stream, sys, out);
}

/* Members m_0 .. m_{p-1} of iteration k. */
void ora_rbmr_members(const ora_params *prm, int64_t n, int32_t p, uint64_t k, uint32_t *mem)
{
    uint32_t sorted[64];
    for (int32_t r = 0; r < p; ++r) {
        uint32_t w[4];
        rbmr_counter(k, (uint32_t)(r / 2), 2u, prm->sys, prm->seed, w);
        const uint64_t u = r % 2 == 0 ? ((uint64_t)w[1] << 32) | w[0] : ((uint64_t)w[3] << 32) | w[2];
        uint64_t v = (uint64_t)(((unsigned __int128)u * (uint64_t)(n - r)) >> 64);
        /* the v-th smallest of the particles not drawn yet: step over every
           drawn particle at or below the running candidate, smallest first */
        for (int32_t q = 0; q < r; ++q)
            if (sorted[q] <= v) ++v;
        mem[r] = (uint32_t)v;
        int32_t q = r;
        while (q > 0 && sorted[q - 1] > mem[r]) {
            sorted[q] = sorted[q - 1];
            --q;
        }
        sorted[q] = mem[r];
    }
}

/* Normals of noise slot r of iteration k. */
static void rbmr_normals(const ora_params *prm, uint64_t k, uint32_t r, double z[4])
{
    uint32_t o[4];
    rbmr_counter(k, r, 3u, prm->sys, prm->seed, o);
    const double two_pi = 6.283185307179586476925286766559;
    for (int h = 0; h < 2; ++h) {
        const double u0 = ora_uniform(o[2 * h]);
        const double u1 = ora_uniform(o[2 * h + 1]);
        const double rr = sqrt(-2.0 * log(u0));
        z[2 * h] = rr * cos(two_pi * u1);
        z[2 * h + 1] = rr * sin(two_pi * u1);
    }
}

/* Iteration k on the given members (any p distinct particles). */
void ora_rbmr_apply(const ora_params *prm, int32_t p, uint64_t k, const uint32_t *mem, double *x)
{
    const int d = prm->d;
    double y[64][3];
    const double sq = sqrt(prm->dt);
    if (prm->kernel == ORA_K_COULOMB_SPLIT) {
        ora_pair_flow(d, prm->dt, x + (int64_t)mem[0] * d, x + (int64_t)mem[1] * d, y[0], y[1]);
    } else {
        for (int32_t r = 0; r < p; ++r) {
            const double *xr = x + (int64_t)mem[r] * d;
            double f[3] = {0.0, 0.0, 0.0};
            for (int32_t q = 0; q < p; ++q) {
                if (q == r) continue;
                double dx[3], kv[3];
                for (int c = 0; c < d; ++c) dx[c] = xr[c] - x[(int64_t)mem[q] * d + c];
                ora_pair_kernel(prm->kernel, d, prm->kparam, dx, kv);
                for (int c = 0; c < d; ++c) f[c] += kv[c];
            }
            for (int c = 0; c < d; ++c) y[r][c] = xr[c] + prm->dt * (-prm->beta * xr[c] + f[c] / (p - 1));
        }
    }
    for (int32_t r = 0; r < p; ++r) {
        double z[4] = {0.0, 0.0, 0.0, 0.0};
        if (prm->sigma != 0.0) rbmr_normals(prm, k, (uint32_t)r, z);
        for (int c = 0; c < d; ++c) {
            double v = y[r][c];
            if (prm->kernel == ORA_K_COULOMB_SPLIT) v += prm->dt * (-prm->beta * v);
            x[(int64_t)mem[r] * d + c] = v + prm->sigma * sq * z[c];
        }
    }
}

/* niter consecutive iterations k0, k0+1, ... */
void ora_rbmr_run(const ora_params *prm, int64_t n, int32_t p, uint64_t k0, int64_t niter, double *x)
{
    uint32_t mem[64];
    for (int64_t t = 0; t < niter; ++t) {
        ora_rbmr_members(prm, n, p, k0 + (uint64_t)t, mem);
        ora_rbmr_apply(prm, p, k0 + (uint64_t)t, mem, x);
    }
}
