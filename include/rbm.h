/*
 * rbm.h -- C ABI of librbm.so: the Random Batch Method RBM-1 (Jin, Li & Liu,
 * arXiv:1812.10575, Sec. 2.1, Algorithm 1) for the binary interacting
 * particle system of eq. (1.2),
 *
 *     dX^i = -grad V(X^i) dt + 1/(N-1) sum_{j != i} K(X^i - X^j) dt + sigma dB^i,
 *
 * on one AMD Instinct MI355X (gfx950).
 *
 * Conventions for every entry point
 *   - Pointers named d_* are DEVICE pointers owned by the caller; the library
 *     never allocates, frees or retains device memory beyond the workspace
 *     the caller hands to rbm_init (which must outlive the context).
 *   - Positions at the boundary are FP32, row-major [N][d], indexed by
 *     particle id 0..N-1.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls only enqueue work on it; nothing is waited for unless stated.
 *   - Argument errors are detected before anything is enqueued and return
 *     RBM_ERR_INVALID / RBM_ERR_UNSUPPORTED / RBM_ERR_WORKSPACE.  HIP launch
 *     failures return RBM_ERR_HIP.  rbm_last_error() returns a thread-local
 *     description of the last failure.  No call aborts or throws.
 *
 * Random numbers (the paper leaves the source open; this library fixes it):
 *   Philox4x32-10 (Salmon et al., SC'11) with key (seed lo32, seed hi32).
 *   PERM word of slot k at step m : Philox(ctr = (k>>2, m, 0, sys))[k & 3]
 *   NOISE of particle i at step m : Philox(ctr = (i, m, 1, sys)), 4 words ->
 *       uniforms u = (2 (w >> 9) + 1) 2^-24 -> Box-Muller pairs (u0,u1), (u2,u3)
 *   Step m orders the particles by the 64-bit key (PERM word of its slot << 32
 *   | id); rank r in that order is the particle's slot at step m+1; the
 *   batches of step m are ranks [qp, qp+p), the last of the floor(N/p)
 *   batches also taking the N mod p leftover ranks.
 */
#ifndef RBM_H
#define RBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RBM_OK = 0,
    RBM_ERR_INVALID = 1,     /* bad argument (null pointer, out-of-range value) */
    RBM_ERR_WORKSPACE = 2,   /* workspace too small or misaligned */
    RBM_ERR_HIP = 3,         /* a HIP runtime call failed */
    RBM_ERR_UNSUPPORTED = 4, /* valid but outside what the kernels implement */
    RBM_ERR_DEVICE = 5       /* a device-side check failed (see rbm_check) */
} rbm_status;

/* Interaction kernels K of eq. (1.2); a = rbm_params.kparam.
 *   RBM_K_GAUSS       K(x) = -x exp(-|x|^2)
 *   RBM_K_SOFTCOULOMB K(x) = x / (|x|^2 + a)   (a = 1: the kernel of Sec. 4.1;
 *                                               small a: softened 1/x of Sec. 4.2)
 *   RBM_K_ATTREP      K(x) = x / (|x|^2 + a) - x
 *   RBM_K_COULOMB_SPLIT K(x) = x / |x|^2 (a must be 0), stepped by the
 *                     splitting of Sec. 2.3 with p = 2 (N even): each pair moves
 *                     by its exact flow over dt (centre fixed, direction kept,
 *                     |X^i - X^j|^2 grows by 4 dt: the scheme of Sec. 4.2 for the
 *                     Dyson Brownian motion), then X += -dt beta X + sigma sqrt(dt) z.
 *                     Forces (rbm_forces, direct_*) are those of x/|x|^2.
 *   RBM_K_WEALTH_SPLIT  K(x) = -a x (a = kappa > 0, the trading interaction
 *                     phi(y) = y^2/2 of the wealth model of Sec. 5), p = 2 (N
 *                     even): each pair moves by its exact flow (mean kept,
 *                     difference times e^{-2 a dt}), then X += -dt beta X and
 *                     the exact multiplicative noise of dX = sigma X dB,
 *                     X *= exp(sigma sqrt(dt) z - sigma^2 dt / 2) (sigma =
 *                     sqrt(2D)).  direct_step does not take this kernel.
 *   RBM_K_HAMILTON    the second-order (Hamiltonian) system of Sec. 4.1 and
 *                     Appendix A, x'' = -beta x + 1/(N-1) sum_j K(x_i - x_j)
 *                     with K(x) = x / (x^2 + a) in one dimension (a = 1: the
 *                     paper's example; a > 0), integrated by Verlet.  d must
 *                     be 2: a record is (x, u), u the Verlet velocity; at
 *                     step 0 u is the initial velocity v_0.  Each step
 *                     (rbm_step and direct_step alike, F the step's force):
 *                       u += h (F - beta x),  x += dt u,  h = dt/2 at step 0
 *                     (step0 = 0 in rbm_init), dt after it, which is
 *                     x_1 = x_0 + dt v_0 + dt^2 F_0 / 2 and x_{m+1} =
 *                     2 x_m - x_{m-1} + dt^2 F_m.  sigma must be 0; any p.
 *                     Forces (rbm_forces, direct_*) are (K(x_i - x_j), 0)
 *                     sums: the velocity component is 0.                  */
typedef enum {
    RBM_K_GAUSS = 0,
    RBM_K_SOFTCOULOMB = 1,
    RBM_K_ATTREP = 2,
    RBM_K_COULOMB_SPLIT = 3,
    RBM_K_WEALTH_SPLIT = 4,
    RBM_K_HAMILTON = 5
} rbm_kernel;

/* Model, method and stream parameters.  V(x) = beta |x|^2 / 2. */
typedef struct {
    int32_t d;        /* space dimension, 1..3 */
    int32_t kernel;   /* rbm_kernel */
    int64_t n;        /* particles N, 2 <= N <= RBM_MAX_N */
    int32_t p;        /* batch size, 2 <= p <= N (p <= RBM_MAX_P_MULTI when N > one bucket) */
    int32_t cv;       /* 0: plain RBM-1 force; 1: learned control variate (d = 2,
                         RBM_K_GAUSS, p <= RBM_MAX_P_CV; see cv_* below) */
    double kparam;    /* kernel softening a >= 0 */
    double beta;      /* external field coefficient: -grad V(x) = -beta x */
    double sigma;     /* noise amplitude sigma >= 0 */
    double dt;        /* time step tau > 0 */
    uint64_t seed;    /* Philox key */
    uint32_t sys;     /* Philox counter word 3 (system index in an ensemble) */
    uint32_t reserved; /* must be 0 */
} rbm_params;

#define RBM_MAX_N (1LL << 25)
#define RBM_MAX_P_MULTI 64
#define RBM_MAX_P_CV 64
#define RBM_CV_NPARAM 6432 /* parameters of one control-variate network */

typedef struct rbm_ctx rbm_ctx;

/* Bytes of device workspace rbm_init needs for these parameters (about
 * 120 B per particle at d = 3 for N above 217,600 with fused steps, of which
 * 32 B per particle are the coarse digits of two banks of 16 key sets; the
 * environment variable RBM_FUSE=0, read here and by rbm_init, plans the
 * unfused order without those buffers). */
rbm_status rbm_workspace_size(const rbm_params *prm, size_t *bytes);

/* Create a context.  d_x0: [N][d] FP32 positions by id.  d_slots: NULL for
 * the identity slot order, else N distinct ids (uint32) giving the id in
 * each slot (the value rbm_perm returns; used to resume a run).  step0: the
 * index m of the first step rbm_step will take (0 <= step0 < 2^32).
 * d_ws: workspace of ws_bytes >= rbm_workspace_size, 256-byte aligned.
 * Enqueues the layout set-up on stream; *out is a host object freed by
 * rbm_destroy. */
rbm_status rbm_init(const rbm_params *prm, const float *d_x0, const uint32_t *d_slots,
                    int64_t step0, void *d_ws, size_t ws_bytes, void *stream,
                    rbm_ctx **out);

/* One RBM-1 step m -> m+1 (Algorithm 1): a fresh random division, batch
 * forces 1/(s-1) sum_{j in batch} K(X_i - X_j) (eq. (2.3), s the batch size),
 * forward Euler-Maruyama update X += dt (-beta X + F) + sigma sqrt(dt) z. */
rbm_status rbm_step(rbm_ctx *ctx, void *stream);

/* nsteps consecutive rbm_step calls (bitwise identical to calling rbm_step
 * nsteps times).  The bucket counts and starts of a step depend only on the
 * step index and the slot indices, so they are computed for groups of up to
 * 16 consecutive steps with one launch of each key kernel.  For N above
 * 217,600 (more than 128 fine buckets), the sort kernel of each step but a
 * group's last writes its records straight into the next step's coarse
 * buckets (one pass over the records fewer); setting the environment
 * variable RBM_FUSE=0 before rbm_init selects the unfused order. */
rbm_status rbm_run(rbm_ctx *ctx, int64_t nsteps, void *stream);

/* Current positions, [N][d] FP32 by id. */
rbm_status rbm_positions(rbm_ctx *ctx, float *d_x, void *stream);

/* Current slot order: d_ids[k] = id of the particle in slot k (N uint32).
 * After a step this is that step's permutation (ids in key order). */
rbm_status rbm_perm(rbm_ctx *ctx, uint32_t *d_ids, void *stream);

/* Batch forces F_i (eq. (2.3)) of the division that step index `step` would
 * draw from the current slot order, at the current positions; [N][d] FP32 by
 * id.  The state is not changed. */
rbm_status rbm_forces(rbm_ctx *ctx, int64_t step, float *d_f, void *stream);

/* Index m of the next step. */
rbm_status rbm_step_index(const rbm_ctx *ctx, int64_t *m);

/* Wait for the stream and report device-side checks (a bucket larger than
 * the on-chip capacity, which by a Chernoff bound on the bucket counts has
 * probability below 1e-15 per step for every supported N; a slot id >= N
 * given to rbm_init): RBM_OK or RBM_ERR_DEVICE. */
rbm_status rbm_check(rbm_ctx *ctx, void *stream);

/* Kernels of one step, for rbm_phase_times (a kernel a step does not need
 * measures 0; the key phases of a group of steps are timed with its first
 * step, so their average over the recorded steps is the cost per step). */
enum {
    RBM_PHASE_KEYCOUNT = 0,  /* fine-bucket histogram of the PERM words per slot tile */
    RBM_PHASE_KEYSUM = 1,    /* fine-bucket totals */
    RBM_PHASE_KEYSTARTS = 2, /* bucket starts and run cursors */
    RBM_PHASE_SCATTER = 3,   /* records to their coarse buckets */
    RBM_PHASE_SPLIT = 4,     /* coarse buckets to fine buckets */
    RBM_PHASE_SORT = 5,      /* in-LDS sort + batch force + update */
    RBM_PHASE_FIXUP = 6,     /* batches cut by fine-bucket boundaries */
    RBM_NPHASES = 7
};

/* Measurement aid: with max_steps > 0, the next max_steps steps taken by
 * rbm_step / rbm_run record a HIP event between consecutive kernels on the
 * stream they run on (events are host-side objects; no device memory).
 * max_steps = 0 stops recording and releases the events. */
rbm_status rbm_timing(rbm_ctx *ctx, int32_t max_steps);

/* Wait for the recorded steps and return, per phase, the mean milliseconds
 * per step (ms[RBM_NPHASES]) over the *steps recorded steps; recording
 * restarts from zero afterwards. */
rbm_status rbm_phase_times(rbm_ctx *ctx, double *ms, int64_t *steps);

/* Free the host context (not the workspace). */
rbm_status rbm_destroy(rbm_ctx *ctx);

/* ---- learned control variate (contexts created with cv = 1) -------------
 * The batch force becomes (RBM-1 applied to the residual kernel, which Sec.
 * 2.3 allows for general kernels K(x, y); unbiased for any weights by
 * Lemma 3.1):
 *   F_i = a(X_i).(S - c(X_i))/(N-1)
 *         + 1/(s-1) sum_{j in batch, j != i} [K(X_i - X_j) - a(X_i).c(X_j)],
 *   S = sum_j c(X_j) (FP64),
 * with MLPs a, c: R^2 -> R^32 (2 -> 64 -> 64 -> 32, GELU in its tanh form,
 * z sigma(2 sqrt(2/pi) z (1 + 0.044715 z^2)), after the hidden layers;
 * outputs read as [component 2][rank 16]) evaluated with BF16 matrix
 * instructions (FP32 accumulation).  A step evaluates c once for every
 * particle and rounds it to BF16 (to nearest even): S sums those rounded
 * values and the batch term uses them, kept in the workspace; a is evaluated
 * once and stays FP32.  The workspace of a cv = 1 context adds 76 bytes per
 * particle.  Parameters of one net, FP32, in order:
 * W1[64][2], b1[64], W2[64][64], b2[64], W3[32][64], b3[32]; a then c.
 * rbm_init initialises them (cv_init with the context's seed). */

/* Glorot-uniform weights (weight q of net n: (2u-1) sqrt(6/(fan_in+fan_out)),
 * u from Philox(ctr = (q, n, 4, 0)), key = seed), zero biases, Adam state
 * reset. */
rbm_status cv_init(rbm_ctx *ctx, uint64_t seed, void *stream);

/* Copy 2 x RBM_CV_NPARAM FP32 parameters in (resets the Adam state) / out. */
rbm_status cv_set_weights(rbm_ctx *ctx, const float *d_w, void *stream);
rbm_status cv_get_weights(rbm_ctx *ctx, float *d_w, void *stream);

/* Network outputs of n points d_x [n][2]: d_a, d_c [n][32] (either may be
 * NULL). */
rbm_status cv_features(rbm_ctx *ctx, const float *d_x, int64_t n, float *d_a, float *d_c,
                       void *stream);

/* Loss L = 1/(2B) sum_pairs sum_k (K_k(x - y) - sum_r a_kr(x) c_kr(y))^2 over
 * the B = npairs pairs (d_x[q], d_y[q]), and its gradient d_g [2][6432]
 * (a then c).  d_loss: one float.  npairs <= 2^24. */
rbm_status cv_grads(rbm_ctx *ctx, const float *d_x, const float *d_y, int64_t npairs,
                    float *d_g, float *d_loss, void *stream);

/* nsteps Adam steps (beta = (0.9, 0.999), eps = 1e-8, learning rate lr) on
 * minibatches of `batch` pairs drawn from the nsnap snapshots d_snap
 * [nsnap][N][2] (positions by id, e.g. saved with rbm_positions during a
 * run): pair q of Adam step t (counted over the context's life) takes
 * Philox(ctr = (q, t, 3, 0)) -> snapshot floor(w0 nsnap / 2^32), particle
 * i = floor(w1 N / 2^32), j' = floor(w2 (N-1) / 2^32), j = j' + [j' >= i].
 * d_loss: NULL or nsteps floats (the minibatch loss before each step). */
rbm_status cv_train(rbm_ctx *ctx, const float *d_snap, int32_t nsnap, int64_t nsteps,
                    int32_t batch, float lr, float *d_loss, void *stream);

/* Measurement of the force error of Lemma 3.1 on a subset: d_out[0] =
 * sum over t < nids of |d_f[d_ids[t]] - d_fref[t]|^2 (d components each,
 * summed in FP64 in a fixed order, so the result does not depend on the
 * launch).  d_f: [n][d] forces by id (e.g. from rbm_forces), d_fref:
 * [nids][d] reference forces (e.g. direct_forces of the same ids), d_out: one
 * double.  An id >= n is not read: it makes d_out[0] NaN.  nids = 0 gives 0
 * (d_ids and d_fref may then be NULL).
 * Errors: RBM_ERR_INVALID for NULL pointers, d outside 1..3, n < 1 or
 * n > 2^31 - 1, nids < 0 or nids > 2^30. */
rbm_status rbm_force_sqerr(const float *d_f, int64_t n, const uint32_t *d_ids, int64_t nids,
                           const float *d_fref, int32_t d, double *d_out, void *stream);

/* ---- batched ensemble -----------------------------------------------------
 * nsys independent RBM-1 systems sharing the model parameters, system s with
 * N_s particles, Philox key seed_s and counter word 3 = s: each follows the
 * definitions of a standalone run with those values (its division is the
 * standalone one bit for bit, and with it every position).  All systems run
 * in one persistent launch: workgroups take work items from a queue ordered
 * by decreasing N_s; an item is one system, or a group of wg / team systems
 * of at most 4 team particles run side by side by teams of threads.  A
 * system run by a whole workgroup stays in LDS for all steps up to
 * tile.lds_max particles (<= RBM_ENS_LDS); larger ones (up to RBM_ENS_MAXN)
 * are streamed through the workspace. */
typedef struct {
    int32_t d;        /* space dimension: 2 */
    int32_t kernel;   /* rbm_kernel */
    int32_t p;        /* batch size, 2 <= p <= min N_s, p <= RBM_MAX_P_MULTI */
    int32_t reserved; /* must be 0 */
    double kparam, beta, sigma, dt;  /* as in rbm_params */
    int64_t nsys;     /* number of systems, >= 1 */
} rbm_ensemble;

/* Launch shape (the autotuner's search space); zeros select the defaults. */
typedef struct {
    int32_t lds_max;  /* a system run by a whole workgroup stays in LDS up to
                         this size (<= 4 wg; default 4 wg); larger ones are
                         streamed */
    int32_t grid;     /* persistent workgroups (default: as many as fit at once) */
    int32_t team;     /* threads per system for systems of at most 4 team
                         particles, run wg / team to a workgroup: a power of
                         two in 64..wg (default 256; wg: one system per
                         workgroup) */
    int32_t bucket;   /* mean bucket of a streamed system, 256..3 wg
                         (default wg); at most 256 buckets per system */
    int32_t wg;       /* threads per workgroup: 1024 (4096 records of LDS, one
                         workgroup per compute unit) or 512 (2048 records, two);
                         0: 1024 */
} rbm_ensemble_tile;

#define RBM_ENS_LDS 4096
#define RBM_ENS_MAXN (256 * 1024)

/* Workspace bytes for these systems (a 256-byte aligned device buffer of
 * about 32 bytes per particle plus the system table); h_n: host array of nsys
 * sizes.  Errors: RBM_ERR_INVALID for a size outside p..RBM_ENS_MAXN,
 * RBM_ERR_UNSUPPORTED for d != 2 or more than 2^31 - 1 particles in all. */
rbm_status ensemble_workspace_size(const rbm_ensemble *e, const int64_t *h_n, size_t *bytes);

/* Runs steps step0 .. step0 + nsteps - 1 of every system.  Each call starts
 * every system with slot k holding particle k (as rbm_init with no slots at
 * step step0), so one call of 2k steps and two calls of k steps differ in
 * their divisions.  h_n, h_seed: host arrays of nsys sizes and Philox keys.
 * d_x: packed FP32 positions [sum N_s][d], system by system, each by
 * particle id; read at the start and overwritten with the final positions.
 * tile: launch shape (NULL: defaults).  graph != 0: the launch is recorded
 * into a hipGraph on a private stream and replayed once (a graph of one
 * kernel node: the same work and time as the direct launch, graph = 0).  Waits for
 * completion and returns RBM_ERR_DEVICE if a device-side check failed. */
rbm_status ensemble_run(const rbm_ensemble *e, const int64_t *h_n, const uint64_t *h_seed,
                        float *d_x, int64_t step0, int64_t nsteps,
                        const rbm_ensemble_tile *tile, void *d_ws, size_t ws_bytes,
                        int32_t graph, void *stream);

/* Exact interaction force of eq. (1.2), F_i = 1/(N-1) sum_{j != i}
 * K(X_i - X_j), for the nids particles listed in d_ids (NULL: all N, in id
 * order).  d_x: [N][d] by id; d_f: [nids][d].  FP32 pair terms, FP64 sums. */
rbm_status direct_forces(const rbm_params *prm, const float *d_x, const uint32_t *d_ids,
                         int64_t nids, float *d_f, void *stream);

/* direct_forces plus d_m2[t] = 1/(N-1) sum_{j != i} |K(X_i - X_j)|^2 for the
 * same particles ([nids] FP32, FP64 sums).  With F_i the exact force, the
 * variance of Lemma 3.1 is Lambda_i = (N-1)/(N-2) (m2_i - |F_i|^2), and the
 * RBM-1 force error has E|F_i^RBM - F_i|^2 = (1/(p-1) - 1/(N-1)) Lambda_i
 * when p divides N.  An id >= N gives NaN outputs. */
rbm_status direct_moments(const rbm_params *prm, const float *d_x, const uint32_t *d_ids,
                          int64_t nids, float *d_f, float *d_m2, void *stream);

/* One step of the fully coupled system with the update and NOISE stream of
 * RBM-1 step `step`: d_x_out = d_x + dt (-beta d_x + F) + sigma sqrt(dt) z
 * (RBM_K_HAMILTON: the Verlet update of step `step`).
 * d_x_out must not alias d_x. */
rbm_status direct_step(const rbm_params *prm, const float *d_x, float *d_x_out,
                       int64_t step, void *stream);

/* Text of a status code, and the last error of this thread. */
const char *rbm_status_str(rbm_status st);
const char *rbm_last_error(void);

/* ------------------------------------------------------------------------
 * RBM-r: random batches with replacement (Sec. 2.2, Algorithms RBM-r' and
 * RBM-r).  Iteration k (0 <= k < 2^48) draws a batch C_k of p distinct
 * particles, uniformly at random and independently of the other iterations,
 * and moves only them by the batch SDE over dt, from the positions the
 * earlier iterations left:
 *   x_i += dt (-beta x_i + 1/(p-1) sum_{j in C_k, j != i} K(x_i - x_j))
 *          + sigma sqrt(dt) z
 * (RBM_K_COULOMB_SPLIT, p = 2: the pair's exact flow over dt, then the field
 * step and the noise, as in the splitting of Sec. 4.2).  N/p iterations
 * stand for one time step dt (RBM-r' reads them as the N/p batches of a
 * step).  Random numbers of iteration k, Philox4x32-10 with the key of
 * rbm_params.seed, counter (k mod 2^32, (k >> 32) | (s << 16), stream, sys):
 *   stream 2, s = b: words (w0..w3) -> U_{2b} = w1:w0, U_{2b+1} = w3:w2;
 *     member r: v = floor(U_r (N - r) / 2^64) and m_r = the v-th smallest
 *     particle not drawn yet (a uniformly random ordered p-subset)
 *   stream 3, s = r: the normals of member r (Box-Muller as for RBM-1)
 * The result is that of running the iterations one after another: the
 * library runs a window of iterations in rounds of disjoint batches, each
 * iteration in the first round in which it is the earliest pending one of
 * all its members, so window and rounds change the speed, never the result.
 *
 * rbm_params: d 1..3, kernel RBM_K_GAUSS .. RBM_K_COULOMB_SPLIT (the latter
 * with p = 2 and kparam = 0), 2 <= p <= min(N, RBM_RBMR_MAX_P), cv = 0.
 * window: iterations per round schedule, 0 for N/p (at most
 * RBM_RBMR_MAX_WINDOW).  rounds: rounds per window across the whole GPU;
 * one workgroup then continues the rounds for what is left (up to 64 more),
 * then runs any rest in order; 0 for (4 + 2p) ceil(window p / N), one more
 * above N = 2^22. */
#define RBM_RBMR_MAX_P 8
#define RBM_RBMR_MAX_WINDOW (1u << 22)
#define RBM_RBMR_MAX_ROUNDS 255

/* Bytes of device workspace rbmr_run needs: 16 N (particle records) +
 * 16 window p (the window's member entries, sorted by particle, and their
 * successors) + 2 x 1024 (ceil(window / 256) + 512) (two round queues of
 * 256 segments) + 4 B (G + 2) (the schedule sort's counts and starts: B <=
 * 8192 buckets of consecutive particles, G = ceil(window / max(4096,
 * ceil(window / 256))) <= 256 counting workgroups) + 1024 (rounds + 2)
 * (queue lengths), each part rounded up to 256. */
rbm_status rbmr_workspace_size(const rbm_params *prm, int64_t window, int32_t rounds, size_t *bytes);

/* Iterations k0 .. k0 + niter - 1 on d_x ([N][d] FP32 positions by particle
 * id, updated in place), enqueued on stream.  d_ws: caller-owned workspace of
 * ws_bytes >= rbmr_workspace_size, 256-byte aligned, no contents carried
 * between calls (so a run split over several calls, k0 continuing, equals
 * one call).  Errors: RBM_ERR_INVALID / RBM_ERR_UNSUPPORTED for parameters
 * outside the limits above, RBM_ERR_WORKSPACE, RBM_ERR_HIP for a failed
 * launch; nothing is enqueued on an argument error. */
rbm_status rbmr_run(const rbm_params *prm, float *d_x, int64_t k0, int64_t niter, int64_t window,
                    int32_t rounds, void *d_ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): rbmr_run
 * with its workspace taken from a buffer inside the library instead of a
 * caller argument.  The buffer is a static device array of
 * RBM_NOALLOC_SCRATCH_BYTES per GPU (held from the first call on that GPU
 * until the process ends); its address is resolved once per device.  The
 * call allocates nothing (no hipMalloc, no allocating library routine).
 * Same arguments, limits, results (bit for bit) and errors as rbmr_run;
 * RBM_ERR_WORKSPACE when rbmr_workspace_size(prm, window, rounds) exceeds
 * RBM_NOALLOC_SCRATCH_BYTES (with the default window N/p, about 36 N bytes
 * for p = 2: N up to 2^20 fits, 2^21 does not).  Every call on one GPU shares that GPU's
 * buffer: calls that overlap on one GPU (on different streams, or from
 * different threads) race and give undefined results; calls in one stream
 * order are safe.  Nothing of a call's buffer contents is carried into the
 * next call. */
#define RBM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
rbm_status rbmr_run_noalloc(const rbm_params *prm, float *d_x, int64_t k0, int64_t niter, int64_t window,
                            int32_t rounds, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RBM_H */
