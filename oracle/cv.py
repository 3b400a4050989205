"""FP64 oracle of the learned control variate for the RBM-1 batch force.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper remarks that the random-batch error C sqrt(tau/p) could be reduced
by variance-reduction techniques (Sec. 2.1, after the cost estimate; Sec. 4.1,
after the CPU-time comparison) and that RBM applies to general kernels
K(x, y) (Sec. 2.3, last item).  The control variate used here splits

    K(x - y) = a(x) . c(y) + [K(x - y) - a(x) . c(y)]

with two small MLPs a, c : R^2 -> R^32 read as [component k = 0, 1][rank r =
0..15].  The separable part is summed exactly (O(N) through S = sum_j c(X_j)),
the residual kernel K_res(x, y) = K(x - y) - a(x) . c(y) by the random batch:

    F_i = a(X_i) . (S - c(X_i)) / (N - 1)
          + 1/(s - 1) sum_{j in batch, j != i} [K(X_i - X_j) - a(X_i) . c(X_j)].

Given the division, the first term is exact; the second is RBM-1 applied to
K_res, so by Lemma 3.1 (valid for general K(x, y)) the force is unbiased for
any weights and its variance is (1/(p-1) - 1/(N-1)) Lambda_i[K_res].

Network: 2 -> 64 -> 64 -> 32, GELU (tanh form) after the two hidden layers,
linear output.  Parameter vector of one net, in this order:
W1[64][2], b1[64], W2[64][64], b2[64], W3[32][64], b3[32] (6432 values).

`use_bf16=True` rounds (to nearest even) exactly the operands the GPU feeds
to its BF16 matrix instructions: W2, W3 and the hidden activations h1, h2 in
the forward pass; dO, delta2, h1, h2 and the weights in every product of the
backward pass (the bias and first-layer gradients stay unrounded).  In the
force (cv_forces, cv_forces_ids, cv_step) it also rounds the output of c to
BF16, as the GPU stores it: S sums the rounded values and the batch term uses
them, so the force stays exactly unbiased; a stays unrounded.
"""
from __future__ import annotations

import math

import numpy as np

from . import philox4x32_10, uniform

NH, NO, RANK, DIM = 64, 32, 16, 2
SIZES = [("W1", (NH, DIM)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
         ("W3", (NO, NH)), ("b3", (NO,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)  # 6432

STREAM_PAIRS = 3
STREAM_INIT = 4


def unpack(theta):
    """Parameter vector -> dict of arrays (views)."""
    out, o = {}, 0
    for name, shp in SIZES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + n], np.float64).reshape(shp)
        o += n
    return out


def bf16(a):
    """Round FP64/FP32 values to the nearest BF16 (ties to even), as FP64."""
    f = np.asarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


GELU_K = 2.0 * math.sqrt(2.0 / math.pi)
GELU_C = 0.044715


def _sigma_v(z):
    z = np.asarray(z, np.float64)
    v = GELU_K * z * (1.0 + GELU_C * z * z)
    from scipy.special import expit  # the logistic function 1 / (1 + e^-v)
    return expit(v)


def gelu(z):
    """GELU in its tanh form, 0.5 z (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3))),
    evaluated as z sigma(v), v = 2 sqrt(2/pi) z (1 + 0.044715 z^2)."""
    return np.asarray(z, np.float64) * _sigma_v(z)


def gelu_grad(z):
    z = np.asarray(z, np.float64)
    s = _sigma_v(z)
    return s + z * s * (1.0 - s) * GELU_K * (1.0 + 3.0 * GELU_C * z * z)


def forward(theta, x, use_bf16=False):
    """One net on points x [n][2]: returns (z1, h1, z2, h2, o) with o [n][32]."""
    p = unpack(theta)
    q = bf16 if use_bf16 else (lambda a: np.asarray(a, np.float64))
    x = np.asarray(x, np.float64)
    z1 = x @ p["W1"].T + p["b1"]
    h1 = gelu(z1)
    z2 = q(h1) @ q(p["W2"]).T + p["b2"]
    h2 = gelu(z2)
    o = q(h2) @ q(p["W3"]).T + p["b3"]
    return z1, h1, z2, h2, o


def features(theta, x, use_bf16=False):
    """Network output [n][2][16]."""
    return forward(theta, x, use_bf16)[4].reshape(-1, DIM, RANK)


def c_features(theta_c, x, use_bf16=False):
    """Output of the c network as the force uses it: [n][2][16], rounded to
    BF16 with use_bf16."""
    c = features(theta_c, x, use_bf16)
    return bf16(c) if use_bf16 else c


def pair_kernel_gauss(dx):
    """K(x) = -x exp(-|x|^2), the Gaussian attraction kernel, rows of dx."""
    r2 = np.sum(dx * dx, axis=1, keepdims=True)
    return -dx * np.exp(-r2)


def loss_and_grads(theta_a, theta_c, x, y, kfun=pair_kernel_gauss, use_bf16=False):
    """L = 1/(2B) sum_pairs sum_k (K_k(x - y) - sum_r a_kr(x) c_kr(y))^2 and
    its gradient with respect to both parameter vectors (backpropagation)."""
    q = bf16 if use_bf16 else (lambda a: np.asarray(a, np.float64))
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    B = x.shape[0]
    fa = forward(theta_a, x, use_bf16)
    fc = forward(theta_c, y, use_bf16)
    a = fa[4].reshape(B, DIM, RANK)
    c = fc[4].reshape(B, DIM, RANK)
    res = kfun(x - y) - np.sum(a * c, axis=2)          # [B][2]
    loss = 0.5 * np.sum(res * res) / B
    dres = res / B
    d_oa = (-dres[:, :, None] * c).reshape(B, NO)
    d_oc = (-dres[:, :, None] * a).reshape(B, NO)
    ga = _backward(theta_a, x, fa, d_oa, q)
    gc = _backward(theta_c, y, fc, d_oc, q)
    return loss, ga, gc


def _backward(theta, x, fw, d_o, q):
    p = unpack(theta)
    z1, h1, z2, h2, _ = fw
    g = {}
    g["W3"] = q(d_o).T @ q(h2)
    g["b3"] = d_o.sum(axis=0)
    dh2 = q(d_o) @ q(p["W3"])
    d2 = dh2 * gelu_grad(z2)
    g["W2"] = q(d2).T @ q(h1)
    g["b2"] = d2.sum(axis=0)
    dh1 = q(d2) @ q(p["W2"])
    d1 = dh1 * gelu_grad(z1)
    g["W1"] = d1.T @ x
    g["b1"] = d1.sum(axis=0)
    return np.concatenate([g[name].ravel() for name, _ in SIZES])


def glorot_init(net: int, seed: int = 1):
    """Glorot-uniform weights, zero biases.  Weight q of net `net` (0: a,
    1: c) is (2u - 1) sqrt(6 / (fan_in + fan_out)) with u the first uniform of
    Philox(ctr = (q, net, 4, 0)), q counting the weights of W1, W2, W3 in
    storage order."""
    theta = np.zeros(NPARAM, np.float64)
    o, qw = 0, 0
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for name, shp in SIZES:
        n = int(np.prod(shp))
        if name.startswith("W"):
            lim = math.sqrt(6.0 / (shp[0] + shp[1]))
            for t in range(n):
                w = philox4x32_10([qw, net, STREAM_INIT, 0], key)[0]
                theta[o + t] = (2.0 * uniform(int(w)) - 1.0) * lim
                qw += 1
        o += n
    return theta


def sample_pairs(step: int, batch: int, nsnap: int, n: int, seed: int = 1):
    """Pair q of minibatch `step`: Philox(ctr = (q, step, 3, 0)) -> words
    (w0, w1, w2); snapshot t = floor(w0 nsnap / 2^32), i = floor(w1 n / 2^32),
    j' = floor(w2 (n - 1) / 2^32), j = j' + [j' >= i] (uniform over j != i)."""
    key = [seed & 0xFFFFFFFF, seed >> 32]
    out = np.zeros((batch, 3), np.int64)
    for qq in range(batch):
        w = philox4x32_10([qq, step, STREAM_PAIRS, 0], key)
        t = (int(w[0]) * nsnap) >> 32
        i = (int(w[1]) * n) >> 32
        jp = (int(w[2]) * (n - 1)) >> 32
        out[qq] = (t, i, jp + (jp >= i))
    return out


def adam(theta, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1).  Returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def cv_forces(theta_a, theta_c, x, perm, p, kfun=pair_kernel_gauss, use_bf16=False):
    """Control-variate batch forces for the division perm (ids in rank
    order, batches as in RBM-1), x [N][2] by id.  The batches of p (all but
    the last) are evaluated together, one batch per row."""
    x = np.asarray(x, np.float64)
    perm = np.asarray(perm, np.int64)
    n = x.shape[0]
    a = features(theta_a, x, use_bf16)     # [N][2][16]
    c = c_features(theta_c, x, use_bf16)
    S = c.sum(axis=0)                       # exact sum (FP64)
    f = np.einsum("ikr,ikr->ik", a, S[None] - c) / (n - 1)
    nb = n // p
    groups = [perm[(nb - 1) * p:][None]]
    if nb > 1:
        groups.append(perm[:(nb - 1) * p].reshape(nb - 1, p))
    for ids in groups:
        nbat, s = ids.shape
        xs = x[ids]                                           # [B][s][2]
        dx = (xs[:, :, None, :] - xs[:, None, :, :]).reshape(-1, 2)
        kv = kfun(dx).reshape(nbat, s, s, 2)                  # K(X_i - X_j)
        ac = np.einsum("bikr,bjkr->bijk", a[ids], c[ids])     # a(X_i) . c(X_j)
        res = kv - ac
        res[:, np.arange(s), np.arange(s), :] = 0.0           # j != i
        f[ids] += res.sum(axis=2) / (s - 1)
    return f


def cv_forces_ids(theta_a, theta_c, x, perm, p, ids, kfun=pair_kernel_gauss, use_bf16=False,
                  chunk=1 << 18):
    """cv_forces for the listed ids only, by the same definitions; the sum S
    of c over all particles is taken in chunks so that large N fit in
    memory."""
    x = np.asarray(x, np.float64)
    perm = np.asarray(perm, np.int64)
    n = x.shape[0]
    S = np.zeros((DIM, RANK))
    for s0 in range(0, n, chunk):
        S += c_features(theta_c, x[s0:s0 + chunk], use_bf16).sum(axis=0)
    rank = np.empty(n, np.int64)
    rank[perm] = np.arange(n)
    nb = n // p
    out = np.zeros((len(ids), DIM))
    for t, i in enumerate(np.asarray(ids, np.int64)):
        q = min(rank[i] // p, nb - 1)
        bs = q * p
        mates = perm[bs:(n if q == nb - 1 else bs + p)]
        a = features(theta_a, x[[i]], use_bf16)[0]
        c = c_features(theta_c, x[mates], use_bf16)
        ci = c_features(theta_c, x[[i]], use_bf16)[0]
        f = np.einsum("kr,kr->k", a, S - ci) / (n - 1)
        res = np.zeros(DIM)
        for jj, j in enumerate(mates):
            if j != i:
                res += kfun((x[i] - x[j])[None])[0] - np.einsum("kr,kr->k", a, c[jj])
        out[t] = f + res / (len(mates) - 1)
    return out


def cv_step(theta_a, theta_c, prm, p, m, x, slots, kfun=pair_kernel_gauss, use_bf16=False):
    """One RBM-1 step with the control-variate force (division and noise as
    in the plain step of rbm_oracle.c).  Returns (x_new, slots_new)."""
    from . import normals, permutation
    x = np.asarray(x, np.float64)
    perm = permutation(prm, m, slots)
    f = cv_forces(theta_a, theta_c, x, perm, p, kfun, use_bf16)
    n, d = x.shape
    z = np.zeros((n, d))
    if prm.sigma != 0.0:
        z = np.array([normals(prm.seed, prm.sys, m, i)[:d] for i in range(n)])
    x1 = x + prm.dt * (-prm.beta * x + f) + prm.sigma * math.sqrt(prm.dt) * z
    return x1, perm
