"""Pins of the FP64 oracle's RBM-r (Sec. 2.2, Algorithm RBM-r): one random
batch of p distinct particles per iteration, drawn with replacement across
iterations, moved by the batch SDE over dt; N/p iterations stand for one
time step.

Each test checks the oracle against something other than itself: the law of
the draw (chi-square over every ordered subset), the inclusion probability,
the exact mean move over all batches (the direct force, as for Lemma 3.1),
conservation of the mean, the law of the noise, and the Dyson Brownian
motion's analytic density of Sec. 4.2 (the RBM-r figure there).
"""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

import rbm_inputs


def _prm(ora, kernel, d=1, **kw):
    base = dict(d=d, kernel=kernel, kparam=1.0, beta=1.0, sigma=0.0, dt=1e-2, seed=1)
    base.update(kw)
    return ora.Params(**base)


@pytest.mark.parametrize("n,p,iters", [(6, 2, 60000), (7, 3, 84000), (5, 5, 24000)])
def test_draw_is_a_uniform_ordered_subset(ora, n, p, iters):
    """Every ordered p-subset of {0..N-1} equally likely (chi-square), members
    distinct and in range."""
    prm = _prm(ora, ora.K_SOFTCOULOMB)
    cells = {c: i for i, c in enumerate(itertools.permutations(range(n), p))}
    counts = np.zeros(len(cells))
    for k in range(iters):
        m = tuple(int(v) for v in ora.rbmr_members(prm, n, p, k))
        counts[cells[m]] += 1
    assert counts.sum() == iters
    assert stats.chisquare(counts).pvalue > 1e-3


def test_draw_at_scale_is_distinct_and_in_range(ora):
    prm = _prm(ora, ora.K_SOFTCOULOMB, seed=9, sys=4)
    n = (1 << 24) + 3
    for p in (2, 8):
        for k in list(range(200)) + [2 ** 32 + 7, 2 ** 47 + 11]:
            m = ora.rbmr_members(prm, n, p, k)
            assert len(set(m.tolist())) == p and int(m.max()) < n


def test_inclusion_probability_and_independence(ora):
    """Each particle is in a batch with probability p/N; the first members
    of consecutive iterations are independent (chi-square on the joint)."""
    n, p, iters = 40, 4, 30000
    prm = _prm(ora, ora.K_SOFTCOULOMB, seed=3)
    hits = np.zeros(n)
    joint = np.zeros((5, 5))
    prev = None
    for k in range(iters):
        m = ora.rbmr_members(prm, n, p, k)
        hits[m] += 1
        cur = int(m[0]) % 5
        if prev is not None:
            joint[prev, cur] += 1
        prev = cur
    assert stats.chisquare(hits).pvalue > 1e-3
    assert abs(hits.sum() / (n * iters) - p / n) < 1e-12
    assert stats.chi2_contingency(joint)[1] > 1e-3


@pytest.mark.parametrize("kernel,d,p", [(0, 2, 2), (2, 3, 3), (1, 1, 4)])
def test_mean_move_over_all_batches_is_the_full_step(ora, kernel, d, p):
    """sigma = 0: averaged over every ordered batch, a particle moves by
    (p/N) dt (-beta x + F) with F the full system's force (it is in the
    batch with probability p/N, and then its batch force is unbiased)."""
    n = 6
    prm = _prm(ora, kernel, d=d, kparam=0.5, beta=0.7, dt=0.05)
    x = rbm_inputs.normal(n, d, seed=11).astype(np.float64)
    acc = np.zeros_like(x)
    cnt = 0
    for m in itertools.permutations(range(n), p):
        acc += ora.rbmr_apply(prm, p, 0, m, x) - x
        cnt += 1
    f = ora.direct_forces(prm, x)
    np.testing.assert_allclose(acc / cnt, (p / n) * prm.dt * (-prm.beta * x + f), rtol=1e-12, atol=1e-15)


def test_full_batch_is_the_direct_step(ora):
    """p = N: the one batch is the whole system, so an iteration is the
    fully coupled Euler step."""
    n = 9
    prm = _prm(ora, ora.K_ATTREP, d=2, kparam=0.1, beta=0.5)
    x = rbm_inputs.normal(n, 2, seed=12).astype(np.float64)
    m = ora.rbmr_members(prm, n, n, 5)
    np.testing.assert_allclose(ora.rbmr_apply(prm, n, 5, m, x), ora.direct_step(prm, 0, x), rtol=1e-13, atol=1e-15)


def test_odd_kernel_keeps_the_mean(ora):
    n = 500
    x0 = rbm_inputs.normal(n, 3, seed=13).astype(np.float64) + 0.2
    for p in (2, 5):
        prm = _prm(ora, ora.K_ATTREP, d=3, kparam=0.01, beta=0.0)
        x = ora.rbmr_run(prm, p, 0, 5000, x0)
        np.testing.assert_allclose(x.mean(axis=0), x0.mean(axis=0), rtol=0, atol=1e-14)
        assert np.abs(x - x0).max() > 1e-3


def test_noise_is_sigma_sqrt_dt_standard_normal(ora):
    """Two particles far apart under the Gaussian kernel feel no force
    (e^{-r^2} underflows); with V = 0 each iteration moves both by
    sigma sqrt(dt) z, z ~ N(0, 1) (KS), independent between slots."""
    prm = _prm(ora, ora.K_GAUSS, d=2, beta=0.0, sigma=0.7, dt=0.04)
    x = np.array([[0.0, 0.0], [100.0, 0.0]])
    inc = []
    for k in range(20000):
        m = ora.rbmr_members(prm, 2, 2, k)
        inc.append((ora.rbmr_apply(prm, 2, k, m, x) - x) / (0.7 * 0.2))
    inc = np.array(inc)
    for r in range(2):
        for c in range(2):
            assert stats.kstest(inc[:, r, c], "norm").pvalue > 1e-3
    assert abs(np.corrcoef(inc[:, 0, 0], inc[:, 1, 0])[0, 1]) < 0.03


@pytest.mark.slow
def test_dyson_rbmr_follows_the_analytic_density(ora):
    """Sec. 4.2 (the RBM-r figure): K = 1/x by the exact pair flow, V = x^2/2,
    sigma = 1/sqrt(N), dt = 1e-3, N/2 iterations per unit dt, from the
    radius-2 semicircle: at t = 0.5 and t = 2 the empirical law is the
    analytic rho(x, t) = sqrt(2 s - x^2)/(s pi), s = 1 + e^{-2t} (KS <= 0.02)."""
    n = 10000
    prm = _prm(ora, ora.K_COULOMB_SPLIT, kparam=0.0, beta=1.0, sigma=1.0 / math.sqrt(n), dt=1e-3)
    x = rbm_inputs.semicircle(n, 2.0, seed=14).astype(np.float64)
    k = 0
    for t_end in (0.5, 2.0):
        iters = int(round(t_end / prm.dt)) * (n // 2) - k
        x = ora.rbmr_run(prm, 2, k, iters, x)
        k += iters
        s = 1 + math.exp(-2 * t_end)
        ks = ora.ks_distance(x[:, 0], lambda v: ora.semicircle_cdf_r(v, math.sqrt(2 * s)))
        assert ks <= 0.02, (t_end, ks)
        assert abs(np.mean(x ** 2) - s / 2) < 0.02, (t_end, np.mean(x ** 2))
