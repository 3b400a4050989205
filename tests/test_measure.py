"""The product's measurement helpers (paper_1812_10575_amd/measure.py), pinned
on the CPU against scipy and closed forms.

The KS distance is checked against scipy.stats.kstest's statistic, the
semicircle CDF against its density (Sec. 4.2) by quadrature and at its ends,
the inverse Gamma CDF against scipy.stats.invgamma and the closed form of
shape 2, the Lemma 3.1 prediction against an exhaustive enumeration of all
divisions of a tiny system written out here, and the slope fit against exact
power laws.
"""
import itertools
import math

import numpy as np
import pytest

from paper_1812_10575_amd import measure

scipy_stats = pytest.importorskip("scipy.stats")
from scipy import integrate  # noqa: E402


def test_ks_matches_scipy_on_normal_samples():
    rng = np.random.default_rng(3)
    for n in (1, 2, 17, 1000, 65537):
        x = rng.standard_normal(n)
        ref = scipy_stats.kstest(x, scipy_stats.norm.cdf).statistic
        assert measure.ks_distance(x, scipy_stats.norm.cdf) == pytest.approx(ref, abs=1e-15)


def test_ks_of_a_shifted_law_and_of_exact_quantiles():
    # samples at the midpoints of N equal-probability cells: D = 1/(2N) exactly
    n = 1000
    u = (np.arange(n) + 0.5) / n
    x = scipy_stats.norm.ppf(u)
    assert measure.ks_distance(x, scipy_stats.norm.cdf) == pytest.approx(0.5 / n, abs=1e-12)
    # all samples far above the law: D -> 1
    assert measure.ks_distance(np.full(10, 50.0), scipy_stats.norm.cdf) == pytest.approx(1.0)
    with pytest.raises(ValueError):
        measure.ks_distance(np.zeros(0), scipy_stats.norm.cdf)


@pytest.mark.parametrize("radius", [math.sqrt(2.0), 2.0, 0.7])
def test_semicircle_cdf_against_its_density(radius):
    R = radius
    dens = lambda v: 2.0 * math.sqrt(max(R * R - v * v, 0.0)) / (math.pi * R * R)  # noqa: E731
    assert measure.semicircle_cdf(-R, R) == pytest.approx(0.0, abs=1e-15)
    assert measure.semicircle_cdf(R, R) == pytest.approx(1.0, abs=1e-15)
    assert measure.semicircle_cdf(0.0, R) == pytest.approx(0.5, abs=1e-15)
    assert measure.semicircle_cdf(-3 * R, R) == 0.0 and measure.semicircle_cdf(3 * R, R) == 1.0
    for v in np.linspace(-R, R, 13):
        ref = integrate.quad(dens, -R, v, epsabs=1e-13, epsrel=1e-13)[0]
        assert measure.semicircle_cdf(v, R) == pytest.approx(ref, abs=1e-10)
    # symmetric law: F(-x) = 1 - F(x)
    v = np.linspace(0, R, 7)
    np.testing.assert_allclose(measure.semicircle_cdf(-v, R), 1.0 - measure.semicircle_cdf(v, R), atol=1e-15)


def test_semicircle_ks_of_exact_samples():
    # inverse-CDF samples of the semicircle (bisection on the closed form)
    R = math.sqrt(2.0)
    n = 4096
    u = (np.arange(n) + 0.5) / n
    lo, hi = np.full(n, -R), np.full(n, R)
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        below = measure.semicircle_cdf(mid, R) < u
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    assert measure.ks_distance(0.5 * (lo + hi), lambda v: measure.semicircle_cdf(v, R)) == pytest.approx(0.5 / n, abs=1e-9)


def test_dyson_radius():
    assert measure.dyson_radius(0.0) == pytest.approx(2.0)
    assert measure.dyson_radius(50.0) == pytest.approx(math.sqrt(2.0))
    t = 0.7
    assert measure.dyson_radius(t) ** 2 == pytest.approx(2.0 * (1.0 + math.exp(-2.0 * t)))


@pytest.mark.parametrize("shape,scale", [(2.0, 0.8), (3.5, 2.0), (1.2, 0.1)])
def test_inverse_gamma_cdf_against_scipy(shape, scale):
    y = np.concatenate([[-1.0, 0.0], np.geomspace(1e-3, 1e3, 41)])
    ref = scipy_stats.invgamma.cdf(y, shape, scale=scale)
    np.testing.assert_allclose(measure.inverse_gamma_cdf(y, shape, scale), ref, rtol=1e-12, atol=1e-15)


def test_inverse_gamma_cdf_shape_two_closed_form():
    # Q(2, z) = e^{-z} (1 + z)
    y = np.geomspace(1e-2, 1e2, 25)
    z = 0.9 / y
    np.testing.assert_allclose(measure.inverse_gamma_cdf(y, 2.0, 0.9), np.exp(-z) * (1 + z), rtol=1e-13)


def test_second_moment_and_rms():
    x = np.array([[3.0, 4.0], [0.0, 0.0], [1.0, 0.0], [0.0, -1.0]])
    assert measure.second_moment(x) == pytest.approx((25 + 0 + 1 + 1) / 4)
    assert measure.second_moment(np.array([1.0, -2.0])) == pytest.approx(2.5)
    y = x + np.array([[1.0, 0.0], [0.0, 2.0], [0.0, 0.0], [0.0, 0.0]])
    assert measure.rms_error(x, y) == pytest.approx(math.sqrt((1 + 4) / 4))
    assert measure.rms_error(np.arange(5.0), np.arange(5.0) + 3) == pytest.approx(3.0)
    with pytest.raises(ValueError):
        measure.rms_error(np.zeros((3, 2)), np.zeros((2, 2)))


def _divisions(ids, p):
    """Every division of ids into batches of p (the last takes the rest)."""
    ids = list(ids)
    if len(ids) < 2 * p:
        yield [ids]
        return
    first = ids[0]
    for mates in itertools.combinations(ids[1:], p - 1):
        rest = [i for i in ids[1:] if i not in mates]
        for tail in _divisions(rest, p):
            yield [[first, *mates]] + tail


@pytest.mark.parametrize("n,p", [(6, 2), (8, 4), (9, 3)])
def test_lemma_3_1_prediction_by_enumeration(n, p):
    rng = np.random.default_rng(11)
    x = rng.standard_normal(n)
    K = lambda v: v / (v * v + 1.0)  # noqa: E731 (an odd kernel in 1-D)
    kij = K(x[:, None] - x[None, :])
    np.fill_diagonal(kij, 0.0)
    fdir = kij.sum(axis=1) / (n - 1)
    # Lambda_i: the variance of K(X_i - X_j) over the other particles j
    lam = np.array([np.sum((np.delete(kij[i], i) - fdir[i]) ** 2) / (n - 2) for i in range(n)])
    err2 = np.zeros(n)
    cnt = 0
    for div in _divisions(range(n), p):
        cnt += 1
        for b in div:
            for i in b:
                f = sum(kij[i, j] for j in b if j != i) / (len(b) - 1)
                err2[i] += (f - fdir[i]) ** 2
    assert all(len(b) == p for div in [next(_divisions(range(n), p))] for b in div)
    assert measure.lemma_3_1_mse(p, n, lam) == pytest.approx(err2.mean() / cnt, rel=1e-12)


def test_loglog_slope_of_power_laws():
    h = np.array([2.0 ** -k for k in range(4, 9)])
    assert measure.loglog_slope(h, 0.2 * h ** 0.5) == pytest.approx(0.5, abs=1e-12)
    assert measure.loglog_slope(h, 3.0 * h ** 2) == pytest.approx(2.0, abs=1e-12)
