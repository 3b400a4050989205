"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: published
known-answer vectors, closed forms, exact combinatorial identities of
Lemma 3.1 (enumerated over every division), conservation laws of the
update, and the error rate of Sec. 4.1 / Theorem 3.1.
"""
import itertools
import math
import os

import numpy as np
import pytest
from scipy import stats

import rbm_inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# helpers: divisions enumerated independently of the oracle
# --------------------------------------------------------------------------

def _equal_partitions(items, p):
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for others in itertools.combinations(rest, p - 1):
        block = (first,) + others
        left = [i for i in rest if i not in others]
        for tail in _equal_partitions(left, p):
            yield [block] + tail


def divisions(n, p):
    """Every division of {0..n-1} into floor(n/p) batches; when p does not
    divide n the last batch has p + n mod p members."""
    if n % p == 0:
        yield from _equal_partitions(list(range(n)), p)
        return
    big = p + n % p
    for bigblock in itertools.combinations(range(n), big):
        rest = [i for i in range(n) if i not in bigblock]
        for part in _equal_partitions(rest, p):
            yield part + [bigblock]


def canon(perm, p):
    """Division of a permutation: consecutive groups of p, remainder merged."""
    n = len(perm)
    nb = n // p
    blocks = [tuple(sorted(perm[q * p:(q + 1) * p])) for q in range(nb - 1)]
    blocks.append(tuple(sorted(perm[(nb - 1) * p:])))
    return tuple(sorted(blocks))


def M(n, p):
    return math.factorial(n) // (math.factorial(p) ** (n // p) * math.factorial(n // p))


# --------------------------------------------------------------------------
# random streams
# --------------------------------------------------------------------------

def test_philox_known_answers(ora):
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        out = ora.philox4x32_10(v[0:4], v[4:6])
        assert [int(o) for o in out] == v[6:10]


def test_uniform_is_24bit_and_exact_in_fp32(ora):
    assert ora.uniform(0) == 2.0 ** -24
    assert ora.uniform(0xFFFFFFFF) == 1.0 - 2.0 ** -24
    assert ora.uniform(0x80000000) == 0.5 + 2.0 ** -24
    rng = np.random.default_rng(5)
    for w in rng.integers(0, 2 ** 32, 2000, dtype=np.uint64):
        u = ora.uniform(int(w))
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u


def test_stream_counter_layout(ora):
    seed, sys = 0x1234567890ABCDEF, 7
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for m in (0, 1, 99):
        for slot in (0, 1, 2, 3, 4, 1023, 12345):
            blk = ora.philox4x32_10([slot >> 2, m, 0, sys], key)
            assert ora.perm_word(seed, sys, m, slot) == int(blk[slot & 3])


def test_box_muller_inverts_to_the_noise_uniforms(ora):
    """z0^2 + z1^2 = -2 ln u0 and atan2(z1, z0) = 2 pi u1 (mod 2 pi) for the
    uniforms of the NOISE block (i, m, 1, sys); same for (z2, z3)."""
    seed, sys = 99, 3
    key = [seed, 0]
    for pid in (0, 5, 77):
        for m in (0, 3):
            blk = ora.philox4x32_10([pid, m, 1, sys], key)
            u = [ora.uniform(int(w)) for w in blk]
            z = ora.normals(seed, sys, m, pid)
            for h in range(2):
                a, b = z[2 * h], z[2 * h + 1]
                assert a * a + b * b == pytest.approx(-2.0 * math.log(u[2 * h]), rel=1e-13)
                ang = math.atan2(b, a) % (2.0 * math.pi)
                assert ang == pytest.approx(2.0 * math.pi * u[2 * h + 1], abs=1e-12)


def test_normals_are_standard_normal(ora):
    z = np.concatenate([ora.normals(1, 0, 0, i) for i in range(16384)])
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 0.02 and abs(z.var() - 1.0) < 0.03


# --------------------------------------------------------------------------
# the model: kernels at points where their values are known in closed form
# --------------------------------------------------------------------------

def test_kernel_closed_forms(ora):
    # Gaussian attraction: |K| peaks at |x| = 1/sqrt 2 with value e^{-1/2}/sqrt 2,
    # pointing to the origin.
    r = 1.0 / math.sqrt(2.0)
    kv = ora.pair_kernel(ora.K_GAUSS, 2, 0.0, [r, 0.0])
    assert kv[0] == pytest.approx(-math.exp(-0.5) / math.sqrt(2.0), rel=1e-15)
    assert kv[1] == 0.0
    # softened Coulomb in 1-D: K(eps) = 1/(2 eps)
    eps = 1e-3
    assert ora.pair_kernel(ora.K_SOFTCOULOMB, 1, eps * eps, [eps])[0] == pytest.approx(1.0 / (2 * eps), rel=1e-14)
    # a = 1 is the kernel of Sec. 4.1, x/(1+x^2): value 1/2 at x = 1
    assert ora.pair_kernel(ora.K_SOFTCOULOMB, 1, 1.0, [1.0])[0] == pytest.approx(0.5, rel=1e-15)
    # attraction-repulsion vanishes on |x|^2 = 1 - a, repels inside, attracts outside
    a = 0.01
    s = math.sqrt(1.0 - a) / math.sqrt(3.0)
    assert np.max(np.abs(ora.pair_kernel(ora.K_ATTREP, 3, a, [s, s, s]))) < 1e-15
    assert ora.pair_kernel(ora.K_ATTREP, 3, a, [0.5, 0, 0])[0] > 0
    assert ora.pair_kernel(ora.K_ATTREP, 3, a, [2.0, 0, 0])[0] < 0
    # every kernel is odd with K(0) = 0
    rng = np.random.default_rng(0)
    for kern, d, a in ((ora.K_GAUSS, 2, 0.0), (ora.K_SOFTCOULOMB, 1, 1e-6), (ora.K_ATTREP, 3, 0.01)):
        assert np.all(ora.pair_kernel(kern, d, a, np.zeros(d)) == 0.0)
        for _ in range(20):
            x = rng.standard_normal(d)
            np.testing.assert_array_equal(ora.pair_kernel(kern, d, a, -x), -ora.pair_kernel(kern, d, a, x))


# --------------------------------------------------------------------------
# the random division (Sec. 2.1) and Lemma 3.1
# --------------------------------------------------------------------------

def test_permutation_is_key_order(ora):
    prm = ora.Params(d=1, kernel=ora.K_GAUSS, kparam=0.0, beta=0.0, sigma=0.0, dt=1e-3, seed=3)
    n = 1000
    rng = np.random.default_rng(1)
    slots = rng.permutation(n).astype(np.uint32)
    perm = ora.permutation(prm, 17, slots)
    assert sorted(perm.tolist()) == list(range(n))
    pos = {int(pid): k for k, pid in enumerate(slots)}
    keys = [(ora.perm_word(3, 0, 17, pos[int(pid)]) << 32) | int(pid) for pid in perm]
    assert all(a < b for a, b in zip(keys, keys[1:]))


@pytest.mark.parametrize("n,p", [(6, 2), (8, 4), (7, 3), (5, 2)])
def test_division_law_is_uniform(ora, n, p):
    """Every division is equally likely (M(n) of them when p | N, Lemma 3.1's
    count), chaining the slot order from step to step as the method does."""
    prm = ora.Params(d=1, kernel=ora.K_GAUSS, kparam=0.0, beta=0.0, sigma=0.0, dt=1e-3, seed=11)
    allv = sorted({tuple(sorted(tuple(sorted(b)) for b in dv)) for dv in divisions(n, p)})
    if n % p == 0:
        assert len(allv) == M(n, p)
    index = {v: k for k, v in enumerate(allv)}
    steps = 2000 * len(allv)
    counts = np.zeros(len(allv))
    slots = np.arange(n, dtype=np.uint32)
    for m in range(steps):
        slots = ora.permutation(prm, m, slots)
        counts[index[canon(slots.tolist(), p)]] += 1
    assert stats.chisquare(counts).pvalue > 1e-4


def test_consecutive_divisions_are_independent(ora):
    prm = ora.Params(d=1, kernel=ora.K_GAUSS, kparam=0.0, beta=0.0, sigma=0.0, dt=1e-3, seed=5)
    n, p = 4, 2
    allv = sorted({canon(list(q), p) for q in itertools.permutations(range(n))})
    index = {v: k for k, v in enumerate(allv)}
    joint = np.zeros((3, 3))
    slots = np.arange(n, dtype=np.uint32)
    prev = None
    for m in range(30000):
        slots = ora.permutation(prm, m, slots)
        cur = index[canon(slots.tolist(), p)]
        if prev is not None:
            joint[prev, cur] += 1
        prev = cur
    assert stats.chisquare(joint.ravel()).pvalue > 1e-4


def test_pair_probability(ora):
    """P(i, j in one batch) = (p-1)/(N-1) (proof of Lemma 3.1)."""
    prm = ora.Params(d=1, kernel=ora.K_GAUSS, kparam=0.0, beta=0.0, sigma=0.0, dt=1e-3, seed=2)
    n, p, steps = 64, 4, 4000
    co = np.zeros((n, n))
    slots = np.arange(n, dtype=np.uint32)
    for m in range(steps):
        slots = ora.permutation(prm, m, slots)
        for q in range(n // p):
            b = slots[q * p:(q + 1) * p]
            co[np.ix_(b, b)] += 1
    e = steps * (p - 1) / (n - 1)
    sd = math.sqrt(steps * (p - 1) / (n - 1) * (1 - (p - 1) / (n - 1)))
    off = co[~np.eye(n, dtype=bool)]
    assert np.max(np.abs(off - e)) < 5.5 * sd
    chi = np.sum((off[: off.size // 2] - e) ** 2 / e)
    assert stats.chi2.sf(chi, off.size // 2) > 1e-4


CASES = [(6, 2, 0, 2), (6, 3, 2, 3), (8, 4, 1, 1), (8, 2, 0, 2), (7, 3, 2, 3), (7, 2, 1, 1)]


@pytest.mark.parametrize("n,p,kern,d", CASES)
def test_lemma_3_1_exactly(ora, n, p, kern, d):
    """Over all divisions: mean of the batch force = direct force, and when
    p | N the variance is (1/(p-1) - 1/(N-1)) Lambda_i (Lemma 3.1)."""
    a = {0: 0.0, 1: 0.5, 2: 0.01}[kern]
    prm = ora.Params(d=d, kernel=kern, kparam=a, beta=1.0, sigma=0.0, dt=1e-3)
    x = rbm_inputs.normal(n, d, seed=n * 10 + p).astype(np.float64)
    fd = ora.direct_forces(prm, x)
    fs = []
    for dv in divisions(n, p):
        perm = np.array([i for b in dv for i in b], np.uint32)
        fs.append(ora.rbm_forces(prm, p, x, perm))
    fs = np.array(fs)
    scale = np.max(np.abs(fd)) + 1.0
    np.testing.assert_allclose(fs.mean(axis=0), fd, rtol=0, atol=1e-13 * scale)
    if n % p == 0:
        var = np.mean(np.sum((fs - fd[None]) ** 2, axis=2), axis=0)
        lam = np.zeros(n)
        for i in range(n):
            kij = np.array([ora.pair_kernel(kern, d, a, x[i] - x[j]) for j in range(n) if j != i])
            lam[i] = np.sum(np.sum((kij - kij.mean(axis=0)) ** 2, axis=1)) / (n - 2)
        pred = (1.0 / (p - 1) - 1.0 / (n - 1)) * lam
        np.testing.assert_allclose(var, pred, rtol=1e-11, atol=1e-14)
        # the moment form of Lambda_i used at scale
        fm, m2 = ora.direct_moments(prm, x)
        np.testing.assert_allclose(fm, fd, rtol=1e-14, atol=1e-16)
        lam2 = (n - 1) / (n - 2) * (m2 - np.sum(fd * fd, axis=1))
        np.testing.assert_allclose((1.0 / (p - 1) - 1.0 / (n - 1)) * lam2, var, rtol=1e-10, atol=1e-14)


def test_single_batch_is_the_direct_sum(ora):
    """p = N: one batch, so the RBM force and step are the full system's."""
    n, d = 50, 2
    prm = ora.Params(d=d, kernel=ora.K_GAUSS, kparam=0.0, beta=1.0, sigma=0.5, dt=1e-3, seed=1)
    x = rbm_inputs.normal(n, d, seed=4)
    perm = ora.permutation(prm, 0, np.arange(n))
    np.testing.assert_allclose(ora.rbm_forces(prm, n, x, perm), ora.direct_forces(prm, x), rtol=1e-12, atol=1e-15)
    x1, _ = ora.rbm_step(prm, n, 0, x, np.arange(n))
    np.testing.assert_allclose(x1, ora.direct_step(prm, 0, x), rtol=1e-13, atol=1e-15)


# --------------------------------------------------------------------------
# the update: exact linear identities
# --------------------------------------------------------------------------

def test_odd_kernel_conserves_the_mean(ora):
    """Odd K: forces cancel inside each batch, so with V = 0 and sigma = 0
    the centre of mass never moves; with V = |x|^2/2 it contracts by
    (1 - dt); with noise it moves by sigma sqrt(dt) mean(z)."""
    n, d = 1000, 3
    x0 = rbm_inputs.normal(n, d, seed=8).astype(np.float64) + 0.3
    prm = ora.Params(d=d, kernel=ora.K_ATTREP, kparam=0.01, beta=0.0, sigma=0.0, dt=1e-3)
    x, _ = ora.rbm_run(prm, 7, 0, 50, x0)
    np.testing.assert_allclose(x.mean(axis=0), x0.mean(axis=0), rtol=0, atol=1e-13)
    prm.beta = 1.0
    x, _ = ora.rbm_run(prm, 7, 0, 50, x0)
    np.testing.assert_allclose(x.mean(axis=0), (1 - 1e-3) ** 50 * x0.mean(axis=0), rtol=1e-12)
    prm.sigma = 0.1
    x1, _ = ora.rbm_step(prm, 7, 3, x0, np.arange(n))
    z = np.array([ora.normals(prm.seed, 0, 3, i)[:d] for i in range(n)])
    want = (1 - 1e-3) * x0.mean(axis=0) + 0.1 * math.sqrt(1e-3) * z.mean(axis=0)
    np.testing.assert_allclose(x1.mean(axis=0), want, rtol=0, atol=1e-14)


def test_second_moment_step_identity(ora):
    """d = 1, V = x^2/2, sigma = 0: X' = (1-dt) X + dt F, hence
    m2' = (1-dt)^2 m2 + 2 dt (1-dt) mean(xF) + dt^2 mean(F^2).  For p = 2 and
    K = 1/x the pair identity x_i K(x_i-x_j) + x_j K(x_j-x_i) = 1 gives
    mean(xF) = 1/2 exactly."""
    n, dt = 4096, 1e-3
    x = rbm_inputs.uniform(n, 1, -3, 3, seed=2).astype(np.float64)
    prm = ora.Params(d=1, kernel=ora.K_SOFTCOULOMB, kparam=0.0, beta=1.0, sigma=0.0, dt=dt, seed=1)
    slots = np.arange(n)
    perm = ora.permutation(prm, 0, slots)
    f = ora.rbm_forces(prm, 2, x, perm)
    assert np.mean(x * f) == pytest.approx(0.5, rel=1e-12)
    x1, _ = ora.rbm_step(prm, 2, 0, x, slots)
    m2, c1, c2 = np.mean(x ** 2), np.mean(x * f), np.mean(f ** 2)
    assert np.mean(x1 ** 2) == pytest.approx((1 - dt) ** 2 * m2 + 2 * dt * (1 - dt) * c1 + dt * dt * c2, rel=1e-12)


def test_resume_from_saved_slots(ora):
    """A run continued from (x, slot order, step index) equals the
    uninterrupted run bit for bit: every random number is a function of
    (seed, step, slot/id)."""
    n, d = 300, 2
    prm = ora.Params(d=d, kernel=ora.K_GAUSS, kparam=0.0, beta=1.0, sigma=0.5, dt=1e-3, seed=1)
    x0 = rbm_inputs.normal(n, d)
    xa, sa = ora.rbm_run(prm, 3, 0, 20, x0)
    xh, sh = ora.rbm_run(prm, 3, 0, 10, x0)
    xb, sb = ora.rbm_run(prm, 3, 10, 10, xh, sh)
    np.testing.assert_array_equal(xa, xb)
    np.testing.assert_array_equal(sa, sb)


# --------------------------------------------------------------------------
# whole runs against the paper's rates and closed forms
# --------------------------------------------------------------------------

@pytest.mark.slow
def test_error_decays_like_sqrt_tau(ora):
    """Sec. 4.1 / Theorem 3.1: with K = x/(1+x^2), V = x^2/2, p = 2 and the
    semicircle initial law of radius 2, the error (the RMS over particles of
    Sec. 4.1) against the fully coupled system at T = 1 falls like tau^(1/2)."""
    n = 256
    x0 = rbm_inputs.semicircle(n, 2.0, seed=3).astype(np.float64)
    ref_prm = ora.Params(d=1, kernel=ora.K_SOFTCOULOMB, kparam=1.0, beta=1.0, sigma=0.0, dt=2.0 ** -12)
    xr = x0.copy()
    for m in range(2 ** 12):
        xr = ora.direct_step(ref_prm, m, xr)
    taus = [2.0 ** -k for k in (4, 5, 6, 7, 8)]
    errs = []
    for tau in taus:
        e2 = []
        for seed in range(1, 9):
            prm = ora.Params(d=1, kernel=ora.K_SOFTCOULOMB, kparam=1.0, beta=1.0, sigma=0.0, dt=tau, seed=seed)
            x, _ = ora.rbm_run(prm, 2, 0, int(round(1.0 / tau)), x0)
            e2.append(ora.rms_error(x, xr) ** 2)
        errs.append(math.sqrt(np.mean(e2)))
    slope = np.polyfit(np.log(taus), np.log(errs), 1)[0]
    assert 0.4 < slope < 0.62, (slope, errs)


@pytest.mark.slow
def test_softened_coulomb_relaxes_to_the_semicircle(ora):
    """Sec. 4.2: with V = x^2/2 and the Coulomb-like kernel, the empirical
    law relaxes to the semicircle rho = sqrt(2 - x^2)/pi; for p = 2 the pair
    identity makes m2(t) = 1/2 + (m2(0) - 1/2) e^{-2t} in the limit of no
    softening."""
    n, dt, a = 8192, 1e-3, 0.05 ** 2
    x0 = rbm_inputs.uniform(n, 1, -3, 3, seed=1).astype(np.float64)
    prm = ora.Params(d=1, kernel=ora.K_SOFTCOULOMB, kparam=a, beta=1.0, sigma=0.0, dt=dt, seed=1)
    m20 = float(np.mean(x0 ** 2))
    x, slots = ora.rbm_run(prm, 2, 0, 500, x0)
    want = 0.5 + (m20 - 0.5) * math.exp(-1.0)
    assert float(np.mean(x ** 2)) == pytest.approx(want, rel=0.03)
    x, slots = ora.rbm_run(prm, 2, 500, 3500, x, slots)
    assert ora.ks_distance(x, ora.semicircle_cdf) < 0.02
    # At equilibrium m2 sits at the fixed point of the exact step identity,
    # m2* = [2 (1-dt) c1 + dt c2] / (2 - dt), with c1 = mean(xF) and
    # c2 = mean(F^2) averaged over steps; softening makes c1 < 1/2.
    c1, c2 = [], []
    for m in range(4000, 4200):
        perm = ora.permutation(prm, m, slots)
        f = ora.rbm_forces(prm, 2, x, perm)
        c1.append(np.mean(x * f))
        c2.append(np.mean(f * f))
        x, slots = ora.rbm_step(prm, 2, m, x, slots)
    m2s = (2 * (1 - dt) * np.mean(c1) + dt * np.mean(c2)) / (2 - dt)
    assert float(np.mean(x ** 2)) == pytest.approx(m2s, abs=0.005)
    assert 0.45 < m2s < 0.5


def test_semicircle_cdf_closed_form(ora):
    """F(-sqrt2) = 0, F(0) = 1/2, F(sqrt2) = 1 and F' = sqrt(2 - x^2)/pi
    (Sec. 4.2), including points at and beyond the support edge."""
    r2 = math.sqrt(2.0)
    assert ora.semicircle_cdf(-r2) == pytest.approx(0.0, abs=1e-15)
    assert ora.semicircle_cdf(0.0) == pytest.approx(0.5, abs=1e-15)
    assert ora.semicircle_cdf(r2) == pytest.approx(1.0, abs=1e-15)
    assert np.all(np.isfinite(ora.semicircle_cdf(np.array([-5.0, -r2, r2, 5.0, np.nextafter(r2, 9)]))))
    xs = np.linspace(-1.3, 1.3, 27)
    h = 1e-6
    dens = (ora.semicircle_cdf(xs + h) - ora.semicircle_cdf(xs - h)) / (2 * h)
    np.testing.assert_allclose(dens, np.sqrt(2 - xs ** 2) / math.pi, rtol=1e-7)
    # total mass 1 and second moment 1/2
    x = np.linspace(-r2, r2, 200001)
    rho = np.sqrt(np.maximum(2 - x ** 2, 0)) / math.pi
    assert np.trapezoid(rho, x) == pytest.approx(1.0, abs=1e-6)
    assert np.trapezoid(x * x * rho, x) == pytest.approx(0.5, abs=1e-6)


def test_ks_distance_matches_the_library_statistic(ora):
    """The KS distance is scipy's two-sided one-sample statistic, on samples
    from the semicircle law and from a shifted law; and the semicircle of
    rbm_inputs lands within the 1% band for 2^20 samples."""
    from scipy import stats
    for shift in (0.0, 0.05):
        x = rbm_inputs.semicircle(20000, radius=math.sqrt(2.0), seed=11).astype(np.float64)[:, 0] + shift
        want = stats.kstest(x, lambda t: ora.semicircle_cdf(t)).statistic
        assert ora.ks_distance(x, ora.semicircle_cdf) == pytest.approx(want, abs=1e-12)
    big = rbm_inputs.semicircle(1 << 20, radius=math.sqrt(2.0), seed=12).astype(np.float64)
    assert ora.ks_distance(big, ora.semicircle_cdf) < 0.01


# --------------------------------------------------------------------------
# splitting with the exact pair flow (Sec. 2.3; the Dyson scheme of Sec. 4.2)
# --------------------------------------------------------------------------

def _rk4_pair(xi, xj, t, nsub=20000):
    """The pair ODE dxi/dt = (xi - xj)/|xi - xj|^2 = -dxj/dt by classical RK4."""
    y = np.concatenate([xi, xj]).astype(np.float64)
    d = len(xi)

    def rhs(v):
        u = v[:d] - v[d:]
        k = u / np.dot(u, u)
        return np.concatenate([k, -k])

    h = t / nsub
    for _ in range(nsub):
        k1 = rhs(y)
        k2 = rhs(y + 0.5 * h * k1)
        k3 = rhs(y + 0.5 * h * k2)
        k4 = rhs(y + h * k3)
        y = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return y[:d], y[d:]


@pytest.mark.parametrize("d", [1, 2, 3])
def test_pair_flow_solves_the_pair_ode(ora, d):
    """The flow is the exact solution of the pair ODE: it agrees with a fine
    RK4 integration, keeps the centre and the direction, and composes (flow
    over t1 then t2 = flow over t1 + t2)."""
    rng = np.random.default_rng(d)
    xi, xj = rng.standard_normal(d), rng.standard_normal(d)
    t = 0.3
    yi, yj = ora.pair_flow(d, t, xi, xj)
    ri, rj = _rk4_pair(xi, xj, t)
    np.testing.assert_allclose(yi, ri, rtol=0, atol=1e-10)
    np.testing.assert_allclose(yj, rj, rtol=0, atol=1e-10)
    np.testing.assert_allclose(yi + yj, xi + xj, rtol=0, atol=1e-15)
    u0, u = xi - xj, yi - yj
    assert np.dot(u, u) == pytest.approx(np.dot(u0, u0) + 4 * t, rel=1e-14)
    np.testing.assert_allclose(u / np.linalg.norm(u), u0 / np.linalg.norm(u0), atol=1e-15)
    ai, aj = ora.pair_flow(d, 0.1, xi, xj)
    bi, bj = ora.pair_flow(d, 0.2, ai, aj)
    np.testing.assert_allclose(bi, yi, rtol=0, atol=1e-14)
    np.testing.assert_allclose(bj, yj, rtol=0, atol=1e-14)
    # coincident particles stay at their centre
    assert np.array_equal(ora.pair_flow(d, 0.1, xi, xi)[0], xi)


def test_split_step_moves_pairs_then_applies_the_field(ora):
    """A split step with sigma = 0: the batches are the pairs of the division,
    each moved by its exact flow, then scaled by (1 - dt beta)."""
    n, dt, beta = 10, 0.01, 1.0
    prm = ora.Params(d=1, kernel=ora.K_COULOMB_SPLIT, kparam=0.0, beta=beta, sigma=0.0, dt=dt, seed=4)
    x = rbm_inputs.normal(n, 1, seed=8).astype(np.float64)
    x1, perm = ora.rbm_step(prm, 2, 0, x, np.arange(n))
    for q in range(0, n, 2):
        i, j = perm[q], perm[q + 1]
        u0, u1 = x[i, 0] - x[j, 0], (x1[i, 0] - x1[j, 0]) / (1 - dt * beta)
        assert u1 * u1 == pytest.approx(u0 * u0 + 4 * dt, rel=1e-13)
        assert (x1[i, 0] + x1[j, 0]) == pytest.approx((1 - dt * beta) * (x[i, 0] + x[j, 0]), abs=1e-14)


def test_semicircle_cdf_of_any_radius(ora):
    for R in (1.0, math.sqrt(2.0), 2.0):
        assert ora.semicircle_cdf_r(-R, R) == pytest.approx(0.0, abs=1e-15)
        assert ora.semicircle_cdf_r(0.0, R) == pytest.approx(0.5, abs=1e-15)
        assert ora.semicircle_cdf_r(R, R) == pytest.approx(1.0, abs=1e-15)
        xs = np.linspace(-0.9 * R, 0.9 * R, 19)
        h = 1e-6
        dens = (ora.semicircle_cdf_r(xs + h, R) - ora.semicircle_cdf_r(xs - h, R)) / (2 * h)
        np.testing.assert_allclose(dens, 2 * np.sqrt(R * R - xs ** 2) / (math.pi * R * R), rtol=1e-7)
    x = np.linspace(-1.4, 1.4, 57)
    np.testing.assert_allclose(ora.semicircle_cdf_r(x, math.sqrt(2.0)), ora.semicircle_cdf(x), atol=1e-15)


def test_dyson_split_follows_the_analytic_density(ora):
    """Sec. 4.2: from the radius-2 semicircle, RBM-1 with the exact pair flow
    (beta = 1, sigma = 1/sqrt(N), tau = 1e-3) follows rho(x, t) =
    sqrt(2 s(t) - x^2) / (s(t) pi), s(t) = 1 + e^{-2t}: KS distance and
    second moment s(t)/2 at t = 0.5 and t = 3."""
    n = 4096
    prm = ora.Params(d=1, kernel=ora.K_COULOMB_SPLIT, kparam=0.0, beta=1.0, sigma=1 / math.sqrt(n),
                     dt=1e-3, seed=3)
    x = rbm_inputs.semicircle(n, 2.0, seed=5).astype(np.float64)
    slots = None
    m = 0
    for t_end in (0.5, 3.0):
        steps = int(round(t_end / 1e-3)) - m
        x, slots = ora.rbm_run(prm, 2, m, steps, x, slots)
        m += steps
        sig = 1 + math.exp(-2 * t_end)
        ks = ora.ks_distance(x[:, 0], lambda v: ora.semicircle_cdf_r(v, math.sqrt(2 * sig)))
        assert ks < 0.02, (t_end, ks)
        assert np.mean(x ** 2) == pytest.approx(sig / 2, abs=0.01), t_end


# --------------------------------------------------------------------------
# the wealth model of Sec. 5: linear trading kernel, multiplicative noise
# --------------------------------------------------------------------------

def test_linear_pair_flow_is_exact(ora):
    """Pair flow of K = -kappa x: RK4 of the pair ODE, the pair's mean kept,
    composition of two flows."""
    rng = np.random.default_rng(7)
    for d in (1, 2):
        xi, xj = rng.standard_normal(d), rng.standard_normal(d)
        kappa, t = 1.3, 0.4
        yi, yj = ora.pair_flow_linear(d, t, kappa, xi, xj)
        y = np.concatenate([xi, xj])
        h = t / 4000
        rhs = lambda v: np.concatenate([-kappa * (v[:d] - v[d:]), -kappa * (v[d:] - v[:d])])
        for _ in range(4000):
            k1 = rhs(y); k2 = rhs(y + 0.5 * h * k1); k3 = rhs(y + 0.5 * h * k2); k4 = rhs(y + h * k3)
            y = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        np.testing.assert_allclose(np.concatenate([yi, yj]), y, rtol=0, atol=1e-12)
        np.testing.assert_allclose(yi + yj, xi + xj, atol=1e-15)
        ai, aj = ora.pair_flow_linear(d, 0.1, kappa, xi, xj)
        bi, bj = ora.pair_flow_linear(d, 0.3, kappa, ai, aj)
        np.testing.assert_allclose(bi, yi, atol=1e-15)


def test_wealth_noise_is_the_exact_geometric_brownian_factor(ora):
    """Equal wealths do not trade, so one step multiplies each by
    exp(sigma sqrt(dt) z - sigma^2 dt / 2): log-normal with the right
    parameters, mean 1."""
    n, sigma, dt = 1 << 16, math.sqrt(2.0), 0.01
    prm = ora.Params(d=1, kernel=ora.K_WEALTH_SPLIT, kparam=1.0, beta=0.0, sigma=sigma, dt=dt, seed=9)
    x1, _ = ora.rbm_step(prm, 2, 4, np.ones((n, 1)), np.arange(n))
    from scipy import stats
    lg = np.log(x1[:, 0])
    assert stats.kstest(lg, "norm", args=(-0.5 * sigma * sigma * dt, sigma * math.sqrt(dt))).pvalue > 1e-3
    assert np.mean(x1) == pytest.approx(1.0, abs=4 * sigma * math.sqrt(dt) / math.sqrt(n))


def test_inverse_gamma_cdf_closed_form(ora):
    """Shape 2: F(y) = (1 + s/y) e^(-s/y); density by differences."""
    y = np.linspace(0.05, 20, 400)
    s = 0.8
    np.testing.assert_allclose(ora.inverse_gamma_cdf(y, 2.0, s), (1 + s / y) * np.exp(-s / y), rtol=1e-13)
    h = 1e-6
    dens = (ora.inverse_gamma_cdf(y + h, 2.0, s) - ora.inverse_gamma_cdf(y - h, 2.0, s)) / (2 * h)
    np.testing.assert_allclose(dens, s * s * y ** -3 * np.exp(-s / y), rtol=1e-6)


def test_wealth_reaches_the_inverse_gamma_equilibrium(ora):
    """Sec. 5 with kappa = D = 1 (sigma = sqrt 2), tau = 1e-3, T = 3, wealth
    started at |N(0,1)|: the empirical law is the inverse Gamma law of shape
    kappa/D + 1 = 2 and scale kappa eta / D, eta the mean wealth."""
    n = 8192
    prm = ora.Params(d=1, kernel=ora.K_WEALTH_SPLIT, kparam=1.0, beta=0.0, sigma=math.sqrt(2.0), dt=1e-3, seed=3)
    x = np.abs(rbm_inputs.normal(n, 1, seed=5).astype(np.float64))
    x1, _ = ora.rbm_run(prm, 2, 0, 3000, x)
    eta = float(x1.mean())
    assert ora.ks_distance(x1[:, 0], lambda v: ora.inverse_gamma_cdf(v, 2.0, eta)) < 0.03
    assert np.all(x1 > 0)


# --------------------------------------------------------------------------
# the second-order (Hamiltonian) system with Verlet (Sec. 4.1, Appendix A)
# --------------------------------------------------------------------------

def _hamilton(ora, dt, seed=1, beta=0.0):
    return ora.Params(d=2, kernel=ora.K_HAMILTON, kparam=1.0, beta=beta, sigma=0.0, dt=dt, seed=seed)


def test_hamiltonian_kernel_acts_between_positions(ora):
    """Records are (x, u): the pair force is (x/(1 + x^2), 0), the Sec. 4.1
    kernel on the position difference, whatever the velocities."""
    for dx, du in [(0.5, 3.0), (-2.0, -1.0), (0.0, 7.0)]:
        k = ora.pair_kernel(ora.K_HAMILTON, 2, 1.0, [dx, du])
        np.testing.assert_array_equal(k, [dx / (1.0 + dx * dx), 0.0])


def test_hamiltonian_rejects_noise_and_other_d(ora):
    with pytest.raises(ValueError):
        ora.Params(d=2, kernel=ora.K_HAMILTON, kparam=1.0, beta=0.0, sigma=0.1, dt=0.1).c()
    with pytest.raises(ValueError):
        ora.Params(d=1, kernel=ora.K_HAMILTON, kparam=1.0, beta=0.0, sigma=0.0, dt=0.1).c()


@pytest.mark.parametrize("p", [2, 3, 0])
def test_verlet_velocity_form_is_the_two_step_recursion(ora, p):
    """The stored (x, u) update is the paper's position-only Verlet scheme,
    X_1 = X_0 + tau V_0 + tau^2 F_0 / 2 and X_{n+1} = 2 X_n - X_{n-1} +
    tau^2 F_n, with F the mean-field force of the step: the full system's
    (p = 0 here) or RBM-1's batch force of that step's division."""
    n, tau = 41, 2.0 ** -5
    s0 = rbm_inputs.hamilton(n, seed=2).astype(np.float64)
    prm = _hamilton(ora, tau, seed=3)
    xs = [s0[:, 0].copy()]
    s, slots = s0.copy(), np.arange(n)
    for m in range(6):
        if p == 0:
            f = ora.direct_forces(prm, s)
            s = ora.direct_step(prm, m, s)
        else:
            f = ora.rbm_forces(prm, p, s, ora.permutation(prm, m, slots))
            s, slots = ora.rbm_step(prm, p, m, s, slots)
        np.testing.assert_array_equal(f[:, 1], 0.0)
        if m == 0:
            want = xs[0] + tau * s0[:, 1] + 0.5 * tau * tau * f[:, 0]
        else:
            want = 2.0 * xs[-1] - xs[-2] + tau * tau * f[:, 0]
        np.testing.assert_allclose(s[:, 0], want, rtol=0, atol=1e-13)
        xs.append(s[:, 0].copy())


def test_direct_verlet_converges_to_the_ode_at_second_order(ora):
    """The full system x'' = (1/(N-1)) sum_j K(x_i - x_j), v(0) = V_0, is
    integrated by scipy's DOP853 to 1e-12; the Verlet positions at T = 1
    approach it like tau^2 (a dropped half kick would make it tau^1, a
    wrong force would not converge)."""
    from scipy.integrate import solve_ivp
    n = 6
    s0 = rbm_inputs.hamilton(n, seed=5).astype(np.float64)

    def rhs(_t, y):
        x = y[:n]
        dx = x[:, None] - x[None, :]
        return np.concatenate([y[n:], (dx / (1.0 + dx * dx)).sum(axis=1) / (n - 1)])

    sol = solve_ivp(rhs, (0.0, 1.0), np.concatenate([s0[:, 0], s0[:, 1]]), method="DOP853",
                    rtol=1e-12, atol=1e-13)
    xt = sol.y[:n, -1]
    errs = []
    for k in (4, 5, 6, 7):
        prm = _hamilton(ora, 2.0 ** -k)
        s = s0.copy()
        for m in range(2 ** k):
            s = ora.direct_step(prm, m, s)
        errs.append(np.abs(s[:, 0] - xt).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(1.9 < o < 2.1 for o in orders), (errs, orders)


def test_hamiltonian_rbm_conserves_momentum(ora):
    """Odd K: the batch forces cancel, so without a field the mean velocity
    stays at its initial value and the centre of mass moves with it:
    mean x_m = mean x_0 + m tau mean v_0.  p = N is the full system."""
    n, tau, steps = 300, 2.0 ** -5, 32
    s0 = rbm_inputs.hamilton(n, seed=6).astype(np.float64) + np.array([0.4, 0.25])
    for p in (2, 5):
        x, _ = ora.rbm_run(_hamilton(ora, tau, seed=p), p, 0, steps, s0)
        np.testing.assert_allclose(x[:, 1].mean(), s0[:, 1].mean(), rtol=0, atol=1e-14)
        np.testing.assert_allclose(x[:, 0].mean(), s0[:, 0].mean() + steps * tau * s0[:, 1].mean(),
                                   rtol=0, atol=1e-13)
    prm = _hamilton(ora, tau, beta=1.0)
    x1, _ = ora.rbm_step(prm, n, 0, s0, np.arange(n))
    np.testing.assert_allclose(x1, ora.direct_step(prm, 0, s0), rtol=1e-13, atol=1e-15)


def test_hamiltonian_centre_of_mass_in_a_harmonic_field(ora):
    """b(x) = -beta x (Appendix A): the batch forces cancel, so the centre of
    mass is a harmonic oscillator, x(T) = x0 cos(wT) + v0 sin(wT)/w with
    w = sqrt(beta); Verlet reaches it at T = 1 to O(tau^2)."""
    n, beta = 200, 2.0
    s0 = rbm_inputs.hamilton(n, seed=7).astype(np.float64) + np.array([0.5, -0.3])
    w = math.sqrt(beta)
    want = s0[:, 0].mean() * math.cos(w) + s0[:, 1].mean() * math.sin(w) / w
    errs = []
    for k in (6, 7):
        x, _ = ora.rbm_run(_hamilton(ora, 2.0 ** -k, seed=2, beta=beta), 3, 0, 2 ** k, s0)
        errs.append(abs(x[:, 0].mean() - want))
    assert errs[0] < 1e-3 and 3.5 < errs[0] / errs[1] < 4.5, errs


@pytest.mark.slow
def test_hamiltonian_rbm_error_decays_like_sqrt_tau(ora):
    """Sec. 4.1 second-order example / Theorem A.1: RBM-1 (p = 2) with Verlet
    against the fully coupled Verlet solution (tau = 2^-11) at T = 1, from
    semicircle positions and N(0, 1) velocities: the RMS error of the
    positions, and of positions and velocities together, falls like
    tau^(1/2) (the slope the text reports; the figure's reference line is
    read as 0.2 tau^(1/2))."""
    n = 256
    s0 = rbm_inputs.hamilton(n, seed=3).astype(np.float64)
    ref = _hamilton(ora, 2.0 ** -11)
    sr = s0.copy()
    for m in range(2 ** 11):
        sr = ora.direct_step(ref, m, sr)
    taus = [2.0 ** -k for k in (4, 5, 6, 7, 8)]
    ex, exu = [], []
    for tau in taus:
        e2, e3 = [], []
        for seed in range(1, 9):
            x, _ = ora.rbm_run(_hamilton(ora, tau, seed=seed), 2, 0, int(round(1.0 / tau)), s0)
            e2.append(ora.rms_error(x[:, 0], sr[:, 0]) ** 2)
            e3.append(ora.rms_error(x, sr) ** 2)
        ex.append(math.sqrt(np.mean(e2)))
        exu.append(math.sqrt(np.mean(e3)))
    for errs in (ex, exu):
        slope = np.polyfit(np.log(taus), np.log(errs), 1)[0]
        assert 0.4 < slope < 0.62, (slope, errs)


@pytest.mark.parametrize("kern,d,p", [(2, 3, 8), (3, 1, 2), (4, 1, 2), (5, 2, 3)])
def test_results_do_not_depend_on_the_thread_count(ora, kern, d, p):
    """The oracle's parallel loops give the same bits on 1 and 5 threads: the
    permutation (a parallel merge of per-thread sorted runs of the unique
    keys against one qsort), the batch forces, every update scheme and the
    direct sum."""
    n = 20011 if kern not in (3, 4) else 20012
    prm = ora.Params(d=d, kernel=kern, kparam={2: 0.01, 3: 0.0, 4: 1.0, 5: 1.0}[kern], beta=0.5,
                     sigma=0.0 if kern == 5 else 0.3, dt=1e-3)
    x = rbm_inputs.normal(n, d, seed=31).astype(np.float64)
    if kern == 4:
        x = np.abs(x) + 0.1
    slots = np.random.default_rng(2).permutation(n).astype(np.uint32)
    old = ora.get_threads()
    try:
        res = []
        for t in (1, 5):
            assert ora.set_threads(t) == t
            xs, ss = ora.rbm_run(prm, p, 3, 2, x, slots)
            fd = ora.direct_forces(prm, x[:2000], np.arange(0, 2000, 7))
            res.append((xs, ss, fd))
    finally:
        ora.set_threads(old)
    assert np.array_equal(res[0][1], res[1][1])
    assert np.array_equal(res[0][0], res[1][0])
    assert np.array_equal(res[0][2], res[1][2])
    # the permutation is the key order (one sequential sort of the keys)
    w = np.array([ora.perm_word(prm.seed, prm.sys, 3, k) for k in range(n)], dtype=np.uint64)
    keys = (w << np.uint64(32)) | slots.astype(np.uint64)
    assert np.array_equal(ora.permutation(prm, 3, slots), (np.sort(keys) & np.uint64(0xffffffff)).astype(np.uint32))
