"""Pins of the control-variate oracle (oracle/cv.py)."""
import itertools
import math

import numpy as np
import pytest

import rbm_inputs
from oracle import cv
from test_oracle_pins import divisions


def rand_theta(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    th = cv.glorot_init(seed % 2, seed=seed) * scale
    p = cv.unpack(th)
    for b in ("b1", "b2", "b3"):
        p[b][...] = 0.3 * rng.standard_normal(p[b].shape)
    return th


@pytest.fixture(scope="module")
def thetas():
    return rand_theta(3), rand_theta(4)


def test_gelu_is_the_tanh_form_and_close_to_the_exact_one():
    """Against torch's own tanh-form GELU, and within the known error of that
    form (< 5e-4) of the exact z Phi(z)."""
    torch = pytest.importorskip("torch")
    z = np.linspace(-7, 7, 2801)
    want = torch.nn.functional.gelu(torch.tensor(z, dtype=torch.float64), approximate="tanh").numpy()
    np.testing.assert_allclose(cv.gelu(z), want, rtol=1e-14, atol=1e-15)
    exact = 0.5 * z * (1 + np.vectorize(math.erf)(z / math.sqrt(2)))
    assert np.max(np.abs(cv.gelu(z) - exact)) < 5e-4


def test_gelu_closed_forms():
    assert cv.gelu(np.array(0.0)) == 0.0
    assert cv.gelu_grad(np.array(0.0)) == pytest.approx(0.5, abs=1e-15)
    assert cv.gelu(np.array(8.0)) == pytest.approx(8.0, rel=1e-12)
    assert cv.gelu(np.array(-8.0)) == pytest.approx(0.0, abs=1e-12)
    z = np.linspace(-4, 4, 41)
    h = 1e-6
    np.testing.assert_allclose(cv.gelu_grad(z), (cv.gelu(z + h) - cv.gelu(z - h)) / (2 * h), rtol=1e-7, atol=1e-9)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -2.5, 3.14159, 1e-20, 6.5e4, -7.77e-3], np.float64)
    rng = np.random.default_rng(0)
    vals = np.concatenate([vals, rng.standard_normal(5000) * 10.0 ** rng.integers(-6, 6, 5000)])
    want = torch.tensor(vals, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cv.bf16(vals), want)
    assert cv.bf16(np.array([1 + 2 ** -8]))[0] == 1.0               # tie to even
    assert cv.bf16(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6   # tie to even


def test_gradients_match_finite_differences(thetas):
    ta, tc = thetas
    rng = np.random.default_rng(1)
    x = rng.standard_normal((5, 2))
    y = rng.standard_normal((5, 2))
    _, ga, gc = cv.loss_and_grads(ta, tc, x, y)
    h = 1e-6
    for theta, g, which in ((ta, ga, 0), (tc, gc, 1)):
        for q in rng.choice(cv.NPARAM, 80, replace=False):
            tp, tm = theta.copy(), theta.copy()
            tp[q] += h
            tm[q] -= h
            if which == 0:
                lp = cv.loss_and_grads(tp, tc, x, y)[0]
                lm = cv.loss_and_grads(tm, tc, x, y)[0]
            else:
                lp = cv.loss_and_grads(ta, tp, x, y)[0]
                lm = cv.loss_and_grads(ta, tm, x, y)[0]
            fd = (lp - lm) / (2 * h)
            assert g[q] == pytest.approx(fd, rel=1e-6, abs=1e-9), (which, q)


def test_loss_is_half_mean_squared_residual(thetas):
    ta, tc = thetas
    rng = np.random.default_rng(2)
    x, y = rng.standard_normal((7, 2)), rng.standard_normal((7, 2))
    a = cv.features(ta, x)
    c = cv.features(tc, y)
    res = cv.pair_kernel_gauss(x - y) - np.sum(a * c, axis=2)
    assert cv.loss_and_grads(ta, tc, x, y)[0] == pytest.approx(0.5 * np.mean(np.sum(res ** 2, axis=1)), rel=1e-14)


def _direct_gauss(x):
    n = x.shape[0]
    f = np.zeros_like(x)
    for i in range(n):
        d = x[i][None] - np.delete(x, i, axis=0)
        f[i] = cv.pair_kernel_gauss(d).sum(axis=0) / (n - 1)
    return f


@pytest.mark.parametrize("use_bf16", [False, True])
@pytest.mark.parametrize("n,p", [(6, 2), (7, 3), (8, 4)])
def test_cv_force_is_unbiased_for_any_weights(thetas, n, p, use_bf16):
    """Over every division, the mean control-variate force is the direct
    force (Lemma 3.1 applied to the residual kernel), and for p | N its
    variance is (1/(p-1) - 1/(N-1)) Lambda_i[K_res].  With use_bf16 the
    networks run on BF16 operands and c is rounded to BF16: the residual
    kernel is then K - a . bf16(c), and the force stays exactly unbiased only
    if S and the batch term take the same rounded c."""
    ta, tc = thetas
    x = rbm_inputs.normal(n, 2, seed=n + 40).astype(np.float64)
    fs = np.array([cv.cv_forces(ta, tc, x, [i for b in dv for i in b], p, use_bf16=use_bf16)
                   for dv in divisions(n, p)])
    fd = _direct_gauss(x)
    np.testing.assert_allclose(fs.mean(axis=0), fd, rtol=0, atol=1e-13)
    if use_bf16:
        c = cv.c_features(tc, x, use_bf16=True)
        assert np.array_equal(cv.bf16(c), c)  # the rounded c are BF16 numbers
        assert not np.array_equal(c, cv.features(tc, x, use_bf16=True))
    if n % p == 0:
        a = cv.features(ta, x, use_bf16)
        c = cv.c_features(tc, x, use_bf16)
        var = np.mean(np.sum((fs - fd[None]) ** 2, axis=2), axis=0)
        for i in range(n):
            js = [j for j in range(n) if j != i]
            kres = cv.pair_kernel_gauss(x[i][None] - x[js]) - np.einsum("kr,jkr->jk", a[i], c[js])
            lam = np.sum((kres - kres.mean(axis=0)) ** 2) / (n - 2)
            assert var[i] == pytest.approx((1 / (p - 1) - 1 / (n - 1)) * lam, rel=1e-10, abs=1e-16)


def test_zero_network_is_plain_rbm():
    import oracle as ora
    n, p = 40, 2
    x = rbm_inputs.normal(n, 2, seed=9).astype(np.float64)
    z = np.zeros(cv.NPARAM)
    prm = ora.Params(d=2, kernel=ora.K_GAUSS, kparam=0.0, beta=1.0, sigma=0.0, dt=1e-3)
    perm = ora.permutation(prm, 3, np.arange(n))
    np.testing.assert_allclose(cv.cv_forces(z, z, x, perm, p), ora.rbm_forces(prm, p, x, perm), rtol=1e-13, atol=1e-15)


def _plain_params(sigma):
    import oracle as ora
    return ora.Params(d=2, kernel=ora.K_GAUSS, kparam=0.0, beta=1.0, sigma=sigma, dt=1e-3, seed=5, sys=2)


@pytest.mark.parametrize("n,p", [(41, 3), (64, 2), (9, 9)])
def test_cv_step_with_zero_networks_is_the_plain_step(n, p):
    """Zero networks make the control-variate force the plain batch force, so
    cv_step (division, update and noise of Algorithm 1) must be the plain
    oracle step: sigma > 0, step m > 0, a slot order that is not the
    identity, and a last batch that takes the remainder."""
    import oracle as ora
    prm = _plain_params(0.5)
    x = rbm_inputs.normal(n, 2, seed=21).astype(np.float64)
    slots = np.random.default_rng(n).permutation(n).astype(np.uint32)
    z = np.zeros(cv.NPARAM)
    x1, s1 = cv.cv_step(z, z, prm, p, 7, x, slots)
    xo, so = ora.rbm_step(prm, p, 7, x, slots)
    assert np.array_equal(s1, so)
    np.testing.assert_allclose(x1, xo, rtol=0, atol=1e-13)
    # the noise is there: the step differs from the noiseless one by sigma sqrt(dt) z
    xq, _ = ora.rbm_step(_plain_params(0.0), p, 7, x, slots)
    zz = np.array([ora.normals(5, 2, 7, i)[:2] for i in range(n)])
    np.testing.assert_allclose(x1 - xq, 0.5 * math.sqrt(1e-3) * zz, rtol=0, atol=1e-13)


def test_cv_step_chain_equals_two_plain_steps():
    import oracle as ora
    n, p = 50, 4
    prm = _plain_params(0.5)
    x = rbm_inputs.normal(n, 2, seed=22).astype(np.float64)
    slots = np.random.default_rng(1).permutation(n).astype(np.uint32)
    z = np.zeros(cv.NPARAM)
    x1, s1 = cv.cv_step(z, z, prm, p, 3, x, slots)
    x2, s2 = cv.cv_step(z, z, prm, p, 4, x1, s1)
    xo, so = ora.rbm_run(prm, p, 3, 2, x, slots)
    assert np.array_equal(s2, so)
    np.testing.assert_allclose(x2, xo, rtol=0, atol=1e-13)


def test_cv_step_moves_by_the_cv_force(thetas):
    """With trained-like networks the step keeps the plain step's division and
    noise and replaces only the force: x1(theta) - x1(0) = dt (F_cv - F_plain)
    on the same division; and averaged over every division of a tiny system
    the control-variate force is the direct force (Lemma 3.1 for K_res),
    which the noiseless step then applies."""
    import oracle as ora
    n, p = 8, 2
    prm = _plain_params(0.5)
    x = rbm_inputs.normal(n, 2, seed=23).astype(np.float64)
    slots = np.arange(n, dtype=np.uint32)
    z = np.zeros(cv.NPARAM)
    ta, tc = thetas
    xa, sa = cv.cv_step(ta, tc, prm, p, 2, x, slots)
    xz, sz = cv.cv_step(z, z, prm, p, 2, x, slots)
    assert np.array_equal(sa, sz)
    fcv = cv.cv_forces(ta, tc, x, sa, p)
    fpl = ora.rbm_forces(prm, p, x, sa)
    np.testing.assert_allclose((xa - xz) / 1e-3, fcv - fpl, rtol=1e-9, atol=1e-9)
    mean = np.zeros((n, 2))
    cnt = 0
    for div in divisions(n, p):
        mean += cv.cv_forces(ta, tc, x, np.concatenate(div), p)
        cnt += 1
    np.testing.assert_allclose(mean / cnt, ora.direct_forces(prm, x), rtol=1e-11, atol=1e-13)


def test_adam_first_step_closed_form():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th, m, v = cv.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=1e-3)
    # m_hat = g, v_hat = g^2: the first step is -lr g / (|g| + eps)
    np.testing.assert_allclose(th, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_glorot_init_statistics():
    th = cv.glorot_init(0, seed=1)
    p = cv.unpack(th)
    for name, (fo, fi) in (("W1", (64, 2)), ("W2", (64, 64)), ("W3", (32, 64))):
        lim = math.sqrt(6 / (fo + fi))
        w = p[name].ravel()
        assert np.max(np.abs(w)) <= lim
        assert abs(w.mean()) < 4 * lim / math.sqrt(3 * w.size)
        if w.size > 1000:
            assert w.var() == pytest.approx(lim * lim / 3, rel=0.1)
    assert np.all(p["b1"] == 0) and np.all(p["b2"] == 0) and np.all(p["b3"] == 0)
    assert not np.array_equal(cv.glorot_init(0, 1), cv.glorot_init(1, 1))


def test_pair_sampler():
    pr = cv.sample_pairs(0, 4000, 3, 50)
    assert np.all(pr[:, 1] != pr[:, 2])
    assert pr[:, 0].min() >= 0 and pr[:, 0].max() <= 2
    assert pr[:, 1].min() >= 0 and pr[:, 1].max() <= 49 and pr[:, 2].max() <= 49
    from scipy import stats
    assert stats.chisquare(np.bincount(pr[:, 1], minlength=50)).pvalue > 1e-4
    assert stats.chisquare(np.bincount(pr[:, 2], minlength=50)).pvalue > 1e-4
    assert not np.array_equal(pr, cv.sample_pairs(1, 4000, 3, 50))


def test_forward_of_a_hand_built_network():
    """A network whose output is known in closed form: hidden unit 0 of layer
    1 carries x0 + 2 x1 + 0.5, hidden unit 3 of layer 2 carries
    -1.5 gelu(z1_0) + 0.25, and output 7 reads 2 gelu(z2_3) - 1; every other
    output is its bias (gelu written here in its tanh form)."""
    th = np.zeros(cv.NPARAM)
    p = cv.unpack(th)
    p["W1"][0] = [1.0, 2.0]
    p["b1"][0] = 0.5
    p["b1"][1:] = -40.0            # other layer-1 units: gelu(-40) = 0 up to 1e-300
    p["W2"][3, 0] = -1.5
    p["b2"][3] = 0.25
    p["b2"][np.arange(64) != 3] = -40.0
    p["W3"][7, 3] = 2.0
    p["b3"][:] = np.arange(32) * 0.01
    p["b3"][7] = -1.0
    x = np.array([[0.3, -0.7], [1.1, 0.4], [-2.0, 0.9]])
    phi = lambda z: 0.5 * (1 + np.tanh(math.sqrt(2 / math.pi) * (z + 0.044715 * z ** 3)))
    z1 = x[:, 0] + 2 * x[:, 1] + 0.5
    z2 = -1.5 * z1 * phi(z1) + 0.25
    o7 = 2 * z2 * phi(z2) - 1.0
    out = cv.forward(th, x)[4]
    np.testing.assert_allclose(out[:, 7], o7, rtol=1e-13, atol=1e-13)
    others = np.delete(out, 7, axis=1)
    np.testing.assert_allclose(others, np.broadcast_to(np.delete(np.arange(32) * 0.01, 7), others.shape),
                               atol=1e-13)
    # the feature layout: output 7 is component k = 0, rank r = 7
    assert np.array_equal(cv.features(th, x)[:, 0, 7], out[:, 7])


def test_forces_for_listed_ids_agree_with_all_forces(thetas):
    ta, tc = thetas
    import oracle as ora
    n, p = 203, 4
    x = rbm_inputs.normal(n, 2, seed=21).astype(np.float64)
    prm = ora.Params(d=2, kernel=ora.K_GAUSS, kparam=0.0, beta=1.0, sigma=0.0, dt=1e-3)
    perm = ora.permutation(prm, 5, np.arange(n))
    ids = [0, 7, 100, int(perm[-1]), int(perm[-5])]  # the last batch has p + 3 members
    full = cv.cv_forces(ta, tc, x, perm, p, use_bf16=True)
    np.testing.assert_allclose(cv.cv_forces_ids(ta, tc, x, perm, p, ids, use_bf16=True, chunk=50), full[ids],
                               rtol=1e-12, atol=1e-14)
