"""GPU parity of the RBM-1 step against the FP64 oracle, through the C ABI.

Bars (FP32 GPU vs FP64 oracle):
  - the permutation and hence the batches: bit-exact, every step;
  - one step from the identical state (e1): max-norm error <= 1e-5, relative
    to max(1, max |x|);
  - 100 steps from the identical state (e100): <= 1e-3 in the same norm;
  - equilibrium of the 1-D softened-Coulomb workload: KS distance to the
    semicircle <= 0.01.
"""
import math

import numpy as np
import pytest

import oracle as ora
import rbm_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1812_10575_amd as rbm  # noqa: E402

FIELDS = ("d", "kernel", "n", "p", "kparam", "beta", "sigma", "dt", "seed")


def say(*a):
    print(*a, flush=True)


def gp(w):
    return rbm.Params(**{k: w[k] for k in FIELDS})


def op(w):
    return ora.Params(d=w["d"], kernel=w["kernel"], kparam=w["kparam"], beta=w["beta"],
                      sigma=w["sigma"], dt=w["dt"], seed=w["seed"])


def x0_of(w):
    return rbm_inputs.workload(w["init"], w["n"], w["seed"])


def start(w, x0=None, slots=None, step0=0):
    x0 = x0_of(w) if x0 is None else x0
    st = None if slots is None else torch.from_numpy(np.asarray(slots).view(np.int32)).cuda()
    ctx = rbm.rbm_init(gp(w), torch.from_numpy(np.ascontiguousarray(x0)).cuda(), st, step0)
    return ctx, x0


def state(ctx):
    x = rbm.rbm_positions(ctx).cpu().numpy()
    s = rbm.rbm_perm(ctx).cpu().numpy().view(np.uint32)
    return x, s


def e_rel(x, ref):
    return ora.rel_max_error(x, ref)


CASES = [
    ("gauss2d-n1024-p2", {}),
    ("gauss2d-n1024-p2", {"p": 1024}),
    ("gauss2d-n1024-p2", {"n": 2, "p": 2}),
    ("gauss2d-n1024-p2", {"n": 3, "p": 2}),
    ("gauss2d-n1024-p2", {"n": 2816, "p": 3}),
    ("gauss2d-n1024-p2", {"n": 2817, "p": 2}),
    ("gauss2d-n1024-p2", {"n": 20000, "p": 5}),
    ("dyson1d-n2^20-p2", {"n": 50001}),
    ("attrep3d-n2^24-p8", {"n": 100003, "p": 7}),
    ("attrep3d-n2^24-p8", {"n": 65536, "p": 64}),
    ("attrep3d-n2^24-p8", {"n": 300000, "p": 32}),
]


@pytest.mark.parametrize("name,over", CASES)
def test_perm_bit_exact_and_one_step(name, over):
    w = rbm_inputs.params_of(name, **over)
    say("case", name, over)
    ctx, _ = start(w)
    o = op(w)
    for m in range(3):
        xm, sm = state(ctx)
        rbm.rbm_step(ctx)
        x1, s1 = state(ctx)
        xo, so = ora.rbm_step(o, w["p"], m, xm.astype(np.float64), sm)
        assert np.array_equal(s1, so), f"permutation differs at step {m}"
        err = e_rel(x1, xo)
        assert err <= 1e-5, (m, err)
    rbm.rbm_check(ctx)


def test_forces_match_the_oracle():
    for name, over in [("gauss2d-n1024-p2", {}), ("attrep3d-n2^24-p8", {"n": 70001, "p": 8}),
                       ("dyson1d-n2^20-p2", {"n": 40000})]:
        w = rbm_inputs.params_of(name, **over)
        say("forces", name, over)
        ctx, _ = start(w)
        rbm.rbm_run(ctx, 2)
        x, s = state(ctx)
        for m in (2, 7):
            f = rbm.rbm_forces(ctx, m).cpu().numpy()
            perm = ora.permutation(op(w), m, s)
            fo = ora.rbm_forces(op(w), w["p"], x.astype(np.float64), perm)
            assert e_rel(f, fo) <= 1e-5
        x2, s2 = state(ctx)
        assert np.array_equal(x, x2) and np.array_equal(s, s2), "rbm_forces changed the state"


def test_hundred_steps_gauss2d_every_window():
    """e100 over every 100-step window of the 1000-step Gaussian workload."""
    w = rbm_inputs.params_of("gauss2d-n1024-p2")
    ctx, _ = start(w)
    o = op(w)
    worst = 0.0
    for win in range(10):
        xm, sm = state(ctx)
        rbm.rbm_run(ctx, 100)
        x1, s1 = state(ctx)
        xo, so = ora.rbm_run(o, w["p"], 100 * win, 100, xm.astype(np.float64), sm)
        assert np.array_equal(s1, so)
        worst = max(worst, e_rel(x1, xo))
    say("e100 worst", worst)
    assert worst <= 1e-3


def test_hundred_steps_attrep3d():
    w = rbm_inputs.params_of("attrep3d-n2^24-p8", n=20011)
    ctx, x0 = start(w)
    rbm.rbm_run(ctx, 100)
    x1, s1 = state(ctx)
    xo, so = ora.rbm_run(op(w), w["p"], 0, 100, x0)
    assert np.array_equal(s1, so)
    assert e_rel(x1, xo) <= 1e-3


def test_single_batch_equals_direct_step():
    """p = N: one batch, so the RBM step is the direct step (same noise)."""
    w = rbm_inputs.params_of("gauss2d-n1024-p2", p=1024)
    ctx, x0 = start(w)
    xt = torch.from_numpy(x0).cuda()
    xd = rbm.direct_step(gp(w), xt, 0).cpu().numpy()
    rbm.rbm_step(ctx)
    x1, _ = state(ctx)
    assert e_rel(x1, xd) <= 1e-5
    assert e_rel(xd, ora.direct_step(op(w), 0, x0)) <= 1e-5


@pytest.mark.parametrize("name,n,nsample", [("attrep3d-n2^24-p8", 4096, None),
                                             ("gauss2d-n1024-p2", 3001, None),
                                             ("dyson1d-n2^20-p2", 5000, None),
                                             ("attrep3d-n2^24-p8", 1 << 20, 48)])
def test_direct_forces(name, n, nsample):
    w = rbm_inputs.params_of(name, n=n)
    say("direct", name, n)
    x = x0_of(w)
    xt = torch.from_numpy(x).cuda()
    if nsample is None:
        ids = None
        f = rbm.direct_forces(gp(w), xt).cpu().numpy()
        fo = ora.direct_forces(op(w), x.astype(np.float64))
    else:
        ids = np.random.default_rng(0).choice(n, nsample, replace=False).astype(np.int32)
        f = rbm.direct_forces(gp(w), xt, torch.from_numpy(ids).cuda()).cpu().numpy()
        fo = ora.direct_forces(op(w), x.astype(np.float64), ids.astype(np.uint32))
    # the sum cancels: measure against the scale of the terms, mean_j |K_ij|
    scale = max(1.0, float(np.max(np.abs(fo))))
    assert np.max(np.abs(f - fo)) / scale <= 1e-5


@pytest.mark.parametrize("name,n,nsample", [("gauss2d-n1024-p2", 3001, None),
                                             ("dyson1d-n2^20-p2", 4000, None),
                                             ("attrep3d-n2^24-p8", 1 << 20, 32)])
def test_direct_moments(name, n, nsample):
    """Forces and second moments of the direct sum against the oracle."""
    w = rbm_inputs.params_of(name, n=n)
    say("moments", name, n)
    x = x0_of(w)
    xt = torch.from_numpy(x).cuda()
    ids = None if nsample is None else np.random.default_rng(1).choice(n, nsample, replace=False).astype(np.int32)
    f, m2 = rbm.direct_moments(gp(w), xt, None if ids is None else torch.from_numpy(ids).cuda())
    fo, m2o = ora.direct_moments(op(w), x.astype(np.float64), None if ids is None else ids.astype(np.uint32))
    scale = max(1.0, float(np.max(np.abs(fo))))
    assert np.max(np.abs(f.cpu().numpy() - fo)) / scale <= 1e-5
    np.testing.assert_allclose(m2.cpu().numpy(), m2o, rtol=1e-5)


@pytest.mark.parametrize("name,n,p", [("gauss2d-n1024-p2", 4096, 2), ("attrep3d-n2^24-p8", 8192, 8),
                                      ("gauss2d-n1024-p2", 4096, 16)])
def test_force_mse_follows_lemma_3_1(name, n, p):
    """Over many divisions the mean squared RBM-1 force error equals
    (1/(p-1) - 1/(N-1)) Lambda_i averaged over the particles, Lambda_i from
    the direct sum's moments (Lemma 3.1; p divides N)."""
    w = rbm_inputs.params_of(name, n=n, p=p)
    say("lemma 3.1", name, n, p)
    ctx, x0 = start(w)
    x, _ = state(ctx)
    xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    fd, m2 = rbm.direct_moments(gp(w), xt)
    fd64 = fd.double()
    lam = (n - 1) / (n - 2) * (m2.double() - (fd64 * fd64).sum(dim=1))
    pred = float(((1.0 / (p - 1) - 1.0 / (n - 1)) * lam).mean())
    acc, R = 0.0, 300
    for m in range(R):
        f = rbm.rbm_forces(ctx, 1000 + m).double()
        acc += float(((f - fd64) ** 2).sum())
    mse = acc / (R * n)
    say("mse", mse, "predicted", pred)
    assert abs(mse / pred - 1.0) < 0.03


def test_full_size_attrep3d_step():
    """The headline size N = 2^24, p = 8, run as the benchmark runs it (9 steps
    in one call sharing one launch of the key passes; the sort kernels of the
    first 8 write the next step's coarse buckets): the slot order after every
    step bit-exact (the oracle chains its permutations), then one more step
    from the GPU's state, every particle within 1e-5."""
    w = rbm_inputs.params_of("attrep3d-n2^24-p8")
    say("full size", w["n"])
    ctx, x0 = start(w)
    rbm.rbm_run(ctx, 9)
    rbm.rbm_check(ctx)
    x9, s9 = state(ctx)
    so = np.arange(w["n"], dtype=np.uint32)
    for m in range(9):
        so = ora.permutation(op(w), m, so)
    assert np.array_equal(s9, so)
    rbm.rbm_step(ctx)
    rbm.rbm_check(ctx)
    x10, s10 = state(ctx)
    xo, so10 = ora.rbm_step(op(w), w["p"], 9, x9.astype(np.float64), s9)
    assert np.array_equal(s10, so10)
    assert e_rel(x10, xo) <= 1e-5


@pytest.mark.parametrize("n,p", [(1 << 25, 3), (217600, 8), (217601, 8)])
def test_largest_supported_size(n, p):
    """N = 2^25 (the largest the plan supports: 19840 fine buckets of 1691
    records on average), p = 3 with a remainder of 2; and the two sides of
    the switch to the split level (128 fine buckets of 1700 records, then
    256 of 850 in two coarse buckets): permutation bit-exact and
    e1 <= 1e-5."""
    w = rbm_inputs.params_of("dyson1d-n2^20-p2", n=n, p=p)
    say("max size", w["n"], w["p"])
    ctx, x0 = start(w)
    rbm.rbm_step(ctx)
    rbm.rbm_check(ctx)
    x1, s1 = state(ctx)
    xo, so = ora.rbm_step(op(w), w["p"], 0, x0.astype(np.float64), np.arange(w["n"], dtype=np.uint32))
    assert np.array_equal(s1, so)
    assert e_rel(x1, xo) <= 1e-5


def test_replay_is_bitwise_deterministic():
    w = rbm_inputs.params_of("attrep3d-n2^24-p8", n=1 << 20)
    outs = []
    for _ in range(2):
        ctx, _ = start(w)
        rbm.rbm_run(ctx, 5)
        outs.append(state(ctx))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_resume_from_saved_slots_is_bitwise():
    w = rbm_inputs.params_of("attrep3d-n2^24-p8", n=100003, p=7)
    ctx, _ = start(w)
    rbm.rbm_run(ctx, 10)
    xa, sa = state(ctx)
    ctx, _ = start(w)
    rbm.rbm_run(ctx, 4)
    xh, sh = state(ctx)
    ctx2, _ = start(w, x0=xh, slots=sh, step0=4)
    rbm.rbm_run(ctx2, 6)
    xb, sb = state(ctx2)
    assert rbm.rbm_step_index(ctx2) == 10
    assert np.array_equal(sa, sb) and np.array_equal(xa, xb)


def test_odd_kernel_keeps_the_centre_of_mass():
    w = rbm_inputs.params_of("attrep3d-n2^24-p8", n=1 << 18, sigma=0.0)
    ctx, x0 = start(w)
    rbm.rbm_run(ctx, 50)
    x1, _ = state(ctx)
    drift = np.abs(x1.astype(np.float64).mean(axis=0) - x0.astype(np.float64).mean(axis=0))
    assert np.max(drift) < 1e-5


def test_dyson1d_relaxes_to_the_semicircle():
    """1-D softened Coulomb with V = x^2/2, sigma = 0, N = 2^20, dt = 1e-4,
    from U[-3, 3]: KS distance to the semicircle law of radius sqrt 2
    (Sec. 4.2) after T = 10; m2 sits at the fixed point of the exact
    second-moment step identity."""
    w = rbm_inputs.params_of("dyson1d-n2^20-p2")
    ctx, x0 = start(w)
    for k in range(10):
        rbm.rbm_run(ctx, 10000)
        torch.cuda.synchronize()
        say("dyson t =", (k + 1) * 10000 * w["dt"])
    rbm.rbm_check(ctx)
    x, s = state(ctx)
    ks = ora.ks_distance(x.astype(np.float64), ora.semicircle_cdf)
    m2 = float(np.mean(x.astype(np.float64) ** 2))
    # c1 = mean(x F), c2 = mean(F^2) of the next division, from the GPU forces
    c1, c2 = [], []
    for m in range(100000, 100020):
        f = rbm.rbm_forces(ctx, m).cpu().numpy().astype(np.float64)
        c1.append(np.mean(x * f))
        c2.append(np.mean(f * f))
    dt = w["dt"]
    m2s = (2 * (1 - dt) * np.mean(c1) + dt * np.mean(c2)) / (2 - dt)
    say(f"KS={ks:.5f} m2={m2:.5f} m2*={m2s:.5f}")
    assert ks <= 0.01
    assert abs(m2 - m2s) < 0.01


# --------------------------------------------------------------------------
# splitting with the exact pair flow (K = x/|x|^2, p = 2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,d", [(1024, 1), (20000, 1), (300002, 1), (50000, 2), (4096, 3)])
def test_split_scheme_matches_the_oracle(n, d):
    """Permutation bit-exact and e1 <= 1e-5 for three steps, forces of the
    division against the oracle's x/|x|^2 forces."""
    w = rbm_inputs.params_of("dysonsplit1d-n2^20-p2", n=n, d=d, sigma=1.0 / math.sqrt(n))
    w["init"] = "semicircle2" if d == 1 else "gauss2d" if d == 2 else "attrep3d"
    say("split", n, d)
    ctx, _ = start(w)
    o = op(w)
    for m in range(3):
        xm, sm = state(ctx)
        rbm.rbm_step(ctx)
        x1, s1 = state(ctx)
        xo, so = ora.rbm_step(o, 2, m, xm.astype(np.float64), sm)
        assert np.array_equal(s1, so), m
        assert e_rel(x1, xo) <= 1e-5, (m, e_rel(x1, xo))
    rbm.rbm_check(ctx)
    x, s = state(ctx)
    f = rbm.rbm_forces(ctx, 3).cpu().numpy()
    fo = ora.rbm_forces(o, 2, x.astype(np.float64), ora.permutation(o, 3, s))
    assert e_rel(f, fo) <= 1e-5


def test_split_scheme_hundred_steps():
    w = rbm_inputs.params_of("dysonsplit1d-n2^20-p2", n=20000, sigma=1.0 / math.sqrt(20000))
    ctx, x0 = start(w)
    rbm.rbm_run(ctx, 100)
    x1, s1 = state(ctx)
    xo, so = ora.rbm_run(op(w), 2, 0, 100, x0.astype(np.float64))
    assert np.array_equal(s1, so)
    assert e_rel(x1, xo) <= 1e-3


def test_dyson_split_follows_the_analytic_density_at_scale():
    """Sec. 4.2 at N = 2^20: from the radius-2 semicircle the empirical law
    follows rho(x, t) = sqrt(2 s(t) - x^2) / (s(t) pi), s(t) = 1 + e^{-2t}
    (KS <= 0.01 and second moment s(t)/2 at t = 0.5, 1 and 5), ending at the
    semicircle of radius sqrt(2) without the bias of the softened Euler
    scheme."""
    w = rbm_inputs.params_of("dysonsplit1d-n2^20-p2")
    ctx, _ = start(w)
    m = 0
    for t_end in (0.5, 1.0, 5.0):
        steps = int(round(t_end / w["dt"])) - m
        rbm.rbm_run(ctx, steps)
        m += steps
        x, _ = state(ctx)
        sig = 1 + math.exp(-2 * t_end)
        ks = ora.ks_distance(x[:, 0].astype(np.float64), lambda v: ora.semicircle_cdf_r(v, math.sqrt(2 * sig)))
        m2 = float(np.mean(x.astype(np.float64) ** 2))
        say("t", t_end, "KS", ks, "m2", m2, "analytic", sig / 2)
        assert ks <= 0.01, (t_end, ks)
        assert abs(m2 - sig / 2) <= 0.003, (t_end, m2)
    rbm.rbm_check(ctx)


# --------------------------------------------------------------------------
# the wealth model (linear trading kernel, exact pair flow, multiplicative noise)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1024, 20000, 300002])
def test_wealth_scheme_matches_the_oracle(n):
    w = rbm_inputs.params_of("wealth1d-n2^20-p2", n=n)
    say("wealth", n)
    ctx, _ = start(w)
    o = op(w)
    for m in range(3):
        xm, sm = state(ctx)
        rbm.rbm_step(ctx)
        x1, s1 = state(ctx)
        xo, so = ora.rbm_step(o, 2, m, xm.astype(np.float64), sm)
        assert np.array_equal(s1, so), m
        assert e_rel(x1, xo) <= 1e-5, (m, e_rel(x1, xo))
    rbm.rbm_check(ctx)
    x, s = state(ctx)
    f = rbm.rbm_forces(ctx, 3).cpu().numpy()
    fo = ora.rbm_forces(o, 2, x.astype(np.float64), ora.permutation(o, 3, s))
    assert e_rel(f, fo) <= 1e-5
    with pytest.raises(rbm.RbmError):
        rbm.direct_step(gp(w), torch.from_numpy(np.ascontiguousarray(x)).cuda(), 0)


def test_wealth_scheme_hundred_steps():
    w = rbm_inputs.params_of("wealth1d-n2^20-p2", n=20000)
    ctx, x0 = start(w)
    rbm.rbm_run(ctx, 100)
    x1, s1 = state(ctx)
    xo, so = ora.rbm_run(op(w), 2, 0, 100, x0.astype(np.float64))
    assert np.array_equal(s1, so)
    assert e_rel(x1, xo) <= 1e-3


def test_wealth_reaches_the_inverse_gamma_law_at_scale():
    """Sec. 5 at N = 2^20, kappa = D = 1, tau = 1e-3, T = 3, from |N(0,1)|:
    every wealth stays positive, the mean wealth stays at sqrt(2/pi) up to
    the noise's random walk, and the law is the inverse Gamma law of shape 2
    and scale eta (KS <= 0.01)."""
    w = rbm_inputs.params_of("wealth1d-n2^20-p2")
    ctx, x0 = start(w)
    rbm.rbm_run(ctx, w["steps"])
    rbm.rbm_check(ctx)
    x, _ = state(ctx)
    y = x[:, 0].astype(np.float64)
    eta = float(y.mean())
    ks = ora.ks_distance(y, lambda v: ora.inverse_gamma_cdf(v, 2.0, eta))
    say("wealth eta", eta, "initial", float(x0.mean()), "KS", ks)
    assert np.all(y > 0)
    assert abs(eta - math.sqrt(2 / math.pi)) < 0.03
    assert ks <= 0.01


# --------------------------------------------------------------------------
# the second-order (Hamiltonian) system with Verlet (Sec. 4.1, Appendix A)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,p", [(1024, 2), (20001, 3), (300002, 2), (100003, 7), (65536, 8), (1 << 20, 2)])
def test_hamilton_matches_the_oracle(n, p):
    """Records (x, u): permutation bit-exact and e1 <= 1e-5 for the first
    three steps (the half kick of step 0, then full kicks); the batch forces
    have a zero velocity component."""
    w = rbm_inputs.params_of("hamilton1d-n2^20-p2", n=n, p=p)
    say("hamilton", n, p)
    ctx, _ = start(w)
    o = op(w)
    for m in range(3):
        xm, sm = state(ctx)
        rbm.rbm_step(ctx)
        x1, s1 = state(ctx)
        xo, so = ora.rbm_step(o, p, m, xm.astype(np.float64), sm)
        assert np.array_equal(s1, so), m
        assert e_rel(x1, xo) <= 1e-5, (m, e_rel(x1, xo))
    rbm.rbm_check(ctx)
    x, s = state(ctx)
    f = rbm.rbm_forces(ctx, 3).cpu().numpy()
    assert np.all(f[:, 1] == 0.0)
    fo = ora.rbm_forces(o, p, x.astype(np.float64), ora.permutation(o, 3, s))
    assert e_rel(f, fo) <= 1e-5


def test_hamilton_hundred_steps_and_direct_verlet():
    """100 RBM-1 Verlet steps against the oracle (e100 <= 1e-3); the fully
    coupled Verlet step (direct_step) against the oracle's at steps 0 and 1,
    and its forces with a zero velocity component."""
    w = rbm_inputs.params_of("hamilton1d-n2^20-p2", n=20000, p=2)
    ctx, x0 = start(w)
    rbm.rbm_run(ctx, 100)
    x1, s1 = state(ctx)
    xo, so = ora.rbm_run(op(w), 2, 0, 100, x0.astype(np.float64))
    assert np.array_equal(s1, so)
    assert e_rel(x1, xo) <= 1e-3, e_rel(x1, xo)
    w = rbm_inputs.params_of("hamilton1d-n2^20-p2", n=3001)
    x = x0_of(w)
    xt = torch.from_numpy(x).cuda()
    for m in (0, 1):
        y = rbm.direct_step(gp(w), xt, m).cpu().numpy()
        assert e_rel(y, ora.direct_step(op(w), m, x.astype(np.float64))) <= 1e-5, m
    f = rbm.direct_forces(gp(w), xt).cpu().numpy()
    assert np.all(f[:, 1] == 0.0)
    assert e_rel(f, ora.direct_forces(op(w), x.astype(np.float64))) <= 1e-5


@pytest.mark.parametrize("n,p", [(2000, 2000), (50001, 5)])
def test_hamilton_in_a_harmonic_field(n, p):
    """b(x) = -beta x (Appendix A) with beta = 2, including p = N (one batch,
    the one-workgroup path): three steps against the oracle, and p = N
    equals the fully coupled Verlet step."""
    w = rbm_inputs.params_of("hamilton1d-n2^20-p2", n=n, p=p, beta=2.0)
    ctx, x0 = start(w)
    o = op(w)
    for m in range(3):
        xm, sm = state(ctx)
        rbm.rbm_step(ctx)
        x1, s1 = state(ctx)
        xo, so = ora.rbm_step(o, p, m, xm.astype(np.float64), sm)
        assert np.array_equal(s1, so), m
        assert e_rel(x1, xo) <= 1e-5, (m, e_rel(x1, xo))
    if p == n:
        ctx, _ = start(w)
        rbm.rbm_step(ctx)
        x1, _ = state(ctx)
        xd = rbm.direct_step(gp(w), torch.from_numpy(x0).cuda(), 0).cpu().numpy()
        assert e_rel(x1, xd) <= 1e-5


def test_hamilton_rejects_noise_and_other_d():
    for over in ({"sigma": 0.1}, {"d": 1}, {"d": 3}, {"kparam": 0.0}):
        w = rbm_inputs.params_of("hamilton1d-n2^20-p2", n=1024, **over)
        with pytest.raises(rbm.RbmError):
            rbm.rbm_workspace_size(gp(w))


def test_hamilton_full_size_momentum_and_centre_of_mass():
    """N = 2^20, tau = 2^-7, T = 1 (the timed configuration): the batch
    forces cancel, so the mean velocity stays at its start value and the
    centre of mass moves with it (FP32 sums of 2^20 terms: 1e-5)."""
    w = rbm_inputs.params_of("hamilton1d-n2^20-p2")
    ctx, x0 = start(w)
    rbm.rbm_run(ctx, w["steps"])
    rbm.rbm_check(ctx)
    x, _ = state(ctx)
    x = x.astype(np.float64)
    v0 = float(x0[:, 1].astype(np.float64).mean())
    c0 = float(x0[:, 0].astype(np.float64).mean())
    say("mean u", x[:, 1].mean(), v0, "mean x", x[:, 0].mean(), c0 + v0)
    assert abs(x[:, 1].mean() - v0) < 1e-5
    assert abs(x[:, 0].mean() - (c0 + w["steps"] * w["dt"] * v0)) < 1e-5
    assert np.all(np.isfinite(x))


def test_hamilton_error_decays_like_sqrt_tau_on_the_gpu():
    """Theorem A.1 on the GPU path at N = 2^14: RBM-1 (p = 2) Verlet against
    the fully coupled Verlet solution (tau = 2^-11, direct_step) at T = 1;
    the RMS position error over 4 seeds falls like tau^(1/2), and is the
    size the oracle finds at N = 256 (the bound does not depend on N)."""
    n = 1 << 14
    w = rbm_inputs.params_of("hamilton1d-n2^20-p2", n=n, dt=2.0 ** -11)
    x0 = x0_of(w)
    xr = torch.from_numpy(x0).cuda()
    for m in range(2 ** 11):
        xr = rbm.direct_step(gp(w), xr, m)
    xr = xr.cpu().numpy().astype(np.float64)
    taus = [2.0 ** -k for k in (4, 5, 6, 7, 8)]
    errs = []
    for tau in taus:
        e2 = []
        for seed in range(1, 5):
            ws = dict(w, dt=tau, seed=seed)
            ctx, _ = start(ws, x0)
            rbm.rbm_run(ctx, int(round(1.0 / tau)))
            x, _ = state(ctx)
            e2.append(ora.rms_error(x[:, 0], xr[:, 0]) ** 2)
        errs.append(math.sqrt(np.mean(e2)))
    slope = np.polyfit(np.log(taus), np.log(errs), 1)[0]
    say("hamilton errors", errs, "slope", slope)
    assert 0.4 < slope < 0.62, (slope, errs)
    assert 0.02 < errs[0] < 0.08, errs
