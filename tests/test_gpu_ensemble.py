"""GPU parity of the batched ensemble (many independent RBM-1 systems in one
persistent launch), through the C ABI.

System s of an ensemble with Philox key k_s must follow the definitions of a
standalone run with seed k_s and counter word 3 = s.  Checked against
  - the standalone GPU path (rbm_init / rbm_run / rbm_positions) of each
    system: the same FP32 operations in the same order, so equal bits;
  - the FP64 oracle for sampled systems: e1 <= 1e-5 and e100 <= 1e-3 in the
    max norm relative to max(1, max |x|), as for a standalone run.
"""
import numpy as np
import pytest

import oracle as ora
import rbm_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1812_10575_amd as rbm  # noqa: E402

PHYS = dict(kparam=0.0, beta=1.0, sigma=0.5, dt=1e-3)


def say(*a):
    print(*a, flush=True)


def make(sizes, p=4, kernel=0, d=2, **over):
    ph = dict(PHYS)
    ph.update(over)
    sizes = np.asarray(sizes, np.int64)
    keys = 1 + np.arange(len(sizes), dtype=np.uint64)
    return rbm.Ensemble(d=d, kernel=kernel, p=p, sizes=sizes, seeds=keys, **ph)


def x0_of(ens, seed=3):
    return rbm_inputs.normal(int(np.sum(ens.sizes)), ens.d, seed)


def run(ens, x0, step0, nsteps, **kw):
    x = torch.from_numpy(np.ascontiguousarray(x0)).cuda()
    rbm.ensemble_run(ens, x, step0, nsteps, **kw)
    return x.cpu().numpy()


def standalone(ens, s, x0, step0, nsteps):
    o = ens.offsets
    prm = rbm.Params(d=ens.d, kernel=ens.kernel, n=int(ens.sizes[s]), p=ens.p, kparam=ens.kparam,
                     beta=ens.beta, sigma=ens.sigma, dt=ens.dt, seed=int(ens.seeds[s]), sys=s)
    ctx = rbm.rbm_init(prm, torch.from_numpy(np.ascontiguousarray(x0[o[s]:o[s + 1]])).cuda(), None, step0)
    rbm.rbm_run(ctx, nsteps)
    return rbm.rbm_positions(ctx).cpu().numpy()


def oracle_run(ens, s, x0, step0, nsteps):
    o = ens.offsets
    prm = ora.Params(d=ens.d, kernel=ens.kernel, kparam=ens.kparam, beta=ens.beta, sigma=ens.sigma,
                     dt=ens.dt, seed=int(ens.seeds[s]), sys=s)
    xo, _ = ora.rbm_run(prm, ens.p, step0, nsteps, x0[o[s]:o[s + 1]].astype(np.float64))
    return xo


# sizes: LDS-resident (<= 4096), streamed (one to many buckets, ragged tails)
SIZES = [4, 7, 64, 100, 257, 1000, 2816, 4096, 4097, 5000, 20011, 65536]


@pytest.mark.parametrize("p", [2, 4, 8, 5])
def test_equals_standalone_runs(p):
    sizes = [p, p + 3] + [n for n in SIZES if n > p + 3]
    ens = make(sizes, p=p)
    x0 = x0_of(ens)
    say("ensemble p", p, "sizes", sizes)
    x = run(ens, x0, 0, 6)
    o = ens.offsets
    for s in range(len(sizes)):
        xs = standalone(ens, s, x0, 0, 6)
        assert np.array_equal(x[o[s]:o[s + 1]], xs), (s, sizes[s], np.abs(x[o[s]:o[s + 1]] - xs).max())


def test_one_step_and_hundred_steps_match_the_oracle():
    ens = make([64, 1000, 4096, 6000, 30000])
    x0 = x0_of(ens, 4)
    o = ens.offsets
    x1 = run(ens, x0, 0, 1)
    for s in range(len(ens.sizes)):
        xo = oracle_run(ens, s, x0, 0, 1)
        assert ora.rel_max_error(x1[o[s]:o[s + 1]], xo) <= 1e-5, s
    x100 = run(ens, x0, 7, 100)
    for s in (0, 1, 3):
        xo = oracle_run(ens, s, x0, 7, 100)
        err = ora.rel_max_error(x100[o[s]:o[s + 1]], xo)
        say("e100 system", s, err)
        assert err <= 1e-3, (s, err)


@pytest.mark.parametrize("kernel,over", [(1, dict(kparam=1e-2, beta=1.0, sigma=0.0)),
                                         (2, dict(kparam=0.01, beta=0.0, sigma=0.1))])
def test_other_kernels(kernel, over):
    ens = make([50, 3000, 9000], p=4, kernel=kernel, **over)
    x0 = x0_of(ens, 5)
    x = run(ens, x0, 3, 4)
    o = ens.offsets
    for s in range(3):
        assert np.array_equal(x[o[s]:o[s + 1]], standalone(ens, s, x0, 3, 4)), s
        assert ora.rel_max_error(x[o[s]:o[s + 1]], oracle_run(ens, s, x0, 3, 4)) <= 1e-4, s


def test_streamed_path_equals_lds_path():
    """lds_max = 64 streams every larger system through global memory: the
    result must not change."""
    ens = make([64, 65, 300, 1500, 4096])
    x0 = x0_of(ens, 6)
    a = run(ens, x0, 0, 5)
    b = run(ens, x0, 0, 5, lds_max=64)
    c = run(ens, x0, 0, 5, lds_max=1024, grid=3)
    d = run(ens, x0, 0, 5, wg=512, lds_max=64)
    assert np.array_equal(a, b) and np.array_equal(a, c) and np.array_equal(a, d)


def test_graph_and_direct_launch_agree_and_replay():
    ens = make(rbm_inputs.ensemble_sizes(40, 64, 8192, seed=2))
    x0 = x0_of(ens, 7)
    a = run(ens, x0, 0, 10, graph=True)
    b = run(ens, x0, 0, 10, graph=False)
    c = run(ens, x0, 0, 10, graph=True)
    assert np.array_equal(a, b) and np.array_equal(a, c)


def test_largest_system_and_single_batches():
    ens = make([rbm.ENS_MAXN, 4, 5, 7], p=4)
    x0 = x0_of(ens, 8)
    x = run(ens, x0, 0, 2)
    o = ens.offsets
    for s in range(4):
        assert np.array_equal(x[o[s]:o[s + 1]], standalone(ens, s, x0, 0, 2)), s
    # a system of p particles is one batch: RBM-1 is the direct step
    prm = ora.Params(d=2, kernel=0, kparam=0.0, beta=1.0, sigma=0.5, dt=1e-3, seed=2, sys=1)
    xd = ora.direct_step(prm, 0, x0[o[1]:o[2]].astype(np.float64))
    assert ora.rel_max_error(x[o[1]:o[2]], ora.rbm_run(prm, 4, 0, 2, x0[o[1]:o[2]].astype(np.float64))[0]) <= 1e-5
    x1 = run(ens, x0, 0, 1)
    assert ora.rel_max_error(x1[o[1]:o[2]], xd) <= 1e-5


def test_zero_steps_and_bad_arguments():
    ens = make([64, 100])
    x0 = x0_of(ens, 9)
    assert np.array_equal(run(ens, x0, 0, 0), x0)
    with pytest.raises(rbm.RbmError):
        run(make([3, 100]), x0_of(make([3, 100])), 0, 1)          # N < p
    with pytest.raises(rbm.RbmError):
        run(make([64, rbm.ENS_MAXN + 1]), np.zeros((64 + rbm.ENS_MAXN + 1, 2), np.float32), 0, 1)
    with pytest.raises(rbm.RbmError):
        run(ens, x0, 0, 1, lds_max=rbm.ENS_LDS + 1)
    with pytest.raises(rbm.RbmError):
        run(ens, x0, 0, 1, wg=512, lds_max=2049)
    with pytest.raises(rbm.RbmError):
        run(ens, x0, 0, 1, wg=256)


def test_every_tile_gives_the_same_result():
    """team, bucket and lds_max change the launch shape, never the result."""
    ens = make(rbm_inputs.ensemble_sizes(24, 64, 20000, seed=4))
    x0 = x0_of(ens, 10)
    ref = run(ens, x0, 2, 4)
    for tile in (dict(team=64), dict(team=128, bucket=1024), dict(team=1024, bucket=3072, lds_max=2048),
                 dict(team=512, bucket=256, lds_max=1), dict(wg=512), dict(wg=512, team=64, bucket=1536),
                 dict(wg=512, team=512, bucket=512, lds_max=600)):
        assert np.array_equal(run(ens, x0, 2, 4, **tile), ref), tile


def test_autotuner_picks_a_valid_tile(tmp_path):
    from paper_1812_10575_amd import autotune
    ens = make(rbm_inputs.ensemble_sizes(64, 64, 30000, seed=6))
    x = torch.from_numpy(x0_of(ens, 11)).cuda()
    x_before = x.clone()
    cache = str(tmp_path / "tune.json")
    tile = autotune.tune(ens, x, probe_steps=3, cache=cache)
    assert torch.equal(x, x_before)
    assert tile in list(autotune.candidates(ens))
    assert autotune.tune(ens, x, cache=cache) == tile  # from the cache
    assert np.array_equal(run(ens, x_before.cpu().numpy(), 0, 3, **tile), run(ens, x_before.cpu().numpy(), 0, 3))


def test_full_ensemble_workload_sampled_systems():
    """The ensemble workload itself (4096 systems, N_s log-uniform on [64,
    65536], 500 steps, one graph-replayed launch with the autotuned tile):
    sampled systems equal their standalone GPU runs bit for bit, and the
    smallest ones stay within 2e-3 of the oracle after 500 steps."""
    from paper_1812_10575_amd import autotune
    E = rbm_inputs.ENSEMBLE
    n, keys, x0 = rbm_inputs.ensemble()
    ens = rbm.Ensemble(d=E["d"], kernel=E["kernel"], p=E["p"], sizes=n, seeds=keys, kparam=E["kparam"],
                       beta=E["beta"], sigma=E["sigma"], dt=E["dt"])
    x = torch.from_numpy(x0).cuda()
    tile = autotune.tune(ens, x)
    say("tile", tile)
    rbm.ensemble_run(ens, x, 0, E["steps"], graph=True, **tile)
    xe = x.cpu().numpy()
    o = ens.offsets
    order = np.argsort(n, kind="stable")
    picks = [order[0], order[1], order[len(n) // 4], order[len(n) // 2], order[-len(n) // 4], order[-1]]
    for s in picks:
        say("system", s, "N", n[s])
        assert np.array_equal(xe[o[s]:o[s + 1]], standalone(ens, s, x0, 0, E["steps"])), s
    for s in picks[:2]:
        err = ora.rel_max_error(xe[o[s]:o[s + 1]], oracle_run(ens, s, x0, 0, E["steps"]))
        say("oracle e500", s, err)
        assert err <= 2e-3
