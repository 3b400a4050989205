"""GPU parity of RBM-r (Sec. 2.2) against the FP64 oracle, through the C ABI.

Bars (FP32 GPU vs FP64 oracle, max-norm relative to max(1, max |x|)):
  - a few windows of iterations: <= 1e-5 per touch of a particle, i.e.
    <= 1e-5 after about one window of N/p iterations, <= 1e-4 after ten;
  - the schedule: any window and round count give the same bits, and a run
    split over calls equals one call;
  - the Dyson Brownian motion at N = 2^20: the analytic density of Sec. 4.2
    at t = 0.5, 1 and 5 (KS <= 0.01).
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


def gpu_run(w, x0, k0, niter, **kw):
    x = torch.from_numpy(np.ascontiguousarray(x0, dtype=np.float32)).cuda()
    rbm.rbmr_run(gp(w), x, k0, niter, **kw)
    torch.cuda.synchronize()
    return x.cpu().numpy()


CASES = [
    # name, overrides, init, iterations (in windows of N/p)
    ("gauss2d-n1024-p2", {}, "gauss2d", 3),
    ("gauss2d-n1024-p2", {"n": 3, "p": 2}, "gauss2d", 40),
    ("gauss2d-n1024-p2", {"n": 8, "p": 8}, "gauss2d", 30),
    ("gauss2d-n1024-p2", {"n": 20001, "p": 5}, "gauss2d", 2),
    ("dyson1d-n2^20-p2", {"n": 50001, "kparam": 1.0, "sigma": 0.1, "dt": 1e-2}, "dyson1d", 2),
    ("attrep3d-n2^24-p8", {"n": 100003, "p": 7}, "attrep3d", 1),
    ("attrep3d-n2^24-p8", {"n": 65536, "p": 3}, "attrep3d", 2),
    ("dysonrbmr1d-n2^20-p2", {"n": 30000, "sigma": 1.0 / math.sqrt(30000)}, "semicircle2", 3),
    ("dysonrbmr1d-n2^20-p2", {"n": 20001, "d": 3, "sigma": 0.05}, "attrep3d", 2),
    ("dysonrbmr1d-n2^20-p2", {"n": 4097, "d": 2, "sigma": 0.0}, "gauss2d", 3),
]


@pytest.mark.parametrize("name,over,init,windows", CASES)
def test_rbmr_matches_the_oracle(name, over, init, windows):
    w = rbm_inputs.params_of(name, **over)
    n, p = w["n"], w["p"]
    niter = windows * max(n // p, 1)
    say("rbmr", name, over, niter)
    x0 = rbm_inputs.workload(init, n, w["seed"])
    xg = gpu_run(w, x0, 5, niter)
    xo = ora.rbmr_run(op(w), p, 5, niter, x0.astype(np.float64))
    e = ora.rel_max_error(xg, xo)
    say("e", e)
    assert e <= 1e-5 * max(windows, 1) * (2 if p > 2 else 1), e


def test_rbmr_ten_windows():
    w = rbm_inputs.params_of("gauss2d-n1024-p2", n=4096)
    x0 = rbm_inputs.workload("gauss2d", 4096, 1)
    niter = 10 * 2048
    e = ora.rel_max_error(gpu_run(w, x0, 0, niter), ora.rbmr_run(op(w), 2, 0, niter, x0.astype(np.float64)))
    assert e <= 1e-4, e


def test_rbmr_schedule_does_not_change_the_bits():
    """Window and round count (down to one round, where most iterations run
    in the ordered tail) and splitting the run over calls give identical
    positions."""
    w = rbm_inputs.params_of("attrep3d-n2^24-p8", n=4096, p=3)
    x0 = rbm_inputs.workload("attrep3d", 4096, 1)
    niter = 5000
    ref = gpu_run(w, x0, 0, niter)
    for kw in ({"window": 1}, {"window": 777}, {"window": 5000, "rounds": 1}, {"rounds": 2}, {"window": 64, "rounds": 255}):
        say("schedule", kw)
        assert np.array_equal(gpu_run(w, x0, 0, niter, **kw), ref), kw
    x = torch.from_numpy(x0).cuda()
    rbm.rbmr_run(gp(w), x, 0, 1234)
    rbm.rbmr_run(gp(w), x, 1234, niter - 1234, window=100)
    assert np.array_equal(x.cpu().numpy(), ref)


def test_rbmr_deep_windows_finish_in_order():
    """N = 8 particles, windows of 1000 pairs: the dependency chains are
    hundreds of iterations deep, so after one round across the GPU the
    finishing workgroup's 64 rounds leave most of each window to its ordered
    part.  Same bits as windows of 4 with 16 rounds, and the oracle's
    sequential run."""
    w = rbm_inputs.params_of("gauss2d-n1024-p2", n=8, p=2)
    x0 = rbm_inputs.workload("gauss2d", 8, 3)
    niter = 3000
    deep = gpu_run(w, x0, 7, niter, window=1000, rounds=1)
    shallow = gpu_run(w, x0, 7, niter, window=4, rounds=16)
    assert np.array_equal(deep, shallow)
    assert ora.rel_max_error(deep, ora.rbmr_run(op(w), 2, 7, niter, x0.astype(np.float64))) <= 1e-4


def test_rbmr_rejects_bad_arguments():
    w = rbm_inputs.params_of("gauss2d-n1024-p2")
    x = torch.zeros((1024, 2), dtype=torch.float32, device="cuda")
    for over in ({"p": 9}, {"kernel": 4}, {"kernel": 5}, {"kernel": 3, "p": 3}, {"sigma": -1.0}):
        with pytest.raises(rbm.RbmError):
            rbm.rbmr_workspace_size(gp(dict(w, **over)))
    for kw in ({"window": -1}, {"window": (1 << 22) + 1}, {"rounds": 256}):
        with pytest.raises(rbm.RbmError):
            rbm.rbmr_run(gp(w), x, 0, 10, **kw)
    with pytest.raises(rbm.RbmError):
        rbm.rbmr_run(gp(w), x, (1 << 48) - 5, 10)
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(rbm.RbmError):
        rbm.rbmr_run(gp(w), x, 0, 10, ws=ws)


def test_rbmr_full_size_window_matches_the_oracle():
    """N = 2^20, p = 2, the timed workload: one window of N/2 iterations from
    the semicircle, every particle against the oracle."""
    w = rbm_inputs.params_of("dysonrbmr1d-n2^20-p2")
    x0 = rbm_inputs.workload(w["init"], w["n"], w["seed"])
    niter = w["n"] // 2
    xg = gpu_run(w, x0, 0, niter)
    xo = ora.rbmr_run(op(w), 2, 0, niter, x0.astype(np.float64))
    e = ora.rel_max_error(xg, xo)
    say("full size e", e)
    assert e <= 1e-5


def test_rbmr_dyson_follows_the_analytic_density_at_scale():
    """Sec. 4.2's RBM-r figure at N = 2^20: N/2 iterations per dt = 1e-3, from
    the radius-2 semicircle; KS to rho(x, t) <= 0.01 and second moment s/2 at
    t = 0.5, 1 and 5."""
    w = rbm_inputs.params_of("dysonrbmr1d-n2^20-p2")
    x = torch.from_numpy(rbm_inputs.workload(w["init"], w["n"], w["seed"])).cuda()
    ws = torch.empty(rbm.rbmr_workspace_size(gp(w)), dtype=torch.uint8, device="cuda")
    per = w["n"] // 2
    k = 0
    for t_end in (0.5, 1.0, 5.0):
        it = int(round(t_end / w["dt"])) * per - k
        rbm.rbmr_run(gp(w), x, k, it, ws=ws)
        k += it
        y = x.cpu().numpy()[:, 0].astype(np.float64)
        s = 1 + math.exp(-2 * t_end)
        ks = ora.ks_distance(y, lambda v: ora.semicircle_cdf_r(v, math.sqrt(2 * s)))
        say("t", t_end, "KS", ks, "m2", float(np.mean(y * y)), s / 2)
        assert ks <= 0.01, (t_end, ks)
        assert abs(float(np.mean(y * y)) - s / 2) <= 0.003


def test_rbmr_largest_system_and_window():
    """N = 2^25 (the largest system), p = 2, one default window of 2^22
    iterations (the largest window): the schedule sort at its limits (8192
    buckets of 4096 particles, 256 counting workgroups); every particle
    against the oracle."""
    n = 1 << 25
    w = rbm_inputs.params_of("dysonrbmr1d-n2^20-p2", n=n, sigma=1.0 / math.sqrt(n))
    x0 = rbm_inputs.workload(w["init"], n, w["seed"])
    niter = 1 << 22
    say("rbmr N = 2^25, one window of", niter)
    xg = gpu_run(w, x0, 11, niter)
    xo = ora.rbmr_run(op(w), 2, 11, niter, x0.astype(np.float64))
    e = ora.rel_max_error(xg, xo)
    say("e", e)
    assert e <= 1e-5


def test_rbmr_dense_window_takes_the_long_list_paths():
    """N = 2^20, p = 8 and a window of 10 N / 8 iterations: each particle is
    in about 10 batches of the window, so a bucket holds more entries than
    its workgroup groups in LDS, most particles' lists are longer than the
    register sort takes (the in-place paths), and the window is about 210
    levels deep (the default 200 rounds, then the finishing workgroup).
    Same bits as windows of N/p, and the oracle."""
    n = 1 << 20
    w = rbm_inputs.params_of("gauss2d-n1024-p2", n=n, p=8)
    x0 = rbm_inputs.workload("gauss2d", n, 4)
    niter = n * 10 // 8
    say("rbmr dense window", n, niter)
    dense = gpu_run(w, x0, 3, niter, window=niter)
    plain = gpu_run(w, x0, 3, niter)
    assert np.array_equal(dense, plain)
    xo = ora.rbmr_run(op(w), 8, 3, niter, x0.astype(np.float64))
    e = ora.rel_max_error(dense, xo)
    say("e", e)
    assert e <= 1e-4
