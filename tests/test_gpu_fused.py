"""Fused steps of one rbm_run call against the same steps taken one call at a time.

In one rbm_run call, the sort kernel of every step but the last writes its
updated records straight into the coarse buckets of the next step (placed
by the cross counts of the key passes, which groups of up to 16 steps share;
a group's last step crosses into the next group, whose key passes are made
in the other bank of key sets); the next step skips the coarse scatter and
its split adds the deferred noise.  A step run on its own (rbm_step) always takes the unfused
order, whose parity with the oracle is tested in test_gpu_rbm.py.  The two
orders do the same arithmetic on the same records, so the bar is bit
equality: positions (velocities for the second-order workload) and the slot
order.  One case is also compared with the oracle directly.
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

FIELDS = ("d", "kernel", "n", "p", "kparam", "beta", "sigma", "dt", "seed")


def say(*a):
    print(*a, flush=True)


def gp(w):
    return rbm.Params(**{k: w[k] for k in FIELDS})


def start(w, x0):
    return rbm.rbm_init(gp(w), torch.from_numpy(np.ascontiguousarray(x0)).cuda(), None, 0)


def state(ctx):
    x = rbm.rbm_positions(ctx).cpu().numpy()
    s = rbm.rbm_perm(ctx).cpu().numpy().view(np.uint32)
    return x, s


# (workload, overrides, steps): every case has more than 128 fine buckets
# (the split level, which fused steps need)
CASES = [
    ("attrep3d-n2^24-p8", {"n": 300007}, 19),              # d = 3, p = 8 unrolled, a group of 16 and three more
    ("attrep3d-n2^24-p8", {"n": 300007, "p": 4}, 40),      # groups in both banks of key sets and back
    ("attrep3d-n2^24-p8", {"n": 1 << 20, "p": 7}, 10),     # the runtime batch loop, a remainder batch
    ("gauss2d-n1024-p2", {"n": 500000, "p": 5}, 8),
    ("dyson1d-n2^20-p2", {"n": 250000, "p": 3}, 8),        # two coarse buckets
    ("dysonsplit1d-n2^20-p2", {}, 8),                      # pairs moved by their exact flow
    ("wealth1d-n2^20-p2", {}, 8),                          # multiplicative noise
    ("hamilton1d-n2^20-p2", {}, 8),                        # Verlet records (x, u)
    ("attrep3d-n2^24-p8", {"n": 300007, "p": 64}, 5),      # the largest batch: one fix-up team per workgroup
    ("attrep3d-n2^24-p8", {"n": 217601}, 6),               # the smallest N with the split level
    ("attrep3d-n2^24-p8", {}, 3),                          # the headline size
    ("dyson1d-n2^20-p2", {"n": 1 << 25, "p": 3}, 3),       # the larger sort capacity
]


@pytest.mark.parametrize("name,over,steps", CASES)
def test_fused_run_equals_single_steps(name, over, steps):
    w = rbm_inputs.params_of(name, **over)
    say("fused", name, over, steps)
    x0 = rbm_inputs.workload(w["init"], w["n"], w["seed"])
    a = start(w, x0)
    rbm.rbm_run(a, steps)
    rbm.rbm_check(a)
    xa, sa = state(a)
    del a
    b = start(w, x0)
    for _ in range(steps):
        rbm.rbm_step(b)
    rbm.rbm_check(b)
    xb, sb = state(b)
    assert np.array_equal(sa, sb), "slot order differs"
    assert np.array_equal(xa.view(np.uint32), xb.view(np.uint32)), "positions differ"


def test_fused_run_matches_the_oracle():
    w = rbm_inputs.params_of("attrep3d-n2^24-p8", n=300007)
    x0 = rbm_inputs.workload(w["init"], w["n"], w["seed"])
    ctx = start(w, x0)
    rbm.rbm_run(ctx, 19)
    rbm.rbm_check(ctx)
    x, s = state(ctx)
    o = ora.Params(d=w["d"], kernel=w["kernel"], kparam=w["kparam"], beta=w["beta"],
                   sigma=w["sigma"], dt=w["dt"], seed=w["seed"])
    xo, so = ora.rbm_run(o, w["p"], 0, 19, x0.astype(np.float64))
    assert np.array_equal(s, so)
    assert ora.rel_max_error(x, xo) <= 1e-4


def test_unfused_order_gives_the_same_bits(monkeypatch):
    """RBM_FUSE=0 (read at rbm_init) plans the unfused order: every step of
    an rbm_run call runs the coarse scatter, groups of 16 steps share one
    bank of key sets.  It gives the same bits as the fused run."""
    w = rbm_inputs.params_of("attrep3d-n2^24-p8", n=300007, p=5)
    x0 = rbm_inputs.workload(w["init"], w["n"], w["seed"])
    a = start(w, x0)
    rbm.rbm_run(a, 21)
    rbm.rbm_check(a)
    xa, sa = state(a)
    del a
    monkeypatch.setenv("RBM_FUSE", "0")
    b = start(w, x0)
    monkeypatch.delenv("RBM_FUSE")
    rbm.rbm_run(b, 21)
    rbm.rbm_check(b)
    xb, sb = state(b)
    assert np.array_equal(sa, sb)
    assert np.array_equal(xa.view(np.uint32), xb.view(np.uint32))


def test_fused_calls_resume_bitwise():
    """Ten steps in one call equal four then six in two calls (each call
    starts from and leaves the state in slot order)."""
    w = rbm_inputs.params_of("attrep3d-n2^24-p8", n=300007, p=7)
    x0 = rbm_inputs.workload(w["init"], w["n"], w["seed"])
    a = start(w, x0)
    rbm.rbm_run(a, 10)
    xa, sa = state(a)
    del a
    b = start(w, x0)
    rbm.rbm_run(b, 4)
    rbm.rbm_run(b, 6)
    rbm.rbm_check(b)
    xb, sb = state(b)
    assert rbm.rbm_step_index(b) == 10
    assert np.array_equal(sa, sb)
    assert np.array_equal(xa.view(np.uint32), xb.view(np.uint32))


def test_forces_after_a_fused_run_match_the_oracle():
    """rbm_forces on the state a fused run leaves (slot order, pending noise
    added by the force path) against the oracle's forces for the same
    division."""
    w = rbm_inputs.params_of("attrep3d-n2^24-p8", n=300007)
    x0 = rbm_inputs.workload(w["init"], w["n"], w["seed"])
    ctx = start(w, x0)
    rbm.rbm_run(ctx, 5)
    rbm.rbm_check(ctx)
    x, s = state(ctx)
    f = rbm.rbm_forces(ctx, 5).cpu().numpy()
    o = ora.Params(d=w["d"], kernel=w["kernel"], kparam=w["kparam"], beta=w["beta"],
                   sigma=w["sigma"], dt=w["dt"], seed=w["seed"])
    perm = ora.permutation(o, 5, s)
    fo = ora.rbm_forces(o, w["p"], x.astype(np.float64), perm)
    assert ora.rel_max_error(f, fo) <= 1e-5
