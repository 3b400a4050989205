"""rbmr_run_noalloc (RBM-r with the library's static per-GPU workspace)
against rbmr_run with a caller workspace, through the C ABI.

The two run the same kernels on the same inputs, so the results must be the
same bits.  Two calls in a row on the one static buffer, the second with a
smaller system, check that nothing of the first call's buffer contents leaks
into the second.
"""
import math

import numpy as np
import pytest

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


def both(w, init, k0, niter):
    x0 = rbm_inputs.workload(init, w["n"], w["seed"])
    xa = torch.from_numpy(np.ascontiguousarray(x0, dtype=np.float32)).cuda()
    xb = xa.clone()
    rbm.rbmr_run(gp(w), xa, k0, niter)
    torch.cuda.synchronize()
    before = torch.cuda.memory_stats().get("allocation.all.allocated", 0)
    rbm.rbmr_run_noalloc(gp(w), xb, k0, niter)
    after = torch.cuda.memory_stats().get("allocation.all.allocated", 0)
    torch.cuda.synchronize()
    assert after == before, "the no-allocation call allocated through torch"
    return xa.cpu().numpy(), xb.cpu().numpy()


def test_noalloc_equals_rbmr_run_on_two_calls():
    # first call: the largest system of the tests, 1-D Dyson at N = 2^20
    # (20 MiB of the 64 MiB buffer)
    w1 = rbm_inputs.params_of("dysonrbmr1d-n2^20-p2")
    need1 = rbm.rbmr_workspace_size(gp(w1))
    assert need1 <= rbm.NOALLOC_SCRATCH_BYTES
    niter1 = 2 * (w1["n"] // w1["p"])
    say("noalloc call 1", w1["n"], w1["d"], niter1)
    a1, b1 = both(w1, "semicircle2", 3, niter1)
    assert np.isfinite(a1).all()
    assert np.array_equal(a1, b1), f"call 1 differs: max {np.max(np.abs(a1 - b1))}"
    # second call: a smaller 2-D system right after, on the same buffer
    w2 = rbm_inputs.params_of("gauss2d-n1024-p2", n=4097, p=3)
    niter2 = 5 * (w2["n"] // w2["p"])
    say("noalloc call 2", w2["n"], w2["d"], niter2)
    a2, b2 = both(w2, "gauss2d", 11, niter2)
    assert np.isfinite(a2).all()
    assert np.array_equal(a2, b2), f"call 2 differs: max {np.max(np.abs(a2 - b2))}"


def test_noalloc_three_dimensions_and_window():
    w = rbm_inputs.params_of("attrep3d-n2^24-p8", n=20001, p=4)
    niter = 3 * (w["n"] // w["p"])
    say("noalloc d=3", w["n"], niter)
    x0 = rbm_inputs.workload("attrep3d", w["n"], w["seed"])
    xa = torch.from_numpy(x0).cuda()
    xb = xa.clone()
    rbm.rbmr_run(gp(w), xa, 0, niter, window=777, rounds=3)
    rbm.rbmr_run_noalloc(gp(w), xb, 0, niter, window=777, rounds=3)
    torch.cuda.synchronize()
    assert np.array_equal(xa.cpu().numpy(), xb.cpu().numpy())


def test_noalloc_rejects_a_run_above_the_buffer():
    # 1-D, N = 2^22, p = 2 needs about 16 N + 16 N + 8 N/2 bytes = 144 MiB > 64 MiB
    w = rbm_inputs.params_of("dysonrbmr1d-n2^20-p2", n=1 << 22, sigma=1.0 / math.sqrt(1 << 22))
    assert rbm.rbmr_workspace_size(gp(w)) > rbm.NOALLOC_SCRATCH_BYTES
    x = torch.zeros((w["n"], 1), dtype=torch.float32, device="cuda")
    with pytest.raises(rbm.RbmError) as ei:
        rbm.rbmr_run_noalloc(gp(w), x, 0, 10)
    assert ei.value.status == rbm.RBM_ERR_WORKSPACE
    assert bool((x == 0).all())
