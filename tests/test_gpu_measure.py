"""The GPU force-error sum rbm_force_sqerr (the force MSE of Lemma 3.1 on a
subset) against an FP64 numpy sum of the same values, through the C ABI."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1812_10575_amd as rbm  # noqa: E402


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("n,nids", [(1, 1), (5000, 1023), (70001, 1025), (70001, 5000), (1 << 20, 65537)])
def test_sqerr_matches_an_fp64_sum(d, n, nids):
    rng = np.random.default_rng(d * 1000 + nids)
    f = rng.standard_normal((n, d)).astype(np.float32) * np.float32(3.0)
    ids = rng.integers(0, n, nids).astype(np.int32)  # repeats allowed
    fref = (f[ids] + rng.standard_normal((nids, d)).astype(np.float32) * np.float32(1e-3)).astype(np.float32)
    fref[::7] = rng.standard_normal((len(fref[::7]), d)).astype(np.float32)
    say("sqerr", d, n, nids)
    out = rbm.rbm_force_sqerr(torch.from_numpy(f).cuda(), torch.from_numpy(ids).cuda(),
                              torch.from_numpy(fref).cuda())
    got = float(out.cpu()[0])
    e = f[ids].astype(np.float64) - fref.astype(np.float64)
    ref = float(np.sum(e * e))
    # both are FP64 sums of the same FP64 terms, in different orders
    assert got == pytest.approx(ref, rel=1e-12, abs=1e-300)


def test_sqerr_empty_and_errors():
    f = torch.ones((10, 2), dtype=torch.float32, device="cuda")
    ids = torch.zeros(0, dtype=torch.int32, device="cuda")
    fref = torch.zeros((0, 2), dtype=torch.float32, device="cuda")
    assert float(rbm.rbm_force_sqerr(f, ids, fref).cpu()[0]) == 0.0
    bad = torch.tensor([3, 10], dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError):
        rbm.rbm_force_sqerr(f, bad, torch.zeros((2, 2), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        rbm.rbm_force_sqerr(f.double(), ids, fref)
    with pytest.raises(ValueError):
        rbm.rbm_force_sqerr(f, ids, torch.zeros((0, 3), dtype=torch.float32, device="cuda"))


def test_sqerr_out_of_range_id_through_the_abi_is_nan():
    """Called through the C ABI without the binding's host check: an id >= n
    is not read and the sum is NaN."""
    f = torch.ones((10, 3), dtype=torch.float32, device="cuda")
    ids = torch.tensor([1, 2, 12, 3], dtype=torch.int32, device="cuda")
    fref = torch.zeros((4, 3), dtype=torch.float32, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = rbm.lib().rbm_force_sqerr(ctypes.c_void_p(f.data_ptr()), 10, ctypes.c_void_p(ids.data_ptr()), 4,
                                   ctypes.c_void_p(fref.data_ptr()), 3, ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == rbm.RBM_OK
    assert np.isnan(float(out.cpu()[0]))
    assert rbm.lib().rbm_force_sqerr(ctypes.c_void_p(f.data_ptr()), 0, ctypes.c_void_p(ids.data_ptr()), 4,
                                     ctypes.c_void_p(fref.data_ptr()), 3, ctypes.c_void_p(out.data_ptr()),
                                     None) == rbm.RBM_ERR_INVALID
