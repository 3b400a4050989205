"""The Gaussian increments of the GPU step, read off directly (the sigma dB
term of eq. (1.2), generated as in the NOISE stream definition: Philox block
(id, m, 1, sys), 24-bit uniforms, Box-Muller).

Runs whose drift is exactly zero and whose noise amplitude sigma sqrt(dt) is
exactly 1 (sigma = 32, dt = 2^-10) make the position change of a step the
normal z(id, m) itself:

  * all particles at the origin: K(0) = 0 for every kernel and V = 0, so a
    step from there moves particle id by z(id, m) exactly (one FP32 multiply
    by 1 and add to 0);
  * K(x) = x / (|x|^2 + a) with a = 1e30: the pair force is below 1e-29 and
    dt F is absorbed by the positions' rounding, so several steps in a row
    add z(id, m), z(id, m + 1), ... (through every reader of the deferred
    noise: the coarse scatter, the split after a fused sort, the
    one-workgroup kernel and rbm_positions);
  * the wealth model (Sec. 5) with every Y = 1: the pair flow keeps 1 and
    the step multiplies by exp(sigma sqrt(dt) z - sigma^2 dt / 2) = e^{z - 1/2}.

The GPU uses the hardware log2, sine and cosine; the bound below is on the
absolute error of z against the oracle's FP64 normals.
"""
import math

import numpy as np
import pytest

import oracle as ora

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_1812_10575_amd as rbm  # noqa: E402

SIGMA, DT = 32.0, 2.0 ** -10  # sigma sqrt(dt) = 1 exactly
Z_TOL = 2e-6


def say(*a):
    print(*a, flush=True)


def normals(seed, sys, m, n, d):
    return np.array([ora.normals(seed, sys, m, i)[:d] for i in range(n)])


@pytest.mark.parametrize("d,n,p", [(1, 1000, 2), (2, 65539, 3), (3, 100003, 8), (3, 2816, 4)])
@pytest.mark.parametrize("m", [0, 7, 1234567])
def test_one_step_from_the_origin_is_the_normal(d, n, p, m):
    prm = rbm.Params(d=d, kernel=rbm.RBM_K_GAUSS, n=n, p=p, kparam=0.0, beta=0.0, sigma=SIGMA, dt=DT,
                     seed=3, sys=1)
    say("noise from origin", d, n, p, m)
    ctx = rbm.rbm_init(prm, torch.zeros((n, d), dtype=torch.float32, device="cuda"), step0=m)
    rbm.rbm_run(ctx, 1)
    z = rbm.rbm_positions(ctx).cpu().numpy().astype(np.float64)
    rbm.rbm_check(ctx)
    zo = normals(3, 1, m, n, d)
    err = np.abs(z - zo)
    say("max |z_gpu - z|", err.max(), "rms", math.sqrt(np.mean(err ** 2)))
    assert err.max() <= Z_TOL


@pytest.mark.parametrize("d,n,p", [(1, 2000, 2), (2, 70001, 4), (3, 1 << 18, 8)])
def test_consecutive_steps_add_the_normals(d, n, p):
    """Four steps of one rbm_run call (the fused path above the one-workgroup
    size: the split adds the noise of the previous step), and four one-step
    calls (the coarse scatter adds it), with rbm_positions adding the last."""
    prm = rbm.Params(d=d, kernel=rbm.RBM_K_SOFTCOULOMB, n=n, p=p, kparam=1e30, beta=0.0, sigma=SIGMA, dt=DT,
                     seed=5, sys=0)
    m0 = 11
    zs = [normals(5, 0, m0 + k, n, d) for k in range(4)]
    x0 = torch.zeros((n, d), dtype=torch.float32, device="cuda")
    # one call of four steps
    say("noise run of 4", d, n, p)
    ctx = rbm.rbm_init(prm, x0, step0=m0)
    rbm.rbm_run(ctx, 4)
    x4 = rbm.rbm_positions(ctx).cpu().numpy().astype(np.float64)
    rbm.rbm_check(ctx)
    ref = zs[0] + zs[1] + zs[2] + zs[3]
    # four z errors plus four FP32 roundings of sums below 24 in magnitude
    assert np.abs(x4 - ref).max() <= 4 * Z_TOL + 4 * 2.0 ** -20
    # four calls of one step: each step's change is its normal
    ctx = rbm.rbm_init(prm, x0, step0=m0)
    prev = np.zeros((n, d))
    for k in range(4):
        rbm.rbm_run(ctx, 1)
        cur = rbm.rbm_positions(ctx).cpu().numpy().astype(np.float64)
        dz = np.abs((cur - prev) - zs[k])
        tol = Z_TOL + np.spacing(np.maximum(np.abs(cur), np.abs(prev)).astype(np.float32)).astype(np.float64)
        say("step", k, "max |dx - z|", dz.max())
        assert np.all(dz <= tol)
        prev = cur
    rbm.rbm_check(ctx)
    assert np.array_equal(prev.astype(np.float32), x4.astype(np.float32))


@pytest.mark.parametrize("m", [0, 3, 99991])
def test_wealth_factor_is_the_exact_lognormal(m):
    n = 50000
    prm = rbm.Params(d=1, kernel=rbm.RBM_K_WEALTH_SPLIT, n=n, p=2, kparam=1.0, beta=0.0, sigma=SIGMA, dt=DT,
                     seed=9, sys=2)
    say("wealth factor", m)
    ctx = rbm.rbm_init(prm, torch.ones((n, 1), dtype=torch.float32, device="cuda"), step0=m)
    rbm.rbm_run(ctx, 1)
    y = rbm.rbm_positions(ctx).cpu().numpy().astype(np.float64)[:, 0]
    rbm.rbm_check(ctx)
    zo = normals(9, 2, m, n, 1)[:, 0]
    assert np.all(y > 0)
    # Y = exp(z - 1/2): z = log Y + 1/2 (the FP32 rounding of Y adds 2^-24
    # relative, i.e. 6e-8 to log Y)
    err = np.abs(np.log(y) + 0.5 - zo)
    say("max |log Y + 1/2 - z|", err.max())
    assert err.max() <= Z_TOL + 1e-7
