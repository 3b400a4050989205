"""FP64 CPU oracle for one RBM-1 step (arXiv:1812.10575, Sec. 2.1, Algorithm 1).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product path
(``paper_1812_10575_amd``) never imports it, and the two share no code.

The arithmetic lives in ``rbm_oracle.c`` (plain C, FP64, no fast-math); this
module only marshals numpy arrays through ctypes and adds the statistics the
paper uses to judge results (Sec. 4: the error measure of Sec. 4.1 and the
semicircle law of Sec. 4.2).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_SANITIZED=1: the ASan/UBSan build (see build.py; needs the sanitizer
# runtime preloaded)
_SANITIZED = os.environ.get("ORACLE_SANITIZED", "") == "1"
_LIB_PATH = os.path.join(_HERE, "liboracle_san.so" if _SANITIZED else "liboracle.so")
_lib = None

K_GAUSS, K_SOFTCOULOMB, K_ATTREP, K_COULOMB_SPLIT, K_WEALTH_SPLIT, K_HAMILTON = 0, 1, 2, 3, 4, 5


class _Params(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("kparam", ctypes.c_double), ("beta", ctypes.c_double),
                ("sigma", ctypes.c_double), ("dt", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("sys", ctypes.c_uint32)]


@dataclass
class Params:
    """Model and stream parameters of eq. (1.2) with V = beta |x|^2 / 2."""
    d: int
    kernel: int
    kparam: float
    beta: float
    sigma: float
    dt: float
    seed: int = 1
    sys: int = 0

    def c(self) -> _Params:
        if self.kernel == K_HAMILTON and (self.d != 2 or self.sigma != 0.0):
            raise ValueError("the Hamiltonian system has records (x, u) (d = 2) and no noise (sigma = 0)")
        return _Params(self.d, self.kernel, self.kparam, self.beta, self.sigma,
                       self.dt, self.seed, self.sys)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b  # noqa: WPS433 (build on first use)
        _b.build(sanitize=_SANITIZED)
    lib = ctypes.CDLL(_LIB_PATH)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    f64p = ctypes.POINTER(ctypes.c_double)
    pp = ctypes.POINTER(_Params)
    lib.ora_philox4x32_10.argtypes = [u32p, u32p, u32p]
    lib.ora_set_threads.argtypes = [ctypes.c_int32]
    lib.ora_get_threads.restype = ctypes.c_int32
    lib.ora_uniform.argtypes = [ctypes.c_uint32]
    lib.ora_uniform.restype = ctypes.c_double
    lib.ora_perm_word.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]
    lib.ora_perm_word.restype = ctypes.c_uint32
    lib.ora_normals.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, f64p]
    lib.ora_pair_kernel.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, f64p, f64p]
    lib.ora_permutation.argtypes = [pp, ctypes.c_int64, ctypes.c_uint32, u32p, u32p]
    lib.ora_batch_of.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int64,
                                 ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    lib.ora_rbm_forces.argtypes = [pp, ctypes.c_int64, ctypes.c_int32, f64p, u32p, f64p]
    lib.ora_direct_forces.argtypes = [pp, ctypes.c_int64, f64p, u32p, ctypes.c_int64, f64p]
    lib.ora_direct_moments.argtypes = [pp, ctypes.c_int64, f64p, u32p, ctypes.c_int64, f64p, f64p]
    lib.ora_pair_flow.argtypes = [ctypes.c_int32, ctypes.c_double, f64p, f64p, f64p, f64p]
    lib.ora_pair_flow_linear.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, f64p, f64p, f64p,
                                         f64p]
    lib.ora_rbm_step.argtypes = [pp, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, f64p, u32p]
    lib.ora_rbm_run.argtypes = [pp, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32,
                                ctypes.c_int64, f64p, u32p]
    lib.ora_direct_step.argtypes = [pp, ctypes.c_int64, ctypes.c_uint32, f64p]
    lib.ora_rbmr_members.argtypes = [pp, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, u32p]
    lib.ora_rbmr_apply.argtypes = [pp, ctypes.c_int32, ctypes.c_uint64, u32p, f64p]
    lib.ora_rbmr_run.argtypes = [pp, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64, f64p]
    _lib = lib
    return lib


def set_threads(n: int) -> int:
    """Threads of the oracle's parallel loops (results do not depend on it);
    returns the count now in use."""
    lib = _load()
    lib.ora_set_threads(int(n))
    return int(lib.ora_get_threads())


def get_threads() -> int:
    return int(_load().ora_get_threads())


def _u32(a):
    return np.ascontiguousarray(a, dtype=np.uint32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


# --------------------------------------------------------------------------
# random streams
# --------------------------------------------------------------------------

def philox4x32_10(ctr, key) -> np.ndarray:
    """One Philox4x32-10 block (Salmon et al., SC'11)."""
    lib = _load()
    c, k, o = _u32(ctr), _u32(key), np.zeros(4, np.uint32)
    assert c.size == 4 and k.size == 2
    lib.ora_philox4x32_10(_p(c, ctypes.c_uint32), _p(k, ctypes.c_uint32), _p(o, ctypes.c_uint32))
    return o


def uniform(w: int) -> float:
    return _load().ora_uniform(int(w) & 0xFFFFFFFF)


def perm_word(seed: int, sys: int, m: int, slot: int) -> int:
    return int(_load().ora_perm_word(seed, sys, m, slot))


def normals(seed: int, sys: int, m: int, pid: int) -> np.ndarray:
    z = np.zeros(4, np.float64)
    _load().ora_normals(seed, sys, m, pid, _p(z, ctypes.c_double))
    return z


def pair_kernel(kernel: int, d: int, a: float, x) -> np.ndarray:
    xv = _f64(x)
    assert xv.size == d
    o = np.zeros(d, np.float64)
    _load().ora_pair_kernel(kernel, d, a, _p(xv, ctypes.c_double), _p(o, ctypes.c_double))
    return o


# --------------------------------------------------------------------------
# the RBM-1 step
# --------------------------------------------------------------------------

def permutation(prm: Params, m: int, slots) -> np.ndarray:
    """Division of step m (Sec. 2.1): ids in ascending key order."""
    s = _u32(slots)
    out = np.zeros_like(s)
    _load().ora_permutation(ctypes.byref(prm.c()), s.size, m, _p(s, ctypes.c_uint32),
                            _p(out, ctypes.c_uint32))
    return out


def batch_of(n: int, p: int, r: int):
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _load().ora_batch_of(n, p, r, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def rbm_forces(prm: Params, p: int, x, perm) -> np.ndarray:
    """Batch forces of eq. (2.3) for the division perm; x is N x d by id."""
    xv, pv = _f64(x), _u32(perm)
    n = pv.size
    f = np.zeros((n, prm.d), np.float64)
    _load().ora_rbm_forces(ctypes.byref(prm.c()), n, p, _p(xv, ctypes.c_double),
                           _p(pv, ctypes.c_uint32), _p(f, ctypes.c_double))
    return f


def direct_forces(prm: Params, x, ids=None) -> np.ndarray:
    """Exact interaction force of eq. (1.2) for the listed ids (all if None)."""
    xv = _f64(x)
    n = xv.shape[0]
    iv = _u32(np.arange(n) if ids is None else ids)
    f = np.zeros((iv.size, prm.d), np.float64)
    _load().ora_direct_forces(ctypes.byref(prm.c()), n, _p(xv, ctypes.c_double),
                              _p(iv, ctypes.c_uint32), iv.size, _p(f, ctypes.c_double))
    return f


def direct_moments(prm: Params, x, ids=None):
    """(F, m2): the exact force of eq. (1.2) and m2_i = 1/(N-1) sum_{j != i}
    |K(X_i - X_j)|^2, so that Lambda_i of Lemma 3.1 is
    (N-1)/(N-2) (m2_i - |F_i|^2)."""
    xv = _f64(x)
    n = xv.shape[0]
    iv = _u32(np.arange(n) if ids is None else ids)
    f = np.zeros((iv.size, prm.d), np.float64)
    m2 = np.zeros(iv.size, np.float64)
    _load().ora_direct_moments(ctypes.byref(prm.c()), n, _p(xv, ctypes.c_double), _p(iv, ctypes.c_uint32),
                               iv.size, _p(f, ctypes.c_double), _p(m2, ctypes.c_double))
    return f, m2


def rbm_step(prm: Params, p: int, m: int, x, slots):
    """One RBM-1 step (Algorithm 1).  Returns (x_new, slots_new)."""
    xv = _f64(x).copy()
    sv = _u32(slots).copy()
    _load().ora_rbm_step(ctypes.byref(prm.c()), sv.size, p, m, _p(xv, ctypes.c_double),
                         _p(sv, ctypes.c_uint32))
    return xv, sv


def rbm_run(prm: Params, p: int, m0: int, nsteps: int, x, slots=None):
    """nsteps RBM-1 steps from step index m0.  Returns (x, slots)."""
    xv = _f64(x).copy()
    n = xv.shape[0]
    sv = _u32(np.arange(n) if slots is None else slots).copy()
    _load().ora_rbm_run(ctypes.byref(prm.c()), n, p, m0, nsteps, _p(xv, ctypes.c_double),
                        _p(sv, ctypes.c_uint32))
    return xv, sv


def direct_step(prm: Params, m: int, x) -> np.ndarray:
    """One step of the fully coupled system, same update and noise as RBM-1."""
    xv = _f64(x).copy()
    _load().ora_direct_step(ctypes.byref(prm.c()), xv.shape[0], m, _p(xv, ctypes.c_double))
    return xv


# --------------------------------------------------------------------------
# RBM-r (Sec. 2.2): one random batch per iteration, drawn with replacement
# --------------------------------------------------------------------------

def _rbmr_check(prm: Params, n: int, p: int):
    if prm.kernel not in (K_GAUSS, K_SOFTCOULOMB, K_ATTREP, K_COULOMB_SPLIT):
        raise ValueError("RBM-r takes the Euler kernels and the split Coulomb kernel")
    if not 2 <= p <= min(n, 64) or (prm.kernel == K_COULOMB_SPLIT and p != 2):
        raise ValueError("p must be in 2..min(N, 64) (2 for the split Coulomb kernel)")


def rbmr_members(prm: Params, n: int, p: int, k: int) -> np.ndarray:
    """Members m_0 .. m_{p-1} of RBM-r iteration k (uint32, draw order)."""
    _rbmr_check(prm, n, p)
    out = np.zeros(p, np.uint32)
    _load().ora_rbmr_members(ctypes.byref(prm.c()), n, p, k, _p(out, ctypes.c_uint32))
    return out


def rbmr_apply(prm: Params, p: int, k: int, members, x) -> np.ndarray:
    """Iteration k of RBM-r on the given members (p distinct ids)."""
    xv = _f64(x).copy()
    mv = _u32(members).copy()
    _rbmr_check(prm, xv.shape[0], p)
    assert mv.size == p and len(set(mv.tolist())) == p and int(mv.max()) < xv.shape[0]
    _load().ora_rbmr_apply(ctypes.byref(prm.c()), p, k, _p(mv, ctypes.c_uint32), _p(xv, ctypes.c_double))
    return xv


def rbmr_run(prm: Params, p: int, k0: int, niter: int, x) -> np.ndarray:
    """niter RBM-r iterations k0, k0+1, ... in sequence."""
    xv = _f64(x).copy()
    _rbmr_check(prm, xv.shape[0], p)
    _load().ora_rbmr_run(ctypes.byref(prm.c()), xv.shape[0], p, k0, niter, _p(xv, ctypes.c_double))
    return xv


# --------------------------------------------------------------------------
# diagnostics
# --------------------------------------------------------------------------

def pair_flow(d: int, t: float, xi, xj):
    """Exact flow over time t of a batch of two particles under
    K(x) = x/|x|^2 (Sec. 2.3 splitting, Sec. 4.2): returns (yi, yj)."""
    a, b = _f64(xi).copy(), _f64(xj).copy()
    yi, yj = np.zeros(d), np.zeros(d)
    _load().ora_pair_flow(d, t, _p(a, ctypes.c_double), _p(b, ctypes.c_double), _p(yi, ctypes.c_double),
                          _p(yj, ctypes.c_double))
    return yi, yj


def pair_flow_linear(d: int, t: float, kappa: float, xi, xj):
    """Exact flow over time t of a pair under K(x) = -kappa x (Sec. 5):
    returns (yi, yj)."""
    a, b = _f64(xi).copy(), _f64(xj).copy()
    yi, yj = np.zeros(d), np.zeros(d)
    _load().ora_pair_flow_linear(d, t, kappa, _p(a, ctypes.c_double), _p(b, ctypes.c_double),
                                 _p(yi, ctypes.c_double), _p(yj, ctypes.c_double))
    return yi, yj


def inverse_gamma_cdf(y, shape, scale):
    """CDF of the inverse Gamma law rho(y) = scale^shape / Gamma(shape)
    y^-(shape+1) e^(-scale/y), y > 0: the equilibrium of the wealth model of
    Sec. 5 has shape kappa/D + 1 and scale kappa eta / D (eta the mean
    wealth)."""
    from scipy.special import gammaincc
    y = np.asarray(y, np.float64)
    out = np.zeros_like(y)
    pos = y > 0
    out[pos] = gammaincc(shape, scale / y[pos])
    return out


def semicircle_cdf_r(x, radius):
    """CDF of the semicircle law of the given radius R,
    rho(x) = 2 sqrt(R^2 - x^2) / (pi R^2); R^2 = 2 sigma(t) gives the
    analytic density of Sec. 4.2, rho(x, t) = sqrt(2 sigma(t) - x^2) /
    (sigma(t) pi), sigma(t) = 1 + e^{-2t}."""
    R = float(radius)
    x = np.clip(np.asarray(x, np.float64), -R, R)
    r = np.sqrt(np.maximum(R * R - x * x, 0.0))
    return 0.5 + x * r / (math.pi * R * R) + np.arcsin(np.clip(x / R, -1.0, 1.0)) / math.pi


def semicircle_cdf(x):
    """CDF of the semicircle law rho(x) = sqrt(2 - x^2) / pi (Sec. 4.2)."""
    x = np.clip(np.asarray(x, np.float64), -math.sqrt(2.0), math.sqrt(2.0))
    r = np.sqrt(np.maximum(2.0 - x * x, 0.0))
    return 0.5 + x * r / (2.0 * math.pi) + np.arcsin(np.clip(x / math.sqrt(2.0), -1.0, 1.0)) / math.pi


def ks_distance(samples, cdf) -> float:
    """Kolmogorov-Smirnov distance between the empirical measure of the
    samples (the empirical measure of eq. (1.5)) and a closed-form CDF."""
    xs = np.sort(np.asarray(samples, np.float64).ravel())
    n = xs.size
    f = cdf(xs)
    k = np.arange(1, n + 1, dtype=np.float64)
    return float(max(np.max(k / n - f), np.max(f - (k - 1) / n)))


def rms_error(x, y) -> float:
    """The error measure of Sec. 4.1: sqrt(mean_i |x_i - y_i|^2)."""
    dx = np.asarray(x, np.float64) - np.asarray(y, np.float64)
    return float(math.sqrt(np.mean(np.sum(dx.reshape(dx.shape[0], -1) ** 2, axis=1))))


def rel_max_error(x, ref) -> float:
    """max_i |x_i - ref_i|_inf / max(1, max_i |ref_i|_inf)."""
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.max(np.abs(x - ref)) / max(1.0, float(np.max(np.abs(ref)))))
