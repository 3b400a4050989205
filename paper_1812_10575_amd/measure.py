"""Measurement helpers of the RBM runs (host side, FP64 numpy).

They judge results the way the paper does, on positions downloaded from the
GPU:

* the error measure of Sec. 4.1, the root mean square over particles of the
  distance to a reference solution (`rms_error`);
* the empirical measure of eq. (1.5) against a closed-form law by the
  Kolmogorov-Smirnov distance (`ks_distance`): the semicircle law of the
  Dyson Brownian motion (Sec. 4.2, `semicircle_cdf`, with the radius of the
  analytic transient `dyson_radius`) and the inverse Gamma equilibrium of the
  wealth model (Sec. 5, `inverse_gamma_cdf`);
* the second moment m2 = mean |x|^2 (`second_moment`), whose relaxation and
  fixed point the Sec. 4.2 runs are checked by;
* the force error on a subset is summed on the GPU (`rbm_force_sqerr` of the
  library); `lemma_3_1_mse` is the variance Lemma 3.1 predicts for it.
"""
from __future__ import annotations

import math

import numpy as np


def _f64(a) -> np.ndarray:
    return np.asarray(a, dtype=np.float64)


def ks_distance(samples, cdf) -> float:
    """sup_x |F_N(x) - F(x)| for the empirical CDF F_N of the samples and a
    continuous CDF F (vectorised callable).  The supremum is reached at a
    sample, just before or at the jump of F_N there: with the samples sorted,
    D = max_k max(k/N - F(x_k), F(x_k) - (k-1)/N), k = 1..N."""
    x = np.sort(_f64(samples).reshape(-1))
    n = x.size
    if n == 0:
        raise ValueError("no samples")
    f = _f64(cdf(x))
    upper = np.arange(1, n + 1, dtype=np.float64) / n - f
    lower = f - np.arange(0, n, dtype=np.float64) / n
    return float(max(upper.max(), lower.max()))


def semicircle_cdf(x, radius: float = math.sqrt(2.0)):
    """CDF of Wigner's semicircle law of radius R, density
    2 sqrt(R^2 - x^2) / (pi R^2) on [-R, R]:
    F(x) = 1/2 + (x sqrt(R^2 - x^2) / R^2 + asin(x / R)) / pi.
    R = sqrt(2) is the equilibrium of the Dyson Brownian motion of Sec. 4.2."""
    R = float(radius)
    if not R > 0:
        raise ValueError("radius must be > 0")
    t = np.clip(_f64(x) / R, -1.0, 1.0)
    return 0.5 + (t * np.sqrt(1.0 - t * t) + np.arcsin(t)) / math.pi


def dyson_radius(t: float, s0: float = 2.0) -> float:
    """Radius of the analytic density of Sec. 4.2 at time t,
    rho(x, t) = sqrt(2 s(t) - x^2) / (s(t) pi) with s(t) = 1 + (s0 - 1) e^{-2t}
    (s0 = 2 for the start from the radius-2 semicircle): R = sqrt(2 s(t))."""
    s = 1.0 + (s0 - 1.0) * math.exp(-2.0 * t)
    return math.sqrt(2.0 * s)


def inverse_gamma_cdf(y, shape: float, scale: float):
    """CDF of the inverse Gamma law with density
    scale^shape / Gamma(shape) y^-(shape+1) exp(-scale / y), y > 0:
    F(y) = Q(shape, scale / y), Q the regularised upper incomplete Gamma
    function (0 for y <= 0).  The equilibrium of the wealth model of Sec. 5
    has shape kappa/D + 1 and scale kappa eta / D."""
    from scipy.special import gammaincc
    y = _f64(y)
    out = np.zeros(y.shape, dtype=np.float64)
    pos = y > 0.0
    out[pos] = gammaincc(float(shape), float(scale) / y[pos])
    return out


def second_moment(x) -> float:
    """m2 = (1/N) sum_i |x_i|^2 (rows are particles)."""
    a = _f64(x)
    a = a.reshape(a.shape[0], -1)
    return float(np.einsum("ij,ij->", a, a) / a.shape[0])


def rms_error(x, ref) -> float:
    """The error measure of Sec. 4.1: sqrt((1/N) sum_i |x_i - ref_i|^2)."""
    a, b = _f64(x), _f64(ref)
    if a.shape != b.shape:
        raise ValueError(f"shapes differ: {a.shape} vs {b.shape}")
    e = (a - b).reshape(a.shape[0], -1)
    return float(math.sqrt(np.einsum("ij,ij->", e, e) / a.shape[0]))


def lemma_3_1_mse(p: int, n: int, lam) -> float:
    """Mean over particles of the variance Lemma 3.1 gives for the RBM-1
    batch force, (1/(p-1) - 1/(N-1)) Lambda_i, with Lambda_i the variance of
    K(X_i - X_j) over the other particles j."""
    if not (2 <= p <= n):
        raise ValueError("need 2 <= p <= N")
    return float((1.0 / (p - 1) - 1.0 / (n - 1)) * np.mean(_f64(lam)))


def loglog_slope(h, err) -> float:
    """Least-squares slope of log(err) against log(h) (the convergence order
    read off the error plots of Sec. 4.1)."""
    lh, le = np.log(_f64(h)), np.log(_f64(err))
    lh = lh - lh.mean()
    return float(np.dot(lh, le - le.mean()) / np.dot(lh, lh))
