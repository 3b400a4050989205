"""Seeded synthetic inputs for the RBM-1 workloads.

This module holds no arithmetic of the method: it only draws initial
particle positions and ensemble sizes.  Both the GPU path's tests and the
oracle receive what it returns, so neither side generates its own inputs.
The draws use numpy's Philox bit generator (a 4x64 counter-based generator,
unrelated to the Philox4x32-10 streams the method itself draws from).

Workload shapes (particles are i.i.d., as the paper assumes for the initial
data of eq. (1.2)):
  gauss2d     d=2, X0 ~ N(0, I)              (Gaussian-attraction workload)
  dyson1d     d=1, X0 ~ U[-3, 3]             (1-D softened-Coulomb workload)
  attrep3d    d=3, X0 ~ N(0, I)              (3-D attraction-repulsion)
  semicircle  d=1, X0 ~ sqrt(4 - x^2)/(2 pi) (the initial law of Sec. 4.1)
  absnormal   d=1, X0 ~ |N(0, 1)|            (initial wealth, Sec. 5)
  hamilton1d  d=2 records (x, v): x semicircle as above, v ~ N(0, 1)
              (the second-order example of Sec. 4.1)
"""
from __future__ import annotations

import numpy as np


def _gen(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(int(seed)))


def normal(n: int, d: int, seed: int = 1) -> np.ndarray:
    """N x d float32 array of i.i.d. standard normals."""
    return _gen(seed).standard_normal((n, d), dtype=np.float32)


def uniform(n: int, d: int, lo: float, hi: float, seed: int = 1) -> np.ndarray:
    """N x d float32 array of i.i.d. U[lo, hi]."""
    u = _gen(seed).random((n, d), dtype=np.float64)
    return (lo + (hi - lo) * u).astype(np.float32)


def semicircle(n: int, radius: float = 2.0, seed: int = 1) -> np.ndarray:
    """N x 1 float32 draws from the semicircle density of the given radius
    (the x-coordinate of a uniform point in the disc of that radius)."""
    g = _gen(seed)
    r = radius * np.sqrt(g.random(n))
    th = 2.0 * np.pi * g.random(n)
    return (r * np.cos(th)).astype(np.float32).reshape(n, 1)


def hamilton(n: int, seed: int = 1) -> np.ndarray:
    """N x 2 float32 records (x, v) of the second-order example of Sec. 4.1:
    x from the radius-2 semicircle, v ~ N(0, 1), independent."""
    return np.concatenate([semicircle(n, 2.0, seed), normal(n, 1, seed + 1)], axis=1)


def ensemble_sizes(s: int, nmin: int = 64, nmax: int = 65536, seed: int = 1) -> np.ndarray:
    """S system sizes, log-uniform on [nmin, nmax] (int64)."""
    u = _gen(seed).random(s)
    n = np.floor(nmin * (nmax / nmin) ** u).astype(np.int64)
    return np.clip(n, nmin, nmax)


def workload(name: str, n: int, seed: int = 1) -> np.ndarray:
    if name == "gauss2d":
        return normal(n, 2, seed)
    if name == "dyson1d":
        return uniform(n, 1, -3.0, 3.0, seed)
    if name == "attrep3d":
        return normal(n, 3, seed)
    if name == "semicircle":
        return semicircle(n, 2.0, seed)
    if name == "semicircle2":  # radius 2: the analytic density of Sec. 4.2 at t = 0
        return semicircle(n, 2.0, seed)
    if name == "absnormal":  # initial wealth |N(0, 1)| (Sec. 5)
        return np.abs(normal(n, 1, seed))
    if name == "hamilton1d":  # (x, v): semicircle positions, normal velocities (Sec. 4.1)
        return hamilton(n, seed)
    raise ValueError(f"unknown workload {name!r}")


# Named workloads: model/method parameters and the initial law.  Kernel
# codes: 0 Gaussian attraction -x exp(-|x|^2), 1 softened Coulomb
# x/(|x|^2 + a), 2 attraction-repulsion x/(|x|^2 + a) - x.
WORKLOADS = {
    # 2-D Gaussian attraction in a harmonic trap, with noise
    "gauss2d-n1024-p2": dict(d=2, kernel=0, n=1024, p=2, kparam=0.0, beta=1.0, sigma=0.5,
                             dt=1e-3, seed=1, init="gauss2d", steps=1000),
    # 1-D softened Coulomb (eps = 1e-3) in a harmonic trap, no noise
    "dyson1d-n2^20-p2": dict(d=1, kernel=1, n=1 << 20, p=2, kparam=1e-6, beta=1.0, sigma=0.0,
                             dt=1e-4, seed=1, init="dyson1d", steps=100000),
    # 1-D Dyson Brownian motion (K = 1/x, V = x^2/2, sigma = 1/sqrt(N)) by the
    # splitting with the exact pair flow, from the radius-2 semicircle
    "dysonsplit1d-n2^20-p2": dict(d=1, kernel=3, n=1 << 20, p=2, kparam=0.0, beta=1.0,
                                  sigma=1.0 / 1024.0, dt=1e-3, seed=1, init="semicircle2", steps=5000),
    # the same Dyson Brownian motion by RBM-r: one random pair per iteration,
    # N/2 iterations per unit dt ("steps" counts such windows)
    "dysonrbmr1d-n2^20-p2": dict(d=1, kernel=3, n=1 << 20, p=2, kparam=0.0, beta=1.0,
                                 sigma=1.0 / 1024.0, dt=1e-3, seed=1, init="semicircle2", steps=5000),
    # wealth model of Sec. 5: kappa = D = 1 (sigma = sqrt 2), quadratic trading,
    # pair flow and exact multiplicative noise, wealth started at |N(0, 1)|
    "wealth1d-n2^20-p2": dict(d=1, kernel=4, n=1 << 20, p=2, kparam=1.0, beta=0.0, sigma=2.0 ** 0.5,
                              dt=1e-3, seed=1, init="absnormal", steps=3000),
    # second-order (Hamiltonian) system of Sec. 4.1: x'' = F with
    # K = x/(1 + x^2), Verlet, T = 1; records (x, u)
    "hamilton1d-n2^20-p2": dict(d=2, kernel=5, n=1 << 20, p=2, kparam=1.0, beta=0.0, sigma=0.0,
                                dt=2.0 ** -7, seed=1, init="hamilton1d", steps=128),
    # the Gaussian workload at 2^22 particles (control-variate comparison)
    "gauss2d-n2^22-p2": dict(d=2, kernel=0, n=1 << 22, p=2, kparam=0.0, beta=1.0, sigma=0.5,
                             dt=1e-3, seed=1, init="gauss2d", steps=1000),
    # 3-D attraction-repulsion, free space, weak noise
    "attrep3d-n2^24-p8": dict(d=3, kernel=2, n=1 << 24, p=8, kparam=0.01, beta=0.0, sigma=0.1,
                              dt=1e-3, seed=1, init="attrep3d", steps=100),
}


# Ensemble of independent 2-D Gaussian systems (the first workload's kernel,
# trap, noise and step), sizes log-uniform on [64, 65536], Philox key of
# system s = 1 + s, initial positions standard normal.
ENSEMBLE = dict(name="gauss2d-ensemble-4096", d=2, kernel=0, p=4, kparam=0.0, beta=1.0, sigma=0.5,
                dt=1e-3, nsys=4096, nmin=64, nmax=65536, steps=500, seed=5)


def ensemble(nsys: int = ENSEMBLE["nsys"], nmin: int = ENSEMBLE["nmin"], nmax: int = ENSEMBLE["nmax"],
             seed: int = ENSEMBLE["seed"]):
    """(sizes int64 [nsys], keys uint64 [nsys], x0 float32 [sum sizes][2])."""
    n = ensemble_sizes(nsys, nmin, nmax, seed)
    keys = 1 + np.arange(nsys, dtype=np.uint64)
    return n, keys, normal(int(n.sum()), 2, seed + 1)


def params_of(name: str, **over) -> dict:
    """Parameter dict of a named workload, with overrides."""
    w = dict(WORKLOADS[name])
    w.update(over)
    return w
