"""Python binding of librbm.so: the RBM-1 step (arXiv:1812.10575, Sec. 2.1,
Algorithm 1) on an AMD Instinct MI355X.

Every function here has the name of a C entry point of ``include/rbm.h`` and
only marshals arguments: torch tensors supply device memory and the current
HIP stream, every step of the method runs in the library's HIP kernels.
There is no fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librbm.so")

RBM_OK, RBM_ERR_INVALID, RBM_ERR_WORKSPACE, RBM_ERR_HIP, RBM_ERR_UNSUPPORTED, RBM_ERR_DEVICE = range(6)
RBM_MAX_N = 1 << 25
RBM_MAX_P_MULTI = 64

# every symbol the header declares
SYMBOLS = (
    "rbm_workspace_size", "rbm_init", "rbm_step", "rbm_run", "rbm_positions", "rbm_perm",
    "rbm_forces", "rbm_step_index", "rbm_check", "rbm_timing", "rbm_phase_times", "rbm_destroy",
    "direct_forces", "direct_step", "rbm_status_str", "rbm_last_error",
    "cv_init", "cv_set_weights", "cv_get_weights", "cv_features", "cv_grads", "cv_train",
    "rbm_force_sqerr", "ensemble_workspace_size", "ensemble_run", "direct_moments",
    "rbmr_workspace_size", "rbmr_run", "rbmr_run_noalloc",
)
ENS_LDS = 4096
ENS_MAXN = 256 * 1024
CV_NPARAM = 6432
RBMR_MAX_P = 8
RBMR_MAX_WINDOW = 1 << 22
NOALLOC_SCRATCH_BYTES = 64 << 20
RBM_K_GAUSS, RBM_K_SOFTCOULOMB, RBM_K_ATTREP, RBM_K_COULOMB_SPLIT, RBM_K_WEALTH_SPLIT, RBM_K_HAMILTON = range(6)
PHASES = ("keycount", "keysum", "keystarts", "scatter", "split", "sort", "fixup")


class RbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class rbm_params(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("kernel", ctypes.c_int32), ("n", ctypes.c_int64),
                ("p", ctypes.c_int32), ("cv", ctypes.c_int32), ("kparam", ctypes.c_double),
                ("beta", ctypes.c_double), ("sigma", ctypes.c_double), ("dt", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("sys", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class rbm_ensemble(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("kernel", ctypes.c_int32), ("p", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("kparam", ctypes.c_double), ("beta", ctypes.c_double),
                ("sigma", ctypes.c_double), ("dt", ctypes.c_double), ("nsys", ctypes.c_int64)]


class rbm_ensemble_tile(ctypes.Structure):
    _fields_ = [("lds_max", ctypes.c_int32), ("grid", ctypes.c_int32), ("team", ctypes.c_int32),
                ("bucket", ctypes.c_int32), ("wg", ctypes.c_int32)]


_lib = None


def lib():
    """Load librbm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1812_10575_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
    pp = ctypes.POINTER(rbm_params)
    sig = {
        "rbm_workspace_size": [pp, ctypes.POINTER(sz)],
        "rbm_init": [pp, vp, vp, i64, vp, sz, vp, ctypes.POINTER(vp)],
        "rbm_step": [vp, vp],
        "rbm_run": [vp, i64, vp],
        "rbm_positions": [vp, vp, vp],
        "rbm_perm": [vp, vp, vp],
        "rbm_forces": [vp, i64, vp, vp],
        "rbm_step_index": [vp, ctypes.POINTER(i64)],
        "rbm_check": [vp, vp],
        "rbm_timing": [vp, ctypes.c_int32],
        "rbm_phase_times": [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)],
        "rbm_destroy": [vp],
        "direct_forces": [pp, vp, vp, i64, vp, vp],
        "direct_moments": [pp, vp, vp, i64, vp, vp, vp],
        "direct_step": [pp, vp, vp, i64, vp],
        "cv_init": [vp, ctypes.c_uint64, vp],
        "cv_set_weights": [vp, vp, vp],
        "cv_get_weights": [vp, vp, vp],
        "cv_features": [vp, vp, i64, vp, vp, vp],
        "cv_grads": [vp, vp, vp, i64, vp, vp, vp],
        "cv_train": [vp, vp, ctypes.c_int32, i64, ctypes.c_int32, ctypes.c_float, vp, vp],
        "rbm_force_sqerr": [vp, i64, vp, i64, vp, ctypes.c_int32, vp, vp],
        "ensemble_workspace_size": [ctypes.POINTER(rbm_ensemble), vp, ctypes.POINTER(sz)],
        "ensemble_run": [ctypes.POINTER(rbm_ensemble), vp, vp, vp, i64, i64,
                         ctypes.POINTER(rbm_ensemble_tile), vp, sz, ctypes.c_int32, vp],
        "rbmr_workspace_size": [pp, i64, ctypes.c_int32, ctypes.POINTER(sz)],
        "rbmr_run": [pp, vp, i64, i64, i64, ctypes.c_int32, vp, sz, vp],
        "rbmr_run_noalloc": [pp, vp, i64, i64, i64, ctypes.c_int32, vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.rbm_status_str.argtypes = [ctypes.c_int]
    L.rbm_status_str.restype = ctypes.c_char_p
    L.rbm_last_error.argtypes = []
    L.rbm_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(st: int):
    if st != RBM_OK:
        L = lib()
        raise RbmError(st, f"{L.rbm_status_str(st).decode()}: {L.rbm_last_error().decode()}")


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


@dataclass
class Params:
    """Parameters of eq. (1.2) with V = beta |x|^2 / 2 and of RBM-1."""
    d: int
    kernel: int
    n: int
    p: int
    kparam: float = 0.0
    beta: float = 0.0
    sigma: float = 0.0
    dt: float = 1e-3
    seed: int = 1
    sys: int = 0
    cv: int = 0

    def c(self) -> rbm_params:
        return rbm_params(self.d, self.kernel, self.n, self.p, self.cv, self.kparam, self.beta,
                          self.sigma, self.dt, self.seed, self.sys, 0)


# --------------------------------------------------------------------------
# entry points (same names as the C ABI)
# --------------------------------------------------------------------------

def rbm_status_str(st: int) -> str:
    return lib().rbm_status_str(st).decode()


def rbm_last_error() -> str:
    return lib().rbm_last_error().decode()


def rbm_workspace_size(prm: Params) -> int:
    n = ctypes.c_size_t()
    _check(lib().rbm_workspace_size(ctypes.byref(prm.c()), ctypes.byref(n)))
    return n.value


def rbm_init(prm: Params, x0, slots=None, step0: int = 0, ws=None, stream=None) -> "Context":
    """Create a context on x0 ([N][d] float32 CUDA tensor, by id)."""
    import torch
    _expect(x0, torch.float32, (prm.n, prm.d), "x0")
    if slots is not None:
        _expect(slots, torch.int32, (prm.n,), "slots")
    nbytes = rbm_workspace_size(prm)
    if ws is None:
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=x0.device)
    base = (ws.data_ptr() + 255) & ~255
    avail = ws.numel() - (base - ws.data_ptr())
    h = ctypes.c_void_p()
    cp = prm.c()
    _check(lib().rbm_init(ctypes.byref(cp), _ptr(x0), _ptr(slots), step0, ctypes.c_void_p(base),
                          avail, _stream(stream), ctypes.byref(h)))
    return Context(prm, h, ws)


def rbm_step(ctx: "Context", stream=None):
    _check(lib().rbm_step(ctx.handle, _stream(stream)))


def rbm_run(ctx: "Context", nsteps: int, stream=None):
    _check(lib().rbm_run(ctx.handle, nsteps, _stream(stream)))


def rbm_positions(ctx: "Context", out=None, stream=None):
    import torch
    if out is None:
        out = torch.empty((ctx.prm.n, ctx.prm.d), dtype=torch.float32, device=ctx.ws.device)
    _expect(out, torch.float32, (ctx.prm.n, ctx.prm.d), "out")
    _check(lib().rbm_positions(ctx.handle, _ptr(out), _stream(stream)))
    return out


def rbm_perm(ctx: "Context", out=None, stream=None):
    import torch
    if out is None:
        out = torch.empty(ctx.prm.n, dtype=torch.int32, device=ctx.ws.device)
    _expect(out, torch.int32, (ctx.prm.n,), "out")
    _check(lib().rbm_perm(ctx.handle, _ptr(out), _stream(stream)))
    return out


def rbm_forces(ctx: "Context", step: int, out=None, stream=None):
    import torch
    if out is None:
        out = torch.empty((ctx.prm.n, ctx.prm.d), dtype=torch.float32, device=ctx.ws.device)
    _expect(out, torch.float32, (ctx.prm.n, ctx.prm.d), "out")
    _check(lib().rbm_forces(ctx.handle, step, _ptr(out), _stream(stream)))
    return out


def rbm_step_index(ctx: "Context") -> int:
    m = ctypes.c_int64()
    _check(lib().rbm_step_index(ctx.handle, ctypes.byref(m)))
    return m.value


def rbm_check(ctx: "Context", stream=None):
    _check(lib().rbm_check(ctx.handle, _stream(stream)))


def rbm_timing(ctx: "Context", max_steps: int):
    _check(lib().rbm_timing(ctx.handle, max_steps))


def rbm_phase_times(ctx: "Context"):
    """(dict phase -> mean ms per step, number of steps recorded)."""
    ms = (ctypes.c_double * len(PHASES))()
    n = ctypes.c_int64()
    _check(lib().rbm_phase_times(ctx.handle, ms, ctypes.byref(n)))
    return dict(zip(PHASES, list(ms))), n.value


def rbm_destroy(ctx: "Context"):
    if ctx.handle is not None:
        _check(lib().rbm_destroy(ctx.handle))
        ctx.handle = None


def direct_forces(prm: Params, x, ids=None, out=None, stream=None):
    import torch
    _expect(x, torch.float32, (prm.n, prm.d), "x")
    nids = prm.n if ids is None else ids.numel()
    if ids is not None:
        _expect(ids, torch.int32, (nids,), "ids")
    if out is None:
        out = torch.empty((nids, prm.d), dtype=torch.float32, device=x.device)
    _expect(out, torch.float32, (nids, prm.d), "out")
    _check(lib().direct_forces(ctypes.byref(prm.c()), _ptr(x), _ptr(ids), nids, _ptr(out),
                               _stream(stream)))
    return out


def direct_moments(prm: Params, x, ids=None, stream=None):
    """(F [nids][d], m2 [nids]): exact forces and 1/(N-1) sum_j |K(X_i - X_j)|^2."""
    import torch
    _expect(x, torch.float32, (prm.n, prm.d), "x")
    nids = prm.n if ids is None else ids.numel()
    if ids is not None:
        _expect(ids, torch.int32, (nids,), "ids")
    f = torch.empty((nids, prm.d), dtype=torch.float32, device=x.device)
    m2 = torch.empty(nids, dtype=torch.float32, device=x.device)
    _check(lib().direct_moments(ctypes.byref(prm.c()), _ptr(x), _ptr(ids), nids, _ptr(f), _ptr(m2),
                                _stream(stream)))
    return f, m2


def direct_step(prm: Params, x, step: int, out=None, stream=None):
    import torch
    _expect(x, torch.float32, (prm.n, prm.d), "x")
    if out is None:
        out = torch.empty_like(x)
    _expect(out, torch.float32, (prm.n, prm.d), "out")
    _check(lib().direct_step(ctypes.byref(prm.c()), _ptr(x), _ptr(out), step, _stream(stream)))
    return out


# ---- RBM-r ------------------------------------------------------------------

def rbmr_workspace_size(prm: Params, window: int = 0, rounds: int = 0) -> int:
    out = ctypes.c_size_t()
    _check(lib().rbmr_workspace_size(ctypes.byref(prm.c()), window, rounds, ctypes.byref(out)))
    return out.value


def rbmr_run(prm: Params, x, k0: int, niter: int, window: int = 0, rounds: int = 0, ws=None, stream=None):
    """RBM-r iterations k0 .. k0 + niter - 1 in place on x ([N][d] FP32 by
    particle id); returns x.  ws: a uint8 device tensor of at least
    rbmr_workspace_size bytes (allocated here if None)."""
    import torch
    _expect(x, torch.float32, (prm.n, prm.d), "x")
    need = rbmr_workspace_size(prm, window, rounds)
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=x.device)
    _check(lib().rbmr_run(ctypes.byref(prm.c()), _ptr(x), k0, niter, window, rounds, _ptr(ws), ws.numel(),
                          _stream(stream)))
    return x


def rbmr_run_noalloc(prm: Params, x, k0: int, niter: int, window: int = 0, rounds: int = 0, stream=None):
    """rbmr_run with the library's static per-GPU workspace (no allocation by
    the library or here); returns x."""
    import torch
    _expect(x, torch.float32, (prm.n, prm.d), "x")
    _check(lib().rbmr_run_noalloc(ctypes.byref(prm.c()), _ptr(x), k0, niter, window, rounds, _stream(stream)))
    return x


# ---- control variate -------------------------------------------------------

def cv_init(ctx: "Context", seed: int, stream=None):
    _check(lib().cv_init(ctx.handle, seed, _stream(stream)))


def cv_set_weights(ctx: "Context", w, stream=None):
    import torch
    _expect(w, torch.float32, (2, CV_NPARAM), "w")
    _check(lib().cv_set_weights(ctx.handle, _ptr(w), _stream(stream)))


def cv_get_weights(ctx: "Context", out=None, stream=None):
    import torch
    if out is None:
        out = torch.empty((2, CV_NPARAM), dtype=torch.float32, device=ctx.ws.device)
    _expect(out, torch.float32, (2, CV_NPARAM), "out")
    _check(lib().cv_get_weights(ctx.handle, _ptr(out), _stream(stream)))
    return out


def cv_features(ctx: "Context", x, stream=None):
    """(a(x), c(x)), each [n][32]."""
    import torch
    n = x.shape[0]
    _expect(x, torch.float32, (n, 2), "x")
    a = torch.empty((n, 32), dtype=torch.float32, device=x.device)
    c = torch.empty((n, 32), dtype=torch.float32, device=x.device)
    _check(lib().cv_features(ctx.handle, _ptr(x), n, _ptr(a), _ptr(c), _stream(stream)))
    return a, c


def cv_grads(ctx: "Context", x, y, stream=None):
    """(loss, gradient [2][6432]) on the pairs (x[q], y[q])."""
    import torch
    n = x.shape[0]
    _expect(x, torch.float32, (n, 2), "x")
    _expect(y, torch.float32, (n, 2), "y")
    g = torch.empty((2, CV_NPARAM), dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    _check(lib().cv_grads(ctx.handle, _ptr(x), _ptr(y), n, _ptr(g), _ptr(loss), _stream(stream)))
    return loss, g


def cv_train(ctx: "Context", snap, nsteps: int, batch: int, lr: float = 1e-3, stream=None):
    """nsteps Adam steps on pairs from snapshots snap [nsnap][N][2]; returns
    the minibatch losses (before each step)."""
    import torch
    nsnap = snap.shape[0]
    _expect(snap, torch.float32, (nsnap, ctx.prm.n, 2), "snap")
    loss = torch.empty(max(nsteps, 1), dtype=torch.float32, device=snap.device)
    _check(lib().cv_train(ctx.handle, _ptr(snap), nsnap, nsteps, batch, lr, _ptr(loss), _stream(stream)))
    return loss[:nsteps]


def rbm_force_sqerr(f, ids, fref, stream=None):
    """sum_t |f[ids[t]] - fref[t]|^2 in FP64 (returns a 1-element CUDA tensor).
    f: [n][d] float32 forces by id; ids: int32 [nids], each in 0..n-1;
    fref: [nids][d] float32."""
    import torch
    if f.dim() != 2:
        raise ValueError(f"f: need a [n][d] tensor, got shape {tuple(f.shape)}")
    n, d = int(f.shape[0]), int(f.shape[1])
    _expect(f, torch.float32, (n, d), "f")
    nids = ids.numel()
    _expect(ids, torch.int32, (nids,), "ids")
    _expect(fref, torch.float32, (nids, d), "fref")
    if nids and (int(ids.min()) < 0 or int(ids.max()) >= n):
        raise ValueError(f"ids must lie in 0..{n - 1}")
    out = torch.empty(1, dtype=torch.float64, device=f.device)
    _check(lib().rbm_force_sqerr(_ptr(f), n, _ptr(ids), nids, _ptr(fref), d, _ptr(out), _stream(stream)))
    return out


# --------------------------------------------------------------------------
# batched ensemble


@dataclass
class Ensemble:
    """Independent RBM-1 systems sharing the model parameters; system s has
    sizes[s] particles and Philox key seeds[s] (counter word 3 = s)."""
    d: int
    kernel: int
    p: int
    sizes: object
    seeds: object
    kparam: float = 0.0
    beta: float = 0.0
    sigma: float = 0.0
    dt: float = 1e-3

    def c(self) -> rbm_ensemble:
        return rbm_ensemble(self.d, self.kernel, self.p, 0, self.kparam, self.beta, self.sigma, self.dt,
                            len(self.sizes))

    def host_arrays(self):
        import numpy as np
        n = np.ascontiguousarray(self.sizes, dtype=np.int64)
        sd = np.ascontiguousarray(self.seeds, dtype=np.uint64)
        if n.shape != sd.shape or n.ndim != 1:
            raise ValueError("sizes and seeds must be 1-D arrays of equal length")
        return n, sd

    @property
    def offsets(self):
        import numpy as np
        n = np.asarray(self.sizes, dtype=np.int64)
        return np.concatenate([[0], np.cumsum(n)])


def ensemble_workspace_size(ens: Ensemble) -> int:
    n, _ = ens.host_arrays()
    out = ctypes.c_size_t()
    _check(lib().ensemble_workspace_size(ctypes.byref(ens.c()), n.ctypes.data_as(ctypes.c_void_p), ctypes.byref(out)))
    return out.value


def ensemble_run(ens: Ensemble, x, step0: int, nsteps: int, lds_max: int = 0, grid: int = 0,
                 team: int = 0, bucket: int = 0, wg: int = 0, graph: bool = True, ws=None, stream=None):
    """Runs steps step0 .. step0 + nsteps - 1 of every system in place on x
    [sum sizes][d] (FP32, system by system, each by particle id).  Returns
    when the launch has completed."""
    import torch
    n, sd = ens.host_arrays()
    tot = int(n.sum())
    _expect(x, torch.float32, (tot, ens.d), "x")
    need = ensemble_workspace_size(ens)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=x.device)
    tile = rbm_ensemble_tile(lds_max, grid, team, bucket, wg)
    _check(lib().ensemble_run(ctypes.byref(ens.c()), n.ctypes.data_as(ctypes.c_void_p),
                              sd.ctypes.data_as(ctypes.c_void_p), _ptr(x), step0, nsteps, ctypes.byref(tile),
                              _ptr(ws), ws.numel(), 1 if graph else 0, _stream(stream)))
    return x


def _expect(t, dtype, shape, name):
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous() or not t.is_cuda:
        raise ValueError(f"{name}: need a contiguous CUDA {dtype} tensor of shape {shape}, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")


@dataclass
class Context:
    """An RBM-1 run: host handle plus the workspace tensor that backs it."""
    prm: Params
    handle: ctypes.c_void_p
    ws: object = field(repr=False)

    def __del__(self):
        try:
            if self.handle is not None and _lib is not None:
                _lib.rbm_destroy(self.handle)
                self.handle = None
        except Exception:
            pass
