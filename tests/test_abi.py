"""Host-side checks of the C ABI (no GPU): the library loads, exports every
entry point the header declares, and rejects bad arguments before anything
is enqueued."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1812_10575_amd as rbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "rbm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", txt, flags=re.M)))


def test_header_declares_the_entry_points():
    fns = header_functions()
    for name in ("rbm_init", "rbm_step", "rbm_run", "direct_step", "direct_forces", "rbm_positions"):
        assert name in fns
    assert set(fns) == set(rbm.SYMBOLS)


def test_library_exports_every_declared_symbol():
    L = rbm.lib()
    for name in header_functions():
        assert hasattr(L, name), name
        assert hasattr(rbm, name), name  # binding has the same names


def P(**kw):
    base = dict(d=3, kernel=rbm.RBM_K_ATTREP, n=1 << 16, p=8, kparam=0.01, beta=0.0, sigma=0.1, dt=1e-3)
    base.update(kw)
    return rbm.Params(**base)


def test_workspace_size_grows_with_n():
    small = rbm.rbm_workspace_size(P(n=1000))
    big = rbm.rbm_workspace_size(P(n=1 << 20))
    assert 0 < small < big
    # state + scratch + staging of 16-byte records at least
    assert big >= 3 * 16 * (1 << 20)


@pytest.mark.parametrize("kw,status", [
    (dict(d=0), rbm.RBM_ERR_INVALID),
    (dict(d=4), rbm.RBM_ERR_INVALID),
    (dict(kernel=7), rbm.RBM_ERR_INVALID),
    (dict(cv=2), rbm.RBM_ERR_INVALID),
    (dict(cv=1), rbm.RBM_ERR_UNSUPPORTED),
    (dict(cv=1, d=2, kernel=rbm.RBM_K_GAUSS, p=65), rbm.RBM_ERR_UNSUPPORTED),
    (dict(n=1, p=2), rbm.RBM_ERR_INVALID),
    (dict(p=1), rbm.RBM_ERR_INVALID),
    (dict(n=100, p=101), rbm.RBM_ERR_INVALID),
    (dict(dt=0.0), rbm.RBM_ERR_INVALID),
    (dict(dt=float("nan")), rbm.RBM_ERR_INVALID),
    (dict(sigma=-1.0), rbm.RBM_ERR_INVALID),
    (dict(kparam=-1.0), rbm.RBM_ERR_INVALID),
    (dict(n=(1 << 25) + 1), rbm.RBM_ERR_UNSUPPORTED),
    (dict(n=100000, p=65), rbm.RBM_ERR_UNSUPPORTED),
])
def test_bad_parameters_are_rejected(kw, status):
    with pytest.raises(rbm.RbmError) as ei:
        rbm.rbm_workspace_size(P(**kw))
    assert ei.value.status == status
    assert rbm.rbm_last_error()


def test_plan_fits_the_kernels_at_every_size():
    """Every supported N gets a bucket plan inside the limits the step
    kernels are built for (at most 32768 fine buckets; the library refuses a
    plan beyond them): the sizes around the switch to the split level at
    217,600, the largest N, powers of two and a log-spaced sweep."""
    ns = {2817, 217600, 217601, 31457280, 31457281, (1 << 25) - 1, 1 << 25}
    ns |= {1 << k for k in range(12, 26)}
    ns |= {int(v) for v in np.geomspace(3000, 1 << 25, 200)}
    for n in sorted(ns):
        assert rbm.rbm_workspace_size(P(n=n)) >= 3 * 16 * n, n


def test_large_p_is_fine_when_one_workgroup_holds_the_system():
    assert rbm.rbm_workspace_size(P(n=2000, p=2000)) > 0


def test_init_checks_before_enqueueing():
    L = rbm.lib()
    prm = P(n=4096).c()
    need = ctypes.c_size_t()
    assert L.rbm_workspace_size(ctypes.byref(prm), ctypes.byref(need)) == rbm.RBM_OK
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x100000)  # never dereferenced: every call below fails its checks first
    assert L.rbm_init(ctypes.byref(prm), None, None, 0, fake, need.value, None, ctypes.byref(h)) == rbm.RBM_ERR_INVALID
    assert L.rbm_init(ctypes.byref(prm), fake, None, 0, fake, need.value - 1, None, ctypes.byref(h)) == rbm.RBM_ERR_WORKSPACE
    assert L.rbm_init(ctypes.byref(prm), fake, None, 0, ctypes.c_void_p(0x100010), need.value, None, ctypes.byref(h)) == rbm.RBM_ERR_WORKSPACE
    assert L.rbm_init(ctypes.byref(prm), fake, None, -1, fake, need.value, None, ctypes.byref(h)) == rbm.RBM_ERR_INVALID
    assert L.rbm_init(ctypes.byref(prm), fake, None, 1 << 32, fake, need.value, None, ctypes.byref(h)) == rbm.RBM_ERR_INVALID
    assert L.rbm_step(None, None) == rbm.RBM_ERR_INVALID
    assert L.rbm_run(None, 3, None) == rbm.RBM_ERR_INVALID
    assert L.direct_step(ctypes.byref(prm), fake, fake, 0, None) == rbm.RBM_ERR_INVALID  # aliasing
    assert L.direct_forces(ctypes.byref(prm), None, None, 0, fake, None) == rbm.RBM_ERR_INVALID


def test_status_strings():
    for st in range(6):
        assert rbm.rbm_status_str(st)
    assert rbm.rbm_status_str(99) == "unknown status"


def test_fused_steps_size_their_buffers(monkeypatch):
    """Fused steps (more than 128 fine buckets, no control variate) hold two
    banks of key sets, the coarse digits of every slot, the cross counts and
    the fix-up positions; RBM_FUSE=0 plans the unfused order without them.
    Below the split level (N <= 217,600) there is nothing to fuse."""
    n = 1 << 20
    fused = rbm.rbm_workspace_size(P(n=n))
    monkeypatch.setenv("RBM_FUSE", "0")
    plain = rbm.rbm_workspace_size(P(n=n))
    small_plain = rbm.rbm_workspace_size(P(n=200000))
    monkeypatch.delenv("RBM_FUSE")
    assert rbm.rbm_workspace_size(P(n=200000)) == small_plain
    # at least 32 key sets of one digit byte per slot and the 4-byte fix-up table
    assert fused - plain >= 32 * n + 4 * n


def _al(v):
    return (v + 255) // 256 * 256


@pytest.mark.parametrize("n,p,window,rounds", [
    (1 << 20, 2, 0, 0), (1 << 20, 8, 1 << 22, 0), (3, 2, 1, 1), (100003, 7, 777, 3), (1 << 25, 2, 0, 0),
    (4097, 3, 5000, 255)])
def test_rbmr_workspace_size_is_the_header_formula(n, p, window, rounds):
    """rbmr_workspace_size against the sum that include/rbm.h states: 16 N +
    16 window p + two queues of 256 segments of ceil(window / 256) + 512
    entries + the schedule sort's counts (B buckets of 2^bsh particles, at
    most 1024 buckets or 4096 particles each; G counting workgroups) + the
    queue lengths, each part rounded up to 256 bytes (host-only call)."""
    prm = rbm.Params(d=1, kernel=rbm.RBM_K_SOFTCOULOMB, n=n, p=p, kparam=1.0, beta=1.0, sigma=0.1, dt=1e-3)
    w = window or min(max(n // p, 1), 1 << 22)
    r = rounds or min((4 + 2 * p) * -(-(w * p) // n) + (1 if n > (1 << 22) else 0), 255)
    bsh = 0
    while -(-n // (1 << bsh)) > 1024 and (1 << bsh) < 4096:
        bsh += 1
    B = -(-n // (1 << bsh))
    G = -(-w // max(4096, -(-w // 256)))
    segcap = -(-w // 256) + 512
    want = (_al(16 * n) + _al(8 * w * p) + 2 * _al(4 * w * p) + _al(4 * B * G) + 2 * _al(4 * B)
            + 2 * _al(4 * 256 * segcap) + _al(4 * 256 * (r + 2)))
    assert rbm.rbmr_workspace_size(prm, window, rounds) == want
