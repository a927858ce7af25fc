"""The C ABI on the CPU: the library loads, exports what include/kubo.h declares,
and rejects bad arguments before any device work (no GPU needed)."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2309_06675_amd import kubo, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "kubo.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kubo_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = kubo.lib()
    names = _declared()
    assert set(kubo.EXPORTED) <= set(names)
    for name in names:
        assert hasattr(L, name), name


def test_status_strings():
    for s in range(7):
        assert kubo.kubo_status_string(s).startswith("KUBO_")
    assert "unknown" in kubo.kubo_status_string(99)


def _desc(n=4, R=None, grid=(4, 4, 4), kb=0, kc=-1):
    if R is None:
        R = synth.cube(1)
    return kubo.make_desc(n, R, grid, kb, kc)


def _plan_status(descs, nf=1, flags=0, tiles=None):
    st, h, ws = kubo.kubo_plan(descs, nf, flags, tiles)
    if h is not None:
        kubo.kubo_plan_destroy(h)
    return st, ws


def test_valid_plan_reports_workspace():
    d, keep = _desc()
    st, ws = _plan_status([d])
    assert st == kubo.KUBO_OK and ws > 0


@pytest.mark.parametrize("bad", ["n0", "nR0", "grid0", "dupR", "notclosed", "slab", "nf0",
                                 "nfbig", "flag", "count0"])
def test_plan_rejects_invalid(bad):
    R = synth.cube(1)
    kw = {}
    nf = 1
    flags = 0
    if bad == "n0":
        kw["n"] = 0
    elif bad == "grid0":
        kw["grid"] = (4, 0, 4)
    elif bad == "dupR":
        kw["R"] = np.concatenate([R, R[:1]])
    elif bad == "notclosed":
        kw["R"] = np.array([[0, 0, 0], [1, 0, 0]], np.int32)
    elif bad == "slab":
        kw["kb"], kw["kc"] = 60, 10
    elif bad == "count0":
        kw["kc"] = 0
    elif bad == "nf0":
        nf = 0
    elif bad == "nfbig":
        nf = 5000
    elif bad == "flag":
        flags = 0x80
    if bad == "nR0":
        d, keep = _desc()
        d.n_R = 0
    else:
        d, keep = _desc(**kw)
    st, _ = _plan_status([d], nf, flags)
    assert st == kubo.KUBO_E_INVALID


def test_plan_rejects_bad_tile():
    d, keep = _desc()
    t = kubo.kubo_tile()
    t.n_orb, t.threads, t.k_block, t.reserved = 4, 96, 8, 0
    assert _plan_status([d], tiles=[t])[0] == kubo.KUBO_E_INVALID
    t.n_orb, t.threads = 40, 64
    assert _plan_status([d], tiles=[t])[0] == kubo.KUBO_E_INVALID


def test_plan_unsupported_size():
    d, keep = _desc(n=600)
    assert _plan_status([d], flags=kubo.KUBO_F_FORWARD_ONLY)[0] == kubo.KUBO_E_UNSUPPORTED


def test_large_n_plans_are_forward_only():
    """128 < n <= 512 runs the large-n pipeline: the plan must be forward-only and not a
    tensor plan; its workspace holds the pipeline's per-k slices."""
    d, keep = _desc(n=200, grid=(3, 2, 2))
    assert _plan_status([d])[0] == kubo.KUBO_E_UNSUPPORTED
    assert _plan_status([d], flags=kubo.KUBO_F_FORWARD_ONLY | kubo.KUBO_F_TENSOR)[0] == \
        kubo.KUBO_E_UNSUPPORTED
    st, ws = _plan_status([d], flags=kubo.KUBO_F_FORWARD_ONLY)
    assert st == kubo.KUBO_OK and ws > 12 * 200 * 200 * 16


def test_null_plan_pointer():
    L = kubo.lib()
    ws = ctypes.c_size_t()
    d, keep = _desc()
    arr = (kubo.kubo_model_desc * 1)(d)
    assert L.kubo_plan(None, arr, 1, 1, 0, None, 0, ctypes.byref(ws)) == kubo.KUBO_E_INVALID
    h = ctypes.c_void_p()
    assert L.kubo_plan(ctypes.byref(h), None, 1, 1, 0, None, 0, ctypes.byref(ws)) == \
        kubo.KUBO_E_INVALID


def test_call_argument_checks_happen_before_device_work():
    d, keep = _desc()
    st, h, wsb = kubo.kubo_plan([d], 1)
    assert st == kubo.KUBO_OK
    try:
        fake = 0x1000  # never dereferenced: every check below fails first
        assert kubo.kubo_ahc(h, 0, fake, 1e-3, 0.0, fake, fake, wsb, None) == kubo.KUBO_E_INVALID
        assert kubo.kubo_ahc(h, fake, fake, -1.0, 0.0, fake, fake, wsb, None) == \
            kubo.KUBO_E_INVALID
        assert kubo.kubo_ahc(h, fake, fake, 1e-3, float("nan"), fake, fake, wsb, None) == \
            kubo.KUBO_E_INVALID
        assert kubo.kubo_ahc(h, fake, fake, 1e-3, 0.0, fake, fake, wsb - 1, None) == \
            kubo.KUBO_E_WORKSPACE
        assert kubo.kubo_ahc(h, fake, fake, 1e-3, 0.0, fake, 0, wsb, None) == \
            kubo.KUBO_E_WORKSPACE
        assert kubo.kubo_ahc_backward(h, fake, fake, 0.0, 0.01, fake, fake, fake, wsb, None) == \
            kubo.KUBO_E_INVALID
        assert kubo.kubo_plan_device_status(h, fake, None) == kubo.KUBO_E_INVALID
        assert kubo.kubo_ahc_noalloc(h, 0, fake, 1e-3, 0.0, fake, 0, None) == kubo.KUBO_E_INVALID
        assert kubo.kubo_ahc_noalloc(None, fake, fake, 1e-3, 0.0, fake, 0, None) == \
            kubo.KUBO_E_INVALID
        st, tk, nm = kubo.kubo_plan_info(h)
        assert st == kubo.KUBO_OK and tk == 64 and nm == 1
    finally:
        kubo.kubo_plan_destroy(h)


def test_plan_info_counts_slabs():
    d1, k1 = _desc(kb=5, kc=20)
    d2, k2 = _desc(n=6, grid=(3, 2, 5))
    st, h, wsb = kubo.kubo_plan([d1, d2], 3)
    assert st == kubo.KUBO_OK
    assert kubo.kubo_plan_info(h)[1:] == (50, 2)
    kubo.kubo_plan_destroy(h)
    kubo.kubo_plan_destroy(None)


def test_kernel_time_slots():
    """which = 0..4 are timing slots (4: the large-n reduction alone); a plan that ran
    nothing reports zero launches without touching a device; other values are invalid."""
    d, keep = _desc(n=200, grid=(3, 2, 2))
    st, h, ws = kubo.kubo_plan([d], 1, kubo.KUBO_F_FORWARD_ONLY | kubo.KUBO_F_TIMING)
    assert st == kubo.KUBO_OK
    for which in range(5):
        st, ms, nl, kp = kubo.kubo_plan_kernel_time(h, which)
        assert st == kubo.KUBO_OK and (ms, nl, kp) == (0.0, 0, 0)
    for which in (-1, 5):
        assert kubo.kubo_plan_kernel_time(h, which)[0] == kubo.KUBO_E_INVALID
    kubo.kubo_plan_destroy(h)


def test_tensor_plan_sizes_and_argument_checks():
    """A KUBO_F_TENSOR plan needs room for a third set of partial Bloch sums and four
    result components; kubo_ahc_tensor on a plan without the flag is rejected before any
    device work."""
    d, keep = _desc(n=4, grid=(4, 3, 2))
    st, h, wsb = kubo.kubo_plan([d], 3, kubo.KUBO_F_FORWARD_ONLY)
    st2, h2, wsb2 = kubo.kubo_plan([d], 3, kubo.KUBO_F_FORWARD_ONLY | kubo.KUBO_F_TENSOR)
    assert st == kubo.KUBO_OK and st2 == kubo.KUBO_OK
    try:
        assert wsb2 > wsb
        fake = 0x1000  # never dereferenced
        assert kubo.kubo_ahc_tensor(h, fake, fake, 1e-3, 0.0, 0, fake, fake, wsb, None) == \
            kubo.KUBO_E_INVALID
        assert kubo.kubo_ahc_tensor(h2, fake, fake, -1.0, 0.0, 0, fake, fake, wsb2, None) == \
            kubo.KUBO_E_INVALID
        assert kubo.kubo_ahc_tensor(h2, fake, fake, 1e-3, 0.0, 0, fake, fake, wsb2 - 1, None) == \
            kubo.KUBO_E_WORKSPACE
    finally:
        kubo.kubo_plan_destroy(h)
        kubo.kubo_plan_destroy(h2)


def test_gf_argument_checks():
    """kubo_ahc_gf rejects bad scalars, NULL node arrays, too many nodes, a short workspace
    and models with more than 32 orbitals before any device work."""
    d, keep = _desc(n=4, grid=(4, 3, 2))
    d40, keep40 = _desc(n=40, grid=(2, 2, 2))
    st, h, wsb = kubo.kubo_plan([d], 3, kubo.KUBO_F_FORWARD_ONLY)
    st2, h2, wsb2 = kubo.kubo_plan([d, d40], 3, kubo.KUBO_F_FORWARD_ONLY)
    assert st == kubo.KUBO_OK and st2 == kubo.KUBO_OK
    try:
        fake = 0x1000  # never dereferenced
        gf = kubo.kubo_ahc_gf
        assert gf(h, fake, fake, -0.1, fake, fake, 4, fake, fake, wsb, None) == kubo.KUBO_E_INVALID
        assert gf(h, fake, fake, float("nan"), fake, fake, 4, fake, fake, wsb, None) == \
            kubo.KUBO_E_INVALID
        assert gf(h, fake, fake, 0.1, 0, fake, 4, fake, fake, wsb, None) == kubo.KUBO_E_INVALID
        assert gf(h, fake, fake, 0.1, fake, 0, 4, fake, fake, wsb, None) == kubo.KUBO_E_INVALID
        assert gf(h, fake, fake, 0.1, fake, fake, 0, fake, fake, wsb, None) == kubo.KUBO_E_INVALID
        assert gf(h, fake, fake, 0.1, fake, fake, kubo.KUBO_GF_MAX_NODES + 1, fake, fake, wsb,
                  None) == kubo.KUBO_E_INVALID
        assert gf(h, fake, fake, 0.1, fake, fake, 4, fake, fake, wsb - 1, None) == \
            kubo.KUBO_E_WORKSPACE
        assert gf(h2, fake, fake, 0.1, fake, fake, 4, fake, fake, wsb2, None) == \
            kubo.KUBO_E_UNSUPPORTED
    finally:
        kubo.kubo_plan_destroy(h)
        kubo.kubo_plan_destroy(h2)
