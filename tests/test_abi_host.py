"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every symbol the
header declares, validates descriptors, and lays out packed buffers exactly as the oracle
indexes groups."""

import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import tucker
from paper_2401_09792_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return B.load()


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "gtucker.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gt_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(lib):
    names = _declared_symbols()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
        assert n in B.SIGNATURES, n


def _plan(lib, descs, iters=3, flags=0, ttm=0, eig64=0):
    arr = (B.ChannelDesc * len(descs))(*[B.ChannelDesc(*d) for d in descs])
    opt = B.FitOptions(iters, ttm, eig64, flags)
    h = C.c_void_p()
    st = lib.gt_plan_create(arr, len(descs), C.byref(opt), C.byref(h))
    return st, h


def test_plan_validation(lib):
    ok = (8, 64, 3276, 12, 8, 16, 12, 4)
    st, h = _plan(lib, [ok])
    assert st == 0
    lib.gt_plan_destroy(h)
    bad = {
        (0, 64, 100, 12, 1, 1, 1, 1): 2,      # nr = 0
        (17, 64, 100, 12, 8, 16, 12, 4): 2,   # nr too large
        (8, 64, 100, 40, 8, 16, 12, 4): 2,    # group too large
        (8, 64, 100, 12, 9, 16, 12, 4): 3,    # m > nr
        (8, 64, 100, 12, 8, 65, 12, 4): 3,    # n > nt
        (8, 64, 100, 12, 8, 16, 13, 4): 3,    # p > group size
        (8, 64, 100, 12, 2, 16, 12, 3): 3,    # ns > min(m, n)
        (8, 64, 100, 12, 8, 16, 12, 0): 3,    # ns = 0
    }
    for d, code in bad.items():
        st, h = _plan(lib, [d])
        assert st == code, (d, st)
    for ttm in (1, 2, 3):                       # 16-bit contraction forms are accepted
        st, h = _plan(lib, [ok], ttm=ttm)
        assert st == 0, ttm
        lib.gt_plan_destroy(h)
    assert _plan(lib, [ok], ttm=4)[0] == 1      # unknown precision
    assert _plan(lib, [ok], iters=-1)[0] == 1
    assert _plan(lib, [ok], flags=4)[0] == 1
    h = C.c_void_p()
    assert lib.gt_plan_create(None, 1, None, C.byref(h)) == 1


def test_offsets_match_oracle_group_layout(lib):
    descs = [(4, 32, 64, 16, 4, 8, 4, 2), (8, 64, 3276, 24, 6, 16, 12, 4),
             (16, 128, 100, 12, 12, 24, 5, 3)]
    st, h = _plan(lib, descs)
    assert st == 0
    ex = dict(x=0, a=0, b=0, c=0, g=0, ht=0, sc=0)
    for ci, (nr, nt, nsc, gs, m, n, p, ns) in enumerate(descs):
        o = B.Offsets()
        assert lib.gt_plan_offsets(h, ci, C.byref(o)) == 0
        starts, sizes = tucker.group_layout(nsc, gs)
        assert o.n_groups == len(starts)
        for k in ex:
            assert getattr(o, k) == ex[k], (ci, k)
        ex["x"] += nsc * nr * nt
        ex["a"] += nr * m
        ex["b"] += nt * n
        ex["c"] += nsc * p
        ex["g"] += len(starts) * p * m * n
        ex["ht"] += nsc * m * n
        ex["sc"] += nsc
    tot = B.Offsets()
    nsm = C.c_int32()
    assert lib.gt_plan_totals(h, C.byref(tot), C.byref(nsm)) == 0
    for k in ex:
        assert getattr(tot, k) == ex[k], k
    assert nsm.value == 4
    wsb = C.c_size_t()
    assert lib.gt_plan_workspace_bytes(h, C.byref(wsb)) == 0 and wsb.value > 0
    o = B.Offsets()
    assert lib.gt_plan_offsets(h, 3, C.byref(o)) == 1
    lib.gt_plan_destroy(h)


def test_calls_reject_bad_workspace_without_launching(lib):
    st, h = _plan(lib, [(4, 32, 64, 16, 4, 8, 4, 2)])
    dummy = C.c_void_p(1 << 20)
    s2 = (C.c_float * 1)(0.1)
    assert lib.gt_sinr_eval(h, dummy, dummy, s2, 1, dummy, None, None, 0, None) == 4
    assert lib.gt_tucker_fit(h, dummy, dummy, dummy, dummy, dummy, None, None, None, 0, None) == 4
    wsb = C.c_size_t()
    lib.gt_plan_workspace_bytes(h, C.byref(wsb))
    # bad noise-variance list is rejected before any launch
    assert lib.gt_sinr_eval(h, dummy, dummy, s2, 0, dummy, None, dummy, wsb.value, None) == 1
    neg = (C.c_float * 1)(-1.0)
    assert lib.gt_sinr_eval(h, dummy, dummy, neg, 1, dummy, None, dummy, wsb.value, None) == 1
    assert lib.gt_tucker_fit_backward(h) == 5
    lib.gt_plan_destroy(h)


def test_status_strings(lib):
    for code in range(8):
        assert lib.gt_status_string(code)
    assert lib.gt_status_string(99) == b"unknown status"


def test_set_tuning_validation(lib):
    st, h = _plan(lib, [(8, 64, 240, 12, 8, 16, 12, 4)] * 16)
    assert st == 0
    for v in ((0, 0, 0), (1, 1, 1), (2, 0, 1)):
        assert lib.gt_plan_set_tuning(h, *v) == 0, v
    for v in ((3, 0, 0), (-1, 0, 0), (0, 2, 0), (0, 0, 2)):
        assert lib.gt_plan_set_tuning(h, *v) == 1, v   # GT_ERR_ARG
    lib.gt_plan_destroy(h)
