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
    opt = B.FitOptions(iters, ttm, eig64, flags, 0)
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
    # the MMSE filter needs a positive noise variance (the covariance is singular without it)
    zero = (C.c_float * 1)(0.0)
    assert lib.gt_sinr_eval(h, dummy, dummy, zero, 1, dummy, None, dummy, wsb.value, None) == 1
    assert lib.gt_tucker_fit_backward(h) == 5
    # the coefficient-vector combinations check the workspace, the pointers and n_pts first
    assert lib.gt_combine_full(h, dummy, dummy, 4, dummy, None, 0, None) == 4
    assert lib.gt_combine_compressed(h, dummy, dummy, dummy, 4, dummy, None, 0, None) == 4
    assert lib.gt_combine_full(h, dummy, dummy, 0, dummy, dummy, wsb.value, None) == 1
    assert lib.gt_combine_full(h, None, dummy, 4, dummy, dummy, wsb.value, None) == 1
    assert lib.gt_combine_compressed(h, dummy, dummy, dummy, (1 << 20) + 1, dummy, dummy,
                                     wsb.value, None) == 1
    lib.gt_plan_destroy(h)


def test_status_strings(lib):
    for code in range(8):
        assert lib.gt_status_string(code)
    assert lib.gt_status_string(99) == b"unknown status"


def test_set_tuning_validation(lib):
    st, h = _plan(lib, [(8, 64, 240, 12, 8, 16, 12, 4)] * 16)
    assert st == 0
    for v in ((0, 0, 0), (1, 1, 1), (2, 0, 1), (0, 0, 2)):
        assert lib.gt_plan_set_tuning(h, *v) == 0, v
    for v in ((3, 0, 0), (-1, 0, 0), (0, 2, 0), (0, 0, 3)):
        assert lib.gt_plan_set_tuning(h, *v) == 1, v   # GT_ERR_ARG
    lib.gt_plan_destroy(h)


def test_set_tuning_rejects_fp32_variants_on_16bit_plans(lib):
    # the prefetching / older B-step kernels and the vector-ALU T pass exist in FP32 only
    st, h = _plan(lib, [(8, 64, 240, 12, 8, 16, 12, 4)] * 16, ttm=1)
    assert st == 0
    assert lib.gt_plan_set_tuning(h, 0, 0, 1) == 0
    for v in ((1, 0, 1), (2, 0, 1), (0, 1, 1)):
        assert lib.gt_plan_set_tuning(h, *v) == 5, v   # GT_ERR_UNSUPPORTED
    lib.gt_plan_destroy(h)


def _plan_dtype(lib, descs, dtype, ttm=0):
    arr = (B.ChannelDesc * len(descs))(*[B.ChannelDesc(*d) for d in descs])
    opt = B.FitOptions(3, ttm, 0, 0, dtype)
    h = C.c_void_p()
    return lib.gt_plan_create(arr, len(descs), C.byref(opt), C.byref(h)), h


def test_c128_plans(lib):
    d = (2, 8, 12, 12, 2, 4, 3, 2)
    assert _plan_dtype(lib, [d], 2)[0] == 1                # unknown dtype: GT_ERR_ARG
    assert _plan_dtype(lib, [d], B.GT_C128, ttm=1)[0] == 5  # 16-bit fit options: unsupported
    st, h = _plan_dtype(lib, [d], B.GT_C128)
    assert st == 0
    st64, h64 = _plan_dtype(lib, [d], B.GT_C64)
    w128, w64 = C.c_size_t(), C.c_size_t()
    lib.gt_plan_workspace_bytes(h, C.byref(w128))
    lib.gt_plan_workspace_bytes(h64, C.byref(w64))
    assert w128.value > w64.value                          # FP64 gradient scratch
    dummy = C.c_void_p(1 << 20)
    # the fit, reconstruction and their adjoints are not provided in FP64: refused, no launch
    assert lib.gt_tucker_fit(h, dummy, dummy, dummy, dummy, dummy, None, None, dummy,
                             w128.value, None) == 5
    assert lib.gt_tucker_reconstruct(h, dummy, dummy, dummy, dummy, dummy, dummy, dummy,
                                     w128.value, None) == 5
    assert lib.gt_tucker_reconstruct_backward(h, *([dummy] * 10), dummy, w128.value, None) == 5
    lib.gt_plan_destroy(h)
    lib.gt_plan_destroy(h64)


def test_api_checks_every_buffer():
    # the Python front end checks sizes and element types before any pointer reaches the
    # library (a CPU plan: nothing is launched)
    import torch

    from paper_2401_09792_amd import api

    d = dict(nr=4, nt=8, nsc=20, group_size=6, m=2, n=3, p=2, ns=2)
    plan = api.Plan([d], iters=2, device="cpu")
    t = plan.totals
    C_ = torch.zeros(t.c, dtype=torch.complex64)
    G = torch.zeros(t.g, dtype=torch.complex64)
    with pytest.raises(ValueError, match="C has"):
        plan.sinr(torch.zeros(t.c - 1, dtype=torch.complex64), G, [0.1])
    with pytest.raises(TypeError, match="G must be"):
        plan.sinr(C_, G.to(torch.complex128), [0.1])
    with pytest.raises(ValueError, match="out has"):
        plan.sinr(C_, G, [0.1, 1.0], out=torch.zeros((1, t.sc, plan.ns_max)))
    with pytest.raises(TypeError, match="status must be"):
        plan.sinr(C_, G, [0.1], status=torch.zeros(1, dtype=torch.int64))
    with pytest.raises(ValueError, match="grad_sinr must have shape"):
        plan.sinr_backward(C_, G, [0.1], torch.zeros((2, t.sc, plan.ns_max)))
    with pytest.raises(ValueError, match="factors"):
        f = plan.empty_factors()
        f["B"] = f["B"][:-1]
        plan.fit(torch.zeros(t.x, dtype=torch.complex64), factors=f)
    with pytest.raises(ValueError, match="grad_Ht has"):
        A, Bm = (torch.zeros(k, dtype=torch.complex64) for k in (t.a, t.b))
        plan.reconstruct_backward(A, Bm, C_, G, grad_Ht=torch.zeros(3, dtype=torch.complex64))
    with pytest.raises(ValueError, match="X has"):
        plan.sinr_full(torch.zeros(t.x + 1, dtype=torch.complex64), [0.1])
    p128 = api.Plan([d], iters=2, device="cpu", dtype="c128")
    with pytest.raises(TypeError, match="complex128"):
        p128.sinr(C_, G, [0.1])


def _plan_descs(lib, descs):
    arr = (B.ChannelDesc * len(descs))(*[B.ChannelDesc(*d) for d in descs])
    opt = B.FitOptions(3, 0, 0, 0, 0)
    h = C.c_void_p()
    return lib.gt_plan_create(arr, len(descs), C.byref(opt), C.byref(h)), h


def test_sharing_labels_are_validated(lib):
    base = (4, 16, 24, 8, 2, 4, 3, 2)
    # channels that share A must agree on (nr, m); those that share B on (nt, n)
    assert _plan_descs(lib, [base + (1, 0, 0), (6, 16, 24, 8, 2, 4, 3, 2, 1, 0, 0)])[0] == 2
    assert _plan_descs(lib, [base + (0, 1, 0), (4, 32, 24, 8, 2, 4, 3, 2, 0, 1, 0)])[0] == 2
    assert _plan_descs(lib, [base + (0, 1, 0), (4, 16, 24, 8, 2, 5, 3, 2, 0, 1, 0)])[0] == 2
    # labels must be >= 0 and the serving flag 0 or 1
    assert _plan_descs(lib, [base + (-1, 0, 0)])[0] == 1
    assert _plan_descs(lib, [base + (0, 0, 2)])[0] == 1
    st, h = _plan_descs(lib, [base + (1, 0, 0), (4, 32, 24, 8, 2, 6, 3, 2, 1, 0, 0)])
    assert st == 0
    wsb = C.c_size_t()
    lib.gt_plan_workspace_bytes(h, C.byref(wsb))
    dummy = C.c_void_p(1 << 20)
    # a plan that shares factors provides no objective trace: refused before any launch
    assert lib.gt_tucker_fit(h, dummy, dummy, dummy, dummy, dummy, dummy, None, dummy,
                             wsb.value, None) == 5
    # and it is not a multi-cell system (unlabelled BSs, no serving links)
    s2 = (C.c_float * 1)(0.1)
    assert lib.gt_sinr_eval_system(h, dummy, dummy, s2, 1, 1, dummy, None, dummy, wsb.value,
                                   None) == 1
    lib.gt_plan_destroy(h)


def test_system_plan_detection(lib):
    # 2 BSs x 1 UE: links (u, k) labelled a_id = u + 1, b_id = k + 1, serving where k == u
    d = lambda u, k, serving: (4, 16, 24, 8, 2, 4, 3, 2, u + 1, k + 1, serving)  # noqa: E731
    st, h = _plan_descs(lib, [d(0, 0, 1), d(0, 1, 0), d(1, 0, 0), d(1, 1, 1)])
    assert st == 0
    wsb = C.c_size_t()
    lib.gt_plan_workspace_bytes(h, C.byref(wsb))
    dummy = C.c_void_p(1 << 20)
    s2 = (C.c_float * 1)(0.1)
    assert lib.gt_sinr_eval_system(h, dummy, dummy, s2, 1, 3, dummy, None, dummy, wsb.value,
                                   None) == 1      # unknown interference mode
    lib.gt_plan_destroy(h)
    # two serving links for one UE: not a system
    st, h = _plan_descs(lib, [d(0, 0, 1), d(0, 1, 1), d(1, 0, 0), d(1, 1, 1)])
    assert st == 0
    assert lib.gt_sinr_eval_system(h, dummy, dummy, s2, 1, 1, dummy, None, dummy, wsb.value,
                                   None) == 1
    lib.gt_plan_destroy(h)
