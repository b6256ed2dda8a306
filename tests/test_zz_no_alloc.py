"""The SINR adjoint in the library's static scratch (gt_sinr_eval_backward_static, the entry
point for callers that cannot allocate device memory) against the workspace entry point
gt_sinr_eval_backward, through the C ABI: two calls in a row on one GPU, the second with a
smaller plan, and a plan too large for the scratch refused before any launch.
"""

import ctypes as C

import numpy as np
import pytest
import torch

from paper_2401_09792_amd import _binding as B
from tests.gpu_util import announce, dev_c64, desc
from tests.test_gpu_backward import _compressed

pytestmark = pytest.mark.gpu


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _packed(plan, descs, seed):
    t = plan.totals
    Cb = np.zeros(t.c, np.complex128)
    Gb = np.zeros(t.g, np.complex128)
    for i, d in enumerate(descs):
        _, Ci, Gi = _compressed(seed + i, d["nsc"], d["group_size"], d["m"], d["n"], d["p"])
        o = plan.offsets(i)
        Cb[o.c:o.c + Ci.size] = Ci.reshape(-1)
        Gb[o.g:o.g + Gi.size] = Gi.reshape(-1)
    return dev_c64(Cb), dev_c64(Gb)


def _static_vs_workspace(gpu_lib, descs, seed):
    plan = gpu_lib.Plan(descs, iters=1)
    Cd, Gd = _packed(plan, descs, seed)
    s2 = [0.05, 0.5]
    g = torch.Generator().manual_seed(seed)
    grad = torch.randn((2, plan.totals.sc, plan.ns_max), generator=g).cuda()
    st_ref = torch.zeros(plan.n_channels, dtype=torch.int32, device="cuda")
    gC, gG = plan.sinr_backward(Cd, Gd, s2, grad, status=st_ref)
    gC2 = torch.full_like(Cd, float("nan"))
    gG2 = torch.full_like(Gd, float("nan"))
    st = torch.zeros(plan.n_channels, dtype=torch.int32, device="cuda")
    lib = B.load()
    rc = lib.gt_sinr_eval_backward_static(
        plan._h, _ptr(Cd), _ptr(Gd), (C.c_float * 2)(*s2), 2, _ptr(grad), _ptr(gC2), _ptr(gG2),
        _ptr(st), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, B.STATUS_NAMES.get(rc, rc)
    torch.cuda.synchronize()
    # the same kernels on the same inputs: identical results
    assert torch.equal(gC2, gC)
    assert torch.equal(gG2, gG)
    assert torch.equal(st, st_ref)


def test_static_adjoint_matches_workspace_adjoint(gpu_lib):
    announce("static-scratch SINR adjoint, two calls")
    # first call: channels on the row-parallel adjoint (m <= 4 and m <= 8) and on the
    # cooperative one (m > 8)
    big = [desc(8, 64, 600, 12, 8, 16, 12, 4), desc(4, 32, 200, 16, 4, 8, 4, 2),
           desc(10, 40, 130, 13, 10, 20, 4, 4)]
    _static_vs_workspace(gpu_lib, big, 1)
    # second call, smaller: the scratch keeps the first call's contents
    _static_vs_workspace(gpu_lib, [desc(6, 24, 50, 10, 6, 12, 4, 3)], 2)


def test_static_adjoint_refuses_plans_beyond_the_scratch(gpu_lib):
    # 24 channels of 8 x 64 x 3276 at ranks (8, 16, 12) need 24 x 3.35 MB of dl/dHt, more than
    # the 64 MiB scratch: refused with GT_ERR_WORKSPACE, nothing launched
    announce("static-scratch SINR adjoint, oversized plan")
    plan = gpu_lib.Plan([desc(8, 64, 3276, 12, 8, 16, 12, 4)] * 24, iters=1)
    lib = B.load()
    dummy = C.c_void_p(1 << 20)
    rc = lib.gt_sinr_eval_backward_static(plan._h, dummy, dummy, (C.c_float * 1)(0.1), 1, dummy,
                                          dummy, dummy, None, None)
    assert rc == 4
