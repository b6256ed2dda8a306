"""Parity of the HIP adjoints (SINR and reconstruction) with the FP64 oracle gradients.

The oracle gradients are pinned by central finite differences and by the closed-form
singular-value gradient (tests/test_oracle_grad.py).  The HIP path runs in FP32, so the
comparison is relative to the largest gradient entry.
"""

import numpy as np
import pytest
import torch

import synthgen
from oracle import grad as ograd, sinr as osinr, tucker
from tests.gpu_util import announce, crandn, desc, dev_c64, host, unpack

pytestmark = pytest.mark.gpu


def _compressed(seed, nsc, gs, m, n, p):
    rng = np.random.default_rng(seed)
    starts, sizes = tucker.group_layout(nsc, gs)
    C = np.zeros((nsc, p), np.complex128)
    for s0, sz in zip(starts, sizes):
        C[s0:s0 + sz, :min(p, sz)] = synthgen.random_unitary(rng, sz, min(p, sz))
    G = crandn(rng, len(starts), p, m, n)
    for g, sz in enumerate(sizes):
        G[g, min(p, sz):] = 0
    return rng, C, G


@pytest.mark.parametrize("shape", [
    # nsc, gs, m, n, p, ns
    (24, 12, 2, 4, 3, 2),
    (40, 12, 8, 16, 12, 4),
    (30, 16, 4, 8, 4, 3),      # short last group
])
def test_sinr_backward_matches_oracle(gpu_lib, shape):
    nsc, gs, m, n, p, ns = shape
    announce(f"sinr backward {shape}")
    rng, C, G = _compressed(5, nsc, gs, m, n, p)
    s2 = [0.05, 0.5]
    gs_r = rng.standard_normal((2, nsc, ns))
    gC_o, gG_o = ograd.sinr_grad(C, G, gs, s2, ns, gs_r)
    plan = gpu_lib.Plan([desc(m, n, nsc, gs, m, n, p, ns)], iters=1)
    gC, gG = plan.sinr_backward(dev_c64(C), dev_c64(G), s2,
                                torch.as_tensor(gs_r, dtype=torch.float32).cuda())
    gC = unpack(plan, 0, host(gC), "c")
    gG = unpack(plan, 0, host(gG), "g")
    assert np.abs(gG - gG_o).max() <= 2e-3 * np.abs(gG_o).max()
    assert np.abs(gC - gC_o).max() <= 2e-3 * np.abs(gC_o).max()


def test_sinr_autograd_function(gpu_lib):
    announce("sinr autograd function")
    nsc, gs, m, n, p, ns = 24, 12, 3, 6, 4, 2
    rng, C, G = _compressed(9, nsc, gs, m, n, p)
    plan = gpu_lib.Plan([desc(m, n, nsc, gs, m, n, p, ns)], iters=1)
    Ct = dev_c64(C).requires_grad_(True)
    Gt = dev_c64(G).requires_grad_(True)
    y = gpu_lib.SinrFn.apply(plan, Ct, Gt, [0.2])
    (y[..., :ns] ** 2).sum().backward()
    gC_o, gG_o = ograd.sinr_grad(C, G, gs, [0.2], ns, 2 * host(y)[..., :ns].astype(np.float64))
    assert np.abs(host(Gt.grad).reshape(G.shape) - gG_o).max() <= 2e-3 * np.abs(gG_o).max()


@pytest.mark.parametrize("shape", [
    # nsc, gs, m, n, p, nr, nt
    (20, 8, 3, 5, 4, 6, 12),
    (30, 12, 10, 20, 6, 12, 64),     # m > 8, a short last group
    (26, 12, 12, 32, 8, 16, 256),    # the largest arrays
])
def test_reconstruct_backward_matches_oracle(gpu_lib, shape):
    announce(f"reconstruct backward {shape}")
    nsc, gs, m, n, p, nr, nt = shape
    rng, C, G = _compressed(13, nsc, gs, m, n, p)
    A = synthgen.random_unitary(rng, nr, m)
    Bm = synthgen.random_unitary(rng, nt, n)
    gHt = crandn(rng, nsc, m, n)
    gX = crandn(rng, nsc, nr, nt)
    ref = ograd.reconstruct_grad(A, Bm, C, G, gs, gHt, gX)
    plan = gpu_lib.Plan([desc(nr, nt, nsc, gs, m, n, p, 2)], iters=1)
    outs = plan.reconstruct_backward(dev_c64(A), dev_c64(Bm), dev_c64(C), dev_c64(G),
                                     dev_c64(gHt), dev_c64(gX))
    for got, r, what in zip(outs, ref, ("a", "b", "c", "g")):
        g = unpack(plan, 0, host(got), what)
        assert np.abs(g - r).max() <= 1e-4 * np.abs(r).max(), what
    # only the compressed-channel gradient
    ref2 = ograd.reconstruct_grad(A, Bm, C, G, gs, gHt, None)
    outs2 = plan.reconstruct_backward(dev_c64(A), dev_c64(Bm), dev_c64(C), dev_c64(G),
                                      dev_c64(gHt), None)
    for got, r, what in zip(outs2, ref2, ("a", "b", "c", "g")):
        g = unpack(plan, 0, host(got), what)
        assert np.abs(g - r).max() <= 1e-4 * max(np.abs(r).max(), 1e-30), what


def test_sinr_mixed_kernel_classes(gpu_lib):
    # one plan whose channels fall in every SINR kernel class (per-lane m <= 4 / 8 with
    # ns <= 2 / 4 / 8, cooperative m > 8 with n <= 32 / 64), interleaved so that the per-class
    # launches cover non-contiguous channels; forward and adjoint per channel against the oracle
    shapes = [  # nsc, gs, m, n, p, ns
        (24, 12, 2, 4, 3, 2), (26, 13, 10, 20, 4, 4), (30, 16, 6, 12, 4, 3),
        (20, 10, 4, 8, 3, 3), (17, 8, 8, 16, 5, 6), (22, 11, 12, 40, 3, 4),
        (9, 9, 3, 6, 2, 1)]
    announce(f"sinr mixed kernel classes {shapes}")
    plan = gpu_lib.Plan([desc(m, n, nsc, gs, m, n, p, ns) for nsc, gs, m, n, p, ns in shapes],
                        iters=1)
    Cb = np.zeros(plan.totals.c, np.complex128)
    Gb = np.zeros(plan.totals.g, np.complex128)
    parts = []
    for i, (nsc, gs, m, n, p, ns) in enumerate(shapes):
        rng, C, G = _compressed(40 + i, nsc, gs, m, n, p)
        o = plan.offsets(i)
        Cb[o.c:o.c + C.size] = C.reshape(-1)
        Gb[o.g:o.g + G.size] = G.reshape(-1)
        parts.append((C, G))
    s2 = [0.05, 0.5]
    sg = host(plan.sinr(dev_c64(Cb), dev_c64(Gb), s2))
    gs_all = np.random.default_rng(3).standard_normal((2, plan.totals.sc, plan.ns_max))
    gC, gG = plan.sinr_backward(dev_c64(Cb), dev_c64(Gb), s2,
                                torch.as_tensor(gs_all, dtype=torch.float32).cuda())
    gC, gG = host(gC), host(gG)
    for i, ((nsc, gs, m, n, p, ns), (C, G)) in enumerate(zip(shapes, parts)):
        o = plan.offsets(i)
        Ht = ograd.compressed_channels_t(torch.as_tensor(C), torch.as_tensor(G), gs).numpy()
        ref = osinr.sinr(Ht, s2, ns)
        got = sg[:, o.sc:o.sc + nsc, :ns]
        err = np.abs(10 * np.log10(got) - 10 * np.log10(ref)).max()
        print(f"[mixed] channel {i} m={m} n={n} ns={ns}: max SINR error {err:.3e} dB", flush=True)
        assert err <= 0.05, (i, err)
        assert np.all(sg[:, o.sc:o.sc + nsc, ns:] == 0)
        gC_o, gG_o = ograd.sinr_grad(C, G, gs, s2, ns, gs_all[:, o.sc:o.sc + nsc, :ns])
        gCi = unpack(plan, i, gC, "c")
        gGi = unpack(plan, i, gG, "g")
        assert np.abs(gGi - gG_o).max() <= 2e-3 * np.abs(gG_o).max(), i
        assert np.abs(gCi - gC_o).max() <= 2e-3 * np.abs(gC_o).max(), i
