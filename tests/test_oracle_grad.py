"""Pins of the FP64 gradient oracle: central finite differences and the closed-form
singular-value gradient (CPU only)."""

import numpy as np
import pytest
import torch

import synthgen
from oracle import grad, sinr, tucker


def _small_compressed(seed=0, m=2, n=4, p=3, gs=12, nsc=12):
    rng = np.random.default_rng(seed)
    C = np.zeros((nsc, p), np.complex128)
    starts, sizes = tucker.group_layout(nsc, gs)
    G = rng.standard_normal((len(starts), p, m, n)) + 1j * rng.standard_normal((len(starts), p, m, n))
    for g, (s0, sz) in enumerate(zip(starts, sizes)):
        C[s0:s0 + sz, :min(p, sz)] = synthgen.random_unitary(rng, sz, min(p, sz))
    return C, G


def test_sinr_gradcheck_fd():
    # compressed SINR chain against central finite differences (2 x 4 compressed
    # channels, one group of 12 subcarriers, 3 core slices, 2 streams)
    C, G = _small_compressed()
    Ct = torch.tensor(C, requires_grad=True)
    Gt = torch.tensor(G, requires_grad=True)
    f = lambda c, g: grad.sinr_compressed_t(c, g, 12, [0.1, 1.0], 2)
    assert torch.autograd.gradcheck(f, (Ct, Gt), eps=1e-6, atol=1e-5, rtol=1e-4)


def test_sinr_grad_matches_closed_form():
    C, G = _small_compressed(seed=1, m=3, n=6, p=4, gs=6, nsc=14)
    rng = np.random.default_rng(2)
    s2 = [0.05, 0.5]
    gs_ = rng.standard_normal((2, 14, 2))
    a = grad.sinr_grad(C, G, 6, s2, 2, gs_)
    b = grad.sinr_grad_closed_form(C, G, 6, s2, 2, gs_)
    for x, y in zip(a, b):
        np.testing.assert_allclose(x, y, rtol=1e-8, atol=1e-8 * np.abs(y).max())


def test_sinr_forward_torch_equals_numpy():
    C, G = _small_compressed(seed=3)
    s2 = [0.2]
    Ht = tucker.compressed_channels(C, G, 12)
    ref = sinr.sinr(Ht, s2, 2)
    got = grad.sinr_compressed_t(torch.tensor(C), torch.tensor(G), 12, s2, 2).numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-10)


def test_reconstruct_gradcheck_fd():
    rng = np.random.default_rng(4)
    C, G = _small_compressed(seed=5, m=2, n=3, p=2, gs=4, nsc=6)
    A = synthgen.random_unitary(rng, 3, 2)
    B = synthgen.random_unitary(rng, 5, 3)
    ts = [torch.tensor(v, requires_grad=True) for v in (A, B, C, G)]
    f = lambda a, b, c, g: grad.reconstruct_t(a, b, c, g, 4)
    assert torch.autograd.gradcheck(f, tuple(ts), eps=1e-6, atol=1e-6, rtol=1e-5)


def test_reconstruct_grad_directional_fd():
    # l = Re<gHt, Ht> + Re<gX, Xhat>; its derivative along a random direction equals
    # Re sum conj(grad) * direction for each of A, B, C, G (central differences, FP64)
    rng = np.random.default_rng(6)
    C, G = _small_compressed(seed=7, m=2, n=3, p=2, gs=4, nsc=6)
    A = synthgen.random_unitary(rng, 3, 2)
    Bm = synthgen.random_unitary(rng, 5, 3)
    gHt = rng.standard_normal((6, 2, 3)) + 1j * rng.standard_normal((6, 2, 3))
    gX = rng.standard_normal((6, 3, 5)) + 1j * rng.standard_normal((6, 3, 5))
    grads = grad.reconstruct_grad(A, Bm, C, G, 4, gHt, gX)

    def loss(a, b, c, g):
        Ht, Xh = tucker.reconstruct(a, b, c, g, 4)
        return float(np.real(np.sum(np.conj(gHt) * Ht) + np.sum(np.conj(gX) * Xh)))

    args = [A, Bm, C, G]
    h = 1e-6
    for i, gr in enumerate(grads):
        d = rng.standard_normal(args[i].shape) + 1j * rng.standard_normal(args[i].shape)
        up = list(args)
        dn = list(args)
        up[i] = args[i] + h * d
        dn[i] = args[i] - h * d
        fd = (loss(*up) - loss(*dn)) / (2 * h)
        an = float(np.real(np.sum(np.conj(gr) * d)))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (i, fd, an)
