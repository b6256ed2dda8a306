"""FP64 gradients of the compressed-domain SINR and of reconstruction (CPU, torch autograd).

Test infrastructure only (see oracle/__init__.py).

The forward functions below restate the chains of Sections 2.2, 3.2 and 3.3 with plain
torch CPU operations in complex128; the gradient is what autograd returns for a given
upstream gradient.  PyTorch's convention holds for complex leaves: the gradient of a real
loss l with respect to z is dl/dRe(z) + i dl/dIm(z).
"""

from __future__ import annotations

import numpy as np
import torch

from .tucker import group_layout


def _group_index(nsc: int, gs: int) -> torch.Tensor:
    starts, sizes = group_layout(nsc, gs)
    idx = np.concatenate([np.full(sz, g) for g, sz in enumerate(sizes)])
    return torch.as_tensor(idx, dtype=torch.long)


def compressed_channels_t(C: torch.Tensor, G: torch.Tensor, gs: int) -> torch.Tensor:
    """Ht_s = sum_q C[s, q] G_g[q]  (equation "compressed matrix SINR reduction")."""
    gi = _group_index(C.shape[0], gs)
    return torch.einsum("sq,sqij->sij", C, G[gi])


def sinr_chain_t(H: torch.Tensor, sigma2_list, ns: int) -> torch.Tensor:
    """SVD precoder + MMSE filter + per-stream SINR (Section 2.2) on a stack of matrices;
    returns [n_snr][nsc][ns]."""
    _, _, Vh = torch.linalg.svd(H, full_matrices=False)
    P = Vh.conj().transpose(-1, -2)[..., :ns]
    HP = H @ P
    M = H.shape[-2]
    eye = torch.eye(M, dtype=H.dtype)
    out = []
    for s2 in sigma2_list:
        Q = HP @ HP.conj().transpose(-1, -2) + float(s2) * eye
        W = torch.linalg.solve(Q, HP)
        WH = W.conj().transpose(-1, -2)
        s = torch.diagonal(WH @ HP, dim1=-2, dim2=-1).abs() ** 2
        wqw = torch.diagonal(WH @ Q @ W, dim1=-2, dim2=-1).real
        out.append(s / (wqw - s))
    return torch.stack(out)


def sinr_compressed_t(C, G, gs, sigma2_list, ns):
    return sinr_chain_t(compressed_channels_t(C, G, gs), sigma2_list, ns)


def sinr_grad(C: np.ndarray, G: np.ndarray, gs: int, sigma2_list, ns: int,
              grad_sinr: np.ndarray):
    """Vector-Jacobian product of the compressed SINR with respect to (C, G)."""
    Ct = torch.tensor(C, dtype=torch.complex128, requires_grad=True)
    Gt = torch.tensor(G, dtype=torch.complex128, requires_grad=True)
    y = sinr_compressed_t(Ct, Gt, gs, sigma2_list, ns)
    y.backward(torch.as_tensor(grad_sinr, dtype=torch.float64))
    return Ct.grad.resolve_conj().numpy().copy(), Gt.grad.resolve_conj().numpy().copy()


def sinr_grad_closed_form(C, G, gs, sigma2_list, ns, grad_sinr):
    """Gradient from SINR_r = sigma_r^2 / sigma^2: dl/dHt_s = sum_r (dl/dsigma_r) u_r v_r^*,
    then pulled back through Ht_s = sum_q C[s, q] G_g[q]."""
    Ht = compressed_channels_t(torch.as_tensor(C), torch.as_tensor(G), gs).numpy()
    U, S, Vh = np.linalg.svd(Ht, full_matrices=False)
    s2 = np.asarray(sigma2_list, dtype=np.float64)
    # dl/dsigma_r = sum_snr g[snr, s, r] * 2 sigma_r / s2
    dsig = np.einsum("ksr,k->sr", grad_sinr, 1.0 / s2) * 2.0 * S[:, :ns]
    gH = np.einsum("sr,sir,srj->sij", dsig, U[:, :, :ns], Vh[:, :ns, :])
    starts, sizes = group_layout(C.shape[0], gs)
    gC = np.zeros_like(C)
    gG = np.zeros_like(G)
    for g, (s0, sz) in enumerate(zip(starts, sizes)):
        for i in range(sz):
            s = s0 + i
            gG[g] += np.conj(C[s])[:, None, None] * gH[s][None]
            gC[s] = np.einsum("ij,qij->q", gH[s], np.conj(G[g]))
    return gC, gG


def reconstruct_t(A, B, C, G, gs):
    """Ht_s = sum_q C[s, q] G_g[q] and Xhat_s = A Ht_s B^*."""
    Ht = compressed_channels_t(C, G, gs)
    Xhat = A @ Ht @ B.conj().transpose(0, 1)
    return Ht, Xhat


def reconstruct_grad(A, B, C, G, gs, grad_Ht, grad_Xhat):
    """Vector-Jacobian product of reconstruction with respect to (A, B, C, G)."""
    ts = [torch.tensor(v, dtype=torch.complex128, requires_grad=True) for v in (A, B, C, G)]
    Ht, Xhat = reconstruct_t(*ts, gs)
    outs, grads = [], []
    if grad_Ht is not None:
        outs.append(Ht)
        grads.append(torch.as_tensor(grad_Ht, dtype=torch.complex128))
    if grad_Xhat is not None:
        outs.append(Xhat)
        grads.append(torch.as_tensor(grad_Xhat, dtype=torch.complex128))
    torch.autograd.backward(outs, grads)
    return [t.grad.resolve_conj().numpy().copy() if t.grad is not None
            else np.zeros(t.shape, np.complex128)
            for t in ts]
