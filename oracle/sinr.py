"""SVD precoding, MMSE equalisation and per-stream SINR, FP64 (Sections 2.2 and 3.3).

Test infrastructure only (see oracle/__init__.py).

Single link per channel matrix (no intra- or inter-cell terms): the covariance is
Q = H P (H P)^* + sigma^2 I.  The same chain is applied to a full channel matrix H_s
(Nr x Nt) or to a compressed one Ht_s (m x n); Section 3.3 shows that the factors A and B
cancel, so the compressed SINR is the chain evaluated on Ht_s.
"""

from __future__ import annotations

import numpy as np


def svd_precoder(H: np.ndarray, ns: int):
    """P = first ns right singular vectors of H (equation "precoding matrix").
    Works on a stack [..., M, N].  Returns (P, singular values)."""
    U, S, Vh = np.linalg.svd(H, full_matrices=False)
    P = np.conj(np.swapaxes(Vh, -1, -2))[..., :ns]
    return P, S


def mmse_sinr(H: np.ndarray, P: np.ndarray, sigma2: float):
    """Per-stream SINR of the MMSE receiver for a single link (stacked over leading axes).

    Q = HP (HP)^* + sigma^2 I        (equation "covariance matrix")
    W = Q^{-1} H P                   (equation "MMSE receive filter")
    s_r = |w_r^* H p_r|^2            (equation "s_r^ij")
    SINR_r = s_r / (w_r^* Q w_r - s_r)   (equation "SINR formula")
    """
    HP = H @ P
    M = H.shape[-2]
    Q = HP @ np.conj(np.swapaxes(HP, -1, -2)) + sigma2 * np.eye(M)
    W = np.linalg.solve(Q, HP)
    WH = np.conj(np.swapaxes(W, -1, -2))
    s = np.abs(np.diagonal(WH @ HP, axis1=-2, axis2=-1)) ** 2
    wqw = np.real(np.diagonal(WH @ Q @ W, axis1=-2, axis2=-1))
    return s / (wqw - s)


def sinr(H: np.ndarray, sigma2_list, ns: int) -> np.ndarray:
    """SINR of every stream for a stack of channel matrices H [nsc][M][N] and every noise
    variance: returns [n_snr][nsc][ns] (linear)."""
    P, _ = svd_precoder(H, ns)
    return np.stack([mmse_sinr(H, P, float(s2)) for s2 in sigma2_list])


def sinr_closed_form(H: np.ndarray, sigma2_list, ns: int) -> np.ndarray:
    """SINR_r = sigma_r^2 / sigma^2 for the single link (derived from the closed form of
    the signal power after the SVD precoder: s_r = sigma_r^4 |u_r^* Q^{-1} u_r|^2)."""
    S = np.linalg.svd(H, compute_uv=False)[..., :ns]
    return np.stack([S ** 2 / float(s2) for s2 in sigma2_list])


def woodbury_inverse(A: np.ndarray, Qt: np.ndarray, sigma2: float) -> np.ndarray:
    """Equation "reduced inversion of interference matrix":
    Q^{-1} ~ (1/s2) I_M - (1/s2) A Qt^{-1} (Qt - s2 I_m) A^*."""
    M, m = A.shape
    inner = np.linalg.solve(Qt, Qt - sigma2 * np.eye(m))
    return (np.eye(M) - A @ inner @ A.conj().T) / sigma2


def compressed_filter(Ht: np.ndarray, Vt: np.ndarray, sigma2: float) -> np.ndarray:
    """Wt = (1/s2) [I_m - Qt^{-1} (Qt - s2 I_m)] Ht Vt, the compressed receive filter
    (Section 3.3, filter matrix), with Qt = Ht Vt (Ht Vt)^* + s2 I_m."""
    m = Ht.shape[0]
    HV = Ht @ Vt
    Qt = HV @ HV.conj().T + sigma2 * np.eye(m)
    inner = np.linalg.solve(Qt, Qt - sigma2 * np.eye(m))
    return (np.eye(m) - inner) @ HV / sigma2
