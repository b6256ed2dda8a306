"""Groupwise Tucker compression of one channel tensor, FP64 (Sections 2.3 and 3.2).

Test infrastructure only (see oracle/__init__.py).

Readings of the paper used here:
  * Mode 3 is the subcarrier axis.  Each group of `gs` consecutive subcarriers is one
    channel tensor X_g (Nr x Nt x size_g) of the groupwise model; all groups of a channel
    share the mode-1 factor A and the mode-2 factor, and own their C_g and core G_g.  The
    last group is short when gs does not divide Nsc, and p_g = min(p, size_g).
  * The model's tensor form X_g ~ G_g x1 A x2 Bt x3 C_g gives H_s ~ A Ht_s Bt^T, while the
    paper's matrix form writes H ~ A Ht B^*.  Both hold with B = conj(Bt).  This module
    works with the tensor-form factor Bt internally and returns the matrix-form B.
  * A shared factor is initialised from the summed mode-n Grams of the tensors that share
    it (HOSVD of the whole channel for A and B); C_g from its own group.
  * Eigenvectors are taken in descending eigenvalue order, each scaled so that its
    largest-modulus entry (lowest index on ties) is real and positive.
  * A fixed number S of sweeps, Gauss-Seidel order A -> B -> C; the core is formed once at
    the end (Algorithm "Groupwise Tucker compression algorithm").
"""

from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

from .tensor import mode_product, norm2, unfold


def group_layout(nsc: int, gs: int) -> Tuple[List[int], List[int]]:
    """Start index and size of each subcarrier group (the loop index sets of the algorithm)."""
    if nsc <= 0 or gs <= 0:
        raise ValueError("nsc and gs must be positive")
    n_groups = -(-nsc // gs)
    starts = [g * gs for g in range(n_groups)]
    sizes = [min(gs, nsc - g * gs) for g in range(n_groups)]
    return starts, sizes


def group_tensors(X: np.ndarray, gs: int) -> List[np.ndarray]:
    """Split X [nsc][nr][nt] into group tensors X_g[i1, i2, i3] = H_{start+i3}[i1, i2]."""
    starts, sizes = group_layout(X.shape[0], gs)
    return [np.transpose(X[s0:s0 + sz], (1, 2, 0)) for s0, sz in zip(starts, sizes)]


def top_eigvecs(M: np.ndarray, r: int) -> Tuple[np.ndarray, np.ndarray]:
    """r principal eigenvectors (and eigenvalues) of a Hermitian matrix, descending order,
    each column scaled so that its largest-modulus entry is real positive."""
    M = 0.5 * (M + M.conj().T)
    w, V = np.linalg.eigh(M)
    w = w[::-1][:r]
    V = V[:, ::-1][:, :r].copy()
    for j in range(V.shape[1]):
        k = int(np.argmax(np.abs(V[:, j])))
        ph = V[k, j] / abs(V[k, j]) if abs(V[k, j]) > 0 else 1.0
        V[:, j] = V[:, j] / ph
    return V, w


def hosvd_init(Xgs: List[np.ndarray], m: int, n: int, p: int):
    """Initial factors from the leading left singular vectors of the mode-n unfoldings
    (Algorithm "HOSVD Algorithm"; first step of the groupwise algorithm)."""
    S1 = sum(unfold(Xg, 0) @ unfold(Xg, 0).conj().T for Xg in Xgs)
    S2 = sum(unfold(Xg, 1) @ unfold(Xg, 1).conj().T for Xg in Xgs)
    A, _ = top_eigvecs(S1, m)
    Bt, _ = top_eigvecs(S2, n)
    Cs = []
    for Xg in Xgs:
        pg = min(p, Xg.shape[2])
        Cg, _ = top_eigvecs(unfold(Xg, 2) @ unfold(Xg, 2).conj().T, pg)
        Cs.append(Cg)
    return A, Bt, Cs


def update_A(Xgs, Bt, Cs, m):
    """Equation "update A": m principal eigenvectors of sum_g M1 M1^*,
    M1 = (X_g x2 Bt^* x3 C_g^*)_(1)."""
    S = 0
    for Xg, Cg in zip(Xgs, Cs):
        M1 = unfold(mode_product(mode_product(Xg, Bt.conj().T, 1), Cg.conj().T, 2), 0)
        S = S + M1 @ M1.conj().T
    return top_eigvecs(S, m)


def update_B(Xgs, A, Cs, n):
    """Equation "update B": n principal eigenvectors of sum_g M2 M2^*,
    M2 = (X_g x1 A^* x3 C_g^*)_(2)."""
    S = 0
    for Xg, Cg in zip(Xgs, Cs):
        M2 = unfold(mode_product(mode_product(Xg, A.conj().T, 0), Cg.conj().T, 2), 1)
        S = S + M2 @ M2.conj().T
    return top_eigvecs(S, n)


def update_C(Xg, A, Bt, pg):
    """Equation "update C": p principal eigenvectors of M3 M3^*,
    M3 = (X_g x1 A^* x2 Bt^*)_(3)."""
    M3 = unfold(mode_product(mode_product(Xg, A.conj().T, 0), Bt.conj().T, 1), 2)
    return top_eigvecs(M3 @ M3.conj().T, pg)


def core(Xg, A, Bt, Cg):
    """Equation "kernel": optimal core G = X x1 A^* x2 B^* x3 C^* (tensor-form factors)."""
    return mode_product(mode_product(mode_product(Xg, A.conj().T, 0), Bt.conj().T, 1),
                        Cg.conj().T, 2)


def objective(Xgs, A, Bt, Cs) -> float:
    """f = sum_g ||X_g||^2 - ||G_g||^2 at the optimal cores (equation "min-max substitite")."""
    return float(sum(norm2(Xg) - norm2(core(Xg, A, Bt, Cg)) for Xg, Cg in zip(Xgs, Cs)))


def to_abi(X_shape, gs, A, Bt, Cs, cores, p) -> Dict[str, np.ndarray]:
    """Pack factors in the library layout: A [nr][m], B [nt][n] (matrix form),
    C [nsc][p] (rows of C_g, zero-padded past p_g), G [groups][p][m][n]."""
    nsc = X_shape[0]
    starts, sizes = group_layout(nsc, gs)
    m = A.shape[1]
    n = Bt.shape[1]
    C = np.zeros((nsc, p), dtype=np.complex128)
    G = np.zeros((len(starts), p, m, n), dtype=np.complex128)
    for g, (s0, sz) in enumerate(zip(starts, sizes)):
        pg = Cs[g].shape[1]
        C[s0:s0 + sz, :pg] = Cs[g]
        G[g, :pg] = np.transpose(cores[g], (2, 0, 1))
    return dict(A=A.copy(), B=Bt.conj().copy(), C=C, G=G)


def fit(X: np.ndarray, gs: int, m: int, n: int, p: int, iters: int,
        warm: Dict[str, np.ndarray] | None = None) -> Dict[str, np.ndarray]:
    """Groupwise Tucker compression (Algorithm "Groupwise Tucker compression algorithm").

    X is [nsc][nr][nt].  Returns A, B (matrix form), C [nsc][p], G [groups][p][m][n] and
    `trace`: the objective f after the initialisation and after each of the 3*iters
    half-steps.  With `warm` (A, B, C in the same layout) the HOSVD step is skipped.
    """
    nsc, nr, nt = X.shape
    if not (1 <= m <= nr and 1 <= n <= nt and 1 <= p <= gs):
        raise ValueError("ranks out of range")
    Xgs = group_tensors(X, gs)
    starts, sizes = group_layout(nsc, gs)
    if warm is None:
        A, Bt, Cs = hosvd_init(Xgs, m, n, p)
    else:
        A = np.array(warm["A"], dtype=np.complex128)
        Bt = np.conj(np.array(warm["B"], dtype=np.complex128))
        Cs = [np.array(warm["C"][s0:s0 + sz, :min(p, sz)], dtype=np.complex128)
              for s0, sz in zip(starts, sizes)]
    trace = [objective(Xgs, A, Bt, Cs)]
    for _ in range(iters):
        A, _ = update_A(Xgs, Bt, Cs, m)
        trace.append(objective(Xgs, A, Bt, Cs))
        Bt, _ = update_B(Xgs, A, Cs, n)
        trace.append(objective(Xgs, A, Bt, Cs))
        Cs = [update_C(Xg, A, Bt, min(p, Xg.shape[2]))[0] for Xg in Xgs]
        trace.append(objective(Xgs, A, Bt, Cs))
    cores = [core(Xg, A, Bt, Cg) for Xg, Cg in zip(Xgs, Cs)]
    out = to_abi(X.shape, gs, A, Bt, Cs, cores, p)
    out["trace"] = np.array(trace)
    out["norm2_X"] = norm2(X)
    return out


def compressed_channels(C: np.ndarray, G: np.ndarray, gs: int) -> np.ndarray:
    """Ht_s = G_g x3 (c^* C_g) with c the selector of subcarrier s, i.e.
    sum_q C[s, q] G_g[q]  (equation "compressed matrix SINR reduction").  [nsc][m][n]."""
    nsc = C.shape[0]
    starts, sizes = group_layout(nsc, gs)
    Ht = np.zeros((nsc,) + G.shape[2:], dtype=np.complex128)
    for g, (s0, sz) in enumerate(zip(starts, sizes)):
        for i in range(sz):
            sel = np.zeros(sz)
            sel[i] = 1.0
            row = sel @ C[s0:s0 + sz]            # c^* C_g  (c real)
            Ht[s0 + i] = np.tensordot(row, G[g], axes=(0, 0))
    return Ht


def combine_full(X: np.ndarray, U: np.ndarray) -> np.ndarray:
    """Channel matrices at general coefficient vectors (Section 2.2, equation "channel
    submatrices, tensor"): H(t) = X x3 u_t = sum_s U[t, s] X_s, with u_t the combining row
    (the row c^*(t) of the tensor form).  X [P][nr][nt], U [T][P]; returns [T][nr][nt]."""
    T = U.shape[0]
    H = np.zeros((T,) + X.shape[1:], dtype=np.complex128)
    for t in range(T):
        for s in range(X.shape[0]):
            H[t] += U[t, s] * X[s]
    return H


def combine_compressed(C: np.ndarray, G: np.ndarray, gs: int, U: np.ndarray) -> np.ndarray:
    """Compressed channel matrices at general coefficient vectors (Section 3.3, equation
    "compressed matrix SINR reduction"): with the groupwise model X_g ~ G_g x1 A x2 Bt x3 C_g,
    the combination of X by the row u_t is A Ht(t) B^H with
    Ht(t) = sum_g G_g x3 (u_t,g C_g), u_t,g the entries of u_t on group g's submatrices.
    C [P][p], G [groups][p][m][n], U [T][P]; returns [T][m][n]."""
    T, P = U.shape
    starts, sizes = group_layout(P, gs)
    Ht = np.zeros((T,) + G.shape[2:], dtype=np.complex128)
    for t in range(T):
        for g, (s0, sz) in enumerate(zip(starts, sizes)):
            row = U[t, s0:s0 + sz] @ C[s0:s0 + sz]     # u_t,g C_g  (length p)
            Ht[t] += np.tensordot(row, G[g], axes=(0, 0))
    return Ht


def reconstruct(A, B, C, G, gs) -> Tuple[np.ndarray, np.ndarray]:
    """Compressed channels Ht [nsc][m][n] and the full reconstruction
    Xhat_g = G_g x1 A x2 Bt x3 C_g (tensor form, Bt = conj(B)) as [nsc][nr][nt]."""
    nsc = C.shape[0]
    starts, sizes = group_layout(nsc, gs)
    Ht = compressed_channels(C, G, gs)
    Bt = np.conj(B)
    Xhat = np.zeros((nsc, A.shape[0], B.shape[0]), dtype=np.complex128)
    for g, (s0, sz) in enumerate(zip(starts, sizes)):
        core_g = np.transpose(G[g], (1, 2, 0))          # m x n x p
        Xg = mode_product(mode_product(mode_product(core_g, A, 0), Bt, 1), C[s0:s0 + sz], 2)
        Xhat[s0:s0 + sz] = np.transpose(Xg, (2, 0, 1))
    return Ht, Xhat
