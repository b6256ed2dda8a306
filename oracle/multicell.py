"""The multi-cell groupwise Tucker model and its SINR with interference, FP64 (Sections 2.2,
3.2 and 3.3).

Test infrastructure only (see oracle/__init__.py).

System: J base stations (BSs), K UEs per cell; UE u = (i, j) is the j-th UE of cell i and is
served by BS i.  The channel between UE u and BS k is X[u, k], stored [nsc][nr][nt] (H_s the
nr x nt receive x transmit matrix of subcarrier s); groups of gs subcarriers are the model's
channel tensors (reading R1 of the single-link oracle).

Factor sharing of the groupwise model (equation "three matrix factorization" and model
"MT_origin"): one mode-1 factor A_u for all channels of UE u (from every BS), one mode-2 factor
B_k for all channels from BS k, and a mode-3 factor and core per (u, k, group).

Readings:
  * A shared factor is initialised from the summed mode-n Grams of the tensors that share it
    (the single-link reading R4, generalised).
  * The sweep follows the algorithm's loop order: every A_[i,j] from the previous B and C,
    then every B_k from the new A and the previous C, then every C from the new A and B.
  * UE (i, j) sees the transmissions listed by `interference_terms`: its own (BS i with its
    own precoder) and, in the paper's experiment protocol, BS k != i with the precoder of the
    first UE of cell k (inter-cell only, no intra-cell interference); mode "all" adds every
    other UE of every cell (equation "signal receiving").
"""

from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np

from .tensor import mode_product, norm2, unfold
from .tucker import group_layout, group_tensors, top_eigvecs

Link = Tuple[int, int]  # (UE index u = i * K + j, BS index k)


def ue_index(i: int, j: int, K: int) -> int:
    return i * K + j


def serving_bs(u: int, K: int) -> int:
    return u // K


def interference_terms(J: int, K: int, mode: str = "paper") -> Dict[int, List[Tuple[int, int]]]:
    """Transmissions seen by each UE: a list of (BS k, UE whose precoder BS k uses), the UE's
    own transmission first.  Modes: "paper" (inter-cell from the first UE of every other cell),
    "all" (every other UE of every cell, intra- and inter-cell), "none" (single link)."""
    if mode not in ("paper", "all", "none"):
        raise ValueError(mode)
    terms = {}
    for i in range(J):
        for j in range(K):
            u = ue_index(i, j, K)
            t = [(i, u)]
            for k in range(J):
                for l in range(K):
                    v = ue_index(k, l, K)
                    if v == u:
                        continue
                    if mode == "all" or (mode == "paper" and k != i and l == 0):
                        t.append((k, v))
            terms[u] = t
    return terms


# ----------------------------------------------------------------------------------------
# Fit (model "MT_origin", equations "update A", "update B", "update C", "kernel")


def _objective(Xg, A, Bt, Cs, a_of, b_of):
    tot = 0.0
    for lk, gs_list in Xg.items():
        u, k = a_of(lk), b_of(lk)
        for X, C in zip(gs_list, Cs[lk]):
            G = mode_product(mode_product(mode_product(X, A[u].conj().T, 0), Bt[k].conj().T, 1),
                             C.conj().T, 2)
            tot += norm2(X) - norm2(G)
    return float(tot)


def fit(X: Dict[Link, np.ndarray], gs: int, m: int, n: int, p: int, iters: int,
        a_of=None, b_of=None):
    """Groupwise Tucker compression of the whole system (Algorithm "Groupwise Tucker
    compression algorithm" over its index sets [i, j] and k).  Returns per UE A[u] (nr x m),
    per BS B[k] (nt x n, matrix form H ~ A Ht B^*), per link C[u, k] ([nsc][p], rows of C_g
    zero-padded past p_g) and G[u, k] ([groups][p][m][n]), and the objective trace after the
    initialisation and after each half-step.

    a_of / b_of map a link to the label of its mode-1 / mode-2 factor (default: the UE and the
    BS, the groupwise model).  Every link its own labels gives the Individual model of
    equation "Tucker decomposition"; one label for all links the Shared model of model "MT1".
    A and B are then keyed by those labels."""
    a_of = a_of or (lambda lk: lk[0])
    b_of = b_of or (lambda lk: lk[1])
    links = sorted(X)
    ues = sorted({a_of(lk) for lk in links})
    bss = sorted({b_of(lk) for lk in links})
    Xg = {lk: group_tensors(X[lk], gs) for lk in links}
    # initialisation from the summed Grams of the sharing tensors
    A, Bt, Cs = {}, {}, {}
    for u in ues:
        S1 = sum(unfold(T, 0) @ unfold(T, 0).conj().T for lk in links if a_of(lk) == u for T in Xg[lk])
        A[u] = top_eigvecs(S1, m)[0]
    for k in bss:
        S2 = sum(unfold(T, 1) @ unfold(T, 1).conj().T for lk in links if b_of(lk) == k for T in Xg[lk])
        Bt[k] = top_eigvecs(S2, n)[0]
    for lk in links:
        Cs[lk] = [top_eigvecs(unfold(T, 2) @ unfold(T, 2).conj().T, min(p, T.shape[2]))[0]
                  for T in Xg[lk]]
    trace = [_objective(Xg, A, Bt, Cs, a_of, b_of)]
    for _ in range(iters):
        newA = {}
        for u in ues:  # equation "update A": sum over the UE's channels from every BS
            S = 0
            for lk in links:
                if a_of(lk) != u:
                    continue
                for T, C in zip(Xg[lk], Cs[lk]):
                    M1 = unfold(mode_product(mode_product(T, Bt[b_of(lk)].conj().T, 1), C.conj().T, 2), 0)
                    S = S + M1 @ M1.conj().T
            newA[u] = top_eigvecs(S, m)[0]
        A = newA
        trace.append(_objective(Xg, A, Bt, Cs, a_of, b_of))
        newB = {}
        for k in bss:  # equation "update B": sum over every UE's channel from BS k
            S = 0
            for lk in links:
                if b_of(lk) != k:
                    continue
                for T, C in zip(Xg[lk], Cs[lk]):
                    M2 = unfold(mode_product(mode_product(T, A[a_of(lk)].conj().T, 0), C.conj().T, 2), 1)
                    S = S + M2 @ M2.conj().T
            newB[k] = top_eigvecs(S, n)[0]
        Bt = newB
        trace.append(_objective(Xg, A, Bt, Cs, a_of, b_of))
        for lk in links:  # equation "update C", per channel tensor
            u, k = a_of(lk), b_of(lk)
            Cs[lk] = []
            for T in Xg[lk]:
                M3 = unfold(mode_product(mode_product(T, A[u].conj().T, 0), Bt[k].conj().T, 1), 2)
                Cs[lk].append(top_eigvecs(M3 @ M3.conj().T, min(p, T.shape[2]))[0])
        trace.append(_objective(Xg, A, Bt, Cs, a_of, b_of))
    # cores (equation "kernel"), packed like the single-link oracle
    C_out, G_out = {}, {}
    for lk in links:
        u, k = a_of(lk), b_of(lk)
        nsc = X[lk].shape[0]
        starts, sizes = group_layout(nsc, gs)
        Cm = np.zeros((nsc, p), np.complex128)
        Gm = np.zeros((len(starts), p, m, n), np.complex128)
        for g, (s0, sz) in enumerate(zip(starts, sizes)):
            C = Cs[lk][g]
            core = mode_product(mode_product(mode_product(Xg[lk][g], A[u].conj().T, 0),
                                             Bt[k].conj().T, 1), C.conj().T, 2)
            Cm[s0:s0 + sz, :C.shape[1]] = C
            Gm[g, :C.shape[1]] = np.transpose(core, (2, 0, 1))
        C_out[lk], G_out[lk] = Cm, Gm
    return dict(A=A, B={k: np.conj(v) for k, v in Bt.items()}, C=C_out, G=G_out,
                trace=np.array(trace))


# ----------------------------------------------------------------------------------------
# SINR with interference (equations "signal receiving", "covariance matrix", "MMSE receive
# filter", "s_r^ij", "SINR formula"; the same chain on the compressed matrices, equations
# "compressed pre" and "Cov")


def precoders(H_serving: np.ndarray, ns: int) -> np.ndarray:
    """First ns right singular vectors of each serving-channel matrix (equation "precoding
    matrix"): [nsc][N][ns]."""
    _, _, Vh = np.linalg.svd(H_serving, full_matrices=False)
    return np.conj(np.swapaxes(Vh[:, :ns, :], 1, 2))


def sinr_system(H: Dict[Link, np.ndarray], J: int, K: int, sigma2_list: Sequence[float], ns: int,
                mode: str = "paper") -> Dict[int, np.ndarray]:
    """Per-stream SINR of every UE, [n_snr][nsc][ns], from the channel matrices H[u, k]
    ([nsc][M][N]; the full channels, or the compressed ones Ht[u, k]).  Each UE's precoder
    comes from its serving channel; UE u sees the transmissions of interference_terms."""
    terms = interference_terms(J, K, mode)
    V = {u: precoders(H[(u, serving_bs(u, K))], ns) for u in terms}
    out = {}
    for u, t in terms.items():
        i = serving_bs(u, K)
        Hs = H[(u, i)]
        nsc, M, _ = Hs.shape
        res = np.zeros((len(sigma2_list), nsc, ns))
        for s in range(nsc):
            G_all = [H[(u, k)][s] @ V[v][s] for k, v in t]
            HP = G_all[0]                                   # desired: H_i^{[i,j]} P^{[i,j]}
            R0 = sum(g @ g.conj().T for g in G_all)
            for a, s2 in enumerate(sigma2_list):
                Q = R0 + s2 * np.eye(M)
                W = np.linalg.solve(Q, HP)
                for r in range(ns):
                    w = W[:, r]
                    sr = abs(np.vdot(w, HP[:, r])) ** 2
                    res[a, s, r] = sr / (np.vdot(w, Q @ w).real - sr)
        out[u] = res
    return out


def storage_ratio_system(J: int, K: int, nr: int, nt: int, nsc: int, gs: int, m: int, n: int,
                         p: int) -> float:
    """R_s of equation "compression ratio" for the system with subcarrier groups: J^2 K links
    of nr x nt x nsc against J K mode-1 factors, J mode-2 factors and, per link and group, a
    core and a mode-3 factor."""
    starts, sizes = group_layout(nsc, gs)
    per_link = sum(m * n * min(p, sz) + sz * min(p, sz) for sz in sizes)
    return (J * J * K * nr * nt * nsc) / (J * J * K * per_link + J * K * nr * m + J * nt * n)
