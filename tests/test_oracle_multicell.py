"""Pins of the multi-cell oracle (oracle/multicell.py) against what the paper and the
mathematics fix: the single-link special case, the textbook MMSE SINR identities with
interference, the cancellation of the shared factors (equations "compressed pre", "Cov",
"reduced inversion of interference matrix"), exact recovery of a planted system, a
non-increasing objective, and the storage formula of Table "storage complexity".
"""

import numpy as np
import pytest

from oracle import metrics, multicell as mc, sinr as osinr, tucker
from synthgen import random_unitary


def _crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _random_system(rng, J, K, nsc, nr, nt, decay=None):
    X = {}
    for u in range(J * K):
        for k in range(J):
            H = _crandn(rng, nsc, nr, nt)
            if decay is not None:
                H = H * (decay[0] ** np.arange(nr))[None, :, None] * (decay[1] ** np.arange(nt))[None, None, :]
            X[(u, k)] = H
    return X


def _planted_system(rng, J, K, nsc, nr, nt, m, n):
    """X[u, k][s] = A_u Ht[u, k][s] B_k^* with orthonormal A_u (per UE) and B_k (per BS)."""
    A = {u: random_unitary(rng, nr, m) for u in range(J * K)}
    B = {k: random_unitary(rng, nt, n) for k in range(J)}
    Ht, X = {}, {}
    for u in range(J * K):
        for k in range(J):
            Ht[(u, k)] = _crandn(rng, nsc, m, n)
            X[(u, k)] = A[u][None] @ Ht[(u, k)] @ B[k].conj().T[None]
    return A, B, Ht, X


def test_interference_terms_protocol():
    J, K = 3, 2
    t = mc.interference_terms(J, K, "paper")
    for i in range(J):
        for j in range(K):
            u = mc.ue_index(i, j, K)
            assert t[u][0] == (i, u)                       # own transmission first
            others = t[u][1:]
            assert sorted(others) == sorted((k, mc.ue_index(k, 0, K)) for k in range(J) if k != i)
    ta = mc.interference_terms(J, K, "all")
    assert all(len(v) == J * K for v in ta.values())
    assert mc.interference_terms(J, K, "none") == {u: [(u // K, u)] for u in range(J * K)}


def test_single_link_system_reduces_to_single_link_oracle():
    rng = np.random.default_rng(3)
    X = _random_system(rng, 1, 1, 30, 4, 10, decay=(0.6, 0.8))
    gs, m, n, p, iters = 8, 3, 5, 4, 4
    sys_fit = mc.fit(X, gs, m, n, p, iters)
    one = tucker.fit(X[(0, 0)], gs, m, n, p, iters)
    np.testing.assert_allclose(sys_fit["trace"], one["trace"], rtol=1e-10, atol=1e-10)
    _, Xh1 = tucker.reconstruct(one["A"], one["B"], one["C"], one["G"], gs)
    _, Xh2 = tucker.reconstruct(sys_fit["A"][0], sys_fit["B"][0], sys_fit["C"][(0, 0)],
                                sys_fit["G"][(0, 0)], gs)
    assert np.linalg.norm(Xh1 - Xh2) <= 1e-10 * np.linalg.norm(X[(0, 0)])
    s2 = [0.1, 1.0]
    got = mc.sinr_system({(0, 0): X[(0, 0)]}, 1, 1, s2, 2)[0]
    np.testing.assert_allclose(got, osinr.sinr(X[(0, 0)], s2, 2), rtol=1e-10)


@pytest.mark.parametrize("ns", [1, 2, 3])
def test_mmse_identity_with_interference(ns):
    # SINR_r = 1 / [(I + G^H R^{-1} G)^{-1}]_rr - 1 with G the desired effective channel and R
    # the interference-plus-noise covariance (for ns = 1: SINR = g^H R^{-1} g)
    rng = np.random.default_rng(10 + ns)
    J, K, nsc, M, N = 3, 2, 3, 4, 6
    H = _random_system(rng, J, K, nsc, M, N)
    s2 = [0.2, 2.0]
    for mode in ("paper", "all"):
        got = mc.sinr_system(H, J, K, s2, ns, mode)
        terms = mc.interference_terms(J, K, mode)
        for u, t in terms.items():
            for s in range(nsc):
                def prec(v):
                    _, _, Vh = np.linalg.svd(H[(v, v // K)][s])
                    return Vh.conj().T[:, :ns]
                Gd = H[(u, t[0][0])][s] @ prec(u)
                for a, sig2 in enumerate(s2):
                    R = sig2 * np.eye(M, dtype=complex)
                    for k, v in t[1:]:
                        Gi = H[(u, k)][s] @ prec(v)
                        R = R + Gi @ Gi.conj().T
                    F = np.eye(ns) + Gd.conj().T @ np.linalg.solve(R, Gd)
                    ref = 1.0 / np.diag(np.linalg.inv(F)).real - 1.0
                    np.testing.assert_allclose(got[u][a, s], ref, rtol=1e-9)


def test_shared_factors_cancel():
    # with A shared per UE and B per BS the SINR of the full channels equals that of the
    # compressed ones (equations "compressed pre", "Cov" and the reduced inversion)
    rng = np.random.default_rng(21)
    J, K, nsc, nr, nt, m, n = 3, 2, 4, 6, 10, 4, 5
    A, B, Ht, X = _planted_system(rng, J, K, nsc, nr, nt, m, n)
    s2 = [0.05, 0.5]
    for mode in ("paper", "all"):
        full = mc.sinr_system(X, J, K, s2, 3, mode)
        comp = mc.sinr_system(Ht, J, K, s2, 3, mode)
        for u in full:
            np.testing.assert_allclose(comp[u], full[u], rtol=1e-9)
    # the cancellation needs B shared per BS: a different B on one interfering link breaks it
    X2 = dict(X)
    B_other = random_unitary(rng, nt, n)
    X2[(0, 1)] = A[0][None] @ Ht[(0, 1)] @ B_other.conj().T[None]
    full2 = mc.sinr_system(X2, J, K, s2, 3, "paper")
    assert np.abs(full2[0] - comp[0]).max() > 1e-3 * np.abs(comp[0]).max()


def test_reduced_inversion_of_interference_matrix():
    # Q^{-1} = (1/s2) I - (1/s2) A Qt^{-1} (Qt - s2 I) A^* for Q = A (Qt - s2 I) A^* + s2 I, and
    # W = A Wt with Wt = (1/s2) (I - Qt^{-1} (Qt - s2 I)) Ht_i Vt  (equation "reduced
    # inversion of interference matrix" and the filter that follows it)
    rng = np.random.default_rng(31)
    nr, m, ns, s2 = 8, 4, 2, 0.3
    A = random_unitary(rng, nr, m)
    Gs = [_crandn(rng, m, ns) for _ in range(3)]          # desired first, then interferers
    Qt = sum(g @ g.conj().T for g in Gs) + s2 * np.eye(m)
    Q = A @ (Qt - s2 * np.eye(m)) @ A.conj().T + s2 * np.eye(nr)
    Qinv = np.eye(nr) / s2 - A @ np.linalg.solve(Qt, Qt - s2 * np.eye(m)) @ A.conj().T / s2
    np.testing.assert_allclose(Qinv, np.linalg.inv(Q), atol=1e-12)
    W = np.linalg.solve(Q, A @ Gs[0])
    Wt = (np.eye(m) - np.linalg.solve(Qt, Qt - s2 * np.eye(m))) @ Gs[0] / s2
    np.testing.assert_allclose(W, A @ Wt, atol=1e-12)


def test_fit_recovers_planted_system_and_decreases():
    rng = np.random.default_rng(41)
    J, K, nsc, nr, nt, gs, m, n, p = 2, 2, 24, 5, 9, 8, 3, 4, 3
    X = {}
    A = {u: random_unitary(rng, nr, m) for u in range(J * K)}
    B = {k: random_unitary(rng, nt, n) for k in range(J)}
    for u in range(J * K):
        for k in range(J):
            starts, sizes = tucker.group_layout(nsc, gs)
            H = np.zeros((nsc, nr, nt), complex)
            for s0, sz in zip(starts, sizes):
                Cg = random_unitary(rng, sz, p)
                core = _crandn(rng, p, m, n)
                Hg = np.einsum("sq,qab->sab", Cg, core)
                H[s0:s0 + sz] = A[u][None] @ Hg @ B[k].conj().T[None]
            X[(u, k)] = H
    r = mc.fit(X, gs, m, n, p, 4)
    tot = sum(np.sum(np.abs(v) ** 2) for v in X.values())
    for (u, k), Xv in X.items():
        _, Xh = tucker.reconstruct(r["A"][u], r["B"][k], r["C"][(u, k)], r["G"][(u, k)], gs)
        assert metrics.nmse(Xv, Xh) < 1e-20
    assert np.all(np.diff(r["trace"]) <= 1e-12 * tot)
    # lossy random system: the objective never increases and ends below the initial value
    X = _random_system(np.random.default_rng(42), 2, 2, 20, 4, 8, decay=(0.7, 0.85))
    r = mc.fit(X, 6, 2, 3, 3, 5)
    tot = sum(np.sum(np.abs(v) ** 2) for v in X.values())
    assert np.all(np.diff(r["trace"]) <= 1e-12 * tot)
    assert r["trace"][-1] < r["trace"][0]


def test_system_storage_ratio_matches_table_formula():
    # one group per link (gs = nsc = P) is the paper's storage formula, which Table 1 pins
    for J, K, M, N, P, m, n, p in ((21, 5, 64, 512, 401, 60, 230, 150), (3, 2, 8, 64, 12, 8, 16, 12)):
        val = mc.storage_ratio_system(J, K, M, N, P, P, m, n, p)
        ref = metrics.storage_ratio_groupwise(J, K, M, N, P, m, n, p)
        assert abs(val - ref) < 1e-12 * ref


def test_individual_and_shared_models_through_the_labels():
    # Individual model (every link its own A and B) = the single-link fit of each link; Shared
    # model (one A and one B for all links) = the single-link groupwise fit of the links
    # concatenated along the subcarrier axis (whole groups per link)
    rng = np.random.default_rng(51)
    X = _random_system(rng, 2, 1, 16, 4, 8, decay=(0.6, 0.8))
    gs, m, n, p, iters = 8, 2, 3, 3, 3
    ind = mc.fit(X, gs, m, n, p, iters, a_of=lambda lk: lk, b_of=lambda lk: lk)
    for lk, Xv in X.items():
        one = tucker.fit(Xv, gs, m, n, p, iters)
        _, Xh1 = tucker.reconstruct(one["A"], one["B"], one["C"], one["G"], gs)
        _, Xh2 = tucker.reconstruct(ind["A"][lk], ind["B"][lk], ind["C"][lk], ind["G"][lk], gs)
        assert np.linalg.norm(Xh1 - Xh2) <= 1e-10 * np.linalg.norm(Xv)
    sh = mc.fit(X, gs, m, n, p, iters, a_of=lambda lk: 0, b_of=lambda lk: 0)
    links = sorted(X)
    cat = np.concatenate([X[lk] for lk in links], axis=0)
    one = tucker.fit(cat, gs, m, n, p, iters)
    np.testing.assert_allclose(sh["trace"], one["trace"], rtol=1e-10, atol=1e-10)
    _, Xh1 = tucker.reconstruct(one["A"], one["B"], one["C"], one["G"], gs)
    Xh2 = np.concatenate([tucker.reconstruct(sh["A"][0], sh["B"][0], sh["C"][lk], sh["G"][lk], gs)[1]
                          for lk in links], axis=0)
    assert np.linalg.norm(Xh1 - Xh2) <= 1e-10 * np.linalg.norm(cat)
