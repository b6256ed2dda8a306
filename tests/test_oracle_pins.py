"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test checks the oracle against something other than itself: closed forms, special
cases that reduce to a textbook or library routine, invariants, brute force on tiny inputs,
and the storage column of Table 1.
"""

import math
import os

import numpy as np
import pytest

import synthgen
from oracle import metrics, sinr, tensor, tucker

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# ----------------------------------------------------------------------------------------
# Section 2.3 primitives


def test_unfold_matches_mode1_index_formula():
    # [X_(1)]_{i1, i2 + I2 (i3 - 1)} = x_{i1 i2 i3}  (1-based in the paper)
    rng = np.random.default_rng(0)
    X = crandn(rng, 3, 4, 5)
    M = tensor.unfold(X, 0)
    for i1 in range(3):
        for i2 in range(4):
            for i3 in range(5):
                assert M[i1, i2 + 4 * i3] == X[i1, i2, i3]
    for mode in range(3):
        assert np.array_equal(tensor.fold(tensor.unfold(X, mode), mode, X.shape), X)


def test_mode_product_unfolding_identity():
    # Y = X x_n U  <=>  Y_(n) = U X_(n)   (Section 2.3)
    rng = np.random.default_rng(1)
    X = crandn(rng, 3, 4, 5)
    for mode, J in ((0, 2), (1, 6), (2, 3)):
        U = crandn(rng, J, X.shape[mode])
        Y = tensor.mode_product(X, U, mode)
        np.testing.assert_allclose(tensor.unfold(Y, mode), U @ tensor.unfold(X, mode),
                                   rtol=1e-13, atol=1e-13)
    # elementwise definition for mode 1 by brute force
    U = crandn(rng, 2, 3)
    Y = tensor.mode_product(X, U, 0)
    for j in range(2):
        for i2 in range(4):
            for i3 in range(5):
                ref = sum(X[i1, i2, i3] * U[j, i1] for i1 in range(3))
                assert abs(Y[j, i2, i3] - ref) < 1e-12


def test_inner_product_and_norm():
    rng = np.random.default_rng(2)
    X, Y = crandn(rng, 2, 3, 4), crandn(rng, 2, 3, 4)
    assert abs(tensor.inner(X, Y) - np.vdot(Y.ravel(), X.ravel())) < 1e-12
    assert abs(tensor.norm2(X) - np.linalg.norm(X.ravel()) ** 2) < 1e-10


def test_top_eigvecs_against_svd_of_factor():
    # eigenvalues of Y Y^* are the squared singular values of Y (a different LAPACK routine)
    rng = np.random.default_rng(3)
    Y = crandn(rng, 7, 20)
    V, w = tucker.top_eigvecs(Y @ Y.conj().T, 4)
    S = np.linalg.svd(Y, compute_uv=False)
    np.testing.assert_allclose(w, S[:4] ** 2, rtol=1e-12)
    np.testing.assert_allclose(V.conj().T @ V, np.eye(4), atol=1e-13)
    R = (Y @ Y.conj().T) @ V - V * w[None, :]
    assert np.abs(R).max() < 1e-11 * w[0]
    for j in range(4):
        k = np.argmax(np.abs(V[:, j]))
        assert abs(V[k, j].imag) < 1e-14 and V[k, j].real > 0


# ----------------------------------------------------------------------------------------
# Section 3.2: fit


def _fit(X, gs, m, n, p, iters):
    r = tucker.fit(X, gs, m, n, p, iters)
    Ht, Xh = tucker.reconstruct(r["A"], r["B"], r["C"], r["G"], gs)
    return r, Ht, Xh


def test_group_layout_short_last_group():
    starts, sizes = tucker.group_layout(3276, 24)
    assert len(starts) == 137 and sizes[-1] == 12 and sum(sizes) == 3276
    starts, sizes = tucker.group_layout(3276, 12)
    assert len(starts) == 273 and set(sizes) == {12}


def test_single_slice_reduces_to_truncated_svd():
    # one subcarrier, mode-3 rank 1: the model is A Ht B^*, whose best approximation is
    # the truncated SVD (Eckart-Young)
    rng = np.random.default_rng(4)
    H = crandn(rng, 6, 9)
    X = H[None]
    r, Ht, Xh = _fit(X, 1, 3, 3, 1, 5)
    S = np.linalg.svd(H, compute_uv=False)
    err = np.sum(np.abs(X - Xh) ** 2)
    assert abs(err - np.sum(S[3:] ** 2)) < 1e-10 * np.sum(S ** 2)
    U, _, Vh = np.linalg.svd(H)
    np.testing.assert_allclose(r["A"] @ r["A"].conj().T, U[:, :3] @ U[:, :3].conj().T,
                               atol=1e-10)
    Bv = Vh.conj().T[:, :3]
    np.testing.assert_allclose(r["B"] @ r["B"].conj().T, Bv @ Bv.conj().T, atol=1e-10)


def test_full_rank_is_exact():
    rng = np.random.default_rng(5)
    X = crandn(rng, 10, 4, 6)          # nsc=10, gs=5 -> two groups
    r, Ht, Xh = _fit(X, 5, 4, 6, 5, 2)
    assert metrics.nmse(X, Xh) < 1e-28


def test_planted_low_rank_recovered():
    rng = np.random.default_rng(6)
    X, A0, B0, C0, G0 = synthgen.planted_tucker(rng, 8, 16, 40, 12, 3, 5, 4)
    r, Ht, Xh = _fit(X, 12, 3, 5, 4, 3)
    assert metrics.nmse(X, Xh) < 1e-24
    np.testing.assert_allclose(r["A"] @ r["A"].conj().T, A0 @ A0.conj().T, atol=1e-11)
    np.testing.assert_allclose(r["B"] @ r["B"].conj().T, B0 @ B0.conj().T, atol=1e-11)
    # compressed channels agree up to the unitary freedom: Ht Ht^* spectra per subcarrier
    Ht0 = tucker.compressed_channels(C0, G0, 12)
    np.testing.assert_allclose(np.linalg.svd(Ht, compute_uv=False),
                               np.linalg.svd(Ht0, compute_uv=False), rtol=1e-9, atol=1e-10)


def test_generator_small_config_is_exactly_representable():
    cfg = synthgen.CONFIGS["small"]
    X = synthgen.make_channel(cfg)
    for Xg in tucker.group_tensors(X, cfg.group_size):
        for mode in range(3):
            s = np.linalg.svd(tensor.unfold(Xg, mode), compute_uv=False)
            assert np.sum(s > 1e-9 * s[0]) <= cfg.n_paths
    r, Ht, Xh = _fit(X, cfg.group_size, cfg.m, cfg.n, cfg.p, cfg.iters)
    assert metrics.nmse(X, Xh) < 1e-24


def _lossy_case():
    rng = np.random.default_rng(7)
    X = crandn(rng, 30, 6, 10)
    return X, 8, 3, 4, 3


def test_factors_orthonormal():
    X, gs, m, n, p = _lossy_case()
    r, _, _ = _fit(X, gs, m, n, p, 4)
    assert np.abs(r["A"].conj().T @ r["A"] - np.eye(m)).max() < 1e-13
    assert np.abs(r["B"].conj().T @ r["B"] - np.eye(n)).max() < 1e-13
    starts, sizes = tucker.group_layout(30, gs)
    for s0, sz in zip(starts, sizes):
        Cg = r["C"][s0:s0 + sz, :min(p, sz)]
        assert np.abs(Cg.conj().T @ Cg - np.eye(Cg.shape[1])).max() < 1e-13


def test_objective_monotone_and_decreasing():
    X, gs, m, n, p = _lossy_case()
    r, _, _ = _fit(X, gs, m, n, p, 10)
    tr = r["trace"]
    assert len(tr) == 1 + 3 * 10
    assert np.all(np.diff(tr) <= 1e-12 * r["norm2_X"])
    assert tr[-1] < tr[0] * (1 - 1e-3)


def test_optimal_core_identity():
    # ||X - Xhat||^2 = ||X||^2 - ||G||^2 at the optimal core (equation "min-max substitite")
    X, gs, m, n, p = _lossy_case()
    r, _, Xh = _fit(X, gs, m, n, p, 3)
    lhs = np.sum(np.abs(X - Xh) ** 2)
    rhs = tensor.norm2(X) - tensor.norm2(r["G"])
    assert abs(lhs - rhs) < 1e-11 * tensor.norm2(X)
    assert abs(lhs - r["trace"][-1]) < 1e-11 * tensor.norm2(X)


def test_updates_are_block_maximisers():
    # each factor update maximises g over its block: random orthonormal competitors and
    # small unitary perturbations never beat it
    X, gs, m, n, p = _lossy_case()
    Xgs = tucker.group_tensors(X, gs)
    rng = np.random.default_rng(8)
    A, Bt, Cs = tucker.hosvd_init(Xgs, m, n, p)
    A1, _ = tucker.update_A(Xgs, Bt, Cs, m)
    f1 = tucker.objective(Xgs, A1, Bt, Cs)
    B1, _ = tucker.update_B(Xgs, A1, Cs, n)
    f2 = tucker.objective(Xgs, A1, B1, Cs)
    for _ in range(20):
        Ar = synthgen.random_unitary(rng, X.shape[1], m)
        assert tucker.objective(Xgs, Ar, Bt, Cs) >= f1 - 1e-12
        Br = synthgen.random_unitary(rng, X.shape[2], n)
        assert tucker.objective(Xgs, A1, Br, Cs) >= f2 - 1e-12
        K = crandn(rng, m, m) * 1e-3
        Ap = A1 @ np.linalg.qr(np.eye(m) + K - K.conj().T)[0]
        Kn = synthgen.random_unitary(rng, X.shape[1], X.shape[1])
        Ap2 = np.linalg.qr(A1 + 1e-3 * Kn[:, :m])[0]
        assert tucker.objective(Xgs, Ap2, Bt, Cs) >= f1 - 1e-12
        assert abs(tucker.objective(Xgs, Ap, Bt, Cs) - f1) < 1e-9   # same subspace


def test_tensor_form_matches_matrix_form():
    # Xhat from G x1 A x2 conj(B) x3 C equals A Ht_s B^* slice by slice
    X, gs, m, n, p = _lossy_case()
    r, Ht, Xh = _fit(X, gs, m, n, p, 2)
    for s in range(X.shape[0]):
        np.testing.assert_allclose(Xh[s], r["A"] @ Ht[s] @ r["B"].conj().T, atol=1e-12)


def test_warm_start_resume_equals_uninterrupted():
    X, gs, m, n, p = _lossy_case()
    full = tucker.fit(X, gs, m, n, p, 6)
    half = tucker.fit(X, gs, m, n, p, 3)
    rest = tucker.fit(X, gs, m, n, p, 3, warm=half)
    np.testing.assert_allclose(rest["trace"][1:], full["trace"][10:], rtol=1e-10)
    np.testing.assert_allclose(rest["A"] @ rest["A"].conj().T,
                               full["A"] @ full["A"].conj().T, atol=1e-9)


# ----------------------------------------------------------------------------------------
# Section 3.3 storage: Table 1


def test_table1_storage_ratios():
    fns = dict(individual=metrics.storage_ratio_individual, shared=metrics.storage_ratio_shared,
               groupwise=metrics.storage_ratio_groupwise)
    rows = 0
    with open(os.path.join(GOLDEN, "table1_storage.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            M, N, P, K, m, n, p, model, rs = line.split()
            val = fns[model](21, int(K), int(M), int(N), int(P), int(m), int(n), int(p))
            assert round(val, 4) == float(rs), (line, val)
            rows += 1
    assert rows == 12


def test_subcarrier_group_storage_ratio():
    # Pinned through the Individual and Shared formulas, whose values the 12 rows of Table 1
    # fix (test above).  One channel compressed as a single group of all its subcarriers is
    # the Individual model with J = K = 1 and P = Nsc.
    for nr, nt, nsc, m, n, p in ((4, 32, 64, 4, 8, 4), (8, 64, 12, 8, 16, 12), (16, 256, 401, 12, 32, 150)):
        one = metrics.storage_ratio_subcarrier_groups(nr, nt, nsc, nsc, m, n, p)
        assert abs(one - metrics.storage_ratio_individual(1, 1, nr, nt, nsc, m, n, p)) < 1e-12 * one
    # Equal groups of gs subcarriers share A and B as the Shared model's K = Nsc / gs tensors
    # of P = gs slices do (J = 1).
    for nr, nt, gs, G, m, n, p in ((4, 32, 16, 4, 4, 8, 4), (8, 64, 12, 273, 8, 16, 12),
                                   (16, 256, 12, 273, 12, 32, 12), (8, 128, 12, 136, 8, 24, 5)):
        val = metrics.storage_ratio_subcarrier_groups(nr, nt, gs * G, gs, m, n, p)
        ref = metrics.storage_ratio_shared(1, G, nr, nt, gs, m, n, p)
        assert abs(val - ref) < 1e-12 * ref, (val, ref)
    # a short last group keeps p_g = min(p, size) slices: 64 subcarriers in groups of 24 leave
    # a group of 16, which with p = 20 keeps 16
    val = metrics.storage_ratio_subcarrier_groups(4, 32, 64, 24, 4, 8, 20)
    full = metrics.storage_ratio_shared(1, 2, 4, 32, 24, 4, 8, 20)  # the two whole groups
    stored_two = 4 * 32 * 48 / full
    last = 4 * 8 * 16 + 16 * 16
    assert abs(val - 4 * 32 * 64 / (stored_two + last)) < 1e-12 * val


# ----------------------------------------------------------------------------------------
# Section 2.2 / 3.3: SINR


def _brute_2x2(H, sigma2):
    """The SINR chain for a 2x2 channel with explicit 2x2 formulas (no LAPACK)."""
    G = H.conj().T @ H
    a, c, b = G[0, 0].real, G[1, 1].real, G[0, 1]
    disc = math.sqrt(((a - c) / 2) ** 2 + abs(b) ** 2)
    lams = [(a + c) / 2 + disc, (a + c) / 2 - disc]
    P = np.zeros((2, 2), dtype=complex)
    for j, lam in enumerate(lams):
        v = np.array([b, lam - a]) if abs(b) > 1e-300 else np.eye(2)[j]
        P[:, j] = v / math.sqrt(abs(v[0]) ** 2 + abs(v[1]) ** 2)
    HP = H @ P
    Q = HP @ HP.conj().T + sigma2 * np.eye(2)
    det = Q[0, 0] * Q[1, 1] - Q[0, 1] * Q[1, 0]
    Qi = np.array([[Q[1, 1], -Q[0, 1]], [-Q[1, 0], Q[0, 0]]]) / det
    W = Qi @ HP
    out = []
    for r in range(2):
        w, h = W[:, r], HP[:, r]
        s = abs(np.vdot(w, h)) ** 2
        out.append(s / (np.vdot(w, Q @ w).real - s))
    return np.array(out), np.sqrt(lams)


def test_sinr_brute_force_2x2():
    rng = np.random.default_rng(9)
    for _ in range(20):
        H = crandn(rng, 2, 2)
        s2 = 10 ** rng.uniform(-2, 1)
        ref, sig = _brute_2x2(H, s2)
        got = sinr.sinr(H[None], [s2], 2)[0, 0]
        np.testing.assert_allclose(got, ref, rtol=1e-10)
        np.testing.assert_allclose(got, sig ** 2 / s2, rtol=1e-10)


def test_sinr_closed_form_general_shapes():
    rng = np.random.default_rng(10)
    for (M, N, ns) in ((4, 8, 2), (8, 16, 4), (12, 32, 8), (8, 64, 4)):
        H = crandn(rng, 5, M, N)
        s2 = [0.01, 0.3, 3.0]
        np.testing.assert_allclose(sinr.sinr(H, s2, ns), sinr.sinr_closed_form(H, s2, ns),
                                   rtol=1e-9)


def test_mmse_identity_any_precoder():
    # SINR_r = 1 / [(I + (HP)^* HP / s2)^{-1}]_rr - 1 for any precoder P
    rng = np.random.default_rng(11)
    H = crandn(rng, 6, 10)
    P = synthgen.random_unitary(rng, 10, 3)
    s2 = 0.2
    got = sinr.mmse_sinr(H, P, s2)
    HP = H @ P
    E = np.linalg.inv(np.eye(3) + HP.conj().T @ HP / s2)
    np.testing.assert_allclose(got, 1.0 / np.real(np.diagonal(E)) - 1.0, rtol=1e-10)


def test_push_through_sinr_gradient_against_finite_differences():
    # with X = (HV^H HV + s2 I)^{-1}, SINR_j = 1 / (s2 X_jj) - 1 (the identity above), so the
    # gradient of sum_j g_j SINR_j in HV (convention dl = Re sum conj(Gbar) dHV) is
    # 2 HV sum_j g_j / (s2 X_jj^2) x_j x_j^H, x_j = X e_j: checked by central differences of the
    # oracle's MMSE chain with the identity precoder (so that H P = HV)
    rng = np.random.default_rng(23)
    m, ns, s2 = 6, 3, 0.4
    HV = crandn(rng, m, ns)
    g = rng.standard_normal(ns)
    P = np.eye(ns)

    def loss(h):
        return float(g @ sinr.mmse_sinr(h, P, s2))

    X = np.linalg.inv(HV.conj().T @ HV + s2 * np.eye(ns))
    gm = sum(g[j] / (s2 * np.real(X[j, j]) ** 2) * np.outer(X[:, j], X[:, j].conj())
             for j in range(ns))
    grad = 2.0 * HV @ gm
    fd = np.zeros_like(HV)
    eps = 1e-6
    for a in range(m):
        for b in range(ns):
            for unit in (1.0, 1j):
                d = np.zeros_like(HV)
                d[a, b] = eps * unit
                fd[a, b] += unit * (loss(HV + d) - loss(HV - d)) / (2 * eps)
    np.testing.assert_allclose(fd, grad, rtol=0, atol=1e-6 * np.abs(grad).max())


def test_factor_cancellation_compressed_equals_full():
    # SINR of A Ht B^* with orthonormal A, B equals the SINR of Ht (Section 3.3)
    rng = np.random.default_rng(12)
    A = synthgen.random_unitary(rng, 16, 6)
    B = synthgen.random_unitary(rng, 40, 10)
    Ht = crandn(rng, 7, 6, 10)
    H = A[None] @ Ht @ B.conj().T[None]
    s2 = [0.05, 1.0]
    np.testing.assert_allclose(sinr.sinr(H, s2, 4), sinr.sinr(Ht, s2, 4), rtol=1e-9)


def test_woodbury_and_compressed_filter():
    rng = np.random.default_rng(13)
    A = synthgen.random_unitary(rng, 16, 6)
    B = synthgen.random_unitary(rng, 40, 10)
    Ht = crandn(rng, 6, 10)
    H = A @ Ht @ B.conj().T
    s2 = 0.3
    Pt, _ = sinr.svd_precoder(Ht, 3)
    P = B @ Pt                                   # V = B Vt (equation "compressed pre")
    HP = H @ P
    Q = HP @ HP.conj().T + s2 * np.eye(16)
    HV = Ht @ Pt
    Qt = HV @ HV.conj().T + s2 * np.eye(6)
    np.testing.assert_allclose(sinr.woodbury_inverse(A, Qt, s2), np.linalg.inv(Q), atol=1e-10)
    W = np.linalg.solve(Q, HP)
    np.testing.assert_allclose(A @ sinr.compressed_filter(Ht, Pt, s2), W, atol=1e-10)


def test_metrics():
    a = np.array([10.0, 100.0])
    b = np.array([10.0, 10.0])
    np.testing.assert_allclose(metrics.db_error(a, b), [0.0, 10.0])
    assert abs(metrics.mean_relative_error(a, b) - 0.45) < 1e-15
    X = np.ones((2, 2, 2))
    assert abs(metrics.nmse(X, 0.9 * X) - 0.01) < 1e-15


# ----------------------------------------------------------------------------------------
# input generator


def test_generator_is_deterministic_and_unit_power():
    cfg = synthgen.CONFIGS["small"]
    a = synthgen.make_channel(cfg)
    b = synthgen.make_channel(cfg)
    assert a.tobytes() == b.tobytes()
    c = synthgen.make_channel(cfg, channel=1)
    assert not np.array_equal(a, c)
    powers = [np.mean(np.abs(synthgen.make_channel(cfg, ch)) ** 2) for ch in range(40)]
    assert 0.6 < np.mean(powers) < 1.4


def test_generator_torch_matches_numpy():
    import torch

    cfg = synthgen.CONFIGS["small"]
    pp = synthgen.draw_paths(synthgen.channel_rng(0, 3), cfg.n_paths, cfg.k_db)
    a = synthgen.build_channel(pp, cfg.nr, cfg.nt, cfg.nsc)
    b = synthgen.build_channel_torch(pp, cfg.nr, cfg.nt, cfg.nsc, "cpu").numpy()
    np.testing.assert_allclose(a, b, atol=1e-12)


# ----------------------------------------------------------------------------------------
# Channels at general coefficient vectors (mode 3 = path / delay submatrices)


def test_combine_selector_rows_give_slices_and_compressed_channels():
    # u_t = e_s picks the slice H_s (equation "channel submatrices, tensor") and the compressed
    # channel Ht_s of equation "compressed matrix SINR reduction" with a selector c
    rng = np.random.default_rng(71)
    X, A, B, C, G = synthgen.planted_tucker(rng, 4, 6, 11, 4, 3, 4, 3)
    eye = np.eye(11, dtype=np.complex128)
    np.testing.assert_array_equal(tucker.combine_full(X, eye), X)
    np.testing.assert_allclose(tucker.combine_compressed(C, G, 4, eye),
                               tucker.compressed_channels(C, G, 4), rtol=0, atol=1e-14)


def test_combine_exact_model_factors_cancel():
    # on a tensor that the groupwise model holds exactly (built slice by slice by the
    # generator), combining the submatrices by any rows equals A Ht(t) B^H with Ht(t) combined
    # from the factors: the identity behind equation "compressed matrix SINR reduction"
    rng = np.random.default_rng(72)
    X, A, B, C, G = synthgen.planted_tucker(rng, 5, 7, 23, 6, 3, 4, 4)  # ragged last group
    U = crandn(rng, 9, 23)
    H = tucker.combine_full(X, U)
    Ht = tucker.combine_compressed(C, G, 6, U)
    assert Ht.shape == (9, 3, 4)
    for t in range(9):
        np.testing.assert_allclose(A @ Ht[t] @ B.conj().T, H[t], rtol=0,
                                   atol=1e-12 * np.abs(H[t]).max())
    # and the combination is linear in the rows
    U2 = crandn(rng, 9, 23)
    np.testing.assert_allclose(tucker.combine_compressed(C, G, 6, U + 2j * U2),
                               Ht + 2j * tucker.combine_compressed(C, G, 6, U2), atol=1e-12)


def test_submatrix_weights_rebuild_the_ofdm_channel():
    # combining the ray submatrices with u_t[l] = exp(-j 2 pi t tau_l / N) gives the channel
    # at subcarrier t of the same rays (the channel-submatrix equation of Section 2.2), which
    # build_channel assembles independently
    pp = synthgen.draw_submatrix_paths(synthgen.channel_rng(9, 0), n_clusters=3, rays=4)
    X = synthgen.build_submatrices(pp, 4, 8)
    assert X.shape == (13, 4, 8)
    H = tucker.combine_full(X, synthgen.submatrix_weights(pp, 16, 16))
    np.testing.assert_allclose(H, synthgen.build_channel(pp, 4, 8, 16), atol=1e-12)
