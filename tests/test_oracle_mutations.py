"""Planted mistakes in the oracle (on the CPU) must be caught by the pins.

Each case swaps one oracle function for a plausible wrong variant (a dropped conjugate, a
wrong index, a dropped term) and checks that the corresponding pin then fails.
"""

import numpy as np
import pytest

import synthgen
from oracle import metrics, sinr, tensor, tucker


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _planted_nmse():
    rng = np.random.default_rng(6)
    X, *_ = synthgen.planted_tucker(rng, 8, 16, 40, 12, 3, 5, 4)
    r = tucker.fit(X, 12, 3, 5, 4, 3)
    _, Xh = tucker.reconstruct(r["A"], r["B"], r["C"], r["G"], 12)
    return metrics.nmse(X, Xh)


def test_pins_catch_missing_conjugate_in_update_B(monkeypatch):
    def bad_update_B(Xgs, A, Cs, n):
        S = 0
        for Xg, Cg in zip(Xgs, Cs):
            M2 = tensor.unfold(tensor.mode_product(tensor.mode_product(Xg, A.T, 0),
                                                   Cg.conj().T, 2), 1)
            S = S + M2 @ M2.conj().T
        return tucker.top_eigvecs(S, n)

    # exact recovery alone does not see it (the mode-2 span survives a transposed A), but
    # the monotone-objective pin on a lossy tensor does
    rng = np.random.default_rng(7)
    X = crandn(rng, 30, 6, 10)
    assert np.diff(tucker.fit(X, 8, 3, 4, 3, 10)["trace"]).max() <= 1e-9
    monkeypatch.setattr(tucker, "update_B", bad_update_B)
    assert np.diff(tucker.fit(X, 8, 3, 4, 3, 10)["trace"]).max() > 1e-3


def test_pins_catch_transposed_core(monkeypatch):
    def bad_core(Xg, A, Bt, Cg):
        return tensor.mode_product(tensor.mode_product(tensor.mode_product(Xg, A.conj().T, 0),
                                                       Bt.T, 1), Cg.conj().T, 2)

    monkeypatch.setattr(tucker, "core", bad_core)
    assert _planted_nmse() > 1e-6


def test_pins_catch_dropped_signal_term_in_sinr(monkeypatch):
    def bad_mmse(H, P, sigma2):
        HP = H @ P
        M = H.shape[-2]
        Q = HP @ np.conj(np.swapaxes(HP, -1, -2)) + sigma2 * np.eye(M)
        W = np.linalg.solve(Q, HP)
        WH = np.conj(np.swapaxes(W, -1, -2))
        s = np.abs(np.diagonal(WH @ HP, axis1=-2, axis2=-1)) ** 2
        return s / np.real(np.diagonal(WH @ Q @ W, axis1=-2, axis2=-1))

    rng = np.random.default_rng(10)
    H = crandn(rng, 5, 8, 16)
    ok = np.allclose(sinr.sinr(H, [0.3], 4), sinr.sinr_closed_form(H, [0.3], 4), rtol=1e-9)
    assert ok
    monkeypatch.setattr(sinr, "mmse_sinr", bad_mmse)
    bad = np.allclose(sinr.sinr(H, [0.3], 4), sinr.sinr_closed_form(H, [0.3], 4), rtol=1e-3)
    assert not bad


def test_pins_catch_wrong_eigen_order(monkeypatch):
    def bad_top(M, r):
        w, V = np.linalg.eigh(0.5 * (M + M.conj().T))
        return V[:, :r], w[:r]                      # smallest instead of largest

    monkeypatch.setattr(tucker, "top_eigvecs", bad_top)
    assert _planted_nmse() > 1e-6
