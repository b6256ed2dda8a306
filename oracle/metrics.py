"""Evaluation metrics (Section 4), FP64.  Test infrastructure only."""

from __future__ import annotations

import numpy as np

from .tucker import group_layout


def nmse(X: np.ndarray, Xhat: np.ndarray) -> float:
    """||X - Xhat||^2 / ||X||^2 as an explicit residual."""
    return float(np.sum(np.abs(X - Xhat) ** 2) / np.sum(np.abs(X) ** 2))


def db_error(sinr_a: np.ndarray, sinr_b: np.ndarray) -> np.ndarray:
    """|10 log10 SINR_a - 10 log10 SINR_b| elementwise."""
    return np.abs(10.0 * np.log10(sinr_a) - 10.0 * np.log10(sinr_b))


def mean_relative_error(sinr_full: np.ndarray, sinr_comp: np.ndarray) -> float:
    """e_c = mean of |(SINR - SINR~) / SINR| (equation "SINR error")."""
    return float(np.mean(np.abs((sinr_full - sinr_comp) / sinr_full)))


def storage_ratio_groupwise(J, K, M, N, P, m, n, p) -> float:
    """R_s of equation "compression ratio" (storage table of Section 3.3): the groupwise
    model keeps J^2 K cores and mode-3 factors, J K mode-1 factors and J mode-2 factors."""
    return (J * J * K * M * N * P) / (J * J * K * (m * n * p + P * p) + J * K * M * m + J * N * n)


def storage_ratio_individual(J, K, M, N, P, m, n, p) -> float:
    """Individual Tucker: every one of the J^2 K channels keeps all three factors."""
    return (J * J * K * M * N * P) / (J * J * K * (m * n * p + P * p + M * m + N * n))


def storage_ratio_shared(J, K, M, N, P, m, n, p) -> float:
    """Shared Tucker: one mode-1 and one mode-2 factor for the whole system."""
    return (J * J * K * M * N * P) / (J * J * K * (m * n * p + P * p) + M * m + N * n)


def storage_ratio_subcarrier_groups(nr, nt, nsc, gs, m, n, p) -> float:
    """Storage ratio of one channel compressed with subcarrier groups: A and B once,
    a core and a mode-3 factor per group (complex entries counted)."""
    starts, sizes = group_layout(nsc, gs)
    comp = nr * m + nt * n
    for sz in sizes:
        pg = min(p, sz)
        comp += m * n * pg + sz * pg
    return (nr * nt * nsc) / comp
