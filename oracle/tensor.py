"""Tensor primitives of Section 2.3 (Preliminaries on Tensors), complex128.

Test infrastructure only (see oracle/__init__.py).
"""

from __future__ import annotations

import numpy as np


def inner(X: np.ndarray, Y: np.ndarray) -> complex:
    """<X, Y> = sum over all indices of x * conj(y)  (Section 2.3, inner product)."""
    return complex(np.sum(X * np.conj(Y)))


def norm2(X: np.ndarray) -> float:
    """||X||^2 = <X, X>  (Section 2.3, induced norm), returned squared."""
    return float(np.real(inner(X, X)))


def unfold(X: np.ndarray, mode: int) -> np.ndarray:
    """Mode-n matricization X_(n) (Section 2.3).

    Rows are indexed by i_n; the remaining indices form the column index with the earlier
    mode varying fastest (the ordering the paper writes for mode 1: column i2 + I2 (i3 - 1)).
    """
    Xm = np.moveaxis(X, mode, 0)
    # after moveaxis the remaining axes keep their order; Fortran order makes the first of
    # them vary fastest
    return Xm.reshape(Xm.shape[0], -1, order="F")


def fold(M: np.ndarray, mode: int, shape) -> np.ndarray:
    """Inverse of unfold for a tensor of the given shape."""
    shape = list(shape)
    rest = [shape[i] for i in range(len(shape)) if i != mode]
    Xm = M.reshape([shape[mode]] + rest, order="F")
    return np.moveaxis(Xm, 0, mode)


def mode_product(X: np.ndarray, U: np.ndarray, mode: int) -> np.ndarray:
    """Mode-n tensor-matrix product X x_n U (Section 2.3).

    (X x_1 U)_{j, i2, i3} = sum_{i1} x_{i1, i2, i3} u_{j, i1}; U is J x I_n and is not
    conjugated.
    """
    Y = np.tensordot(U, X, axes=(1, mode))   # new axis first
    return np.moveaxis(Y, 0, mode)
