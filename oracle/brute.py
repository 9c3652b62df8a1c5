"""Dense brute-force definitions (numpy, FP64) used to pin the oracle.

TEST INFRASTRUCTURE ONLY (see :mod:`oracle`).

These follow the matrix formulation of the suite (Section 4): the mode-n
matricization, the Kronecker product and the Khatri-Rao product (Section
4.5), and MTTKRP as X_(n) times the Khatri-Rao product of the other
factors (Section 4.6, eq. mttkrp-init). They materialise the dense tensor,
so they only run on tiny shapes.

Reading of the garbled matricization shape (Section 4, which prints
X_(n) with the I_n axis last): X_(n) has I_n rows and prod_{k!=n} I_k
columns, because the product with the (prod_{k!=n} I_k) x R Khatri-Rao
matrix must conform and Alg. 6 returns an I x R matrix. Columns are ordered
with the lowest remaining mode fastest, which pairs with the eq. 's
reverse operand order U^(N) (.) ... (.) U^(1).
"""
from __future__ import annotations

from typing import Sequence

import numpy as np


def dense(dims: Sequence[int], inds, vals) -> np.ndarray:
    """Dense FP64 tensor of a COO list; repeated coordinates are summed."""
    X = np.zeros(tuple(int(d) for d in dims), dtype=np.float64)
    np.add.at(X, tuple(np.asarray(i, dtype=np.int64) for i in inds), np.asarray(vals, dtype=np.float64))
    return X


def unfold(X: np.ndarray, n: int) -> np.ndarray:
    """Mode-n matricization: rows = i_n, columns = the other modes with the
    lowest-numbered mode varying fastest."""
    return np.reshape(np.moveaxis(X, n, 0), (X.shape[n], -1), order="F")


def kronecker(U: np.ndarray, V: np.ndarray) -> np.ndarray:
    """Kronecker product (Section 4.5): block (i, j) of the result is U[i, j] * V."""
    I, J = U.shape
    K, L = V.shape
    out = np.empty((I * K, J * L), dtype=np.float64)
    for i in range(I):
        for j in range(J):
            out[i * K:(i + 1) * K, j * L:(j + 1) * L] = U[i, j] * V
    return out


def khatri_rao(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Khatri-Rao product (Section 4.5): column r is kron(a_r, b_r)."""
    if A.shape[1] != B.shape[1]:
        raise ValueError("Khatri-Rao operands need the same number of columns")
    cols = [kronecker(A[:, r:r + 1], B[:, r:r + 1])[:, 0] for r in range(A.shape[1])]
    return np.stack(cols, axis=1) if cols else np.zeros((A.shape[0] * B.shape[0], 0))


def khatri_rao_chain(mats) -> np.ndarray:
    out = np.asarray(mats[0], dtype=np.float64)
    for m in mats[1:]:
        out = khatri_rao(out, np.asarray(m, dtype=np.float64))
    return out


def mttkrp_dense(X: np.ndarray, factors, n: int) -> np.ndarray:
    """eq. mttkrp-init: X_(n) (U^(N) (.) ... (.) U^(n+1) (.) U^(n-1) (.) ... (.) U^(1))."""
    others = [np.asarray(factors[k], dtype=np.float64) for k in reversed(range(X.ndim)) if k != n]
    if not others:
        raise ValueError("order-1 tensors have no Khatri-Rao operand")
    return unfold(X, n) @ khatri_rao_chain(others)


def mttkrp_dense_c_order(X: np.ndarray, factors, n: int) -> np.ndarray:
    """The same product with a C-order unfolding (last mode fastest) paired with
    the forward operand order U^(1) (.) ... (.) U^(N)."""
    others = [np.asarray(factors[k], dtype=np.float64) for k in range(X.ndim) if k != n]
    Xn = np.moveaxis(X, n, 0).reshape(X.shape[n], -1)
    return Xn @ khatri_rao_chain(others)


def cp_full(factors) -> np.ndarray:
    """Dense rank-R CP tensor sum_r a^(1)_r o ... o a^(N)_r, built by outer products."""
    R = factors[0].shape[1]
    X = 0.0
    for r in range(R):
        t = np.asarray(factors[0][:, r], dtype=np.float64)
        for f in factors[1:]:
            t = np.multiply.outer(t, np.asarray(f[:, r], dtype=np.float64))
        X = X + t
    return X
