"""The sparse embedding matrix of Definition 2.1 and the products the method forms.

S in R^{s x n} has, in each column i, the value signs[i,g]/sqrt(gamma) at row
rows[i,g] (g < gamma) and zeros elsewhere. Products are taken with scipy.sparse as a
library primitive; no blocking or reordering beyond the definition.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def embedding_matrix(rows: np.ndarray, signs: np.ndarray, s: int) -> sp.csr_matrix:
    """S (s x n) as a sparse matrix (Definition 2.1)."""
    n, gamma = rows.shape
    vals = signs.astype(np.float64).ravel() * (1.0 / np.sqrt(float(gamma)))
    cols = np.repeat(np.arange(n), gamma)
    return sp.csr_matrix((vals, (rows.ravel().astype(np.int64), cols)), shape=(s, n))


def dense_embedding(rows, signs, s) -> np.ndarray:
    return embedding_matrix(rows, signs, s).toarray()


def right_sketch(a: np.ndarray, rows: np.ndarray, signs: np.ndarray, s: int) -> np.ndarray:
    """C = A S^T (Algorithm 1; Algorithm 3 names it A-tilde):
    column j of C sums sign/sqrt(gamma) * A[:, i] over the columns i that S maps to j."""
    S = embedding_matrix(rows, signs, s)
    return np.asarray((S @ a.T).T)


def left_sketch(rows: np.ndarray, signs: np.ndarray, s: int, x: np.ndarray) -> np.ndarray:
    """S X for a tall X (n x k): W = S C and C~ = Phi C (Algorithm 1),
    A^ = Phi A~ (Algorithm 3)."""
    S = embedding_matrix(rows, signs, s)
    return np.asarray(S @ x)
