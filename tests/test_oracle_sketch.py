"""Pins of the sparse embedding products (Definition 2.1, Algorithm 1)."""
import numpy as np
import pytest

from oracle import rng, sketch


def _column_of_s(rows, signs, i, s):
    """Column i of S read straight off the index draw."""
    col = np.zeros(s)
    g = rows.shape[1]
    for r, sg in zip(rows[i], signs[i]):
        col[r] += sg / np.sqrt(g)
    return col


def test_columns_have_unit_norm():
    rows, signs = rng.sketch_indices(3, 300, 32, 8)
    S = sketch.dense_embedding(rows, signs, 32)
    assert np.allclose((S * S).sum(axis=0), 1.0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("k,l", [(0, 5), (7, 2), (19, 19)])
def test_right_sketch_of_elementary_matrix(k, l):
    # (e_k e_l^T) S^T = e_k (S e_l)^T : one nonzero row holding column l of S.
    n, s = 20, 8
    rows, signs = rng.sketch_indices(4, n, s, 3)
    a = np.zeros((n, n))
    a[k, l] = 1.0
    c = sketch.right_sketch(a, rows, signs, s)
    want = np.zeros((n, s))
    want[k] = _column_of_s(rows, signs, l, s)
    assert np.array_equal(c, want)


def test_left_sketch_of_elementary_matrix():
    # S (e_l e_c^T) places column l of S into column c
    n, s = 30, 10
    rows, signs = rng.sketch_indices(6, n, s, 4)
    x = np.zeros((n, 3))
    x[11, 2] = 1.0
    y = sketch.left_sketch(rows, signs, s, x)
    want = np.zeros((s, 3))
    want[:, 2] = _column_of_s(rows, signs, 11, s)
    assert np.array_equal(y, want)


def test_right_sketch_brute_force():
    # C[r, j] = sum over (i, g) with rows[i, g] = j of signs[i, g] / sqrt(gamma) * A[r, i]
    n, s, gamma = 13, 5, 2
    rows, signs = rng.sketch_indices(8, n, s, gamma)
    a = np.random.default_rng(0).standard_normal((7, n))
    want = np.zeros((7, s))
    for r in range(7):
        for i in range(n):
            for g in range(gamma):
                want[r, rows[i, g]] += signs[i, g] / np.sqrt(gamma) * a[r, i]
    assert np.allclose(sketch.right_sketch(a, rows, signs, s), want, rtol=0, atol=1e-14)


def test_embedding_preserves_norms_on_average():
    # E ||S x||^2 = ||x||^2 for a fixed x (independent columns, unit norm, random signs)
    x = np.random.default_rng(1).standard_normal(400)
    vals = []
    for seed in range(200):
        rows, signs = rng.sketch_indices(1000 + seed, 400, 40, 4)
        vals.append(np.linalg.norm(sketch.left_sketch(rows, signs, 40, x[:, None])) ** 2)
    assert abs(np.mean(vals) / (x @ x) - 1.0) < 0.05


def test_embedding_matrix_entries_follow_the_draws():
    # column i of S holds sign(i, g) / sqrt(gamma) at row rows(i, g) for the gamma draws, and
    # nothing else (Definition 2.1); each column has unit norm since its rows are distinct
    rows = np.array([[0, 3], [2, 1], [3, 0]])
    signs = np.array([[1, -1], [-1, -1], [1, 1]], dtype=np.int8)
    S = sketch.embedding_matrix(rows, signs, 4).toarray()
    r = 1.0 / np.sqrt(2.0)
    want = np.array([[r, 0, r], [0, -r, 0], [0, -r, 0], [-r, 0, r]])
    assert np.array_equal(S, want)
    assert np.allclose(np.linalg.norm(S, axis=0), 1.0)
