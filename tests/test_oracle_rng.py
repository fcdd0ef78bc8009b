"""Pins of the oracle's SplitMix64 and of the Definition 2.1 index draw."""
import os

import numpy as np
import pytest

from oracle import rng


def _golden(golden_dir):
    with open(os.path.join(golden_dir, "splitmix64_seed1234567.txt")) as f:
        return [int(t) for t in f.read().split("\n") if t and not t.startswith("#")]


def test_splitmix64_known_answer(golden_dir):
    assert rng.splitmix64_outputs(1234567, 5) == _golden(golden_dir)


def test_counter_form_matches_stream(golden_dir):
    # output a of the stream is fmix(seed + a * golden): the counter-based form
    g = _golden(golden_dir)
    assert [rng.stream_output(1234567, a) for a in range(1, 6)] == g


@pytest.mark.parametrize("n,s,gamma,seed", [(50, 8, 8, 1), (200, 16, 4, 7), (64, 64, 1, 3), (37, 5, 3, 2**64 - 1)])
def test_vectorised_draw_equals_loop(n, s, gamma, seed):
    r1, g1 = rng.sketch_indices(seed, n, s, gamma)
    r2, g2 = rng.sketch_indices_loop(seed, n, s, gamma)
    assert np.array_equal(r1, r2) and np.array_equal(g1, g2)


def test_definition_2_1_structure():
    # gamma distinct rows per column, all in range, signs +-1
    rows, signs = rng.sketch_indices(11, 5000, 64, 8)
    assert rows.shape == (5000, 8) and rows.dtype == np.int32
    assert rows.min() >= 0 and rows.max() < 64
    srt = np.sort(rows, axis=1)
    assert (np.diff(srt, axis=1) > 0).all()
    assert set(np.unique(signs)) == {-1, 1}


def test_uniform_rows_and_fair_signs():
    # chi-square of row counts and a binomial check of the signs
    n, s, gamma = 40000, 128, 8
    rows, signs = rng.sketch_indices(5, n, s, gamma)
    counts = np.bincount(rows.ravel(), minlength=s)
    expect = n * gamma / s
    chi2 = float(((counts - expect) ** 2 / expect).sum())
    # 127 dof: mean 127, sd ~16; allow 5 sd. (Without replacement lowers the variance.)
    assert chi2 < 127 + 5 * 16
    frac = (signs == 1).mean()
    assert abs(frac - 0.5) < 5 * 0.5 / np.sqrt(signs.size)


def test_gamma_equal_s_is_a_permutation():
    rows, _ = rng.sketch_indices(9, 100, 6, 6)
    assert (np.sort(rows, axis=1) == np.arange(6)).all()


def test_invalid_gamma():
    with pytest.raises(ValueError):
        rng.sketch_indices(1, 10, 4, 5)


def test_probe_uniforms_are_the_counter_stream():
    # the vectorised draw equals the plain definition, element by element
    seed, n, N = 987654321, 7, 3
    U1, U2 = rng.probe_uniforms(seed, n, N)
    for j in range(N):
        key = rng.stream_output(seed ^ rng.PROBE_DOMAIN, j + 1)
        for i in range(n):
            u1 = rng.stream_output(key, 2 * i + 1)
            u2 = rng.stream_output(key, 2 * i + 2)
            assert U1[j, i] == ((u1 >> 11) + 1) * 2.0 ** -53
            assert U2[j, i] == (u2 >> 11) * 2.0 ** -53
    assert U1.min() > 0.0 and U1.max() <= 1.0 and U2.min() >= 0.0 and U2.max() < 1.0


def test_gaussian_probes_are_standard_normal():
    # moments and the Kolmogorov-Smirnov distance of 200 000 draws against N(0, 1)
    from scipy import stats
    g = rng.gaussian_probes(2405, 2000, 100).ravel()
    assert abs(g.mean()) < 5 / np.sqrt(g.size)
    assert abs(g.var() - 1.0) < 5 * np.sqrt(2.0 / g.size)
    assert stats.kstest(g, "norm").pvalue > 1e-3
    # distinct seeds and the sketch domain give different draws
    assert not np.array_equal(rng.gaussian_probes(1, 50, 2), rng.gaussian_probes(2, 50, 2))
