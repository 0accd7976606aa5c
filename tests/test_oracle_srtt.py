"""Pins for the SRTT sketch operator (CPU only).

§3.4 names subsampled randomized trigonometric transforms as the cheaper sketch for very
large m.  The oracle's operator is G = sqrt(m/c) R F D with F the orthonormal DCT-II,
written from the cosine definition; it is pinned against scipy's FFT-based DCT, against
orthogonality of the full transform, and by the statistics of its random parts.
"""
import numpy as np
import pytest
import scipy.fft as sfft
from scipy import stats

from oracle.icur import exact_relative_error, iterative_cur
from oracle.rng import g_scale, make_G, srtt_G, srtt_rows, srtt_signs
from paper_2509_21963_amd import workloads as W


@pytest.mark.parametrize("m,c,seed", [(97, 11, 3), (1000, 55, 0), (4096, 35, 9), (40000, 110, 1)])
def test_matches_fft_dct_of_signed_input(m, c, seed):
    x = np.random.default_rng(seed).standard_normal((m, 3))
    G = srtt_G(seed, c, m)
    y = sfft.dct(srtt_signs(seed, m)[:, None] * x, type=2, norm="ortho", axis=0)
    want = y[srtt_rows(seed, c, m)] * np.sqrt(m / c)
    np.testing.assert_allclose(G @ x, want, rtol=0, atol=1e-11 * np.abs(x).sum(axis=0).max())


@pytest.mark.parametrize("m", [1, 2, 7, 64, 300])
def test_full_transform_is_orthogonal(m):
    G = srtt_G(5, m, m)
    np.testing.assert_allclose(G @ G.T, np.eye(m), atol=1e-12)


def test_rows_are_distinct_sorted_and_uniform():
    m, c = 50, 10
    counts = np.zeros(m)
    for seed in range(2000):
        r = srtt_rows(seed, c, m)
        assert len(r) == c and len(set(r.tolist())) == c
        assert np.all(np.diff(r) > 0) and r.min() >= 0 and r.max() < m
        counts[r] += 1
    exp = 2000 * c / m
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert stats.chi2.sf(chi2, m - 1) > 1e-4
    assert len(srtt_rows(0, 30, 30)) == 30


def test_signs_are_balanced():
    d = srtt_signs(8, 100000)
    assert set(np.unique(d).tolist()) == {-1.0, 1.0}
    assert abs(d.mean()) < 5.0 / np.sqrt(d.size)


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_sketch_scale_preserves_norms_in_expectation(kind):
    # E ||G x||^2 = g_scale^2 ||x||^2 over the operator's randomness
    m, c = 400, 22
    x = np.random.default_rng(2).standard_normal(m)
    vals = [np.sum((make_G(s, c, m, kind) @ x) ** 2) for s in range(300)]
    ratio = np.mean(vals) / (g_scale(kind, c) ** 2 * np.sum(x ** 2))
    assert abs(ratio - 1.0) < 0.1


def test_iterative_cur_with_srtt():
    A = W.exact_lowrank(400, 300, 30, seed=5)
    out = iterative_cur(A, 1e-10, 10, kind=2, seed=4)
    assert out["rank"] == 30
    assert exact_relative_error(A, out["I"], out["J"], out["U"]) < 1e-12
    B, _ = W.planted_geometric(500, 400, 20.0, seed=2)
    out = iterative_cur(B, 1e-5, 16, kind=2, seed=1)
    err = exact_relative_error(B, out["I"], out["J"], out["U"])
    assert out["rho"] <= 1e-5 and 0.5 <= out["rho"] / err <= 2.0
