"""Pins for the oracle's random sketch operator (CPU only)."""
import itertools

import numpy as np
import pytest
from scipy import stats

from oracle.rng import (gaussian_G, make_G, philox4x32_10, round_to_bf16,
                        sparse_sign_G, sparse_sign_pattern)


# Known-answer vectors published with the Random123 library for philox4x32 with 10
# rounds: (counter words, key words) -> output words.
PHILOX_KAT = [
    ((0x00000000, 0x00000000, 0x00000000, 0x00000000), (0x00000000, 0x00000000),
     (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff, 0xffffffff, 0xffffffff, 0xffffffff), (0xffffffff, 0xffffffff),
     (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
]


@pytest.mark.parametrize("ctr,key,expect", PHILOX_KAT)
def test_philox_known_answers(ctr, key, expect):
    out = philox4x32_10(*[np.array([v], dtype=np.uint64) for v in ctr], *key)
    assert tuple(int(o[0]) for o in out) == expect


def test_bf16_rounding_round_to_nearest_even():
    one = 1.0
    ulp = 2.0 ** -7                        # BF16 spacing just above 1
    cases = {
        one: one,
        one + ulp / 2: one,                # tie -> even (1.0)
        one + 3 * ulp / 2: one + 2 * ulp,  # tie -> even (1 + 2 ulp)
        one + ulp / 2 + 2 ** -20: one + ulp,   # above the tie -> up
        one + ulp / 4: one,
        -(one + 3 * ulp / 4): -(one + ulp),
        0.0: 0.0,
    }
    for x, want in cases.items():
        assert round_to_bf16(np.array([x]))[0] == want, x


def test_gaussian_values_are_bf16_and_standard_normal():
    G = gaussian_G(seed=123, c=64, m=4000)
    bits = G.astype(np.float32).view(np.uint32)
    assert np.all(bits & 0xFFFF == 0)                    # exactly representable in BF16
    assert np.all(G.astype(np.float32).astype(np.float64) == G)
    z = G.ravel()
    n = z.size
    assert abs(z.mean()) < 5.0 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5.0 * np.sqrt(2.0 / n) + 1e-4   # + BF16 rounding bias
    # distribution: BF16 rounding moves values by < 2^-8 relative, far below what a
    # Kolmogorov-Smirnov test at this n can see
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # entries are independent of position: different seeds and positions differ
    G2 = gaussian_G(seed=124, c=64, m=4000)
    assert np.mean(G == G2) < 0.01
    assert abs(np.corrcoef(G[0], G[1])[0, 1]) < 0.1


def test_gaussian_entry_depends_only_on_seed_row_and_column():
    G = gaussian_G(seed=7, c=10, m=50)
    H = gaussian_G(seed=7, c=20, m=80)
    assert np.array_equal(G, H[:10, :50])


@pytest.mark.parametrize("c,zeta", [(110, 8), (35, 8), (5, 8), (1, 8), (70, 3)])
def test_sparse_sign_columns_have_distinct_rows(c, zeta):
    rows, signs = sparse_sign_pattern(seed=9, c=c, m=3000, zeta=zeta)
    z = min(c, zeta)
    assert rows.shape == (3000, z)
    assert rows.min() >= 0 and rows.max() < c
    for r in rows:
        assert len(set(r.tolist())) == z
    assert set(np.unique(signs).tolist()) <= {-1.0, 1.0}
    G = sparse_sign_G(seed=9, c=c, m=3000, zeta=zeta)
    assert np.all(np.count_nonzero(G, axis=0) == z)
    assert np.all(np.abs(G[G != 0]) == 1.0)


def test_sparse_sign_rows_and_signs_are_uniform():
    c, zeta, m = 110, 8, 20000
    rows, signs = sparse_sign_pattern(seed=3, c=c, m=m, zeta=zeta)
    counts = np.bincount(rows.ravel(), minlength=c)
    chi2 = ((counts - m * zeta / c) ** 2 / (m * zeta / c)).sum()
    assert stats.chi2.sf(chi2, c - 1) > 1e-4
    assert abs(signs.mean()) < 5.0 / np.sqrt(signs.size)


def test_floyd_sampling_gives_uniform_subsets():
    # c = 5, zeta = 2: each of the 10 subsets should appear with probability 1/10
    rows, _ = sparse_sign_pattern(seed=11, c=5, m=50000, zeta=2)
    keys = [tuple(sorted(r)) for r in rows.tolist()]
    subsets = list(itertools.combinations(range(5), 2))
    counts = np.array([keys.count(s) for s in subsets])
    chi2 = ((counts - 5000.0) ** 2 / 5000.0).sum()
    assert stats.chi2.sf(chi2, len(subsets) - 1) > 1e-4


def test_make_G_dispatch():
    assert np.array_equal(make_G(1, 4, 9, 0), gaussian_G(1, 4, 9))
    assert np.array_equal(make_G(1, 4, 9, 1), sparse_sign_G(1, 4, 9))
    with pytest.raises(ValueError):
        make_G(1, 4, 9, 3)
