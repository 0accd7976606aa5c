"""Pins for the oracle's LU-with-partial-pivoting index selection (CPU only)."""
import itertools

import numpy as np
import pytest
import scipy.linalg

from oracle.lupp import lupp_pivots


def lapack_pivot_order(T):
    """Pivot order of LAPACK getrf (via scipy) on T: replay its row interchanges."""
    _, piv = scipy.linalg.lu_factor(T, check_finite=False)
    perm = np.arange(T.shape[0])
    for i, p in enumerate(piv):
        perm[[i, p]] = perm[[p, i]]
    return perm[:min(T.shape)].tolist()


def brute_force_pivots(T, steps, exclude=()):
    """Step t picks the eligible row i maximising |det T([p_0..p_{t-1}, i], 0..t)|:
    the Schur-complement entry that partial pivoting compares equals that determinant
    divided by a factor common to all candidates."""
    N, K = T.shape
    chosen = []
    for t in range(min(steps, K)):
        best, arg = -1.0, None
        for i in range(N):
            if i in chosen or i in exclude:
                continue
            d = abs(np.linalg.det(T[np.ix_(chosen + [i], list(range(t + 1)))]))
            if d > best:
                best, arg = d, i
        if arg is None or best == 0.0:
            break
        chosen.append(arg)
    return chosen


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("shape", [(40, 7), (300, 55), (1000, 110), (64, 64)])
def test_matches_lapack_getrf(seed, shape):
    T = np.random.default_rng(seed).standard_normal(shape)
    piv, margins = lupp_pivots(T, shape[1], return_margins=True)
    ref = lapack_pivot_order(T)
    # blocked LAPACK rounds differently; compare up to the first near tie
    k = next((i for i, mg in enumerate(margins) if mg < 1e-8), len(piv))
    assert piv[:k] == ref[:k]
    assert k >= min(len(piv), 5)


@pytest.mark.parametrize("seed", range(20))
def test_matches_brute_force_determinants(seed):
    g = np.random.default_rng(100 + seed)
    N, K = int(g.integers(3, 9)), int(g.integers(1, 5))
    T = g.standard_normal((N, K))
    steps = int(g.integers(1, K + 1))
    excl = [int(x) for x in g.choice(N, size=int(g.integers(0, max(1, N - K + 1))), replace=False)]
    assert lupp_pivots(T, steps, exclude=excl) == brute_force_pivots(T, steps, excl)


def test_excluded_rows_are_never_chosen():
    T = np.random.default_rng(5).standard_normal((50, 10))
    first = lupp_pivots(T, 10)
    again = lupp_pivots(T, 10, exclude=first[:3])
    assert not set(first[:3]) & set(again)
    assert again == brute_force_pivots(T, 10, first[:3])


def test_ties_go_to_lowest_index():
    T = np.array([[1.0, 2.0], [-3.0, 0.5], [3.0, 1.0], [0.0, 0.0]])
    assert lupp_pivots(T, 1) == [1]
    assert lupp_pivots(np.ones((4, 1)), 1) == [0]


def test_stops_at_zero_pivot_and_exhaustion():
    assert lupp_pivots(np.zeros((5, 3)), 3) == []
    u = np.array([1.0, 2.0, 3.0, 4.0])
    T = np.outer(u, [1.0, -2.0, 0.5])          # rank one: one pivot, then exact zeros
    assert lupp_pivots(T, 3) == [3]
    assert lupp_pivots(np.eye(3), 3, exclude=[0, 1, 2]) == []
    assert len(lupp_pivots(np.random.default_rng(0).standard_normal((4, 6)), 6)) == 4


def test_steps_limit_and_margins():
    T = np.random.default_rng(8).standard_normal((200, 12))
    piv, mg = lupp_pivots(T, 5, return_margins=True)
    assert len(piv) == 5 and len(mg) == 5
    assert all(0.0 <= x <= 1.0 for x in mg)
    assert piv == lupp_pivots(T, 12)[:5]
