"""Pins for the oracle's QR with column pivoting selection (CPU only).

QRCP is Alg. 1's alternative to LUPP for both selections (§5.3).  Its pivots are
checked against LAPACK's geqp3 (through scipy) and against brute force: step t picks the
candidate that maximises the volume det Gram(X[:, P_t + [j]]).
"""
import itertools

import numpy as np
import pytest
import scipy.linalg as sl

from oracle.icur import exact_relative_error, iterative_cur
from oracle.qrcp import qrcp_pivots
from paper_2509_21963_amd import workloads as W


@pytest.mark.parametrize("seed,shape", [(0, (12, 80)), (1, (35, 500)), (2, (8, 8)), (3, (20, 21))])
def test_matches_lapack_geqp3(seed, shape):
    rng = np.random.default_rng(seed)
    K, N = shape
    X = rng.standard_normal((K, N)) * np.exp(rng.standard_normal(N))[None, :]
    ours = qrcp_pivots(X.T, K)
    lapack = sl.qr(X, pivoting=True, mode="r")[1][:K]
    assert ours == lapack.tolist()


@pytest.mark.parametrize("seed", range(5))
def test_matches_brute_force_volumes(seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((4, 9))
    ours = qrcp_pivots(X.T, 4)
    P = []
    for t in range(4):
        vol = {j: np.linalg.det(X[:, P + [j]].T @ X[:, P + [j]]) for j in range(9) if j not in P}
        P.append(max(vol, key=lambda j: (vol[j], -j)))
    assert ours == P


def test_exclusions_ties_and_early_stop():
    rng = np.random.default_rng(7)
    X = rng.standard_normal((6, 40))
    ex = [5, 9, 33]
    got = qrcp_pivots(X.T, 6, exclude=ex)
    keep = [j for j in range(40) if j not in ex]
    sub = qrcp_pivots(X[:, keep].T, 6)
    assert got == [keep[j] for j in sub]
    # equal norms: the lowest index wins
    E = np.eye(3)
    assert qrcp_pivots(np.hstack([E, E]).T, 3) == [0, 1, 2]
    # only three nonzero candidates: the selection ends after them
    Z = np.zeros((5, 10))
    Z[:, [2, 4, 7]] = rng.standard_normal((5, 3))
    assert sorted(qrcp_pivots(Z.T, 5)) == [2, 4, 7]


def test_margins():
    X = np.diag([3.0, 2.0, 1.0])
    piv, marg = qrcp_pivots(X.T, 3, return_margins=True)
    assert piv == [0, 1, 2]
    np.testing.assert_allclose(marg, [1 - 2 / 3, 1 - 1 / 2, 1.0])


@pytest.mark.parametrize("kind", [0, 1])
def test_iterative_cur_with_qrcp_recovers_exactly_low_rank(kind):
    A = W.exact_lowrank(300, 200, 24, seed=4)
    out = iterative_cur(A, 1e-10, 8, kind=kind, seed=2, selection="qrcp")
    assert out["rank"] == 24
    assert exact_relative_error(A, out["I"], out["J"], out["U"]) < 1e-12


def test_iterative_cur_with_qrcp_meets_tolerance_like_lupp():
    # §5.3: QRCP and LUPP selections give IterativeCUR the same quality
    A, _ = W.planted_geometric(400, 300, 20.0, seed=3)
    q = iterative_cur(A, 1e-6, 10, seed=1, selection="qrcp")
    l = iterative_cur(A, 1e-6, 10, seed=1)
    eq = exact_relative_error(A, q["I"], q["J"], q["U"])
    assert q["rho"] <= 1e-6 and 0.5 <= q["rho"] / eq <= 2.0
    assert abs(q["rank"] - l["rank"]) <= 10
