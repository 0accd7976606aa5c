"""Pins for the oracle's IterativeCUR loop (CPU only).

Each test checks the oracle against something other than itself: the paper's worked
examples, identities the paper proves, closed forms, and library routines.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle.icur import (cur_residual, exact_relative_error, iterative_cur, pinv_svd,
                         risk_aware_factor, sketch_rows)
from oracle.rng import gaussian_G, sparse_sign_G, sparse_sign_pattern
from paper_2509_21963_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_sketch_rows():
    # c = floor(1.1 b) for the block sizes the paper and its workloads use
    assert [sketch_rows(b) for b in (1, 5, 32, 50, 64, 100, 128, 250, 500)] == \
        [1, 5, 35, 55, 70, 110, 140, 275, 550]


def test_example_3_1_worked_example():
    ex = json.load(open(os.path.join(GOLDEN, "example31.json")))
    A = np.array(ex["A"])
    g = np.array(ex["g"])[None, :]
    out = iterative_cur(A, 1e-300, 1, G=g, max_rank=2, record=True)
    np.testing.assert_allclose(out["X0"][0], ex["sketched_residual_before"], atol=1e-14)
    h1, h2 = out["history"]
    assert h1["J_k"] == [ex["iter1_column"]]
    assert h1["I_k"] == [ex["iter1_row"]]
    np.testing.assert_allclose(h1["S_col"][0], ex["sketched_residual_after_iter1"],
                               atol=1e-14)
    assert h2["J_k"] == [ex["iter2_column"]]
    assert out["status"] == "maxrank" and out["rank"] == 2


def test_dependent_selection_avoids_singular_core():
    # 2 x (n+1) matrix of §3.2: rows chosen from the chosen column give a nonzero core,
    # where independent norm-based choices give the singular core A(1,1) = 0.
    n, eta = 9, 0.1
    A = np.zeros((2, n + 1))
    A[0, 1:] = 1.0 / math.sqrt(n)
    A[1, 0] = 1.0 / math.sqrt(n) + eta
    out = iterative_cur(A, 1e-300, 1, G=np.ones((1, 2)), max_rank=1)
    assert out["J"] == [0] and out["I"] == [1]
    assert A[1, 0] != 0 and out["U"][0, 0] == pytest.approx(1.0 / A[1, 0])
    row_indep = int(np.argmax(np.linalg.norm(A, axis=1)))
    col_indep = int(np.argmax(np.linalg.norm(A, axis=0)))
    assert A[row_indep, col_indep] == 0.0


def _small_planted(seed=0, m=120, n=90):
    A, _ = W.planted_geometric(m, n, decades_per=12.0, seed=seed)
    return A


@pytest.mark.parametrize("kind", [0, 1])
def test_residuals_match_closed_forms_and_schur_zeros(kind):
    A = _small_planted(1, 200, 150)
    # tol well above the FP64 rounding floor and rank well below min(m, n), so every
    # residual entry is meaningful
    out = iterative_cur(A, 1e-6, 6, kind=kind, seed=4, record=True)
    assert out["rank"] < 120
    G = out["G"]
    I, J = [], []
    U = np.zeros((0, 0))
    scale = np.linalg.norm(A)
    eps = 2.0 ** -52
    X0 = out["X0"]
    for h in out["history"]:
        # S^row is the full residual of the previous iterate at the new columns; the
        # two evaluations differ by rounding of the product C U R(:,J_k), bounded
        # componentwise by (inner dims + 2) eps |C| |U| |R(:,J_k)|
        S_prev = cur_residual(A, I, J, U)
        Jk = h["J_k"]
        if J:
            bound = (2 * len(J) + 2) * eps * (np.abs(A[:, Jk]) + np.abs(A[:, J]) @ (
                np.abs(U) @ np.abs(A[np.ix_(I, Jk)])))
        else:
            bound = np.zeros_like(h["S_row"])
        assert np.all(np.abs(h["S_row"] - S_prev[:, Jk]) <= bound)
        I, J = I + h["I_k"], J + Jk
        U = pinv_svd(A[np.ix_(I, J)])
        S = cur_residual(A, I, J, U)
        # S^col is G times the full residual ("use GC_k from GA"), up to rounding of
        # the triple products (componentwise bound) and of the pseudo-inverse
        r, m = len(J), A.shape[0]
        CUR_abs = np.abs(A[:, J]) @ (np.abs(U) @ np.abs(A[I, :]))
        bound = (2 * r + m + 4) * eps * (np.abs(X0) + np.abs(X0[:, J]) @ (
            np.abs(U) @ np.abs(A[I, :])) + np.abs(G) @ (np.abs(A) + CUR_abs))
        assert np.all(np.abs(h["S_col"] - G @ S) <= bound)
        if h["rho"] > 1e-3:             # early iterations: the bound is tight enough to
            assert np.linalg.norm(bound) < 0.05 * np.linalg.norm(h["S_col"])  # catch a slip
        # the residual vanishes on the selected rows and columns (§3.2.2)
        assert np.abs(S[I, :]).max() < 1e-10 * scale
        assert np.abs(S[:, J]).max() < 1e-10 * scale
        assert np.all(np.abs(h["S_col"][:, J]) <= bound[:, J])
        # rho is a difference of nearly equal terms: compare on the scale of ||GA||
        assert abs(h["rho"] - np.linalg.norm(G @ S) / np.linalg.norm(X0)) <= \
            2 * np.linalg.norm(bound) / np.linalg.norm(X0)


def test_residual_recurrence_lemma():
    # §4.2: A - A_{I u I+, J u J+} = S - S(:,J+) S(I+,J+)^+ S(I+,:), S = A - A_{I,J}
    g = np.random.default_rng(2)
    A = g.standard_normal((30, 25)) @ np.diag(0.7 ** np.arange(25)) @ g.standard_normal((25, 25))
    I, J = [3, 17, 8, 22, 0], [5, 1, 19, 11, 24]
    Ip, Jp = [9, 13, 27], [2, 7, 16]
    S = cur_residual(A, I, J, pinv_svd(A[np.ix_(I, J)]))
    lhs = cur_residual(A, I + Ip, J + Jp, pinv_svd(A[np.ix_(I + Ip, J + Jp)]))
    rhs = S - S[:, Jp] @ pinv_svd(S[np.ix_(Ip, Jp)]) @ S[Ip, :]
    np.testing.assert_allclose(lhs, rhs, atol=1e-9 * np.linalg.norm(A))


def test_pinv_matches_moore_penrose_conditions():
    g = np.random.default_rng(3)
    for M in (g.standard_normal((7, 7)), g.standard_normal((6, 4)) @ g.standard_normal((4, 6))):
        P = pinv_svd(M)
        np.testing.assert_allclose(M @ P @ M, M, atol=1e-10)
        np.testing.assert_allclose(P @ M @ P, P, atol=1e-10)
        np.testing.assert_allclose((M @ P).T, M @ P, atol=1e-10)
        np.testing.assert_allclose((P @ M).T, P @ M, atol=1e-10)


@pytest.mark.parametrize("kind", [0, 1])
def test_exact_recovery_of_exactly_low_rank(kind):
    # §5.1: on an exactly low-rank matrix IterativeCUR returns the true rank with an
    # error near machine precision
    b, q = 10, 3
    A = W.exact_lowrank(200, 150, b * q, seed=5)
    out = iterative_cur(A, 1e-10, b, kind=kind, seed=1)
    assert out["rank"] == b * q
    assert out["rho"] < 1e-12
    assert exact_relative_error(A, out["I"], out["J"], out["U"]) < 1e-12


def test_accuracy_respects_svd_lower_bounds():
    # Eckart-Young (§2.1): a rank-k approximation cannot beat the SVD tail
    A, sigma = W.planted_geometric(300, 200, decades_per=40.0, seed=2)
    out = iterative_cur(A, 1e-3, 10, seed=2)
    k = out["rank"]
    assert k < sigma.size
    err = exact_relative_error(A, out["I"], out["J"], out["U"])
    tail = math.sqrt((sigma[k:] ** 2).sum() / (sigma ** 2).sum())
    assert err >= tail * (1 - 1e-9)
    S = cur_residual(A, out["I"], out["J"], out["U"])
    assert np.linalg.norm(S, 2) >= sigma[k] * (1 - 1e-9)
    # closed form for sigma_i = q^i, q = 10^(-1/40), i < N: the squared relative tail is
    # (q^(2k) - q^(2N)) / (1 - q^(2N))
    q2, N = 10.0 ** (-2.0 / 40.0), sigma.size
    assert tail == pytest.approx(math.sqrt((q2 ** k - q2 ** N) / (1 - q2 ** N)), rel=1e-9)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("which", ["planted", "rbf"])
def test_estimator_within_factor_two_and_tolerance_met(seed, which):
    if which == "planted":
        A = _small_planted(seed, 400, 300)
        tol, b = 1e-6, 20
    else:
        A = W.rbf(500, 400, seed)
        tol, b = 1e-4, 10
    out = iterative_cur(A, tol, b, kind=seed % 2, seed=seed)
    err = exact_relative_error(A, out["I"], out["J"], out["U"])
    assert out["status"] == "ok" and out["rho"] <= tol
    assert 0.5 <= out["rho"] / err <= 2.0
    assert err <= 2.0 * tol


def test_gratton_tail_bound_holds_for_fresh_sketches():
    # Theorem 3.1 of §3.3 (Gratton and Titley-Peloquin): with G of variance-1/c
    # Gaussian entries, P[||GA||_F <= ||A||_F / tau] <= exp(-c (tau^2-1)^2 / (4 tau^4)).
    # Fresh seeds, fixed A, tau = 2, c = 5: the bound is exp(-5*9/64) = 0.495.
    A = _small_planted(0, 200, 50)
    c, tau, fails, trials = 5, 2.0, 0, 300
    for s in range(trials):
        G = gaussian_G(10_000 + s, c, A.shape[0]) / math.sqrt(c)
        fails += np.linalg.norm(G @ A) <= np.linalg.norm(A) / tau
    bound = math.exp(-c * (tau ** 2 - 1) ** 2 / (4 * tau ** 4))
    assert fails / trials <= bound


def test_risk_aware_threshold_worked_value():
    # §3.3: alpha = 1e-10, c = 100 (delta = 0) means dividing eps by 4.98
    assert 1.0 / risk_aware_factor(1e-10, 0.0, 100) == pytest.approx(4.98, abs=0.005)
    assert risk_aware_factor(0.0, 0.0, 10) == 1.0
    with pytest.raises(ValueError):
        risk_aware_factor(1e-10, 0.0, 90)          # needs c > -4 ln(alpha) = 92.1
    A = _small_planted(0, 300, 250)
    plain = iterative_cur(A, 1e-4, 90, seed=1)          # c = 99 > 92.1
    risk = iterative_cur(A, 1e-4, 90, seed=1, alpha=1e-10)
    assert risk["rho"] <= 1e-4 / 4.98 and risk["rank"] >= plain["rank"]


def test_sketch_products_follow_their_definitions():
    g = np.random.default_rng(6)
    A = g.integers(-50, 50, size=(300, 40)).astype(np.float64)
    c = sketch_rows(10)
    # sparse-sign: X0 = sum over rows i of A of sign * A(i,:) added into zeta rows
    rows, signs = sparse_sign_pattern(3, c, 300, 8)
    X = np.zeros((c, 40))
    for i in range(300):
        for t in range(rows.shape[1]):
            X[rows[i, t]] += signs[i, t] * A[i]
    out = iterative_cur(A, 0.5, 10, kind=1, seed=3)
    assert np.array_equal(out["X0"], X)              # integer data: exact
    assert np.array_equal(out["G"], sparse_sign_G(3, c, 300))
    # Gaussian: entrywise sum of products, exact for integer A and BF16 G at this size
    Gg = gaussian_G(4, c, 300)
    Xg = np.array([[sum(Gg[r, i] * A[i, j] for i in range(300)) for j in range(40)]
                   for r in range(c)])
    out = iterative_cur(A, 0.5, 10, kind=0, seed=4)
    assert np.array_equal(out["X0"], Xg)


def test_degenerate_inputs():
    out = iterative_cur(np.zeros((20, 10)), 1e-3, 4)
    assert out["rank"] == 0 and out["rho"] == 0.0 and out["status"] == "ok"
    A = np.ones((20, 10))
    A[3, 4] = np.nan
    with pytest.raises(FloatingPointError):
        iterative_cur(A, 1e-3, 4)
    with pytest.raises(ValueError):
        iterative_cur(np.ones((5, 5)), 1e-3, 6)
    with pytest.raises(ValueError):
        iterative_cur(np.ones((5, 5)), 0.0, 2)
    # rank one: one pivot per block, then an exactly-zero residual
    out = iterative_cur(np.outer(np.arange(1.0, 9.0), np.arange(1.0, 6.0)), 1e-12, 3)
    assert out["rank"] == 1 and out["rho"] == 0.0


def test_max_rank_cap_and_full_rank_exhaustion():
    A = W.rbf(80, 60, seed=1, h=0.05)
    out = iterative_cur(A, 1e-14, 7, max_rank=20)
    assert out["status"] == "maxrank" and out["rank"] == 20
    # r not a multiple of b: the last block is shortened
    A = np.random.default_rng(0).standard_normal((30, 23))
    out = iterative_cur(A, 1e-13, 5)
    assert out["rank"] == 23 and out["rho"] < 1e-12


def test_same_seed_same_result_and_block_size_one():
    A = _small_planted(3)
    a = iterative_cur(A, 1e-5, 8, seed=11)
    b = iterative_cur(A, 1e-5, 8, seed=11)
    assert a["I"] == b["I"] and a["J"] == b["J"] and a["rho"] == b["rho"]
    one = iterative_cur(A, 1e-3, 1, seed=2)
    assert one["status"] == "ok"
    assert len(set(one["I"])) == one["rank"] and len(set(one["J"])) == one["rank"]
