"""Pins for the oracle's replay mode (CPU only).

Replay runs the oracle's selections with the pivots given by the caller, so another
implementation's choices can be checked one pivot at a time along its own trajectory.
It is pinned by brute force (every replayed value is a ratio of determinants, computed
here without any elimination) and by reproducing the oracle's own run bit for bit.
"""
import itertools

import numpy as np
import pytest

from oracle.icur import iterative_cur
from oracle.lupp import lupp_pivots, lupp_replay
from oracle.qrcp import qrcp_pivots
from paper_2509_21963_amd import workloads as W


def _det(M):
    return np.linalg.det(M) if M.size else 1.0


@pytest.mark.parametrize("seed", range(6))
def test_lupp_replay_values_are_determinant_ratios(seed):
    # the Schur-complement entry of candidate i at step t, after pivots P_t, equals
    # det(T[P_t + [i], :t+1]) / det(T[P_t, :t]); this holds for any pivot sequence, so a
    # random (non-argmax) sequence checks the replay's elimination
    rng = np.random.default_rng(seed)
    T = rng.standard_normal((7, 4))
    forced = list(rng.permutation(7)[:4])
    recs = lupp_replay(T, forced)
    for t, rec in enumerate(recs):
        P = forced[:t]
        den = _det(T[np.ix_(P, range(t))])
        vals = {i: abs(_det(T[np.ix_(P + [i], range(t + 1))]) / den)
                for i in range(7) if i not in P}
        assert rec["value"] == pytest.approx(vals[forced[t]], rel=1e-10)
        assert rec["best_value"] == pytest.approx(max(vals.values()), rel=1e-10)
        assert vals[rec["best"]] == pytest.approx(max(vals.values()), rel=1e-10)


@pytest.mark.parametrize("seed", range(4))
def test_lupp_replay_of_its_own_pivots(seed):
    rng = np.random.default_rng(seed)
    T = rng.standard_normal((200, 12))
    ex = [3, 17, 150]
    piv, marg = lupp_pivots(T, 12, exclude=ex, return_margins=True)
    recs = lupp_replay(T, piv, exclude=ex)
    assert [r["best"] for r in recs] == piv
    assert all(r["value"] == r["best_value"] for r in recs)
    np.testing.assert_array_equal([1 - r["second_value"] / r["best_value"] for r in recs], marg)


def test_lupp_replay_rejects_ineligible_pivots():
    T = np.random.default_rng(1).standard_normal((10, 3))
    with pytest.raises(ValueError):
        lupp_replay(T, [2, 2])
    with pytest.raises(ValueError):
        lupp_replay(T, [4], exclude=[4])
    with pytest.raises(ValueError):
        lupp_replay(np.zeros((4, 2)), [1])


@pytest.mark.parametrize("selection", ["lupp", "qrcp"])
@pytest.mark.parametrize("kind", [0, 1])
def test_replaying_its_own_choices_reproduces_the_run(selection, kind):
    A, _ = W.planted_geometric(300, 220, 15.0, seed=2)
    ref = iterative_cur(A, 1e-7, 12, kind=kind, seed=5, record=True, selection=selection)
    forced = [(h["J_k"], h["I_k"]) for h in ref["history"]]
    rep = iterative_cur(A, 1e-7, 12, kind=kind, seed=5, forced=forced, selection=selection)
    assert rep["I"] == ref["I"] and rep["J"] == ref["J"] and rep["blocks"] == ref["blocks"]
    np.testing.assert_array_equal(rep["U"], ref["U"])
    assert rep["rho"] == ref["rho"]
    for h in rep["history"]:
        for rec in h["col_replay"] + h["row_replay"]:
            assert rec["pick"] == rec["best"] and rec["value"] == rec["best_value"]
    # forcing only the first block, the rest selects as usual: the same run again
    part = iterative_cur(A, 1e-7, 12, kind=kind, seed=5, forced=forced[:1], selection=selection)
    assert part["I"] == ref["I"] and part["J"] == ref["J"] and part["rho"] == ref["rho"]


def test_replay_records_a_choice_that_is_not_the_argmax():
    # force the runner-up column at the first step: the record shows it, the run goes on
    # along the forced trajectory, and the result is still a CUR with the Schur zeros
    A, _ = W.planted_geometric(200, 150, 10.0, seed=1)
    ref = iterative_cur(A, 1e-5, 5, seed=3, record=True)
    h = ref["history"][0]
    S0 = ref["X0"]
    mag = np.abs(S0[0])
    runner_up = int(np.argsort(-mag)[1])
    Jk = [runner_up] + [j for j in h["J_k"] if j != runner_up][:4]
    T = A[:, Jk]
    Ik = lupp_pivots(T, len(Jk))
    rep = iterative_cur(A, 1e-5, 5, seed=3, forced=[(Jk, Ik)])
    first = rep["history"][0]["col_replay"][0]
    assert first["pick"] == runner_up and first["best"] == h["J_k"][0]
    assert first["value"] < first["best_value"]
    I, J, U = rep["I"], rep["J"], rep["U"]
    Res = A - A[:, J] @ U @ A[I, :]
    assert np.abs(Res[I, :]).max() < 1e-9 * np.abs(A).max()
    assert np.abs(Res[:, J]).max() < 1e-9 * np.abs(A).max()


def test_qrcp_replay_values_are_volume_ratios():
    # QRCP step t: the trailing norm of candidate j after pivots P_t is
    # sqrt(det Gram(P_t + [j]) / det Gram(P_t)) for any pivot sequence
    from oracle.icur import _qrcp_replay
    rng = np.random.default_rng(4)
    T = rng.standard_normal((8, 5))
    forced = [6, 1, 3, 0]
    recs = _qrcp_replay(T, forced)
    X = T.T
    for t, rec in enumerate(recs):
        P = forced[:t]
        gP = _det(X[:, P].T @ X[:, P])
        vals = {j: np.sqrt(_det(X[:, P + [j]].T @ X[:, P + [j]]) / gP) for j in range(8) if j not in P}
        assert rec["value"] == pytest.approx(vals[forced[t]], rel=1e-9)
        assert rec["best_value"] == pytest.approx(max(vals.values()), rel=1e-9)
    own = qrcp_pivots(T, 5)
    assert [r["best"] for r in _qrcp_replay(T, own)] == own
