"""Pivot-by-pivot parity of a GPU run with the FP64 oracle (test helper, no tests here).

The GPU's index blocks are replayed through the oracle (`iterative_cur(forced=...)`):
at every LUPP step the oracle evaluates, along the GPU's own trajectory, the value of
the candidate the GPU chose and the best and second-best eligible values.  Both sides
carry rounding, so each value is known up to a noise bound `noise`:
  * the GPU's choice is valid when   value >= best - 2 noise   (it lies in the tied set);
  * the step is pinned when          second < best - 2 noise   (only the oracle's argmax
    is valid, so validity means the GPU chose exactly the oracle's pivot).

Noise bounds (absolute, per candidate i at step t of a selection on T, the N x K
candidate matrix, P the t pivots so far): an input perturbation of size d0 in every
entry of T moves the step-t Schur complement v_i = T(i,t) - x_i T(P,t) by at most
d0 (1 + ||x_i||_1) (1 + ||y||_1), x_i = T(i,0:t) T(P,0:t)^{-1}, y = T(P,0:t)^{-1} T(P,t)
(first order).  A choice is valid when its interval meets the best candidate's; a step
is pinned when no other interval reaches the best one's.  (QRCP steps use the cruder
factor (1 + a_t)^2, a_t = t max|T| ||T(P,0:t)^{-1}||_1.)  The input perturbation d0:
  column steps: (eta + 4 cond 2^-52) max|X0|, with eta the sketch rounding of the form
    relative to max|X0| (see sketch_eta) and cond = cond(A(I,J)) of the cross before
    the block: the oracle forms S^col = X0 - X0(:,J) A(I,J)^+ A(I,:), whose rounding
    grows with cond; the GPU's residual form does not, so the oracle's term dominates;
  row steps: (eta_row + 4 sqrt(r + 1) cond 2^-52) max|A| (the row residual involves no
    sketch; with FP64 factors both sides form it in FP64 from the same FP32 values, and
    eta_row covers the rounding of FP32 factors, see residual_eta).
  With QRCP the compared values are residual 2-norms of K-vectors, so both bounds are
  multiplied by sqrt(K).
"""
import math

import numpy as np

from oracle.icur import iterative_cur

EPS64 = 2.0 ** -52
EPS32 = 2.0 ** -24


def sketch_eta(terms, chunk=128, sparse=False):
    """Rounding of the GPU sketch relative to max|X0|, with a factor 16 of headroom.

    Dense forms: each product of a BF16 piece sum with the BF16-valued G carries the
    pieces' truncation, 2^-(8 T + 1) relative (T = 1, 2; three pieces are exact); FP32
    sums over `chunk` rows add about sqrt(chunk) 2^-24 relative (random-walk growth of
    the partial sums), FP64 across chunks.  The CSR sketch is FP64 throughout.
    """
    if sparse:
        return 16 * 64 * EPS64
    trunc = 0.0 if terms in (0, 3) else 2.0 ** -(8 * terms + 1)
    return 16 * (trunc + math.sqrt(chunk) * EPS32)


def residual_eta(terms):
    """Rounding of the FP32-factor residual products relative to the scale of A, with a
    factor 4 of headroom.

    The factors are stored in FP32 (2^-24 relative) and both operands of the two large
    products are cut into `terms` BF16 pieces (2^-(8 T + 1) relative each; T = 0 means FP32
    matrix cores, no cut); FP32 sums over 32-deep chunks add about sqrt(32) 2^-24.
    """
    trunc = 0.0 if terms == 0 else 2.0 * 2.0 ** -(8 * terms + 1)
    return 4 * (trunc + EPS32 + math.sqrt(32) * EPS32)


def blocks_of(rank, b, max_rank=None, sizes=None):
    """Block sizes of a run: the reported ones, else b per block (the last one short)."""
    if sizes:
        assert sum(sizes) == rank
        return list(sizes)
    out, r = [], 0
    cap = rank if max_rank is None else max_rank
    while r < rank:
        s = min(b, cap - r, rank - r)
        out.append(s)
        r += s
    return out


def growth(T, piv):
    """(1 + a_t)^2 for every step t of a selection on T (N x K) with the pivots `piv`,
    a_t = t max|T| ||T(piv[:t], :t)^{-1}||_1 (1 at t = 0): a cheap upper bound of the
    factor step_margins computes exactly (used for QRCP)."""
    T = np.asarray(T, dtype=np.float64)
    tmax = float(np.abs(T).max()) if T.size else 0.0
    out = []
    for t in range(len(piv)):
        if t == 0:
            out.append(1.0)
            continue
        B = T[np.ix_(list(piv[:t]), list(range(t)))]
        try:
            inv1 = float(np.abs(np.linalg.inv(B)).sum(axis=0).max())
        except np.linalg.LinAlgError:
            inv1 = float("inf")
        a = t * tmax * inv1
        out.append((1.0 + a) ** 2)
    return out


def lupp_steps_with_noise(T, piv, exclude, d0):
    """For each step t of LUPP on T (N x K) with the given pivots: the step-t Schur
    complements v_i of every eligible candidate and their noise bounds
    n_i = d0 (1 + ||x_i||_1) (1 + ||y||_1) with x_i = T(i, 0:t) T(P, 0:t)^{-1},
    y = T(P, 0:t)^{-1} T(P, t).  Yields (eligible indices, |v|, n) per step.

    v comes from right-looking elimination along the given pivots (rounding near
    t 2^-52 max|T|, whatever the conditioning of T(P, 0:t)); x and y, which only size the
    noise, come from solves with T(P, 0:t)."""
    T = np.asarray(T, dtype=np.float64)
    N = T.shape[0]
    elig = np.ones(N, dtype=bool)
    ex = np.asarray(list(exclude), dtype=np.int64)
    if ex.size:
        elig[ex] = False
    S = T.copy()  # Schur complements, columns t.. current
    P = []
    for t in range(len(piv)):
        if t == 0:
            xn = np.zeros(N)
            yn = 0.0
        else:
            B = T[np.ix_(P, list(range(t)))]
            try:
                y = np.linalg.solve(B, T[P, t])
                X = np.linalg.solve(B.T, T[:, :t].T).T
            except np.linalg.LinAlgError:
                y = np.full(t, np.inf)
                X = np.full((N, t), np.inf)
            xn = np.abs(X).sum(axis=1)
            yn = float(np.abs(y).sum())
        idx = np.nonzero(elig)[0]
        yield idx, np.abs(S[idx, t]), d0 * (1.0 + xn[idx]) * (1.0 + yn)
        p = int(piv[t])
        if t + 1 < S.shape[1] and S[p, t] != 0.0:
            f = S[:, t] / S[p, t]
            S[:, t + 1:] -= np.outer(f, S[p, t + 1:])
        elig[p] = False
        P.append(p)


def replay(A64, I, J, blocks, tol, b, kind, seed, eta, zeta=8, selection="lupp",
           denominator="GA", max_rank=None, eta_row=0.0, alpha=0.0):
    """Replay the GPU's blocks through the oracle and check every pivot.

    Returns (stats, rep) with stats = {"col_pinned", "col_tied", "row_pinned", "row_tied"}
    and rep the oracle's replay.  Raises AssertionError at the first invalid choice.
    """
    I, J = [int(x) for x in I], [int(x) for x in J]
    forced, o = [], 0
    for s in blocks:
        forced.append((J[o:o + s], I[o:o + s]))
        o += s
    assert o == len(I) == len(J)
    rep = iterative_cur(A64, tol, b, kind=kind, seed=seed, zeta=zeta, forced=forced,
                        selection=selection, denominator=denominator, max_rank=max_rank, alpha=alpha)
    x0max = float(np.abs(rep["X0"]).max())
    amax = float(np.abs(A64).max())
    stats = {"col_pinned": 0, "col_tied": 0, "row_pinned": 0, "row_tied": 0}
    cond, Ic, Jc = 1.0, [], []
    assert len(rep["history"]) >= len(forced), (
        "the oracle stops after %d blocks along this trajectory, the GPU ran %d" % (len(rep["history"]), len(forced)))
    for k, (Jk, Ik) in enumerate(forced):
        h = rep["history"][k]
        noise = {"col": (eta + 4 * cond * EPS64) * x0max,
                 "row": (eta_row + 4 * math.sqrt(len(Ic) + 1) * cond * EPS64) * amax}
        if selection == "qrcp":
            # QRCP compares residual 2-norms of K-vectors: their error is up to sqrt(K)
            # times an entry's
            noise = {"col": noise["col"] * math.sqrt(rep["X0"].shape[0]),
                     "row": noise["row"] * math.sqrt(len(Jk))}
        # the candidate matrices of the block: (S^col)^T before it, and S^row
        Tcol = (rep["X0"] if k == 0 else rep["history"][k - 1]["S_col"]).T
        for side, T, piv, excl, recs in (("col", Tcol, Jk, Jc, h["col_replay"]),
                                         ("row", h["S_row"], Ik, Ic, h["row_replay"])):
            if selection == "qrcp":
                amp = growth(T, piv)
                for t, rec in enumerate(recs):
                    lim = rec["best_value"] - 2 * noise[side] * amp[t]
                    assert rec["value"] >= lim, (
                        "block %d %s step %d: GPU chose %d (|v| = %.6e), oracle's best %d (%.6e)"
                        % (k, side, t, rec["pick"], rec["value"], rec["best"], rec["best_value"]))
                    if rec["second_value"] < lim:
                        assert rec["pick"] == rec["best"]
                        stats[side + "_pinned"] += 1
                    else:
                        stats[side + "_tied"] += 1
                continue
            for t, (idx, av, nz) in enumerate(lupp_steps_with_noise(T, piv, excl, noise[side])):
                pick = int(piv[t])
                b = int(np.argmax(av))
                lo_best = av[b] - nz[b]
                j = int(np.searchsorted(idx, pick))
                assert j < idx.size and idx[j] == pick
                assert av[j] + nz[j] >= lo_best, (
                    "block %d %s step %d: GPU chose %d (|v| = %.6e +- %.2e), oracle's best %d (%.6e +- %.2e)"
                    % (k, side, t, pick, av[j], nz[j], idx[b], av[b], nz[b]))
                others = np.delete(np.arange(idx.size), b)
                if others.size == 0 or np.max(av[others] + nz[others]) < lo_best:
                    assert pick == idx[b]
                    stats[side + "_pinned"] += 1
                else:
                    stats[side + "_tied"] += 1
        Ic += Ik
        Jc += Jk
        cond = float(np.linalg.cond(A64[np.ix_(Ic, Jc)]))
    return stats, rep


def all_pinned(A64, ora, tol, b, kind, seed, eta, **kw):
    """True when every step of the oracle's own run is pinned under the noise model of
    `replay`: an input with well-separated pivots, whose whole index sets are unique."""
    blocks = [len(h["I_k"]) for h in ora["history"]]
    stats, _ = replay(A64, ora["I"], ora["J"], blocks, tol, b, kind, seed, eta, **kw)
    return stats["col_tied"] == 0 and stats["row_tied"] == 0, stats
