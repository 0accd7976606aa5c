"""IterativeCUR, plain FP64 reference (oracle side; test infrastructure).

Follows Alg. 1 of the paper step by step:

  c = floor(1.1 b) sketch rows                       (§1.1 Notation; §3.4)
  G (c x m), drawn once and recycled                 (Alg. 1; §3.2.1)
  X0 = S_0^col = G A,  rho_0 = 1                     (Alg. 1, initial sketch)
  while rho > eps:                                   (Alg. 1 loop)
      J_k = LUPP pivots of (S^col)^T                 (column selection, §3.2.1)
      S^row = A(:,J_k) - C U R(:,J_k)                (row residual, previous C, U, R)
      I_k = LUPP pivots of S^row                     (row selection, §3.2.2)
      I = [I, I_k], J = [J, J_k]
      U = A(I,J)^+ ,  C = A(:,J),  R = A(I,:)        (core and factors, §2.2)
      S^col = G A - (G C) U R, with G C = X0(:,J)    (column residual, "use GC from GA")
      rho = ||S^col||_F / ||G A||_F                  (estimator, §3.3)

Readings where the paper is silent or inconsistent (each is listed in the design doc):
  * c = (11 b) // 10 in integer arithmetic;
  * G is c x m (Alg. 1 prints c x n, which cannot multiply A from the left);
  * the loop stops when rho <= eps (Alg. 1 "while rho > eps"), rho uses ||G A||_F;
  * U = A(I,J)^+ is the SVD pseudo-inverse with singular values below
    r * 2^-52 * sigma_max dropped;
  * a block whose row selection returns fewer pivots than its column selection keeps
    only as many columns as rows; an empty block, or |J| reaching max_rank, ends the
    loop (max_rank defaults to min(m, n));
  * ||G A||_F = 0 returns rank 0 and rho 0; a non-finite ||G A||_F is an error.

Options beyond the default loop:
  * selection="qrcp": QR with column pivoting in place of LUPP for both selections
    (Alg. 1 names it as the alternative; §5.3);
  * denominator="A": rho = ||S^col||_F / (s_G ||A||_F) with s_G the scale of G
    (E ||G x||^2 = s_G^2 ||x||^2), the estimate the Corollary of §3.3 bounds (the §5
    footnote on the denominator); with a Gaussian G this is ||G' (A - CUR)||_F / ||A||_F
    for G' = G / sqrt(c), whose entries have the Corollary's variance 1/c;
  * forced=[(J_1, I_1), (J_2, I_2), ...]: replay mode.  Block k uses the given index
    blocks instead of its own selections, and records beside them what the selection
    would have seen (`lupp_replay` / per-step best and second-best values), so the
    choices of another implementation can be checked one pivot at a time along its own
    trajectory.  Blocks after the forced ones select as usual.
"""
import math

import numpy as np

from .lupp import lupp_pivots, lupp_replay
from .qrcp import qrcp_pivots
from .rng import g_scale, make_G


def sketch_rows(b):
    """c = floor(1.1 b), computed exactly as (11 b) // 10."""
    return (11 * int(b)) // 10


def pinv_svd(M):
    """Moore-Penrose pseudo-inverse through the SVD; singular values at or below
    max(shape) * 2^-52 * sigma_max are treated as zero."""
    M = np.asarray(M, dtype=np.float64)
    if M.size == 0:
        return np.zeros((M.shape[1], M.shape[0]))
    Uu, s, Vt = np.linalg.svd(M, full_matrices=False)
    cut = max(M.shape) * 2.0 ** -52 * (s[0] if s.size else 0.0)
    inv = np.zeros_like(s)
    keep = s > cut
    inv[keep] = 1.0 / s[keep]
    return (Vt.T * inv) @ Uu.T


def risk_aware_factor(alpha, delta, c):
    """Threshold multiplier xi = (1 + delta) sqrt(1 - 2 sqrt(-ln(alpha) / c)) of the
    risk-aware stopping rule (§3.3, Corollary); stop at rho <= xi * eps.  Requires
    c > -4 ln(alpha).  alpha = 0 switches the adjustment off (xi = 1)."""
    if alpha == 0:
        return 1.0
    if not (0.0 < alpha < 1.0) or delta < 0:
        raise ValueError("need 0 < alpha < 1 and delta >= 0")
    if not c > -4.0 * math.log(alpha):
        raise ValueError("risk-aware threshold needs c > -4 ln(alpha)")
    return (1.0 + delta) * math.sqrt(1.0 - 2.0 * math.sqrt(-math.log(alpha) / c))


def cur_residual(A, I, J, U):
    """Full residual S = A - A(:,J) U A(I,:) (§1.1 Notation)."""
    A = np.asarray(A, dtype=np.float64)
    if len(J) == 0:
        return A.copy()
    return A - A[:, J] @ (U @ A[I, :])


def exact_relative_error(A, I, J, U):
    """||A - C U R||_F / ||A||_F."""
    A = np.asarray(A, dtype=np.float64)
    return np.linalg.norm(cur_residual(A, I, J, U)) / np.linalg.norm(A)


def _qrcp_replay(T, forced, exclude=()):
    """Replay of QRCP with the pivot of each step given: per step the given pivot's
    trailing norm beside the best eligible one (same records as lupp_replay)."""
    X = np.array(np.asarray(T, dtype=np.float64).T, copy=True)
    K, N = X.shape
    avail = np.ones(N, dtype=bool)
    ex = np.asarray(list(exclude), dtype=np.int64)
    if ex.size:
        avail[ex] = False
    recs = []
    for t, p in enumerate(forced):
        p = int(p)
        if not (0 <= p < N) or not avail[p]:
            raise ValueError("forced pivot %d at step %d is not an eligible candidate" % (p, t))
        nrm = np.sqrt(np.sum(X[t:, :] ** 2, axis=0))
        nrm[~avail] = -1.0
        b = int(np.argmax(nrm))
        rest = nrm.copy()
        rest[b] = -1.0
        recs.append({"pick": p, "value": nrm[p], "best": b, "best_value": nrm[b],
                     "second_value": max(rest.max(), 0.0)})
        if nrm[p] == 0.0:
            raise ValueError("forced pivot %d at step %d has a zero residual" % (p, t))
        avail[p] = False
        x = X[t:, p]
        alpha = np.linalg.norm(x)
        v = x.copy()
        v[0] = x[0] + (1.0 if x[0] >= 0 else -1.0) * alpha
        X[t:, :] -= (2.0 / (v @ v)) * np.outer(v, v @ X[t:, :])
    return recs


def iterative_cur(A, tol, b, kind=0, seed=0, zeta=8, max_rank=None, G=None,
                  alpha=0.0, delta=0.0, record=False, selection="lupp", denominator="GA",
                  forced=None):
    """IterativeCUR of Alg. 1 on the dense m x n matrix A.

    Returns a dict with I, J (pivot order), U (|J| x |J|), rank, rho (final estimate),
    status ("ok"; "maxrank" when |J| reached max_rank first; "stalled" when a block
    came back empty), X0 = G A, G, blocks (sizes of the index blocks) and, when
    record=True (always in replay mode), per-iteration history entries
    {"J_k", "I_k", "rho", "col_margins", "row_margins"}; replayed blocks also carry
    "col_replay" and "row_replay" (per-step records of the forced choices).
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    b = int(b)
    if not (1 <= b <= min(m, n)):
        raise ValueError("need 1 <= b <= min(m, n)")
    if not (math.isfinite(tol) and tol > 0):
        raise ValueError("tol must be finite and positive")
    if selection not in ("lupp", "qrcp"):
        raise ValueError("selection is lupp or qrcp")
    if denominator not in ("GA", "A"):
        raise ValueError("denominator is GA or A")
    if alpha != 0 and G is None and kind != 0:
        raise ValueError("risk-aware stopping (§3.3 Corollary) holds for the Gaussian sketch only")
    pick = lupp_pivots if selection == "lupp" else qrcp_pivots
    replay = lupp_replay if selection == "lupp" else _qrcp_replay
    forced = list(forced or [])
    if forced:
        record = True
    c = sketch_rows(b)
    if max_rank is None:
        max_rank = min(m, n)
    max_rank = min(int(max_rank), m, n)
    if G is None:
        G = make_G(seed, c, m, kind, zeta)
    G = np.asarray(G, dtype=np.float64)
    c = G.shape[0]
    xi = risk_aware_factor(alpha, delta, c)

    X0 = G @ A
    g = np.linalg.norm(X0)
    if not math.isfinite(g):
        raise FloatingPointError("non-finite sketch norm")
    out = {"I": [], "J": [], "U": np.zeros((0, 0)), "rank": 0, "rho": 0.0,
           "status": "ok", "history": [], "X0": X0, "G": G, "blocks": []}
    if g == 0.0:
        return out
    denom = g if denominator == "GA" else g_scale(kind, c, zeta) * np.linalg.norm(A)

    S = X0
    rho = 1.0 if denominator == "GA" else g / denom
    I, J = [], []
    U = np.zeros((0, 0))
    while rho > xi * tol and len(J) < max_rank:
        s = min(b, max_rank - len(J))
        k = len(out["blocks"])
        entry = {}
        if k < len(forced):
            Jk, Ik = [int(x) for x in forced[k][0]], [int(x) for x in forced[k][1]]
            if not (1 <= len(Jk) == len(Ik) <= s):
                raise ValueError("forced block %d must hold 1..%d column and row indices" % (k, s))
            entry["col_replay"] = replay(S.T, Jk, exclude=J)
            cm = [1.0 - r["second_value"] / r["best_value"] if r["best_value"] > 0 else 0.0
                  for r in entry["col_replay"]]
        else:
            Jk, cm = pick(S.T, s, exclude=J, return_margins=True)
            if not Jk:
                break
        if J:
            Sr = A[:, Jk] - A[:, J] @ (U @ A[np.ix_(I, Jk)])
        else:
            Sr = A[:, Jk].copy()
        if k < len(forced):
            entry["row_replay"] = replay(Sr, Ik, exclude=I)
            rm = [1.0 - r["second_value"] / r["best_value"] if r["best_value"] > 0 else 0.0
                  for r in entry["row_replay"]]
        else:
            Ik, rm = pick(Sr, len(Jk), exclude=I, return_margins=True)
            Jk = Jk[:len(Ik)]
            if not Ik:
                break
        I = I + Ik
        J = J + Jk
        out["blocks"].append(len(Ik))
        U = pinv_svd(A[np.ix_(I, J)])
        S = X0 - (X0[:, J] @ U) @ A[I, :]
        rho = np.linalg.norm(S) / denom
        if record:
            entry.update({"J_k": list(Jk), "I_k": list(Ik), "rho": rho,
                          "col_margins": cm[:len(Ik)], "row_margins": rm,
                          "S_row": Sr, "S_col": S})
            out["history"].append(entry)
    if rho <= xi * tol:
        status = "ok"
    elif len(J) >= max_rank:
        status = "maxrank"
    else:
        status = "stalled"
    out.update(I=I, J=J, U=U, rank=len(J), rho=rho, status=status)
    return out
