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
"""
import math

import numpy as np

from .lupp import lupp_pivots
from .rng import make_G


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


def iterative_cur(A, tol, b, kind=0, seed=0, zeta=8, max_rank=None, G=None,
                  alpha=0.0, delta=0.0, record=False):
    """IterativeCUR of Alg. 1 on the dense m x n matrix A.

    Returns a dict with I, J (pivot order), U (|J| x |J|), rank, rho (final estimate),
    status ("ok"; "maxrank" when |J| reached max_rank first; "stalled" when a block
    came back empty), X0 = G A, G and, when record=True, per-iteration history entries
    {"J_k", "I_k", "rho", "col_margins", "row_margins"}.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    b = int(b)
    if not (1 <= b <= min(m, n)):
        raise ValueError("need 1 <= b <= min(m, n)")
    if not (math.isfinite(tol) and tol > 0):
        raise ValueError("tol must be finite and positive")
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
           "status": "ok", "history": [], "X0": X0, "G": G}
    if g == 0.0:
        return out

    S = X0
    rho = 1.0
    I, J = [], []
    U = np.zeros((0, 0))
    while rho > xi * tol and len(J) < max_rank:
        s = min(b, max_rank - len(J))
        Jk, cm = lupp_pivots(S.T, s, exclude=J, return_margins=True)
        if not Jk:
            break
        if J:
            Sr = A[:, Jk] - A[:, J] @ (U @ A[np.ix_(I, Jk)])
        else:
            Sr = A[:, Jk].copy()
        Ik, rm = lupp_pivots(Sr, len(Jk), exclude=I, return_margins=True)
        Jk = Jk[:len(Ik)]
        if not Ik:
            break
        I = I + Ik
        J = J + Jk
        U = pinv_svd(A[np.ix_(I, J)])
        S = X0 - (X0[:, J] @ U) @ A[I, :]
        rho = np.linalg.norm(S) / g
        if record:
            out["history"].append({"J_k": list(Jk), "I_k": list(Ik), "rho": rho,
                                   "col_margins": cm[:len(Ik)], "row_margins": rm,
                                   "S_row": Sr, "S_col": S})
    if rho <= xi * tol:
        status = "ok"
    elif len(J) >= max_rank:
        status = "maxrank"
    else:
        status = "stalled"
    out.update(I=I, J=J, U=U, rank=len(J), rho=rho, status=status)
    return out
