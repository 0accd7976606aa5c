"""Index selection by LU with partial pivoting (oracle side; test infrastructure).

IterativeCUR selects its b new column indices by LUPP on the sketched residual and its
b new row indices by LUPP on the row residual (Alg. 1, the "Column Selection" and "Row
Selection" steps; §3.2.1 and §3.2.2).  Only the pivot order is used.

Readings of what the paper leaves open:
* candidates are the rows of T (N x K); pivots are taken for columns 0, 1, ... in turn,
  the first `steps` of them (b new indices per iteration, §1.1 Notation);
* ties in |T[i, t]| go to the lowest row index (the BLAS i?amax convention);
* rows already selected in earlier iterations are excluded (they are exact zeros of the
  residual, §3.2.2; excluding them guards against rounding);
* a step whose best candidate is exactly zero, or that has no candidate left, ends the
  selection early.

Arithmetic: FP64, textbook right-looking elimination.  At step t with pivot row p every
remaining row i is updated as  l = T[i,t] / T[p,t];  T[i,j] = T[i,j] - (l * T[p,j])
for j > t, with the product rounded before the subtraction (no fused multiply-add).

Replay: `lupp_replay` runs the same elimination with the pivot of each step given by
the caller (for instance the choices another implementation made) and records, per
step, the given pivot's |T[p,t]| beside the best eligible |T[i,t]|.  With the argmax
pivots it is lupp_pivots itself, step for step.
"""
import numpy as np


def _eliminate(T, avail, p, t):
    """Right-looking update of the eligible rows with pivot row p at column t."""
    N, K = T.shape
    rows = np.nonzero(avail)[0]
    if rows.size and t + 1 < K:
        l = T[rows, t] / T[p, t]
        prod = l[:, None] * T[p, t + 1:][None, :]
        T[np.ix_(rows, np.arange(t + 1, K))] = T[np.ix_(rows, np.arange(t + 1, K))] - prod


def _step_scan(T, avail, t):
    """(argmax index, best |T[i,t]|, second best) over the eligible rows."""
    mag = np.abs(T[:, t])
    mag[~avail] = -1.0
    p = int(np.argmax(mag))            # first index of the maximum
    best = mag[p]
    rest = mag.copy()
    rest[p] = -1.0
    return p, best, rest.max()


def lupp_pivots(T, steps, exclude=(), return_margins=False):
    """Pivot rows of LU with partial pivoting applied to the N x K matrix T.

    Returns the list of chosen row indices in pivot order (length <= min(steps, K)).
    With return_margins=True also returns, per step, 1 - |second best| / |best| over
    the eligible candidates (1.0 when there is a single candidate).
    """
    T = np.array(T, dtype=np.float64, copy=True)
    N, K = T.shape
    steps = min(int(steps), K)
    avail = np.ones(N, dtype=bool)
    ex = np.asarray(list(exclude), dtype=np.int64)
    if ex.size:
        avail[ex] = False
    piv, margins = [], []
    for t in range(steps):
        if not avail.any():
            break
        p, best, second = _step_scan(T, avail, t)
        if best == 0.0:
            break
        if return_margins:
            margins.append(1.0 if second < 0 else 1.0 - second / best)
        piv.append(p)
        avail[p] = False
        _eliminate(T, avail, p, t)
    if return_margins:
        return piv, margins
    return piv


def lupp_replay(T, forced, exclude=()):
    """LUPP elimination of the N x K matrix T with the pivot of step t set to forced[t].

    Returns one record per forced step: {"pick": forced[t], "value": |T[pick, t]|,
    "best": argmax index over the eligible rows, "best_value", "second_value"} where the
    values are those of the partially eliminated T at that step.  A forced pivot that is
    excluded, already chosen or out of range raises ValueError; so does a zero pivot
    value (the elimination cannot continue).
    """
    T = np.array(T, dtype=np.float64, copy=True)
    N, K = T.shape
    if len(forced) > K:
        raise ValueError("more forced pivots than columns")
    avail = np.ones(N, dtype=bool)
    ex = np.asarray(list(exclude), dtype=np.int64)
    if ex.size:
        avail[ex] = False
    recs = []
    for t, p in enumerate(forced):
        p = int(p)
        if not (0 <= p < N) or not avail[p]:
            raise ValueError("forced pivot %d at step %d is not an eligible candidate" % (p, t))
        b, best, second = _step_scan(T, avail, t)
        val = abs(T[p, t])
        recs.append({"pick": p, "value": val, "best": b, "best_value": best,
                     "second_value": max(second, 0.0)})
        if val == 0.0:
            raise ValueError("forced pivot %d at step %d is exactly zero" % (p, t))
        avail[p] = False
        _eliminate(T, avail, p, t)
    return recs
