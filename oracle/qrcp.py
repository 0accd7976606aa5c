"""Index selection by QR with column pivoting (oracle side; test infrastructure).

Alg. 1 names LUPP as the default selection and QRCP as an alternative for both the
column and the row selection; §5.3 compares the two (and finds them equal in quality).
The candidates are the rows of T (N x K), as for `lupp_pivots`: the column selection
passes (S^col)^T, the row selection passes S^row, and QRCP pivots over the columns of
X = T^T (Businger-Golub column pivoting).

Arithmetic: FP64 Householder QR.  At step t the trailing parts X[t:, j] of the eligible
columns are the components of the candidates orthogonal to the span of the columns
already chosen; their norms are recomputed from them at every step (no downdating), the
largest is the pivot (ties to the lowest index), and a Householder reflector that maps
the pivot's trailing part onto e_1 is applied to the trailing rows of every column.
A step whose best norm is exactly zero, or that has no candidate left, ends the
selection.  Candidates in `exclude` are never chosen.
"""
import numpy as np


def _householder(x):
    """v, beta with (I - beta v v^T) x = -sign(x0) ||x|| e_1 (v[0] = 1 scaling free)."""
    alpha = np.linalg.norm(x)
    v = x.copy()
    s = 1.0 if x[0] >= 0 else -1.0
    v[0] = x[0] + s * alpha
    vv = v @ v
    beta = 0.0 if vv == 0.0 else 2.0 / vv
    return v, beta


def qrcp_pivots(T, steps, exclude=(), return_margins=False):
    """Pivot order of QR with column pivoting applied to X = T^T (T is N x K, one row per
    candidate).  Returns the chosen candidate indices (length <= min(steps, K)) and, with
    return_margins=True, per step 1 - (second best norm) / (best norm)."""
    X = np.array(np.asarray(T, dtype=np.float64).T, copy=True)   # K x N
    K, N = X.shape
    steps = min(int(steps), K)
    avail = np.ones(N, dtype=bool)
    ex = np.asarray(list(exclude), dtype=np.int64)
    if ex.size:
        avail[ex] = False
    piv, margins = [], []
    for t in range(steps):
        if not avail.any():
            break
        nrm = np.sqrt(np.sum(X[t:, :] ** 2, axis=0))
        nrm[~avail] = -1.0
        p = int(np.argmax(nrm))
        best = nrm[p]
        if best == 0.0:
            break
        if return_margins:
            rest = nrm.copy()
            rest[p] = -1.0
            second = rest.max()
            margins.append(1.0 if second < 0 else 1.0 - second / best)
        piv.append(p)
        avail[p] = False
        v, beta = _householder(X[t:, p])
        X[t:, :] -= beta * np.outer(v, v @ X[t:, :])
    if return_margins:
        return piv, margins
    return piv
