"""IterativeCUR on a CSR matrix (icur_run_csr) against the FP64 oracle (GPU).

The oracle runs on the dense copy of the same FP32 values.  The CSR sketch accumulates
in FP64 (exact products with the +-1 or BF16-valued G).  Every pivot is replayed through
the oracle along the GPU's trajectory (tests/_replay.py), U is compared with the
oracle's pseudo-inverse of the cross, and the result is checked as in the dense tests
(true error <= 2 tol, rho within a factor 2 of it).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle.icur import exact_relative_error, iterative_cur, pinv_svd   # noqa: E402
from paper_2509_21963_amd import workloads as W               # noqa: E402
from _replay import replay, sketch_eta                          # noqa: E402


@pytest.fixture(scope="module")
def icur():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_21963_amd import icur as m
    m.load()
    return m


def dev_csr(rowptr, colind, vals):
    return (torch.from_numpy(rowptr).cuda(), torch.from_numpy(colind).cuda(), torch.from_numpy(vals).cuda())


def run_and_check(icur, A, tol, b, kind, seed, **kw):
    rowptr, colind, vals = W.csr_to_f32(A)
    D = W.csr_dense64(rowptr, colind, vals, A.shape)
    got = icur.run_csr(*dev_csr(rowptr, colind, vals), A.shape, tol, b, kind, seed, **kw)
    I, J = got["I"].tolist(), got["J"].tolist()
    r = got["rank"]
    assert len(set(I)) == r and len(set(J)) == r
    # every pivot replayed through the oracle (tests/_replay.py); the CSR sketch is FP64
    stats, rep = replay(D, I, J, got["info"]["block_sizes"], tol, b, kind, seed, sketch_eta(3, sparse=True))
    got["parity"] = stats
    print("pivot parity", stats)
    assert stats["col_pinned"] > 0 and stats["row_pinned"] > 0
    ora = iterative_cur(D, tol, b, kind=kind, seed=seed, record=True)
    err = exact_relative_error(D, I, J, got["U"]) if r else 1.0
    if r:
        core = D[np.ix_(I, J)]
        Uo = pinv_svd(core)
        assert np.abs(got["U"] - Uo).max() <= 16 * r * np.linalg.cond(core) * 2.0 ** -52 * np.abs(Uo).max()
    return got, ora, err, D


@pytest.mark.parametrize("kind", [0, 1])
def test_sparse_low_rank_plus_noise(icur, kind):
    A = W.sparse_lowrank(3000, 2000, r=30, q_per_row=50, seed=1)
    got, ora, err, _ = run_and_check(icur, A, 1e-6, 10, kind, 3)
    assert got["status"] == "ok" and got["rank"] == 30 and ora["rank"] == 30
    assert err < 1e-6 and got["rho"] < 1e-6


@pytest.mark.parametrize("kind,tol", [(1, 1e-4), (0, 1e-6)])
def test_sparse_decaying_spectrum(icur, kind, tol):
    A = W.sparse_lowrank(2500, 1800, r=120, q_per_row=60, seed=2, decay=1.0 / 15)
    got, ora, err, _ = run_and_check(icur, A, tol, 16, kind, 5)
    assert got["status"] == "ok"
    assert err <= 2 * tol and 0.5 <= got["rho"] / err <= 2.0


def test_sparse_matches_dense_path(icur):
    A = W.sparse_lowrank(2000, 1500, r=40, q_per_row=40, seed=4, decay=1.0 / 20)
    rowptr, colind, vals = W.csr_to_f32(A)
    D32 = W.csr_dense64(rowptr, colind, vals, A.shape).astype(np.float32)
    a = icur.run_csr(*dev_csr(rowptr, colind, vals), A.shape, 1e-4, 8, 1, 9)
    b = icur.run(torch.from_numpy(D32).cuda(), 1e-4, 8, 1, 9)
    # same stopping point; the estimates agree to the dense form's sketch noise (FP32
    # sums over 128-row blocks, about 1e-6 of ||G A||), the CSR sketch being FP64
    assert a["rank"] == b["rank"]
    assert a["rho"] <= 1e-4 and b["rho"] <= 1e-4
    assert abs(a["rho"] - b["rho"]) <= 1e-6
    assert a["J"].tolist()[:8] == b["J"].tolist()[:8]


def test_sparse_edge_cases(icur):
    import scipy.sparse as sp
    # empty rows and columns, a column-heavy and a row-heavy part
    g = np.random.default_rng(0)
    D = np.zeros((400, 300))
    D[::3, :200] = g.standard_normal((134, 200))
    D[:, 250] = g.standard_normal(400)
    A = sp.csr_matrix(D)
    got, ora, err, _ = run_and_check(icur, A, 1e-8, 12, 1, 1)
    # exact rank 135 = 11 blocks + 3: the oracle fills the last block with rounding-noise
    # pivots (its pseudo-inverse drops them again); the GPU ends the row selection at a
    # numerically zero pivot, so its rank is the exact rank
    assert got["rank"] == np.linalg.matrix_rank(D) <= ora["rank"] and err < 1e-8
    # the zero matrix (no entries)
    rowptr = np.zeros(51, np.int64)
    out = icur.run_csr(torch.from_numpy(rowptr).cuda(), torch.zeros(0, dtype=torch.int32, device="cuda"),
                       torch.zeros(0, dtype=torch.float32, device="cuda"), (50, 40), 1e-3, 4)
    assert out["rank"] == 0 and out["rho"] == 0.0 and out["status"] == "ok"


@pytest.mark.parametrize("defect", ["unsorted", "duplicate", "range", "rowptr"])
def test_non_canonical_csr_is_rejected(icur, defect):
    rowptr = np.array([0, 2, 4, 5], np.int64)
    colind = np.array([0, 2, 1, 3, 0], np.int32)
    vals = np.ones(5, np.float32)
    if defect == "unsorted":
        colind[:2] = [2, 0]
    elif defect == "duplicate":
        colind[:2] = [1, 1]
    elif defect == "range":
        colind[4] = 4
    else:
        rowptr[3] = 4
    with pytest.raises(icur.IcurError) as e:
        icur.run_csr(*dev_csr(rowptr, colind, vals), (3, 4), 1e-3, 2)
    assert e.value.status == icur.ERR_ARG


def test_sparse_device_outputs(icur):
    # device_outputs = 1: the same I, J and U, written to device memory
    A = W.sparse_lowrank(2000, 1500, r=40, q_per_row=40, seed=4, decay=1.0 / 20)
    rowptr, colind, vals = W.csr_to_f32(A)
    args = dev_csr(rowptr, colind, vals)
    h = icur.run_csr(*args, A.shape, 1e-4, 8, 1, 9)
    d = icur.run_csr(*args, A.shape, 1e-4, 8, 1, 9, device_outputs=True)
    assert d["U"].is_cuda and h["rank"] == d["rank"] and h["rho"] == d["rho"]
    assert np.array_equal(h["I"], d["I"].cpu().numpy()) and np.array_equal(h["J"], d["J"].cpu().numpy())
    assert np.array_equal(h["U"], d["U"].cpu().numpy())
