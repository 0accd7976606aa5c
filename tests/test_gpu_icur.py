"""End-to-end parity of icur_run with the FP64 oracle (GPU).

IterativeCUR is a greedy, randomized iteration, so the HIP path and the oracle agree on
the unique part of the result and are checked for validity on the rest:
  * every pivot of every block is replayed through the oracle along the GPU's own
    trajectory (tests/_replay.py): each GPU choice lies in the set the oracle's values
    allow within the rounding of both sides, and equals the oracle's argmax wherever
    that set has one member ("pinned" steps; each test reports how many);
  * U equals the oracle's pseudo-inverse of the same cross A(I,J) to cond 2^-52;
  * the final exact error ||A - CUR||_F / ||A||_F (computed on the host in FP64 from the
    GPU's I, J, U) is at most 2 tol (the estimate's spread; see the risk-aware tests
    for the tol bar itself), and the estimate rho is within a factor 2 of it;
  * the residual vanishes on the selected rows and columns.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle.icur import exact_relative_error, iterative_cur, pinv_svd   # noqa: E402
from paper_2509_21963_amd import workloads as W               # noqa: E402
from _replay import residual_eta, replay, sketch_eta                          # noqa: E402


@pytest.fixture(scope="module")
def icur():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_21963_amd import icur as m
    m.load()
    return m


def form_eta(got, tol, precision, sketch_fp32=False):
    """Sketch rounding of the run's form (see tests/_replay.py)."""
    chunk = 32 if tol < 1e-4 else 128
    if precision:
        return sketch_eta(got["info"]["split_terms"], chunk)
    return sketch_eta(0 if sketch_fp32 else 3, 32 if sketch_fp32 else chunk)


def check_against_oracle(icur, A32, tol, b, kind, seed, precision=0, eta=None, eta_row=0.0, **kw):
    selection = "qrcp" if kw.get("selection") == 1 else "lupp"
    A64 = A32.astype(np.float64)
    got = icur.run(torch.from_numpy(A32).cuda(), tol, b, kind, seed, precision, **kw)
    r = got["rank"]
    I, J, U = got["I"].tolist(), got["J"].tolist(), got["U"]
    assert len(set(I)) == r and len(set(J)) == r
    if eta is None:
        eta = form_eta(got, tol, precision, kw.get("sketch_fp32", False))
        # FP32 factors (the precision form's default, or residual_fp64 = -1): the residual
        # products' rounding enters the row residual directly and the sketched residual
        # through Ur_k
        if got["info"]["residual_terms"] >= 0:
            er = residual_eta(got["info"]["residual_terms"])
            eta_row = max(eta_row, er)
            eta = eta + 4 * er
    # every pivot of the GPU run, replayed through the oracle along the GPU's trajectory
    denominator = "A" if kw.get("denominator") == 1 else "GA"
    stats, rep = replay(A64, I, J, got["info"]["block_sizes"], tol, b, kind, seed, eta,
                        zeta=kw.get("zeta") or 8, max_rank=kw.get("max_rank") or None, eta_row=eta_row,
                        selection=selection, denominator=denominator)
    got["parity"] = stats
    print("pivot parity", stats)
    assert stats["col_pinned"] > 0 and stats["row_pinned"] > 0
    ora = iterative_cur(A64, tol, b, kind=kind, seed=seed, record=True,
                        max_rank=kw.get("max_rank") or None, selection=selection, denominator=denominator)
    # U against the oracle's pseudo-inverse of the same cross: both are backward stable,
    # so they differ by at most a few cond(A(I,J)) 2^-52 relative
    err = exact_relative_error(A64, I, J, U) if r else 1.0
    if r:
        core = A64[np.ix_(I, J)]
        Uo = pinv_svd(core)
        assert np.abs(U - Uo).max() <= 16 * r * np.linalg.cond(core) * 2.0 ** -52 * np.abs(Uo).max()
    return got, ora, err


def test_planted_spectrum_2000x1500_fp32(icur):
    # tol 1e-6 on a cross with condition ~1e8: the residual factors run in FP64
    A, _ = W.planted_geometric(2000, 1500, 40.0, seed=0)
    A32, _ = W.to_f32(A)
    got, ora, err = check_against_oracle(icur, A32, 1e-6, 50, 0, 0)
    assert got["status"] == "ok" and got["rho"] <= 1e-6
    assert err <= 2e-6 and 0.5 <= got["rho"] / err <= 2.0
    assert abs(got["rank"] - ora["rank"]) <= 50
    assert got["info"]["iterations"] == len(got["info"]["rho"])


@pytest.mark.parametrize("res64", [1, -1])
def test_residual_factor_precision_switch(icur, res64):
    # tol 1e-4 is well above the FP32 floor: both factor precisions meet it
    A, _ = W.planted_geometric(1200, 1000, 30.0, seed=6)
    A32, _ = W.to_f32(A)
    # FP32 factors on the FP32 matrix cores (plain form, residual_fp64 = -1): the row
    # residual carries their rounding; N_k^{-1} S(I_k,:) stays FP64
    got, ora, err = check_against_oracle(icur, A32, 1e-4, 32, 0, 6, residual_fp64=res64)
    assert got["status"] == "ok" and err <= 2e-4 and 0.5 <= got["rho"] / err <= 2.0


@pytest.mark.parametrize("form,tol", [(0, 1e-6), (1, 1e-4)])
def test_exact_rank_inside_a_block(icur, form, tol):
    # rank 25 with b = 10: the third block holds 5 real pivots and then noise (the FP32
    # rounding of A, near 1e-7, and the form's own rounding).  The block stays stable
    # (the row selection ends at a numerically zero pivot when the noise is the factors'
    # rounding) and the loop stops after it
    A32, _ = W.to_f32(W.exact_lowrank(500, 400, 25, seed=8))
    got = icur.run(torch.from_numpy(A32).cuda(), tol, 10, 1, 2, precision=form)
    A = A32.astype(np.float64)
    err = exact_relative_error(A, got["I"].tolist(), got["J"].tolist(), got["U"])
    assert got["status"] == "ok" and 25 <= got["rank"] <= 30
    assert err < tol and got["rho"] < tol


@pytest.mark.parametrize("kind", [0, 1])
def test_exact_low_rank_recovery(icur, kind):
    A32, _ = W.to_f32(W.exact_lowrank(400, 300, 30, seed=5))
    got, ora, err = check_against_oracle(icur, A32, 1e-5, 10, kind, 1)
    assert got["rank"] == 30
    assert err < 1e-5 and got["rho"] < 1e-5


@pytest.mark.parametrize("seed", [0, 1])
def test_rbf_sparse_sign(icur, seed):
    A32, _ = W.to_f32(W.rbf(1500, 1200, seed))
    got, ora, err = check_against_oracle(icur, A32, 1e-4, 20, 1, seed)
    assert got["status"] == "ok"
    assert err <= 2e-4 and 0.5 <= got["rho"] / err <= 2.0


@pytest.mark.parametrize("tol", [1e-2, 1e-3, 1e-5])
def test_bf16_split_form(icur, tol):
    A, _ = W.planted_geometric(3000, 2000, 60.0, seed=3)
    A32, _ = W.to_f32(A)
    got, ora, err = check_against_oracle(icur, A32, tol, 64, 0, 3, precision=1)
    assert got["status"] == "ok"
    assert err <= 2 * tol and 0.5 <= got["rho"] / err <= 2.0
    assert got["info"]["split_terms"] == (1 if tol >= 1e-1 else 2 if tol >= 5e-4 else 3)
    assert got["info"]["residual_terms"] == (2 if tol >= 1e-1 else 3 if tol >= 1e-4 else -1)


@pytest.mark.parametrize("kind", [0, 1])
def test_qrcp_selection_matches_oracle(icur, kind):
    # Alg. 1 with QRCP for both selections (§5.3): every pivot replayed through the
    # oracle's QRCP along the GPU's trajectory, and the same quality as LUPP
    A, _ = W.planted_geometric(1500, 1200, 30.0, seed=5)
    A32, _ = W.to_f32(A)
    got, ora, err = check_against_oracle(icur, A32, 1e-5, 32, kind, 2, selection=1)
    lu = icur.run(torch.from_numpy(A32).cuda(), 1e-5, 32, kind, 2)
    assert got["status"] == "ok" and err <= 2e-5 and 0.5 <= got["rho"] / err <= 2.0
    assert abs(got["rank"] - ora["rank"]) <= 32 and abs(got["rank"] - lu["rank"]) <= 64


@pytest.mark.parametrize("denominator", [0, 1])
def test_srtt_sketch_matches_oracle(icur, denominator):
    # the SRTT operator (FP32 values on FP32 matrix cores, 32-deep chunks summed in FP64):
    # every pivot replayed through the oracle's SRTT run
    A, _ = W.planted_geometric(2000, 1500, 30.0, seed=7)
    A32, _ = W.to_f32(A)
    got, ora, err = check_against_oracle(icur, A32, 1e-5, 40, icur.SRTT, 4, eta=sketch_eta(0, 32),
                                         denominator=denominator)
    assert got["status"] == "ok" and err <= 2e-5 and 0.5 <= got["rho"] / err <= 2.0
    assert abs(got["rank"] - ora["rank"]) <= 40


def test_fp32_matrix_core_sketch_option(icur):
    A32, _ = W.to_f32(W.planted_geometric(800, 600, 30.0, seed=4)[0])
    got, ora, err = check_against_oracle(icur, A32, 1e-5, 16, 0, 4, sketch_fp32=True)
    assert err <= 2e-5


def test_dense_sketch_runs_on_the_sketch_kernel(icur):
    # G A of the BF16-exact operators goes through the dedicated streaming kernel (not the
    # general product) for row-aligned inputs, in both forms and in the grouped batch
    g = torch.Generator(device="cuda").manual_seed(3)
    A = torch.randn(2000, 1500, generator=g, device="cuda", dtype=torch.float32)
    for kind in (0, 1):
        for precision in (icur.FP32, icur.BF16_SPLIT):
            icur.run(A, 1e-2, 50, kind, 0, precision=precision)
            assert icur.last_info()["sketch_kernel"] == 1, (kind, precision)
    icur.run(A, 1e-2, 50, icur.SRTT, 0)
    assert icur.last_info()["sketch_kernel"] == 0  # the SRTT operator runs on the general product
    mats = [A[:700, :600].contiguous(), A[:900, :1200].contiguous(), A[:520, :804].contiguous()]
    icur.run_batched(mats, [1e-2] * 3, 32)
    assert icur.last_info()["sketch_kernel"] == 3


@pytest.mark.parametrize("b", [129, 250, 512])
def test_large_blocks_blocked_pivot_inverse(icur, b):
    # blocks above 128 invert their pivot blocks (and the core's diagonal blocks) by 2 x 2
    # block elimination over 128-wide in-order Gauss-Jordan tiles: every pivot replayed,
    # and U against the oracle's pseudo-inverse of the cross (check_against_oracle)
    A, _ = W.planted_geometric(1800, 1400, 45.0, seed=11)
    A32, _ = W.to_f32(A)
    got, ora, err = check_against_oracle(icur, A32, 1e-6, b, 0, 5)
    assert got["status"] == "ok" and got["rank"] >= b
    assert err <= 2e-6 and got["rho"] <= 1e-6


def test_schur_zeros_of_the_result(icur):
    A32, _ = W.to_f32(W.rbf(900, 700, 2))
    got = icur.run(torch.from_numpy(A32).cuda(), 1e-5, 16, 0, 7)
    A = A32.astype(np.float64)
    I, J, U = got["I"], got["J"], got["U"]
    S = A - A[:, J] @ U @ A[I, :]
    scale = np.abs(A).max()
    assert np.abs(S[I, :]).max() < 1e-9 * scale * np.linalg.cond(A[np.ix_(I, J)])
    assert np.abs(S[:, J]).max() < 1e-9 * scale * np.linalg.cond(A[np.ix_(I, J)])


def test_degenerate_and_edge_cases(icur):
    z = torch.zeros((300, 200), dtype=torch.float32, device="cuda")
    out = icur.run(z, 1e-3, 8)
    assert out["rank"] == 0 and out["rho"] == 0.0 and out["status"] == "ok"
    bad = torch.ones((300, 200), dtype=torch.float32, device="cuda")
    bad[5, 7] = float("nan")
    with pytest.raises(icur.IcurError) as e:
        icur.run(bad, 1e-3, 8)
    assert e.value.status == icur.ERR_NONFINITE
    # a tolerance the empty approximation already meets (rho starts at 1): no iteration,
    # and the sketch norm is still checked
    with pytest.raises(icur.IcurError) as e:
        icur.run(bad, 1.0, 8)
    assert e.value.status == icur.ERR_NONFINITE
    # max_rank cap
    A32, _ = W.to_f32(W.rbf(400, 300, 1, h=0.05))
    out = icur.run(torch.from_numpy(A32).cuda(), 1.0, 8)
    assert out["rank"] == 0 and out["status"] == "ok" and out["info"]["iterations"] == 0
    assert out["info"]["sketch_norm"] > 0.0
    out = icur.run(torch.from_numpy(A32).cuda(), 1e-12, 7, max_rank=20)
    assert out["status"] == "maxrank" and out["rank"] == 20
    # exhaustion of a full-rank matrix with a shortened last block (23 = 4*5 + 3)
    R32 = np.random.default_rng(0).standard_normal((30, 23)).astype(np.float32)
    out = icur.run(torch.from_numpy(R32).cuda(), 1e-12, 5)
    assert out["rank"] == 23
    # block 1 and the smallest shapes
    out = icur.run(torch.from_numpy(W.to_f32(W.rbf(50, 40, 3))[0]).cuda(), 1e-3, 1)
    assert out["status"] == "ok" and out["rank"] >= 1
    one = torch.full((1, 1), 2.0, device="cuda")
    out = icur.run(one, 1e-3, 1)
    assert out["rank"] == 1 and out["I"].tolist() == [0] and out["U"][0, 0] == 0.5


def test_repeatable_and_seed_dependent(icur):
    A = torch.from_numpy(W.to_f32(W.rbf(1000, 800, 5))[0]).cuda()
    a = icur.run(A, 1e-4, 10, 0, 11)
    b = icur.run(A, 1e-4, 10, 0, 11)
    c = icur.run(A, 1e-4, 10, 0, 12)
    assert a["I"].tolist() == b["I"].tolist() and a["J"].tolist() == b["J"].tolist()
    assert a["rho"] == b["rho"]
    assert a["J"].tolist() != c["J"].tolist()


def test_risk_aware_threshold(icur):
    A32, _ = W.to_f32(W.planted_geometric(600, 500, 30.0, seed=1)[0])
    out = icur.run(torch.from_numpy(A32).cuda(), 1e-4, 91, alpha=1e-10)   # c = 100
    assert out["info"]["threshold"] == pytest.approx(1e-4 / 4.98, rel=1e-3)
    assert out["rho"] <= 1e-4 / 4.98


def test_strided_input_leading_dimension(icur):
    big = torch.from_numpy(W.to_f32(W.rbf(600, 900, 4))[0]).cuda()
    view = big[:, :700]                     # lda = 900 > n = 700
    A32 = np.ascontiguousarray(big.cpu().numpy()[:, :700])
    a = icur.run(view, 1e-4, 12, 0, 2)
    b = icur.run(torch.from_numpy(A32).cuda(), 1e-4, 12, 0, 2)
    assert a["J"].tolist() == b["J"].tolist() and a["I"].tolist() == b["I"].tolist()


def test_smooth_kernel_estimate_matches_oracle(icur):
    # RBF kernel: the pivots of one block of 100 decay by about five orders, so N_k is
    # ill-conditioned.  The estimate after the first block must agree with the oracle's
    # (an N_k^{-1} rounded to FP32 before it multiplies puts an error near 1e-2 on it and
    # costs a second iteration); same rank, same iteration count
    A32, _ = W.to_f32(W.rbf(6000, 5000, seed=0))
    got, ora, err = check_against_oracle(icur, A32, 1e-4, 100, 1, 0, zeta=8)
    assert got["status"] == "ok"
    assert got["rank"] == ora["rank"]
    assert got["info"]["iterations"] == len(ora["history"])
    assert 0.8 <= got["rho"] / ora["rho"] <= 1.25
    assert err <= 2e-4 and 0.5 <= got["rho"] / err <= 2.0


def test_deep_products_on_the_native_gemm(icur, monkeypatch):
    # ICUR_NATIVE_GEMM=1 runs the deep residual products and the core's block products on
    # the library's own FP64 matrix-core kernel instead of rocBLAS: the same parity bar
    monkeypatch.setenv("ICUR_NATIVE_GEMM", "1")
    A, _ = W.planted_geometric(3000, 2500, 80.0, seed=4)
    A32, _ = W.to_f32(A)
    got, ora, err = check_against_oracle(icur, A32, 1e-6, 128, 0, 3)
    assert got["rank"] >= 512 and got["info"]["iterations"] >= 4
    assert got["status"] == "ok" and err <= 2e-6 and 0.5 <= got["rho"] / err <= 2.0
    assert abs(got["rank"] - ora["rank"]) <= 128


def test_deep_products_on_the_library_gemm(icur):
    # blocks of 128 rows and ranks past 256: the row residual and the residual at the new
    # rows run as library FP64 GEMMs (depth >= 256), the others on the short-M kernel
    A, _ = W.planted_geometric(3000, 2500, 80.0, seed=4)
    A32, _ = W.to_f32(A)
    got, ora, err = check_against_oracle(icur, A32, 1e-6, 128, 0, 3)
    assert got["rank"] >= 512 and got["info"]["iterations"] >= 4
    assert got["status"] == "ok" and err <= 2e-6 and 0.5 <= got["rho"] / err <= 2.0
    assert abs(got["rank"] - ora["rank"]) <= 128


@pytest.mark.parametrize("shape,tol,b", [((400, 300), 1e-3, 8), ((2000, 1500), 1e-6, 64)])
def test_device_outputs_equal_host_outputs(icur, shape, tol, b):
    # device_outputs = 1 writes I, J and U to device memory instead of the host (the small
    # case goes through the pinned staging area on the host path, the large one past it);
    # the values are the same bytes
    A32, _ = W.to_f32(W.planted_geometric(shape[0], shape[1], 40.0 if shape[0] < 1000 else 100.0, seed=2)[0])
    A = torch.from_numpy(A32).cuda()
    h = icur.run(A, tol, b, 0, 5)
    d = icur.run(A, tol, b, 0, 5, device_outputs=True)
    assert d["U"].is_cuda and d["I"].is_cuda
    assert h["rank"] == d["rank"] and h["rho"] == d["rho"] and h["status"] == d["status"]
    assert np.array_equal(h["I"], d["I"].cpu().numpy()) and np.array_equal(h["J"], d["J"].cpu().numpy())
    assert np.array_equal(h["U"], d["U"].cpu().numpy())
    if shape[0] == 2000:
        assert h["rank"] * h["rank"] * 8 > 2 << 20
