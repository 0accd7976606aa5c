"""Step-by-step parity of the HIP path with the FP64 oracle (GPU).

Each §8(a) step of Alg. 1 is called through its C-ABI entry point on seeded inputs and
compared element by element with the oracle on the same inputs:
  sketch operator G     bit-exact (integer generator, BF16 values)
  G A                   within the FP32 accumulation bound (+ BF16 piece truncation)
  LUPP pivots           bit-exact pivot order (FP64 on both sides, same operation order)
  gathers               bit-exact copies
  residual products     within the FP32 / BF16-piece bound; the FP64 products the loop
                        runs by default (both the library route and the short-M kernel)
                        within the FP64 accumulation bound
  FP64 core update      the oracle's pseudo-inverse within FP64 rounding times the
                        block's condition number
Sizes span several tiles and a ragged tail.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle.icur import pinv_svd                           # noqa: E402
from oracle.lupp import lupp_pivots                        # noqa: E402
from oracle.rng import gaussian_G, sparse_sign_pattern, sparse_sign_G  # noqa: E402

U24 = 2.0 ** -24       # FP32 unit roundoff
U8 = 2.0 ** -8         # BF16 unit roundoff


@pytest.fixture(scope="module")
def icur():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_21963_amd import icur as m
    m.load()
    return m


def bf16_bits(values):
    f = np.asarray(values, dtype=np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


# ----------------------------------------------------------------- sketch operator
@pytest.mark.parametrize("c,m,seed", [(55, 2000, 0), (7, 333, 12345), (140, 1000, 2**40 + 7), (1, 5, 3)])
def test_gaussian_sketch_operator_bit_exact(icur, c, m, seed):
    G, _, _ = icur.make_sketch(seed, c, m, icur.GAUSSIAN)
    got = G.cpu().numpy().view(np.uint16)
    want = bf16_bits(gaussian_G(seed, c, m))
    assert np.array_equal(got, want)


@pytest.mark.parametrize("c,m,zeta,seed", [(110, 4000, 8, 0), (35, 777, 8, 9), (5, 100, 8, 1),
                                           (70, 1000, 3, 2**33)])
def test_sparse_sign_operator_bit_exact(icur, c, m, zeta, seed):
    G, rows, signs = icur.make_sketch(seed, c, m, icur.SPARSE_SIGN, zeta, want_dense=True,
                                      want_pattern=True)
    orows, osigns = sparse_sign_pattern(seed, c, m, zeta)
    assert np.array_equal(rows.cpu().numpy().astype(np.int64), orows)
    bits = signs.cpu().numpy()
    for t in range(orows.shape[1]):
        assert np.array_equal(np.where((bits >> t) & 1, -1.0, 1.0), osigns[:, t])
    assert np.array_equal(G.cpu().numpy().view(np.uint16), bf16_bits(sparse_sign_G(seed, c, m, zeta)))


# ----------------------------------------------------------------- X0 = G A
def _product_bound(Gd, A, K, pieces):
    """Elementwise bound for the FP32 computation of G A: truncation of A to `pieces`
    BF16 pieces (none for 3 or for FP32 products) plus FP32 accumulation over K terms."""
    trunc = {0: 0.0, 1: U8, 2: U8 ** 2, 3: 0.0}[pieces]
    return (trunc + (K + 3) * U24) * (np.abs(Gd) @ np.abs(A))


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("terms", [0, 1, 2, 3])
@pytest.mark.parametrize("c,m,n", [(55, 2000, 1500), (7, 333, 97), (140, 1000, 700), (110, 4096, 130)])
def test_sketch_product(icur, kind, terms, c, m, n):
    rng = np.random.default_rng(c * 1000 + m)
    A32 = rng.standard_normal((m, n)).astype(np.float32)
    A = A32.astype(np.float64)
    G, _, _ = icur.make_sketch(5, c, m, kind)
    Gd = gaussian_G(5, c, m) if kind == 0 else sparse_sign_G(5, c, m)
    X0, nsq = icur.sketch(G, dev(A32), terms)
    X0 = X0.cpu().numpy().astype(np.float64)
    want = Gd @ A
    bound = _product_bound(Gd, A, m, terms)
    assert np.all(np.abs(X0 - want) <= bound)
    assert nsq == pytest.approx(float((X0 ** 2).sum()), rel=1e-12)
    if terms in (0, 3):
        # typical error is far inside the worst-case bound
        assert np.linalg.norm(X0 - want) <= 4 * np.sqrt(m) * U24 * np.linalg.norm(np.abs(Gd) @ np.abs(A))


def test_sketch_exact_on_integer_data(icur):
    # integer A with |sums| < 2^24: every partial sum is exact in FP32
    rng = np.random.default_rng(3)
    m, n, c = 1200, 300, 70
    A32 = rng.integers(-20, 20, size=(m, n)).astype(np.float32)
    G, _, _ = icur.make_sketch(8, c, m, icur.SPARSE_SIGN)
    X0, _ = icur.sketch(G, dev(A32), 3)
    assert np.array_equal(X0.cpu().numpy().astype(np.float64), sparse_sign_G(8, c, m) @ A32.astype(np.float64))


# ----------------------------------------------------------------- LUPP selection
LUPP_CASES = [
    # K, N, steps, excluded fraction, seed
    (55, 1500, 50, 0.0, 0),
    (33, 300, 33, 0.1, 1),        # ragged last panel
    (16, 257, 16, 0.0, 2),        # one panel, ragged groups
    (1, 40, 1, 0.0, 3),
    (110, 40000, 100, 0.01, 4),   # column selection at the 40000-column RBF shape
    (40, 6000, 40, 0.0, 9),       # two rows per thread
    (48, 12000, 48, 0.05, 10),    # four rows per thread, 256 threads
    (64, 70000, 64, 0.0, 5),      # four rows per thread, 512 threads
    (40, 30000, 40, 0.02, 12),    # two rows per thread, 256 threads, 59 workgroups
    (70, 200000, 64, 0.001, 6),
    (20, 300000, 20, 0.0, 7),
    (130, 5000, 128, 0.2, 8),     # 8 panels
    (600, 2000, 600, 0.0, 11),    # pivot rows of 37 panels: more than 64 KB of LDS
]


@pytest.mark.parametrize("K,N,steps,frac,seed", LUPP_CASES)
def test_lupp_pivots_bit_exact(icur, K, N, steps, frac, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((K, N)).astype(np.float32)
    excl = (rng.random(N) < frac)
    excl_idx = np.nonzero(excl)[0].tolist()
    got = icur.lupp(dev(X), steps, dev(excl.astype(np.uint8)) if frac else None)
    want = lupp_pivots(X.astype(np.float64).T, steps, exclude=excl_idx)
    assert got.tolist() == want


def test_lupp_degenerate_inputs(icur):
    # rank one with power-of-two entries: every elimination step is exact, so the
    # Schur complement is exactly zero after one pivot and the selection stops
    u = (2.0 ** np.random.default_rng(1).permutation(np.arange(-20, 20))).astype(np.float32)
    X = np.stack([u, -2 * u, 0.5 * u])
    assert icur.lupp(dev(X), 3).tolist() == [int(np.argmax(u))]
    # rank one in general: rounding leaves a tiny Schur complement; same pivots as FP64
    v = np.arange(1.0, 301.0, dtype=np.float32)
    Xv = np.stack([v, -2 * v, 0.5 * v])
    assert icur.lupp(dev(Xv), 3).tolist() == lupp_pivots(Xv.astype(np.float64).T, 3)
    assert icur.lupp(dev(np.zeros((4, 100), np.float32)), 4).tolist() == []
    ties = np.ones((2, 600), np.float32)                      # ties -> lowest index
    assert icur.lupp(dev(ties), 1).tolist() == [0]
    excl = np.ones(50, np.uint8)
    excl[[7, 31]] = 0                                         # only two candidates
    Y = np.random.default_rng(0).standard_normal((5, 50)).astype(np.float32)
    got = icur.lupp(dev(Y), 5, dev(excl)).tolist()
    assert got == lupp_pivots(Y.astype(np.float64).T, 5, exclude=np.nonzero(excl)[0].tolist())
    assert len(got) == 2
    # the Schur complement becomes exactly zero in the middle of the second panel: the
    # selection ends there, in every workgroup at once
    Z = np.zeros((40, 20000), np.float32)
    Z[:21] = np.random.default_rng(2).standard_normal((21, 20000))
    got = icur.lupp(dev(Z), 40).tolist()
    assert got == lupp_pivots(Z.astype(np.float64).T, 40) and len(got) == 21


def test_lupp_repeatable(icur):
    X = dev(np.random.default_rng(9).standard_normal((110, 40000)).astype(np.float32))
    a = icur.lupp(X, 100)
    b = icur.lupp(X, 100)
    assert a.tolist() == b.tolist()


# ----------------------------------------------------------------- gathers
def test_gathers_bit_exact(icur):
    rng = np.random.default_rng(4)
    m, n = 1001, 777
    A32 = rng.standard_normal((m, n)).astype(np.float32)
    A = dev(A32)
    cols = rng.choice(n, 37, replace=False)
    rows = rng.choice(m, 41, replace=False)
    Ct = icur.gather_cols_T(A, dev(cols.astype(np.int64))).cpu().numpy()
    R = icur.gather_rows(A, dev(rows.astype(np.int64))).cpu().numpy()
    assert np.array_equal(Ct, A32[:, cols].T)
    assert np.array_equal(R, A32[rows, :])


# ----------------------------------------------------------------- residual products
def _residual_bound(X, W, B, K, terms):
    trunc = {0: U24, 1: 3 * U8, 2: 3 * U8 ** 2, 3: 4 * U24}[terms]
    return (trunc + (K + 3) * U24) * (np.abs(X) + np.abs(W) @ np.abs(B))


@pytest.mark.parametrize("terms", [0, 1, 2, 3])
@pytest.mark.parametrize("M,K,N", [(110, 100, 40000 // 8), (140, 700, 3001), (100, 0, 500),
                                   (5, 33, 64), (160, 250, 1000), (200, 96, 513)])
def test_residual_product(icur, terms, M, K, N):
    rng = np.random.default_rng(M + K + N)
    W = rng.standard_normal((M, K))
    B32 = rng.standard_normal((K, N)).astype(np.float32)
    X32 = rng.standard_normal((M, N)).astype(np.float32)
    out, nsq = icur.residual(dev(X32), dev(W), dev(B32), terms)
    got = out.cpu().numpy().astype(np.float64)
    X, B = X32.astype(np.float64), B32.astype(np.float64)
    want = X - W @ B
    assert np.all(np.abs(got - want) <= _residual_bound(X, W, B, K, terms))
    assert nsq == pytest.approx(float((got ** 2).sum()), rel=1e-12)


@pytest.mark.parametrize("M,K,N,inplace", [
    (110, 100, 40000, True),    # column residual shape of the 40000^2 run: library route (wide rows)
    (128, 512, 3001, True),     # deep products of tall blocks: library route
    (128, 512, 3001, False),    # same shape with a separate X: short-M kernel
    (100, 0, 700, True),        # empty depth
    (32, 700, 5000, True),      # short blocks stay on the short-M kernel
    (35, 33, 8191, False),      # ragged tails
    (140, 128, 40000, None),    # plain product OUT = W B (Ur_k = N_k^{-1} S(I_k,:))
])
def test_residual_product_fp64(icur, M, K, N, inplace):
    # the default residual-form arithmetic: FP64 factors and FP64 output; exact products
    # summed in FP64, so |error| <= (K + 2) 2^-52 (|X| + |W| |B|) elementwise
    rng = np.random.default_rng(M * 7 + K + N)
    W = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    X = rng.standard_normal((M, N))
    Wd, Bd = dev(W), dev(B)
    if inplace is None:
        out, nsq = icur.residual_f64(None, Wd, Bd)
        want = W @ B
        bound = (K + 2) * 2.0 ** -52 * (np.abs(W) @ np.abs(B))
    else:
        Xd = dev(X)
        out, nsq = icur.residual_f64(Xd, Wd, Bd, out=Xd if inplace else None)
        want = X - W @ B
        bound = (K + 2) * 2.0 ** -52 * (np.abs(X) + np.abs(W) @ np.abs(B))
    got = out.cpu().numpy()
    assert np.all(np.abs(got - want) <= bound)
    assert nsq == pytest.approx(float((got ** 2).sum()), rel=1e-12)


# ----------------------------------------------------------------- SRTT operator
@pytest.mark.parametrize("c,m,seed", [(11, 97, 3), (110, 40000, 0), (35, 8000, 5), (64, 64, 1)])
def test_srtt_operator_matches_oracle(icur, c, m, seed):
    # kept rows bit-exact (integer generator); entries the oracle's FP64 cosines rounded to
    # FP32 (device cos within a few FP64 ulps, far below the FP32 rounding)
    from oracle.rng import srtt_G, srtt_rows
    G, rows = icur.make_srtt(seed, c, m)
    assert rows.cpu().numpy().tolist() == srtt_rows(seed, c, m).tolist()
    want = srtt_G(seed, c, m)
    got = G.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - want) <= U24 * np.abs(want) + 1e-15)


# ----------------------------------------------------------------- QRCP selection
@pytest.mark.parametrize("K,N,steps,excl_frac,seed", [
    (55, 1500, 50, 0.0, 0), (110, 40000, 100, 0.01, 1), (16, 257, 16, 0.0, 2), (1, 40, 1, 0.0, 3),
    (35, 8000, 32, 0.1, 4), (140, 5000, 128, 0.0, 5)])
def test_qrcp_pivots_match_oracle(icur, K, N, steps, excl_frac, seed):
    # generic inputs (norm ties only at rounding level): the pivot order of the GPU's
    # orthogonalised residuals equals the oracle's Householder QRCP
    from oracle.qrcp import qrcp_pivots
    rng = np.random.default_rng(seed)
    X = (rng.standard_normal((K, N)) * np.exp(rng.standard_normal(N))[None, :]).astype(np.float32)
    ex = rng.random(N) < excl_frac
    exd = dev(ex.astype(np.uint8)) if excl_frac else None
    got = icur.qrcp(dev(X), steps, exd).tolist()
    want = qrcp_pivots(X.astype(np.float64).T, steps, exclude=np.nonzero(ex)[0].tolist())
    assert got == want


def test_qrcp_degenerate_inputs(icur):
    # three nonzero candidates among zeros: the selection ends after them
    X = np.zeros((5, 30), np.float32)
    X[:, [4, 9, 20]] = np.random.default_rng(0).standard_normal((5, 3)).astype(np.float32)
    assert sorted(icur.qrcp(dev(X), 5).tolist()) == [4, 9, 20]
    # equal norms: the lowest index
    E = np.hstack([np.eye(3), np.eye(3)]).astype(np.float32)
    assert icur.qrcp(dev(E), 3).tolist() == [0, 1, 2]


# ----------------------------------------------------------------- FP64 core update
@pytest.mark.parametrize("r,k", [(0, 5), (40, 10), (150, 64), (300, 128), (64, 130)])
def test_core_update_block_inverse(icur, r, k):
    # the bordered core against the oracle's core (the SVD pseudo-inverse of the whole
    # cross, which it recomputes every iteration): both are backward stable, so they
    # differ by a few cond 2^-52 relative
    rng = np.random.default_rng(r + k)
    n = r + k
    M = rng.standard_normal((n, n)) + 4 * np.sqrt(n) * np.eye(n)   # well conditioned
    A11, A12, A21, A22 = M[:r, :r], M[:r, r:], M[r:, :r], M[r:, r:]
    Ucap = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    U11 = pinv_svd(A11) if r else np.zeros((0, 0))
    if r:
        Ucap[:r, :r] = torch.from_numpy(U11).cuda()
    Y = U11 @ A12 if r else np.zeros((0, k))
    icur.core_update(Ucap, r, k, dev(Y), dev(A21), dev(A22))
    got = Ucap.cpu().numpy()
    want = pinv_svd(M)
    kappa = np.linalg.cond(M)
    assert np.abs(got - want).max() <= 16 * n * kappa * 2.0 ** -52 * np.abs(want).max()


@pytest.mark.parametrize("case", ["cond1e2", "cond1e6", "lupp_cross"])
def test_core_update_chain_matches_oracle_recompute(icur, case):
    # grow the core block by block, as the loop would, and compare with the oracle's
    # pseudo-inverse recomputed from scratch at every size.  Random crosses of condition
    # 1e2 and 1e6, and the cross the oracle's own selections build at tol 1e-6 on a planted
    # spectrum sigma_i = exp(-i/22) (its rows and columns in selection order, the order the
    # loop borders in; cond about 6e8): there the Schur complements stay well scaled
    # although the cross is not.  Pushed to tol 1e-9 the same spectrum gives a cross of
    # cond 5e19, numerically singular in FP64, where bordering (like any explicit inverse)
    # no longer tracks the pseudo-inverse to a bound linear in cond.
    if case == "lupp_cross":
        from oracle.icur import iterative_cur
        from paper_2509_21963_amd import workloads as W
        A, _ = W.planted_geometric(600, 500, 22.0, seed=3)
        ora = iterative_cur(A, 1e-6, 40, seed=1)
        M = A[np.ix_(ora["I"], ora["J"])]
        n, k = M.shape[0], 40
    else:
        cond_target = 1e2 if case == "cond1e2" else 1e6
        rng = np.random.default_rng(int(np.log10(cond_target)))
        n, k = 200, 40
        Q1, _ = np.linalg.qr(rng.standard_normal((n, n)))
        Q2, _ = np.linalg.qr(rng.standard_normal((n, n)))
        M = (Q1 * np.logspace(0, -np.log10(cond_target), n)) @ Q2.T
    Ucap = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    for r in range(0, n, k):
        kk = min(k, n - r)
        A12, A21, A22 = M[:r, r:r + kk], M[r:r + kk, :r], M[r:r + kk, r:r + kk]
        Ucur = Ucap[:r, :r].cpu().numpy()
        icur.core_update(Ucap, r, kk, dev(Ucur @ A12 if r else np.zeros((0, kk))), dev(A21), dev(A22))
        sub = M[:r + kk, :r + kk]
        want = pinv_svd(sub)
        got = Ucap[:r + kk, :r + kk].cpu().numpy()
        kappa = np.linalg.cond(sub)
        # each update adds about n kappa 2^-52 |U| and carries the earlier error on, so
        # the bound grows with the number of blocks
        blocks = r // k + 1
        assert np.abs(got - want).max() <= 16 * n * blocks * kappa * 2.0 ** -52 * np.abs(want).max(), (r, kappa)
    print("core chain %s: %d blocks, final cond %.2e" % (case, blocks, kappa))
