"""Step-by-step parity of the HIP path with the FP64 oracle (GPU).

Each §8(a) step of Alg. 1 is called through its C-ABI entry point on seeded inputs and
compared element by element with the oracle on the same inputs:
  sketch operator G     bit-exact (integer generator, BF16 values)
  G A                   within the FP32 accumulation bound (+ BF16 piece truncation)
  LUPP pivots           bit-exact pivot order (FP64 on both sides, same operation order)
  gathers               bit-exact copies
  residual products     within the FP32 / BF16-piece bound
  FP64 core update      within FP64 rounding times the block's condition number
Sizes span several tiles and a ragged tail.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

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


# ----------------------------------------------------------------- FP64 core update
@pytest.mark.parametrize("r,k", [(0, 5), (40, 10), (150, 64), (300, 128), (64, 130)])
def test_core_update_block_inverse(icur, r, k):
    rng = np.random.default_rng(r + k)
    n = r + k
    M = rng.standard_normal((n, n)) + 4 * np.sqrt(n) * np.eye(n)   # well conditioned
    A11, A12, A21, A22 = M[:r, :r], M[:r, r:], M[r:, :r], M[r:, r:]
    Ucap = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    if r:
        Ucap[:r, :r] = torch.from_numpy(np.linalg.inv(A11)).cuda()
    Y = np.linalg.inv(A11) @ A12 if r else np.zeros((0, k))
    icur.core_update(Ucap, r, k, dev(Y), dev(A21), dev(A22))
    got = Ucap.cpu().numpy()
    want = np.linalg.inv(M)
    kappa = np.linalg.cond(M)
    assert np.abs(got - want).max() <= 1e-13 * kappa * np.abs(want).max() * n
