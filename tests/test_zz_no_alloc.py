"""icur_lupp_noalloc (the entry point that allocates nothing) against icur_lupp (GPU).

Both calls go through the C-ABI on the same seeded inputs; the pivots must be identical
(both are bit-exact FP64 LUPP).  Two calls in a row, the second on a smaller input, show
that nothing left in the shared scratch area by the first call leaks into the second.
Also checked: the oracle's pivots, and the size limit (an argument error, before any
device work).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle.lupp import lupp_pivots  # noqa: E402


@pytest.fixture(scope="module")
def icur():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_21963_amd import icur as m
    m.load()
    m.init_noalloc()
    return m


def _case(K, N, frac, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((K, N)).astype(np.float32)
    excl = (rng.random(N) < frac).astype(np.uint8)
    return X, excl


@pytest.mark.parametrize("first,second", [
    ((110, 40000, 100, 0.01, 4), (55, 1500, 50, 0.0, 0)),     # C2 column selection, then C1-sized
    ((64, 70000, 64, 0.0, 5), (33, 300, 33, 0.1, 1)),          # several workgroups, then one
])
def test_noalloc_matches_allocating_entry(icur, first, second):
    print("noalloc case", first, second, flush=True)
    for K, N, steps, frac, seed in (first, second):
        X, excl = _case(K, N, frac, seed)
        Xd = torch.from_numpy(X).cuda()
        ex = torch.from_numpy(excl).cuda() if frac else None
        want = icur.lupp(Xd, steps, ex)
        piv = torch.full((steps,), -1, dtype=torch.int64, device="cuda")
        npiv = icur.lupp_noalloc(Xd, steps, piv, ex)
        got = piv[:npiv].cpu().numpy()
        assert got.tolist() == want.tolist()
        if N <= 40000:
            ora = lupp_pivots(X.astype(np.float64).T, steps, exclude=np.nonzero(excl)[0].tolist())
            assert got.tolist() == ora


def test_noalloc_rejects_requests_above_its_scratch(icur):
    # checked before any device work: a pointer that is never dereferenced will do
    import ctypes
    lib = icur.load()
    fake = ctypes.c_void_p(0x1000)
    npiv = ctypes.c_int32(-1)
    # 256 steps over 40000 candidates need about 87 MB, above the 48 MiB area
    st = lib.icur_lupp_noalloc(fake, 256, 40000, 40000, 256, None, fake, ctypes.byref(npiv), None)
    assert st == icur.ERR_ARG and b"scratch" in lib.icur_last_error()
    st = lib.icur_lupp_noalloc(fake, 300, 1000, 1000, 257, None, fake, ctypes.byref(npiv), None)
    assert st == icur.ERR_ARG                      # steps above 256
    st = lib.icur_lupp_noalloc(fake, 8, 8, 8, 9, None, fake, ctypes.byref(npiv), None)
    assert st == icur.ERR_ARG                      # steps > K
    assert npiv.value == -1                        # nothing written on an argument error
