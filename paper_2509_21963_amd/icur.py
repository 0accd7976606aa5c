"""Python binding of libicur (ctypes).

Argument marshalling only: every step of IterativeCUR runs in the HIP kernels of
libicur.so.  Device buffers are torch CUDA (HIP) tensors; the binding passes their
pointers and the current torch stream.  If the library has not been built this module
raises on import of the library (there is no fallback path).

Function names follow the C entry points in include/icur.h without the `icur_` prefix.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libicur.so")

OK, MAXRANK, STALLED = 0, 1, 2
ERR_ARG, ERR_NONFINITE, ERR_NOMEM, ERR_HIP, ERR_UNSUPPORTED = -1, -2, -3, -4, -5
GAUSSIAN, SPARSE_SIGN, SRTT = 0, 1, 2
FP32, BF16_SPLIT = 0, 1
DENOM_GA, DENOM_A = 0, 1
LUPP, QRCP = 0, 1

_STATUS_NAMES = {0: "ok", 1: "maxrank", 2: "stalled", -1: "bad argument",
                 -2: "non-finite input", -3: "out of device memory", -4: "HIP error",
                 -5: "unsupported shape"}


class IcurError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("libicur: %s (%d): %s" % (_STATUS_NAMES.get(status, "?"), status, message))
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("zeta", ctypes.c_int32),
                ("max_rank", ctypes.c_int64), ("stream", ctypes.c_void_p),
                ("alpha", ctypes.c_double), ("delta", ctypes.c_double),
                ("split_terms", ctypes.c_int32), ("sketch_fp32", ctypes.c_int32),
                ("residual_fp64", ctypes.c_int32), ("batch_workers", ctypes.c_int32),
                ("denominator", ctypes.c_int32), ("selection", ctypes.c_int32),
                ("device_outputs", ctypes.c_int32), ("pad_opts", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("split_terms", ctypes.c_int32),
                ("sketch_norm", ctypes.c_double), ("threshold", ctypes.c_double),
                ("ms_total", ctypes.c_double), ("ms_sketch", ctypes.c_double),
                ("ms_select", ctypes.c_double), ("ms_residual", ctypes.c_double),
                ("ms_core", ctypes.c_double), ("ms_sketch_product", ctypes.c_double),
                ("n_rho", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("rho", ctypes.c_double * 512),
                ("block_sizes", ctypes.c_int32 * 512),
                ("ms_products", ctypes.c_double), ("product_bytes", ctypes.c_double),
                ("product_launches", ctypes.c_int32), ("group_iterations", ctypes.c_int32),
                ("ms_setup", ctypes.c_double), ("ms_results", ctypes.c_double),
                ("ms_stage", ctypes.c_double * 5), ("tiles", ctypes.c_int32 * 4),
                ("sketch_kernel", ctypes.c_int32), ("residual_terms", ctypes.c_int32),
                ("stage_bytes", ctypes.c_double * 5), ("graph_iterations", ctypes.c_int32),
                ("pad3", ctypes.c_int32)]


_lib = None
EXPORTS = ["icur_run", "icur_run_csr", "icur_run_batched", "icur_last_info", "icur_last_error", "icur_release",
           "icur_make_sketch", "icur_sketch", "icur_lupp", "icur_residual", "icur_gather",
           "icur_core_update", "icur_init_noalloc", "icur_lupp_noalloc", "icur_residual_f64", "icur_qrcp",
           "icur_make_srtt"]


def load(path=LIB_PATH):
    """Load libicur.so (once).  Raises FileNotFoundError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            "libicur.so not found at %s; build it with `python -m paper_2509_21963_amd.build`" % path)
    lib = ctypes.CDLL(path)
    P, I64, I32, D, U64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64
    lib.icur_run.argtypes = [P, I64, I64, I64, D, I32, I32, U64, ctypes.POINTER(Opts), P, P, P,
                             ctypes.POINTER(I64), ctypes.POINTER(D)]
    lib.icur_run_csr.argtypes = [P, P, P, I64, I64, I64, D, I32, I32, U64, ctypes.POINTER(Opts), P, P, P,
                                 ctypes.POINTER(I64), ctypes.POINTER(D)]
    lib.icur_run_batched.argtypes = [I32, P, P, P, P, P, I32, I32, P, ctypes.POINTER(Opts), P, P, P, P, P, P, P]
    lib.icur_last_info.argtypes = [ctypes.POINTER(Info)]
    lib.icur_last_error.restype = ctypes.c_char_p
    lib.icur_make_sketch.argtypes = [U64, I64, I64, I32, I32, P, P, P, P]
    lib.icur_sketch.argtypes = [P, I64, P, I64, I64, I64, I32, P, ctypes.POINTER(D), P]
    lib.icur_lupp.argtypes = [P, I64, I64, I64, I32, P, P, ctypes.POINTER(I32), P]
    lib.icur_residual.argtypes = [P, I64, P, I64, P, I64, I64, I64, I64, I32, P, I64,
                                  ctypes.POINTER(D), P]
    lib.icur_make_srtt.argtypes = [U64, I64, I64, P, P, P]
    lib.icur_qrcp.argtypes = [P, I64, I64, I64, I32, P, P, ctypes.POINTER(I32), P]
    lib.icur_residual_f64.argtypes = [P, I64, P, I64, P, I64, I64, I64, I64, P, I64, ctypes.POINTER(D), P]
    lib.icur_gather.argtypes = [P, I64, I64, I64, P, P, I64, P, I64, P, I64, P]
    lib.icur_core_update.argtypes = [P, I64, I64, I64, P, P, P, ctypes.POINTER(D), P]
    lib.icur_init_noalloc.argtypes = []
    lib.icur_lupp_noalloc.argtypes = [P, I64, I64, I64, I32, P, P, ctypes.POINTER(I32), P]
    for name in EXPORTS:
        if name not in ("icur_last_error",):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status, allow_warnings=False):
    if status < 0 or (status > 0 and not allow_warnings):
        raise IcurError(status, load().icur_last_error().decode())
    return status


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _require(t, dtype, name):
    import torch
    if t.device.type != "cuda":
        raise ValueError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s must be %s" % (name, dtype))
    if t.dim() == 2 and t.stride(1) != 1:
        raise ValueError("%s must be row-major with unit column stride" % name)


def _outputs(rmax, device_outputs, device):
    """I, J and U buffers of a single call: numpy arrays, or device tensors."""
    import torch
    if device_outputs:
        return (torch.empty(max(rmax, 1), dtype=torch.int64, device=device),
                torch.empty(max(rmax, 1), dtype=torch.int64, device=device),
                torch.empty(max(rmax * rmax, 1), dtype=torch.float64, device=device))
    return np.zeros(rmax, np.int64), np.zeros(rmax, np.int64), np.zeros(rmax * rmax, np.float64)


def _addr(x):
    return ctypes.c_void_p(x.data_ptr()) if hasattr(x, "data_ptr") else x.ctypes.data_as(ctypes.c_void_p)


def _single_result(I, J, U, r, rho, st):
    return {"I": I[:r].clone() if hasattr(I, "clone") else I[:r].copy(),
            "J": J[:r].clone() if hasattr(J, "clone") else J[:r].copy(),
            "U": U[:r * r].reshape(r, r).clone() if hasattr(U, "clone") else U[:r * r].reshape(r, r).copy(),
            "rank": r, "rho": rho, "status": _STATUS_NAMES[st], "info": last_info()}


def run(A, tol, block, sketch_kind=GAUSSIAN, seed=0, precision=FP32, zeta=0, max_rank=0,
        alpha=0.0, delta=0.0, split_terms=0, sketch_fp32=False, residual_fp64=0, denominator=DENOM_GA,
        selection=LUPP, device_outputs=False):
    """icur_run on the m x n FP32 device tensor A.  Returns a dict with I, J (int64
    numpy arrays, selection order), U (rank x rank float64 numpy array), rank, rho
    (final estimate), status ("ok", "maxrank" or "stalled") and info (per-call
    statistics).  With device_outputs, I, J and U are device tensors on A's device."""
    import torch
    lib = load()
    _require(A, torch.float32, "A")
    m, n = A.shape
    rmax = min(m, n) if max_rank == 0 else min(int(max_rank), m, n)
    I, J, U = _outputs(rmax, device_outputs, A.device)
    rank = ctypes.c_int64(0)
    rho = ctypes.c_double(0.0)
    o = Opts(precision, zeta, max_rank, _stream(), alpha, delta, split_terms, 1 if sketch_fp32 else 0,
             int(residual_fp64), 0, int(denominator), int(selection), 1 if device_outputs else 0)
    st = lib.icur_run(_ptr(A), m, n, A.stride(0), float(tol), int(block), int(sketch_kind),
                      ctypes.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), ctypes.byref(o),
                      _addr(I), _addr(J), _addr(U), ctypes.byref(rank), ctypes.byref(rho))
    _check(st, allow_warnings=True)
    return _single_result(I, J, U, rank.value, rho.value, st)


def run_csr(rowptr, colind, vals, shape, tol, block, sketch_kind=SPARSE_SIGN, seed=0, precision=FP32,
            zeta=0, max_rank=0, alpha=0.0, delta=0.0, split_terms=0, residual_fp64=0, denominator=DENOM_GA,
            selection=LUPP, device_outputs=False):
    """icur_run_csr on device CSR arrays (rowptr int64, colind int32, vals float32) of an
    m x n matrix.  Returns the same dict as run()."""
    import torch
    lib = load()
    m, n = shape
    if rowptr.dtype != torch.int64 or colind.dtype != torch.int32 or vals.dtype != torch.float32:
        raise ValueError("CSR arrays must be int64 rowptr, int32 colind, float32 vals")
    for t, name in ((rowptr, "rowptr"), (colind, "colind"), (vals, "vals")):
        if t.device.type != "cuda" or not t.is_contiguous():
            raise ValueError("%s must be a contiguous device tensor" % name)
    nnz = colind.numel()
    rmax = min(m, n) if max_rank == 0 else min(int(max_rank), m, n)
    I, J, U = _outputs(rmax, device_outputs, vals.device)
    rank = ctypes.c_int64(0)
    rho = ctypes.c_double(0.0)
    o = Opts(precision, zeta, max_rank, _stream(), alpha, delta, split_terms, 0, int(residual_fp64), 0,
             int(denominator), int(selection), 1 if device_outputs else 0)
    st = lib.icur_run_csr(_ptr(rowptr), _ptr(colind), _ptr(vals), m, n, nnz, float(tol), int(block),
                          int(sketch_kind), ctypes.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), ctypes.byref(o),
                          _addr(I), _addr(J), _addr(U), ctypes.byref(rank), ctypes.byref(rho))
    _check(st, allow_warnings=True)
    return _single_result(I, J, U, rank.value, rho.value, st)


def run_batched(As, tols, block, sketch_kind=GAUSSIAN, seeds=None, precision=FP32, zeta=0, max_rank=0,
                alpha=0.0, delta=0.0, split_terms=0, residual_fp64=0, workers=0, check=True,
                denominator=DENOM_GA, device_outputs=False):
    """icur_run_batched on a list of m_i x n_i FP32 device tensors with per-matrix tolerances
    (and seeds, default 0..count-1).  Returns a list of dicts like run() (without info), each
    with its own "status"; raises on a failed matrix when check is True.  With
    device_outputs the pools (and so I, J, U) are device tensors on the first matrix's
    device."""
    import torch
    lib = load()
    count = len(As)
    if len(tols) != count:
        raise ValueError("need one tolerance per matrix")
    seeds = list(range(count)) if seeds is None else list(seeds)
    if len(seeds) != count:
        raise ValueError("need one seed per matrix")
    for i, A in enumerate(As):
        _require(A, torch.float32, "A[%d]" % i)
    ptrs = (ctypes.c_void_p * max(count, 1))(*[A.data_ptr() for A in As])
    m = np.array([A.shape[0] for A in As], np.int64)
    n = np.array([A.shape[1] for A in As], np.int64)
    lda = np.array([A.stride(0) for A in As], np.int64)
    tol = np.array(tols, np.float64)
    sd = np.array([int(x) & 0xFFFFFFFFFFFFFFFF for x in seeds], np.uint64)
    cap = np.minimum(m, n) if max_rank == 0 else np.minimum(np.minimum(m, n), int(max_rank))
    offs = np.zeros(count + 1, np.int64)
    offs[1:] = np.cumsum(cap)
    uoffs = np.zeros(count + 1, np.int64)
    uoffs[1:] = np.cumsum(cap * cap)
    if device_outputs and count:
        dev = As[0].device
        I = torch.empty(max(int(offs[-1]), 1), dtype=torch.int64, device=dev)
        J = torch.empty(max(int(offs[-1]), 1), dtype=torch.int64, device=dev)
        U = torch.empty(max(int(uoffs[-1]), 1), dtype=torch.float64, device=dev)
    else:
        I = np.empty(max(int(offs[-1]), 1), np.int64)
        J = np.empty(max(int(offs[-1]), 1), np.int64)
        U = np.empty(max(int(uoffs[-1]), 1), np.float64)
    rank = np.zeros(max(count, 1), np.int64)
    est = np.zeros(max(count, 1), np.float64)
    status = np.zeros(max(count, 1), np.int32)
    o = Opts(precision, zeta, max_rank, _stream(), alpha, delta, split_terms, 0, int(residual_fp64), int(workers),
             int(denominator), LUPP, 1 if device_outputs else 0)
    c_ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    st = lib.icur_run_batched(count, ptrs, c_ptr(m), c_ptr(n), c_ptr(lda), c_ptr(tol), int(block), int(sketch_kind),
                              c_ptr(sd), ctypes.byref(o), _addr(I), _addr(J), _addr(U), c_ptr(offs), c_ptr(rank),
                              c_ptr(est), c_ptr(status))
    if check:
        _check(st)
    out = []
    for i in range(count):
        r = int(rank[i])
        # views into the pools (the pools live as long as any view does)
        out.append({"I": I[offs[i]:offs[i] + r], "J": J[offs[i]:offs[i] + r],
                    "U": U[uoffs[i]:uoffs[i] + r * r].reshape(r, r), "rank": r, "rho": float(est[i]),
                    "status": _STATUS_NAMES.get(int(status[i]), str(int(status[i])))})
    return out


def last_info():
    info = Info()
    load().icur_last_info(ctypes.byref(info))
    d = {k: getattr(info, k) for k, _ in Info._fields_ if k not in ("rho", "pad", "pad3", "block_sizes", "ms_stage", "tiles", "stage_bytes")}
    d["ms_stage"] = list(info.ms_stage)
    d["stage_bytes"] = list(info.stage_bytes)
    d["tiles"] = list(info.tiles)
    d["rho"] = list(info.rho[:info.n_rho])
    d["block_sizes"] = list(info.block_sizes[:info.n_rho])
    return d


def release():
    _check(load().icur_release())


def make_sketch(seed, c, m, kind=GAUSSIAN, zeta=0, want_dense=True, want_pattern=False):
    """icur_make_sketch: returns (G_bf16 uint16 c x m or None, rows uint8 m x z or None,
    signs uint8 m or None) as device tensors (int16 holds the BF16 bit patterns)."""
    import torch
    lib = load()
    G = torch.empty((c, m), dtype=torch.int16, device="cuda") if want_dense else None
    z = min(zeta if zeta > 0 else 8, c)
    rows = torch.empty((m, z), dtype=torch.uint8, device="cuda") if want_pattern else None
    signs = torch.empty((m,), dtype=torch.uint8, device="cuda") if want_pattern else None
    _check(lib.icur_make_sketch(ctypes.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), c, m, kind, zeta,
                                _ptr(G), _ptr(rows), _ptr(signs), _stream()))
    return G, rows, signs


def make_srtt(seed, c, m, want_dense=True):
    """icur_make_srtt: returns (G c x m FP32 device tensor or None, rows int64 device tensor)."""
    import torch
    lib = load()
    G = torch.empty((c, m), dtype=torch.float32, device="cuda") if want_dense else None
    rows = torch.empty((c,), dtype=torch.int64, device="cuda")
    _check(lib.icur_make_srtt(ctypes.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), c, m, _ptr(G), _ptr(rows), _stream()))
    return G, rows


def sketch(G, A, terms):
    """icur_sketch: X0 = G A (c x n FP32 device tensor) and ||X0||_F^2."""
    import torch
    lib = load()
    _require(A, torch.float32, "A")
    c, m = G.shape
    n = A.shape[1]
    if A.shape[0] != m:
        raise ValueError("shape mismatch")
    X0 = torch.empty((c, n), dtype=torch.float32, device="cuda")
    nsq = ctypes.c_double(0.0)
    _check(lib.icur_sketch(_ptr(G), c, _ptr(A), m, n, A.stride(0), terms, _ptr(X0),
                           ctypes.byref(nsq), _stream()))
    return X0, nsq.value


def lupp(X, steps, excluded=None):
    """icur_lupp on the K x N FP32 device tensor X (candidates along N): returns the
    pivot order as an int64 numpy array."""
    import torch
    lib = load()
    _require(X, torch.float32, "X")
    K, N = X.shape
    piv = torch.zeros((steps,), dtype=torch.int64, device="cuda")
    npiv = ctypes.c_int32(0)
    if excluded is not None and (excluded.dtype != torch.uint8 or excluded.numel() != N):
        raise ValueError("excluded must be a uint8 device tensor of length N")
    _check(lib.icur_lupp(_ptr(X), K, N, X.stride(0), steps, _ptr(excluded), _ptr(piv),
                         ctypes.byref(npiv), _stream()))
    return piv[:npiv.value].cpu().numpy()


def qrcp(X, steps, excluded=None):
    """icur_qrcp on the K x N FP32 device tensor X (candidates along N): returns the pivot
    order as an int64 numpy array."""
    import torch
    lib = load()
    _require(X, torch.float32, "X")
    K, N = X.shape
    piv = torch.zeros((steps,), dtype=torch.int64, device="cuda")
    npiv = ctypes.c_int32(0)
    if excluded is not None and (excluded.dtype != torch.uint8 or excluded.numel() != N):
        raise ValueError("excluded must be a uint8 device tensor of length N")
    _check(lib.icur_qrcp(_ptr(X), K, N, X.stride(0), steps, _ptr(excluded), _ptr(piv), ctypes.byref(npiv),
                         _stream()))
    return piv[:npiv.value].cpu().numpy()


def lupp_noalloc(X, steps, piv, excluded=None):
    """icur_lupp_noalloc on the K x N FP32 device tensor X into the caller's int64 device
    tensor piv (capacity >= steps): the library allocates nothing.  Returns the pivot
    count."""
    import torch
    lib = load()
    _require(X, torch.float32, "X")
    K, N = X.shape
    if piv.dtype != torch.int64 or piv.device.type != "cuda" or piv.numel() < steps:
        raise ValueError("piv must be an int64 device tensor with at least `steps` entries")
    if excluded is not None and (excluded.dtype != torch.uint8 or excluded.numel() != N):
        raise ValueError("excluded must be a uint8 device tensor of length N")
    npiv = ctypes.c_int32(0)
    _check(lib.icur_lupp_noalloc(_ptr(X), K, N, X.stride(0), steps, _ptr(excluded), _ptr(piv),
                                 ctypes.byref(npiv), _stream()))
    return npiv.value


def init_noalloc():
    """icur_init_noalloc: look up the fixed scratch area on the current device."""
    _check(load().icur_init_noalloc())


def residual(X, W, B, terms):
    """icur_residual: OUT = X - W B with W FP64 (M x K), B FP32 (K x N), X FP32 (M x N)
    or None.  Returns (OUT, ||OUT||_F^2)."""
    import torch
    lib = load()
    M, K = W.shape
    N = B.shape[1]
    OUT = torch.empty((M, N), dtype=torch.float32, device="cuda")
    nsq = ctypes.c_double(0.0)
    _check(lib.icur_residual(_ptr(X), X.stride(0) if X is not None else N, _ptr(W),
                             W.stride(0) if K > 0 else 1, _ptr(B), B.stride(0), M, K, N, terms,
                             _ptr(OUT), N, ctypes.byref(nsq), _stream()))
    return OUT, nsq.value


def residual_f64(X, W, B, out=None):
    """icur_residual_f64: OUT = X - W B (FP64 device tensors; X may be `out` for in place,
    or None for OUT = W B).  Returns (OUT, ||OUT||_F^2)."""
    import torch
    lib = load()
    M, K = W.shape
    N = B.shape[1]
    OUT = out if out is not None else torch.empty((M, N), dtype=torch.float64, device="cuda")
    nsq = ctypes.c_double(0.0)
    _check(lib.icur_residual_f64(_ptr(X), X.stride(0) if X is not None else N, _ptr(W),
                                 W.stride(0) if K > 0 else 1, _ptr(B), B.stride(0) if K > 0 else N,
                                 M, K, N, _ptr(OUT), OUT.stride(0), ctypes.byref(nsq), _stream()))
    return OUT, nsq.value


def gather_cols_T(A, cols):
    import torch
    lib = load()
    m, n = A.shape
    k = cols.numel()
    Ct = torch.empty((k, m), dtype=torch.float32, device="cuda")
    _check(lib.icur_gather(_ptr(A), m, n, A.stride(0), _ptr(cols), None, k, _ptr(Ct), m, None, 0,
                           _stream()))
    return Ct


def gather_rows(A, rows):
    import torch
    lib = load()
    m, n = A.shape
    k = rows.numel()
    R = torch.empty((k, n), dtype=torch.float32, device="cuda")
    _check(lib.icur_gather(_ptr(A), m, n, A.stride(0), None, _ptr(rows), k, None, 0, _ptr(R), n,
                           _stream()))
    return R


def core_update(U, r, k, Y, A21, A22):
    """icur_core_update in place on the FP64 device tensor U ((r+k) x (r+k) or larger,
    row-major).  Returns rcond of the new diagonal block."""
    lib = load()
    rc = ctypes.c_double(0.0)
    _check(lib.icur_core_update(_ptr(U), U.stride(0), r, k, _ptr(Y), _ptr(A21), _ptr(A22),
                                ctypes.byref(rc), _stream()))
    return rc.value
