"""The C-ABI library loads and exports every symbol include/icur.h declares; argument
errors are reported before any device work (CPU only: no compute call reaches a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "icur.h")


def _lib():
    from paper_2509_21963_amd import icur
    if not os.path.exists(icur.LIB_PATH):
        from paper_2509_21963_amd import build
        build.build()
    return icur, icur.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(icur_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for want in ("icur_run", "icur_run_csr", "icur_run_batched", "icur_lupp", "icur_sketch", "icur_residual", "icur_gather",
                 "icur_core_update", "icur_make_sketch", "icur_release", "icur_last_error",
                 "icur_last_info"):
        assert want in names


def test_library_exports_every_declared_symbol():
    icur, lib = _lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(icur.EXPORTS) == set(declared_functions())


def _c_layout(struct, fields):
    """sizeof and field offsets of a header struct, from a C program built with gcc."""
    import subprocess
    import tempfile
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "icur.h"', 'int main(void) {',
             '  printf("%%zu\\n", sizeof(%s));' % struct]
    lines += ['  printf("%%zu\\n", offsetof(%s, %s));' % (struct, f) for f in fields]
    lines += ['  return 0;', '}']
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
        open(src, "w").write("\n".join(lines) + "\n")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(x) for x in out[1:]]


@pytest.mark.parametrize("struct,cls", [("icur_opts", "Opts"), ("icur_info", "Info")])
def test_struct_layouts_match_header(struct, cls):
    # the binding's ctypes mirrors are laid out as the C compiler lays out the header's
    icur, _ = _lib()
    C = getattr(icur, cls)
    names = [f[0] for f in C._fields_]
    size, offs = _c_layout(struct, names)
    assert ctypes.sizeof(C) == size
    assert [getattr(C, f).offset for f in names] == offs


FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: validation precedes device work


def _run_args(lib, m=10, n=8, lda=8, tol=1e-3, block=2, kind=0, opts=None):
    I = np.zeros(64, np.int64)
    J = np.zeros(64, np.int64)
    U = np.zeros(64 * 64)
    rank = ctypes.c_int64(-1)
    rho = ctypes.c_double(-1.0)
    st = lib.icur_run(FAKE, m, n, lda, tol, block, kind, ctypes.c_uint64(0), opts,
                      I.ctypes.data_as(ctypes.c_void_p), J.ctypes.data_as(ctypes.c_void_p),
                      U.ctypes.data_as(ctypes.c_void_p), ctypes.byref(rank), ctypes.byref(rho))
    return st, rank.value


@pytest.mark.parametrize("kw", [
    dict(m=0), dict(n=0), dict(lda=7), dict(tol=0.0), dict(tol=float("nan")),
    dict(tol=float("inf")), dict(block=0), dict(block=9), dict(kind=3),
])
def test_run_rejects_bad_arguments_before_device_work(kw):
    icur, lib = _lib()
    st, rank = _run_args(lib, **kw)
    assert st == icur.ERR_ARG
    assert rank == -1                      # nothing written
    assert lib.icur_last_error()


def test_run_rejects_bad_options():
    icur, lib = _lib()
    for o in (icur.Opts(precision=5), icur.Opts(zeta=9), icur.Opts(split_terms=4),
              icur.Opts(max_rank=-1), icur.Opts(alpha=1e-10),     # c = 2 < -4 ln(alpha)
              icur.Opts(residual_fp64=2), icur.Opts(zeta=-1), icur.Opts(batch_workers=17),
              icur.Opts(batch_workers=-1), icur.Opts(denominator=2), icur.Opts(denominator=-1),
              icur.Opts(selection=2), icur.Opts(selection=-1), icur.Opts(device_outputs=2)):
        st, _ = _run_args(lib, opts=ctypes.byref(o))
        assert st == icur.ERR_ARG, (o.precision, o.zeta)
    # the SRTT operator needs c <= m
    st, _ = _run_args(lib, m=19, n=30, lda=30, block=19, kind=2)   # c = 20 > m
    assert st == icur.ERR_ARG
    # risk-aware stopping is for the Gaussian sketch (the section 3.3 Corollary)
    o = icur.Opts(alpha=0.2)
    st, _ = _run_args(lib, m=100, n=100, lda=100, block=20, kind=1, opts=ctypes.byref(o))
    assert st == icur.ERR_ARG
    # sparse-sign needs c <= 255
    st, _ = _run_args(lib, m=300, n=300, lda=300, block=240, kind=1)
    assert st == icur.ERR_ARG
    # pivot blocks are inverted by one workgroup: b <= 512, rejected before device work
    st, rank = _run_args(lib, m=1000, n=1000, lda=1000, block=513)
    assert st == icur.ERR_ARG and rank == -1


def test_step_entry_points_reject_bad_shapes():
    icur, lib = _lib()
    n = ctypes.c_int32(0)
    assert lib.icur_lupp(FAKE, 4, 10, 9, 2, None, FAKE, ctypes.byref(n), None) == icur.ERR_ARG
    assert lib.icur_lupp(FAKE, 4, 10, 10, 5, None, FAKE, ctypes.byref(n), None) == icur.ERR_ARG
    assert lib.icur_sketch(FAKE, 0, FAKE, 5, 5, 5, 0, FAKE, None, None) == icur.ERR_ARG
    assert lib.icur_sketch(FAKE, 3, FAKE, 5, 5, 5, 4, FAKE, None, None) == icur.ERR_ARG
    assert lib.icur_residual(None, 4, FAKE, 3, FAKE, 4, 2, 3, 4, 0, FAKE, 3, None, None) == icur.ERR_ARG
    assert lib.icur_gather(FAKE, 4, 4, 4, FAKE, FAKE, 2, FAKE, 4, FAKE, 4, None) == icur.ERR_ARG
    assert lib.icur_core_update(FAKE, 3, 2, 2, FAKE, FAKE, FAKE, None, None) == icur.ERR_ARG
    assert lib.icur_make_sketch(ctypes.c_uint64(0), 3, 5, 7, 0, FAKE, None, None, None) == icur.ERR_ARG


def test_run_csr_rejects_bad_arguments_before_device_work():
    icur, lib = _lib()
    I = np.zeros(8, np.int64)
    J = np.zeros(8, np.int64)
    U = np.zeros(64)
    rank = ctypes.c_int64(-1)
    rho = ctypes.c_double(0.0)

    def call(rowptr=FAKE, colind=FAKE, vals=FAKE, m=10, n=8, nnz=20, tol=1e-3, block=4, kind=1):
        return lib.icur_run_csr(rowptr, colind, vals, m, n, nnz, tol, block, kind, ctypes.c_uint64(0), None,
                                I.ctypes.data_as(ctypes.c_void_p), J.ctypes.data_as(ctypes.c_void_p),
                                U.ctypes.data_as(ctypes.c_void_p), ctypes.byref(rank), ctypes.byref(rho))
    for kw in (dict(rowptr=None), dict(colind=None), dict(vals=None), dict(nnz=-1), dict(nnz=2 ** 31),
               dict(m=0), dict(n=0), dict(tol=0.0), dict(block=0), dict(block=9), dict(kind=3)):
        assert call(**kw) == icur.ERR_ARG, kw
        assert rank.value == -1


def test_run_batched_rejects_bad_arguments_before_device_work():
    icur, lib = _lib()
    count = 3

    def arr(values, dt):
        a = np.array(values, dt)
        return a, a.ctypes.data_as(ctypes.c_void_p)

    def call(ms=(10, 12, 9), ns=(8, 8, 7), ldas=(8, 8, 7), tols=(1e-3, 1e-3, 1e-3), caps=(8, 8, 7), block=2,
             cnt=count, first_off=0, ptrs=True):
        keep = []
        P = (ctypes.c_void_p * count)(*([0x1000] * count))
        m_, pm = arr(ms, np.int64)
        n_, pn = arr(ns, np.int64)
        l_, pl = arr(ldas, np.int64)
        t_, pt = arr(tols, np.float64)
        s_, ps = arr([0] * count, np.uint64)
        offs = np.zeros(count + 1, np.int64)
        offs[1:] = np.cumsum(caps)
        offs[0] = first_off
        I = np.zeros(64, np.int64)
        J = np.zeros(64, np.int64)
        U = np.zeros(4096)
        rank = np.full(count, -1, np.int64)
        est = np.zeros(count)
        status = np.full(count, 99, np.int32)
        keep += [m_, n_, l_, t_, s_]
        c = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        st = lib.icur_run_batched(cnt, P if ptrs else None, pm, pn, pl, pt, block, 0, ps, None, c(I), c(J), c(U),
                                  c(offs), c(rank), c(est), c(status))
        return st, rank, status

    for kw in (dict(cnt=-1), dict(ptrs=False), dict(ms=(10, 0, 9)), dict(ldas=(8, 7, 7)),
               dict(tols=(1e-3, float("nan"), 1e-3)), dict(caps=(8, 7, 7)), dict(block=8), dict(first_off=1)):
        st, rank, status = call(**kw)
        assert st == icur.ERR_ARG, kw
        assert (rank == -1).all() and (status == 99).all(), kw   # nothing ran, nothing written
    st, _, _ = call(ms=(10, 0, 9))
    assert b"matrix 1" in lib.icur_last_error()
    # count 0 is a no-op
    assert call(cnt=0)[0] == icur.OK
