"""Host-only checks of the C ABI library: it loads, exports what the header
declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ftm.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(ftm_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def L():
    from paper_2508_10202_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libftm.so is not built: run __graft_entry__.build()")
    return _lib.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("ftm_setup_operator", "ftm_matvec", "ftm_rmatvec", "ftm_destroy_operator"):
        assert want in names


def test_library_exports_every_declared_symbol(L):
    from paper_2508_10202_amd import _lib
    names = _declared()
    assert set(names) == set(_lib.EXPORTS)
    for n in names:
        assert hasattr(L, n), n


def test_status_strings(L):
    assert L.ftm_status_string(0) == b"ok"
    assert L.ftm_status_string(1) == b"invalid argument"
    assert L.ftm_status_string(99) == b"unknown status"


def _setup(L, out, F, Nt, Nd, Nm, fwd=None, adj=None, spectra=0, max_rhs=1):
    return L.ftm_setup_operator(out, F, Nt, Nd, Nm, fwd, adj, spectra, max_rhs, None)


def test_setup_rejects_bad_arguments_without_a_gpu(L):
    from paper_2508_10202_amd._lib import ERR_INVALID, ERR_UNSUPPORTED, FtmPrecision
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: every case fails validation first
    assert _setup(L, None, fake, 4, 2, 3) == ERR_INVALID
    assert _setup(L, ctypes.byref(h), None, 4, 2, 3) == ERR_INVALID
    assert _setup(L, ctypes.byref(h), fake, 0, 2, 3) == ERR_INVALID
    assert _setup(L, ctypes.byref(h), fake, 4, 0, 3) == ERR_INVALID
    assert _setup(L, ctypes.byref(h), fake, 4, 2, 3, max_rhs=0) == ERR_INVALID
    assert b"max_rhs" in L.ftm_last_error()
    # no transform length of at most 4096 covers Nt above 2048
    assert _setup(L, ctypes.byref(h), fake, 2049, 2, 3) == ERR_UNSUPPORTED
    assert _setup(L, ctypes.byref(h), fake, 4096, 2, 3) == ERR_UNSUPPORTED
    assert _setup(L, ctypes.byref(h), fake, 4, 2, 3, spectra=1 << 5) == ERR_INVALID
    bad = FtmPrecision(0, 0, 0, 0, 0, 1)      # FP64 product with FP32 accumulation
    assert _setup(L, ctypes.byref(h), fake, 4, 2, 3, fwd=ctypes.byref(bad)) == ERR_INVALID
    bad = FtmPrecision(0, 0, 2, 0, 0, 0)      # FP16 product with FP64 accumulation
    assert _setup(L, ctypes.byref(h), fake, 4, 2, 3, adj=ctypes.byref(bad)) == ERR_INVALID
    bad = FtmPrecision(0, 7, 0, 0, 0, 0)
    assert _setup(L, ctypes.byref(h), fake, 4, 2, 3, fwd=ctypes.byref(bad)) == ERR_INVALID
    assert h.value is None


def test_calls_on_null_operator(L):
    from paper_2508_10202_amd._lib import ERR_INVALID, OK
    fake = ctypes.c_void_p(0x1000)
    assert L.ftm_matvec(None, fake, fake, 1, None) == ERR_INVALID
    assert L.ftm_rmatvec(None, fake, fake, 1, None) == ERR_INVALID
    assert L.ftm_set_precision(None, None, None) == ERR_INVALID
    assert L.ftm_get_spectrum(None, 0, 0, 1, fake, None) == ERR_INVALID
    assert L.ftm_operator_info(None, None, None, None, None, None) == ERR_INVALID
    assert L.ftm_destroy_operator(None) == OK


def test_precision_strings():
    from paper_2508_10202_amd import BF16, F16, F32, F64, Precision
    p = Precision.parse("dssdd")
    assert (p.pad, p.fft, p.gemv, p.ifft, p.unpad, p.accum) == (F64, F32, F32, F64, F64, F32)
    assert str(p) == "dssdd"
    q = Precision.parse("dhbsd+a32")
    assert (q.fft, q.gemv, q.ifft, q.accum) == (F16, BF16, F32, F32)
    assert str(Precision.parse("ddsdd+a64")) == "ddsdd+a64"
    assert Precision.parse("ddddd") == Precision()
    for bad in ("dddd", "dxddd", "ddddd+a16"):
        with pytest.raises(ValueError):
            Precision.parse(bad)


def test_server_rejects_bad_arguments_without_a_gpu(L):
    from paper_2508_10202_amd._lib import ERR_INVALID
    h = ctypes.c_void_p()
    assert L.ftm_server_create(None, 1 << 20, 2, 8) == ERR_INVALID
    assert L.ftm_server_create(ctypes.byref(h), 100, 2, 8) == ERR_INVALID     # budget < 4 KiB
    assert L.ftm_server_create(ctypes.byref(h), 1 << 20, 0, 8) == ERR_INVALID
    assert L.ftm_server_create(ctypes.byref(h), 1 << 20, 17, 8) == ERR_INVALID
    assert L.ftm_server_create(ctypes.byref(h), 1 << 20, 2, 0) == ERR_INVALID
    t = ctypes.c_uint64()
    fake = ctypes.c_void_p(0x1000)
    assert L.ftm_server_submit(None, fake, 0, fake, fake, 1, None, ctypes.byref(t)) == ERR_INVALID
    done = ctypes.c_int32()
    assert L.ftm_server_poll(None, 1, ctypes.byref(done), None) == ERR_INVALID
    assert L.ftm_server_destroy(None) == 0


def test_sbgemv_rejects_bad_arguments_without_a_gpu(L):
    from paper_2508_10202_amd._lib import ERR_INVALID, OK
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every case fails validation (or does nothing)
    one = ctypes.c_double(1.0)
    a = ctypes.cast(ctypes.pointer(one), ctypes.c_void_p)

    def call(type_=1, op=1, m=4, n=8, lda=4, sa=32, sx=4, sy=8, batch=2, alpha=a, A=fake, x=fake, y=fake):
        return L.ftm_sbgemv(type_, op, m, n, alpha, A, lda, sa, x, sx, a, y, sy, batch, None)

    assert call(type_=4) == ERR_INVALID
    assert call(op=3) == ERR_INVALID
    assert call(m=-1) == ERR_INVALID
    assert call(A=None) == ERR_INVALID
    assert call(alpha=None) == ERR_INVALID
    assert call(lda=3) == ERR_INVALID                       # lda < m
    assert call(sa=31) == ERR_INVALID                       # matrices overlap
    assert call(sx=3) == ERR_INVALID                        # op T reads m = 4 entries of x
    assert call(op=0, sx=4, sy=4) == ERR_INVALID            # op N reads n = 8 entries of x
    assert call(sy=7) == ERR_INVALID
    assert call(m=1 << 31, lda=1 << 31) == ERR_INVALID
    assert call(m=0) == OK and call(n=0) == OK and call(batch=0) == OK
    assert call(batch=1, sa=0, sx=0, sy=0, A=None) == ERR_INVALID


def test_binding_constants_match_the_header():
    from paper_2508_10202_amd import _lib
    text = open(HEADER).read()

    def enum(name):
        return int(re.search(r"\b%s\s*=\s*(\d+)" % name, text).group(1))
    assert (enum("FTM_TYPE_S"), enum("FTM_TYPE_D"), enum("FTM_TYPE_C"), enum("FTM_TYPE_Z")) == \
        (_lib.TYPE_S, _lib.TYPE_D, _lib.TYPE_C, _lib.TYPE_Z)
    assert (enum("FTM_OP_N"), enum("FTM_OP_T"), enum("FTM_OP_C")) == (_lib.OP_N, _lib.OP_T, _lib.OP_C)
    assert (enum("FTM_F64"), enum("FTM_F32"), enum("FTM_F16"), enum("FTM_BF16")) == \
        (_lib.F64, _lib.F32, _lib.F16, _lib.BF16)
    assert (enum("FTM_RHS_AUTO"), enum("FTM_RHS_GEMV"), enum("FTM_RHS_GEMM")) == \
        (_lib.RHS_AUTO, _lib.RHS_GEMV, _lib.RHS_GEMM)
    m = re.search(r"#define FTM_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == _lib.SCRATCH_BYTES
