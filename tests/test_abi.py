"""Host-side checks of the C-ABI library (no GPU needed).

* librsvd.so loads and exports every function declared in include/rsvd.h;
* argument validation returns the documented negative codes before any
  device work (a dummy non-null handle is enough for invalid arguments);
* the workspace query is a pure function that grows with the problem.
"""

import ctypes
import os
import re

import pytest

from paper_1502_05366_amd import _lib

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = os.path.join(os.path.dirname(HERE), "include", "rsvd.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(rsvd_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    # and the binding declares exactly those
    assert sorted(_lib.SIGNATURES) == names


FAKE = ctypes.c_void_p(0x1000)   # never dereferenced on the invalid-argument paths
NULLP = None
PTR = ctypes.c_void_p(0x2000)


def svd_call(lib, **kw):
    a = dict(h=FAKE, dtype=0, m=100, n=80, k=10, p=5, q=1, seed=1, A=PTR, lda=80, U=PTR, ldu=10,
             S=PTR, V=PTR, ldv=10, work=PTR, wb=1 << 40, info=PTR, stream=NULLP)
    a.update(kw)
    return lib.rsvd_svd(a['h'], a['dtype'], a['m'], a['n'], a['k'], a['p'], a['q'], a['seed'],
                        a['A'], a['lda'], a['U'], a['ldu'], a['S'], a['V'], a['ldv'], a['work'],
                        a['wb'], a['info'], a['stream'])


@pytest.mark.parametrize("kw,code", [
    (dict(h=NULLP), -1), (dict(dtype=7), -2), (dict(dtype=2, lda=81), -10), (dict(m=0), -3), (dict(n=-1), -4),
    (dict(k=0), -5), (dict(k=81), -5), (dict(p=-1), -6), (dict(q=-2), -7),
    (dict(A=NULLP), -9), (dict(lda=79), -10), (dict(U=NULLP), -11), (dict(ldu=9), -12),
    (dict(S=NULLP), -13), (dict(V=NULLP), -14), (dict(ldv=3), -15), (dict(work=NULLP), -16),
    (dict(info=NULLP), -18), (dict(wb=16), 2), (dict(k=580, p=10, m=1000, n=800, lda=800, ldu=580,
                                                     ldv=580), 3),
])
def test_svd_argument_codes(lib, kw, code):
    assert svd_call(lib, **kw) == code


def test_id_cur_argument_codes(lib):
    assert lib.rsvd_id(FAKE, 0, 50, 40, 5, 5, 1, 1, PTR, 40, NULLP, PTR, 35, PTR, 1 << 40, PTR,
                       NULLP) == -11
    assert lib.rsvd_id(FAKE, 0, 50, 40, 5, 5, 1, 1, PTR, 40, PTR, PTR, 34, PTR, 1 << 40, PTR,
                       NULLP) == -13
    assert lib.rsvd_cur(FAKE, 1, 50, 40, 5, 5, 1, 1, PTR, 40, PTR, PTR, PTR, 4, PTR, 1 << 40,
                        PTR, NULLP) == -14
    assert lib.rsvd_cur(FAKE, 1, 50, 40, 5, 5, 1, 1, PTR, 40, PTR, PTR, PTR, 5, PTR, 8,
                        PTR, NULLP) == 2


def test_mixed_precision_argument_codes(lib):
    # rsvd_svd_ex: FP8 needs its column scales (and only FP8 takes them), an
    # FP8 A needs lda % 16 == 0; the basis output needs ldqb >= l
    def ex(dtype=3, lda=96, scale=PTR, Qb=NULLP, ldqb=0, m=100, n=80, k=10, p=5):
        return lib.rsvd_svd_ex(FAKE, dtype, m, n, k, p, 1, 1, PTR, lda, scale, PTR, k, PTR, PTR, k,
                               Qb, ldqb, PTR, 1 << 40, PTR, NULLP)
    assert ex(scale=NULLP) == -11
    assert ex(dtype=0, lda=80) == -11
    assert ex(lda=88) == -10
    assert ex(Qb=PTR, ldqb=14) == -18
    assert ex(k=580, p=10, m=1000, n=800, lda=800) == 3
    # F8E4M3 is refused by the entry points that take no scales
    assert svd_call(lib, dtype=3) == 3
    assert lib.rsvd_workspace_bytes(1, 3, 100, 80, 10, 5, 1) > 0
    assert lib.rsvd_workspace_bytes(2, 3, 100, 80, 10, 5, 1) == 0
    # rsvd_quantize: BF16 or E4M3 from FP64; E4M3 needs the scale output
    assert lib.rsvd_quantize(FAKE, 0, 10, 10, PTR, 10, PTR, 10, PTR, NULLP) == -2
    assert lib.rsvd_quantize(FAKE, 3, 10, 10, PTR, 10, PTR, 10, NULLP, NULLP) == -9
    assert lib.rsvd_quantize(FAKE, 2, 10, 10, PTR, 9, PTR, 10, NULLP, NULLP) == -6
    # rsvd_pass_f8: lda a multiple of 16, scales required, l <= 576
    assert lib.rsvd_pass_f8(FAKE, 0, 100, 80, 10, PTR, 88, PTR, PTR, 10, PTR, 10, 0, PTR, 1 << 40,
                            NULLP) == -7
    assert lib.rsvd_pass_f8(FAKE, 0, 100, 80, 10, PTR, 96, NULLP, PTR, 10, PTR, 10, 0, PTR,
                            1 << 40, NULLP) == -8
    assert lib.rsvd_pass_f8(FAKE, 0, 1000, 800, 600, PTR, 800, PTR, PTR, 600, PTR, 600, 0, PTR,
                            1 << 40, NULLP) == 3
    assert lib.rsvd_pass_f8_workspace_bytes(1, 100, 80, 10) > 0


def test_status_strings(lib):
    assert lib.rsvd_status_string(0) == b"ok"
    assert lib.rsvd_status_string(-3) == b"invalid argument"
    assert lib.rsvd_status_string(2) == b"workspace too small"


def test_workspace_query(lib):
    w = lib.rsvd_workspace_bytes
    assert w(1, 0, 100, 80, 10, 5, 1) > 0
    assert w(0, 0, 100, 80, 10, 5, 1) == 0           # no op selected
    assert w(1, 0, 100, 80, 90, 5, 1) == 0           # k > min(m, n)
    small = w(1, 0, 2000, 1000, 20, 10, 1)
    big = w(1, 0, 20000, 10000, 200, 20, 2)
    assert big > small
    # the FP64 C2 sizes fit comfortably in one GPU's HBM
    assert w(7, 0, 20000, 10000, 200, 20, 2) < 4 << 30
    assert w(7, 1, 20000, 10000, 200, 20, 2) < w(7, 0, 20000, 10000, 200, 20, 2)
    assert w(4, 0, 300, 200, 10, 5, 1) == w(6, 0, 300, 200, 10, 5, 1)


def test_step_workspace_queries(lib):
    assert lib.rsvd_orth_workspace_bytes(0, 1000, 30) > 0
    assert lib.rsvd_orth_workspace_bytes(0, 10, 30) == 0
    assert lib.rsvd_orth_workspace_bytes(0, 1000, 300) > 0       # column blocks above 256
    assert lib.rsvd_orth_workspace_bytes(0, 1000, 600) == 0      # above 576
    assert lib.rsvd_small_svd_workspace_bytes(220) >= 2 * 220 * 220 * 8
    assert lib.rsvd_small_svd_workspace_bytes(576) >= 2 * 576 * 576 * 8
    assert lib.rsvd_small_svd_workspace_bytes(577) == 0
    assert lib.rsvd_cpqr_workspace_bytes(220, 10000, 200) > 0
    assert lib.rsvd_cpqr_workspace_bytes(220, 10000, 300) == 0
    assert lib.rsvd_pass_workspace_bytes(0, 0, 20000, 10000, 220) > 0


def grad_call(lib, **kw):
    a = dict(h=FAKE, dtype=0, m=100, n=80, k=10, p=5, q=1, seed=1, A=PTR, lda=80, dU=PTR, lddu=10,
             dS=PTR, dV=PTR, lddv=10, dres=PTR, dA=PTR, ldda=80, U=NULLP, ldu=10, S=NULLP,
             V=NULLP, ldv=10, r2=NULLP, work=PTR, wb=1 << 40, info=PTR, stream=NULLP)
    a.update(kw)
    return lib.rsvd_svd_grad(a['h'], a['dtype'], a['m'], a['n'], a['k'], a['p'], a['q'],
                             a['seed'], a['A'], a['lda'], a['dU'], a['lddu'], a['dS'], a['dV'],
                             a['lddv'], a['dres'], a['dA'], a['ldda'], a['U'], a['ldu'], a['S'],
                             a['V'], a['ldv'], a['r2'], a['work'], a['wb'], a['info'],
                             a['stream'])


@pytest.mark.parametrize("kw,code", [
    (dict(h=NULLP), -1), (dict(dtype=7), -2), (dict(dtype=1), 3), (dict(dtype=2), 3),
    (dict(m=0), -3), (dict(n=0), -4), (dict(k=81), -5), (dict(p=-1), -6), (dict(q=-1), -7),
    (dict(q=9), 3), (dict(A=NULLP), -9), (dict(lda=79), -10), (dict(lddu=9), -12),
    (dict(lddv=9), -15), (dict(ldda=79), -18), (dict(U=PTR, ldu=9), -20),
    (dict(V=PTR, ldv=9), -23), (dict(dA=NULLP), -17), (dict(work=NULLP), -25),
    (dict(info=NULLP), -27), (dict(wb=16), 2),
    (dict(k=250, p=10, m=400, n=300, lda=300, ldda=300, lddu=250, lddv=250), 3),
])
def test_svd_grad_argument_codes(lib, kw, code):
    assert grad_call(lib, **kw) == code


def test_svd_grad_workspace_query(lib):
    w = lib.rsvd_svd_grad_workspace_bytes
    assert w(0, 300, 200, 10, 6, 2) > w(0, 300, 200, 10, 6, 1) > 0
    assert w(1, 300, 200, 10, 6, 1) == 0        # FP64 only
    assert w(0, 300, 200, 10, 6, 9) == 0        # q <= 8
    # the FP64 8192 x 4096, k = 64, p = 16, q = 2 case
    assert w(0, 8192, 4096, 64, 16, 2) < 256 << 20


def test_batch_create_argument_codes(lib):
    import numpy as np
    m = np.array([100, 50], dtype=np.int64)
    n = np.array([80, 40], dtype=np.int64)
    k = np.array([10, 5], dtype=np.int32)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    plan = ctypes.c_void_p()
    cr = lib.rsvd_batch_create
    assert cr(NULLP, 2, P(m), P(n), P(k), 8, 1, ctypes.byref(plan)) == -1
    assert cr(FAKE, 0, P(m), P(n), P(k), 8, 1, ctypes.byref(plan)) == -2
    assert cr(FAKE, 2, NULLP, P(n), P(k), 8, 1, ctypes.byref(plan)) == -3
    assert cr(FAKE, 2, P(m), NULLP, P(k), 8, 1, ctypes.byref(plan)) == -4
    assert cr(FAKE, 2, P(m), P(n), NULLP, 8, 1, ctypes.byref(plan)) == -5
    assert cr(FAKE, 2, P(m), P(n), P(k), -1, 1, ctypes.byref(plan)) == -6
    assert cr(FAKE, 2, P(m), P(n), P(k), 8, -1, ctypes.byref(plan)) == -7
    assert cr(FAKE, 2, P(m), P(n), P(k), 8, 1, NULLP) == -8
    bad_k = np.array([10, 41], dtype=np.int32)            # k > min(m, n)
    assert cr(FAKE, 2, P(m), P(n), P(bad_k), 8, 1, ctypes.byref(plan)) == -5
    bad_m = np.array([100, 0], dtype=np.int64)
    assert cr(FAKE, 2, P(bad_m), P(n), P(k), 8, 1, ctypes.byref(plan)) == -3
    m2 = np.array([200, 50], dtype=np.int64)
    n2 = np.array([100, 40], dtype=np.int64)
    huge = np.array([74, 5], dtype=np.int32)              # l = 82 -> lp 96: unsupported
    assert cr(FAKE, 2, P(m2), P(n2), P(huge), 8, 1, ctypes.byref(plan)) == 3
    assert lib.rsvd_batch_workspace_bytes(NULLP) == 0
    assert lib.rsvd_batch_svd(NULLP, 1, PTR, PTR, PTR, PTR, PTR, 1, PTR, NULLP) == -1
    assert lib.rsvd_batch_prepare(NULLP, PTR, 1, NULLP) == -1
    assert lib.rsvd_batch_set_variants(NULLP, PTR) == -1
