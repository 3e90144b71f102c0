"""The C ABI without a GPU: the library loads, exports every symbol the header
declares, and rejects bad arguments on the host before launching anything."""

import ctypes
import os
import re

import pytest

from paper_2409_19402_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "projprod.h")

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH),
                                reason="libprojprod.so not built")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pq_[a-z0-9_]+)\s*\(", text)))


def test_header_symbols_exported():
    lib = _lib.load()
    names = declared_symbols()
    assert len(names) >= 17
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.SIGNATURES), "binding signatures must cover the header"


def test_status_strings():
    lib = _lib.load()
    assert lib.pq_version() >= 100
    for code in range(0, -12, -1):
        assert lib.pq_status_string(code)
    assert b"unknown" in lib.pq_status_string(-99)


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


def rc(name, *args):
    return getattr(_lib.load(), name)(*args)


def test_validation_errors():
    # null pointers
    assert rc("pq_hat", None, 0, FAKE, FAKE, 4, 4, 8, 2, 0, None) == -1
    # p > n3 and p < 1
    assert rc("pq_hat", FAKE, 0, FAKE, ctypes.c_void_p(0x2000), 4, 4, 8, 9, 0, None) == -3
    assert rc("pq_hat", FAKE, 0, FAKE, ctypes.c_void_p(0x2000), 4, 4, 8, 0, 0, None) == -3
    # non-positive size
    assert rc("pq_hat", FAKE, 0, FAKE, ctypes.c_void_p(0x2000), 0, 4, 8, 2, 0, None) == -2
    # dtype
    assert rc("pq_hat", FAKE, 7, FAKE, ctypes.c_void_p(0x2000), 4, 4, 8, 2, 0, None) == -5
    assert rc("pq_unhat", FAKE, FAKE, ctypes.c_void_p(0x2000), 2, 4, 4, 8, 2, 0, None) == -5
    # precision mode on float64 data
    assert rc("pq_hat", FAKE, 1, FAKE, ctypes.c_void_p(0x2000), 4, 4, 8, 2, 2, None) == -6
    # alias: output == input
    assert rc("pq_hat", FAKE, 0, ctypes.c_void_p(0x3000), FAKE, 4, 4, 8, 2, 0, None) == -7
    # k out of range
    for k in (0, 5):
        assert rc("pq_tsvdq", FAKE, 0, ctypes.c_void_p(0x2000), 4, 6, 8, 2, k, 0,
                  ctypes.c_void_p(0x3000), ctypes.c_void_p(0x4000), ctypes.c_void_p(0x5000),
                  None, None, None, None, 0.0, 0, None, ctypes.c_void_p(0x6000), 1 << 30,
                  None) in (-4, -2)
    # workspace too small
    assert rc("pq_qprod", FAKE, ctypes.c_void_p(0x2000), 0, ctypes.c_void_p(0x3000),
              ctypes.c_void_p(0x4000), 4, 3, 5, 8, 2, 0, None, None, ctypes.c_void_p(0x5000), 16,
              None) == -8
    # shape: m of B must match (facewise shapes come from the caller, so check p)
    assert rc("pq_qprod_backward", FAKE, FAKE, FAKE, FAKE, None, None, 0, 4, 3, 5, 8, 9,
              ctypes.c_void_p(0x2000), None, None, ctypes.c_void_p(0x5000), 1 << 30, None) == -3


def test_workspace_queries_monotone():
    lib = _lib.load()
    a = lib.pq_qprod_workspace(32, 24, 20, 16, 4, 0)
    b = lib.pq_qprod_workspace(64, 24, 20, 16, 4, 0)
    assert 0 < a < b
    assert lib.pq_qprod_workspace(32, 24, 20, 16, 4, 1) > a  # float64 needs more
    # the transform-domain intermediate (the fused kernel runs without it)
    assert lib.pq_proj_workspace(100, 100, 64, 16, 0) == 100 * 100 * 16 * 4
    assert lib.pq_proj_workspace(100, 100, 64, 40, 1) == 100 * 100 * 40 * 8
    assert lib.pq_tsvdq_workspace(240, 320, 200, 20, 10, 0) > 2 * 240 * 320 * 20 * 4


def _instances(specs):
    arr = (_lib.PQInstance * len(specs))()
    for i, (n1, n2, n3, n4, p, k) in enumerate(specs):
        x = arr[i]
        x.n1, x.n2, x.n3, x.n4, x.p, x.k = n1, n2, n3, n4, p, k
        x.A, x.Q = 0x1000 * (i + 1), 0x100000 * (i + 1)
        if n4:
            x.B, x.C = 0x2000000 + i, 0x3000000 + i
        if k:
            x.Uhat, x.s, x.Vhat = 0x4000000 + i, 0x5000000 + i, 0x6000000 + i
    return arr


def test_batched_validation():
    lib = _lib.load()
    nb = ctypes.c_size_t()
    good = _instances([(64, 80, 32, 70, 8, 4), (100, 50, 20, 0, 5, 2)])
    assert lib.pq_batched_workspace(ctypes.byref(good), 2, ctypes.byref(nb)) == 0
    assert nb.value > 0
    one = ctypes.c_size_t()
    assert lib.pq_batched_workspace(ctypes.byref(good), 1, ctypes.byref(one)) == 0
    assert 0 < one.value < nb.value
    assert lib.pq_batched_workspace(None, 2, ctypes.byref(nb)) == -1
    assert lib.pq_batched_workspace(ctypes.byref(good), 0, ctypes.byref(nb)) == -11
    assert lib.pq_batched_workspace(_instances([(100, 50, 20, 0, 5, 60)]), 1, ctypes.byref(nb)) == -4
    assert lib.pq_batched_workspace(_instances([(100, 50, 20, 0, 25, 2)]), 1, ctypes.byref(nb)) == -3
    assert lib.pq_batched_workspace(_instances([(600, 50, 20, 0, 5, 2)]), 1, ctypes.byref(nb)) == -10
    assert lib.pq_batched_workspace(_instances([(60, 50, 20, 0, 5, 0)]), 1, ctypes.byref(nb)) == -11
    half = _instances([(64, 80, 32, 70, 8, 4)])
    half[0].C = None  # B without C
    assert lib.pq_batched_workspace(ctypes.byref(half), 1, ctypes.byref(nb)) == -1
    # planning validates before touching the device
    h = ctypes.c_void_p()
    assert lib.pq_batched_plan(ctypes.byref(good), 2, 0, 0.0, None, None, 0, None, ctypes.byref(h)) == -1
    assert lib.pq_batched_run(None, None) == -1
    assert lib.pq_batched_destroy(None) == -1


def test_check_q_flag_and_u3_validation():
    F2 = ctypes.c_void_p(0x2000)
    F3 = ctypes.c_void_p(0x3000)
    assert rc("pq_check_q_flag", None, 0, 8, 2, 1e-6, F2, F3, None) == -1
    assert rc("pq_check_q_flag", FAKE, 0, 8, 2, 1e-6, None, F3, None) == -1
    assert rc("pq_check_q_flag", FAKE, 2, 8, 2, 1e-6, F2, F3, None) == -5
    assert rc("pq_check_q_flag", FAKE, 0, 8, 9, 1e-6, F2, F3, None) == -3
    assert rc("pq_check_q_flag", FAKE, 0, 8, 2, -1.0, F2, F3, None) == -11
    assert rc("pq_check_q_flag", FAKE, 0, 8, 2, float("nan"), F2, F3, None) == -11
    # the U3 Gram product runs over n1 n2 tubes with a 32-bit depth: an area
    # of 2^31 or more is refused before anything else is looked at
    assert rc("pq_u3", FAKE, 0, 65536, 32768, 8, 4, F2, None, None, None, 0, None) == -10
    assert rc("pq_u3", FAKE, 0, 65536, 32767, 8, 4, F2, None, None, None, 0, None) == -8


def test_qprod_noalloc_validation():
    F = [ctypes.c_void_p(0x1000 * (i + 1)) for i in range(4)]
    # a workspace beyond the library's fixed array is refused on the host
    assert rc("pq_qprod_noalloc", F[0], F[1], 0, F[2], F[3], 2048, 2048, 2048, 64, 32, 0, None, None,
              None) == -10
    # sizes large enough to overflow a byte count are refused too
    assert rc("pq_qprod_noalloc", F[0], F[1], 0, F[2], F[3], 1 << 40, 1 << 40, 8, 8, 2, 0, None, None,
              None) == -10
    assert rc("pq_qprod_noalloc", None, F[1], 0, F[2], F[3], 8, 8, 8, 8, 2, 0, None, None, None) == -1
    assert rc("pq_qprod_noalloc", F[0], F[1], 0, F[2], F[3], 8, 8, 8, 8, 9, 0, None, None, None) == -3
    assert rc("pq_qprod_noalloc", F[0], F[1], 5, F[2], F[3], 8, 8, 8, 8, 2, 0, None, None, None) == -5
    assert rc("pq_qprod_noalloc", F[0], F[1], 0, F[2], F[3], 0, 8, 8, 8, 2, 0, None, None, None) == -2
