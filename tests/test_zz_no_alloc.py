"""pq_qprod_noalloc (the projected product of Def. 3.1 with its workspace in
the library's fixed scratch array) against pq_qprod with a caller-provided
workspace, through the C ABI: two calls in a row, the second smaller, in
float32, bfloat16 and float64, and the size limit."""

import ctypes

import numpy as np
import pytest

from helpers import dev, devq, host, say
from paper_2409_19402_amd import _lib, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _with_ws(torch, lib, A, B, Q, dt, n1, m, n2, n3, p, prec, C):
    nb = lib.pq_qprod_workspace(n1, m, n2, n3, p, dt)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    rc = lib.pq_qprod(_ptr(A), _ptr(B), dt, _ptr(Q), _ptr(C), n1, m, n2, n3, p, prec, None, None,
                      _ptr(ws), nb, _stream(torch))
    assert rc == 0, rc


def _no_ws(torch, lib, A, B, Q, dt, n1, m, n2, n3, p, prec, C):
    rc = lib.pq_qprod_noalloc(_ptr(A), _ptr(B), dt, _ptr(Q), _ptr(C), n1, m, n2, n3, p, prec, None, None,
                              _stream(torch))
    assert rc == 0, rc


@pytest.mark.parametrize("kind", ["f32", "bf16x3", "bf16", "f64"])
def test_noalloc_matches_workspace_call(torch_dev, kind):
    torch = torch_dev
    lib = _lib.load()
    rng = np.random.default_rng(41)
    dt = {"f32": 0, "bf16x3": 0, "bf16": 2, "f64": 1}[kind]
    prec = {"f32": 0, "bf16x3": 2, "bf16": 0, "f64": 0}[kind]
    # the second call is smaller than the first, so that a stale tail of the
    # first call's intermediates would show
    for (n1, m, n2, n3, p) in [(256, 128, 256, 128, 16), (70, 33, 45, 40, 9)]:
        say(f"  noalloc {kind}: {n1}x{m}x{n3} * {m}x{n2}x{n3}, p={p}")
        A = synth.gaussian(rng, n1, m, n3)
        B = synth.gaussian(rng, m, n2, n3)
        Q = synth.random_orthonormal(rng, n3, p)
        if kind == "f64":
            Ad, Bd = dev(A, torch.float64), dev(B, torch.float64)
            Qd, od = devq(Q.astype(np.float64)), torch.float64
        elif kind == "bf16":
            Ad, Bd = dev(A, torch.bfloat16), dev(B, torch.bfloat16)
            Qd, od = devq(Q.astype(np.float32)), torch.float32
        else:
            Ad, Bd = dev(A), dev(B)
            Qd, od = devq(Q.astype(np.float32)), torch.float32
        ref = torch.empty((n3, n2, n1), dtype=od, device="cuda")
        out = torch.full((n3, n2, n1), float("nan"), dtype=od, device="cuda")
        _with_ws(torch, lib, Ad, Bd, Qd, dt, n1, m, n2, n3, p, prec, ref)
        _no_ws(torch, lib, Ad, Bd, Qd, dt, n1, m, n2, n3, p, prec, out)
        torch.cuda.synchronize()
        # the same kernels on the same inputs: the same bits
        assert torch.equal(out, ref)
        assert bool(torch.isfinite(out).all())


def test_noalloc_limit(torch_dev):
    lib = _lib.load()
    F = [ctypes.c_void_p(0x1000 * (i + 1)) for i in range(5)]
    # workspace beyond the fixed array: refused before anything is enqueued
    big = lib.pq_qprod_workspace(2048, 2048, 2048, 64, 32, 0)
    assert big > (64 << 20)
    assert lib.pq_qprod_noalloc(F[0], F[1], 0, F[2], F[3], 2048, 2048, 2048, 64, 32, 0, None, None, None) == -10
    # argument errors come first, as in pq_qprod
    assert lib.pq_qprod_noalloc(None, F[1], 0, F[2], F[3], 8, 8, 8, 8, 2, 0, None, None, None) == -1
    assert lib.pq_qprod_noalloc(F[0], F[1], 0, F[2], F[3], 8, 8, 8, 8, 9, 0, None, None, None) == -3
