"""Python binding of the projprod C ABI: argument checks and marshalling only.

Tensors are torch tensors on a ROCm device, indexed like the paper,
X[i, j, t] for an n1 x n2 x n3 tensor, and stored face-major (strides
(1, n1, n1*n2)): ``empty(n1, n2, n3)`` makes one, ``from_storage(S)`` views a
contiguous (n3, n2, n1) tensor as one.  Q is a contiguous (n3, p) tensor.
float32, bfloat16 (inputs) and float64 are accepted; results are float32
(float64 for float64 inputs).  Every call is enqueued on the current stream;
PyTorch only provides memory and the stream, the arithmetic runs in the HIP
kernels of libprojprod.so.
"""

from collections import namedtuple

import torch

from . import _lib
from ._lib import PQ_F32, PQ_F64, PQ_BF16, PREC, call

__all__ = [
    "empty", "from_storage", "is_face_major", "to_face_major", "to_tube_major",
    "autotune", "autotune_save", "autotune_load",
    "check_q", "check_q_flag", "orthonormalize_q", "hat", "unhat", "proj", "facewise",
    "qprod", "qprod_backward", "proj_backward", "tsvdq", "TSVDQ", "QProd", "Proj",
    "Batch", "batched", "u3",
]

_DT = {torch.float32: PQ_F32, torch.float64: PQ_F64, torch.bfloat16: PQ_BF16}


def _stream(device):
    return ctypes_stream(torch.cuda.current_stream(device))


def ctypes_stream(s):
    return s.cuda_stream


def empty(n1, n2, n3, dtype=torch.float32, device="cuda"):
    """An uninitialised face-major n1 x n2 x n3 tensor."""
    return torch.empty((n3, n2, n1), dtype=dtype, device=device).permute(2, 1, 0)


def from_storage(S):
    """View a contiguous (n3, n2, n1) tensor as the face-major n1 x n2 x n3 tensor."""
    if S.dim() != 3 or not S.is_contiguous():
        raise ValueError("from_storage expects a contiguous 3-d tensor")
    return S.permute(2, 1, 0)


def is_face_major(X):
    if X.dim() != 3:
        return False
    n1, n2, n3 = X.shape
    want = (1, n1, n1 * n2)
    return all(s == w or d == 1 for s, w, d in zip(X.stride(), want, X.shape))


def _tensor(X, name, dtypes=(torch.float32, torch.float64, torch.bfloat16)):
    if not isinstance(X, torch.Tensor) or X.device.type != "cuda":
        raise TypeError(f"{name} must be a torch tensor on a ROCm device")
    if X.dtype not in dtypes:
        raise TypeError(f"{name}: dtype {X.dtype} not supported")
    if not is_face_major(X):
        raise ValueError(f"{name} must be face-major (strides (1, n1, n1*n2)); "
                         "see binding.empty / binding.from_storage")
    return X


def _q(Q, dtype):
    if not isinstance(Q, torch.Tensor) or Q.device.type != "cuda" or Q.dim() != 2:
        raise TypeError("Q must be a 2-d torch tensor (n3, p) on a ROCm device")
    want = torch.float64 if dtype == torch.float64 else torch.float32
    if Q.dtype != want:
        raise TypeError(f"Q must be {want} for {dtype} data")
    if not Q.is_contiguous():
        raise ValueError("Q must be a contiguous (n3, p) tensor (row-major)")
    return Q


def _out_dtype(dtype):
    return torch.float64 if dtype == torch.float64 else torch.float32


def _ws(nbytes, device):
    if nbytes == 0:
        return None, 0
    buf = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
    return buf, int(nbytes)


def _ptr(X):
    return None if X is None else X.data_ptr()


def autotune(on=True):
    """Switch the library's launch-configuration autotuner on or off: while on,
    a call whose launch shape has no recorded choice times the candidate
    configurations (synchronising the stream) and records the fastest."""
    _lib.load().pq_autotune_enable(1 if on else 0)


def autotune_save(path):
    call("pq_autotune_save", str(path).encode())


def autotune_load(path):
    call("pq_autotune_load", str(path).encode())


def check_q(Q):
    """float64 max |Q^T Q - I| as a 0-d device tensor (Def. 3.1 precondition)."""
    if Q.dtype not in (torch.float32, torch.float64):
        raise TypeError("Q must be float32 or float64")
    Q = _q(Q, Q.dtype)
    out = torch.empty((), dtype=torch.float64, device=Q.device)
    call("pq_check_q", _ptr(Q), _DT[Q.dtype], Q.shape[0], Q.shape[1], _ptr(out), _stream(Q.device))
    return out


def check_q_flag(Q, tol):
    """(dist, flag): the float64 distance max |Q^T Q - I| as a 0-d device
    tensor and an int32 device flag, 1 when the distance exceeds tol or is not
    a number (the Def. 3.1 precondition checked on the device, without a host
    round trip)."""
    if Q.dtype not in (torch.float32, torch.float64):
        raise TypeError("Q must be float32 or float64")
    Q = _q(Q, Q.dtype)
    dist = torch.empty((), dtype=torch.float64, device=Q.device)
    flag = torch.empty((), dtype=torch.int32, device=Q.device)
    call("pq_check_q_flag", _ptr(Q), _DT[Q.dtype], Q.shape[0], Q.shape[1], float(tol), _ptr(dist),
         _ptr(flag), _stream(Q.device))
    return dist, flag


def orthonormalize_q(Q, out=None):
    """(Qout, info): Q re-orthonormalised by CholeskyQR2 in float64 (the Q
    factor of the thin QR with positive diagonal R; float32 Q gives float32
    Qout), and an int32 device tensor info[0] = 0, or c + 1 for a column c
    numerically dependent on the earlier ones (Qout is then not written).
    `out` (optional, may be Q itself) receives the result."""
    if Q.dtype not in (torch.float32, torch.float64):
        raise TypeError("Q must be float32 or float64")
    Q = _q(Q, Q.dtype)
    n3, p = Q.shape
    if out is None:
        out = torch.empty_like(Q)
    elif out.dtype != Q.dtype or tuple(out.shape) != (n3, p) or not out.is_contiguous():
        raise ValueError("out must be a contiguous tensor of Q's shape and dtype")
    info = torch.empty(1, dtype=torch.int32, device=Q.device)
    lib = _lib.load()
    wsb, nb = _ws(lib.pq_orthonormalize_q_workspace(n3, p), Q.device)
    call("pq_orthonormalize_q", _ptr(Q), _DT[Q.dtype], n3, p, _ptr(out), _ptr(info), _ptr(wsb), nb,
         _stream(Q.device))
    return out, info


def hat(A, Q, prec="default"):
    """A x_3 Q^T: n1 x n2 x p transform-domain tensor."""
    _tensor(A, "A")
    _q(Q, A.dtype)
    n1, n2, n3 = A.shape
    if Q.shape[0] != n3:
        raise ValueError("Q must have n3 rows")
    p = Q.shape[1]
    Ah = empty(n1, n2, p, _out_dtype(A.dtype), A.device)
    call("pq_hat", _ptr(A), _DT[A.dtype], _ptr(Q), _ptr(Ah), n1, n2, n3, p, PREC[prec],
         _stream(A.device))
    return Ah


def unhat(Ah, Q, prec="default"):
    """Ah x_3 Q: back to the spatial domain, n1 x n2 x n3."""
    _tensor(Ah, "Ahat", (torch.float32, torch.float64))
    _q(Q, Ah.dtype)
    n1, n2, p = Ah.shape
    n3 = Q.shape[0]
    if Q.shape[1] != p:
        raise ValueError("Q must have p columns")
    A = empty(n1, n2, n3, Ah.dtype, Ah.device)
    call("pq_unhat", _ptr(Ah), _ptr(Q), _ptr(A), _DT[Ah.dtype], n1, n2, n3, p, PREC[prec],
         _stream(Ah.device))
    return A


def _proj_fwd(A, Q, prec):
    _tensor(A, "A")
    _q(Q, A.dtype)
    n1, n2, n3 = A.shape
    p = Q.shape[1]
    if Q.shape[0] != n3:
        raise ValueError("Q must have n3 rows")
    out = empty(n1, n2, n3, _out_dtype(A.dtype), A.device)
    lib = _lib.load()
    wsb, nb = _ws(lib.pq_proj_workspace(n1, n2, n3, p, _DT[A.dtype]), A.device)
    call("pq_proj", _ptr(A), _DT[A.dtype], _ptr(Q), _ptr(out), n1, n2, n3, p, PREC[prec],
         _ptr(wsb), nb, _stream(A.device))
    return out


def facewise(Ah, Bh, prec="default"):
    """Facewise product (Def. 2.3) of two n1 x m x p and m x n2 x p tensors."""
    _tensor(Ah, "Ahat", (torch.float32, torch.float64))
    _tensor(Bh, "Bhat", (Ah.dtype,))
    n1, m, p = Ah.shape
    if Bh.shape[0] != m or Bh.shape[2] != p:
        raise ValueError("facewise: shapes do not agree")
    n2 = Bh.shape[1]
    Ch = empty(n1, n2, p, Ah.dtype, Ah.device)
    call("pq_facewise", _ptr(Ah), _ptr(Bh), _ptr(Ch), _DT[Ah.dtype], n1, m, n2, p, PREC[prec],
         _stream(Ah.device))
    return Ch


def _qprod_fwd(A, B, Q, prec, save=False):
    _tensor(A, "A")
    _tensor(B, "B", (A.dtype,))
    _q(Q, A.dtype)
    n1, m, n3 = A.shape
    if B.shape[0] != m or B.shape[2] != n3:
        raise ValueError("qprod: A is n1 x m x n3 and B must be m x n2 x n3")
    n2 = B.shape[1]
    if Q.shape[0] != n3:
        raise ValueError("Q must have n3 rows")
    p = Q.shape[1]
    od = _out_dtype(A.dtype)
    C = empty(n1, n2, n3, od, A.device)
    Ah = empty(n1, m, p, od, A.device) if save else None
    Bh = empty(m, n2, p, od, A.device) if save else None
    lib = _lib.load()
    wsb, nb = _ws(lib.pq_qprod_workspace(n1, m, n2, n3, p, _DT[A.dtype]), A.device)
    call("pq_qprod", _ptr(A), _ptr(B), _DT[A.dtype], _ptr(Q), _ptr(C), n1, m, n2, n3, p,
         PREC[prec], _ptr(Ah), _ptr(Bh), _ptr(wsb), nb, _stream(A.device))
    return C, Ah, Bh


def qprod_noalloc(A, B, Q, prec="default"):
    """A *_Q B through pq_qprod_noalloc: the library's fixed scratch array
    instead of a workspace (forward only; the output C is still allocated
    here, as the caller's)."""
    _tensor(A, "A")
    _tensor(B, "B", (A.dtype,))
    _q(Q, A.dtype)
    n1, m, n3 = A.shape
    if B.shape[0] != m or B.shape[2] != n3:
        raise ValueError("qprod: A is n1 x m x n3 and B must be m x n2 x n3")
    n2 = B.shape[1]
    if Q.shape[0] != n3:
        raise ValueError("Q must have n3 rows")
    p = Q.shape[1]
    C = empty(n1, n2, n3, _out_dtype(A.dtype), A.device)
    call("pq_qprod_noalloc", _ptr(A), _ptr(B), _DT[A.dtype], _ptr(Q), _ptr(C), n1, m, n2, n3, p,
         PREC[prec], None, None, _stream(A.device))
    return C


PQ_LAYOUT_FACE_MAJOR, PQ_LAYOUT_TUBE_MAJOR = 0, 1


def to_face_major(X):
    """A face-major copy of X (n1, n2, n3): a contiguous (C-order, tube-major)
    tensor is converted by the library's relayout kernel."""
    if not isinstance(X, torch.Tensor) or X.device.type != "cuda" or X.dtype not in _DT:
        raise TypeError("X must be a float32, float64 or bfloat16 torch tensor on a ROCm device")
    if X.dim() != 3 or not X.is_contiguous():
        raise ValueError("to_face_major expects a contiguous (n1, n2, n3) tensor")
    n1, n2, n3 = X.shape
    out = empty(n1, n2, n3, X.dtype, X.device)
    call("pq_relayout", _ptr(X), PQ_LAYOUT_TUBE_MAJOR, _ptr(out), _DT[X.dtype], n1, n2, n3, _stream(X.device))
    return out


def to_tube_major(X):
    """A contiguous (C-order) copy of the face-major tensor X (n1, n2, n3)."""
    _tensor(X, "X")
    if not is_face_major(X):
        raise ValueError("to_tube_major expects a face-major tensor")
    n1, n2, n3 = X.shape
    out = torch.empty((n1, n2, n3), dtype=X.dtype, device=X.device)
    call("pq_relayout", _ptr(X), PQ_LAYOUT_FACE_MAJOR, _ptr(out), _DT[X.dtype], n1, n2, n3, _stream(X.device))
    return out


def _face_major(G):
    # the adjoint kernels read face-major storage; autograd may hand over any
    # layout: C order goes through the relayout kernel, any other strides are
    # first made contiguous
    if is_face_major(G):
        return G
    return to_face_major(G if G.is_contiguous() else G.contiguous())


def qprod_backward(G, A, B, Q, Ahat=None, Bhat=None, need=(True, True, True)):
    """(dA, dB, dQ) of L given G = dL/dC for C = A *_Q B; entries of `need`
    that are False come back as None."""
    for X, nm in ((G, "G"), (A, "A"), (B, "B")):
        _tensor(X, nm, (torch.float32, torch.float64))
    _q(Q, A.dtype)
    n1, m, n3 = A.shape
    n2 = B.shape[1]
    p = Q.shape[1]
    dt = A.dtype
    dA = empty(n1, m, n3, dt, A.device) if need[0] else None
    dB = empty(m, n2, n3, dt, A.device) if need[1] else None
    dQ = torch.empty((n3, p), dtype=dt, device=A.device) if need[2] else None
    lib = _lib.load()
    wsb, nb = _ws(lib.pq_qprod_backward_workspace(n1, m, n2, n3, p, _DT[dt]), A.device)
    call("pq_qprod_backward", _ptr(G), _ptr(A), _ptr(B), _ptr(Q), _ptr(Ahat), _ptr(Bhat), _DT[dt],
         n1, m, n2, n3, p, _ptr(dA), _ptr(dB), _ptr(dQ), _ptr(wsb), nb, _stream(A.device))
    return dA, dB, dQ


def proj_backward(G, A, Q, need=(True, True)):
    _tensor(G, "G", (torch.float32, torch.float64))
    _tensor(A, "A", (G.dtype,))
    _q(Q, G.dtype)
    n1, n2, n3 = A.shape
    p = Q.shape[1]
    dA = empty(n1, n2, n3, G.dtype, G.device) if need[0] else None
    dQ = torch.empty((n3, p), dtype=G.dtype, device=G.device) if need[1] else None
    lib = _lib.load()
    wsb, nb = _ws(lib.pq_proj_backward_workspace(n1, n2, n3, p, _DT[G.dtype]), G.device)
    call("pq_proj_backward", _ptr(G), _ptr(A), _ptr(Q), _DT[G.dtype], n1, n2, n3, p, _ptr(dA),
         _ptr(dQ), _ptr(wsb), nb, _stream(G.device))
    return dA, dQ


class QProd(torch.autograd.Function):
    """C = A *_Q B (Def. 3.1) with the hand-written adjoint for dA, dB, dQ."""

    @staticmethod
    def forward(ctx, A, B, Q, prec="default"):
        C, Ah, Bh = _qprod_fwd(A, B, Q, prec, save=True)
        ctx.save_for_backward(A, B, Q, Ah, Bh)
        return C

    @staticmethod
    def backward(ctx, G):
        A, B, Q, Ah, Bh = ctx.saved_tensors
        need = ctx.needs_input_grad[:3]
        dA, dB, dQ = qprod_backward(_face_major(G.to(Ah.dtype)), A, B, Q, Ah, Bh, need)
        return dA, dB, dQ, None


class Proj(torch.autograd.Function):
    """A x_3 Q Q^T with the hand-written adjoint for dA and dQ."""

    @staticmethod
    def forward(ctx, A, Q, prec="default"):
        ctx.save_for_backward(A, Q)
        return _proj_fwd(A, Q, prec)

    @staticmethod
    def backward(ctx, G):
        A, Q = ctx.saved_tensors
        need = ctx.needs_input_grad[:2]
        dA, dQ = proj_backward(_face_major(G.to(Q.dtype)), A, Q, need)
        return dA, dQ, None


def qprod(A, B, Q, prec="default"):
    """A *_Q B (Def. 3.1); differentiable in A, B and Q (float32/float64)."""
    if torch.is_grad_enabled() and any(x.requires_grad for x in (A, B, Q)):
        return QProd.apply(A, B, Q, prec)
    return _qprod_fwd(A, B, Q, prec)[0]


def proj(A, Q, prec="default"):
    """A x_3 Q Q^T; differentiable in A and Q (float32/float64)."""
    if torch.is_grad_enabled() and any(x.requires_grad for x in (A, Q)):
        return Proj.apply(A, Q, prec)
    return _proj_fwd(A, Q, prec)


TSVDQ = namedtuple("TSVDQ", "Uhat s Vhat Uk Sk Vk Ak info")


Q_KINDS = {"identity": 0, "dct": 1}


def build_q(kind, n3, p, dtype=torch.float32, device="cuda"):
    """Q (n3, p) of a fixed transform of Sec. 5: "identity" or "dct" (the
    first p rows of the orthonormal DCT-II matrix, transposed)."""
    if kind not in Q_KINDS:
        raise ValueError(f"kind must be one of {sorted(Q_KINDS)}")
    Q = torch.empty((n3, p), dtype=dtype, device=device)
    call("pq_build_q", Q_KINDS[kind], n3, p, _DT[dtype], _ptr(Q), _stream(Q.device))
    return Q


def _info(info, n, dev):
    """The caller's int32 info tensor of n entries (every entry is written by
    the library), or a new uninitialised one."""
    if info is None:
        return torch.empty(n, dtype=torch.int32, device=dev)
    if info.dtype != torch.int32 or info.numel() != n or not info.is_contiguous() or info.device != dev:
        raise ValueError(f"info must be a contiguous int32 tensor of {n} entries on the data's device")
    return info


def u3(A, p, info=None):
    """Q = U3(:, :p) of A (Thm. 4.3): the leading p left singular vectors of
    the mode-3 unfolding, as an (n3, p) tensor (float32, or float64 for
    float64 data), with the eigenvalues sigma_i(A_(3))^2 (p,) and the Jacobi
    info int32[3] (`info`, when given, receives it)."""
    _tensor(A, "A", (torch.float32, torch.float64))
    n1, n2, n3 = A.shape
    dev = A.device
    Q = torch.empty((n3, p), dtype=A.dtype, device=dev)
    lam = torch.empty(p, dtype=A.dtype, device=dev)
    info = _info(info, 3, dev)
    lib = _lib.load()
    wsb, nb = _ws(lib.pq_u3_workspace(n1, n2, n3, p, _DT[A.dtype]), dev)
    call("pq_u3", _ptr(A), _DT[A.dtype], n1, n2, n3, p, _ptr(Q), _ptr(lam), _ptr(info), _ptr(wsb), nb,
         _stream(dev))
    return Q, lam, info


def tsvdq(A, Q, k, prec="default", spatial=False, approx=False, tol=0.0, max_sweeps=0, info=None):
    """Truncated *_Q-SVD (Alg. 4.1).  Returns TSVDQ(Uhat n1 x k x p,
    s (k, p), Vhat n2 x k x p, Uk, Sk (k, n3), Vk [spatial=True], Ak
    [approx=True], info = int32 device tensor [max sweeps, unconverged faces,
    total sweeps] (`info`, when given, receives it))."""
    _tensor(A, "A")
    _q(Q, A.dtype)
    n1, n2, n3 = A.shape
    if Q.shape[0] != n3:
        raise ValueError("Q must have n3 rows")
    p = Q.shape[1]
    od = _out_dtype(A.dtype)
    dev = A.device
    Uh = empty(n1, k, p, od, dev)
    Vh = empty(n2, k, p, od, dev)
    s = torch.empty((p, k), dtype=od, device=dev)
    Uk = empty(n1, k, n3, od, dev) if spatial else None
    Vk = empty(n2, k, n3, od, dev) if spatial else None
    Sk = torch.empty((n3, k), dtype=od, device=dev) if spatial else None
    Ak = empty(n1, n2, n3, od, dev) if approx else None
    info = _info(info, 3, dev)
    lib = _lib.load()
    wsb, nb = _ws(lib.pq_tsvdq_workspace(n1, n2, n3, p, k, _DT[A.dtype]), dev)
    call("pq_tsvdq", _ptr(A), _DT[A.dtype], _ptr(Q), n1, n2, n3, p, k, PREC[prec], _ptr(Uh),
         _ptr(s), _ptr(Vh), _ptr(Uk), _ptr(Sk), _ptr(Vk), _ptr(Ak), float(tol), int(max_sweeps),
         _ptr(info), _ptr(wsb), nb, _stream(dev))
    return TSVDQ(Uh, s.t(), Vh, Uk, None if Sk is None else Sk.t(), Vk, Ak, info)


def tsvdq_backward(A, Q, k, Gbar=None, sbar=None, need=(True, True), gap_tol=0.0, tol=0.0,
                   max_sweeps=0, info=None):
    """(dA, dQ, info) of L given Gbar = dL/dA_k (n1 x n2 x n3) and/or
    sbar = dL/ds ((k, p), as tsvdq returns s), for the rank-k tSVDQ of A;
    entries of `need` that are False come back as None.  info is the int32
    device tensor [max sweeps, unconverged faces, total sweeps, dropped
    near-degenerate pairs] (`info`, when given, receives it)."""
    _tensor(A, "A", (torch.float32, torch.float64))
    _q(Q, A.dtype)
    n1, n2, n3 = A.shape
    p = Q.shape[1]
    dt = A.dtype
    if Gbar is not None:
        if tuple(Gbar.shape) != (n1, n2, n3):
            raise ValueError("Gbar must have the shape of A")
        Gbar = _tensor(_face_major(Gbar.to(dt)), "Gbar", (dt,))
    if sbar is not None:
        if tuple(sbar.shape) != (k, p):
            raise ValueError("sbar must be (k, p)")
        sbar = sbar.to(dt).t().contiguous()  # element (j, l) at j + l k
    dA = empty(n1, n2, n3, dt, A.device) if need[0] else None
    dQ = torch.empty((n3, p), dtype=dt, device=A.device) if need[1] else None
    info = _info(info, 4, A.device)
    lib = _lib.load()
    wsb, nb = _ws(lib.pq_tsvdq_backward_workspace(n1, n2, n3, p, k, _DT[dt]), A.device)
    call("pq_tsvdq_backward", _ptr(A), _DT[dt], _ptr(Q), n1, n2, n3, p, k, _ptr(Gbar), _ptr(sbar),
         _ptr(dA), _ptr(dQ), float(gap_tol), float(tol), int(max_sweeps), _ptr(info), _ptr(wsb), nb,
         _stream(A.device))
    return dA, dQ, info


class TSVDQApprox(torch.autograd.Function):
    """(A_k, s) of the rank-k tSVDQ (Alg. 4.1, Thm. 4.2) with the hand-written
    adjoint for dA and dQ."""

    @staticmethod
    def forward(ctx, A, Q, k, prec="default"):
        out = tsvdq(A, Q, k, prec=prec, approx=True)
        ctx.save_for_backward(A, Q)
        ctx.k = k
        return out.Ak, out.s

    @staticmethod
    def backward(ctx, gAk, gs):
        A, Q = ctx.saved_tensors
        need = ctx.needs_input_grad[:2]
        dA, dQ, _ = tsvdq_backward(A, Q, ctx.k, Gbar=gAk, sbar=gs, need=need)
        return dA, dQ, None, None


def tsvdq_approx(A, Q, k, prec="default"):
    """(A_k, s) of the rank-k tSVDQ; differentiable in A and Q (float32/float64)."""
    if torch.is_grad_enabled() and any(x.requires_grad for x in (A, Q)):
        return TSVDQApprox.apply(A, Q, k, prec)
    out = tsvdq(A, Q, k, prec=prec, approx=True)
    return out.Ak, out.s


SVDII = namedtuple("SVDII", "Uhat s Vhat rho Ak info")


def svdii(A, Q, gamma, kmax=None, prec="default", approx=False, tol=0.0, max_sweeps=0, info=None):
    """*_Q-SVDII (Alg. 4.2): per-face ranks rho from one energy threshold
    gamma over the singular values of every face.  Returns SVDII(Uhat
    n1 x kmax x p, s (kmax, p), Vhat n2 x kmax x p with face l's columns
    beyond min(rho_l, kmax) zero, rho (int32 device tensor of p, before the
    kmax cap), Ak [approx=True], info); kmax defaults to min(n1, n2)."""
    _tensor(A, "A")
    _q(Q, A.dtype)
    n1, n2, n3 = A.shape
    if Q.shape[0] != n3:
        raise ValueError("Q must have n3 rows")
    p = Q.shape[1]
    k = min(n1, n2) if kmax is None else int(kmax)
    od = _out_dtype(A.dtype)
    dev = A.device
    Uh = empty(n1, k, p, od, dev)
    Vh = empty(n2, k, p, od, dev)
    s = torch.empty((p, k), dtype=od, device=dev)
    rho = torch.empty(p, dtype=torch.int32, device=dev)
    Ak = empty(n1, n2, n3, od, dev) if approx else None
    info = _info(info, 3, dev)
    lib = _lib.load()
    wsb, nb = _ws(lib.pq_svdii_workspace(n1, n2, n3, p, k, _DT[A.dtype]), dev)
    call("pq_svdii", _ptr(A), _DT[A.dtype], _ptr(Q), n1, n2, n3, p, float(gamma), k, PREC[prec],
         _ptr(Uh), _ptr(s), _ptr(Vh), _ptr(rho), _ptr(Ak), float(tol), int(max_sweeps), _ptr(info),
         _ptr(wsb), nb, _stream(dev))
    return SVDII(Uh, s.t(), Vh, rho, Ak, info)


class Batch:
    """A planned batch of uneven instances (pq_batched_plan).

    ``outputs[i]`` holds instance i's results: ``C`` (A *_Q B, when B was
    given) and ``Uhat``, ``s`` (k, p), ``Vhat`` (when k was given).  The plan
    already ran the batch once; ``run()`` replays the captured graph on the
    current stream, reading the same input tensors (update them in place) and
    writing the same output tensors.  ``info`` is the int32 device tensor of
    sweep statistics over every face, as in tsvdq."""

    def __init__(self, instances, max_sweeps=0, tol=0.0):
        lib = _lib.load()
        self._keep = []
        self.outputs = []
        arr = (_lib.PQInstance * len(instances))()
        dev = None
        for i, inst in enumerate(instances):
            A, Q = inst["A"], inst["Q"]
            _tensor(A, "A", (torch.float32,))
            _q(Q, torch.float32)
            dev = A.device
            n1, n2, n3 = A.shape
            if Q.shape[0] != n3:
                raise ValueError("Q must have n3 rows")
            p = Q.shape[1]
            out = {}
            x = arr[i]
            x.n1, x.n2, x.n3, x.p = n1, n2, n3, p
            x.A, x.Q = _ptr(A), _ptr(Q)
            self._keep += [A, Q]
            B = inst.get("B")
            if B is not None:
                _tensor(B, "B", (torch.float32,))
                if B.shape[0] != n2 or B.shape[2] != n3:
                    raise ValueError("B must be n2 x n4 x n3")
                n4 = B.shape[1]
                C = empty(n1, n4, n3, torch.float32, dev)
                x.n4, x.B, x.C = n4, _ptr(B), _ptr(C)
                out["C"] = C
                self._keep += [B, C]
            k = inst.get("k")
            if k is not None:
                Uh = empty(n1, k, p, torch.float32, dev)
                Vh = empty(n2, k, p, torch.float32, dev)
                s = torch.empty((p, k), dtype=torch.float32, device=dev)
                x.k, x.Uhat, x.s, x.Vhat = k, _ptr(Uh), _ptr(s), _ptr(Vh)
                out.update(Uhat=Uh, s=s.t(), Vhat=Vh)
                self._keep += [Uh, Vh, s]
            self.outputs.append(out)
        nbytes = _lib.ctypes.c_size_t()
        call("pq_batched_workspace", _lib.ctypes.byref(arr), len(instances), _lib.ctypes.byref(nbytes))
        self._ws, nb = _ws(nbytes.value, dev)
        self.info = torch.empty(3, dtype=torch.int32, device=dev)
        self._arr = arr
        h = _lib.ctypes.c_void_p()
        call("pq_batched_plan", _lib.ctypes.byref(arr), len(instances), int(max_sweeps), float(tol),
             _ptr(self.info), _ptr(self._ws), nb, _stream(dev), _lib.ctypes.byref(h))
        self._h = h
        self._dev = dev
        self.workspace_bytes = nb

    def run(self):
        call("pq_batched_run", self._h, _stream(self._dev))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            torch.cuda.synchronize(self._dev)
            _lib.load().pq_batched_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # interpreter shutdown
            pass


def batched(instances, max_sweeps=0, tol=0.0):
    """Plan (and run once) a batch: ``instances`` is a list of dicts with
    "A" (n1 x n2 x n3), "Q" (n3 x p), optionally "B" (n2 x n4 x n3) for
    A *_Q B and "k" for the rank-k tSVDQ of A.  Returns a Batch."""
    return Batch(instances, max_sweeps, tol)
