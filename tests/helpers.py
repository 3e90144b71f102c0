"""Shared helpers of the GPU parity tests (marshalling between numpy face-major
storage and device tensors; error norms)."""

import sys

import numpy as np

from paper_2409_19402_amd import synth


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(storage, dtype=None):
    """numpy face-major storage (n3, n2, n1) -> face-major device tensor."""
    import torch
    from paper_2409_19402_amd import binding
    t = torch.from_numpy(np.ascontiguousarray(storage))
    if dtype is not None:
        t = t.to(dtype)
    return binding.from_storage(t.cuda())


def dev_bf16(bits_storage):
    """uint16 bfloat16 patterns (n3, n2, n1) -> face-major torch.bfloat16 tensor."""
    import torch
    from paper_2409_19402_amd import binding
    t = torch.from_numpy(np.ascontiguousarray(bits_storage).view(np.int16)).cuda()
    return binding.from_storage(t.view(torch.bfloat16))


def devq(Q):
    import torch
    return torch.from_numpy(np.ascontiguousarray(Q)).cuda()


def host(X):
    """device tensor (any layout) -> numpy float64 array of its logical shape."""
    return X.detach().double().cpu().numpy()


def rel(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.linalg.norm((x - ref).ravel())
    n = np.linalg.norm(ref.ravel())
    return d / n if n > 0 else d


def logical(storage):
    return synth.logical(storage)


def relmax(x, ref):
    """max |x - ref| / max |ref|: the element-wise companion of rel(), which
    catches an error confined to a few elements (one ragged strip, one face)
    that a whole-tensor norm would average away."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    m = float(np.max(np.abs(ref))) if ref.size else 0.0
    d = float(np.max(np.abs(x - ref))) if ref.size else 0.0
    return d / m if m > 0 else d
