"""Seeded synthetic inputs shaped like the paper's workloads.

This module builds inputs only: tensors, orthonormal Q matrices, targets.  It
holds none of the projected-product arithmetic and imports neither the GPU
binding nor the oracle, so both sides can take their inputs from it.

Every tensor is returned in face-major storage: a C-contiguous numpy array of
shape (n3, n2, n1), whose element [t, j, i] is the paper's A(i, j, t)
(Def. 2.1 order: i fastest, then j, then t).  ``logical(x)`` gives the
(n1, n2, n3) view the oracle indexes.

Recipes (the paper's data sets are not available; these stand in for them):

* gaussian: i.i.d. N(0, 1).
* random orthonormal Q: the Q factor of the Householder QR of a seeded
  n3 x p Gaussian, columns signed so that diag(R) > 0 (the 'random
  orthogonal' transformation of Sec. 5.1.1).
* video: a height x width x frames clip, a sum of separable components
  (an axis-aligned 2-D Gaussian blob times a slowly drifting temporal cosine)
  plus N(0, var) noise; stands in for the grey-scale videos of Sec. 5.2.
* hyperspectral: a pixels x pixels x bands cube, Dirichlet(0.5) abundances
  over endmember spectra that are each a sum of Gaussian bumps across the
  bands, plus N(0, var) noise, rounded to bfloat16; stands in for the
  hyperspectral image of Sec. 5.3.
* U3 Q: the leading p left singular vectors of the mode-3 unfolding (the
  data-dependent transformation of Sec. 5.1.1 and Thm. 4.3), computed in
  float64 from the eigen-decomposition of A_(3) A_(3)^T and signed so that
  each column's largest-magnitude entry is positive.
"""

import numpy as np


def logical(x):
    """(n3, n2, n1) face-major storage -> (n1, n2, n3) logical view."""
    return np.transpose(x, (2, 1, 0))


def storage(a):
    """(n1, n2, n3) logical array -> C-contiguous (n3, n2, n1) storage."""
    return np.ascontiguousarray(np.transpose(a, (2, 1, 0)))


def gaussian(rng, n1, n2, n3, dtype=np.float32):
    return rng.standard_normal((n3, n2, n1)).astype(dtype)


def random_orthonormal(rng, n3, p, dtype=np.float64):
    X = rng.standard_normal((n3, p))
    Qm, R = np.linalg.qr(X)
    sgn = np.sign(np.diag(R))
    sgn[sgn == 0] = 1.0
    return (Qm * sgn).astype(dtype)


def bf16_bits(x):
    """Round float32 values to bfloat16 (round to nearest, ties to even);
    returns the 16-bit patterns as uint16."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    lsb = (u >> 16) & 1
    r = (u + np.uint32(0x7FFF) + lsb) >> 16
    nan = np.isnan(np.asarray(x, dtype=np.float32))
    r = np.where(nan, (u >> 16) | 0x40, r)
    return r.astype(np.uint16)


def bf16_to_f32(bits):
    return (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def video(rng, n1=240, n2=320, n3=200, components=10, noise_var=1e-2):
    """Video-shaped tensor (height x width x frames), float32 face-major."""
    x = np.arange(n1, dtype=np.float64)
    y = np.arange(n2, dtype=np.float64)
    t = np.arange(n3, dtype=np.float64)
    gx = np.empty((components, n1))
    gy = np.empty((components, n2))
    h = np.empty((components, n3))
    for c in range(components):
        amp = rng.uniform(0.5, 2.0)
        cx, cy = rng.uniform(0, n1), rng.uniform(0, n2)
        sx, sy = rng.uniform(8, 40), rng.uniform(8, 40)
        f, phi = rng.uniform(0.5, 4.0), rng.uniform(0, 2 * np.pi)
        gx[c] = amp * np.exp(-((x - cx) ** 2) / (2 * sx * sx))
        gy[c] = np.exp(-((y - cy) ** 2) / (2 * sy * sy))
        h[c] = np.cos(2 * np.pi * f * t / n3 + phi)
    A = np.einsum("ct,cy,cx->tyx", h, gy, gx)
    A += np.sqrt(noise_var) * rng.standard_normal(A.shape)
    return A.astype(np.float32)


def hyperspectral(rng, n1=512, n2=512, n3=224, endmembers=8, bumps=3,
                  alpha=0.5, noise_var=1e-3):
    """Hyperspectral-shaped cube, rounded to bfloat16.

    Returns (bits, values): uint16 bfloat16 patterns and the same values as
    float32, both face-major (n3, n2, n1)."""
    lam = np.arange(n3, dtype=np.float64)
    spectra = np.zeros((endmembers, n3))
    for e in range(endmembers):
        for _ in range(bumps):
            mu = rng.uniform(0, n3 - 1)
            w = rng.uniform(4, 30)
            hgt = rng.uniform(0.2, 1.0)
            spectra[e] += hgt * np.exp(-((lam - mu) ** 2) / (2 * w * w))
    abund = rng.dirichlet(alpha * np.ones(endmembers), size=(n2, n1))  # (n2, n1, E)
    A = np.einsum("el,yxe->lyx", spectra, abund)
    A += np.sqrt(noise_var) * rng.standard_normal(A.shape)
    bits = bf16_bits(A.astype(np.float32))
    return bits, bf16_to_f32(bits)


def u3_leading(A_storage, p):
    """Leading p left singular vectors of the mode-3 unfolding, float64.

    A_storage is face-major (n3, n2, n1); its reshape to (n3, n1*n2) is the
    mode-3 unfolding with columns in the order of Def. 2.1."""
    n3 = A_storage.shape[0]
    X = np.asarray(A_storage, dtype=np.float64).reshape(n3, -1)
    gram = X @ X.T
    w, V = np.linalg.eigh(gram)
    V = V[:, ::-1][:, :p]
    idx = np.argmax(np.abs(V), axis=0)
    sgn = np.sign(V[idx, np.arange(p)])
    sgn[sgn == 0] = 1.0
    return V * sgn


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

def tiny(seed=1):
    """Tiny plain-method case, float64: A 32x24x16, B 24x20x16, Q 16x4, k=5."""
    rng = np.random.default_rng(seed)
    A = gaussian(rng, 32, 24, 16, np.float64)
    B = gaussian(rng, 24, 20, 16, np.float64)
    Q = random_orthonormal(rng, 16, 4)
    return dict(A=A, B=B, Q=Q, k=5)


def video_case(seed=2, n1=240, n2=320, n3=200, p=20, k=10):
    """Video-shaped tSVDQ, float32: A 240x320x200, Q = U3(:, :20), k=10."""
    rng = np.random.default_rng(seed)
    A = video(rng, n1, n2, n3)
    Q = u3_leading(A, p).astype(np.float32)
    return dict(A=A, Q=Q, k=k)


def hyperspectral_case(seed=3, n1=512, n2=512, n3=224, p=32, k=16):
    """Hyperspectral-shaped case: A 512x512x224 in bfloat16, Q = U3(:, :32)
    of the rounded data, k=16."""
    rng = np.random.default_rng(seed)
    bits, vals = hyperspectral(rng, n1, n2, n3)
    Q = u3_leading(vals, p).astype(np.float32)
    return dict(A_bits=bits, A=vals, Q=Q, k=k)


def batched_shapes(seed=4, count=64, lo=64, hi=512, n3_lo=32, n3_hi=256,
                   p_lo=4, p_hi=32):
    """Shapes of the uneven batch: n1, n2, n4 ~ U{lo..hi}, n3 ~ U{n3_lo..n3_hi},
    p ~ U{p_lo..min(p_hi, n3)}, k = max(1, p // 2).  Instance i multiplies
    A_i (n1 x n2 x n3) by B_i (n2 x n4 x n3)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n1, n2, n4 = (int(v) for v in rng.integers(lo, hi + 1, size=3))
        n3 = int(rng.integers(n3_lo, n3_hi + 1))
        p = int(rng.integers(p_lo, min(p_hi, n3) + 1))
        out.append(dict(n1=n1, n2=n2, n3=n3, n4=n4, p=p, k=max(1, p // 2)))
    return out


def batched_instance(seed, index, shape):
    """Inputs of one batched instance: A, B i.i.d. N(0,1) float32 and a random
    orthonormal Q (float32), from a stream keyed by (seed, index)."""
    rng = np.random.default_rng([seed, index])
    A = gaussian(rng, shape["n1"], shape["n2"], shape["n3"])
    B = gaussian(rng, shape["n2"], shape["n4"], shape["n3"])
    Q = random_orthonormal(rng, shape["n3"], shape["p"]).astype(np.float32)
    return dict(A=A, B=B, Q=Q, k=shape["k"])


def differentiation_case(seed=5, n1=256, m=128, n2=256, n3=128, p=16):
    """Differentiation case: A 256x128x128, B 128x256x128, Q 128x16, target T
    256x256x128, all float32; loss ||A *_Q B - T||_F^2."""
    rng = np.random.default_rng(seed)
    A = gaussian(rng, n1, m, n3)
    B = gaussian(rng, m, n2, n3)
    Q = random_orthonormal(rng, n3, p).astype(np.float32)
    T = gaussian(rng, n1, n2, n3)
    return dict(A=A, B=B, Q=Q, T=T)
