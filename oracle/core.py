"""Products of the paper, written out from their definitions (float64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""

import numpy as np


def _f64(x):
    return np.asarray(x, dtype=np.float64)


def fro2(A):
    """Squared Frobenius norm, summed over frontal slices (Sec. 2)."""
    A = _f64(A)
    return float(np.sum(A * A))


def unfold3(A):
    """Mode-3 unfolding A_(3) in R^{n3 x n1 n2} (Def. 2.1).

    Column J(i, j) = i + j*n1 (0-based) holds the tube A[i, j, :].
    """
    A = _f64(A)
    n1, n2, n3 = A.shape
    # Fortran-order reshape makes the first index fastest: row i + j*n1.
    return A.reshape(n1 * n2, n3, order="F").T


def fold3(M, n1, n2):
    """Inverse of unfold3 (Def. 2.1): an n x (n1 n2) matrix -> n1 x n2 x n."""
    M = _f64(M)
    n = M.shape[0]
    return M.T.reshape(n1, n2, n, order="F")


def mode3(A, M):
    """Mode-3 product A x_3 M = fold(M A_(3)) (Def. 2.2), M is p x n3."""
    A = _f64(A)
    n1, n2, _ = A.shape
    return fold3(_f64(M) @ unfold3(A), n1, n2)


def facewise(A, B):
    """Facewise product (Def. 2.3): (A tri B)[:, :, i] = A[:, :, i] B[:, :, i]."""
    A = _f64(A)
    B = _f64(B)
    if A.shape[1] != B.shape[0] or A.shape[2] != B.shape[2]:
        raise ValueError("facewise: inner or third dimension mismatch")
    out = np.empty((A.shape[0], B.shape[1], A.shape[2]))
    for i in range(A.shape[2]):
        out[:, :, i] = A[:, :, i] @ B[:, :, i]
    return out


def mprod(A, B, M):
    """*_M product with invertible n3 x n3 M (Def. 2.4):
    ((A x_3 M) tri (B x_3 M)) x_3 M^{-1}."""
    M = _f64(M)
    return mode3(facewise(mode3(A, M), mode3(B, M)), np.linalg.inv(M))


def hat(A, Q):
    """Transform-domain tensor A x_3 Q^H (Def. 3.1 and the 'hat' convention
    that follows it).  Q is n3 x p with orthonormal columns; the result has p
    frontal slices."""
    return mode3(A, _f64(Q).T)


def unhat(Ah, Q):
    """Return to the spatial domain: Ah x_3 Q (Def. 3.1, Alg. 4.1 step 4)."""
    return mode3(Ah, _f64(Q))


def qprod(A, B, Q):
    """Projected product A *_Q B = [(A x_3 Q^H) tri (B x_3 Q^H)] x_3 Q
    (Def. 3.1)."""
    return unhat(facewise(hat(A, Q), hat(B, Q)), Q)


def proj(A, Q):
    """Orthogonal projection of the tubes onto range(Q):
    (A x_3 Q^H) x_3 Q = A x_3 Q Q^H (Sec. 3, after Fig. 3.1)."""
    return unhat(hat(A, Q), Q)


def identity_tensor(m, Q):
    """*_Q identity (Def. 3.2): every transform-domain face is I_m, so
    I = I_hat x_3 Q."""
    Q = _f64(Q)
    p = Q.shape[1]
    Ih = np.repeat(np.eye(m)[:, :, None], p, axis=2)
    return unhat(Ih, Q)


def ftranspose(A, Q):
    """*_Q (conjugate) transpose (Def. 3.3): transpose every transform-domain
    face, then return to the spatial domain."""
    Ah = hat(A, Q)
    return unhat(np.transpose(Ah, (1, 0, 2)), Q)


def check_q(Q):
    """Distance of Q from the Stiefel manifold, max_ij |(Q^T Q - I)_ij|
    (the precondition Q in St_{n3,p} of Def. 3.1)."""
    Q = _f64(Q)
    return float(np.max(np.abs(Q.T @ Q - np.eye(Q.shape[1]))))


def orthonormalize_q(Q):
    """Q with its columns re-orthonormalised, as a repair of the precondition
    Q in St_{n3,p} of Def. 3.1 (the paper itself assumes that precondition
    and gives no repair): CholeskyQR2, i.e. twice W <- W R^{-1} with R the
    upper Cholesky factor (positive diagonal) of W^T W, starting from W = Q.
    Returns (W, 0), or (None, c + 1) when the pivot of column c is not above
    64 eps times that column's squared norm in either pass."""
    W = _f64(Q).copy()
    eps = np.finfo(np.float64).eps
    for _ in range(2):
        G = W.T @ W
        p = G.shape[0]
        R = np.zeros_like(G)
        for c in range(p):
            d = G[c, c] - R[:c, c] @ R[:c, c]
            if not d > 64.0 * eps * G[c, c]:
                return None, c + 1
            R[c, c] = np.sqrt(d)
            for b in range(c + 1, p):
                R[c, b] = (G[c, b] - R[:c, c] @ R[:c, b]) / R[c, c]
        # rows of W solve x R = w: W R^{-1} column by column
        X = np.empty_like(W)
        for c in range(p):
            X[:, c] = (W[:, c] - X[:, :c] @ R[:c, c]) / R[c, c]
        W = X
    return W, 0


def u3(A, p):
    """Q = U3(:, :p): the leading p left singular vectors of the mode-3
    unfolding A_(3) (the data-dependent transform of Thm. 4.3 and Cor. 4.1),
    with each column signed so that its largest-magnitude entry is positive
    (the first such entry on ties).  Returns (Q, sigma^2) with sigma the
    leading p singular values of A_(3)."""
    A = _f64(A)
    U, S, _ = np.linalg.svd(unfold3(A), full_matrices=False)
    Q = U[:, :p].copy()
    for j in range(p):
        i = int(np.argmax(np.abs(Q[:, j])))
        if Q[i, j] < 0:
            Q[:, j] = -Q[:, j]
    return Q, S[:p] ** 2


def identity_q(n3, p):
    """The first p columns of I_n3 (the control transform of Sec. 5)."""
    return np.eye(n3)[:, :p]


def dct_q(n3, p):
    """The transposed first p rows of the orthonormal DCT-II matrix C
    (Sec. 5.1.1): C[l, t] = w_l cos(pi (2t + 1) l / (2 n3)), w_0 = sqrt(1/n3),
    w_l = sqrt(2/n3); Q = C[:p, :]^T, written out from that definition."""
    C = np.zeros((n3, n3))
    for l in range(n3):
        w = np.sqrt(1.0 / n3) if l == 0 else np.sqrt(2.0 / n3)
        for t in range(n3):
            C[l, t] = w * np.cos(np.pi * (2 * t + 1) * l / (2 * n3))
    return C[:p, :].T
