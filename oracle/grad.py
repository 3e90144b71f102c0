"""Adjoints of the projected product and of the projection, float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper defines the forward maps only; the gradients follow from Def. 3.1
by the chain rule.  Writing C_(3) = Q Ch_(3), Ch = Ah tri Bh,
Ah_(3) = Q^T A_(3), Bh_(3) = Q^T B_(3) and G = dL/dC:

    dCh    = G x_3 Q^T
    dAh_l  = dCh_l Bh_l^T          dBh_l = Ah_l^T dCh_l      (each face l)
    dA     = dAh x_3 Q             dB    = dBh x_3 Q
    dQ     = G_(3) Ch_(3)^T + A_(3) dAh_(3)^T + B_(3) dBh_(3)^T

(the Euclidean gradient of Q treated as a free n3 x p matrix).  For
P = A x_3 Q Q^T:  dA = G x_3 Q Q^T and dQ = G_(3) A_(3)^T Q + A_(3) G_(3)^T Q.
"""

import numpy as np

from .core import hat, unhat, facewise, unfold3, _f64


def qprod_backward(G, A, B, Q):
    G, A, B, Q = _f64(G), _f64(A), _f64(B), _f64(Q)
    Ah, Bh = hat(A, Q), hat(B, Q)
    Ch = facewise(Ah, Bh)
    dCh = hat(G, Q)
    dAh = facewise(dCh, np.transpose(Bh, (1, 0, 2)))
    dBh = facewise(np.transpose(Ah, (1, 0, 2)), dCh)
    dA = unhat(dAh, Q)
    dB = unhat(dBh, Q)
    dQ = (unfold3(G) @ unfold3(Ch).T
          + unfold3(A) @ unfold3(dAh).T
          + unfold3(B) @ unfold3(dBh).T)
    return dA, dB, dQ


def proj_backward(G, A, Q):
    G, A, Q = _f64(G), _f64(A), _f64(Q)
    dA = unhat(hat(G, Q), Q)
    G3, A3 = unfold3(G), unfold3(A)
    dQ = G3 @ (A3.T @ Q) + A3 @ (G3.T @ Q)
    return dA, dQ


def tsvdq_backward(A, Q, k, Gbar=None, sbar=None):
    """Adjoint of the truncated tSVDQ (Alg. 4.1) as a map (A, Q) -> (A_k, s),
    A_k the approximation of Thm. 4.2 and s (k x p) the kept transform-domain
    singular values: returns (dA, dQ) of L = <Gbar, A_k> + <sbar, s>.

    The paper differentiates nothing; this is first-order perturbation theory
    of each face's SVD.  For a face M = Ah_l (n1 x n2) with full SVD
    M = U diag(sigma) V^T (sigma_i taken as 0 past min(n1, n2)) and a
    perturbation with a = U^T dM V, the kept values move by a_ii and the
    rank-k truncation T(M) moves, in the same bases, by
        a_ij                                            i, j < k
        sigma_i (sigma_i a_ij + sigma_j a_ji) / (sigma_i^2 - sigma_j^2)   i < k <= j
        sigma_j (sigma_j a_ij + sigma_i a_ji) / (sigma_j^2 - sigma_i^2)   j < k <= i
        0                                               i, j >= k
    (defined when sigma_k-1 > sigma_k).  Transposing these coefficients gives
    the face gradient; the chain rule through Ah = A x_3 Q^T and
    A_k = T(Ah) x_3 Q supplies dA and the Euclidean dQ.
    """
    A, Q = _f64(A), _f64(Q)
    n1, n2, _ = A.shape
    p = Q.shape[1]
    if not (1 <= k <= min(n1, n2)):
        raise ValueError("k must lie in 1..min(n1, n2)")
    Ah = hat(A, Q)
    Gh = hat(_f64(Gbar), Q) if Gbar is not None else np.zeros_like(Ah)
    sb = _f64(sbar) if sbar is not None else np.zeros((k, p))
    dAh = np.zeros_like(Ah)
    Akh = np.zeros_like(Ah)
    r = min(n1, n2)
    for l in range(p):
        U, S, Vt = np.linalg.svd(Ah[:, :, l], full_matrices=True)
        V = Vt.T
        s_row = np.zeros(n1)
        s_row[:r] = S
        s_col = np.zeros(n2)
        s_col[:r] = S
        g = U.T @ Gh[:, :, l] @ V
        Ab = np.zeros((n1, n2))
        Ab[:k, :k] = g[:k, :k]
        for c in range(k):
            sc2 = S[c] ** 2
            Ab[c, c] += sb[c, l]
            # kept row c, discarded column j
            for j in range(k, n2):
                den = sc2 - s_col[j] ** 2
                Ab[c, j] += sc2 * g[c, j] / den
                if j < n1:
                    Ab[j, c] += S[c] * s_col[j] * g[c, j] / den
            # discarded row i, kept column c
            for i in range(k, n1):
                den = sc2 - s_row[i] ** 2
                Ab[i, c] += sc2 * g[i, c] / den
                if i < n2:
                    Ab[c, i] += S[c] * s_row[i] * g[i, c] / den
        dAh[:, :, l] = U @ Ab @ Vt
        Akh[:, :, l] = (U[:, :k] * S[:k]) @ Vt[:k, :]
    dA = unhat(dAh, Q)
    dQ = unfold3(A) @ unfold3(dAh).T
    if Gbar is not None:
        dQ += unfold3(_f64(Gbar)) @ unfold3(Akh).T
    return dA, dQ
