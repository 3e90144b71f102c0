"""Truncated tSVDQ (Alg. 4.1), its error identity (Thm. 4.2) and the
tSVDQ-II (Alg. 4.2), float64 on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""

from dataclasses import dataclass

import numpy as np

from .core import hat, unhat, facewise, proj, fro2, _f64


@dataclass
class TSVDQResult:
    Uhat: np.ndarray   # n1 x k x p   transform-domain left factors
    s: np.ndarray      # k x p        singular values, descending per face
    Vhat: np.ndarray   # n2 x k x p   transform-domain right factors
    Uk: np.ndarray     # n1 x k x n3  spatial factors (Alg. 4.1 step 4)
    Sk: np.ndarray     # k x k x n3   f-diagonal (Def. 3.5)
    Vk: np.ndarray     # n2 x k x n3
    Ak: np.ndarray     # n1 x n2 x n3 the rank-k approximation U_k *_Q S_k *_Q V_k^H
    s_all: np.ndarray  # min(n1,n2) x p, every singular value of every face


def tsvdq(A, Q, k):
    """Truncated *_Q-SVD (Alg. 4.1).

    1. move to the transform domain, Ah = A x_3 Q^H;
    2. a truncated matrix SVD of each of the p frontal slices (LAPACK gesdd,
       singular values in descending order as Def. 4.1 requires);
    3. return to the spatial domain with x_3 Q.
    The approximation A_k = (Uh_k tri Sh_k tri Vh_k^H) x_3 Q is the one that
    Thm. 4.2 is about.
    """
    A = _f64(A)
    Q = _f64(Q)
    n1, n2, n3 = A.shape
    if not (1 <= k <= min(n1, n2)):
        raise ValueError("k must lie in 1..min(n1, n2) (Alg. 4.1 inputs)")
    Ah = hat(A, Q)
    p = Ah.shape[2]
    r = min(n1, n2)
    Uh = np.zeros((n1, k, p))
    Vh = np.zeros((n2, k, p))
    s = np.zeros((k, p))
    s_all = np.zeros((r, p))
    for i in range(p):
        U, S, Vt = np.linalg.svd(Ah[:, :, i], full_matrices=False)
        Uh[:, :, i] = U[:, :k]
        Vh[:, :, i] = Vt[:k, :].T
        s[:, i] = S[:k]
        s_all[:, i] = S
    Sh = np.zeros((k, k, p))
    for i in range(p):
        Sh[:, :, i] = np.diag(s[:, i])
    Uk = unhat(Uh, Q)
    Sk = unhat(Sh, Q)
    Vk = unhat(Vh, Q)
    Vh_T = np.transpose(Vh, (1, 0, 2))  # facewise transpose (Def. 3.3)
    Ak = unhat(facewise(facewise(Uh, Sh), Vh_T), Q)
    return TSVDQResult(Uh, s, Vh, Uk, Sk, Vk, Ak, s_all)


def tsvdq_error_terms(A, Q, k, s_all=None):
    """The two terms of the Thm. 4.2 error identity,
    ||A - A_k||^2 = sum_{j>k} ||S_jj||^2 + ||A x_3 (I - Q Q^H)||^2.

    The spatial singular tube S_jj = Sh_jj x_3 Q has the same norm as its
    transform-domain tube because Q has orthonormal columns, so the first
    term is the sum of the squares of the discarded facewise singular values.
    """
    A = _f64(A)
    if s_all is None:
        Ah = hat(A, Q)
        s_all = np.stack([np.linalg.svd(Ah[:, :, i], compute_uv=False)
                          for i in range(Ah.shape[2])], axis=1)
    eckart_young = float(np.sum(s_all[k:, :] ** 2))
    projection = fro2(A - proj(A, Q))
    return eckart_young, projection


def relative_error(A, Atilde):
    """RE = ||A - Atilde||_F / ||A||_F (Sec. 5.1.2)."""
    A = _f64(A)
    return float(np.sqrt(fro2(A - _f64(Atilde)) / fro2(A)))


def tsvdq_ii(A, Q, gamma):
    """*_Q-SVDII (Alg. 4.2): one global energy threshold over all
    transform-domain singular values, giving a rank rho_i per face.

    Returns (rho, Ak): the multirank (Def. 4.3) and the approximation
    sum over faces of the rank-rho_i truncations, mapped back with x_3 Q.
    Ties in the global order are broken by face-major index order
    (the permutation of Alg. 4.2 is not unique on ties).
    """
    A = _f64(A)
    Q = _f64(Q)
    if not (0.0 < gamma <= 1.0):
        raise ValueError("gamma must lie in (0, 1]")
    Ah = hat(A, Q)
    n1, n2, p = Ah.shape
    svds = [np.linalg.svd(Ah[:, :, i], full_matrices=False) for i in range(p)]
    r = min(n1, n2)
    # global descending order of every (j, i) singular value
    vals = np.array([svds[i][1][j] for i in range(p) for j in range(r)])
    owner = np.array([i for i in range(p) for j in range(r)])
    order = np.argsort(-vals, kind="stable")
    energy = np.cumsum(vals[order] ** 2) / np.sum(vals ** 2)
    # first K with cumulative energy >= gamma (clamped: rounding can leave the
    # full sum a hair below 1)
    K = min(int(np.searchsorted(energy, gamma)) + 1, vals.size)
    rho = np.zeros(p, dtype=np.int64)
    for idx in order[:K]:
        rho[owner[idx]] += 1
    Akh = np.zeros((n1, n2, p))
    for i in range(p):
        U, S, Vt = svds[i]
        ri = int(rho[i])
        Akh[:, :, i] = (U[:, :ri] * S[:ri]) @ Vt[:ri, :]
    return rho, unhat(Akh, Q)


def _unfold(A, mode):
    """Mode-i unfolding: the mode-i fibres as columns (any fixed column order
    serves, the left singular vectors do not depend on it)."""
    return np.moveaxis(A, mode, 0).reshape(A.shape[mode], -1)


def hosvd(A, k1, k2, k3):
    """Truncated HOSVD of multilinear rank (k1, k2, k3) (Sec. 4.2): U_i the
    leading left singular vectors of each unfolding, core
    G = A x_1 U1^T x_2 U2^T x_3 U3^T, and A_k = G x_1 U1 x_2 U2 x_3 U3.
    Used only to check Thm. 4.6 against the tSVDQ."""
    A = _f64(A)
    Us = []
    for mode, k in enumerate((k1, k2, k3)):
        U, _, _ = np.linalg.svd(_unfold(A, mode), full_matrices=False)
        Us.append(U[:, :k])
    G = np.einsum("ijt,ia,jb,tc->abc", A, Us[0], Us[1], Us[2])
    return np.einsum("abc,ia,jb,tc->ijt", G, Us[0], Us[1], Us[2])
