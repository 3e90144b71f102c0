"""FP64 CPU oracle for the projected tensor-tensor product and the truncated tSVDQ.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain, obviously-correct
reference that the GPU library is checked against.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path (the HIP library and its Python binding) never does, and the
oracle never imports the product path.  The two share no code; they meet only
through the seeded input generators, which hold none of the method's
arithmetic.

Everything is numpy float64 (LAPACK for the per-face SVD).  Tensors are numpy
arrays with the paper's logical index order A[i, j, t] (i < n1, j < n2,
t < n3), real-valued throughout (the paper restricts its experiments to real
transformations, Sec. 5.1.1), so Q^H = Q^T.

Every function cites the definition, equation, algorithm or theorem of
Keegan & Newman, "Projected Tensor-Tensor Products for Efficient Computation
of Optimal Multiway Data Representations" (arXiv:2409.19402) that it follows.
Parity status of each function is listed in ``PARITY`` below.
"""

from .core import (  # noqa: F401
    unfold3, fold3, mode3, facewise, mprod, hat, unhat, qprod, proj,
    identity_tensor, ftranspose, check_q, fro2, u3, identity_q, dct_q, orthonormalize_q,
)
from .tsvdq import (  # noqa: F401
    tsvdq, tsvdq_error_terms, relative_error, tsvdq_ii, TSVDQResult, hosvd,
)
from .grad import qprod_backward, proj_backward, tsvdq_backward  # noqa: F401

# Which pin holds each oracle function (see tests/test_oracle_pins.py).
PARITY = {
    "u3": "pinned: Gram eigen-decomposition (independent route), orthonormality, "
          "Cor 4.1 face norms",
    "unfold3/fold3/mode3": "pinned: Appendix A printed tubes; brute-force loops",
    "facewise": "pinned: brute-force loops",
    "mprod": "pinned: Appendix A printed a*_M b",
    "hat/unhat/qprod/proj": "pinned: Appendix A printed values, brute force, "
                            "Q=I reduction, square-orthogonal reduction to *_M, "
                            "Sec. 3.2 splitting identities",
    "tsvdq": "pinned: Example 4.1 printed errors, Thm 4.2 identity, Cor 4.1, "
             "Eckart-Young optimality, full-rank reduction to proj",
    "tsvdq_ii": "pinned: Thm 4.5 (SVDII error <= tSVDQ error at equal storage), "
                "gamma=1 reduction, the exact K and multirank of diagonal faces with gamma "
                "strictly between consecutive energy fractions (ties ordered face-major)",
    "relative_error": "pinned: Example 4.1 (RE = sqrt(3)/2 and sqrt(2)/2 from the printed squared "
                      "errors and the printed entries) and closed forms",
    "qprod_backward/proj_backward": "pinned: central finite differences (tiny tensors, and "
                                    "qprod_backward at the full differentiation size) and "
                                    "torch CPU float64 autograd",
    "tsvdq_backward": "pinned: central finite differences of <Gbar, A_k> + <sbar, s> "
                      "(tall, wide and square faces, k = 1 and k = min(n1, n2)) and "
                      "torch CPU float64 autograd through torch.linalg.svd",
    "check_q": "pinned: closed form on constructed matrices",
    "orthonormalize_q": "pinned: numpy's Householder thin QR (library routine, sign-fixed to a "
                        "positive diagonal R), orthonormal input returned unchanged, dependent "
                        "column reported",
    "identity_q/dct_q": "pinned: scipy's orthonormal DCT-II of the identity (library routine), "
                        "the n3 = 2 Haar closed form, orthonormal columns",
    "hosvd": "pinned: full multilinear rank reproduces A, the rank-(n1, n2, p) case equals "
             "the projection onto U3 (Thm. 4.3), and the truncation-error bound by the "
             "discarded mode singular values",
}
