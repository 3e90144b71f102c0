/*
 * projprod.h — C ABI of the MI355X (gfx950) library for the projected
 * tensor-tensor product *_Q and the truncated tSVDQ built on it
 * (Keegan & Newman, "Projected Tensor-Tensor Products for Efficient
 * Computation of Optimal Multiway Data Representations", arXiv:2409.19402).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Tensors are real, third order, stored FACE-MAJOR: element (i, j, t) of an
 * n1 x n2 x n3 tensor sits at offset i + j*n1 + t*n1*n2 (0-based; the
 * column order of the mode-3 unfolding, Def. 2.1).  Each frontal slice is a
 * contiguous column-major n1 x n2 matrix, and row t of the n3 x (n1 n2)
 * row-major matrix seen by the kernels is frontal slice t.
 *
 * Q is an n3 x p matrix with orthonormal columns (Q in St_{n3,p}, Def. 3.1),
 * stored ROW-MAJOR: Q(t, l) at t*p + l.  1 <= p <= n3.
 *
 * Every pointer argument is a DEVICE pointer owned by the caller, except where
 * a comment says "host".  Entry points never allocate and never synchronise;
 * all work is enqueued on `stream` in order.  (Where a Jacobi sweep launch
 * would hold two or more visits per CU -- tSVDQ, SVDII and their adjoint on
 * many large faces -- the sweeps fork from `stream` onto a second stream of
 * the library's, one per device and host thread created on first use
 * outside graph capture, and join back into `stream` before the call's next
 * step: ordering with respect to `stream` is unchanged, and under graph
 * capture the fork and join become graph dependencies.)  Inputs are read only; outputs
 * must not overlap inputs (PQ_ERR_ALIAS is returned for exact pointer
 * equality; partial overlap is the caller's responsibility).  Scratch memory
 * is passed in `ws` (device, 256-byte aligned) of `ws_bytes` bytes; the
 * matching *_workspace query returns the size needed.  The return value
 * reports errors the host can detect (shapes, dtypes, null pointers, too
 * small a workspace, a failed launch); nothing is launched when it is not
 * PQ_OK.  Conditions only the device can see (Jacobi non-convergence) are
 * written to device memory the caller passes.
 *
 * Data types (dtype arguments): PQ_F32, PQ_F64, PQ_BF16 (bfloat16 bit
 * patterns, inputs only).  A float64 call keeps every operand and result in
 * float64.  A float32 call takes float32 or bfloat16 tensor inputs, float32 Q
 * and writes float32 results.
 *
 * Precision modes (prec arguments, float32 calls only) select how the dense
 * contractions run on the matrix cores:
 *   PQ_PREC_DEFAULT  float32 MFMA (float64 calls: float64 arithmetic)
 *   PQ_PREC_BF16     one bfloat16 MFMA pass, float32 accumulation
 *   PQ_PREC_BF16X3   split-bfloat16 compensated products, x = x_hi + x_lo,
 *                    x*y ~ x_hi y_hi + x_hi y_lo + x_lo y_hi (3 passes); when
 *                    the tensor operand is already bfloat16 the other operand
 *                    is split three ways instead, which is exact in float32
 *   PQ_PREC_BF16X6   three-way split of both operands, 6 passes
 * The modes apply to the forward transform A x_3 Q^T (pq_hat and the
 * transform steps of pq_qprod, pq_proj, pq_tsvdq and pq_svdii), to the
 * facewise product (pq_facewise and the facewise step of pq_qprod) and to the
 * return transform (pq_unhat for p <= 32; float32 above).  Inside pq_qprod,
 * pq_proj, pq_tsvdq and pq_svdii the return transform of the X3 mode runs as
 * X6: it is bound by its writes, so the extra products are free, and they
 * keep the error of the whole chain well inside the float32 tolerance.  The fused
 * projection, the tSVDQ's own factor products and the adjoints run on
 * float32 MFMA in every mode.
 */
#ifndef PROJPROD_H
#define PROJPROD_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define PQ_OK               0
#define PQ_ERR_NULL        -1  /* a required pointer is NULL                     */
#define PQ_ERR_SHAPE       -2  /* a size is < 1, or sizes do not agree           */
#define PQ_ERR_P           -3  /* p < 1 or p > n3                                */
#define PQ_ERR_K           -4  /* k < 1 or k > min(n1, n2)                       */
#define PQ_ERR_DTYPE       -5  /* unsupported dtype combination                  */
#define PQ_ERR_PREC        -6  /* unsupported precision mode for this call       */
#define PQ_ERR_ALIAS       -7  /* an output pointer equals an input pointer      */
#define PQ_ERR_WORKSPACE   -8  /* ws is NULL or ws_bytes too small               */
#define PQ_ERR_HIP         -9  /* a kernel launch failed (see pq_last_hip_error) */
#define PQ_ERR_UNSUPPORTED -10 /* size beyond what this build supports          */
#define PQ_ERR_ARG         -11 /* another argument out of range                  */

/* ---- dtypes and precision modes ------------------------------------------ */
#define PQ_F32  0
#define PQ_F64  1
#define PQ_BF16 2

#define PQ_PREC_DEFAULT 0
#define PQ_PREC_BF16    1
#define PQ_PREC_BF16X3  2
#define PQ_PREC_BF16X6  3

/* Library version (major*10000 + minor*100 + patch). */
int pq_version(void);

/* Static text for a status code; never NULL. */
const char* pq_status_string(int code);

/* The hipError_t of the last failed launch on the calling thread (0 if none). */
int pq_last_hip_error(void);

/* ---- launch-configuration autotuner --------------------------------------- */
/*
 * The library keeps a process-wide table from a launch shape (kernel family,
 * precision mode and sizes) to the fastest of that kernel's candidate launch
 * configurations (vectors per lane, waves per workgroup).  While
 * pq_autotune_enable(1) is in force, a call whose launch shape is not yet in
 * the table times every candidate on its stream (this synchronises the
 * stream; the call's outputs are still written correctly) and records the
 * fastest; otherwise the recorded choice, or a built-in default, is used
 * without synchronising.  pq_autotune_save / pq_autotune_load write and read
 * the table as text ("key choice" per line; host path).  pq_autotune_entries
 * returns the number of recorded shapes.
 */
int pq_autotune_enable(int on);
int pq_autotune_entries(void);
int pq_autotune_save(const char* path);
int pq_autotune_load(const char* path);

/* ---- per-launch timing ---------------------------------------------------- */
/*
 * While enabled, every kernel launch the library makes is bracketed by two
 * hipEvents recorded on the caller's stream (events come from a pool owned by
 * the library; no device memory is allocated); the back-to-back sweep
 * launches of the Jacobi share one pair per phase and count as the launches
 * they are.  Nothing is recorded while the stream is being captured into a
 * graph.  pq_profile_query waits for the recorded events of the launches
 * named `name` (e.g. "hat", "unhat", "facewise_gemm", "jacobi_gram_f32"),
 * and returns their summed duration in milliseconds and their count.  pq_profile_names writes the
 * comma-separated names seen since the last reset into buf (host, len bytes).
 * pq_profile_reset forgets the records.  Process-wide; calls are serialised.
 */
int pq_profile_enable(int on);
int pq_profile_reset(void);
int pq_profile_query(const char* name, double* total_ms, int* launches);
int pq_profile_names(char* buf, size_t len);

/* ---- Q intake ------------------------------------------------------------ */
/*
 * Distance of Q from the Stiefel manifold, max_ij |(Q^T Q - I_p)_ij|, in
 * float64 (precondition Q in St_{n3,p} of Def. 3.1).  q_dtype is PQ_F32 or
 * PQ_F64.  Writes one double to out_dev.  Workspace: none.
 */
int pq_check_q(const void* Q, int q_dtype, int64_t n3, int64_t p,
               double* out_dev, hipStream_t stream);

/*
 * The same precondition as a device-side status flag.  The products and the
 * tSVDQ do not check Q themselves (a check costs a launch and Q is usually
 * reused across many calls); a caller that wants the check in front of them
 * without a host round trip -- inside a captured graph, or in a loop that
 * polls the flag later -- enqueues this call first on the same stream.
 * Writes the distance max_ij |(Q^T Q - I_p)_ij| to dist_dev (one double, as
 * pq_check_q) and to flag_dev (one int32) 1 when that distance exceeds tol or
 * is not a number, 0 otherwise.  tol >= 0, else PQ_ERR_ARG (NaN included).
 * q_dtype PQ_F32 or PQ_F64.  Workspace: none.
 */
int pq_check_q_flag(const void* Q, int q_dtype, int64_t n3, int64_t p, double tol,
                    double* dist_dev, int* flag_dev, hipStream_t stream);

/*
 * Q (n3 x p, row-major, q_dtype F32 or F64) of one of the fixed transforms
 * that Sec. 5 compares with the data-dependent U3 (pq_u3):
 *   PQ_Q_IDENTITY  the first p columns of I_n3;
 *   PQ_Q_DCT       the first p rows of the orthonormal DCT-II matrix C,
 *                  transposed: Q(t, l) = C(l, t) = w_l cos(pi (2t + 1) l /
 *                  (2 n3)), w_0 = sqrt(1/n3), w_l = sqrt(2/n3) (the real
 *                  stand-in for the t-product's DFT).
 * Both have orthonormal columns.  Returns PQ_ERR_ARG for another kind.
 */
#define PQ_Q_IDENTITY 0
#define PQ_Q_DCT      1
int pq_build_q(int kind, int64_t n3, int64_t p, int q_dtype, void* Q, hipStream_t stream);

/*
 * Re-orthonormalisation of Q (the optional repair of the St_{n3,p}
 * precondition of Def. 3.1): Qout = Q R^{-1} by CholeskyQR2 in float64 --
 * twice G = W^T W, G = R^T R (upper Cholesky factor, positive diagonal),
 * W <- W R^{-1}, starting from W = Q -- so that Qout has orthonormal columns
 * spanning those of Q (for float32 Q to float32 rounding of the float64
 * result).  For full-rank Q this is the Q factor of the thin QR
 * decomposition whose R has a positive diagonal.
 * Q, Qout: n3 x p row-major, q_dtype F32 or F64; Qout may be Q itself.
 * 1 <= p <= min(n3, 128), else PQ_ERR_P / PQ_ERR_UNSUPPORTED.
 * info_dev: one int32 in device memory; 0, or c + 1 when column c (0-based)
 * is numerically dependent on the earlier ones (its pivot is not above
 * 64 eps times its squared norm, in either pass); Qout is then left
 * unwritten.  Accurate for condition numbers of Q up to about 1e7 (the
 * first pass squares it).  Workspace: pq_orthonormalize_q_workspace bytes
 * (n3 p doubles).  One workgroup: an intake step, not a hot loop.
 */
size_t pq_orthonormalize_q_workspace(int64_t n3, int64_t p);
int pq_orthonormalize_q(const void* Q, int q_dtype, int64_t n3, int64_t p, void* Qout, int* info_dev,
                        void* ws, size_t ws_bytes, hipStream_t stream);

/* ---- layouts ---------------------------------------------------------------- */
/*
 * Every tensor argument of this library is in the paper's order (Def. 2.1):
 * element (i, j, t) of an n1 x n2 x n3 tensor at i + n1 (j + n2 t), each
 * frontal slice a contiguous column-major matrix (PQ_LAYOUT_FACE_MAJOR).
 * Data held in numpy / torch C order of an (n1, n2, n3) array, element at
 * t + n3 (j + n2 i) (PQ_LAYOUT_TUBE_MAJOR), is converted with pq_relayout.
 *
 * dst = src in the other layout: src_layout names src's (the one given or
 * PQ_ERR_ARG), dst gets the other.  dtype F32, F64 or BF16 (bits copied
 * unchanged); dst must not overlap src (PQ_ERR_ALIAS).  A transpose of
 * each (i, t) plane through LDS: one read and one write of the tensor.
 * Workspace: none.  PQ_ERR_UNSUPPORTED when ceil(n1 / 32) > 65535.
 */
#define PQ_LAYOUT_FACE_MAJOR 0
#define PQ_LAYOUT_TUBE_MAJOR 1
int pq_relayout(const void* src, int src_layout, void* dst, int dtype, int64_t n1, int64_t n2, int64_t n3,
                hipStream_t stream);

/* ---- mode-3 transforms (Def. 2.2 with M = Q^T and M = Q) ----------------- */
/*
 * Ahat = A x_3 Q^T (the "hat" transform after Def. 3.1; Alg. 4.1 step 2).
 * A: n1 x n2 x n3 face-major, dtype a_dtype (F32, BF16 or F64).
 * Ahat: n1 x n2 x p face-major, float32 (float64 when a_dtype is F64).
 */
int pq_hat(const void* A, int a_dtype, const void* Q, void* Ahat,
           int64_t n1, int64_t n2, int64_t n3, int64_t p, int prec,
           hipStream_t stream);

/*
 * A = Ahat x_3 Q (the return to the spatial domain in Def. 3.1 and
 * Alg. 4.1 step 4).  Ahat: n1 x n2 x p; A: n1 x n2 x n3; both of dtype
 * (F32 or F64).
 */
int pq_unhat(const void* Ahat, const void* Q, void* A, int dtype,
             int64_t n1, int64_t n2, int64_t n3, int64_t p, int prec,
             hipStream_t stream);

/*
 * out = A x_3 Q Q^T, the orthogonal projection of every tube onto range(Q)
 * (the remark after Fig. 3.1).  A: a_dtype (F32, BF16 or F64); out float32
 * (float64 for F64).  With pq_proj_workspace bytes of ws it runs the two
 * streaming transforms (the precision mode applies to the first); with no
 * (or too small a) workspace and p <= 32 on float32/bf16 data it runs a
 * fused single-pass kernel (float32 MFMA, mode ignored); otherwise it
 * returns PQ_ERR_WORKSPACE.
 */
size_t pq_proj_workspace(int64_t n1, int64_t n2, int64_t n3, int64_t p, int a_dtype);
int pq_proj(const void* A, int a_dtype, const void* Q, void* out,
            int64_t n1, int64_t n2, int64_t n3, int64_t p, int prec,
            void* ws, size_t ws_bytes, hipStream_t stream);

/* ---- facewise product (Def. 2.3) ----------------------------------------- */
/*
 * Ch(:,:,l) = Ah(:,:,l) Bh(:,:,l) for l < p.  Ah: n1 x m x p, Bh: m x n2 x p,
 * Ch: n1 x n2 x p, all face-major, dtype F32 or F64.
 */
int pq_facewise(const void* Ah, const void* Bh, void* Ch, int dtype,
                int64_t n1, int64_t m, int64_t n2, int64_t p, int prec,
                hipStream_t stream);

/* ---- the projected product (Def. 3.1) ------------------------------------ */
/*
 * C = A *_Q B = [(A x_3 Q^T) tri (B x_3 Q^T)] x_3 Q.
 * A: n1 x m x n3, B: m x n2 x n3 (ab_dtype F32, BF16 or F64; both the same),
 * C: n1 x n2 x n3 (float32, or float64 for F64).
 * Ahat_out (n1 x m x p) and Bhat_out (m x n2 x p) are optional (NULL = not
 * wanted); when given, the transform-domain inputs are left there for a later
 * pq_qprod_backward.  Workspace: pq_qprod_workspace bytes.
 */
size_t pq_qprod_workspace(int64_t n1, int64_t m, int64_t n2, int64_t n3, int64_t p,
                          int ab_dtype);
int pq_qprod(const void* A, const void* B, int ab_dtype, const void* Q, void* C,
             int64_t n1, int64_t m, int64_t n2, int64_t n3, int64_t p, int prec,
             void* Ahat_out, void* Bhat_out,
             void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * pq_qprod for callers that cannot allocate device memory (code being
 * captured into a graph, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, kernels and results as pq_qprod, with the
 * workspace taken from a fixed array inside the library instead of a ws
 * argument.  The array holds PQ_QPROD_NOALLOC_MAX_BYTES (64 MiB) on every
 * GPU the call runs on, from the first call on that GPU until the process
 * ends; sizes whose workspace (pq_qprod_workspace) exceeds it return
 * PQ_ERR_UNSUPPORTED before anything is enqueued.  The first call on a device
 * looks up the array's address with that device current (the stream must
 * belong to the current device).  Nothing in the array needs to start at
 * zero: each call writes every byte it reads.  Every call on one GPU shares
 * that GPU's array, so calls that may overlap in time on one GPU (different
 * streams, or threads without ordering) race and must be serialised by the
 * caller.  Allocates nothing; never synchronises.
 */
#define PQ_QPROD_NOALLOC_MAX_BYTES ((size_t)64 << 20)
int pq_qprod_noalloc(const void* A, const void* B, int ab_dtype, const void* Q, void* C,
                     int64_t n1, int64_t m, int64_t n2, int64_t n3, int64_t p, int prec,
                     void* Ahat_out, void* Bhat_out, hipStream_t stream);

/*
 * Adjoint of pq_qprod (chain rule through Def. 3.1).  G = dL/dC is
 * n1 x n2 x n3.  With dCh = G x_3 Q^T:
 *   dAh_l = dCh_l Bh_l^T,  dBh_l = Ah_l^T dCh_l,  dA = dAh x_3 Q,
 *   dB = dBh x_3 Q,  dQ = G_(3) Ch_(3)^T + A_(3) dAh_(3)^T + B_(3) dBh_(3)^T.
 * dA (n1 x m x n3), dB (m x n2 x n3), dQ (n3 x p row-major) may each be NULL
 * (= not needed).  Ahat/Bhat may be NULL, in which case they are recomputed.
 * dtype F32 or F64 for every operand.  dQ is reduced in a fixed order, so
 * repeated calls give bit-identical results.  Workspace:
 * pq_qprod_backward_workspace bytes.
 */
size_t pq_qprod_backward_workspace(int64_t n1, int64_t m, int64_t n2, int64_t n3,
                                   int64_t p, int dtype);
int pq_qprod_backward(const void* G, const void* A, const void* B, const void* Q,
                      const void* Ahat, const void* Bhat, int dtype,
                      int64_t n1, int64_t m, int64_t n2, int64_t n3, int64_t p,
                      void* dA, void* dB, void* dQ,
                      void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Adjoint of pq_proj: dA = G x_3 Q Q^T, dQ = G_(3) A_(3)^T Q + A_(3) G_(3)^T Q.
 * dA or dQ may be NULL.  dtype F32 or F64.  Workspace:
 * pq_proj_backward_workspace bytes.
 */
size_t pq_proj_backward_workspace(int64_t n1, int64_t n2, int64_t n3, int64_t p, int dtype);
int pq_proj_backward(const void* G, const void* A, const void* Q, int dtype,
                     int64_t n1, int64_t n2, int64_t n3, int64_t p,
                     void* dA, void* dQ, void* ws, size_t ws_bytes,
                     hipStream_t stream);

/* ---- the data-dependent transform Q = U3 (Thm. 4.3, Cor. 4.1) ------------ */
/*
 * Q = U3(:, 1:p), the leading p left singular vectors of the mode-3
 * unfolding A_(3) (n3 x n1 n2): the choice of Q that Thm. 4.3 shows optimal
 * for the projection error.  A: n1 x n2 x n3 face-major, a_dtype F32 or
 * F64.  Computed as the top-p eigenvectors of the Gram matrix
 * A_(3) A_(3)^T (matrix-core product split over the n1 n2 tubes, slices
 * summed in float64) by one-sided Jacobi (F32 data: float32 Gram-form
 * sweeps to 1e-5, at most 10, on the Gram matrix rounded to float32, then
 * float64 Gram-form sweeps to 1e-10, at most 6; F64 data: float64
 * Gram-form sweeps to 1e-13, at most 16, then float64 vector-form sweeps
 * to 1e-13, at most 6, only if the Gram form stopped short); each column is
 * signed so that its largest-magnitude entry (the first on ties) is
 * positive.
 * Outputs (float32 for F32 data, float64 for F64): Q n3 x p row-major;
 * lambda (may be NULL) p values, the eigenvalues sigma_i(A_(3))^2 as
 * Rayleigh quotients, descending.  info_dev (device int[3], may be NULL) as
 * in pq_tsvdq.  Eigenvectors of (nearly) equal eigenvalues are determined
 * only up to a rotation within their span.  Workspace: pq_u3_workspace.
 */
size_t pq_u3_workspace(int64_t n1, int64_t n2, int64_t n3, int64_t p, int a_dtype);
int pq_u3(const void* A, int a_dtype, int64_t n1, int64_t n2, int64_t n3, int64_t p, void* Q, void* lambda,
          int* info_dev, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---- truncated tSVDQ (Alg. 4.1) ------------------------------------------ */
/*
 * Truncated *_Q-SVD of A (n1 x n2 x n3, a_dtype F32, BF16 or F64) with rank
 * k per face, 1 <= k <= min(n1, n2).
 *   step 2: Ahat = A x_3 Q^T;
 *   step 3: every face Ahat_l ~ Uhat_l diag(s_l) Vhat_l^T, the exact rank-k
 *           truncation (one-sided Jacobi: for float32 data, float32 sweeps
 *           to a coarse threshold and then float64 polishing sweeps on Gram
 *           matrices; for float64 data, float64 sweeps on Gram matrices to
 *           1e-10 and then float64 sweeps on the vectors themselves to tol);
 *   step 4 (optional outputs): Uk = Uhat x_3 Q, the diagonal tubes of
 *           S_k = Shat x_3 Q, Vk = Vhat x_3 Q, and the approximation
 *           A_k = (Uhat tri Shat tri Vhat^T) x_3 Q of Thm. 4.2.
 * Outputs (float32, or float64 for F64):
 *   Uhat n1 x k x p, s k x p (element (j, l) at j + l*k, descending in j),
 *   Vhat n2 x k x p — required;
 *   Uk n1 x k x n3, Sk k x n3 (element (j, t) at j + t*k), Vk n2 x k x n3,
 *   Ak n1 x n2 x n3 — each optional (NULL).
 * Singular vectors of a face whose singular value is zero (rank-deficient
 * faces) are written as zero vectors.  tol is the Jacobi stopping threshold
 * on |a_i . a_j| / (|a_i| |a_j|) of the final (float64) sweeps (<= 0 selects
 * 1e-13; two singular vectors come out coupled by about tol / (2 x the
 * relative gap of their singular values); for F32 and BF16 data the final
 * sweeps work on Gram matrices of the vectors, rotate down to
 * max(tol, 1e-10) and, ahead of the Rayleigh-Ritz step on the leading
 * k + 8 vectors, stop once a sweep started from squared cosines of at most
 * 1e-5, which it squares),
 * max_sweeps caps the sweeps of each phase (<= 0: 10 for float32 data,
 * whose float64 phase takes at most 4 ahead of the Rayleigh-Ritz step; 30
 * for float64 data, whose Gram phase takes at most 16 and whose vector
 * phase at most 6; at most 100).  info_dev (device int[3], may be NULL)
 * receives [0] = the largest number of sweeps any face used (all phases),
 * [1] = the number of faces whose last phase hit max_sweeps before
 * converging (their outputs are still written) and [2] = the sweeps summed
 * over the faces.  Workspace: pq_tsvdq_workspace bytes.
 */
size_t pq_tsvdq_workspace(int64_t n1, int64_t n2, int64_t n3, int64_t p, int64_t k,
                          int a_dtype);
int pq_tsvdq(const void* A, int a_dtype, const void* Q,
             int64_t n1, int64_t n2, int64_t n3, int64_t p, int64_t k, int prec,
             void* Uhat, void* s, void* Vhat,
             void* Uk, void* Sk, void* Vk, void* Ak,
             double tol, int max_sweeps, int* info_dev,
             void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * *_Q-SVDII of A (Sec. 4.1, Alg. 4.2): the facewise SVD of Ahat = A x_3 Q^T
 * as in pq_tsvdq, then one energy threshold over the singular values of all
 * p faces together.  The r p values (r = min(n1, n2)) are put in one
 * descending order (equal values ordered face-major: face l's value j at
 * position j + l r of the flattened list), K is the smallest count whose
 * squared values sum to at least gamma times the sum of all of them
 * (0 < gamma <= 1; K = r p when rounding leaves every partial sum short),
 * and rho_l = how many of face l's values are among the first K (the
 * *_Q-multirank of the approximation, Def. 4.3).  Face l keeps its leading
 * min(rho_l, kmax) singular triplets, 1 <= kmax <= r; pass kmax = r for the
 * untruncated algorithm.  The selection runs in float64 on the GPU.
 * Outputs (float32, or float64 for F64; same layout as pq_tsvdq with k =
 * kmax): Uhat n1 x kmax x p, s kmax x p, Vhat n2 x kmax x p — required; the
 * columns of face l beyond min(rho_l, kmax) are zero.  rho_dev (device
 * int[p], may be NULL) receives rho before the kmax cap.  Ak (n1 x n2 x n3,
 * optional) receives (Uhat tri Shat tri Vhat^T) x_3 Q, whose error obeys
 * Thm. 4.4.  prec, tol, max_sweeps and info_dev as in pq_tsvdq.  Returns
 * PQ_ERR_ARG for gamma outside (0, 1].  Workspace: pq_svdii_workspace bytes.
 */
size_t pq_svdii_workspace(int64_t n1, int64_t n2, int64_t n3, int64_t p, int64_t kmax,
                          int a_dtype);
int pq_svdii(const void* A, int a_dtype, const void* Q,
             int64_t n1, int64_t n2, int64_t n3, int64_t p, double gamma, int64_t kmax,
             int prec, void* Uhat, void* s, void* Vhat, int* rho_dev, void* Ak,
             double tol, int max_sweeps, int* info_dev,
             void* ws, size_t ws_bytes, hipStream_t stream);


/*
 * Adjoint of the truncated tSVDQ viewed as the map (A, Q) -> (A_k, s):
 * A_k = (Uhat tri Shat tri Vhat^T) x_3 Q the approximation of Thm. 4.2 and
 * s (k x p) the kept transform-domain singular values of Alg. 4.1 step 3.
 * Given Gbar = dL/dA_k (n1 x n2 x n3) and/or sbar = dL/ds (k x p, element
 * (j, l) at j + l*k), writes dA = dL/dA (n1 x n2 x n3) and/or dQ = dL/dQ
 * (n3 x p row-major, the Euclidean gradient of Q as a free matrix).  The
 * paper differentiates nothing; this follows from first-order perturbation
 * of each face's SVD: the derivative of the rank-k truncation of a face is
 * that of its spectral projector, which couples each kept value sigma_c
 * with each discarded one sigma_j through 1 / (sigma_c^2 - sigma_j^2), and
 * with the null space through 1 / sigma_c^2.  It exists when every face has
 * sigma_k > sigma_k+1; pairs with |sigma_c^2 - sigma_j^2| <= gap_tol
 * sigma_c^2 have their coupling dropped (gap_tol <= 0 selects 1e-8) and are
 * counted.  Losses of A_k and s are the ones whose gradient is well defined
 * (the factors themselves are fixed only up to signs and rotations).
 * The facewise SVD is recomputed with every singular vector of the shorter
 * side kept.  The coefficients divide by the spectral gaps, so float32
 * arithmetic anywhere on the path (the transforms included) would leave
 * errors of about 1e-7 / (relative gap); float32 data are therefore widened
 * and the whole computation runs in float64 (tol and max_sweeps as for
 * float64 data in pq_tsvdq), the gradients rounded to float32 at the end.
 * a_dtype F32 or F64; Gbar, sbar, dA and dQ have the output type of
 * pq_tsvdq.  Gbar or sbar may
 * be NULL (not both), dA or dQ may be NULL (not both).  info_dev (device
 * int[4], may be NULL): [0..2] as in pq_tsvdq, [3] = the pairs whose
 * coupling was dropped.  Workspace: pq_tsvdq_backward_workspace bytes.
 */
size_t pq_tsvdq_backward_workspace(int64_t n1, int64_t n2, int64_t n3, int64_t p, int64_t k,
                                   int a_dtype);
int pq_tsvdq_backward(const void* A, int a_dtype, const void* Q,
                      int64_t n1, int64_t n2, int64_t n3, int64_t p, int64_t k,
                      const void* Gbar, const void* sbar, void* dA, void* dQ,
                      double gap_tol, double tol, int max_sweeps, int* info_dev,
                      void* ws, size_t ws_bytes, hipStream_t stream);


/* ---- batched form: many uneven instances in one captured graph ----------- */
/*
 * Instance i of a batch (all float32, face-major, device pointers owned by
 * the caller): A (n1 x n2 x n3), Q (n3 x p, row-major, orthonormal columns,
 * p <= n3), and
 *   - the projected product C = A *_Q B (Def. 3.1) with B (n2 x n4 x n3) and
 *     C (n1 x n4 x n3): B and C both given, or both NULL;
 *   - the truncated tSVDQ of A with rank k per face (Alg. 4.1 steps 2-3, the
 *     same outputs and layout as pq_tsvdq): Uhat (n1 x k x p), s (k x p),
 *     Vhat (n2 x k x p) all given, or all NULL; 1 <= k <= min(n1, n2) and
 *     max(n1, n2) <= 512 (PQ_ERR_UNSUPPORTED otherwise).
 * An instance must ask for at least one of the two.
 */
typedef struct {
  int64_t n1, n2, n3, n4, p, k;
  const void* A;
  const void* B;
  const void* Q;
  void* C;
  void* Uhat;
  void* s;
  void* Vhat;
} pq_instance;

typedef struct pq_batch_s* pq_batch;

/* Workspace bytes for a batch of count instances (validates them). */
int pq_batched_workspace(const pq_instance* inst, int count, size_t* bytes);

/*
 * Plans a batch: copies the face table into ws, runs every instance once on
 * `stream` (the outputs of this run are valid; while pq_autotune_enable(1)
 * is in force, launch shapes not yet in the autotuner's table are tuned
 * here), then captures the same launch sequence into a hipGraph on a private
 * stream and instantiates it.  Synchronises `stream`; allocates host memory
 * for the handle only.  The faces' Jacobi sweeps run in two parts on two
 * streams (a stream and events created and destroyed by this call; the
 * graph keeps the two parts as parallel branches).  The transforms, the facewise products and the
 * back-projections of all instances run as grouped launches (one per
 * vector width for the transforms; back-projections of more than 32 faces
 * per instance), and the Jacobi sweeps and finishing steps of all tSVDQ
 * instances as grouped launches over every face at once.  max_sweeps
 * (<= 0: 10) and tol (<= 0: 1e-13) as in pq_tsvdq; info_dev (device int[3],
 * may be NULL) receives the sweep statistics over all faces, as in pq_tsvdq.
 * Every pointer of inst[] and ws is baked into the graph: they must stay
 * valid until pq_batched_destroy, and each run reads and writes them again.
 */
int pq_batched_plan(const pq_instance* inst, int count, int max_sweeps, double tol, int* info_dev,
                    void* ws, size_t ws_bytes, hipStream_t stream, pq_batch* out);

/* Replays the planned batch on `stream` (one hipGraphLaunch; asynchronous). */
int pq_batched_run(pq_batch batch, hipStream_t stream);

/* Frees the graph and the handle (host call; no replay may be in flight). */
int pq_batched_destroy(pq_batch batch);

#ifdef __cplusplus
}
#endif

#endif /* PROJPROD_H */
