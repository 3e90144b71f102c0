// C ABI of the projprod library: argument validation, workspace layout and
// the order of kernel launches for each call.  Every step of every call runs
// in the kernels of this library; nothing here touches tensor data.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/projprod.h"
#include "internal.hpp"

using pq::Gemm;
using pq::Prec;

namespace pq {
namespace {
thread_local int g_last_hip = 0;
}  // namespace
int note_hip_error(hipError_t e) {
  g_last_hip = static_cast<int>(e);
  return PQ_ERR_HIP;
}
}  // namespace pq

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int hip_status(hipError_t e) { return e == hipSuccess ? PQ_OK : pq::note_hip_error(e); }

#define PQ_TRY(expr)                        \
  do {                                      \
    int _rc = hip_status(expr);             \
    if (_rc != PQ_OK) return _rc;           \
  } while (0)

#define PQ_CHECK(expr)                      \
  do {                                      \
    int _rc = (expr);                       \
    if (_rc != PQ_OK) return _rc;           \
  } while (0)

#define PQ_PROF(name, stream) pq::ProfScope _pq_prof_scope(name, stream)

constexpr int64_t kMaxDim = (int64_t)1 << 30;

int check_dims(std::initializer_list<int64_t> dims) {
  for (int64_t d : dims)
    if (d < 1) return PQ_ERR_SHAPE;
  for (int64_t d : dims)
    if (d > kMaxDim) return PQ_ERR_UNSUPPORTED;
  return PQ_OK;
}

int check_p(int64_t n3, int64_t p) { return (p < 1 || p > n3) ? PQ_ERR_P : PQ_OK; }

// elements of an area must stay addressable with 32-bit GEMM sizes
int check_area(int64_t a, int64_t b) { return (a * b >= ((int64_t)1 << 31)) ? PQ_ERR_UNSUPPORTED : PQ_OK; }

bool is_f64(int dtype) { return dtype == PQ_F64; }
size_t elem(int dtype) { return dtype == PQ_F64 ? 8 : 4; }

// tensor input dtype (F32, BF16 or F64)
int check_in_dtype(int dt) { return (dt == PQ_F32 || dt == PQ_F64 || dt == PQ_BF16) ? PQ_OK : PQ_ERR_DTYPE; }
// dtype of arithmetic-only arguments (F32 or F64)
int check_ar_dtype(int dt) { return (dt == PQ_F32 || dt == PQ_F64) ? PQ_OK : PQ_ERR_DTYPE; }

int check_prec(int prec, int dtype) {
  if (prec < PQ_PREC_DEFAULT || prec > PQ_PREC_BF16X6) return PQ_ERR_PREC;
  if (dtype == PQ_F64 && prec != PQ_PREC_DEFAULT) return PQ_ERR_PREC;
  return PQ_OK;
}

int no_alias(const void* out, std::initializer_list<const void*> ins) {
  if (!out) return PQ_OK;
  for (const void* in : ins)
    if (in && in == out) return PQ_ERR_ALIAS;
  return PQ_OK;
}

// Bump allocator over the caller's workspace.
struct Arena {
  char* base;
  size_t cap, used = 0;
  Arena(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
  void* take(size_t bytes) {
    void* p = base ? base + used : nullptr;
    used += align_up(bytes);
    return p;
  }
  bool fits() const { return used <= cap; }
};

constexpr int kDefaultSweeps32 = 10;  // per phase; float32 faces need 6-11 coarse sweeps to 1e-5 (the float64 phase continues from where they stop)
constexpr int kDefaultSweeps64 = 30;
// Jacobi thresholds on |a.c| / (|a||c|): the float32 phase stops at the coarse
// one, the float64 phase polishes to the default final one.
constexpr double kCoarseTol32 = 1e-5;
constexpr int kPolishSweeps = 6;  // float64 phase from the coarse threshold
// the top-block polish ahead of the Ritz step of a plain truncation (1-2
// sweeps from the float32 stop, the rest margin)
constexpr int kTopPolishSweeps = 4;
constexpr double kPolishTol = 1e-13;
// The float64 sweeps of float32 data run on Gram matrices, whose rotation
// angles come from G as updated within a visit: their stopping test is
// floored here (the coupling it leaves, about tol / (2 x relative gap), is
// still far below float32 resolution).
constexpr double kGramTolFloor = 1e-10;
// sweep cap of the Gram-form phase of float64 data (from scratch: 6-12)
constexpr int kGramSweeps64 = 16;
constexpr int kMaxSweepsCap = 100;
// widest Q that pq_orthonormalize_q takes (its Cholesky factor lives in LDS)
constexpr int64_t kOrthoMaxP = 128;
// relative gap |lambda_c - lambda_j| / lambda_c at or under which the adjoint
// of the truncation drops the coupling of a kept and a discarded pair
constexpr double kDefaultGapTol = 1e-8;

// split-K slices of a reduction over K: 512 of K per slice, 256 when the
// product has at most 32 rows (the dQ products, M = p, on the narrow GEMM
// tile: twice the workgroups for the same partial-sum traffic per row)
int ksplit_for(int64_t K, int64_t M = 64) {
  return (int)std::clamp<int64_t>(K / (M <= 32 ? 256 : 512), 1, 1024);
}

// bytes of the transform and Jacobi buffers (take_sweep_bufs takes them in
// this order)
size_t sweep_bytes(bool f64, int64_t N, int64_t p) {
  return align_up(elem(f64 ? PQ_F64 : PQ_F32) * N * p)     // Ah
         + (f64 ? 0 : align_up(4 * N * p))                 // float32 Jacobi vectors
         + align_up(8 * N * p)                             // float64 Jacobi vectors
         + align_up(sizeof(int) * p) * 2                   // sweeps per face, both phases
         + align_up(sizeof(int) * p * kMaxSweepsCap);      // per-sweep rotation flags
}

// ---- dispatch by dtype -------------------------------------------------------
hipError_t do_hat(const void* A, int a_dtype, const void* Q, void* Ah, int64_t N, int n3, int p,
                  Prec prec, hipStream_t s) {
  PQ_PROF("hat", s);
  if (a_dtype == PQ_F64)
    return pq::hat_f64(static_cast<const double*>(A), static_cast<const double*>(Q),
                       static_cast<double*>(Ah), N, n3, p, s);
  return pq::hat_f32(A, a_dtype == PQ_BF16, static_cast<const float*>(Q), static_cast<float*>(Ah), N,
                     n3, p, prec, s);
}

// Precision of the back-projection inside a composite call: the split x3
// mode runs it as x6, which keeps the error of the whole chain (transform,
// facewise step, back-projection) well inside the float32 tolerance.  The
// return transform is bound by its float32 writes: in the split modes the
// autotuner also times its float32 kernels and keeps the faster.
Prec back_prec(Prec p) { return p == Prec::BF16x3 ? Prec::BF16x6 : p; }

hipError_t do_unhat(const void* Ah, const void* Q, void* A, int dtype, int64_t N, int n3, int p,
                    Prec prec, hipStream_t s) {
  PQ_PROF("unhat", s);
  if (dtype == PQ_F64)
    return pq::unhat_f64(static_cast<const double*>(Ah), static_cast<const double*>(Q),
                         static_cast<double*>(A), N, n3, p, s);
  return pq::unhat_f32(static_cast<const float*>(Ah), static_cast<const float*>(Q),
                       static_cast<float*>(A), N, n3, p, prec, s);
}

hipError_t do_gemm(const char* name, const Gemm& g, int dtype, Prec prec, hipStream_t s) {
  PQ_PROF(name, s);
  return dtype == PQ_F64 ? pq::gemm_f64(g, s) : pq::gemm_f32(g, prec, s);
}

hipError_t do_sum(const void* parts, int nparts, int64_t stride, int64_t count, void* out, int dtype,
                  hipStream_t s) {
  PQ_PROF("sum_partials", s);
  if (dtype == PQ_F64)
    return pq::sum_partials_f64(static_cast<const double*>(parts), nparts, stride, count,
                                static_cast<double*>(out), s);
  return pq::sum_partials_f32(static_cast<const float*>(parts), nparts, stride, count,
                              static_cast<float*>(out), s);
}

// Facewise C_l = op(A_l) op(B_l) over p faces with face-major operands.
Gemm face_gemm(bool ta, bool tb, int M, int N, int K, const void* A, int64_t lda, int64_t sA,
               const void* B, int64_t ldb, int64_t sB, void* C, int64_t ldc, int64_t sC, int p) {
  Gemm g{};
  g.ta = ta; g.tb = tb; g.M = M; g.N = N; g.K = K;
  g.A = A; g.lda = lda; g.sA = sA;
  g.B = B; g.ldb = ldb; g.sB = sB;
  g.C = C; g.ldc = ldc; g.sC = sC;
  g.batch = p; g.ksplit = 1; g.sSplit = 0;
  return g;
}

// dQ^T (p x n3, column-major = dQ row-major) partial: Xh_(3) (p x K) times
// Y_(3)^T (K x n3); both operands are row-major (rows x K) in storage.
Gemm dq_gemm(const void* Xh, const void* Y, int p, int n3, int64_t K, void* parts, int ks) {
  Gemm g{};
  g.ta = true; g.tb = false; g.M = p; g.N = n3; g.K = (int)K;
  g.A = Xh; g.lda = K; g.sA = 0;
  g.B = Y; g.ldb = K; g.sB = 0;
  g.C = parts; g.ldc = p; g.sC = 0;
  g.batch = 1; g.ksplit = ks; g.sSplit = (int64_t)p * n3;
  return g;
}

}  // namespace

extern "C" {

int pq_version(void) { return 100; }

const char* pq_status_string(int code) {
  switch (code) {
    case PQ_OK: return "ok";
    case PQ_ERR_NULL: return "a required pointer is NULL";
    case PQ_ERR_SHAPE: return "a size is < 1 or the sizes do not agree";
    case PQ_ERR_P: return "p must satisfy 1 <= p <= n3";
    case PQ_ERR_K: return "k must satisfy 1 <= k <= min(n1, n2)";
    case PQ_ERR_DTYPE: return "unsupported dtype combination";
    case PQ_ERR_PREC: return "unsupported precision mode for this call";
    case PQ_ERR_ALIAS: return "an output pointer equals an input pointer";
    case PQ_ERR_WORKSPACE: return "workspace missing or too small";
    case PQ_ERR_HIP: return "a HIP launch failed";
    case PQ_ERR_UNSUPPORTED: return "size beyond what this build supports";
    case PQ_ERR_ARG: return "argument out of range";
    default: return "unknown status code";
  }
}

int pq_last_hip_error(void) { return pq::g_last_hip; }

int pq_autotune_enable(int on) {
  pq::tune_enable(on != 0);
  return PQ_OK;
}

int pq_autotune_entries(void) { return pq::tune_entries(); }

int pq_autotune_save(const char* path) {
  if (!path) return PQ_ERR_NULL;
  return pq::tune_save(path) ? PQ_OK : PQ_ERR_ARG;
}

int pq_autotune_load(const char* path) {
  if (!path) return PQ_ERR_NULL;
  return pq::tune_load(path) ? PQ_OK : PQ_ERR_ARG;
}

int pq_profile_enable(int on) {
  pq::prof_enable(on != 0);
  return PQ_OK;
}

int pq_profile_reset(void) {
  pq::prof_reset();
  return PQ_OK;
}

int pq_profile_query(const char* name, double* total_ms, int* launches) {
  if (!name || !total_ms || !launches) return PQ_ERR_NULL;
  PQ_TRY(pq::prof_query(name, total_ms, launches));
  return PQ_OK;
}

int pq_profile_names(char* buf, size_t len) {
  if (!buf || len == 0) return PQ_ERR_NULL;
  return pq::prof_names(buf, len) ? PQ_OK : PQ_ERR_ARG;
}

int pq_check_q(const void* Q, int q_dtype, int64_t n3, int64_t p, double* out_dev, hipStream_t stream) {
  if (!Q || !out_dev) return PQ_ERR_NULL;
  PQ_CHECK(check_ar_dtype(q_dtype));
  PQ_CHECK(check_dims({n3}));
  PQ_CHECK(check_p(n3, p));
  PQ_PROF("check_q", stream);
  PQ_TRY(pq::check_q_launch(Q, is_f64(q_dtype), (int)n3, (int)p, out_dev, stream));
  return PQ_OK;
}

int pq_check_q_flag(const void* Q, int q_dtype, int64_t n3, int64_t p, double tol, double* dist_dev, int* flag_dev,
                    hipStream_t stream) {
  if (!Q || !dist_dev || !flag_dev) return PQ_ERR_NULL;
  PQ_CHECK(check_ar_dtype(q_dtype));
  PQ_CHECK(check_dims({n3}));
  PQ_CHECK(check_p(n3, p));
  if (!(tol >= 0.0)) return PQ_ERR_ARG;
  PQ_PROF("check_q", stream);
  PQ_TRY(pq::check_q_launch(Q, is_f64(q_dtype), (int)n3, (int)p, dist_dev, stream));
  PQ_TRY(pq::check_q_flag(dist_dev, tol, flag_dev, stream));
  return PQ_OK;
}

int pq_build_q(int kind, int64_t n3, int64_t p, int q_dtype, void* Q, hipStream_t stream) {
  if (!Q) return PQ_ERR_NULL;
  if (kind != PQ_Q_IDENTITY && kind != PQ_Q_DCT) return PQ_ERR_ARG;
  PQ_CHECK(check_ar_dtype(q_dtype));
  PQ_CHECK(check_dims({n3}));
  PQ_CHECK(check_p(n3, p));
  PQ_PROF("build_q", stream);
  PQ_TRY(pq::build_q(kind, is_f64(q_dtype), (int)n3, (int)p, Q, stream));
  return PQ_OK;
}

int pq_relayout(const void* src, int src_layout, void* dst, int dtype, int64_t n1, int64_t n2, int64_t n3,
                hipStream_t stream) {
  if (!src || !dst) return PQ_ERR_NULL;
  if (src_layout != PQ_LAYOUT_FACE_MAJOR && src_layout != PQ_LAYOUT_TUBE_MAJOR) return PQ_ERR_ARG;
  PQ_CHECK(check_in_dtype(dtype));
  PQ_CHECK(check_dims({n1, n2, n3}));
  PQ_CHECK(no_alias(dst, {src}));
  // grid: (ceil(n3 / 32) n2, ceil(n1 / 32)); the second dimension is limited to 65535
  if ((n1 + 31) / 32 > 65535 || (n3 + 31) / 32 * n2 > INT32_MAX) return PQ_ERR_UNSUPPORTED;
  const int bytes = dtype == PQ_F64 ? 8 : dtype == PQ_BF16 ? 2 : 4;
  PQ_PROF("relayout", stream);
  PQ_TRY(pq::relayout(src, dst, bytes, src_layout == PQ_LAYOUT_TUBE_MAJOR, (int)n1, (int)n2, (int)n3, stream));
  return PQ_OK;
}

size_t pq_orthonormalize_q_workspace(int64_t n3, int64_t p) { return align_up(8 * (size_t)n3 * p); }

int pq_orthonormalize_q(const void* Q, int q_dtype, int64_t n3, int64_t p, void* Qout, int* info_dev, void* ws,
                        size_t ws_bytes, hipStream_t stream) {
  if (!Q || !Qout || !info_dev) return PQ_ERR_NULL;
  PQ_CHECK(check_ar_dtype(q_dtype));
  PQ_CHECK(check_dims({n3}));
  PQ_CHECK(check_p(n3, p));
  if (p > kOrthoMaxP) return PQ_ERR_UNSUPPORTED;
  if (!ws || ws_bytes < pq_orthonormalize_q_workspace(n3, p)) return PQ_ERR_WORKSPACE;
  PQ_PROF("orthonormalize_q", stream);
  PQ_TRY(pq::cholqr2(Q, is_f64(q_dtype), (int)n3, (int)p, static_cast<double*>(ws), Qout, info_dev, stream));
  return PQ_OK;
}

int pq_hat(const void* A, int a_dtype, const void* Q, void* Ahat, int64_t n1, int64_t n2, int64_t n3,
           int64_t p, int prec, hipStream_t stream) {
  if (!A || !Q || !Ahat) return PQ_ERR_NULL;
  PQ_CHECK(check_in_dtype(a_dtype));
  PQ_CHECK(check_dims({n1, n2, n3}));
  PQ_CHECK(check_p(n3, p));
  PQ_CHECK(check_prec(prec, a_dtype));
  PQ_CHECK(no_alias(Ahat, {A, Q}));
  PQ_TRY(do_hat(A, a_dtype, Q, Ahat, n1 * n2, (int)n3, (int)p, (Prec)prec, stream));
  return PQ_OK;
}

int pq_unhat(const void* Ahat, const void* Q, void* A, int dtype, int64_t n1, int64_t n2, int64_t n3,
             int64_t p, int prec, hipStream_t stream) {
  if (!A || !Q || !Ahat) return PQ_ERR_NULL;
  PQ_CHECK(check_ar_dtype(dtype));
  PQ_CHECK(check_dims({n1, n2, n3}));
  PQ_CHECK(check_p(n3, p));
  PQ_CHECK(check_prec(prec, dtype));
  PQ_CHECK(no_alias(A, {Ahat, Q}));
  if (p > 512 && dtype != PQ_F64) return PQ_ERR_UNSUPPORTED;
  PQ_TRY(do_unhat(Ahat, Q, A, dtype, n1 * n2, (int)n3, (int)p, (Prec)prec, stream));
  return PQ_OK;
}

size_t pq_proj_workspace(int64_t n1, int64_t n2, int64_t n3, int64_t p, int a_dtype) {
  (void)n3;
  return align_up((size_t)n1 * n2 * p * elem(a_dtype == PQ_F64 ? PQ_F64 : PQ_F32));
}

int pq_proj(const void* A, int a_dtype, const void* Q, void* out, int64_t n1, int64_t n2, int64_t n3,
            int64_t p, int prec, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!A || !Q || !out) return PQ_ERR_NULL;
  PQ_CHECK(check_in_dtype(a_dtype));
  PQ_CHECK(check_dims({n1, n2, n3}));
  PQ_CHECK(check_p(n3, p));
  PQ_CHECK(check_prec(prec, a_dtype));
  PQ_CHECK(no_alias(out, {A, Q}));
  const int64_t N = n1 * n2;
  const size_t need = pq_proj_workspace(n1, n2, n3, p, a_dtype);
  // with the workspace: the two streaming transforms (faster than the fused
  // kernel on gfx950, and they honour the precision mode); without it: the
  // fused kernel (p <= 32)
  if (!ws || ws_bytes < need) {
    if (a_dtype != PQ_F64 && pq::proj_fused_ok((int)n3, (int)p)) {
      PQ_PROF("proj_fused", stream);
      PQ_TRY(pq::proj_fused_f32(A, a_dtype == PQ_BF16, static_cast<const float*>(Q),
                                static_cast<float*>(out), N, (int)n3, (int)p, (Prec)prec, stream));
      return PQ_OK;
    }
    return PQ_ERR_WORKSPACE;
  }
  if (p > 512 && a_dtype != PQ_F64) return PQ_ERR_UNSUPPORTED;
  const int dt = a_dtype == PQ_F64 ? PQ_F64 : PQ_F32;
  PQ_TRY(do_hat(A, a_dtype, Q, ws, N, (int)n3, (int)p, (Prec)prec, stream));
  PQ_TRY(do_unhat(ws, Q, out, dt, N, (int)n3, (int)p, back_prec((Prec)prec), stream));
  return PQ_OK;
}

int pq_facewise(const void* Ah, const void* Bh, void* Ch, int dtype, int64_t n1, int64_t m, int64_t n2,
                int64_t p, int prec, hipStream_t stream) {
  if (!Ah || !Bh || !Ch) return PQ_ERR_NULL;
  PQ_CHECK(check_ar_dtype(dtype));
  PQ_CHECK(check_dims({n1, m, n2, p}));
  PQ_CHECK(check_prec(prec, dtype));
  PQ_CHECK(no_alias(Ch, {Ah, Bh}));
  Gemm g = face_gemm(false, false, (int)n1, (int)n2, (int)m, Ah, n1, n1 * m, Bh, m, m * n2, Ch, n1,
                     n1 * n2, (int)p);
  PQ_TRY(do_gemm("facewise_gemm", g, dtype, (Prec)prec, stream));
  return PQ_OK;
}

size_t pq_qprod_workspace(int64_t n1, int64_t m, int64_t n2, int64_t n3, int64_t p, int ab_dtype) {
  (void)n3;
  const size_t e = elem(ab_dtype);
  return align_up(e * n1 * m * p) + align_up(e * m * n2 * p) + align_up(e * n1 * n2 * p);
}

int pq_qprod(const void* A, const void* B, int ab_dtype, const void* Q, void* C, int64_t n1, int64_t m,
             int64_t n2, int64_t n3, int64_t p, int prec, void* Ahat_out, void* Bhat_out, void* ws,
             size_t ws_bytes, hipStream_t stream) {
  if (!A || !B || !Q || !C) return PQ_ERR_NULL;
  PQ_CHECK(check_in_dtype(ab_dtype));
  PQ_CHECK(check_dims({n1, m, n2, n3}));
  PQ_CHECK(check_p(n3, p));
  PQ_CHECK(check_prec(prec, ab_dtype));
  PQ_CHECK(no_alias(C, {A, B, Q, Ahat_out, Bhat_out}));
  PQ_CHECK(no_alias(Ahat_out, {A, B, Q}));
  PQ_CHECK(no_alias(Bhat_out, {A, B, Q, Ahat_out}));
  if (p > 512 && ab_dtype != PQ_F64) return PQ_ERR_UNSUPPORTED;
  if (!ws || ws_bytes < pq_qprod_workspace(n1, m, n2, n3, p, ab_dtype)) return PQ_ERR_WORKSPACE;
  const int dt = ab_dtype == PQ_F64 ? PQ_F64 : PQ_F32;
  const size_t e = elem(dt);
  Arena ar(ws, ws_bytes);
  void* Ah = ar.take(e * n1 * m * p);
  void* Bh = ar.take(e * m * n2 * p);
  void* Ch = ar.take(e * n1 * n2 * p);
  if (Ahat_out) Ah = Ahat_out;
  if (Bhat_out) Bh = Bhat_out;
  const Prec pr = (Prec)prec;
  PQ_TRY(do_hat(A, ab_dtype, Q, Ah, n1 * m, (int)n3, (int)p, pr, stream));
  PQ_TRY(do_hat(B, ab_dtype, Q, Bh, m * n2, (int)n3, (int)p, pr, stream));
  Gemm g = face_gemm(false, false, (int)n1, (int)n2, (int)m, Ah, n1, n1 * m, Bh, m, m * n2, Ch, n1,
                     n1 * n2, (int)p);
  PQ_TRY(do_gemm("facewise_gemm", g, dt, pr, stream));
  PQ_TRY(do_unhat(Ch, Q, C, dt, n1 * n2, (int)n3, (int)p, back_prec(pr), stream));
  return PQ_OK;
}

size_t pq_qprod_backward_workspace(int64_t n1, int64_t m, int64_t n2, int64_t n3, int64_t p, int dtype) {
  const size_t e = elem(dtype);
  size_t bytes = align_up(e * n1 * m * p) + align_up(e * m * n2 * p)   // Ah, Bh
                 + align_up(e * n1 * n2 * p) + align_up(e * n1 * n2 * p)  // Ch, dCh
                 + align_up(e * n1 * m * p) + align_up(e * m * n2 * p);   // dAh, dBh
  const int parts = ksplit_for(n1 * n2, p) + ksplit_for(n1 * m, p) + ksplit_for(m * n2, p);
  bytes += align_up(e * (size_t)parts * p * n3);
  return bytes;
}

int pq_qprod_backward(const void* G, const void* A, const void* B, const void* Q, const void* Ahat,
                      const void* Bhat, int dtype, int64_t n1, int64_t m, int64_t n2, int64_t n3,
                      int64_t p, void* dA, void* dB, void* dQ, void* ws, size_t ws_bytes,
                      hipStream_t stream) {
  if (!G || !Q) return PQ_ERR_NULL;
  if ((!Ahat || dQ) && !A) return PQ_ERR_NULL;
  if ((!Bhat || dQ) && !B) return PQ_ERR_NULL;
  PQ_CHECK(check_ar_dtype(dtype));
  PQ_CHECK(check_dims({n1, m, n2, n3}));
  PQ_CHECK(check_p(n3, p));
  PQ_CHECK(check_area(n1, n2));
  PQ_CHECK(check_area(n1, m));
  PQ_CHECK(check_area(m, n2));
  for (const void* o : {dA, dB, dQ}) PQ_CHECK(no_alias(o, {G, A, B, Q, Ahat, Bhat}));
  if ((dA && (dA == dB || dA == dQ)) || (dB && dB == dQ)) return PQ_ERR_ALIAS;
  if (p > 512 && dtype != PQ_F64) return PQ_ERR_UNSUPPORTED;
  if (!ws || ws_bytes < pq_qprod_backward_workspace(n1, m, n2, n3, p, dtype)) return PQ_ERR_WORKSPACE;
  if (!dA && !dB && !dQ) return PQ_OK;
  const size_t e = elem(dtype);
  Arena ar(ws, ws_bytes);
  void* Ah_ws = ar.take(e * n1 * m * p);
  void* Bh_ws = ar.take(e * m * n2 * p);
  void* Ch = ar.take(e * n1 * n2 * p);
  void* dCh = ar.take(e * n1 * n2 * p);
  void* dAh = ar.take(e * n1 * m * p);
  void* dBh = ar.take(e * m * n2 * p);
  const int ks1 = ksplit_for(n1 * n2, p), ks2 = ksplit_for(n1 * m, p), ks3 = ksplit_for(m * n2, p);
  void* parts = ar.take(e * (size_t)(ks1 + ks2 + ks3) * p * n3);
  const Prec pr = Prec::Default;
  const void* Ah = Ahat;
  const void* Bh = Bhat;
  if (!Ah) {
    PQ_TRY(do_hat(A, dtype, Q, Ah_ws, n1 * m, (int)n3, (int)p, pr, stream));
    Ah = Ah_ws;
  }
  if (!Bh) {
    PQ_TRY(do_hat(B, dtype, Q, Bh_ws, m * n2, (int)n3, (int)p, pr, stream));
    Bh = Bh_ws;
  }
  // dCh = G x_3 Q^T
  PQ_TRY(do_hat(G, dtype, Q, dCh, n1 * n2, (int)n3, (int)p, pr, stream));
  const bool need_dAh = dA || dQ, need_dBh = dB || dQ;
  if (need_dAh) {  // dAh_l = dCh_l Bh_l^T   (n1 x m)
    Gemm g = face_gemm(false, true, (int)n1, (int)m, (int)n2, dCh, n1, n1 * n2, Bh, m, m * n2, dAh, n1,
                       n1 * m, (int)p);
    PQ_TRY(do_gemm("adjoint_gemm", g, dtype, pr, stream));
  }
  if (need_dBh) {  // dBh_l = Ah_l^T dCh_l   (m x n2)
    Gemm g = face_gemm(true, false, (int)m, (int)n2, (int)n1, Ah, n1, n1 * m, dCh, n1, n1 * n2, dBh, m,
                       m * n2, (int)p);
    PQ_TRY(do_gemm("adjoint_gemm", g, dtype, pr, stream));
  }
  if (dA) PQ_TRY(do_unhat(dAh, Q, dA, dtype, n1 * m, (int)n3, (int)p, pr, stream));
  if (dB) PQ_TRY(do_unhat(dBh, Q, dB, dtype, m * n2, (int)n3, (int)p, pr, stream));
  if (dQ) {
    Gemm fw = face_gemm(false, false, (int)n1, (int)n2, (int)m, Ah, n1, n1 * m, Bh, m, m * n2, Ch, n1,
                        n1 * n2, (int)p);
    PQ_TRY(do_gemm("facewise_gemm", fw, dtype, pr, stream));
    char* pb = static_cast<char*>(parts);
    const size_t slab = e * (size_t)p * n3;
    PQ_TRY(do_gemm("dq_gemm", dq_gemm(Ch, G, (int)p, (int)n3, n1 * n2, pb, ks1), dtype, pr, stream));
    PQ_TRY(do_gemm("dq_gemm", dq_gemm(dAh, A, (int)p, (int)n3, n1 * m, pb + slab * ks1, ks2), dtype, pr, stream));
    PQ_TRY(do_gemm("dq_gemm", dq_gemm(dBh, B, (int)p, (int)n3, m * n2, pb + slab * (ks1 + ks2), ks3), dtype, pr,
                   stream));
    PQ_TRY(do_sum(parts, ks1 + ks2 + ks3, p * n3, p * n3, dQ, dtype, stream));
  }
  return PQ_OK;
}

size_t pq_proj_backward_workspace(int64_t n1, int64_t n2, int64_t n3, int64_t p, int dtype) {
  const size_t e = elem(dtype);
  const int ks = ksplit_for(n1 * n2, p);
  return align_up(e * n1 * n2 * p) * 2 + align_up(e * (size_t)2 * ks * p * n3);
}

int pq_proj_backward(const void* G, const void* A, const void* Q, int dtype, int64_t n1, int64_t n2,
                     int64_t n3, int64_t p, void* dA, void* dQ, void* ws, size_t ws_bytes,
                     hipStream_t stream) {
  if (!G || !Q || (dQ && !A)) return PQ_ERR_NULL;
  PQ_CHECK(check_ar_dtype(dtype));
  PQ_CHECK(check_dims({n1, n2, n3}));
  PQ_CHECK(check_p(n3, p));
  PQ_CHECK(check_area(n1, n2));
  for (const void* o : {dA, dQ}) PQ_CHECK(no_alias(o, {G, A, Q}));
  if (dA && dA == dQ) return PQ_ERR_ALIAS;
  if (p > 512 && dtype != PQ_F64) return PQ_ERR_UNSUPPORTED;
  if (!ws || ws_bytes < pq_proj_backward_workspace(n1, n2, n3, p, dtype)) return PQ_ERR_WORKSPACE;
  const size_t e = elem(dtype);
  const int64_t N = n1 * n2;
  Arena ar(ws, ws_bytes);
  void* Ah = ar.take(e * N * p);
  void* Gh = ar.take(e * N * p);
  const int ks = ksplit_for(N, p);
  void* parts = ar.take(e * (size_t)2 * ks * p * n3);
  const Prec pr = Prec::Default;
  PQ_TRY(do_hat(G, dtype, Q, Gh, N, (int)n3, (int)p, pr, stream));
  if (dA) PQ_TRY(do_unhat(Gh, Q, dA, dtype, N, (int)n3, (int)p, pr, stream));
  if (dQ) {
    PQ_TRY(do_hat(A, dtype, Q, Ah, N, (int)n3, (int)p, pr, stream));
    char* pb = static_cast<char*>(parts);
    const size_t slab = e * (size_t)p * n3;
    // dQ^T = Ah_(3) G_(3)^T + Gh_(3) A_(3)^T
    PQ_TRY(do_gemm("dq_gemm", dq_gemm(Ah, G, (int)p, (int)n3, N, pb, ks), dtype, pr, stream));
    PQ_TRY(do_gemm("dq_gemm", dq_gemm(Gh, A, (int)p, (int)n3, N, pb + slab * ks, ks), dtype, pr, stream));
    PQ_TRY(do_sum(parts, 2 * ks, p * n3, p * n3, dQ, dtype, stream));
  }
  return PQ_OK;
}

size_t pq_u3_workspace(int64_t n1, int64_t n2, int64_t n3, int64_t p, int a_dtype) {
  const int64_t N = n1 * n2;
  const int ks = ksplit_for(N);
  const size_t e = elem(a_dtype == PQ_F64 ? PQ_F64 : PQ_F32);
  return align_up(e * (size_t)ks * n3 * n3)   // split-K slices of the Gram matrix
         + align_up(8 * (size_t)n3 * n3) * 2  // Gram matrix (float64) and the Jacobi copy
         + align_up(sizeof(int) * 2)          // sweeps used
         + align_up(sizeof(int) * kMaxSweepsCap)
         + align_up(8 * (size_t)n3 * p)       // the p leading eigenvectors
         + align_up(8 * (size_t)n3);          // norms of the converged columns
}

int pq_u3(const void* A, int a_dtype, int64_t n1, int64_t n2, int64_t n3, int64_t p, void* Q, void* lambda,
          int* info_dev, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!A || !Q) return PQ_ERR_NULL;
  if (a_dtype != PQ_F32 && a_dtype != PQ_F64) return PQ_ERR_DTYPE;
  PQ_CHECK(check_dims({n1, n2, n3}));
  PQ_CHECK(check_p(n3, p));
  PQ_CHECK(check_area(n1, n2));  // the Gram product's depth is n1 n2
  if (n3 > 4096) return PQ_ERR_UNSUPPORTED;
  for (const void* o : {Q, lambda})
    if (o && o == A) return PQ_ERR_ALIAS;
  if (lambda && lambda == Q) return PQ_ERR_ALIAS;
  if (!ws || ws_bytes < pq_u3_workspace(n1, n2, n3, p, a_dtype)) return PQ_ERR_WORKSPACE;
  const bool f64 = a_dtype == PQ_F64;
  const int64_t N = n1 * n2;
  const int ks = ksplit_for(N);
  const int in3 = (int)n3, ip = (int)p;
  const size_t e = elem(f64 ? PQ_F64 : PQ_F32);
  Arena ar(ws, ws_bytes);
  void* parts = ar.take(e * (size_t)ks * n3 * n3);
  double* G = static_cast<double*>(ar.take(8 * (size_t)n3 * n3));
  double* W = static_cast<double*>(ar.take(8 * (size_t)n3 * n3));
  int* used = static_cast<int*>(ar.take(sizeof(int) * 2));
  int* flags = static_cast<int*>(ar.take(sizeof(int) * kMaxSweepsCap));
  double* F = static_cast<double*>(ar.take(8 * (size_t)n3 * p));
  double* sig = static_cast<double*>(ar.take(8 * (size_t)n3));
  // Gram matrix A_(3) A_(3)^T: split-K over the n1 n2 tubes, slices summed in
  // a fixed order in float64
  PQ_TRY(do_gemm("u3_gram", dq_gemm(A, A, in3, in3, N, parts, ks), f64 ? PQ_F64 : PQ_F32, Prec::Default, stream));
  {
    PQ_PROF("sum_partials", stream);
    if (f64) PQ_TRY(pq::sum_partials_f64(static_cast<const double*>(parts), ks, n3 * n3, n3 * n3, G, stream));
    else PQ_TRY(pq::sum_to_f64(static_cast<const float*>(parts), ks, n3 * n3, n3 * n3, G, stream));
  }
  // its eigenvectors: one-sided Jacobi on the symmetric positive semidefinite
  // G (converged columns are lambda_j u_j).  float32 data: the sweep phases
  // of the float32 tSVDQ, float32 sweeps to the coarse threshold on G rounded
  // to float32 (no coarser than the float32 products that formed it), then
  // float64 Gram-form sweeps to 1e-10; float64 data: the phases of the
  // float64 tSVDQ, float64 Gram-form sweeps to 1e-13, then vector-form sweeps
  // (angles from the vectors themselves) only if the Gram form stopped short.
  if (!f64) {
    float* W32 = static_cast<float*>(parts);  // the slices are summed: their space is free
    PQ_TRY(pq::grad_narrow(G, W32, n3 * n3, stream));
    PQ_TRY(pq::jacobi_sweeps_f32(W32, 1, in3, in3, kDefaultSweeps32, kCoarseTol32, 0.0, used, flags, stream));
    {
      PQ_PROF("jacobi_widen", stream);
      PQ_TRY(pq::jacobi_widen(W32, W, n3 * n3, stream));
    }
    PQ_TRY(pq::jacobi_gram_sweeps_f64(W, 1, in3, in3, kPolishSweeps, kGramTolFloor, 0.0, 0, used + 1, flags,
                                      stream));
  } else {
    PQ_TRY(hipMemcpyAsync(W, G, 8 * (size_t)n3 * n3, hipMemcpyDeviceToDevice, stream));
    PQ_TRY(pq::jacobi_gram_sweeps_f64(W, 1, in3, in3, kGramSweeps64, kPolishTol, 0.0, 0, used, flags, stream));
    PQ_TRY(pq::jacobi_sweeps_f64(W, 1, in3, in3, kPolishSweeps, kPolishTol, used + 1, flags, used, kGramSweeps64,
                                 stream));
  }
  {
    PQ_PROF("jacobi_finalize", stream);
    PQ_TRY(pq::jacobi_norms_f64(W, 1, in3, in3, sig, nullptr, stream));
    PQ_TRY(pq::jacobi_finalize_f64(W, sig, 1, in3, in3, ip, nullptr, 0, F, nullptr, stream));
  }
  {
    PQ_PROF("u3_finish", stream);
    PQ_TRY(pq::u3_finish(F, G, in3, ip, Q, lambda, f64, stream));
  }
  if (info_dev) {
    if (f64) PQ_TRY(pq::jacobi_info(used, used + 1, 1, kGramSweeps64, kPolishSweeps, info_dev, stream));
    else PQ_TRY(pq::jacobi_info(used, used + 1, 1, kDefaultSweeps32, kPolishSweeps, info_dev, stream));
  }
  return PQ_OK;
}

size_t pq_tsvdq_workspace(int64_t n1, int64_t n2, int64_t n3, int64_t p, int64_t k, int a_dtype) {
  (void)n3;
  const bool f64 = a_dtype == PQ_F64;
  const size_t e = elem(f64 ? PQ_F64 : PQ_F32);
  const int64_t mx = std::max(n1, n2), mn = std::min(n1, n2);
  const int64_t kr = pq::ritz_cols(k, mn);
  return sweep_bytes(f64, n1 * n2, p)
         + align_up(8 * mn * p)                           // every singular value
         + align_up(sizeof(int) * mn * p)                 // top-block positions
         + align_up(8 * mx * kr * p)                      // top-kr Jacobi vectors
         + align_up(8 * mn * kr * p)                      // other side (float64)
         + align_up(e * mn * k * p)                       // other side, ordered, unscaled
         + align_up(e * n1 * n2 * p);                     // transform-domain A_k
}

size_t pq_svdii_workspace(int64_t n1, int64_t n2, int64_t n3, int64_t p, int64_t kmax, int a_dtype) {
  const int64_t mn = std::min(n1, n2);
  return pq_tsvdq_workspace(n1, n2, n3, p, kmax, a_dtype)
         + align_up(sizeof(int) * mn * p)  // global ranks
         + align_up(8 * mn * p)            // energies in descending order
         + align_up(sizeof(int) * p);      // multirank when the caller keeps none
}

}  // extern "C"

namespace {

// Transform and Jacobi buffers: Ah, the float32 working copy (float32 data),
// the float64 vectors, sweep counters of both phases and rotation flags.
struct SweepBufs {
  void* Ah;
  float* W32;
  double* W64;
  int* used1;
  int* used2;
  int* flags;
};

SweepBufs take_sweep_bufs(Arena& ar, bool f64, int64_t N, int64_t p) {
  SweepBufs b;
  b.Ah = ar.take(elem(f64 ? PQ_F64 : PQ_F32) * N * p);
  b.W32 = f64 ? nullptr : static_cast<float*>(ar.take(4 * N * p));
  b.W64 = static_cast<double*>(ar.take(8 * N * p));
  b.used1 = static_cast<int*>(ar.take(sizeof(int) * p));
  b.used2 = static_cast<int*>(ar.take(sizeof(int) * p));
  b.flags = static_cast<int*>(ar.take(sizeof(int) * p * kMaxSweepsCap));
  return b;
}

// Step 2 of Alg. 4.1 and the Jacobi sweeps of step 3: b.Ah = A x_3 Q^T and
// b.W64 = the converged vectors of every face (the shorter side's: columns
// of each face when n1 >= n2, rows otherwise); sweep statistics to info_dev.
// wide: float32 data (a_dtype PQ_F32) factorised in float64 as if widened
// (Q is then float64, and so is the transform)
int converge(const void* A, int a_dtype, const void* Q, int64_t n1, int64_t n2, int64_t n3, int64_t p, Prec pr,
             double tol, int max_sweeps, const SweepBufs& b, int* info_dev, hipStream_t stream,
             bool wide = false, int ntop = 0, double* top_nrm = nullptr, int* top_pos = nullptr) {
  const bool f64 = a_dtype == PQ_F64 || wide;
  const int64_t N = n1 * n2;
  const int in1 = (int)n1, in2 = (int)n2, ip = (int)p;
  const int nv = (int)std::min(n1, n2), L = (int)std::max(n1, n2);
  if (wide) {
    PQ_PROF("hat", stream);
    PQ_TRY(pq::hat_f64_wide(static_cast<const float*>(A), static_cast<const double*>(Q),
                            static_cast<double*>(b.Ah), N, (int)n3, ip, stream));
  } else {
    PQ_TRY(do_hat(A, a_dtype, Q, b.Ah, N, (int)n3, ip, pr, stream));
  }
  if (f64) {
    PQ_PROF("jacobi_prep", stream);
    PQ_TRY(pq::jacobi_prep_f64(static_cast<const double*>(b.Ah), b.W64, in1, in2, ip, stream));
  } else {
    {
      PQ_PROF("jacobi_prep", stream);
      PQ_TRY(pq::jacobi_prep_f32(static_cast<const float*>(b.Ah), b.W32, in1, in2, ip, stream));
    }
    // float32 sweeps down to a coarse threshold (each launch profiled inside)
    PQ_TRY(pq::jacobi_sweeps_f32(b.W32, ip, nv, L, max_sweeps, kCoarseTol32,
                                 ntop > 0 ? pq::kCoarseStop32 : kCoarseTol32, b.used1, b.flags, stream));
    PQ_PROF("jacobi_widen", stream);
    if (ntop > 0)
      PQ_TRY(pq::jacobi_widen_top(b.W32, b.W64, nullptr, ip, nv, L, nv, 16 * ntop, top_nrm, top_pos, stream));
    else PQ_TRY(pq::jacobi_widen(b.W32, b.W64, N * p, stream));
  }
  // float64 sweeps to tol (each launch profiled inside)
  // float64 data: Gram-form sweeps to tol (the stopping test is evaluated on
  // G freshly formed from the vectors, as accurate as their dot products),
  // then vector-form sweeps (rotation angles from the vectors themselves) to
  // tol for the faces the Gram form left unconverged; float32 data:
  // Gram-form float64 sweeps to max(tol, 1e-10)
  const int max1 = f64 ? std::min(max_sweeps, kGramSweeps64) : max_sweeps;
  const int max2 = std::min(max_sweeps, (!f64 && ntop > 0) ? kTopPolishSweeps : kPolishSweeps);
  if (f64) {
    PQ_TRY(pq::jacobi_gram_sweeps_f64(b.W64, ip, nv, L, max1, tol, 0.0, 0, b.used1, b.flags, stream));
    PQ_TRY(pq::jacobi_sweeps_f64(b.W64, ip, nv, L, max2, tol, b.used2, b.flags, b.used1, max1, stream));
  } else {
    // rotations down to max(tol, 1e-10); the top-block polish ahead of the
    // Ritz step stops at kPolishStop32, a polish of every pair (the SVDII
    // selection ranks the column norms themselves) at that same floor
    const double ptol = std::max(tol, kGramTolFloor);
    PQ_TRY(pq::jacobi_gram_sweeps_f64(b.W64, ip, nv, L, max2, ptol, ntop > 0 ? pq::kPolishStop32 : ptol, ntop,
                                      b.used2, b.flags, stream));
  }
  if (info_dev) PQ_TRY(pq::jacobi_info(b.used1, b.used2, ip, max1, max2, info_dev, stream));
  return PQ_OK;
}

// Steps 2-3 of Alg. 4.1 (gamma <= 0: rank k on every face) or of Alg. 4.2
// (gamma in (0, 1]: per-face ranks rho from one energy threshold over every
// face, each face keeping min(rho_i, k) columns, zero columns after), then
// the approximation of Thm. 4.2 when Ak is given.  Arguments are validated
// by the callers; the workspace is carved from ar.
int facewise_svd(const void* A, int a_dtype, const void* Q, int64_t n1, int64_t n2, int64_t n3, int64_t p,
                 int64_t k, Prec pr, double gamma, int* rho, void* Uhat, void* s, void* Vhat, void* Ak,
                 double tol, int max_sweeps, int* info_dev, Arena& ar, hipStream_t stream) {
  const bool f64 = a_dtype == PQ_F64;
  const int dt = f64 ? PQ_F64 : PQ_F32;
  const size_t e = elem(dt);
  const int64_t N = n1 * n2;
  const int64_t mx = std::max(n1, n2), mn = std::min(n1, n2);
  const SweepBufs b = take_sweep_bufs(ar, f64, N, p);
  const int kr = pq::ritz_cols(k, mn);  // columns of the Rayleigh-Ritz step
  double* sig = static_cast<double*>(ar.take(8 * mn * p));
  int* tpos = static_cast<int*>(ar.take(sizeof(int) * mn * p));
  double* Ft = static_cast<double*>(ar.take(8 * mx * kr * p));
  double* Y = static_cast<double*>(ar.take(8 * mn * kr * p));
  void* Ys = ar.take(e * mn * k * p);
  void* Akh = ar.take(e * N * p);
  const bool select = gamma > 0.0;
  int* rank = select ? static_cast<int*>(ar.take(sizeof(int) * mn * p)) : nullptr;
  double* e2 = select ? static_cast<double*>(ar.take(8 * mn * p)) : nullptr;
  int* rho_ws = select ? static_cast<int*>(ar.take(sizeof(int) * p)) : nullptr;
  if (select && !rho) rho = rho_ws;
  const int in1 = (int)n1, in2 = (int)n2, ip = (int)p, ik = (int)k;
  const void* Ah = b.Ah;
  double* W64 = b.W64;
  // float32 data of a plain truncation: the float64 polish only separates
  // the leading blocks, which hold the Ritz step's kr columns; the SVDII
  // selection ranks every singular value and keeps every pair
  const int ntop = select ? 0 : pq::top_blocks(kr);
  PQ_CHECK(converge(A, a_dtype, Q, n1, n2, n3, p, pr, tol, max_sweeps, b, info_dev, stream, false, ntop, sig,
                    tpos));
  const bool cols = n1 >= n2;
  const int nv = (int)mn, L = (int)mx;
  void* Fo = cols ? Uhat : Vhat;     // side given by the Jacobi vectors
  void* Other = cols ? Vhat : Uhat;  // side given by one more product
  {
    PQ_PROF("jacobi_norms", stream);
    PQ_TRY(pq::jacobi_norms_f64(W64, ip, nv, L, sig, rank, stream));
  }
  if (select) {
    PQ_PROF("svdii_select", stream);
    PQ_TRY(pq::jacobi_select(sig, ip, nv, gamma, rank, e2, rho, stream));
  }
  {
    PQ_PROF("jacobi_finalize", stream);
    PQ_TRY(pq::jacobi_finalize_f64(W64, sig, ip, nv, L, kr, select ? rho : nullptr, pq::kRitzExtra, Ft, nullptr,
                                   stream));
  }
  {  // Y = Ah_l^T Ft_l (n2 x kr) or Ah_l Ft_l (n1 x kr), float64 accumulation
    PQ_PROF("factor_product", stream);
    if (f64) PQ_TRY(pq::jacobi_factor_f64(static_cast<const double*>(Ah), Ft, Y, in1, in2, kr, ip, cols, stream));
    else PQ_TRY(pq::jacobi_factor_f32(static_cast<const float*>(Ah), Ft, Y, in1, in2, kr, ip, cols, stream));
  }
  {  // Rayleigh-Ritz on the kr columns, the leading k kept
    PQ_PROF("jacobi_refine", stream);
    if (f64)
      PQ_TRY(pq::jacobi_refine_f64(Y, Ft, nv, L, kr, ik, ip, select ? rho : nullptr, pq::kRitzExtra, tol,
                                   static_cast<double*>(s), static_cast<double*>(Other), static_cast<double*>(Fo),
                                   static_cast<double*>(Ys), stream));
    else
      PQ_TRY(pq::jacobi_refine_f32(Y, Ft, nv, L, kr, ik, ip, select ? rho : nullptr, pq::kRitzExtra, tol,
                                   static_cast<float*>(s), static_cast<float*>(Other), static_cast<float*>(Fo),
                                   static_cast<float*>(Ys), stream));
  }
  // step 4 and the approximation of Thm. 4.2 (zero columns add nothing)
  if (Ak) {
    // Akh_l = Uhat_l Ys_l^T (cols) or Ys_l Vhat_l^T (rows): both Uhat S Vhat^T
    Gemm g = cols ? face_gemm(false, true, in1, in2, ik, Fo, n1, n1 * k, Ys, n2, n2 * k, Akh, n1, N, ip)
                  : face_gemm(false, true, in1, in2, ik, Ys, n1, n1 * k, Fo, n2, n2 * k, Akh, n1, N, ip);
    PQ_TRY(do_gemm("approx_gemm", g, dt, Prec::Default, stream));
    PQ_TRY(do_unhat(Akh, Q, Ak, dt, N, (int)n3, ip, back_prec(pr), stream));
  }
  return PQ_OK;
}

// argument checks shared by pq_tsvdq and pq_svdii
int check_svd_args(const void* A, int a_dtype, const void* Q, int64_t n1, int64_t n2, int64_t n3, int64_t p,
                   int64_t k, int prec, std::initializer_list<const void*> outs) {
  PQ_CHECK(check_in_dtype(a_dtype));
  PQ_CHECK(check_dims({n1, n2, n3}));
  PQ_CHECK(check_p(n3, p));
  PQ_CHECK(check_area(n1, n2));
  if (k < 1 || k > std::min(n1, n2)) return PQ_ERR_K;
  PQ_CHECK(check_prec(prec, a_dtype));
  for (const void* o : outs)
    if (o && (o == A || o == Q)) return PQ_ERR_ALIAS;
  if (std::min(n1, n2) > 4096) return PQ_ERR_UNSUPPORTED;
  if (p > 512 && a_dtype != PQ_F64) return PQ_ERR_UNSUPPORTED;
  return PQ_OK;
}

int sweep_defaults(int a_dtype, double& tol, int& max_sweeps) {
  if (max_sweeps <= 0) max_sweeps = a_dtype == PQ_F64 ? kDefaultSweeps64 : kDefaultSweeps32;
  if (max_sweeps > kMaxSweepsCap) return PQ_ERR_ARG;
  if (tol <= 0.0) tol = kPolishTol;
  return PQ_OK;
}

}  // namespace

extern "C" {

int pq_tsvdq(const void* A, int a_dtype, const void* Q, int64_t n1, int64_t n2, int64_t n3, int64_t p,
             int64_t k, int prec, void* Uhat, void* s, void* Vhat, void* Uk, void* Sk, void* Vk, void* Ak,
             double tol, int max_sweeps, int* info_dev, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!A || !Q || !Uhat || !s || !Vhat) return PQ_ERR_NULL;
  PQ_CHECK(check_svd_args(A, a_dtype, Q, n1, n2, n3, p, k, prec, {Uhat, s, Vhat, Uk, Sk, Vk, Ak}));
  if (!ws || ws_bytes < pq_tsvdq_workspace(n1, n2, n3, p, k, a_dtype)) return PQ_ERR_WORKSPACE;
  PQ_CHECK(sweep_defaults(a_dtype, tol, max_sweeps));
  const Prec pr = (Prec)prec;
  const int dt = a_dtype == PQ_F64 ? PQ_F64 : PQ_F32;
  Arena ar(ws, ws_bytes);
  PQ_CHECK(facewise_svd(A, a_dtype, Q, n1, n2, n3, p, k, pr, 0.0, nullptr, Uhat, s, Vhat, Ak, tol, max_sweeps,
                        info_dev, ar, stream));
  const int ip = (int)p;
  if (Uk) PQ_TRY(do_unhat(Uhat, Q, Uk, dt, n1 * k, (int)n3, ip, back_prec(pr), stream));
  if (Vk) PQ_TRY(do_unhat(Vhat, Q, Vk, dt, n2 * k, (int)n3, ip, back_prec(pr), stream));
  if (Sk) PQ_TRY(do_unhat(s, Q, Sk, dt, k, (int)n3, ip, back_prec(pr), stream));
  return PQ_OK;
}

int pq_svdii(const void* A, int a_dtype, const void* Q, int64_t n1, int64_t n2, int64_t n3, int64_t p,
             double gamma, int64_t kmax, int prec, void* Uhat, void* s, void* Vhat, int* rho_dev, void* Ak,
             double tol, int max_sweeps, int* info_dev, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!A || !Q || !Uhat || !s || !Vhat) return PQ_ERR_NULL;
  if (!(gamma > 0.0 && gamma <= 1.0)) return PQ_ERR_ARG;
  PQ_CHECK(check_svd_args(A, a_dtype, Q, n1, n2, n3, p, kmax, prec, {Uhat, s, Vhat, rho_dev, Ak}));
  if (!ws || ws_bytes < pq_svdii_workspace(n1, n2, n3, p, kmax, a_dtype)) return PQ_ERR_WORKSPACE;
  PQ_CHECK(sweep_defaults(a_dtype, tol, max_sweeps));
  Arena ar(ws, ws_bytes);
  return facewise_svd(A, a_dtype, Q, n1, n2, n3, p, kmax, (Prec)prec, gamma, rho_dev, Uhat, s, Vhat, Ak, tol,
                      max_sweeps, info_dev, ar, stream);
}

size_t pq_tsvdq_backward_workspace(int64_t n1, int64_t n2, int64_t n3, int64_t p, int64_t k, int a_dtype) {
  const bool f64 = a_dtype == PQ_F64;
  const size_t e = elem(f64 ? PQ_F64 : PQ_F32);
  const int64_t N = n1 * n2, L = std::max(n1, n2), S = std::min(n1, n2);
  const int ks = ksplit_for(N, p);
  return (f64 ? 0 : align_up(8 * n3 * p) + align_up(8 * k * p))  // widened Q and sbar
         + sweep_bytes(true, N, p)                  // transform and Jacobi buffers (float64)
         + align_up(8 * S * p) * 2                  // norms, sorted singular values
         + align_up(8 * L * S * p)                  // every normalised Jacobi vector
         + align_up(sizeof(int) * p)                // near-degenerate pairs per face
         + align_up(8 * N * p)                      // Gh
         + align_up(8 * N * p) * 2                  // the face gradient and transform-domain A_k
         + (f64 ? 0 : align_up(4 * N * p) * 2)      // ... rounded to float32
         + align_up(8 * S * S * p)                  // Yall
         + align_up(8 * S * k * p) * 6              // H, P1, Ba, Bb, E, Ep
         + align_up(8 * L * k * p) * 2              // Ra, UE
         + align_up(8 * L * 2 * k * p)              // [U_K X]
         + align_up(8 * S * 2 * k * p)              // [N Y]
         + align_up(e * (size_t)ks * p * n3) * 2;   // split-K slices of the two dQ terms
}

int pq_tsvdq_backward(const void* A, int a_dtype, const void* Q, int64_t n1, int64_t n2, int64_t n3, int64_t p,
                      int64_t k, const void* Gbar, const void* sbar, void* dA, void* dQ, double gap_tol, double tol,
                      int max_sweeps, int* info_dev, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!A || !Q) return PQ_ERR_NULL;
  if (!Gbar && !sbar) return PQ_ERR_NULL;  // nothing to propagate
  if (!dA && !dQ) return PQ_ERR_NULL;      // nothing asked for
  if (a_dtype != PQ_F32 && a_dtype != PQ_F64) return PQ_ERR_DTYPE;
  PQ_CHECK(check_svd_args(A, a_dtype, Q, n1, n2, n3, p, k, PQ_PREC_DEFAULT, {dA, dQ}));
  for (const void* o : {dA, dQ})
    if (o && (o == Gbar || o == sbar)) return PQ_ERR_ALIAS;
  if (dA && dA == dQ) return PQ_ERR_ALIAS;
  if (!ws || ws_bytes < pq_tsvdq_backward_workspace(n1, n2, n3, p, k, a_dtype)) return PQ_ERR_WORKSPACE;
  PQ_CHECK(sweep_defaults(PQ_F64, tol, max_sweeps));
  if (gap_tol <= 0.0) gap_tol = kDefaultGapTol;
  const bool f64 = a_dtype == PQ_F64;
  const int dt = f64 ? PQ_F64 : PQ_F32;
  const size_t e = elem(dt);
  const int64_t N = n1 * n2;
  const int L = (int)std::max(n1, n2), S = (int)std::min(n1, n2);
  const int ip = (int)p, ik = (int)k, in3 = (int)n3;
  const int ks = ksplit_for(N, p);
  const bool cols = n1 >= n2;
  const bool has_g = Gbar != nullptr;
  const Prec pr = Prec::Default;
  Arena ar(ws, ws_bytes);
  // The adjoint's coefficients divide by the gaps of the face spectra, so
  // float32 arithmetic anywhere from the data to the face gradient (the
  // transforms included) would leave errors of about 1e-7 / (relative gap).
  // float32 data are exact in float64: they are widened (A and Gbar inside
  // the float64 transform, Q and sbar here), and everything up to the face
  // gradient runs in float64; the two transforms back (dA, dQ), where no gap
  // enters any more, run in the data's type.
  const double* Q64 = static_cast<const double*>(Q);
  const double* s64 = static_cast<const double*>(sbar);
  if (!f64) {
    double* q64 = static_cast<double*>(ar.take(8 * n3 * p));
    double* sb64 = static_cast<double*>(ar.take(8 * k * p));
    PQ_PROF("grad_elementwise", stream);
    PQ_TRY(pq::jacobi_widen(static_cast<const float*>(Q), q64, n3 * p, stream));
    if (sbar) PQ_TRY(pq::jacobi_widen(static_cast<const float*>(sbar), sb64, k * p, stream));
    Q64 = q64;
    s64 = sbar ? sb64 : nullptr;
  }
  const SweepBufs b = take_sweep_bufs(ar, true, N, p);
  double* sig = static_cast<double*>(ar.take(8 * (size_t)S * p));
  double* sigs = static_cast<double*>(ar.take(8 * (size_t)S * p));
  double* U = static_cast<double*>(ar.take(8 * (size_t)L * S * p));
  int* cnt = static_cast<int*>(ar.take(sizeof(int) * p));
  double* Gh = static_cast<double*>(ar.take(8 * N * p));
  double* Mbar = static_cast<double*>(ar.take(8 * N * p));
  double* Akh = static_cast<double*>(ar.take(8 * N * p));
  float* Mbar32 = f64 ? nullptr : static_cast<float*>(ar.take(4 * N * p));
  float* Akh32 = f64 ? nullptr : static_cast<float*>(ar.take(4 * N * p));
  double* Yall = static_cast<double*>(ar.take(8 * (size_t)S * S * p));
  double* H = static_cast<double*>(ar.take(8 * (size_t)S * k * p));
  double* P1 = static_cast<double*>(ar.take(8 * (size_t)S * k * p));
  double* Ba = static_cast<double*>(ar.take(8 * (size_t)S * k * p));
  double* Bb = static_cast<double*>(ar.take(8 * (size_t)S * k * p));
  double* E = static_cast<double*>(ar.take(8 * (size_t)S * k * p));
  double* Ep = static_cast<double*>(ar.take(8 * (size_t)S * k * p));
  double* Ra = static_cast<double*>(ar.take(8 * (size_t)L * k * p));
  double* UE = static_cast<double*>(ar.take(8 * (size_t)L * k * p));
  double* LHS = static_cast<double*>(ar.take(8 * (size_t)L * 2 * k * p));
  double* RHS = static_cast<double*>(ar.take(8 * (size_t)S * 2 * k * p));
  char* parts = static_cast<char*>(ar.take(e * (size_t)ks * p * n3 * 2));
  const int64_t sU = (int64_t)L * S, sY = (int64_t)S * S, sK = (int64_t)S * k, sR = (int64_t)L * k;
  // the forward factorisation in float64: every singular vector of the
  // Jacobi side
  PQ_CHECK(converge(A, dt, Q64, n1, n2, n3, p, pr, tol, max_sweeps, b, info_dev, stream, !f64));
  {
    PQ_PROF("jacobi_finalize", stream);
    PQ_TRY(pq::jacobi_norms_f64(b.W64, ip, S, L, sig, nullptr, stream));
    PQ_TRY(pq::jacobi_finalize_f64(b.W64, sig, ip, S, L, S, nullptr, 0, U, sigs, stream));
  }
  const double* M = static_cast<const double*>(b.Ah);
  // M_t is the face (cols) or its transpose; op(M_t^T) is the face with
  // transpose flag `cols`, op(M_t) with `!cols`.  Yall = M_t^T U, Y = its
  // first k columns.
  PQ_TRY(do_gemm("grad_gemm", face_gemm(cols, false, S, S, L, M, n1, N, U, L, sU, Yall, S, sY, ip), PQ_F64, pr,
                 stream));
  if (has_g) {
    if (f64) {
      PQ_TRY(do_hat(Gbar, PQ_F64, Q64, Gh, N, in3, ip, pr, stream));
    } else {
      PQ_PROF("hat", stream);
      PQ_TRY(pq::hat_f64_wide(static_cast<const float*>(Gbar), Q64, Gh, N, in3, ip, stream));
    }
    // H = G_t^T U_K;  Ra = G_t Y;  Ba = U^T Ra;  Bb = Yall^T H
    PQ_TRY(do_gemm("grad_gemm", face_gemm(cols, false, S, ik, L, Gh, n1, N, U, L, sU, H, S, sK, ip), PQ_F64, pr,
                   stream));
    PQ_TRY(do_gemm("grad_gemm", face_gemm(!cols, false, L, ik, S, Gh, n1, N, Yall, S, sY, Ra, L, sR, ip), PQ_F64,
                   pr, stream));
    PQ_TRY(do_gemm("grad_gemm", face_gemm(true, false, S, ik, L, U, L, sU, Ra, L, sR, Ba, S, sK, ip), PQ_F64, pr,
                   stream));
    PQ_TRY(do_gemm("grad_gemm", face_gemm(true, false, S, ik, S, Yall, S, sY, H, S, sK, Bb, S, sK, ip), PQ_F64, pr,
                   stream));
    {
      PQ_PROF("grad_elementwise", stream);
      PQ_TRY(pq::grad_coef(Ba, Bb, sigs, ip, S, ik, gap_tol, E, Ep, cnt, true, stream));
    }
    // X = Ra diag(1/lambda) + U E into the second half of LHS;  P1 = Yall Ep
    PQ_TRY(do_gemm("grad_gemm", face_gemm(false, false, L, ik, S, U, L, sU, E, S, sK, UE, L, sR, ip), PQ_F64, pr,
                   stream));
    PQ_TRY(do_gemm("grad_gemm", face_gemm(false, false, S, ik, S, Yall, S, sY, Ep, S, sK, P1, S, sK, ip), PQ_F64,
                   pr, stream));
    pq::ProfScope prof_elementwise("grad_elementwise", stream, 3);
    PQ_TRY(pq::grad_xcombine(Ra, UE, U, sigs, ip, L, S, ik, LHS, true, stream));
    PQ_TRY(pq::grad_ncombine(H, P1, Yall, s64, sigs, ip, S, S, ik, RHS, true, false, stream));
    if (info_dev) PQ_TRY(pq::grad_count(cnt, ip, info_dev + 3, stream));
  } else {
    pq::ProfScope prof_elementwise("grad_elementwise", stream, 3);
    PQ_TRY(pq::grad_xcombine(nullptr, nullptr, U, sigs, ip, L, S, ik, LHS, true, stream));
    PQ_TRY(pq::grad_ncombine(nullptr, nullptr, Yall, s64, sigs, ip, S, S, ik, RHS, true, false, stream));
    if (info_dev) PQ_TRY(pq::grad_count(cnt, 0, info_dev + 3, stream));
  }
  // the face gradient: dM_t = [U_K X][N Y]^T, written as the face itself
  {
    Gemm g = cols ? face_gemm(false, true, L, S, 2 * ik, LHS, L, (int64_t)L * 2 * k, RHS, S, (int64_t)S * 2 * k,
                              Mbar, n1, N, ip)
                  : face_gemm(false, true, S, L, 2 * ik, RHS, S, (int64_t)S * 2 * k, LHS, L, (int64_t)L * 2 * k,
                              Mbar, n1, N, ip);
    PQ_TRY(do_gemm("grad_gemm", g, PQ_F64, pr, stream));
  }
  // the transforms back run in the data's type, on its own A, Q and Gbar
  const void* Mb = Mbar;
  if (!f64) {
    PQ_PROF("grad_elementwise", stream);
    PQ_TRY(pq::grad_narrow(Mbar, Mbar32, N * p, stream));
    Mb = Mbar32;
  }
  if (dA) PQ_TRY(do_unhat(Mb, Q, dA, dt, N, in3, ip, pr, stream));
  if (dQ) {
    // dQ^T = Mbar_(3) A_(3)^T + Akh_(3) Gbar_(3)^T
    const size_t slab = e * (size_t)p * n3;
    PQ_TRY(do_gemm("dq_gemm", dq_gemm(Mb, A, ip, in3, N, parts, ks), dt, pr, stream));
    int nparts = ks;
    if (has_g) {
      // Akh = U_K Y^T (cols) or Y U_K^T (rows): the transform-domain A_k
      Gemm g = cols ? face_gemm(false, true, L, S, ik, U, L, sU, Yall, S, sY, Akh, n1, N, ip)
                    : face_gemm(false, true, S, L, ik, Yall, S, sY, U, L, sU, Akh, n1, N, ip);
      PQ_TRY(do_gemm("approx_gemm", g, PQ_F64, pr, stream));
      const void* Ak = Akh;
      if (!f64) {
        PQ_PROF("grad_elementwise", stream);
        PQ_TRY(pq::grad_narrow(Akh, Akh32, N * p, stream));
        Ak = Akh32;
      }
      PQ_TRY(do_gemm("dq_gemm", dq_gemm(Ak, Gbar, ip, in3, N, parts + slab * ks, ks), dt, pr, stream));
      nparts += ks;
    }
    PQ_TRY(do_sum(parts, nparts, p * n3, p * n3, dQ, dt, stream));
  }
  return PQ_OK;
}

}  // extern "C"
