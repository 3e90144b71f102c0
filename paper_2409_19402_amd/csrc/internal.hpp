// Host-side launchers of the projprod kernels.  Tensors are seen as row-major
// matrices: an n1 x n2 x n3 face-major tensor is the n3 x N matrix (N = n1*n2)
// whose row t is frontal slice t; Q is n3 x p row-major.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <functional>
#include <string>
#include <vector>

namespace pq {

enum class Prec : int { Default = 0, BF16 = 1, BF16x3 = 2, BF16x6 = 3 };

// ---- launch-configuration autotuner (tune.cpp) ------------------------------
// launch(c) enqueues candidate configuration c (0 <= c < ncand) on s.  The
// recorded choice for key is used; with none recorded and tuning switched on
// every candidate is timed (synchronising s) and the fastest recorded;
// otherwise candidate dflt is used.
hipError_t tuned_launch(const std::string& key, int ncand, int dflt, hipStream_t s,
                        const std::function<hipError_t(int)>& launch);
void tune_enable(bool on);
int tune_entries();
bool tune_save(const char* path);
bool tune_load(const char* path);

// ---- per-launch profiler (prof.cpp) ---------------------------------------
// While enabled, a ProfScope records a hipEvent on s at construction and at
// destruction; the pair is kept under `name` (a string literal) and counts as
// `launches` launches.
class ProfScope {
 public:
  ProfScope(const char* name, hipStream_t s, int launches = 1);
  ~ProfScope();
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;

 private:
  const char* name_;
  hipStream_t s_;
  int count_;
  hipEvent_t a_ = nullptr;
};
// While a ProfMute lives, the ProfScopes of its host thread record nothing
// (launches that an enclosing scope on another stream already brackets).
class ProfMute {
 public:
  ProfMute();
  ~ProfMute();
  ProfMute(const ProfMute&) = delete;
  ProfMute& operator=(const ProfMute&) = delete;
};
void prof_enable(bool on);
void prof_reset();
hipError_t prof_query(const char* name, double* total_ms, int* launches);
bool prof_names(char* buf, size_t len);

// ---- mode-3 transforms (transform.hip) -----------------------------------
// Ah (p x N) = Q^T (p x n3) * A (n3 x N); A is float32 or bfloat16 bits.
hipError_t hat_f32(const void* A, bool a_bf16, const float* Q, float* Ah,
                   int64_t N, int n3, int p, Prec prec, hipStream_t s);
hipError_t hat_f64(const double* A, const double* Q, double* Ah,
                   int64_t N, int n3, int p, hipStream_t s);
// the float64 transform of float32 data (each element widened exactly)
hipError_t hat_f64_wide(const float* A, const double* Q, double* Ah, int64_t N, int n3, int p, hipStream_t s);
// A (n3 x N) = Q (n3 x p) * Ah (p x N)
hipError_t unhat_f32(const float* Ah, const float* Q, float* A,
                     int64_t N, int n3, int p, Prec prec, hipStream_t s);
hipError_t unhat_f64(const double* Ah, const double* Q, double* A,
                     int64_t N, int n3, int p, hipStream_t s);
// out (n3 x N) = Q Q^T A in one pass; valid when proj_fused_ok(n3, p).
bool proj_fused_ok(int n3, int p);
hipError_t proj_fused_f32(const void* A, bool a_bf16, const float* Q, float* out,
                          int64_t N, int n3, int p, Prec prec, hipStream_t s);

// ---- batched GEMM (gemm.hip) ----------------------------------------------
// For every batch b: C_b = op(A_b) op(B_b), column-major operands;
// op(X) = X^T when the flag is set.  op(A) is M x K, op(B) is K x N.
// With ksplit > 1 the K range is cut into ksplit slices and slice z writes
// its partial product to C + z * sSplit (to be summed by sum_partials).
struct Gemm {
  bool ta, tb;
  int M, N, K;
  const void* A; int64_t lda, sA;
  const void* B; int64_t ldb, sB;
  void* C; int64_t ldc, sC;
  int batch;
  int ksplit; int64_t sSplit;
};
hipError_t gemm_f32(const Gemm& g, Prec prec, hipStream_t s);
// Many float32 products C_z = A_z B_z (no transposes, column-major) of
// different shapes in one launch: descs (device) one per product, tiles
// (device) one per 128 x 128 output tile {product, tile row, tile column,
// batch entry}, in the order the host wants them started.
struct GemmDesc {
  const float* A;
  const float* B;
  float* C;
  int M, N, K;
  int64_t lda, sA, ldb, sB, ldc, sC;
  int vec4;  // operands allow 16-byte loads (gemm_vec4_ok)
};
struct GemmTile {
  int desc, tx, ty, z;
};
bool gemm_vec4_ok(const GemmDesc& d);
hipError_t gemm_f32_grouped(const GemmDesc* descs, const GemmTile* tiles, int ntiles, hipStream_t s);
hipError_t gemm_f64(const Gemm& g, hipStream_t s);
// out[e] = sum_{z < nparts} parts[z * stride + e] for e < count, fixed order
hipError_t sum_partials_f32(const float* parts, int nparts, int64_t stride,
                            int64_t count, float* out, hipStream_t s);
hipError_t sum_partials_f64(const double* parts, int nparts, int64_t stride,
                            int64_t count, double* out, hipStream_t s);
// the same for float32 slices, summed in float64
hipError_t sum_to_f64(const float* parts, int nparts, int64_t stride, int64_t count, double* out, hipStream_t s);

// ---- Q = U3 (misc.hip) ---------------------------------------------------------
// Q (n3 x p row-major, float32 or float64) from the p normalised eigenvectors
// F (vector-major, n3 each): columns signed so that the largest-magnitude
// entry is positive; lambda[r] = f_r^T G f_r (G n3 x n3)
hipError_t u3_finish(const double* F, const double* G, int n3, int p, void* Q, void* lambda, bool f64,
                     hipStream_t s);
// max |(Q^T Q - I)_ab| into out[0] (float64): two launches, the first clears out
hipError_t check_q_launch(const void* Q, bool f64, int n3, int p, double* out, hipStream_t s);
hipError_t check_q_flag(const double* dist, double tol, int* flag, hipStream_t s);
// dst = src in the other layout: tube-major (t + n3 (j + n2 i)) to face-major
// (i + n1 (j + n2 t)) when to_face, the reverse otherwise; elements of
// elem_bytes (2, 4 or 8) bytes; (ceil(n3 / 32) n2, ceil(n1 / 32)) workgroups
hipError_t relayout(const void* src, void* dst, int elem_bytes, bool to_face, int n1, int n2, int n3, hipStream_t s);
// Qout = Q R^{-1} by CholeskyQR2 in float64 (one workgroup; p <= 128; W:
// n3 p doubles of scratch); info[0] = 0, or c + 1 for a column c that is
// numerically dependent on the earlier ones (Qout then unwritten)
hipError_t cholqr2(const void* Q, bool f64, int n3, int p, double* W, void* Qout, int* info, hipStream_t s);
// Q (n3 x p row-major) of a fixed transform: kind 0 identity, 1 DCT-II
hipError_t build_q(int kind, bool f64, int n3, int p, void* Q, hipStream_t s);

// ---- facewise one-sided Jacobi SVD (jacobi.hip) -----------------------------
// W holds, for each of p faces, nv vectors of length L (vector j of face l at
// W + (l*nv + j)*L).  prep copies the faces of Ah (n1 x n2 x p, face-major)
// into W: the columns when n1 >= n2 (nv = n2, L = n1), else the rows
// (nv = n1, L = n2).
hipError_t jacobi_prep_f32(const float* Ah, float* W, int n1, int n2, int p, hipStream_t s);
hipError_t jacobi_prep_f64(const double* Ah, double* W, int n1, int n2, int p, hipStream_t s);
// Orthogonalises the nv vectors of every face; sweeps_used[l] gets the sweep
// count of face l, or max_sweeps + 1 when it stopped without converging.
// flags: p * max_sweeps ints of scratch.  A face stops after a sweep that
// rotated nothing or, with stop2 > 0, after a sweep whose largest cosine c
// had c^2 <= stop2 (near convergence a sweep squares c, so the sweep itself
// brought the face to about stop2); pairs rotate down to tol either way.
hipError_t jacobi_sweeps_f32(float* W, int p, int nv, int L, int max_sweeps, double tol, double stop2,
                             int* sweeps_used, int* flags, hipStream_t s);
// Grouped Jacobi over faces of different sizes (the batched form): faces[f]
// (device) gives face f's element offset in W, its vector count and length.
// nb_max is the largest block count (ceil(nv / 16), rounded up to even) over
// the faces and L_max the largest length (any length: vectors too long to
// stage in LDS are read from the L2).
struct JFace {
  int64_t off;
  int nv, L;
};
// Many float32 mode-3 transforms in one launch each (the batched form): a
// descriptor per tensor (in: A for the forward transform, Chat for the
// return one; Q; out; N = n1 n2 tubes; n3; p) and one entry per workgroup
// (x: strip of 32 vec tubes for the forward transform, group of four such
// strips for the return one; y: 32-row chunk of p for the forward
// transform; 0 for the return one, whose workgroups write every output
// tile of their strips).  The return transform
// keeps a strip's p <= 32 rows in registers: larger p is not grouped.
struct XformDesc {
  const float* in;
  const float* Q;
  float* out;
  int64_t N;
  int n3, p;
};
struct XformTile {
  int64_t x;
  int desc, y;
};
// tubes per lane for a tensor: 4, 2 or 1, the widest accesses (16, 8 or 4
// bytes) that N and both pointers allow (the tiles of one launch share it)
int xform_group_vec(const XformDesc& d);
int unhat_group_vec(const XformDesc& d);
void hat_group_tiles(const XformDesc& d, int desc, std::vector<XformTile>& tiles);
void unhat_group_tiles(const XformDesc& d, int desc, std::vector<XformTile>& tiles);
hipError_t hat_grouped(const XformDesc* d, const XformTile* t, int ntiles, int vec, hipStream_t s);
hipError_t unhat_grouped(const XformDesc* d, const XformTile* t, int ntiles, int vec, size_t q_bytes,
                         hipStream_t s);
// LDS bytes of a return transform's Q staged in LDS
size_t unhat_group_q_bytes(const XformDesc& d);
// Visits of a grouped sweep listed per round, so that a launch has one
// workgroup per visit that exists (faces of fewer blocks have fewer rounds
// and pairs): entry (f << kVisitShift) | slot names face f of the table and
// its visit slot; round r's entries are dev[off[r] .. off[r + 1]) (off on
// the host, one more value than rounds).  Built by jacobi_visit_list with the
// same ntop as the launches that use it.
constexpr int kVisitShift = 6;
struct VisitList {
  const int* dev = nullptr;
  const int* off = nullptr;
};
// the visit list of the grouped sweeps over faces (host copy of the face
// table); false when the table is too large to list
bool jacobi_visit_list(const JFace* faces, int nfaces, int ntop, std::vector<int>& entries, std::vector<int>& off,
                       const std::vector<char>* pick = nullptr);
// vl: the sweep's visit list (nullptr: every face at the largest face's
// rounds and slots, idle workgroups exiting at once)
// A second stream for the grouped sweeps: the faces split in two
// halves with visit lists of their own (vla, vlb), the first half's rounds
// on the caller's stream and the second's on s2, between a fork and a join
// event, so that one half's memory phases (staging, write-back) overlap the
// other's rotation rounds.  Used when a launch would hold two or more
// visits per CU; otherwise the sweeps run the full list on one stream.
constexpr int kSweepParts = 2;  // three or four parts measured no faster
struct SweepPair {
  hipStream_t s2[kSweepParts - 1] = {};
  hipEvent_t fork = nullptr, join[kSweepParts - 1] = {};
  const VisitList* vl[kSweepParts] = {};
};
hipError_t jacobi_gram_grouped_f32(float* W, const JFace* faces, int nfaces, int nb_max, int L_max,
                                   int max_sweeps, double tol, double stop2, int* used, int* flags,
                                   const VisitList* vl, hipStream_t s, const SweepPair* sp = nullptr);
// ntop (1 or 2; 0 = every pair): the top-block schedule, which visits only
// the pairs with a vector in the first ntop 16-vector blocks of a face
hipError_t jacobi_gram_grouped_f64(double* W, const JFace* faces, int nfaces, int nb_max, int L_max,
                                   int max_sweeps, double tol, double stop2, int ntop, int* used, int* flags,
                                   const VisitList* vl, hipStream_t s, const SweepPair* sp = nullptr);
// float64 sweeps in the Gram-matrix form (the polishing sweeps of float32
// data); ntop as above
hipError_t jacobi_gram_sweeps_f64(double* W, int p, int nv, int L, int max_sweeps, double tol, double stop2,
                                  int ntop, int* used, int* flags, hipStream_t s);
// prior (may be null): a face with prior[f] <= prior_max converged in an
// earlier phase and is left alone (sweeps_used[f] = 0)
hipError_t jacobi_sweeps_f64(double* W, int p, int nv, int L, int max_sweeps, double tol,
                             int* sweeps_used, int* flags, const int* prior, int prior_max, hipStream_t s);
// Column norms, descending order, top k normalised vectors F (L x k x p).
// norms of all nv vectors of every face into sig (nv x p, float64); rank
// (n = nv p ints, may be null) cleared for jacobi_select
hipError_t jacobi_norms_f64(const double* W, int p, int nv, int L, double* sig, int* rank, hipStream_t s);
// the top k of each face by sig, normalised into F (L x k x p); a face keeps
// min(k, kface[f] + extra) vectors when kface is given, zero columns after
// them; sig_sorted (k x p, may be null) receives the matching norms (0 past
// them)
hipError_t jacobi_finalize_f64(const double* W, const double* sig, int p, int nv, int L, int k, const int* kface,
                              int extra, double* F, double* sig_sorted, hipStream_t s);
// *_Q-SVDII selection over the n = p nv values of sig (rank cleared by
// jacobi_norms_f64): rho[f] = face f's values among the first K of the
// descending order, K the first count whose energy reaches gamma of the
// total; e2 is n doubles of scratch
hipError_t jacobi_select(const double* sig, int p, int nv, double gamma, int* rank, double* e2, int* rho,
                         hipStream_t s);
// The Rayleigh-Ritz step of the truncation: float64 Jacobi on the k columns
// of Y (m1 x k x p), each rotation applied to F (m2 x k x p) too; writes the
// leading kout <= k of the results: s (kout x p, descending), Other = Y / s,
// Fo = F and Ys = Y, in descending order of s, in the output type.  With
// kface given a face works on min(k, kface[f] + extra) columns and keeps
// min(kout, kface[f]), zero columns after them.
hipError_t jacobi_refine_f32(double* Y, double* F, int m1, int m2, int k, int kout, int p, const int* kface,
                             int extra, double tol, float* s_out, float* Other, float* Fo, float* Ys,
                             hipStream_t s);
hipError_t jacobi_refine_f64(double* Y, double* F, int m1, int m2, int k, int kout, int p, const int* kface,
                             int extra, double tol, double* s_out, double* Other, double* Fo, double* Ys,
                             hipStream_t s);
// Columns of the Rayleigh-Ritz step for a rank-k truncation of faces with nv
// singular values: k plus kRitzExtra more, at most nv.  The leading k of the
// Ritz values and vectors on the span of the top k + kRitzExtra Jacobi vectors
// (with the transform-domain face itself in the products) are first-order
// sensitive to the Jacobi's own rounding only through the gap between the
// k-th and the (k + kRitzExtra + 1)-th singular value, instead of the gap
// between the k-th and the (k + 1)-th.
constexpr int kRitzExtra = 8;
// Prediction threshold of the float64 top-block polish of float32 data (c^2
// of the largest cosine before rotation, with the rotations themselves going
// down to 1e-10): a face stops after the sweep that started from
// c^2 <= 1e-5, which leaves its leading vectors at cosines of about 1e-5
// against all others.  The Rayleigh-Ritz step that follows is accurate to
// second order in those cosines; measured, the sweeps that would continue
// (one more on most faces) change no A_k by more than rounding.
constexpr double kPolishStop32 = 1e-5;
// Prediction threshold of the float32 sweeps ahead of that polish (their
// rotations still go down to 1e-5): the leading vectors by norm must hold
// the Ritz step's columns when the polish takes over.  Measured on the
// batched test instances: 1e-4 and 3e-4 change no result; 1e-3 moved one
// instance whose Ritz columns (15) nearly fill its single leading block by
// 2.5e-5, so the threshold keeps a factor of ten from there.
constexpr double kCoarseStop32 = 1e-4;
inline int ritz_cols(int64_t k, int64_t nv) { return (int)(k + kRitzExtra < nv ? k + kRitzExtra : nv); }
// The finishing steps of the truncation (norms, the top kr normalised vectors
// F, Y = Ah^T F or Ah F, the Ritz step keeping kout) for many faces of
// different shapes, one launch each: every face described by a FinFace in a
// device table.
struct FinFace {
  const double* w;  // Jacobi vectors: nv x L, vector-major (nv = min(n1, n2), L = max)
  const float* ah;  // the transform-domain face: n1 x n2, column-major
  double* sig;      // nv norms (scratch)
  double* ft;       // kr columns of L (scratch)
  double* y;        // kr columns of nv (scratch)
  float* s;         // kout singular values
  float* other;     // kout columns of nv: Y / s (the side of Y)
  float* fo;        // kout columns of L: F (the side of the Jacobi vectors)
  float* ys;        // kout columns of nv: Y (scratch for A_k)
  int n1, n2, kr, kout;
};
// maxima over the table's faces: n1, n2, nv = min(n1, n2), nvL = n1 + n2, kr
struct FinMax {
  int n1 = 1, n2 = 1, nv = 1, nvL = 2, kr = 1;
};
hipError_t jacobi_finish_grouped(const FinFace* tab, int nfaces, const FinMax& m, double tol, hipStream_t s);
// y[i] = x[i] for i < n (float32 -> float64)
hipError_t jacobi_widen(const float* x, double* y, int64_t n, hipStream_t s);
// the same per face (faces: the table of the grouped form, or null for p =
// nfaces faces of nv_u x L_u), the ntop16 vectors of largest norm moved to
// the front in descending order (the leading blocks of the top-block
// schedule), the others after them in their own order; nrm (doubles) and
// pos (ints): nfaces x nv_max of scratch each; nv_max <= 4096
hipError_t jacobi_widen_top(const float* W32, double* W64, const JFace* faces, int nfaces, int nv_u, int L_u,
                            int nv_max, int ntop16, double* nrm, int* pos, hipStream_t s);
// leading 16-vector blocks of the top-block polish for a Ritz step on kr
// columns: 1 or 2, or 0 (the full schedule) when kr needs more.  The
// polish makes the leading vectors orthogonal to the others; it does not
// move a leading singular direction that the float32 sweeps left among the
// trailing vectors into the leading blocks, so the blocks hold kr + 8
// vectors: the kr of largest norm and a margin against that.
inline int top_blocks(int kr) { return kr + 8 <= 16 ? 1 : kr + 8 <= 32 ? 2 : 0; }
// Y = Ah_l^T F_l (cols: Y n2 x k, F n1 x k) or Ah_l F_l (rows: Y n1 x k,
// F n2 x k) per face, float64 accumulation and result
hipError_t jacobi_factor_f32(const float* Ah, const double* F, double* Y, int n1, int n2, int k, int p,
                             bool cols, hipStream_t s);
hipError_t jacobi_factor_f64(const double* Ah, const double* F, double* Y, int n1, int n2, int k, int p,
                             bool cols, hipStream_t s);
// info[0] = the most sweeps a face used over both phases (used2 may be
// NULL; max1 and max2 are the phases' caps), info[1] = #faces whose last
// phase did not converge, info[2] = the sweeps summed over the faces.
// ---- adjoint of the truncated tSVDQ (svdgrad.hip) -------------------------
hipError_t grad_narrow(const double* x, float* y, int64_t n, hipStream_t s);
// E and Ep (nv x k x p) from Ba = U^T Ra, Bb = Yall^T H and the sorted
// singular values sig (nv x p); cnt[f] = pairs of face f whose gap fell
// under gap_tol
hipError_t grad_coef(const void* Ba, const void* Bb, const double* sig, int p, int nv, int k, double gap_tol,
                     void* E, void* Ep, int* cnt, bool f64, hipStream_t s);
// LHS (L x 2k x p) = [U_K, R diag(1/lambda) + UE] (R null: zero second half)
hipError_t grad_xcombine(const void* R, const void* UE, const void* U, const double* sig, int p, int L, int nv, int k,
                         void* LHS, bool f64, hipStream_t s);
// RHS (S x 2k x p) = [H + P1 + Y diag(sbar / sigma), Y] (null terms are 0;
// Y is read from Yall, S x S per face)
hipError_t grad_ncombine(const void* H, const void* P1, const void* Y, const void* sbar, const double* sig, int p,
                         int S, int nv, int k, void* RHS, bool f64, bool sbar_f32, hipStream_t s);
// out[0] = sum of cnt[0..p)
hipError_t grad_count(const int* cnt, int p, int* out, hipStream_t s);

// records e as the last failed HIP call of this thread (pq_last_hip_error)
// and returns PQ_ERR_HIP
int note_hip_error(hipError_t e);

hipError_t jacobi_info(const int* used1, const int* used2, int p, int max1, int max2, int* info,
                       hipStream_t s);

}  // namespace pq
