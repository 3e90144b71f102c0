// Facewise truncated SVD of the transform-domain faces (Alg. 4.1 step 3) by
// one-sided (Hestenes) Jacobi.
//
// Each face contributes nv = min(n1, n2) vectors of length L = max(n1, n2)
// (its columns when n1 >= n2, its rows otherwise).  For a pair (a, c) a wave
// forms alpha = |a|^2, beta = |c|^2, gamma = a.c with float64 accumulation
// and a DPP reduction across its lanes, computes in float64 the plane
// rotation that zeroes gamma, and applies it.  Converged vectors are mutually
// orthogonal; their norms are the singular values and, normalised, they are
// the singular vectors of their side.  A face has converged after a sweep in
// which no pair had |gamma| > tol sqrt(alpha beta), or (the sweeps of
// float32 data) after a sweep whose largest |gamma| / sqrt(alpha beta) was
// at most sqrt(tol), which by quadratic convergence leaves it near tol.
//
// Schedule (block form): the nv vectors are cut into nb blocks of b vectors
// (nb even; vectors past nv are zero and never rotate; b = 4 per wave, one
// pair per 16-lane row).  One launch is one
// round of a round-robin tournament over the blocks: workgroup (x, face)
// stages the 2b vectors of block pair x in LDS.  In the first round of a sweep
// it runs a full round-robin over all 2b vectors (every block takes part in
// that round, so every pair inside a block is visited once per sweep); in the
// other rounds only the b*b pairs between its two blocks are left, visited in
// b rounds with the first block's vectors kept in registers.  nb - 1 launches
// make a sweep.  With nb == 2 one workgroup holds the whole face and loops
// over sweeps by itself.  Vectors longer than 1024 fall back to a form with
// one workgroup per face and the pairs read from global memory.
//
// Precision: float32 faces are first swept with float32 storage down to a
// coarse threshold, then the vectors are promoted to float64 and polished by
// float64 sweeps (quadratic convergence: a few sweeps).  The residual coupling
// of two singular vectors at convergence is about tol / (2 x relative gap of
// their singular values); float32 storage cannot push tol much below 1e-7,
// which on the nearly flat spectra of noise faces (relative gaps of 1e-3)
// would leave the rank-k truncation visibly mixed.
//
// The factor on the other side is Y = Ahat F (or Ahat^T F) for the top-k
// Jacobi vectors F, formed with float64 accumulation.  A last small float64
// Jacobi on the k columns of Y, applying each rotation to F as well, makes
// both factors orthonormal to working precision without changing Y F^T; its
// column norms are the singular values.
#include <algorithm>
#include <climits>

#include <type_traits>

#include "common.hpp"
#include "internal.hpp"

namespace pq {
namespace {

constexpr int kJacobiThreads = 1024;

// circle-method round robin over n (even) players: pair `pi` of round `r`
// (0 <= r < n - 1, 0 <= pi < n / 2)
__device__ __forceinline__ void circle_pair(int n, int r, int pi, int& a, int& c) {
  if (pi == 0) {
    a = n - 1;
    c = r;
  } else {
    a = r + pi;
    if (a >= n - 1) a -= n - 1;
    c = r - pi;
    if (c < 0) c += n - 1;
  }
}

struct Rot {
  double c, s;
  bool on;
};

__device__ __forceinline__ Rot rotation(double al, double be, double ga, double tol) {
  Rot q{1.0, 0.0, false};
  if (ga != 0.0 && fabs(ga) > tol * sqrt(al) * sqrt(be)) {
    const double zeta = (be - al) / (2.0 * ga);
    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    q.c = 1.0 / sqrt(1.0 + t * t);
    q.s = q.c * t;
    q.on = true;
  }
  return q;
}

// Row-granular pairs: every 16-lane row of a wave owns one pair, so a wave
// rotates four pairs with the same instructions.  Lane g of a row holds, of
// each of its two vectors, elements 64c + 4g + j (c < R, j < 4): four
// consecutive values per 64-element chunk, read from LDS as one 16-byte load.
// Sums over the 16 lanes of a row use DPP within the row and leave the result
// in every lane of the row.
__device__ __forceinline__ double row_total(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return v;
}

template <typename T, int R>
__device__ __forceinline__ bool rotate_row_pair(T (&xa)[4 * R], T (&xc)[4 * R], double tol) {
  double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
  for (int i = 0; i < 4 * R; ++i) {
    const double a = (double)xa[i], c = (double)xc[i];
    al = fma(a, a, al);
    be = fma(c, c, be);
    ga = fma(a, c, ga);
  }
  al = row_total(al);
  be = row_total(be);
  ga = row_total(ga);
  // rotate when |gamma| > tol sqrt(alpha beta)
  if (!(ga * ga > tol * tol * al * be)) return false;
  const double zeta = (be - al) / (2.0 * ga);
  const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  // the rotation is applied in float64 and rounded once: an exactly
  // orthogonal update, so the residual |gamma| left behind is at the rounding
  // floor of the storage type even for pairs of very different norms
  const double cs = 1.0 / sqrt(1.0 + t * t);
  const double sn = cs * t;
#pragma unroll
  for (int i = 0; i < 4 * R; ++i) {
    const double a = (double)xa[i], c = (double)xc[i];
    xa[i] = static_cast<T>(cs * a - sn * c);
    xc[i] = static_cast<T>(sn * a + cs * c);
  }
  return true;
}

template <typename T, int R>
__device__ __forceinline__ void row_load(const T* v, int g, T (&x)[4 * R]) {
#pragma unroll
  for (int c = 0; c < R; ++c)
#pragma unroll
    for (int j = 0; j < 4; ++j) x[4 * c + j] = v[64 * c + 4 * g + j];
}
template <typename T, int R>
__device__ __forceinline__ void row_store(T* v, int g, const T (&x)[4 * R]) {
#pragma unroll
  for (int c = 0; c < R; ++c)
#pragma unroll
    for (int j = 0; j < 4; ++j) v[64 * c + 4 * g + j] = x[4 * c + j];
}

constexpr int kPairsPerWave = 4;

template <typename T, int R>
__global__ __launch_bounds__(256) void jacobi_block_kernel(T* __restrict__ W, int nv, int L, int nb,
                                                            int round, int sweep, int max_sweeps,
                                                            double tol, int* __restrict__ flags,
                                                            int* __restrict__ sweeps_used,
                                                            const int* __restrict__ prior, int prior_max) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* V = reinterpret_cast<T*>(smem_raw);
  __shared__ int any_rot;
  constexpr int Lp = 64 * R;
  const int NW = blockDim.x >> 6;
  const int b = NW * kPairsPerWave;  // vectors per block = pairs per round
  const int nvl = 2 * b;
  const int face = blockIdx.y;
  const bool whole = nb == 2;
  if (prior && prior[face] <= prior_max) {  // converged in an earlier phase: no sweep
    if (whole && threadIdx.x == 0) sweeps_used[face] = 0;
    return;
  }
  if (!whole && sweep > 0 && flags[face * max_sweeps + sweep - 1] == 0) return;
  int I, J;
  circle_pair(nb, round, blockIdx.x, I, J);
  T* Wf = W + (int64_t)face * nv * L;
  for (int idx = threadIdx.x; idx < nvl * Lp; idx += blockDim.x) {
    const int u = idx / Lp, e = idx - u * Lp;
    const int g = (u < b) ? I * b + u : J * b + (u - b);
    T v = T(0);
    if (g < nv && e < L) v = Wf[(int64_t)g * L + e];
    V[idx] = v;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int gl = lane & 15;                          // lane within the row
  const int pi = wave * kPairsPerWave + (lane >> 4);  // this row's pair
  int sw = 0;
  bool converged = false;
  do {
    if (threadIdx.x == 0) any_rot = 0;
    __syncthreads();
    bool mine = false;
    if (whole || round == 0) {
      for (int r = 0; r < nvl - 1; ++r) {
        int ia, ic;
        circle_pair(nvl, r, pi, ia, ic);
        T xa[4 * R], xc[4 * R];
        row_load<T, R>(V + ia * Lp, gl, xa);
        row_load<T, R>(V + ic * Lp, gl, xc);
        if (rotate_row_pair<T, R>(xa, xc, tol)) {
          row_store<T, R>(V + ia * Lp, gl, xa);
          row_store<T, R>(V + ic * Lp, gl, xc);
          mine = true;
        }
        __syncthreads();
      }
    } else {
      T xi[4 * R];
      row_load<T, R>(V + pi * Lp, gl, xi);
      for (int r = 0, ic = b + pi; r < b; ++r, ic = (ic + 1 == 2 * b) ? b : ic + 1) {
        T xc[4 * R];
        row_load<T, R>(V + ic * Lp, gl, xc);
        if (rotate_row_pair<T, R>(xi, xc, tol)) {
          row_store<T, R>(V + ic * Lp, gl, xc);
          mine = true;
        }
        __syncthreads();
      }
      row_store<T, R>(V + pi * Lp, gl, xi);
    }
    if (mine) any_rot = 1;
    __syncthreads();
    ++sw;
    const int rotated = any_rot;
    __syncthreads();
    if (!rotated) converged = true;
    else if (!whole && threadIdx.x == 0) flags[face * max_sweeps + sweep] = 1;
    if (!whole) break;
  } while (!converged && sw < max_sweeps);
  for (int idx = threadIdx.x; idx < nvl * Lp; idx += blockDim.x) {
    const int u = idx / Lp, e = idx - u * Lp;
    const int g = (u < b) ? I * b + u : J * b + (u - b);
    if (g < nv && e < L) Wf[(int64_t)g * L + e] = V[idx];
  }
  if (whole && threadIdx.x == 0) sweeps_used[face] = converged ? sw : max_sweeps + 1;
}

// Long vectors: one workgroup per face, pairs read from global memory.
template <typename T>
__global__ __launch_bounds__(kJacobiThreads) void jacobi_global_kernel(T* __restrict__ W, int nv, int L,
                                                                       int max_sweeps, double tol,
                                                                       int* __restrict__ sweeps_used,
                                                                       const int* __restrict__ prior,
                                                                       int prior_max) {
  constexpr int NW = kJacobiThreads / 64;
  __shared__ int any_rot;
  const int face = blockIdx.x;
  if (prior && prior[face] <= prior_max) {  // converged in an earlier phase: no sweep
    if (threadIdx.x == 0) sweeps_used[face] = 0;
    return;
  }
  T* Wf = W + (int64_t)face * nv * L;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nvp = nv + (nv & 1);
  int sweep = 0;
  bool converged = false;
  while (sweep < max_sweeps) {
    if (threadIdx.x == 0) any_rot = 0;
    __syncthreads();
    for (int round = 0; round < nvp - 1; ++round) {
      for (int pi = wave; pi < nvp / 2; pi += NW) {
        int a, c;
        circle_pair(nvp, round, pi, a, c);
        if (a >= nv || c >= nv) continue;
        T* va = Wf + (int64_t)a * L;
        T* vc = Wf + (int64_t)c * L;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int e = lane; e < L; e += 64) {
          const double x = va[e], y = vc[e];
          al = fma(x, x, al);
          be = fma(y, y, be);
          ga = fma(x, y, ga);
        }
        const Rot q = rotation(wave_total(al), wave_total(be), wave_total(ga), tol);
        if (q.on) {
          for (int e = lane; e < L; e += 64) {
            const double x = va[e], y = vc[e];
            va[e] = static_cast<T>(q.c * x - q.s * y);
            vc[e] = static_cast<T>(q.s * x + q.c * y);
          }
          if (lane == 0) any_rot = 1;
        }
      }
      __syncthreads();
    }
    ++sweep;
    const int any = any_rot;
    __syncthreads();
    if (!any) {
      converged = true;
      break;
    }
  }
  if (threadIdx.x == 0) sweeps_used[face] = converged ? sweep : max_sweeps + 1;
}

// ---- Gram-matrix block step ---------------------------------------------
// One workgroup of four waves per (block pair, face).  The 2b = 32 vectors of
// blocks I and J are staged in LDS; their Gram matrix G = X^T X is formed on
// MFMA (v_mfma_f32_16x16x4f32 for float32 vectors, v_mfma_f64_16x16x4f64 for
// float64; one 16x16 tile per wave, the lower off-diagonal tile mirrored from
// the upper one).  If no pair this visit covers has |g_ac| > tol sqrt(g_aa
// g_cc) in the freshly formed G, the visit ends there (the face's sweep flag
// is left alone).  Otherwise the rotations are run on G alone, in float64:
// each round takes 16 disjoint pairs, computes their angles from G's entries
// and applies G <- J^T G J (one 2x2 block of G per pair of pairs and thread)
// and V <- V J.  The vectors are touched once more, at the end: X <- X V on
// the same MFMA, written back to global memory.  A rotation costs O(32) work
// on G instead of O(L) on the vectors.
//
// Pairs: the first launch of a sweep runs a full round robin over the 32
// vectors (so every pair inside a block is visited once per sweep), the
// others the 16 x 16 pairs between their two blocks in 16 rounds.
//
// A face table (nullable) gives every face its own offset, vector count and
// length; without one, face f is the f-th block of nv x L elements.

constexpr int kGB = 16;        // vectors per block
constexpr int kG2 = 2 * kGB;   // vectors per block pair = Gram order
constexpr int kGld = kG2 + 1;  // row stride of G and V in LDS (doubles): no bank conflicts on columns
constexpr int kGMat = kG2 * kGld;
// LDS head of a visit: NB copies of G in the angle type (float32 for float32
// data; with two copies each round reads one and writes the other, with one
// a round reads, synchronises and writes), V in float64 (updated in place:
// every entry is read and written by one thread only) and a flag word.  The
// four waves' partial Gram tiles (4 x 3 x 4 x 64 values of T) are staged in
// the G and V area before G is formed.
template <typename T, int NB>
__host__ __device__ constexpr size_t gram_g_bytes() {
  return ((size_t)NB * kGMat * sizeof(T) + 15) & ~(size_t)15;
}
// (after the flag word: the rotations of the last two rounds, 2 x 16 pairs
// of (c, s) in the angle type)
constexpr size_t kRotBytes = 2 * 16 * 2 * sizeof(double);
template <typename T, int NB>
__host__ __device__ constexpr size_t gram_head() {
  return gram_g_bytes<T, NB>() + sizeof(double) * kGMat + 16 + kRotBytes;
}
template <typename T, int NB>
__host__ __device__ constexpr bool gram_partials_fit() {
  return sizeof(T) * 4 * 3 * 4 * 64 <= gram_head<T, NB>() - 16;
}

__device__ __forceinline__ JFace face_of(const JFace* tab, int f, int nv, int L) {
  if (tab) return tab[f];
  return JFace{(int64_t)f * nv * L, nv, L};
}

// LDS row stride of the staged vectors: 16-byte reads of 16 rows hit
// distinct banks
template <typename T>
__host__ __device__ __forceinline__ int gram_ldx(int L) {
  return ((L + 15) & ~15) + (sizeof(T) == 4 ? 4 : 2);
}

template <typename T, int NB, bool ST>
__host__ __device__ __forceinline__ size_t gram_lds_bytes(int L) {
  return gram_head<T, NB>() + (ST ? sizeof(T) * (size_t)kG2 * gram_ldx<T>(L) : 0);
}

template <typename T> struct GramMfma;
// Output layout of the 16x16x4 MFMAs: lane L holds column L mod 16 of D, in
// rows row(L / 16, j) for its four values j (float32: 4 (L / 16) + j;
// float64: L / 16 + 4 j).
template <> struct GramMfma<float> {
  typedef f32x4 acc_t;
  typedef float4 vec_t;  // 16-byte global/LDS chunk
  static constexpr int kVec = 4;
  static __device__ __forceinline__ int row(int kq, int j) { return 4 * kq + j; }
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ vec_t zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
};
template <> struct GramMfma<double> {
  typedef f64x4 acc_t;
  typedef double2 vec_t;
  static constexpr int kVec = 2;
  static __device__ __forceinline__ int row(int kq, int j) { return kq + 4 * j; }
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ vec_t zero() { return make_double2(0.0, 0.0); }
};

// 1/sqrt(x) for positive normal float64 x: the hardware estimate and NS
// Newton steps (each squares the relative error).
template <int NS>
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int i = 0; i < NS; ++i) y = y * fma(-0.5 * x * y, y, 1.5);
  return y;
}

// Rotation (cos, sin) that zeroes gamma of the pair with squared norms alpha,
// beta; (1, 0) when |gamma| <= tol sqrt(alpha beta).  With tau = beta - alpha
// and d = sqrt(tau^2 + 4 gamma^2): cos(2 theta) = |tau| / d, cos^2(theta) =
// (1 + cos 2 theta) / 2 and sin(theta) = sign(tau) gamma / (d cos theta): the
// rotation with |theta| <= pi/4.  Computed without branches.
template <int NS>
__device__ __forceinline__ double2 gram_rotation(double al, double be, double ga, double tol2) {
  const bool on = ga * ga > tol2 * al * be;
  const double g = on ? ga : 1.0;  // keeps the arithmetic finite when off
  const double tau = be - al;
  const double r = rsq_nr<NS>(fma(tau, tau, 4.0 * g * g));
  const double h = fma(0.5 * fabs(tau), r, 0.5);
  const double y = rsq_nr<NS>(h);
  const double cs = h * y, sn = (tau >= 0.0 ? g : -g) * r * y;
  return on ? make_double2(cs, sn) : make_double2(1.0, 0.0);
}

// The rotation of rotation() (same test, same annihilating angle up to the
// choice at beta = alpha) through gram_rotation: reciprocal square roots
// refined by two Newton steps instead of a chain of float64 square roots and
// divisions, for the latency-bound refinement rounds.
__device__ __forceinline__ Rot rotation_rsq(double al, double be, double ga, double tol) {
  Rot q{1.0, 0.0, false};
  const double tol2 = tol * tol;
  if (ga != 0.0 && ga * ga > tol2 * al * be) {
    const double2 cs = gram_rotation<2>(al, be, ga, tol2);
    q.c = cs.x;
    q.s = cs.y;
    q.on = true;
  }
  return q;
}

// The same rotation in float32 (the coarse sweeps of float32 data): the
// hardware reciprocal square root without refinement, about 1e-7 relative,
// far below the coarse stopping threshold.  A rotation that is off, or
// whose gamma^2 underflows, is the identity.  The result is selected
// arithmetically so that the compiler keeps the loop free of branches.
__device__ __forceinline__ float2 gram_rotation_f32(float al, float be, float ga, float tol2) {
  const bool on = ga * ga > tol2 * al * be;
  const float g = on ? ga : 1.0f;
  const float tau = be - al;
  const float r = __builtin_amdgcn_rsqf(fmaf(tau, tau, 4.0f * g * g));
  const float h = fmaf(0.5f * fabsf(tau), r, 0.5f);
  const float y = __builtin_amdgcn_rsqf(h);
  const float onf = on ? 1.0f : 0.0f;
  const float cs = fmaf(onf, fmaf(h, y, -1.0f), 1.0f);
  const float sn = onf * ((tau >= 0.0f ? g : -g) * r * y);
  return make_float2(cs, sn);
}

__device__ __forceinline__ void gram_pair(bool full, int r, int P, int& a, int& c) {
  if (full) {
    circle_pair(kG2, r, P, a, c);
  } else {
    a = P;
    c = kGB + ((P + r) & (kGB - 1));
  }
}

// Workgroup -> (face, block pair): workgroups are dealt to the XCDs in turn
// (workgroup w runs on XCD w mod 8), so face f takes the workgroups of XCD
// f mod 8 and its vectors stay in that XCD's L2 from launch to launch.
constexpr int kXcds = 8;

__host__ __device__ __forceinline__ int gram_grid(int nfaces, int npair) {
  return kXcds * ((nfaces + kXcds - 1) / kXcds) * npair;
}

// Adjacent-lane swap (lanes 2i <-> 2i + 1) on the VALU.
__device__ __forceinline__ float swap_pair(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xf, 0xf, false));
}
__device__ __forceinline__ double swap_pair(double v) { return dpp_f64<0xB1>(v); }

// Top-block schedule of a sweep (ntop = 1 or 2 leading blocks, on a face of
// nb >= 2 ntop + 2 blocks; other faces keep the full schedule): only the
// pairs with at least one vector in the leading blocks are visited.  Round r
// < nb - ntop pairs leading block t = pair with trailing block ntop + (r + t)
// mod (nb - ntop), so that the visits of a round touch distinct blocks; with
// two leading blocks one more round visits (0, 1).  The first visit of each
// leading block in a sweep (round 0) and the (0, 1) visit run the full round
// robin over their 32 vectors, which covers the pairs inside the blocks.
// Launches per sweep: nb - ntop (+ 1 for two leading blocks), ntop visits
// each.  Used for the float64 polishing of float32 data once the leading
// blocks hold the vectors of largest norm: the Ritz step that follows needs
// only those to be orthogonal to all others.
__host__ __device__ __forceinline__ bool top_schedule(int ntop, int nb) {
  return (ntop == 1 || ntop == 2) && nb >= 2 * ntop + 2;
}
__host__ __device__ __forceinline__ int top_rounds(int ntop, int nb) { return nb - ntop + (ntop > 1 ? 1 : 0); }

// visit `pair` of round `round`: blocks (I, J) and whether it runs the full
// round robin; false when the slot is idle
__host__ __device__ __forceinline__ bool top_pair(int ntop, int nb, int round, int pair, int& I, int& J,
                                                    bool& full) {
  const int nbot = nb - ntop;
  if (pair >= ntop || round >= top_rounds(ntop, nb)) return false;
  if (round < nbot) {
    I = pair;
    J = ntop + (round + pair) % nbot;
    full = round == 0;
    return true;
  }
  if (pair > 0) return false;
  I = 0;
  J = 1;
  full = true;
  return true;
}

// Rounds of the eight-wave visit with fixed addresses.  The 32 vectors of a
// visit sit in slots 0..31 (block I in 0..15, block J in 16..31).  A round
// rotates 16 fixed pairs of slots; afterwards every element moves to slot
// sigma(slot), so that the same slot pairs hold new pairs of vectors in the
// next round.  Intra rounds (the first 15 of a full visit) pair slots q and
// 15 - q of each block, and sigma keeps slot 0 of a block and cycles its
// slots 1..15 (the circle method on 16 vectors, in both blocks at once):
// every pair inside a block once in 15 rounds.  Cross rounds pair slot i
// with slot 16 + i, and sigma moves the J slots down by one: every (I, J)
// pair once in 16 rounds.  Each phase returns every element to its own slot.
// G is held as one 2 x 2 block ("quad") per pair of slot pairs (k, k2): the
// entries (u_k, u_k2), (u_k, w_k2), (w_k, u_k2), (w_k, w_k2) of pair k's
// slots u_k, w_k and pair k2's, so that a thread updates its quad from the
// quad itself and the rotations of k and k2, and writes each entry to the
// quad and position that hold it in the next round: addresses fixed for the
// whole phase.
struct GSlot {
  int pair, side;  // slot pair holding the slot, and which of its two slots
};
__device__ __forceinline__ GSlot gslot(bool intra, int s) {
  const int b = s >> 4, q = s & 15;
  if (intra) return q < 8 ? GSlot{8 * b + q, 0} : GSlot{8 * b + 15 - q, 1};
  return GSlot{q, b};
}
__device__ __forceinline__ int gslot_of(bool intra, int k, int side) {
  if (intra) return 16 * (k >> 3) + (side ? 15 - (k & 7) : (k & 7));
  return k + 16 * side;
}
__device__ __forceinline__ int gsigma(bool intra, int s) {
  const int q = s & 15;
  if (intra) return (s & 16) | (q == 0 ? 0 : q == 15 ? 1 : q + 1);
  return s < 16 ? s : 16 + ((q - 1) & 15);
}
// element index of entry (slot a, slot b) in the quad array
__device__ __forceinline__ int gquad_index(bool intra, int a, int b) {
  const GSlot x = gslot(intra, a), y = gslot(intra, b);
  return 4 * (16 * x.pair + y.pair) + 2 * x.side + y.side;
}
// vector (0..31) in slot u_k (side 0) or w_k (side 1) of pair k at round r
// of a phase
__device__ __forceinline__ int gslot_vector(bool intra, int k, int side, int r) {
  if (intra) {
    const int q = side ? 15 - (k & 7) : (k & 7);
    int v = q;
    if (q > 0) {
      v = q - 1 - r + 15;  // 1 + ((q - 1 - r) mod 15), r < 15
      if (v >= 15) v -= 15;
      ++v;
    }
    return 16 * (k >> 3) + v;
  }
  return side ? 16 + ((k + r) & 15) : k;
}
template <typename R>
__device__ __forceinline__ void load_quad(const R* p, R (&q)[4]) {
  if constexpr (sizeof(R) == 4) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    q[0] = v.x;
    q[1] = v.y;
    q[2] = v.z;
    q[3] = v.w;
  } else {
    const double2 a = *reinterpret_cast<const double2*>(p), b = *reinterpret_cast<const double2*>(p + 2);
    q[0] = a.x;
    q[1] = a.y;
    q[2] = b.x;
    q[3] = b.y;
  }
}

// Largest of the 64 lanes' non-negative values on the VALU (DPP, the
// pattern of wave_total; lanes a step leaves out read 0, neutral here),
// returned wave-uniform.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, false));
}
__device__ __forceinline__ float wave_max_nonneg(float v) {
  v = fmaxf(v, dpp_f32<0xB1>(v));
  v = fmaxf(v, dpp_f32<0x4E>(v));
  v = fmaxf(v, dpp_f32<0x141>(v));
  v = fmaxf(v, dpp_f32<0x140>(v));
  v = fmaxf(v, dpp_f32<0x142, 0xA>(v));
  v = fmaxf(v, dpp_f32<0x143, 0xC>(v));
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

template <typename T, int NB, bool ST, int NW>
__global__ __launch_bounds__(64 * NW) void jacobi_gram_kernel(T* __restrict__ W, const JFace* __restrict__ faces,
                                                              int nfaces, int npair, int nv_u, int L_u, int round,
                                                              int sweep, int max_sweeps, double tol, float skip2,
                                                              int ntop, int* __restrict__ flags,
                                                              const int* __restrict__ visits) {
  typedef GramMfma<T> M;
  typedef typename M::vec_t vec_t;
  constexpr int VEC = M::kVec;
  constexpr bool F32 = sizeof(T) == 4;
  constexpr int NT = 64 * NW;    // threads of a visit
  constexpr int VPW = kG2 / NW;  // staged vectors per wave
  // G and the angle arithmetic: float32 in the coarse sweeps of float32 data,
  // float64 in the polishing sweeps; V is float64 in both
  typedef typename std::conditional<F32, float, double>::type R;
  static_assert(NB == 1 || NB == 2, "one or two copies of G");
  static_assert(NW == 4 || NW == 8, "four or eight waves per visit");
  static_assert(gram_partials_fit<T, NB>(), "partial tiles exceed the G/V area");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* Gb = reinterpret_cast<R*>(smem_raw);  // G copies at Gb (and Gb + kGMat)
  double* V = reinterpret_cast<double*>(smem_raw + gram_g_bytes<R, NB>());
  int* any_rot = reinterpret_cast<int*>(V + kGMat);
  // ST: the 32 vectors are staged in LDS; otherwise the Gram step and X V
  // read them from global memory (the L2) and the visit needs only the head,
  // so that several visits share a CU
  T* X = reinterpret_cast<T*>(smem_raw + gram_head<R, NB>());

  int f, pair;
  if (visits) {
    // listed visit: face index and slot
    const int v = visits[blockIdx.x];
    if (v < 0) return;
    f = v >> kVisitShift;
    pair = v & ((1 << kVisitShift) - 1);
  } else {
    const int xcd = blockIdx.x % kXcds, m = blockIdx.x / kXcds;
    f = xcd + kXcds * (m / npair);
    pair = m % npair;
    if (f >= nfaces) return;
  }
  const JFace fd = face_of(faces, f, nv_u, L_u);
  const int nv = fd.nv, L = fd.L;
  int nb = (nv + kGB - 1) / kGB;
  nb += nb & 1;
  int I, J;
  bool full = round == 0;
  if (top_schedule(ntop, nb)) {
    if (!top_pair(ntop, nb, round, pair, I, J, full)) return;
  } else {
    if (round >= nb - 1 || pair >= nb / 2) return;
    circle_pair(nb, round, pair, I, J);
  }
  if (sweep > 0 && __int_as_float(flags[f * max_sweeps + sweep - 1]) <= skip2) return;
  const int Lp = (L + 15) & ~15;
  const int ldx = gram_ldx<T>(L);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  T* Wf = W + fd.off;
  auto gvec = [&](int u) { return u < kGB ? I * kGB + u : J * kGB + (u - kGB); };

  if constexpr (ST) {
    // stage the 32 vectors (wave w takes vectors w, w + NW, ...), zero past
    // nv; each lane issues the loads of its vectors before their LDS stores,
    // with clamped addresses and out-of-range values masked
    if (L % VEC == 0 && fd.off % VEC == 0) {
      const int nq = L / VEC;
      // two 64-chunk columns per pass: all loads of a lane in flight at once
      for (int q0 = 0; q0 < nq; q0 += 128) {
        vec_t buf[2][VPW];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int qc = min(q0 + 64 * h + lane, nq - 1);
#pragma unroll
          for (int i = 0; i < VPW; ++i) {
            const int g = gvec(wave + NW * i);
            const vec_t v = *reinterpret_cast<const vec_t*>(Wf + (int64_t)min(g, nv - 1) * L + VEC * qc);
            buf[h][i] = g < nv ? v : M::zero();
          }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int q = q0 + 64 * h + lane;
          if (q < nq) {
#pragma unroll
            for (int i = 0; i < VPW; ++i) *reinterpret_cast<vec_t*>(X + (wave + NW * i) * ldx + VEC * q) = buf[h][i];
          }
        }
      }
    } else {
      for (int e0 = 0; e0 < L; e0 += 64) {
        const int e = e0 + lane, ec = min(e, L - 1);
        T buf[VPW];
#pragma unroll
        for (int i = 0; i < VPW; ++i) {
          const int g = gvec(wave + NW * i);
          const T v = Wf[(int64_t)min(g, nv - 1) * L + ec];
          buf[i] = g < nv ? v : T(0);
        }
        if (e < L) {
#pragma unroll
          for (int i = 0; i < VPW; ++i) X[(wave + NW * i) * ldx + e] = buf[i];
        }
      }
    }
    if (Lp > L) {
      for (int e = tid; e < kG2 * 16; e += NT) {
        const int u = e >> 4, c = L + (e & 15);
        if (c < Lp) X[u * ldx + c] = T(0);
      }
    }
  }
  __syncthreads();

  // G = X^T X.  Wave w takes the 16-element chunks w, w + NW, ... of the
  // vectors and forms the three distinct 16 x 16 tiles (0,0), (0,1), (1,1)
  // of its chunks' contribution: per chunk, 8 operand reads feed 12 MFMAs,
  // and each tile has four independent accumulation chains.  MFMA t of a
  // chunk takes element 4 kq + t of the chunk from the lanes of k-group kq:
  // the chunk's 16 elements in some order, the same for both operands.  The
  // waves' partial tiles meet in LDS (the G and V area, free until here;
  // with eight waves, waves 4-7 first fold theirs into waves 0-3) and are
  // summed in a fixed order.
  {
    typedef typename M::acc_t acc_t;
    acc_t acc[3][4];
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[q][t] = acc_t{0, 0, 0, 0};
    auto mma3 = [&](const T (&a0)[4], const T (&a1)[4]) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        acc[0][t] = M::mma(a0[t], a0[t], acc[0][t]);
        acc[1][t] = M::mma(a0[t], a1[t], acc[1][t]);
        acc[2][t] = M::mma(a1[t], a1[t], acc[2][t]);
      }
    };
    if constexpr (ST) {
      const T* x0 = X + r16 * ldx + 4 * kq;
      const T* x1 = X + (16 + r16) * ldx + 4 * kq;
#pragma unroll 2
      for (int s0 = 16 * wave; s0 < Lp; s0 += 16 * NW) {
        T a0[4], a1[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          a0[t] = x0[s0 + t];
          a1[t] = x1[s0 + t];
        }
        mma3(a0, a1);
      }
    } else {
      // rows r16 of both blocks, elements 4 kq + t of each chunk, from the
      // L2; the next chunk's loads are issued before this chunk's MFMAs
      const int g0 = gvec(r16), g1 = gvec(16 + r16);
      const T* w0 = Wf + (int64_t)min(g0, nv - 1) * L;
      const T* w1 = Wf + (int64_t)min(g1, nv - 1) * L;
      auto fetch = [&](int s0, T (&a0)[4], T (&a1)[4]) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int e = s0 + 4 * kq + t, ec = min(e, L - 1);
          const T v0 = w0[ec], v1 = w1[ec];
          a0[t] = (g0 < nv && e < L) ? v0 : T(0);
          a1[t] = (g1 < nv && e < L) ? v1 : T(0);
        }
      };
      T n0[4], n1[4];
      int s0 = 16 * wave;
      if (s0 < Lp) fetch(s0, n0, n1);
      for (; s0 < Lp; s0 += 16 * NW) {
        T a0[4], a1[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          a0[t] = n0[t];
          a1[t] = n1[t];
        }
        if (s0 + 16 * NW < Lp) fetch(s0 + 16 * NW, n0, n1);
        mma3(a0, a1);
      }
    }
    T* part = reinterpret_cast<T*>(smem_raw);  // [wave][tile][j][lane], waves 0-3
    acc_t sum[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) sum[q] = (acc[q][0] + acc[q][1]) + (acc[q][2] + acc[q][3]);
    if constexpr (NW == 8) {
      if (wave >= 4) {
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) part[(((wave - 4) * 3 + q) * 4 + jj) * 64 + lane] = sum[q][jj];
      }
      __syncthreads();
      // (each of waves 0-3 then reads and rewrites only its own region:
      // no barrier between the read and the write below)
      if (wave < 4) {
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) sum[q][jj] += part[((wave * 3 + q) * 4 + jj) * 64 + lane];
      }
    }
    if (wave < 4) {
#pragma unroll
      for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) part[((wave * 3 + q) * 4 + jj) * 64 + lane] = sum[q][jj];
    }
    __syncthreads();
    // the 768 entries (tile q, value jj, lane ln) summed over the four waves
    constexpr int kPer = (3 * 256 + NT - 1) / NT;
    R gsum[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int e = tid + NT * i;
      if (e < 3 * 256) {
        const int q = e >> 8, jj = (e >> 6) & 3, ln = e & 63;
        gsum[i] = (R)((part[((0 * 3 + q) * 4 + jj) * 64 + ln] + part[((1 * 3 + q) * 4 + jj) * 64 + ln]) +
                      (part[((2 * 3 + q) * 4 + jj) * 64 + ln] + part[((3 * 3 + q) * 4 + jj) * 64 + ln]));
      }
    }
    __syncthreads();
    // lane ln of value jj holds G[16 ti + row(ln / 16, jj)][16 tj + ln mod 16]
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int e = tid + NT * i;
      if (e < 3 * 256) {
        const int q = e >> 8, jj = (e >> 6) & 3, ln = e & 63;
        const int ti = q == 2 ? 1 : 0, tj = q == 0 ? 0 : 1;
        const int row = 16 * ti + M::row(ln >> 4, jj), col = 16 * tj + (ln & 15);
        if (ti != tj || row <= col) {
          if constexpr (NW == 8) {
            // the quads of the first round's slot pairs
            Gb[gquad_index(full, row, col)] = gsum[i];
            Gb[gquad_index(full, col, row)] = gsum[i];
          } else {
            Gb[row * kGld + col] = gsum[i];
            Gb[col * kGld + row] = gsum[i];
          }
        }
      }
    }
    for (int e = tid; e < kG2 * kG2; e += NT) V[(e >> 5) * kGld + (e & 31)] = ((e >> 5) == (e & 31)) ? 1.0 : 0.0;
    if (tid == 0) *any_rot = 0;
  }
  __syncthreads();

  // does any pair of this visit need a rotation?  The largest squared
  // cosine g^2 / (g_aa g_cc) of the pairs this visit covers (0 for zero or
  // non-finite columns) is taken as float bits, whose integer order is the
  // order of non-negative floats, and the visits of a sweep leave the face's
  // largest in its flag word
  const double tol2 = tol * tol;
  {
    float mx = 0.f;
    auto gat = [&](int a, int b) -> R {
      if constexpr (NW == 8)
        return Gb[gquad_index(full, a, b)];
      else
        return Gb[a * kGld + b];
    };
    auto cos2 = [&](int i, int c) {
      const double g = gat(i, c);
      // the hardware reciprocal (about 1e-15 relative): the value only meets thresholds
      const double r = g * g * __builtin_amdgcn_rcp((double)gat(i, i) * (double)gat(c, c));
      return r > 0.0 ? (float)r : 0.f;  // NaN (0 / 0 included) never asks for a rotation
    };
    if (full) {
      for (int e = tid; e < kG2 * kG2; e += NT) {
        const int i = e >> 5, c = e & 31;
        if (i < c) mx = fmaxf(mx, cos2(i, c));
      }
    } else if (tid < kGB * kGB) {
      mx = cos2(tid >> 4, kGB + (tid & 15));
    }
    // one LDS atomic per wave
    mx = wave_max_nonneg(mx);
    if (lane == 0 && mx > (float)tol2) atomicMax(any_rot, __float_as_int(mx));
    __syncthreads();
    if (*any_rot == 0) return;  // the block pair is converged: nothing to do
  }
  if (tid == 0) atomicMax(&flags[f * max_sweeps + sweep], *any_rot);

  if constexpr (NW == 4) {
    // Rounds on G.  Each round reads the current copy of G and writes every
    // entry of the other, so one barrier per round suffices.  Thread (P, P2)
    // (P2 = lane mod 16) computes the rotation of pair P2, takes pair P's from
    // lane P of its wave, writes its own 2x2 block of J^T G J (rows of pair P,
    // columns of pair P2: threads (P, P2) and (P2, P) write mirror blocks, equal
    // up to rounding), and rows P2 and P2 + 16 of V J in the columns of pair P.
    // In float32 the rotation applied to V is renormalised in float64 (first
    // order in cos^2 + sin^2 - 1, exact to 1e-14), so V stays orthogonal to
    // float64 precision whatever the float32 angle arithmetic does.  The work
    // per round is a few dozen instructions per thread: at wave64 on 16-lane
    // SIMDs every instruction costs four cycles, and the instruction count is
    // what bounds the round.
    const int P = tid >> 4, P2 = tid & 15;
    const int nrounds = full ? kG2 - 1 : kGB;
    const R tol2r = (R)tol2;
    const int vr0 = P2 * kGld, vr1 = (P2 + 16) * kGld;
    // V J of a round is applied during the next round (after the barrier that
    // ends it, before the one that ends the next), off the angle arithmetic's
    // path: the entries a thread updates are its own within a round, and the
    // barriers order the updates of one entry across rounds
    int pa = 0, pc = 0;
    double pvc = 1.0, pvs = 0.0;
    auto apply_v = [&]() {
      const double v0a = V[vr0 + pa], v0c = V[vr0 + pc];
      const double v1a = V[vr1 + pa], v1c = V[vr1 + pc];
      V[vr0 + pa] = pvc * v0a - pvs * v0c;
      V[vr0 + pc] = pvs * v0a + pvc * v0c;
      V[vr1 + pa] = pvc * v1a - pvs * v1c;
      V[vr1 + pc] = pvs * v1a + pvc * v1c;
    };
    int cur = 0;
    for (int r = 0; r < nrounds; ++r) {
      const R* G = Gb + (NB == 2 ? cur : 0) * kGMat;
      R* Gn = Gb + (NB == 2 ? cur ^ 1 : 0) * kGMat;
      int a1, c1, a2, c2;
      gram_pair(full, r, P, a1, c1);
      gram_pair(full, r, P2, a2, c2);
      // row offsets on the full-rate 24-bit multiplier
      const int ra1 = __mul24(a1, kGld), rc1 = __mul24(c1, kGld);
      const int ra2 = __mul24(a2, kGld), rc2 = __mul24(c2, kGld);
      const R m00 = G[ra1 + a2], m01 = G[ra1 + c2];
      const R m10 = G[rc1 + a2], m11 = G[rc1 + c2];
      const R al2 = G[ra2 + a2], be2 = G[rc2 + c2], ga2 = G[ra2 + c2];
      if (r > 0) apply_v();
      R c2r, s2r;
      if constexpr (F32) {
        const float2 q2 = gram_rotation_f32(al2, be2, ga2, tol2r);
        c2r = q2.x;
        s2r = q2.y;
      } else {
        const double2 q2 = gram_rotation<2>(al2, be2, ga2, tol2);
        c2r = q2.x;
        s2r = q2.y;
      }
      const R c1r = __shfl(c2r, P), s1r = __shfl(s2r, P);
      const R t00 = c2r * m00 - s2r * m01, t01 = s2r * m00 + c2r * m01;
      const R t10 = c2r * m10 - s2r * m11, t11 = s2r * m10 + c2r * m11;
      const bool own = P == P2 && s1r != R(0);  // the rotation annihilates its own off-diagonal entry
      const R g00 = c1r * t00 - s1r * t10;
      const R g01 = own ? R(0) : c1r * t01 - s1r * t11;
      const R g10 = own ? R(0) : s1r * t00 + c1r * t10;
      const R g11 = s1r * t01 + c1r * t11;
      if constexpr (NB == 1) __syncthreads();  // every read of the round before any write
      Gn[ra1 + a2] = g00;
      Gn[ra1 + c2] = g01;
      Gn[rc1 + a2] = g10;
      Gn[rc1 + c2] = g11;
      pa = a1;
      pc = c1;
      pvc = c1r;
      pvs = s1r;
      if constexpr (F32) {
        const double nf = fma(-0.5, fma(pvc, pvc, pvs * pvs), 1.5);
        pvc *= nf;
        pvs *= nf;
      }
      cur ^= 1;
      __syncthreads();
    }
    apply_v();
    __syncthreads();

  } else {
    // Eight waves: waves 0-3 update G, one quad per thread (thread (k, k2),
    // k = tid / 16, k2 = tid mod 16), with the fixed-address rounds described
    // above; waves 4-7 update V, two rows of one slot pair's two columns per
    // thread, applying each round's rotations during the next round (V keeps
    // the vectors' own numbering: a thread maps its pair's slots to vectors).
    // A G thread computes pair k2's rotation from quad (k2, k2) and takes
    // pair k's from the lane that holds quad (k, k).  Per round and thread:
    // two quad reads, the angle, sixteen multiply-adds and four writes.
    const R tol2r = (R)tol2;
    const bool gw = tid < 256;
    const int k = (tid >> 4) & 15, k2 = tid & 15;
    const int srcl = (17 * k) & 63;  // lane of this wave with quad (k, k)
    R* rot = reinterpret_cast<R*>(reinterpret_cast<unsigned char*>(any_rot) + 16);
    // where this thread's four entries go: after an intra round, after the
    // last intra round (into the cross rounds' quads), after a cross round
    int tgI[4], tgT[4], tgC[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int aI = gsigma(true, gslot_of(true, k, e >> 1)), bI = gsigma(true, gslot_of(true, k2, e & 1));
      tgI[e] = gquad_index(true, aI, bI);
      tgT[e] = gquad_index(false, aI, bI);
      const int aC = gsigma(false, gslot_of(false, k, e >> 1)), bC = gsigma(false, gslot_of(false, k2, e & 1));
      tgC[e] = gquad_index(false, aC, bC);
    }
    const int own4 = 4 * (16 * k + k2), diag4 = 4 * 17 * k2;
    const int vt = tid - 256, vrow = (vt >> 4) * kGld, vp = vt & 15;
    auto apply_v = [&](bool intra, int r, int buf) {
      // the four V entries and the rotation are read together (one LDS
      // round trip, not one per dependent group), then updated
      const int ca = gslot_vector(intra, vp, 0, r), cw = gslot_vector(intra, vp, 1, r);
      double va[2], vw[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int o = vrow + 16 * kGld * h;
        va[h] = V[o + ca];
        vw[h] = V[o + cw];
      }
      double c = (double)rot[buf * 32 + 2 * vp], sn = (double)rot[buf * 32 + 2 * vp + 1];
      if constexpr (F32) {
        // float32 angles renormalised in float64 (first order in
        // c^2 + s^2 - 1, exact to 1e-14): V stays orthogonal to float64
        // precision whatever the float32 arithmetic does
        const double nf = fma(-0.5, fma(c, c, sn * sn), 1.5);
        c *= nf;
        sn *= nf;
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int o = vrow + 16 * kGld * h;
        V[o + ca] = c * va[h] - sn * vw[h];
        V[o + cw] = sn * va[h] + c * vw[h];
      }
    };
    int cur = 0, rr = 0;
    // one round with write targets tg; the V waves apply round rr - 1 (of
    // phase pv_intra, round pv_r within it; pv_r < 0: none)
    auto do_round = [&](const int (&tg)[4], bool pv_intra, int pv_r) {
      const R* G = Gb + (NB == 2 ? cur : 0) * 1024;
      R* Gn = Gb + (NB == 2 ? cur ^ 1 : 0) * 1024;
      R g[4], c2r = R(1), s2r = R(0);
      if (gw) {
        R m[4], d[4];
        load_quad(G + own4, m);
        load_quad(G + diag4, d);
        if constexpr (F32) {
          const float2 q2 = gram_rotation_f32(d[0], d[3], d[1], tol2r);
          c2r = q2.x;
          s2r = q2.y;
        } else {
          const double2 q2 = gram_rotation<2>(d[0], d[3], d[1], tol2);
          c2r = q2.x;
          s2r = q2.y;
        }
        const R c1r = __shfl(c2r, srcl), s1r = __shfl(s2r, srcl);
        const R t00 = c2r * m[0] - s2r * m[1], t01 = s2r * m[0] + c2r * m[1];
        const R t10 = c2r * m[2] - s2r * m[3], t11 = s2r * m[2] + c2r * m[3];
        const bool own = k == k2 && s1r != R(0);  // the rotation annihilates its own off-diagonal entries
        g[0] = c1r * t00 - s1r * t10;
        g[1] = own ? R(0) : c1r * t01 - s1r * t11;
        g[2] = own ? R(0) : s1r * t00 + c1r * t10;
        g[3] = s1r * t01 + c1r * t11;
      } else if (pv_r >= 0) {
        apply_v(pv_intra, pv_r, (rr - 1) & 1);
      }
      if constexpr (NB == 1) __syncthreads();  // every read of the round before any write
      if (gw) {
#pragma unroll
        for (int e = 0; e < 4; ++e) Gn[tg[e]] = g[e];
        if (tid < 16) {
          rot[(rr & 1) * 32 + 2 * k2] = c2r;
          rot[(rr & 1) * 32 + 2 * k2 + 1] = s2r;
        }
      }
      cur ^= 1;
      ++rr;
      __syncthreads();
    };
    if (full) {
      do_round(tgI, true, -1);
      for (int r = 1; r < kGB - 2; ++r) do_round(tgI, true, r - 1);
      do_round(tgT, true, kGB - 3);
      do_round(tgC, true, kGB - 2);
    } else {
      do_round(tgC, false, -1);
    }
    for (int r = 1; r < kGB; ++r) do_round(tgC, false, r - 1);
    if (!gw) apply_v(false, kGB - 1, (rr - 1) & 1);
    __syncthreads();
  }

  // X <- X V: D[c][e] = sum_a V[a][c] X[a][e]; wave w takes the 16-element
  // column tiles te = w, w + NW, ... and both row tiles tc of each.
  T va[2][8];
#pragma unroll
  for (int tc = 0; tc < 2; ++tc)
#pragma unroll
    for (int s = 0; s < 8; ++s) va[tc][s] = (T)V[(4 * s + kq) * kGld + 16 * tc + r16];
  // (without staging: tile te's 8 rows per lane come from the L2, the next
  // tile's issued before this tile's MFMAs; the tiles of one launch are
  // disjoint column ranges, read before they are written)
  T nb8[8];
  auto fetch_tile = [&](int te, T (&xb)[8]) {
    const int e = 16 * te + r16, ec = min(e, L - 1);
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int g = gvec(4 * s + kq);
      const T v = Wf[(int64_t)min(g, nv - 1) * L + ec];
      xb[s] = (g < nv && e < L) ? v : T(0);
    }
  };
  if constexpr (!ST) {
    if (wave < (Lp >> 4)) fetch_tile(wave, nb8);
  }
  for (int te = wave; te < (Lp >> 4); te += NW) {
    T xb[8];
    if constexpr (ST) {
#pragma unroll
      for (int s = 0; s < 8; ++s) xb[s] = X[(4 * s + kq) * ldx + 16 * te + r16];
    } else {
#pragma unroll
      for (int s = 0; s < 8; ++s) xb[s] = nb8[s];
      if (te + NW < (Lp >> 4)) fetch_tile(te + NW, nb8);
    }
    const int e = 16 * te + r16;
    // the two row tiles as interleaved, independent MFMA chains
    typename M::acc_t acc[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
    for (int s = 0; s < 8; ++s) {
#pragma unroll
      for (int tc = 0; tc < 2; ++tc) acc[tc] = M::mma(va[tc][s], xb[s], acc[tc]);
    }
    if (e < L) {
#pragma unroll
      for (int tc = 0; tc < 2; ++tc)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int g = gvec(16 * tc + M::row(kq, j));
          if (g < nv) Wf[(int64_t)g * L + e] = acc[tc][j];
        }
    }
  }
}

__global__ void zero_ints_kernel(int* __restrict__ x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0;
}

// sweeps_used[l] from the per-sweep rotation flags: the first sweep without a
// rotation ends the iteration (it is counted); none means not converged.
__global__ void count_sweeps_kernel(const int* __restrict__ flags, int p, int max_sweeps, float skip2,
                                    int* __restrict__ sweeps_used, const int* __restrict__ prior = nullptr,
                                    int prior_max = 0) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= p) return;
  if (prior && prior[l] <= prior_max) {  // skipped: converged in an earlier phase
    sweeps_used[l] = 0;
    return;
  }
  int u = max_sweeps + 1;
  for (int s = 0; s < max_sweeps; ++s) {
    if (__int_as_float(flags[l * max_sweeps + s]) <= skip2) {
      u = s + 1;
      break;
    }
  }
  sweeps_used[l] = u;
}

// W face l (nv x L, vector-major) <- transpose of Ah face l (n1 x n2 column
// major), i.e. vector i = row i.  32x32 tiles through LDS.
template <typename T>
__global__ __launch_bounds__(256) void transpose_faces_kernel(const T* __restrict__ Ah,
                                                              T* __restrict__ W, int n1, int n2) {
  __shared__ T tile[32][33];
  const int l = blockIdx.z;
  const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
  const T* src = Ah + (int64_t)l * n1 * n2;
  T* dst = W + (int64_t)l * n1 * n2;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int i = i0 + tx, j = j0 + r;
    if (i < n1 && j < n2) tile[r][tx] = src[i + (int64_t)j * n1];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = i0 + r, j = j0 + tx;
    if (i < n1 && j < n2) dst[j + (int64_t)i * n2] = tile[tx][r];
  }
}

// Norms of the converged vectors: one wave per vector, sig[f * nv + j];
// rank (when given) is cleared for the selection that follows.
template <typename T>
__global__ __launch_bounds__(256) void norms_kernel(const T* __restrict__ W, int nv, int L, double* __restrict__ sig,
                                                    int* __restrict__ rank) {
  const int face = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= nv) return;
  const T* v = W + ((int64_t)face * nv + j) * L;
  double acc = 0.0;
  for (int e = lane; e < L; e += 64) {
    const double x = (double)v[e];
    acc = fma(x, x, acc);
  }
  acc = wave_total(acc);
  if (lane == 0) {
    sig[(int64_t)face * nv + j] = sqrt(acc);
    if (rank) rank[(int64_t)face * nv + j] = 0;
  }
}

// Descending order of each face's norms (ties by index) and the leading
// vectors normalised into F (L x k x p); a face keeps min(k, kface[f] +
// extra) vectors when kface is given, the rest of its k columns are zero, as
// is a zero vector.  Workgroup (f, c) writes the columns [16 c, 16 c + 16) of
// face f (each workgroup ranks the face's norms itself).
constexpr int kFinCols = 16;

// One face: Wf its nv vectors of L, sigf their norms, Ff its k columns of L,
// sig_sortedf (nullable) its k sorted norms; kf of the k columns are kept.
template <typename T>
__device__ __forceinline__ void finalize_face(const T* __restrict__ Wf, const double* __restrict__ sigf, int nv, int L,
                                              int k, int kf, T* __restrict__ Ff, double* __restrict__ sig_sortedf,
                                              int r0, double* sig, int* order) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = threadIdx.x; j < nv; j += 256) sig[j] = sigf[j];
  if (threadIdx.x < kFinCols) order[threadIdx.x] = -1;  // stays -1 only for NaN norms
  __syncthreads();
  for (int j = threadIdx.x; j < nv; j += 256) {
    const double v = sig[j];
    int r = 0;
    for (int i = 0; i < nv; ++i) r += (sig[i] > v) || (sig[i] == v && i < j);
    if (r >= r0 && r < min(k, r0 + kFinCols)) order[r - r0] = j;
  }
  __syncthreads();
  for (int r = r0 + wave; r < min(k, r0 + kFinCols); r += 4) {
    T* dst = Ff + (int64_t)r * L;
    const int j = order[r - r0];
    if (r >= kf || j < 0) {
      for (int e = lane; e < L; e += 64) dst[e] = T(0);
      if (sig_sortedf && lane == 0) sig_sortedf[r] = 0.0;
      continue;
    }
    const double v = sig[j];
    if (sig_sortedf && lane == 0) sig_sortedf[r] = v;
    const double inv = v > 0.0 ? 1.0 / v : 0.0;
    for (int e = lane; e < L; e += 64) dst[e] = static_cast<T>(inv * (double)Wf[(int64_t)j * L + e]);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void finalize_kernel(const T* __restrict__ W, const double* __restrict__ sig_all,
                                                       int nv, int L, int k, const int* __restrict__ kface,
                                                       int extra, T* __restrict__ F,
                                                       double* __restrict__ sig_sorted) {
  extern __shared__ double fin_sig[];  // nv doubles
  __shared__ int order[kFinCols];
  const int face = blockIdx.x;
  const int kf = kface ? max(0, min(k, kface[face] + extra)) : k;
  finalize_face<T>(W + (int64_t)face * nv * L, sig_all + (int64_t)face * nv, nv, L, k, kf, F + (int64_t)face * k * L,
                   sig_sorted ? sig_sorted + (int64_t)face * k : nullptr, blockIdx.y * kFinCols, fin_sig, order);
}

// ---- global selection of *_Q-SVDII (Alg. 4.2) ------------------------------
// rank[i] += how many of sig[c], c in this block's column range, come before
// sig[i] in the descending order of all n values (ties by index; the values
// are face-major, face f's at f * nv + j).  Every rank lies in [0, n - 1]
// whatever the values are.
__global__ __launch_bounds__(256) void rank_kernel(const double* __restrict__ sig, int n, int cols,
                                                   int* __restrict__ rank) {
  __shared__ double tile[256];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const double v = i < n ? sig[i] : 0.0;
  const int c_begin = blockIdx.y * cols, c_end = min(n, c_begin + cols);
  int r = 0;
  for (int c0 = c_begin; c0 < c_end; c0 += 256) {
    __syncthreads();
    tile[threadIdx.x] = c0 + (int)threadIdx.x < c_end ? sig[c0 + threadIdx.x] : 0.0;
    __syncthreads();
    const int cn = min(256, c_end - c0);
    for (int c = 0; c < cn; ++c) {
      const double w = tile[c];
      r += (w > v) || (w == v && c0 + c < i);
    }
  }
  if (i < n && r) atomicAdd(&rank[i], r);
}

// One workgroup: the squared values scattered by rank into descending order
// (e2, n doubles), their running sum, K = the first count whose running sum
// reaches gamma times the total (n when rounding leaves it short), and
// rho[f] = how many of face f's values are among the first K.
constexpr int kSelThreads = 1024;

__global__ __launch_bounds__(kSelThreads) void select_kernel(const double* __restrict__ sig,
                                                             const int* __restrict__ rank, int n, int p, int nv,
                                                             double gamma, double* __restrict__ e2,
                                                             int* __restrict__ rho) {
  __shared__ double part[kSelThreads];
  __shared__ int kfirst;
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += kSelThreads) {
    const double v = sig[i];
    e2[rank[i]] = v * v;
  }
  if (tid == 0) kfirst = n;
  __syncthreads();
  // chunk totals, an inclusive scan of them, then each chunk walked again
  const int chunk = (n + kSelThreads - 1) / kSelThreads;
  const int b0 = min(n, tid * chunk), b1 = min(n, b0 + chunk);
  double s = 0.0;
  for (int i = b0; i < b1; ++i) s += e2[i];
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < kSelThreads; off <<= 1) {
    const double add = tid >= off ? part[tid - off] : 0.0;
    __syncthreads();
    part[tid] += add;
    __syncthreads();
  }
  const double target = gamma * part[kSelThreads - 1];
  double run = tid > 0 ? part[tid - 1] : 0.0;
  for (int i = b0; i < b1; ++i) {
    run += e2[i];
    if (run >= target) {
      atomicMin(&kfirst, i + 1);
      break;
    }
  }
  __syncthreads();
  const int K = kfirst;
  // one wave per face
  const int lane = tid & 63;
  for (int f = tid >> 6; f < p; f += kSelThreads / 64) {
    int c = 0;
    for (int j = lane; j < nv; j += 64) c += rank[(int64_t)f * nv + j] < K;
    c = (int)wave_total((double)c);  // exact: counts stay far below 2^53
    if (lane == 0) rho[f] = c;
  }
}

// Rayleigh-Ritz step of the truncation: Jacobi on the k columns of Y (m1 x
// k, face-major) with every rotation also applied to the k columns of F (m2
// x k); then norms, descending order and the leading kout of the results
// (type TO): s (kout), Other = Y / s, Fo = F, Ys = Y, in that order, each
// face's outputs kout apart.  With kface given a face works on min(k,
// kface[f] + extra) columns (the rest are zero) and keeps min(kout,
// kface[f]); its other output columns are zero.  The columns stay in global
// memory (the form for k columns that do not fit in LDS); 16 waves per face,
// one pair per wave at a time.
constexpr int kRefineWaves = 16;

template <typename T, typename TO>
__global__ __launch_bounds__(64 * kRefineWaves) void refine_kernel(T* __restrict__ Y, T* __restrict__ F, int m1,
                                                     int m2, int k, int kout, const int* __restrict__ kface,
                                                     int extra, double tol, int max_sweeps,
                                                     TO* __restrict__ s_out, TO* __restrict__ Other,
                                                     TO* __restrict__ Fo, TO* __restrict__ Ys) {
  extern __shared__ double sig[];  // k doubles, then k ints
  int* order = reinterpret_cast<int*>(sig + k);
  __shared__ int any_rot;
  const int face = blockIdx.x;
  T* Yf = Y + (int64_t)face * m1 * k;
  T* Ff = F + (int64_t)face * m2 * k;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kf = kface ? max(0, min(k, kface[face] + extra)) : k;  // columns past kf are zero
  const int ko = kface ? max(0, min(kout, kface[face])) : kout;     // kept columns
  const int kp = kf + (kf & 1);
  for (int sweep = 0; sweep < max_sweeps && kf > 1; ++sweep) {
    if (threadIdx.x == 0) any_rot = 0;
    __syncthreads();
    for (int r = 0; r < kp - 1; ++r) {
      for (int pi = wave; pi < kp / 2; pi += kRefineWaves) {
        int a, c;
        circle_pair(kp, r, pi, a, c);
        if (a >= kf || c >= kf) continue;
        T* ya = Yf + (int64_t)a * m1;
        T* yc = Yf + (int64_t)c * m1;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int e = lane; e < m1; e += 64) {
          const double x = ya[e], y = yc[e];
          al = fma(x, x, al);
          be = fma(y, y, be);
          ga = fma(x, y, ga);
        }
        const Rot q = rotation_rsq(wave_total(al), wave_total(be), wave_total(ga), tol);
        if (q.on) {
          for (int e = lane; e < m1; e += 64) {
            const double x = ya[e], y = yc[e];
            ya[e] = static_cast<T>(q.c * x - q.s * y);
            yc[e] = static_cast<T>(q.s * x + q.c * y);
          }
          T* fa = Ff + (int64_t)a * m2;
          T* fc = Ff + (int64_t)c * m2;
          for (int e = lane; e < m2; e += 64) {
            const double x = fa[e], y = fc[e];
            fa[e] = static_cast<T>(q.c * x - q.s * y);
            fc[e] = static_cast<T>(q.s * x + q.c * y);
          }
          if (lane == 0) any_rot = 1;
        }
      }
      __syncthreads();
    }
    const int any = any_rot;
    __syncthreads();
    if (!any) break;
  }
  for (int j = wave; j < k; j += kRefineWaves) {
    double acc = 0.0;
    for (int e = lane; e < m1; e += 64) {
      const double x = Yf[(int64_t)j * m1 + e];
      acc = fma(x, x, acc);
    }
    acc = wave_total(acc);
    if (lane == 0) sig[j] = sqrt(acc);
  }
  for (int r = threadIdx.x; r < k; r += 64 * kRefineWaves) order[r] = -1;
  __syncthreads();
  for (int j = threadIdx.x; j < k; j += 64 * kRefineWaves) {
    const double v = sig[j];
    int r = 0;
    for (int i = 0; i < k; ++i) r += (sig[i] > v) || (sig[i] == v && i < j);
    order[r] = j;
  }
  __syncthreads();
  for (int r = wave; r < kout; r += kRefineWaves) {
    // equal ranks arise only from NaN norms; such a slot reads column r
    const int j = order[r] >= 0 && order[r] < k ? order[r] : r;
    const bool keep = r < ko;
    const double v = keep ? sig[j] : 0.0;
    const double inv = v > 0.0 ? 1.0 / v : 0.0;
    if (lane == 0) s_out[(int64_t)face * kout + r] = static_cast<TO>(v);
    const T* yj = Yf + (int64_t)j * m1;
    TO* o = Other + ((int64_t)face * kout + r) * m1;
    TO* ys = Ys + ((int64_t)face * kout + r) * m1;
    for (int e = lane; e < m1; e += 64) {
      const double x = keep ? (double)yj[e] : 0.0;
      ys[e] = static_cast<TO>(x);
      o[e] = static_cast<TO>(inv * x);
    }
    const T* fj = Ff + (int64_t)j * m2;
    TO* fo = Fo + ((int64_t)face * kout + r) * m2;
    for (int e = lane; e < m2; e += 64) fo[e] = static_cast<TO>(keep ? (double)fj[e] : 0.0);
  }
}

// The float32 -> float64 copy of the Jacobi vectors for the top-block
// polishing sweeps, in three launches: the squared norm of every vector
// (one wave per vector), the target position of every vector (one workgroup
// per face: the ntop16 of largest norm, ties by index and a NaN norm counting
// as the smallest, go to the front in descending order of norm, the others
// follow in their own order), and the permuted copy (one wave per vector).
// Per-face arrays (norms, positions) are ld entries apart.
__global__ __launch_bounds__(256) void top_norms_kernel(const float* __restrict__ W32, const JFace* __restrict__ faces,
                                                        int nv_u, int L_u, int ld, double* __restrict__ nrm) {
  const JFace fd = face_of(faces, blockIdx.y, nv_u, L_u);
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (j >= fd.nv) return;
  const float* v = W32 + fd.off + (int64_t)j * fd.L;
  double acc = 0.0;
  for (int e = lane; e < fd.L; e += 64) {
    const double x = (double)v[e];
    acc = fma(x, x, acc);
  }
  acc = wave_total(acc);
  if (lane == 0) nrm[(int64_t)blockIdx.y * ld + j] = acc == acc ? acc : -1.0;
}

__global__ __launch_bounds__(256) void top_perm_kernel(const double* __restrict__ nrm_g, const JFace* __restrict__ faces,
                                                       int nv_u, int L_u, int ld, int ntop16, int* __restrict__ pos_g) {
  extern __shared__ double tp_smem[];  // nv norms, then nv ranks
  const int nv = face_of(faces, blockIdx.x, nv_u, L_u).nv;
  double* nrm = tp_smem;
  int* rank = reinterpret_cast<int*>(tp_smem + nv);
  for (int j = threadIdx.x; j < nv; j += 256) nrm[j] = nrm_g[(int64_t)blockIdx.x * ld + j];
  __syncthreads();
  for (int j = threadIdx.x; j < nv; j += 256) {
    const double v = nrm[j];
    int r = 0;
    for (int i = 0; i < nv; ++i) r += (nrm[i] > v) || (nrm[i] == v && i < j);
    rank[j] = r;
  }
  __syncthreads();
  const int nt = min(ntop16, nv);
  for (int j = threadIdx.x; j < nv; j += 256) {
    int to = rank[j];
    if (to >= nt) {  // after the leading nt, in index order
      int c = 0;
      for (int i = 0; i < j; ++i) c += rank[i] >= nt;
      to = nt + c;
    }
    pos_g[(int64_t)blockIdx.x * ld + j] = to;
  }
}

__global__ __launch_bounds__(256) void top_copy_kernel(const float* __restrict__ W32, double* __restrict__ W64,
                                                       const JFace* __restrict__ faces, int nv_u, int L_u, int ld,
                                                       const int* __restrict__ pos_g) {
  const JFace fd = face_of(faces, blockIdx.y, nv_u, L_u);
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (j >= fd.nv) return;
  const int to = pos_g[(int64_t)blockIdx.y * ld + j];
  const float* src = W32 + fd.off + (int64_t)j * fd.L;
  double* dst = W64 + fd.off + (int64_t)to * fd.L;
  for (int e = lane; e < fd.L; e += 64) dst[e] = (double)src[e];
}

// float32 -> float64 copy of the Jacobi vectors (the float64 polishing sweeps)
__global__ __launch_bounds__(256) void widen_kernel(const float* __restrict__ x, double* __restrict__ y,
                                                    int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = (double)x[i];
}

// Y(:, c) = Ah_l^T F(:, c) (Ah face n1 x n2, F n1 x k, Y n2 x k) with float64
// accumulation: one wave per column j2 of the face, lanes over i.  One face:
// a its matrix, f its F, y its Y.
template <typename TA>
__device__ __forceinline__ void factor_t_face(const TA* __restrict__ a0, const double* __restrict__ f,
                                              double* __restrict__ y, int n1, int n2, int k, int j2) {
  const int lane = threadIdx.x & 63;
  if (j2 >= n2) return;
  const TA* a = a0 + (int64_t)j2 * n1;
  for (int c0 = 0; c0 < k; c0 += 8) {
    double acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = 0.0;
    for (int i = lane; i < n1; i += 64) {
      const double x = (double)a[i];
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (c0 + c < k) acc[c] = fma(x, f[(int64_t)(c0 + c) * n1 + i], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const double t = wave_total(acc[c]);
      if (lane == 0 && c0 + c < k) y[(int64_t)(c0 + c) * n2 + j2] = t;
    }
  }
}

template <typename TA>
__global__ __launch_bounds__(256) void factor_t_kernel(const TA* __restrict__ Ah, const double* __restrict__ F,
                                                       double* __restrict__ Y, int n1, int n2, int k) {
  const int face = blockIdx.y;
  factor_t_face<TA>(Ah + (int64_t)face * n1 * n2, F + (int64_t)face * n1 * k, Y + (int64_t)face * n2 * k, n1, n2, k,
                    blockIdx.x * 4 + (threadIdx.x >> 6));
}


// Y (n1 x k per face) = Ah_l (n1 x n2) F_l (n2 x k) with float64
// accumulation: a workgroup takes 64 rows and 16 columns; its four waves take
// quarters of the j range (lane = row, coalesced loads of Ah), stage their
// chunks of F in LDS (read back as broadcasts) and sum their partials
// through LDS at the end.  One face: a its matrix, f its F, y its Y; rows
// from 64 bx, columns from c0.
constexpr int kFactorJC = 32;
struct FactorRowsLds {
  double Fs[4][kFactorJC][16];
  double red[3][16][64];
};

template <typename TA>
__device__ __forceinline__ void factor_rows_face(const TA* __restrict__ a, const double* __restrict__ f,
                                                 double* __restrict__ y, int n1, int n2, int k, int bx, int c0,
                                                 FactorRowsLds& sm) {
  constexpr int JC = kFactorJC;
  const int kc = min(16, k - c0);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = bx * 64 + lane;
  const int jq = (n2 + 3) / 4;
  const int jb = wave * jq, je = min(n2, jb + jq);
  double acc[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) acc[c] = 0.0;
  const int nchunk = (jq + JC - 1) / JC;  // the same for every wave
  for (int ch = 0; ch < nchunk; ++ch) {
    const int j0 = jb + ch * JC;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < JC * 16 / 64; ++t) {
      const int e = lane + 64 * t, jj = e >> 4, c = e & 15;
      const int jg = j0 + jj;
      sm.Fs[wave][jj][c] = (jg < je && c < kc) ? f[(int64_t)(c0 + c) * n2 + jg] : 0.0;
    }
    __syncthreads();
    // the chunk's 32 loads of this row issued together (clamped addresses;
    // rows of F past je are zero in LDS, so the clamped values add nothing)
    const int ic = min(i, n1 - 1);
    double xs[JC];
#pragma unroll
    for (int jj = 0; jj < JC; ++jj) xs[jj] = (double)a[ic + (int64_t)min(j0 + jj, n2 - 1) * n1];
#pragma unroll
    for (int jj = 0; jj < JC; ++jj)
#pragma unroll
      for (int c = 0; c < 16; ++c) acc[c] = fma(xs[jj], sm.Fs[wave][jj][c], acc[c]);
  }
  if (wave > 0) {
#pragma unroll
    for (int c = 0; c < 16; ++c) sm.red[wave - 1][c][lane] = acc[c];
  }
  __syncthreads();
  if (wave == 0 && i < n1) {
#pragma unroll
    for (int c = 0; c < 16; ++c)
      if (c < kc)
        y[(int64_t)(c0 + c) * n1 + i] = acc[c] + sm.red[0][c][lane] + sm.red[1][c][lane] + sm.red[2][c][lane];
  }
}

template <typename TA>
__global__ __launch_bounds__(256) void factor_rows_kernel(const TA* __restrict__ Ah, const double* __restrict__ F,
                                                          double* __restrict__ Y, int n1, int n2, int k) {
  __shared__ FactorRowsLds sm;
  const int face = blockIdx.y;
  factor_rows_face<TA>(Ah + (int64_t)face * n1 * n2, F + (int64_t)face * n2 * k, Y + (int64_t)face * n1 * k, n1, n2,
                       k, blockIdx.x, blockIdx.z * 16, sm);
}

// The refinement of refine_kernel with the k columns of Y and F of the face
// held in LDS and one wave per pair (16 waves): the face's k columns cost
// 8 k (m1 + m2) bytes.  A face works on min(k, kface[f] + extra) columns
// when kface is given (the rest are zero, never rotate, and sort last) and
// keeps min(kout, kface[f]) of them.
// FG: only Y is held in LDS and F is rotated in place in global memory (the
// L2), for faces whose k columns of both do not fit.
// One face: yg its k columns of Y (m1), fg its k columns of F (m2), kf
// columns worked on, ko kept; outputs s_f (kout), other_f, ys_f (kout x m1),
// fo_f (kout x m2).  rl_smem: the dynamic LDS of the form.
template <typename TO, bool FG>
__device__ __forceinline__ void refine_face(const double* __restrict__ yg, double* __restrict__ fg, int m1, int m2,
                                            int k, int kout, int kf, int ko, double tol, int max_sweeps,
                                            TO* __restrict__ s_f, TO* __restrict__ other_f, TO* __restrict__ fo_f,
                                            TO* __restrict__ ys_f, double* rl_smem, int& any_rot) {
  double* Yf = rl_smem;  // k columns of m1
  double* Ff = FG ? fg : Yf + (int64_t)k * m1;  // k columns of m2
  double* sig = FG ? Yf + (int64_t)k * m1 : Ff + (int64_t)k * m2;
  int* order = reinterpret_cast<int*>(sig + k);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < k * m1; e += 1024) Yf[e] = yg[e];
  if constexpr (!FG) {
    for (int e = tid; e < k * m2; e += 1024) Ff[e] = fg[e];
  }
  __syncthreads();
  const int kp = kf + (kf & 1);
  for (int sweep = 0; sweep < max_sweeps && kf > 1; ++sweep) {
    if (tid == 0) any_rot = 0;
    __syncthreads();
    for (int r = 0; r < kp - 1; ++r) {
      for (int pi = wave; pi < kp / 2; pi += 16) {
        int a, c;
        circle_pair(kp, r, pi, a, c);
        if (a >= kf || c >= kf) continue;
        double* ya = Yf + (int64_t)a * m1;
        double* yc = Yf + (int64_t)c * m1;
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll 4
        for (int e = lane; e < m1; e += 64) {
          const double x = ya[e], y = yc[e];
          al = fma(x, x, al);
          be = fma(y, y, be);
          ga = fma(x, y, ga);
        }
        const Rot q = rotation_rsq(wave_total(al), wave_total(be), wave_total(ga), tol);
        if (q.on) {
#pragma unroll 4
          for (int e = lane; e < m1; e += 64) {
            const double x = ya[e], y = yc[e];
            ya[e] = q.c * x - q.s * y;
            yc[e] = q.s * x + q.c * y;
          }
          double* fa = Ff + (int64_t)a * m2;
          double* fc = Ff + (int64_t)c * m2;
#pragma unroll 4
          for (int e = lane; e < m2; e += 64) {
            const double x = fa[e], y = fc[e];
            fa[e] = q.c * x - q.s * y;
            fc[e] = q.s * x + q.c * y;
          }
          if (lane == 0) any_rot = 1;
        }
      }
      __syncthreads();
    }
    const int any = any_rot;
    __syncthreads();
    if (!any) break;
  }
  for (int c = wave; c < k; c += 16) {
    double acc = 0.0;
    for (int e = lane; e < m1; e += 64) {
      const double x = Yf[(int64_t)c * m1 + e];
      acc = fma(x, x, acc);
    }
    acc = wave_total(acc);
    if (lane == 0) sig[c] = sqrt(acc);
  }
  for (int r = tid; r < k; r += 1024) order[r] = -1;
  __syncthreads();
  for (int c = tid; c < k; c += 1024) {
    const double v = sig[c];
    int r = 0;
    for (int i = 0; i < k; ++i) r += (sig[i] > v) || (sig[i] == v && i < c);
    order[r] = c;
  }
  __syncthreads();
  for (int r = wave; r < kout; r += 16) {
    // equal ranks arise only from NaN norms; such a slot reads column r
    const int c = order[r] >= 0 && order[r] < k ? order[r] : r;
    const bool keep = r < ko;
    const double v = keep ? sig[c] : 0.0;
    const double inv = v > 0.0 ? 1.0 / v : 0.0;
    if (lane == 0) s_f[r] = static_cast<TO>(v);
    TO* o = other_f + (int64_t)r * m1;
    TO* ys = ys_f + (int64_t)r * m1;
    for (int e = lane; e < m1; e += 64) {
      const double x = keep ? Yf[(int64_t)c * m1 + e] : 0.0;
      ys[e] = static_cast<TO>(x);
      o[e] = static_cast<TO>(inv * x);
    }
    TO* fo = fo_f + (int64_t)r * m2;
    for (int e = lane; e < m2; e += 64) fo[e] = static_cast<TO>(keep ? Ff[(int64_t)c * m2 + e] : 0.0);
  }
}

template <typename TO, bool FG>
__global__ __launch_bounds__(1024) void refine_lds_kernel(const double* __restrict__ Yg, double* __restrict__ Fg,
                                                          int m1, int m2, int k, int kout,
                                                          const int* __restrict__ kface, int extra, double tol,
                                                          int max_sweeps, TO* __restrict__ s_out,
                                                          TO* __restrict__ Other, TO* __restrict__ Fo,
                                                          TO* __restrict__ Ys) {
  extern __shared__ double rl_smem[];
  __shared__ int any_rot;
  const int face = blockIdx.x;
  const int kf = kface ? max(0, min(k, kface[face] + extra)) : k;
  const int ko = kface ? max(0, min(kout, kface[face])) : kout;
  refine_face<TO, FG>(Yg + (int64_t)face * m1 * k, Fg + (int64_t)face * m2 * k, m1, m2, k, kout, kf, ko, tol,
                      max_sweeps, s_out + (int64_t)face * kout, Other + (int64_t)face * kout * m1,
                      Fo + (int64_t)face * kout * m2, Ys + (int64_t)face * kout * m1, rl_smem, any_rot);
}

// ---- the finishing steps of many faces of different shapes in one launch each
// (the batched form): a device table of FinFace entries (internal.hpp).
__global__ __launch_bounds__(256) void fin_norms_kernel(const FinFace* __restrict__ tab) {
  const FinFace t = tab[blockIdx.y];
  const int nv = min(t.n1, t.n2), L = max(t.n1, t.n2);
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (j >= nv) return;
  const double* v = t.w + (int64_t)j * L;
  double acc = 0.0;
  for (int e = lane; e < L; e += 64) acc = fma(v[e], v[e], acc);
  acc = wave_total(acc);
  if (lane == 0) t.sig[j] = sqrt(acc);
}

__global__ __launch_bounds__(256) void fin_finalize_kernel(const FinFace* __restrict__ tab) {
  extern __shared__ double fin_sig_g[];
  __shared__ int order[kFinCols];
  const FinFace t = tab[blockIdx.x];
  const int r0 = blockIdx.y * kFinCols;
  if (r0 >= t.kr) return;
  const int nv = min(t.n1, t.n2), L = max(t.n1, t.n2);
  finalize_face<double>(t.w, t.sig, nv, L, t.kr, t.kr, t.ft, nullptr, r0, fin_sig_g, order);
}

// cols faces (n1 >= n2): Y = Ah^T F; rows faces: Y = Ah F; each launch
// passes over the faces of the other orientation
__global__ __launch_bounds__(256) void fin_factor_t_kernel(const FinFace* __restrict__ tab) {
  const FinFace t = tab[blockIdx.y];
  if (t.n1 < t.n2) return;
  factor_t_face<float>(t.ah, t.ft, t.y, t.n1, t.n2, t.kr, blockIdx.x * 4 + (threadIdx.x >> 6));
}

__global__ __launch_bounds__(256) void fin_factor_rows_kernel(const FinFace* __restrict__ tab) {
  __shared__ FactorRowsLds sm;
  const FinFace t = tab[blockIdx.y];
  if (t.n1 >= t.n2 || blockIdx.x * 64 >= t.n1 || (int)blockIdx.z * 16 >= t.kr) return;
  factor_rows_face<float>(t.ah, t.ft, t.y, t.n1, t.n2, t.kr, blockIdx.x, blockIdx.z * 16, sm);
}

template <bool FG>
__global__ __launch_bounds__(1024) void fin_refine_kernel(const FinFace* __restrict__ tab, double tol,
                                                          int max_sweeps) {
  extern __shared__ double rl_smem_g[];
  __shared__ int any_rot;
  const FinFace t = tab[blockIdx.x];
  const int nv = min(t.n1, t.n2), L = max(t.n1, t.n2);
  refine_face<float, FG>(t.y, t.ft, nv, L, t.kr, t.kout, t.kr, t.kout, tol, max_sweeps, t.s, t.other, t.fo, t.ys,
                         rl_smem_g, any_rot);
}

// one workgroup of kInfoThreads: each thread takes every kInfoThreads-th
// face, then the three integers are combined through LDS (order-free:
// maximum and sums of integers)
constexpr int kInfoThreads = 256;
__global__ __launch_bounds__(kInfoThreads) void info_kernel(const int* __restrict__ used1,
                                                            const int* __restrict__ used2, int p, int max1,
                                                            int max2, int* __restrict__ info) {
  __shared__ int acc[3];
  if (threadIdx.x == 0) acc[0] = acc[1] = acc[2] = 0;
  __syncthreads();
  int mx = 0, bad = 0, total = 0;
  for (int l = threadIdx.x; l < p; l += kInfoThreads) {
    const int u1 = used1[l];
    int n = min(u1, max1);
    bool conv = u1 <= max1;
    if (used2) {
      const int u2 = used2[l];
      n += min(u2, max2);
      conv = u2 <= max2;
    }
    if (!conv) ++bad;
    mx = max(mx, n);
    total += n;
  }
  atomicMax(&acc[0], mx);
  atomicAdd(&acc[1], bad);
  atomicAdd(&acc[2], total);
  __syncthreads();
  if (threadIdx.x == 0) {
    info[0] = acc[0];
    info[1] = acc[1];
    info[2] = acc[2];
  }
}

constexpr size_t kLdsCap = 131072;

template <typename T>
constexpr const char* block_name() {
  return sizeof(T) == 8 ? "jacobi_block_f64" : "jacobi_block_f32";
}

template <typename T, int R>
hipError_t block_sweeps(T* W, int p, int nv, int L, int nw, int max_sweeps, double tol, int* used,
                        int* flags, const int* prior, int prior_max, hipStream_t s) {
  const int b = nw * kPairsPerWave;
  int nb = (nv + b - 1) / b;
  nb += nb & 1;
  const size_t lds = sizeof(T) * (size_t)2 * b * 64 * R;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&jacobi_block_kernel<T, R>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsCap);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const dim3 block((unsigned)(64 * nw));
  if (nb == 2) {
    ProfScope prof(block_name<T>(), s);
    jacobi_block_kernel<T, R><<<dim3(1, p), block, lds, s>>>(W, nv, L, nb, 0, 0, max_sweeps, tol, flags,
                                                              used, prior, prior_max);
    return hipGetLastError();
  }
  const int nflags = p * max_sweeps;
  {
    ProfScope prof("jacobi_flags", s);
    zero_ints_kernel<<<(nflags + 255) / 256, 256, 0, s>>>(flags, nflags);
  }
  {
    ProfScope prof(block_name<T>(), s, max_sweeps * (nb - 1));
    for (int sw = 0; sw < max_sweeps; ++sw)
      for (int round = 0; round < nb - 1; ++round)
        jacobi_block_kernel<T, R><<<dim3(nb / 2, p), block, lds, s>>>(W, nv, L, nb, round, sw, max_sweeps,
                                                                       tol, flags, used, prior, prior_max);
  }
  {
    ProfScope prof("jacobi_flags", s);
    count_sweeps_kernel<<<(p + 63) / 64, 64, 0, s>>>(flags, p, max_sweeps, 0.f, used, prior, prior_max);
  }
  return hipGetLastError();
}

// Sweeps in the Gram form: max_sweeps x (nb - 1) launches; a face whose
// sweep rotated nothing is skipped by the later launches.
// The dynamic LDS the kernel may use: the largest of 160, 128 and 64 KiB
// that the device accepts (set once per process and instantiation).
template <typename T, int NB, bool ST, int NW = 4>
size_t gram_lds_cap() {
  static size_t cap = 0;
  if (cap == 0) {
    for (size_t c : {(size_t)160 * 1024, (size_t)128 * 1024, (size_t)64 * 1024}) {
      if (hipFuncSetAttribute(reinterpret_cast<const void*>(&jacobi_gram_kernel<T, NB, ST, NW>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)c) == hipSuccess) {
        cap = c;
        break;
      }
      (void)hipGetLastError();  // clear the refused request
    }
  }
  return cap;
}

// Visit forms: the 32 vectors staged in LDS with two copies of G, staged
// with one copy of G (float32 only: one more barrier per round, half the
// head), or not staged (the Gram step and X V read the L2; only the head in
// LDS).  A launch with at most one visit per CU stages its vectors; with more
// visits than CUs, float32 takes the form that lets two visits share a CU
// (staged, with one copy of G where two do not fit in half a CU's LDS).
// float64 vectors of 512 elements fill a CU's LDS when staged; unstaged they
// let two visits share a CU but wait on the L2, which measured 8% slower at
// two visits per CU (512-vector faces, 512 visits per launch) and 10% faster
// with more than four per CU (the batched form): float64 stays staged unless
// a launch has more than four visits per CU.  Vectors too long to stage at
// all are never staged.
enum class GramForm { Staged2, Staged1, Stream };
constexpr int kSplitVisitsPerCu = 256;  // CUs of the device
constexpr size_t kHalfCuLds = 80 * 1024;

template <typename T>
GramForm gram_form(int L, int grid) {
  const size_t two = gram_lds_bytes<T, 2, true>(L);
  const bool many = grid > 256;
  const bool fits2 = two <= gram_lds_cap<T, 2, true>();
  if constexpr (sizeof(T) == 4) {
    const size_t one = gram_lds_bytes<T, 1, true>(L);
    const bool fits1 = one <= gram_lds_cap<T, 1, true>();
    if (fits2 && (!many || two <= kHalfCuLds)) return GramForm::Staged2;
    if (fits1 && (one <= kHalfCuLds || !fits2)) return GramForm::Staged1;
    if (fits2 && !many) return GramForm::Staged2;
    return GramForm::Stream;
  } else {
    if (fits2 && (grid <= 4 * 256 || two <= kHalfCuLds)) return GramForm::Staged2;
    return GramForm::Stream;
  }
}

// launches of one sweep and visit slots per face: the full schedule of the
// largest face, or the top-block schedule (whose smaller faces, on the full
// schedule, fit in as many slots and rounds: nb <= 2 ntop blocks take at most
// ntop slots and 2 ntop - 1 <= top_rounds rounds)
inline void sweep_shape(int ntop, int nb_max, int& rounds, int& slots) {
  if (top_schedule(ntop, nb_max)) {
    rounds = top_rounds(ntop, nb_max);
    slots = ntop;
  } else {
    rounds = nb_max - 1;
    slots = nb_max / 2;
  }
}

template <typename T, int NB, bool ST, int NW>
void gram_launch_all(T* W, const JFace* faces, int nfaces, int nv_u, int L_u, int nb_max, int L_max, int max_sweeps,
                     double tol, float skip2, int ntop, int* flags, const VisitList* vl, hipStream_t s) {
  const size_t lds = gram_lds_bytes<T, NB, ST>(L_max);
  (void)gram_lds_cap<T, NB, ST, NW>();  // sets the kernel's LDS limit once
  int rounds, slots;
  sweep_shape(ntop, nb_max, rounds, slots);
  if (!top_schedule(ntop, nb_max)) ntop = 0;
  for (int sw = 0; sw < max_sweeps; ++sw)
    for (int round = 0; round < rounds; ++round) {
      unsigned grid = (unsigned)gram_grid(nfaces, slots);
      const int* visits = nullptr;
      if (vl) {
        grid = (unsigned)(vl->off[round + 1] - vl->off[round]);
        visits = vl->dev + vl->off[round];
        if (grid == 0) continue;
      }
      jacobi_gram_kernel<T, NB, ST, NW><<<grid, 64 * NW, lds, s>>>(W, faces, nfaces, slots, nv_u, L_u, round, sw,
                                                                   max_sweeps, tol, skip2, ntop, flags, visits);
    }
}

// launches of a sweep
int sweep_launches(int ntop, int nb_max, const VisitList* vl) {
  int rounds, slots;
  sweep_shape(ntop, nb_max, rounds, slots);
  if (!vl) return rounds;
  int n = 0;
  for (int r = 0; r < rounds; ++r) n += vl->off[r + 1] > vl->off[r];
  return n;
}

// Stopping rule of the Gram-form sweeps.  A face stops after a sweep in
// which no pair needed a rotation (largest squared cosine <= tol^2 on its
// flag word).  With a prediction threshold stop2 > 0 it also stops after a
// sweep whose largest cosine c before rotation had c^2 <= stop2: near
// convergence a cyclic Jacobi sweep squares the largest cosine (the
// quadratic convergence of the cyclic method), so that sweep itself left the
// face at cosines of about stop2, and the sweeps that would only take it
// further are not run.  Pairs are still rotated down to tol within the
// sweeps that do run.  The float32 data's phases predict (their result is
// settled by the float64 Ritz step on the transform-domain face); float64
// data and the U3 eigenvectors confirm (stop2 = 0).
inline float sweep_skip2(double tol, double stop2) { return (float)(stop2 > 0.0 ? std::max(tol * tol, stop2) : tol * tol); }

template <typename T>
hipError_t gram_sweeps(T* W, const JFace* faces, int nfaces, int nv_u, int L_u, int nb_max, int L_max,
                       int max_sweeps, double tol, double stop2, int ntop, int* used, int* flags, hipStream_t s,
                       const VisitList* vl = nullptr, const SweepPair* sp = nullptr, int form_grid = 0) {
  const int nflags = nfaces * max_sweeps;
  {
    ProfScope prof("jacobi_flags", s);
    zero_ints_kernel<<<(nflags + 255) / 256, 256, 0, s>>>(flags, nflags);
  }
  int rounds, slots;
  sweep_shape(ntop, nb_max, rounds, slots);
  // the top-block polish has two visits per face: staged whenever the
  // vectors fit (measured 1% faster than the unstaged form on the batched
  // workload, 11% on the hyperspectral one)
  const GramForm form = (sizeof(T) == 8 && top_schedule(ntop, nb_max) &&
                         gram_lds_bytes<T, 2, true>(L_max) <= gram_lds_cap<T, 2, true>())
                            ? GramForm::Staged2
                            : gram_form<T>(L_max, form_grid > 0 ? form_grid : gram_grid(nfaces, slots));
  const float skip2 = sweep_skip2(tol, stop2);
  // The faces in two parts on two streams (sp) when a launch would hold two
  // or more visits per CU: the visits of one launch start together and move
  // through the same phases at once, so that the memory system idles during
  // the rotation rounds and is flooded by the write-backs; two independent
  // chains of launches fall out of step and overlap the two.  Measured: the
  // batched workload's float32 sweeps 62.7 -> 58.0 ms, the hyperspectral
  // faces (512 visits per launch, split by face halves) 7.59 -> 6.85 ms; a
  // launch with fewer visits than CUs only gains dispatch cost (video 1.89
  // -> 2.10 ms), hence the threshold.
  bool split = sp != nullptr;
  int split_visits = 0;
  for (int k = 0; split && k < kSweepParts; ++k) {
    split = sp->vl[k] != nullptr && (k == 0 || sp->s2[k - 1] != nullptr);
    if (split) split_visits += sp->vl[k]->off[1] - sp->vl[k]->off[0];
  }
  split = split && split_visits >= 2 * kSplitVisitsPerCu;
  // every launch of the sweeps over visit list l on stream st, in the form
  // chosen (staged visits get eight waves: two per SIMD hide each other's
  // latency)
  auto launch = [&](const VisitList* l, hipStream_t st) {
    if (form == GramForm::Stream) {
      gram_launch_all<T, 2, false, 4>(W, faces, nfaces, nv_u, L_u, nb_max, L_max, max_sweeps, tol, skip2, ntop,
                                       flags, l, st);
    } else if constexpr (sizeof(T) == 4) {
      if (form == GramForm::Staged1)
        gram_launch_all<T, 1, true, 8>(W, faces, nfaces, nv_u, L_u, nb_max, L_max, max_sweeps, tol, skip2, ntop,
                                       flags, l, st);
      else
        gram_launch_all<T, 2, true, 8>(W, faces, nfaces, nv_u, L_u, nb_max, L_max, max_sweeps, tol, skip2, ntop,
                                       flags, l, st);
    } else {
      gram_launch_all<T, 2, true, 8>(W, faces, nfaces, nv_u, L_u, nb_max, L_max, max_sweeps, tol, skip2, ntop, flags,
                                     l, st);
    }
  };
  {
    int nl = 0;
    if (split)
      for (int k = 0; k < kSweepParts; ++k) nl += sweep_launches(ntop, nb_max, sp->vl[k]);
    else
      nl = sweep_launches(ntop, nb_max, vl);
    ProfScope prof(sizeof(T) == 8 ? "jacobi_gram_f64" : "jacobi_gram_f32", s, max_sweeps * nl);
    if (split) {
      hipError_t e = hipEventRecord(sp->fork, s);
      for (int k = 1; k < kSweepParts && e == hipSuccess; ++k) e = hipStreamWaitEvent(sp->s2[k - 1], sp->fork, 0);
      if (e != hipSuccess) return e;
      for (int k = 0; k < kSweepParts; ++k) launch(sp->vl[k], k == 0 ? s : sp->s2[k - 1]);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      for (int k = 1; k < kSweepParts; ++k) {
        if ((e = hipEventRecord(sp->join[k - 1], sp->s2[k - 1])) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(s, sp->join[k - 1], 0)) != hipSuccess) return e;
      }
    } else {
      launch(vl, s);
    }
  }
  {
    ProfScope prof("jacobi_flags", s);
    count_sweeps_kernel<<<(nfaces + 63) / 64, 64, 0, s>>>(flags, nfaces, max_sweeps, skip2, used);
  }
  return hipGetLastError();
}

// The second stream of a single call's split sweeps: one per device and host
// thread, created on first use outside graph capture and kept for the
// thread's life (null where it cannot be had: the sweeps then run on one
// stream).
struct DevicePair {
  hipStream_t s2 = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  bool tried = false;
};
constexpr int kMaxDevices = 64;
const DevicePair* device_pair(hipStream_t s) {
  thread_local DevicePair pairs[kMaxDevices];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  DevicePair& d = pairs[dev];
  if (d.s2) return &d;
  if (d.tried) return nullptr;
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess || st != hipStreamCaptureStatusNone) return nullptr;
  d.tried = true;
  hipError_t e = hipStreamCreateWithFlags(&d.s2, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&d.fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&d.join, hipEventDisableTiming);
  if (e != hipSuccess) {
    if (d.fork) hipEventDestroy(d.fork);
    if (d.join) hipEventDestroy(d.join);
    if (d.s2) hipStreamDestroy(d.s2);
    d = DevicePair{};
    d.tried = true;
    (void)hipGetLastError();
    return nullptr;
  }
  return &d;
}

// p faces of nv vectors of length L.  Where a launch would hold two or more
// visits per CU, the two halves of the face range run on two streams (the
// reason is given at gram_sweeps), under one profiler bracket on s.
template <typename T>
hipError_t gram_sweeps_uniform(T* W, int p, int nv, int L, int max_sweeps, double tol, double stop2, int ntop,
                               int* used, int* flags, hipStream_t s) {
  int nb = (nv + kGB - 1) / kGB;
  nb += nb & 1;
  int rounds, slots;
  sweep_shape(ntop, nb, rounds, slots);
  const DevicePair* dp = nullptr;
  if (p >= 2 && gram_grid(p, slots) >= 2 * kSplitVisitsPerCu) dp = device_pair(s);
  if (!dp) return gram_sweeps<T>(W, nullptr, p, nv, L, nb, L, max_sweeps, tol, stop2, ntop, used, flags, s);
  const int h = p / 2;
  ProfScope prof(sizeof(T) == 8 ? "jacobi_gram_f64" : "jacobi_gram_f32", s, 2 * max_sweeps * rounds);
  ProfMute mute;
  hipError_t e = hipEventRecord(dp->fork, s);
  if (e == hipSuccess) e = hipStreamWaitEvent(dp->s2, dp->fork, 0);
  // the visit form of the whole set's launches (two halves share the CUs)
  const int grid = gram_grid(p, slots);
  if (e == hipSuccess)
    e = gram_sweeps<T>(W, nullptr, h, nv, L, nb, L, max_sweeps, tol, stop2, ntop, used, flags, s, nullptr, nullptr,
                       grid);
  if (e == hipSuccess)
    e = gram_sweeps<T>(W + (size_t)h * nv * L, nullptr, p - h, nv, L, nb, L, max_sweeps, tol, stop2, ntop, used + h,
                       flags + (size_t)h * max_sweeps, dp->s2, nullptr, nullptr, grid);
  if (e == hipSuccess) e = hipEventRecord(dp->join, dp->s2);
  if (e == hipSuccess) e = hipStreamWaitEvent(s, dp->join, 0);
  return e;
}

// waves per workgroup (4 vectors of a block each): blocks of 16 vectors, fewer
// for faces of fewer than 32 vectors, and the 2b staged vectors within the
// LDS budget
template <typename T>
int pick_waves(int nv, int Lp) {
  int nw = std::min(4, std::max(1, (nv + 7) / 8));
  while (nw > 1 && sizeof(T) * (size_t)2 * kPairsPerWave * nw * Lp > kLdsCap) --nw;
  return nw;
}

template <typename T>
hipError_t sweeps(T* W, int p, int nv, int L, int max_sweeps, double tol, int* used, int* flags,
                  const int* prior, int prior_max, hipStream_t s) {
  const int R = (L + 63) / 64;
  int Rk = 0;
  for (int c : {1, 2, 3, 4, 5, 6, 8, 10, 12, 16})
    if (!Rk && R <= c) Rk = c;
  if (Rk > 0 && sizeof(T) * (size_t)2 * kPairsPerWave * 64 * Rk <= kLdsCap) {
    const int nw = pick_waves<T>(nv, 64 * Rk);
    switch (Rk) {
      case 1: return block_sweeps<T, 1>(W, p, nv, L, nw, max_sweeps, tol, used, flags, prior, prior_max, s);
      case 2: return block_sweeps<T, 2>(W, p, nv, L, nw, max_sweeps, tol, used, flags, prior, prior_max, s);
      case 3: return block_sweeps<T, 3>(W, p, nv, L, nw, max_sweeps, tol, used, flags, prior, prior_max, s);
      case 4: return block_sweeps<T, 4>(W, p, nv, L, nw, max_sweeps, tol, used, flags, prior, prior_max, s);
      case 5: return block_sweeps<T, 5>(W, p, nv, L, nw, max_sweeps, tol, used, flags, prior, prior_max, s);
      case 6: return block_sweeps<T, 6>(W, p, nv, L, nw, max_sweeps, tol, used, flags, prior, prior_max, s);
      case 8: return block_sweeps<T, 8>(W, p, nv, L, nw, max_sweeps, tol, used, flags, prior, prior_max, s);
      case 10: return block_sweeps<T, 10>(W, p, nv, L, nw, max_sweeps, tol, used, flags, prior, prior_max, s);
      case 12: return block_sweeps<T, 12>(W, p, nv, L, nw, max_sweeps, tol, used, flags, prior, prior_max, s);
      default: return block_sweeps<T, 16>(W, p, nv, L, nw, max_sweeps, tol, used, flags, prior, prior_max, s);
    }
  }
  ProfScope prof(sizeof(T) == 8 ? "jacobi_global_f64" : "jacobi_global_f32", s);
  jacobi_global_kernel<T><<<p, kJacobiThreads, 0, s>>>(W, nv, L, max_sweeps, tol, used, prior, prior_max);
  return hipGetLastError();
}

template <typename T>
hipError_t prep(const T* Ah, T* W, int n1, int n2, int p, hipStream_t s) {
  if (n1 >= n2) {
    return hipMemcpyAsync(W, Ah, sizeof(T) * (size_t)n1 * n2 * p, hipMemcpyDeviceToDevice, s);
  }
  dim3 grid((unsigned)((n1 + 31) / 32), (unsigned)((n2 + 31) / 32), (unsigned)p);
  transpose_faces_kernel<T><<<grid, 256, 0, s>>>(Ah, W, n1, n2);
  return hipGetLastError();
}

template <typename T>
hipError_t finalize(const T* W, const double* sig, int p, int nv, int L, int k, const int* kface, int extra, T* F,
                    double* sig_sorted, hipStream_t s) {
  const size_t lds = sizeof(double) * (size_t)nv;
  finalize_kernel<T><<<dim3((unsigned)p, (unsigned)((k + kFinCols - 1) / kFinCols)), 256, lds, s>>>(
      W, sig, nv, L, k, kface, extra, F, sig_sorted);
  return hipGetLastError();
}

template <typename TO>
hipError_t refine(double* Y, double* F, int m1, int m2, int k, int kout, int p, const int* kface, int extra,
                  double tol, TO* s_out, TO* Other, TO* Fo, TO* Ys, hipStream_t s) {
  // dynamic LDS up to 159 KiB (the kernel's static word fits in the rest)
  constexpr size_t kLdsCap = 159 * 1024;
  const size_t tail = (sizeof(double) + sizeof(int)) * (size_t)k;
  const size_t lds_both = sizeof(double) * (size_t)k * (m1 + m2) + tail;
  const size_t lds_y = sizeof(double) * (size_t)k * m1 + tail;
  static const hipError_t attr = [] {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&refine_lds_kernel<TO, false>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsCap);
    if (e == hipSuccess)
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(&refine_lds_kernel<TO, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsCap);
    if (e != hipSuccess) (void)hipGetLastError();  // clear a refused request: the global form runs instead
    return e;
  }();
  if (attr == hipSuccess && lds_both <= kLdsCap) {
    refine_lds_kernel<TO, false><<<p, 1024, lds_both, s>>>(Y, F, m1, m2, k, kout, kface, extra, tol, 12, s_out, Other,
                                                          Fo, Ys);
  } else if (attr == hipSuccess && lds_y <= kLdsCap) {
    refine_lds_kernel<TO, true><<<p, 1024, lds_y, s>>>(Y, F, m1, m2, k, kout, kface, extra, tol, 12, s_out, Other,
                                                         Fo, Ys);
  } else {
    const size_t lds = (sizeof(double) + sizeof(int)) * (size_t)k;
    refine_kernel<double, TO><<<p, 64 * kRefineWaves, lds, s>>>(Y, F, m1, m2, k, kout, kface, extra, tol, 12,
                                                               s_out, Other, Fo, Ys);
  }
  return hipGetLastError();
}

template <typename TA>
hipError_t factor(const TA* Ah, const double* F, double* Y, int n1, int n2, int k, int p, bool cols,
                  hipStream_t s) {
  if (cols) {
    factor_t_kernel<TA><<<dim3((unsigned)((n2 + 3) / 4), (unsigned)p), 256, 0, s>>>(Ah, F, Y, n1, n2, k);
  } else {
    factor_rows_kernel<TA><<<dim3((unsigned)((n1 + 63) / 64), (unsigned)p, (unsigned)((k + 15) / 16)), 256, 0,
                             s>>>(Ah, F, Y, n1, n2, k);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t jacobi_prep_f32(const float* Ah, float* W, int n1, int n2, int p, hipStream_t s) {
  return prep<float>(Ah, W, n1, n2, p, s);
}
hipError_t jacobi_prep_f64(const double* Ah, double* W, int n1, int n2, int p, hipStream_t s) {
  return prep<double>(Ah, W, n1, n2, p, s);
}
hipError_t jacobi_sweeps_f32(float* W, int p, int nv, int L, int max_sweeps, double tol, double stop2, int* used,
                             int* flags, hipStream_t s) {
  return gram_sweeps_uniform<float>(W, p, nv, L, max_sweeps, tol, stop2, 0, used, flags, s);
}
hipError_t jacobi_sweeps_f64(double* W, int p, int nv, int L, int max_sweeps, double tol, int* used,
                             int* flags, const int* prior, int prior_max, hipStream_t s) {
  return sweeps<double>(W, p, nv, L, max_sweeps, tol, used, flags, prior, prior_max, s);
}
hipError_t jacobi_gram_grouped_f32(float* W, const JFace* faces, int nfaces, int nb_max, int L_max,
                                   int max_sweeps, double tol, double stop2, int* used, int* flags,
                                   const VisitList* vl, hipStream_t s, const SweepPair* sp) {
  return gram_sweeps<float>(W, faces, nfaces, 0, 0, nb_max, L_max, max_sweeps, tol, stop2, 0, used, flags, s, vl,
                            sp);
}
hipError_t jacobi_gram_grouped_f64(double* W, const JFace* faces, int nfaces, int nb_max, int L_max,
                                   int max_sweeps, double tol, double stop2, int ntop, int* used, int* flags,
                                   const VisitList* vl, hipStream_t s, const SweepPair* sp) {
  return gram_sweeps<double>(W, faces, nfaces, 0, 0, nb_max, L_max, max_sweeps, tol, stop2, ntop, used, flags,
                             s, vl, sp);
}
bool jacobi_visit_list(const JFace* faces, int nfaces, int ntop, std::vector<int>& entries, std::vector<int>& off,
                       const std::vector<char>* pick) {
  entries.clear();
  off.assign(1, 0);
  if (nfaces < 0 || nfaces > (INT_MAX >> kVisitShift)) return false;
  auto blocks = [](int nv) {
    const int nb = (nv + kGB - 1) / kGB;
    return nb + (nb & 1);
  };
  int nb_max = 2;
  for (int f = 0; f < nfaces; ++f) nb_max = std::max(nb_max, blocks(faces[f].nv));
  int rounds, slots;
  sweep_shape(ntop, nb_max, rounds, slots);
  if (!top_schedule(ntop, nb_max)) ntop = 0;
  if (slots > (1 << kVisitShift)) return false;
  // longest vectors first within a round
  std::vector<int> order((size_t)nfaces);
  for (int f = 0; f < nfaces; ++f) order[(size_t)f] = f;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return faces[a].L > faces[b].L; });
  for (int r = 0; r < rounds; ++r) {
    for (const int f : order) {
      if (pick && !(*pick)[(size_t)f]) continue;
      const int nb = blocks(faces[f].nv);
      for (int pair = 0; pair < slots; ++pair) {
        bool valid;
        if (top_schedule(ntop, nb)) {
          int I, J;
          bool full;
          valid = top_pair(ntop, nb, r, pair, I, J, full);
        } else {
          valid = r < nb - 1 && pair < nb / 2;
        }
        if (valid) entries.push_back((f << kVisitShift) | pair);
      }
    }
    off.push_back((int)entries.size());
  }
  return true;
}
hipError_t jacobi_gram_sweeps_f64(double* W, int p, int nv, int L, int max_sweeps, double tol, double stop2,
                                  int ntop, int* used, int* flags, hipStream_t s) {
  return gram_sweeps_uniform<double>(W, p, nv, L, max_sweeps, tol, stop2, ntop, used, flags, s);
}
hipError_t jacobi_norms_f64(const double* W, int p, int nv, int L, double* sig, int* rank, hipStream_t s) {
  norms_kernel<double><<<dim3((unsigned)((nv + 3) / 4), (unsigned)p), 256, 0, s>>>(W, nv, L, sig, rank);
  return hipGetLastError();
}
hipError_t jacobi_finalize_f64(const double* W, const double* sig, int p, int nv, int L, int k, const int* kface,
                              int extra, double* F, double* sig_sorted, hipStream_t s) {
  return finalize<double>(W, sig, p, nv, L, k, kface, extra, F, sig_sorted, s);
}
hipError_t jacobi_select(const double* sig, int p, int nv, double gamma, int* rank, double* e2, int* rho,
                         hipStream_t s) {
  const int n = p * nv;
  const int bx = (n + 255) / 256;
  // split the comparison columns so that the grid holds about 2048 blocks
  const int by = std::max(1, std::min(bx, (2048 + bx - 1) / bx));
  const int cols = ((n + by - 1) / by + 255) / 256 * 256;
  rank_kernel<<<dim3((unsigned)bx, (unsigned)((n + cols - 1) / cols)), 256, 0, s>>>(sig, n, cols, rank);
  select_kernel<<<1, kSelThreads, 0, s>>>(sig, rank, n, p, nv, gamma, e2, rho);
  return hipGetLastError();
}
hipError_t jacobi_refine_f32(double* Y, double* F, int m1, int m2, int k, int kout, int p, const int* kface,
                             int extra, double tol, float* s_out, float* Other, float* Fo, float* Ys,
                             hipStream_t s) {
  return refine<float>(Y, F, m1, m2, k, kout, p, kface, extra, tol, s_out, Other, Fo, Ys, s);
}
hipError_t jacobi_refine_f64(double* Y, double* F, int m1, int m2, int k, int kout, int p, const int* kface,
                             int extra, double tol, double* s_out, double* Other, double* Fo, double* Ys,
                             hipStream_t s) {
  return refine<double>(Y, F, m1, m2, k, kout, p, kface, extra, tol, s_out, Other, Fo, Ys, s);
}
hipError_t jacobi_finish_grouped(const FinFace* tab, int nfaces, const FinMax& m, double tol, hipStream_t s) {
  if (nfaces <= 0) return hipSuccess;
  // norms of every vector, the top kr normalised (finalize ranks a face's nv
  // norms in LDS), the products with the transform-domain faces, the Ritz step
  fin_norms_kernel<<<dim3((unsigned)((m.nv + 3) / 4), (unsigned)nfaces), 256, 0, s>>>(tab);
  fin_finalize_kernel<<<dim3((unsigned)nfaces, (unsigned)((m.kr + kFinCols - 1) / kFinCols)), 256,
                        sizeof(double) * (size_t)m.nv, s>>>(tab);
  fin_factor_t_kernel<<<dim3((unsigned)((m.n2 + 3) / 4), (unsigned)nfaces), 256, 0, s>>>(tab);
  fin_factor_rows_kernel<<<dim3((unsigned)((m.n1 + 63) / 64), (unsigned)nfaces, (unsigned)((m.kr + 15) / 16)), 256, 0,
                           s>>>(tab);
  constexpr size_t kLdsCap = 159 * 1024;
  const size_t tail = (sizeof(double) + sizeof(int)) * (size_t)m.kr;
  const size_t both = sizeof(double) * (size_t)m.kr * m.nvL + tail;
  const size_t yonly = sizeof(double) * (size_t)m.kr * m.nv + tail;
  static const hipError_t attr = [] {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fin_refine_kernel<false>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsCap);
    if (e == hipSuccess)
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fin_refine_kernel<true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsCap);
    return e;
  }();
  if (attr != hipSuccess) return attr;
  if (both <= kLdsCap) {
    fin_refine_kernel<false><<<(unsigned)nfaces, 1024, both, s>>>(tab, tol, 12);
  } else if (yonly <= kLdsCap) {
    fin_refine_kernel<true><<<(unsigned)nfaces, 1024, yonly, s>>>(tab, tol, 12);
  } else {
    return hipErrorInvalidValue;  // beyond what the batched form's size cap admits
  }
  return hipGetLastError();
}

hipError_t jacobi_widen_top(const float* W32, double* W64, const JFace* faces, int nfaces, int nv_u, int L_u,
                            int nv_max, int ntop16, double* nrm, int* pos, hipStream_t s) {
  const dim3 grid((unsigned)((nv_max + 3) / 4), (unsigned)nfaces);
  top_norms_kernel<<<grid, 256, 0, s>>>(W32, faces, nv_u, L_u, nv_max, nrm);
  top_perm_kernel<<<(unsigned)nfaces, 256, (sizeof(double) + sizeof(int)) * (size_t)nv_max, s>>>(
      nrm, faces, nv_u, L_u, nv_max, ntop16, pos);
  top_copy_kernel<<<grid, 256, 0, s>>>(W32, W64, faces, nv_u, L_u, nv_max, pos);
  return hipGetLastError();
}
hipError_t jacobi_widen(const float* x, double* y, int64_t n, hipStream_t s) {
  widen_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, y, n);
  return hipGetLastError();
}
hipError_t jacobi_factor_f32(const float* Ah, const double* F, double* Y, int n1, int n2, int k, int p,
                             bool cols, hipStream_t s) {
  return factor<float>(Ah, F, Y, n1, n2, k, p, cols, s);
}
hipError_t jacobi_factor_f64(const double* Ah, const double* F, double* Y, int n1, int n2, int k, int p,
                             bool cols, hipStream_t s) {
  return factor<double>(Ah, F, Y, n1, n2, k, p, cols, s);
}
hipError_t jacobi_info(const int* used1, const int* used2, int p, int max1, int max2, int* info,
                       hipStream_t s) {
  info_kernel<<<1, kInfoThreads, 0, s>>>(used1, used2, p, max1, max2, info);
  return hipGetLastError();
}

}  // namespace pq
