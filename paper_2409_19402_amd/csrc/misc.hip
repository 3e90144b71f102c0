// The float64 Stiefel check of Q (precondition of Def. 3.1), the fixed
// transforms used as Q in the experiments of Sec. 5 (identity, DCT) and the
// last step of the construction of Q = U3 (Thm. 4.3).
#include "common.hpp"
#include "internal.hpp"

namespace pq {
namespace {

// max over a <= b of |(Q^T Q - I)_ab| in float64: one wave per column pair
// (lanes over t), the maximum folded into out[0] by an integer atomic on the
// bit pattern (non-negative doubles order as their bits do); out[0] is
// cleared by clear_q_kernel first.
template <typename TQ>
__global__ __launch_bounds__(256) void check_q_kernel(const TQ* __restrict__ Q, int n3, int p,
                                                      unsigned long long* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t pair = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t npair = (int64_t)p * (p + 1) / 2;
  if (pair >= npair) return;
  // pair -> (a, b), a <= b, row by row of the upper triangle
  int a = 0;
  int64_t rest = pair;
  while (rest >= p - a) {
    rest -= p - a;
    ++a;
  }
  const int b = a + (int)rest;
  double acc = 0.0;
  for (int t = lane; t < n3; t += 64)
    acc = fma((double)Q[(int64_t)t * p + a], (double)Q[(int64_t)t * p + b], acc);
  acc = wave_total(acc);
  if (lane == 0) {
    const double d = fabs(a == b ? acc - 1.0 : acc);
    atomicMax(out, (unsigned long long)__double_as_longlong(d));
  }
}

__global__ void clear_q_kernel(unsigned long long* __restrict__ out) {
  if (threadIdx.x == 0) out[0] = 0ull;
}

// flag[0] = 1 when the distance dist[0] exceeds tol or is not a number
// (a NaN's bit pattern wins the integer maximum above), else 0
__global__ void q_flag_kernel(const double* __restrict__ dist, double tol, int* __restrict__ flag) {
  if (threadIdx.x == 0) flag[0] = (dist[0] <= tol) ? 0 : 1;
}

// Layout conversion between the paper's face-major order (element (i, j, t)
// at i + n1 (j + n2 t)) and tube-major order (t + n3 (j + n2 i): numpy's
// C order of an n1 x n2 x n3 array).  For each j it is a transpose of the
// (i, t) plane: 32 x 32 tiles through LDS, loads and stores both coalesced
// (lanes along the contiguous index of each side).  E is the element's bit
// pattern (2, 4 or 8 bytes).
template <typename E, bool TO_FACE>
__global__ __launch_bounds__(256) void relayout_kernel(const E* __restrict__ src, E* __restrict__ dst, int n1,
                                                       int n2, int n3, int tiles_t) {
  __shared__ E tile[32][33];
  const int j = blockIdx.x / tiles_t, t0 = (blockIdx.x % tiles_t) * 32, i0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int64_t face = (int64_t)n1 * n2;
  // tile[r][c] holds element (i0 + r, t0 + c) when converting to face-major,
  // element (i0 + c, t0 + r) otherwise; either way the stores read tile[tx][r]
  for (int r = ty; r < 32; r += 8) {
    if (TO_FACE) {
      const int i = i0 + r, t = t0 + tx;
      if (i < n1 && t < n3) tile[r][tx] = src[t + (int64_t)n3 * (j + (int64_t)n2 * i)];
    } else {
      const int i = i0 + tx, t = t0 + r;
      if (i < n1 && t < n3) tile[r][tx] = src[i + (int64_t)n1 * j + face * t];
    }
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    if (TO_FACE) {
      const int i = i0 + tx, t = t0 + r;
      if (i < n1 && t < n3) dst[i + (int64_t)n1 * j + face * t] = tile[tx][r];
    } else {
      const int i = i0 + r, t = t0 + tx;
      if (i < n1 && t < n3) dst[t + (int64_t)n3 * (j + (int64_t)n2 * i)] = tile[tx][r];
    }
  }
}

// CholeskyQR2 of Q (n3 x p row-major) in float64, one workgroup: W = Q
// (widened), then twice G = W^T W, G = R^T R (Cholesky, R upper triangular
// with a positive diagonal, in LDS), W <- W R^{-1}; Qout = W in Q's type.
// info[0] = 0, or c + 1 when the pivot of column c in either pass is not
// above 64 eps times that column's squared norm (Q numerically rank
// deficient): the kernel then stops and leaves Qout unwritten.  Q is read in
// full before Qout is written, so the two may be the same array.
constexpr int kQrThreads = 1024;

template <typename TQ>
__global__ __launch_bounds__(kQrThreads) void cholqr2_kernel(const TQ* __restrict__ Q, int n3, int p,
                                                           double* __restrict__ W, TQ* __restrict__ Qout,
                                                           int* __restrict__ info) {
  extern __shared__ double R[];  // p x p, row a at R + a p; then the p squared column norms
  double* gd = R + (size_t)p * p;
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int64_t n = (int64_t)n3 * p;
  for (int64_t e = tid; e < n; e += kQrThreads) W[e] = (double)Q[e];
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    // G = W^T W, upper triangle
    for (int e = tid; e < p * p; e += kQrThreads) {
      const int a = e / p, b = e - a * p;
      if (a <= b) {
        double g = 0.0;
        for (int t = 0; t < n3; ++t) g = fma(W[(int64_t)t * p + a], W[(int64_t)t * p + b], g);
        R[e] = g;
        if (a == b) gd[a] = g;
      }
    }
    __syncthreads();
    // upper Cholesky G = R^T R, right-looking, column by column
    for (int c = 0; c < p; ++c) {
      if (tid == 0) {
        // the column's squared norm less its projection on the earlier columns
        const double d = R[c * p + c];
        if (!(d > 64.0 * 2.220446049250313e-16 * gd[c])) bad = c + 1;
        else R[c * p + c] = sqrt(d);
      }
      __syncthreads();
      if (bad) break;
      const double rcc = R[c * p + c];
      for (int b = c + 1 + tid; b < p; b += kQrThreads) R[c * p + b] /= rcc;
      __syncthreads();
      // trailing update G[a][b] -= R[c][a] R[c][b] for c < a <= b
      const int m = p - c - 1;
      for (int e = tid; e < m * m; e += kQrThreads) {
        const int a = c + 1 + e / m, b = c + 1 + e % m;
        if (a <= b) R[a * p + b] -= R[c * p + a] * R[c * p + b];
      }
      __syncthreads();
    }
    if (bad) break;
    // W <- W R^{-1}: row t solves x R = w by forward substitution
    for (int t = tid; t < n3; t += kQrThreads) {
      double* w = W + (int64_t)t * p;
      for (int c = 0; c < p; ++c) {
        double x = w[c];
        for (int k = 0; k < c; ++k) x = fma(-w[k], R[k * p + c], x);
        w[c] = x / R[c * p + c];
      }
    }
    __syncthreads();
  }
  if (tid == 0) info[0] = bad;
  if (bad) return;
  for (int64_t e = tid; e < n; e += kQrThreads) Qout[e] = static_cast<TQ>(W[e]);
}

// Q (n3 x p row-major) of a fixed transform: kind 0 the first p columns of
// the identity, kind 1 the first p rows of the orthonormal DCT-II matrix C
// (n3 x n3), transposed: Q(t, l) = C(l, t) = w_l cos(pi (2t + 1) l / (2 n3)),
// w_0 = sqrt(1 / n3), w_l = sqrt(2 / n3).  The cosine takes the angle as an
// exact rational multiple of pi (the integer (2t + 1) l reduced mod 4 n3).
template <typename TO>
__global__ __launch_bounds__(256) void build_q_kernel(int kind, int n3, int p, TO* __restrict__ Q) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)n3 * p) return;
  const int t = (int)(e / p), l = (int)(e - (int64_t)t * p);
  double v;
  if (kind == 0) {
    v = t == l ? 1.0 : 0.0;
  } else {
    const int64_t m = ((int64_t)(2 * t + 1) * l) % (4 * (int64_t)n3);
    const double w = l == 0 ? sqrt(1.0 / n3) : sqrt(2.0 / n3);
    v = w * cospi((double)m / (2.0 * n3));
  }
  Q[e] = static_cast<TO>(v);
}

// Column r of Q from the r-th normalised eigenvector f = F[r * n3 .. +n3):
// signed so that its largest-magnitude entry (the first on ties) is positive,
// written row-major (Q[t * p + r]); lambda[r] = f^T G f (Rayleigh quotient,
// G the n3 x n3 Gram matrix, column-major).  One workgroup per column.
template <typename TO>
__global__ __launch_bounds__(256) void u3_finish_kernel(const double* __restrict__ F, const double* __restrict__ G,
                                                        int n3, int p, TO* __restrict__ Q, TO* __restrict__ lambda) {
  extern __shared__ double fs[];  // the eigenvector (n3 doubles)
  __shared__ double rv[256];
  __shared__ int ri[256];
  const int r = blockIdx.x;
  const double* f = F + (int64_t)r * n3;
  for (int i = threadIdx.x; i < n3; i += 256) fs[i] = f[i];
  __syncthreads();
  double best = -1.0;
  int bi = 0;
  double quad = 0.0;
  for (int i = threadIdx.x; i < n3; i += 256) {
    const double a = fabs(fs[i]);
    if (a > best) { best = a; bi = i; }
    // (G f)_i: eight chains over j (mod 8), eight loads of column i in
    // flight, summed in a fixed order
    const double* gc = G + i;
    double c8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int j = 0;
    for (; j + 7 < n3; j += 8) {
      double g[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) g[c] = gc[(int64_t)(j + c) * n3];
#pragma unroll
      for (int c = 0; c < 8; ++c) c8[c] = fma(g[c], fs[j + c], c8[c]);
    }
    for (int c = 0; j < n3; ++j, ++c) c8[c] = fma(gc[(int64_t)j * n3], fs[j], c8[c]);
    const double gi = ((c8[0] + c8[1]) + (c8[2] + c8[3])) + ((c8[4] + c8[5]) + (c8[6] + c8[7]));
    quad = fma(fs[i], gi, quad);
  }
  rv[threadIdx.x] = best;
  ri[threadIdx.x] = bi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double a = rv[threadIdx.x + w];
      const int b = ri[threadIdx.x + w];
      if (a > rv[threadIdx.x] || (a == rv[threadIdx.x] && b < ri[threadIdx.x])) {
        rv[threadIdx.x] = a;
        ri[threadIdx.x] = b;
      }
    }
    __syncthreads();
  }
  const double sgn = fs[ri[0]] < 0.0 ? -1.0 : 1.0;
  __syncthreads();
  rv[threadIdx.x] = quad;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) rv[threadIdx.x] += rv[threadIdx.x + w];
    __syncthreads();
  }
  for (int t = threadIdx.x; t < n3; t += 256) Q[(int64_t)t * p + r] = static_cast<TO>(sgn * fs[t]);
  if (threadIdx.x == 0 && lambda) lambda[r] = static_cast<TO>(rv[0]);
}

}  // namespace

hipError_t check_q_launch(const void* Q, bool f64, int n3, int p, double* out, hipStream_t s) {
  unsigned long long* bits = reinterpret_cast<unsigned long long*>(out);
  clear_q_kernel<<<1, 64, 0, s>>>(bits);
  const int64_t npair = (int64_t)p * (p + 1) / 2;
  const unsigned grid = (unsigned)((npair + 3) / 4);
  if (f64) check_q_kernel<double><<<grid, 256, 0, s>>>(static_cast<const double*>(Q), n3, p, bits);
  else check_q_kernel<float><<<grid, 256, 0, s>>>(static_cast<const float*>(Q), n3, p, bits);
  return hipGetLastError();
}

hipError_t check_q_flag(const double* dist, double tol, int* flag, hipStream_t s) {
  q_flag_kernel<<<1, 64, 0, s>>>(dist, tol, flag);
  return hipGetLastError();
}

template <typename E>
hipError_t relayout_go(const void* src, void* dst, bool to_face, int n1, int n2, int n3, hipStream_t s) {
  const int tiles_t = (n3 + 31) / 32;
  const dim3 grid((unsigned)((int64_t)tiles_t * n2), (unsigned)((n1 + 31) / 32));
  if (to_face)
    relayout_kernel<E, true><<<grid, 256, 0, s>>>(static_cast<const E*>(src), static_cast<E*>(dst), n1, n2, n3,
                                                 tiles_t);
  else
    relayout_kernel<E, false><<<grid, 256, 0, s>>>(static_cast<const E*>(src), static_cast<E*>(dst), n1, n2, n3,
                                                  tiles_t);
  return hipGetLastError();
}

hipError_t relayout(const void* src, void* dst, int elem_bytes, bool to_face, int n1, int n2, int n3, hipStream_t s) {
  switch (elem_bytes) {
    case 2: return relayout_go<uint16_t>(src, dst, to_face, n1, n2, n3, s);
    case 4: return relayout_go<uint32_t>(src, dst, to_face, n1, n2, n3, s);
    default: return relayout_go<uint64_t>(src, dst, to_face, n1, n2, n3, s);
  }
}

hipError_t cholqr2(const void* Q, bool f64, int n3, int p, double* W, void* Qout, int* info, hipStream_t s) {
  const size_t lds = sizeof(double) * ((size_t)p * p + p);
  const void* fn = f64 ? reinterpret_cast<const void*>(&cholqr2_kernel<double>)
                       : reinterpret_cast<const void*>(&cholqr2_kernel<float>);
  if (lds > 48 * 1024) {
    const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (f64)
    cholqr2_kernel<double><<<1, kQrThreads, lds, s>>>(static_cast<const double*>(Q), n3, p, W,
                                                      static_cast<double*>(Qout), info);
  else
    cholqr2_kernel<float><<<1, kQrThreads, lds, s>>>(static_cast<const float*>(Q), n3, p, W,
                                                     static_cast<float*>(Qout), info);
  return hipGetLastError();
}

hipError_t build_q(int kind, bool f64, int n3, int p, void* Q, hipStream_t s) {
  const unsigned grid = (unsigned)(((int64_t)n3 * p + 255) / 256);
  if (f64) build_q_kernel<double><<<grid, 256, 0, s>>>(kind, n3, p, static_cast<double*>(Q));
  else build_q_kernel<float><<<grid, 256, 0, s>>>(kind, n3, p, static_cast<float*>(Q));
  return hipGetLastError();
}

hipError_t u3_finish(const double* F, const double* G, int n3, int p, void* Q, void* lambda, bool f64,
                     hipStream_t s) {
  const size_t lds = 8 * (size_t)n3;  // n3 <= 4096: at most 32 KB
  if (f64)
    u3_finish_kernel<double><<<p, 256, lds, s>>>(F, G, n3, p, static_cast<double*>(Q), static_cast<double*>(lambda));
  else
    u3_finish_kernel<float><<<p, 256, lds, s>>>(F, G, n3, p, static_cast<float*>(Q), static_cast<float*>(lambda));
  return hipGetLastError();
}

}  // namespace pq
