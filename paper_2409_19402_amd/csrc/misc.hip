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

// out[e] = sum over z of parts[z * stride + e], accumulated in float64 in a
// fixed order (the split-K slices of a float32 product)
__global__ __launch_bounds__(256) void sum_to_f64_kernel(const float* __restrict__ parts, int nparts,
                                                         int64_t stride, int64_t count, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= count) return;
  double acc = 0.0;
  for (int z = 0; z < nparts; ++z) acc += (double)parts[(int64_t)z * stride + e];
  out[e] = acc;
}

// Column r of Q from the r-th normalised eigenvector f = F[r * n3 .. +n3):
// signed so that its largest-magnitude entry (the first on ties) is positive,
// written row-major (Q[t * p + r]); lambda[r] = f^T G f (Rayleigh quotient,
// G the n3 x n3 Gram matrix, column-major).  One workgroup per column.
template <typename TO>
__global__ __launch_bounds__(256) void u3_finish_kernel(const double* __restrict__ F, const double* __restrict__ G,
                                                        int n3, int p, TO* __restrict__ Q, TO* __restrict__ lambda) {
  __shared__ double rv[256];
  __shared__ int ri[256];
  const int r = blockIdx.x;
  const double* f = F + (int64_t)r * n3;
  double best = -1.0;
  int bi = 0;
  double quad = 0.0;
  for (int i = threadIdx.x; i < n3; i += 256) {
    const double a = fabs(f[i]);
    if (a > best) { best = a; bi = i; }
    double gi = 0.0;  // (G f)_i
    for (int j = 0; j < n3; ++j) gi = fma(G[i + (int64_t)j * n3], f[j], gi);
    quad = fma(f[i], gi, quad);
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
  const double sgn = f[ri[0]] < 0.0 ? -1.0 : 1.0;
  __syncthreads();
  rv[threadIdx.x] = quad;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) rv[threadIdx.x] += rv[threadIdx.x + w];
    __syncthreads();
  }
  for (int t = threadIdx.x; t < n3; t += 256) Q[(int64_t)t * p + r] = static_cast<TO>(sgn * f[t]);
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

hipError_t build_q(int kind, bool f64, int n3, int p, void* Q, hipStream_t s) {
  const unsigned grid = (unsigned)(((int64_t)n3 * p + 255) / 256);
  if (f64) build_q_kernel<double><<<grid, 256, 0, s>>>(kind, n3, p, static_cast<double*>(Q));
  else build_q_kernel<float><<<grid, 256, 0, s>>>(kind, n3, p, static_cast<float*>(Q));
  return hipGetLastError();
}

hipError_t sum_to_f64(const float* parts, int nparts, int64_t stride, int64_t count, double* out, hipStream_t s) {
  sum_to_f64_kernel<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(parts, nparts, stride, count, out);
  return hipGetLastError();
}

hipError_t u3_finish(const double* F, const double* G, int n3, int p, void* Q, void* lambda, bool f64,
                     hipStream_t s) {
  if (f64)
    u3_finish_kernel<double><<<p, 256, 0, s>>>(F, G, n3, p, static_cast<double*>(Q), static_cast<double*>(lambda));
  else
    u3_finish_kernel<float><<<p, 256, 0, s>>>(F, G, n3, p, static_cast<float*>(Q), static_cast<float*>(lambda));
  return hipGetLastError();
}

}  // namespace pq
