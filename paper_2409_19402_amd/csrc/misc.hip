// The float64 Stiefel check of Q (precondition of Def. 3.1) and the last step
// of the construction of Q = U3 (Thm. 4.3).
#include "common.hpp"
#include "internal.hpp"

namespace pq {
namespace {

template <typename TQ>
__global__ __launch_bounds__(256) void check_q_kernel(const TQ* __restrict__ Q, int n3, int p,
                                                      double* __restrict__ out) {
  __shared__ double red[256];
  double mx = 0.0;
  const int64_t npair = (int64_t)p * p;
  for (int64_t e = threadIdx.x; e < npair; e += 256) {
    const int a = (int)(e / p), b = (int)(e - (int64_t)a * p);
    if (b < a) continue;
    double acc = 0.0;
    for (int t = 0; t < n3; ++t)
      acc = fma((double)Q[(int64_t)t * p + a], (double)Q[(int64_t)t * p + b], acc);
    if (a == b) acc -= 1.0;
    mx = fmax(mx, fabs(acc));
  }
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
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
  if (f64) check_q_kernel<double><<<1, 256, 0, s>>>(static_cast<const double*>(Q), n3, p, out);
  else check_q_kernel<float><<<1, 256, 0, s>>>(static_cast<const float*>(Q), n3, p, out);
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
