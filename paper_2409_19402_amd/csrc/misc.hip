// Small kernels around the hot path: the float64 Stiefel check of Q
// (precondition of Def. 3.1) and the column scaling that turns the products
// A^T U (or A V) of the truncated SVD into singular vectors.
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

template <typename T>
__global__ __launch_bounds__(256) void scale_cols_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                         int64_t rows, int k, int64_t total,
                                                         const T* __restrict__ scale) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int64_t col = e / rows;  // = j + l*k
  out[e] = in[e] * scale[col];
  (void)k;
}

}  // namespace

hipError_t check_q_launch(const void* Q, bool f64, int n3, int p, double* out, hipStream_t s) {
  if (f64) check_q_kernel<double><<<1, 256, 0, s>>>(static_cast<const double*>(Q), n3, p, out);
  else check_q_kernel<float><<<1, 256, 0, s>>>(static_cast<const float*>(Q), n3, p, out);
  return hipGetLastError();
}

hipError_t scale_cols_f32(const float* in, float* out, int64_t rows, int k, int p, const float* scale,
                          hipStream_t s) {
  const int64_t total = rows * k * (int64_t)p;
  scale_cols_kernel<float><<<(unsigned)((total + 255) / 256), 256, 0, s>>>(in, out, rows, k, total, scale);
  return hipGetLastError();
}

hipError_t scale_cols_f64(const double* in, double* out, int64_t rows, int k, int p,
                          const double* scale, hipStream_t s) {
  const int64_t total = rows * k * (int64_t)p;
  scale_cols_kernel<double><<<(unsigned)((total + 255) / 256), 256, 0, s>>>(in, out, rows, k, total, scale);
  return hipGetLastError();
}

}  // namespace pq
