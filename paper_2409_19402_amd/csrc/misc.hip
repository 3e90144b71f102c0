// The float64 Stiefel check of Q (precondition of Def. 3.1).
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

}  // namespace

hipError_t check_q_launch(const void* Q, bool f64, int n3, int p, double* out, hipStream_t s) {
  if (f64) check_q_kernel<double><<<1, 256, 0, s>>>(static_cast<const double*>(Q), n3, p, out);
  else check_q_kernel<float><<<1, 256, 0, s>>>(static_cast<const float*>(Q), n3, p, out);
  return hipGetLastError();
}

}  // namespace pq
