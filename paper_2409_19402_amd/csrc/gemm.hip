// Batched dense GEMM for the facewise product (Def. 2.3) and the other
// contractions of the path (the transposed facewise products of the adjoint,
// the split-K reductions over the n1 n2 tubes that give dQ, the factor
// products of the truncated SVD).
//
// float32: a 64x64 output tile per 256-thread workgroup, 16-deep K tiles
// staged through LDS, one 32x32 tile per wave on v_mfma_f32_32x32x2f32.  The
// MFMA computes the transposed tile (rows = output columns), so the 32 lanes
// that share an accumulator register hold 32 consecutive rows of the
// column-major output and stores coalesce.
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace pq {
namespace {

constexpr int kTM = 64, kTN = 64, kTK = 16;

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_f32_kernel(Gemm g, int kchunk) {
  __shared__ float As[kTK][kTM + 4];
  __shared__ float Bs[kTK][kTN + 4];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int nl = lane & 31, kh = lane >> 5;
  const int wm = wave & 1, wn = wave >> 1;
  const int zb = blockIdx.z % g.batch, zs = blockIdx.z / g.batch;
  const int m0 = blockIdx.x * kTM, n0 = blockIdx.y * kTN;
  const int kbeg = zs * kchunk, kend = min(g.K, kbeg + kchunk);
  const float* A = static_cast<const float*>(g.A) + (int64_t)zb * g.sA;
  const float* B = static_cast<const float*>(g.B) + (int64_t)zb * g.sB;
  float* C = static_cast<float*>(g.C) + (int64_t)zb * g.sC + (int64_t)zs * g.sSplit;
  f32x16 acc;
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = 0.f;
  for (int k0 = kbeg; k0 < kend; k0 += kTK) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = tid + 256 * i;
      int m, k;
      if (TA) { k = e & 15; m = e >> 4; } else { m = e & 63; k = e >> 6; }
      const int gm = m0 + m, gk = k0 + k;
      float v = 0.f;
      if (gm < g.M && gk < kend) v = TA ? A[gk + (int64_t)gm * g.lda] : A[gm + (int64_t)gk * g.lda];
      As[k][m] = v;
      int n;
      if (TB) { n = e & 63; k = e >> 6; } else { k = e & 15; n = e >> 4; }
      const int gn = n0 + n;
      const int gk2 = k0 + k;
      float w = 0.f;
      if (gn < g.N && gk2 < kend) w = TB ? B[gn + (int64_t)gk2 * g.ldb] : B[gk2 + (int64_t)gn * g.ldb];
      Bs[k][n] = w;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kTK; kk += 2) {
      const float a = Bs[kk + kh][wn * 32 + nl];  // rows of the transposed tile: output columns
      const float b = As[kk + kh][wm * 32 + nl];  // columns of the transposed tile: output rows
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const int gm = m0 + wm * 32 + nl;
  if (gm >= g.M) return;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int gn = n0 + wn * 32 + 8 * (j >> 2) + 4 * kh + (j & 3);
    if (gn < g.N) C[gm + (int64_t)gn * g.ldc] = acc[j];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void gemm_generic_kernel(Gemm g, int kchunk) {
  const int zb = blockIdx.z % g.batch, zs = blockIdx.z / g.batch;
  const int m = blockIdx.x * 16 + (threadIdx.x & 15);
  const int n = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (m >= g.M || n >= g.N) return;
  const T* A = static_cast<const T*>(g.A) + (int64_t)zb * g.sA;
  const T* B = static_cast<const T*>(g.B) + (int64_t)zb * g.sB;
  T* C = static_cast<T*>(g.C) + (int64_t)zb * g.sC + (int64_t)zs * g.sSplit;
  const int kbeg = zs * kchunk, kend = min(g.K, kbeg + kchunk);
  T acc = T(0);
  for (int k = kbeg; k < kend; ++k) {
    const T a = g.ta ? A[k + (int64_t)m * g.lda] : A[m + (int64_t)k * g.lda];
    const T b = g.tb ? B[n + (int64_t)k * g.ldb] : B[k + (int64_t)n * g.ldb];
    acc = fma(a, b, acc);
  }
  C[m + (int64_t)n * g.ldc] = acc;
}

template <typename T>
__global__ __launch_bounds__(256) void sum_partials_kernel(const T* __restrict__ parts, int nparts,
                                                           int64_t stride, int64_t count,
                                                           T* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= count) return;
  T acc = T(0);
  for (int z = 0; z < nparts; ++z) acc += parts[(int64_t)z * stride + e];
  out[e] = acc;
}

int chunk_for(const Gemm& g, int align) {
  const int ks = std::max(1, g.ksplit);
  int c = (g.K + ks - 1) / ks;
  c = (c + align - 1) / align * align;
  return std::max(c, align);
}

}  // namespace

hipError_t gemm_f32(const Gemm& g, Prec prec, hipStream_t s) {
  (void)prec;
  const int kchunk = chunk_for(g, kTK);
  dim3 grid((unsigned)((g.M + kTM - 1) / kTM), (unsigned)((g.N + kTN - 1) / kTN),
            (unsigned)(g.batch * std::max(1, g.ksplit)));
  if (!g.ta && !g.tb) gemm_f32_kernel<false, false><<<grid, 256, 0, s>>>(g, kchunk);
  else if (!g.ta && g.tb) gemm_f32_kernel<false, true><<<grid, 256, 0, s>>>(g, kchunk);
  else if (g.ta && !g.tb) gemm_f32_kernel<true, false><<<grid, 256, 0, s>>>(g, kchunk);
  else gemm_f32_kernel<true, true><<<grid, 256, 0, s>>>(g, kchunk);
  return hipGetLastError();
}

hipError_t gemm_f64(const Gemm& g, hipStream_t s) {
  const int kchunk = chunk_for(g, 1);
  dim3 grid((unsigned)((g.M + 15) / 16), (unsigned)((g.N + 15) / 16),
            (unsigned)(g.batch * std::max(1, g.ksplit)));
  gemm_generic_kernel<double><<<grid, 256, 0, s>>>(g, kchunk);
  return hipGetLastError();
}

hipError_t sum_partials_f32(const float* parts, int nparts, int64_t stride, int64_t count,
                            float* out, hipStream_t s) {
  sum_partials_kernel<float><<<(unsigned)((count + 255) / 256), 256, 0, s>>>(parts, nparts, stride,
                                                                           count, out);
  return hipGetLastError();
}

hipError_t sum_partials_f64(const double* parts, int nparts, int64_t stride, int64_t count,
                            double* out, hipStream_t s) {
  sum_partials_kernel<double><<<(unsigned)((count + 255) / 256), 256, 0, s>>>(parts, nparts, stride,
                                                                            count, out);
  return hipGetLastError();
}

}  // namespace pq
