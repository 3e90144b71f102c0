// Mode-3 transforms of the projected product (Def. 2.2 with M = Q^T and
// M = Q; Def. 3.1): hat, unhat and the fused projection, on gfx950.
//
// Storage: an n1 x n2 x n3 face-major tensor is the row-major n3 x N matrix
// (N = n1 n2) whose row t is frontal slice t, so a transform is a skinny
// GEMM whose long dimension runs along the contiguous tube index.  A wave
// owns a strip of 32*VEC consecutive tubes; per MFMA step it reads two rows
// of the strip with VEC-wide coalesced loads, and the VEC columns of every
// lane become VEC independent 32x32x2 float32 MFMAs (the tube index of MFMA
// column n, sub-step q is 32*VEC*strip + VEC*n + q), so results leave the
// accumulators as VEC-wide contiguous stores too.
#include <algorithm>
#include <initializer_list>

#include "common.hpp"
#include "internal.hpp"

namespace pq {
namespace {

constexpr int kKC = 128;  // rows of Q staged in LDS per chunk (hat)

// acc[q] += Q(rows kc.., lc + m)^T * A(rows kc.., strip) over `rows` rows;
// Qs is the LDS copy of those rows of the 32-column chunk, leading dim ldq.
template <int VEC, typename TIn>
__device__ __forceinline__ void hat_accumulate(const TIn* __restrict__ Ap, int64_t N, bool active,
                                               int rows, int rows_valid, const float* Qs, int ldq,
                                               int n, int kh, f32x16 (&acc)[VEC]) {
  int r = 0;
  for (; r + 16 <= rows_valid; r += 16) {
    float b[8][VEC];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      if (active) {
        load_vec<VEC>(Ap + (int64_t)(r + 2 * s + kh) * N, b[s]);
      } else {
#pragma unroll
        for (int q = 0; q < VEC; ++q) b[s][q] = 0.f;
      }
    }
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const float a = Qs[(r + 2 * s + kh) * ldq + n];
#pragma unroll
      for (int q = 0; q < VEC; ++q)
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b[s][q], acc[q], 0, 0, 0);
    }
  }
  for (; r < rows_valid; r += 2) {
    const int t = r + kh;
    float b[VEC];
    if (active && t < rows_valid) {
      load_vec<VEC>(Ap + (int64_t)t * N, b);
    } else {
#pragma unroll
      for (int q = 0; q < VEC; ++q) b[q] = 0.f;
    }
    const float a = Qs[t * ldq + n];  // row rows_valid of Qs is zero-filled
#pragma unroll
    for (int q = 0; q < VEC; ++q)
      acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b[q], acc[q], 0, 0, 0);
  }
  (void)rows;
}

template <int VEC, int WAVES, typename TIn>
__global__ __launch_bounds__(WAVES * 64) void hat_f32_kernel(const TIn* __restrict__ A,
                                                             const float* __restrict__ Q,
                                                             float* __restrict__ Ah, int64_t N,
                                                             int n3, int p) {
  __shared__ float Qs[(kKC + 2) * 32];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = lane & 31, kh = lane >> 5;
  const int lc = blockIdx.y * 32;
  const int64_t xl = ((int64_t)blockIdx.x * WAVES + wave) * (32 * VEC) + (int64_t)VEC * n;
  const bool active = xl < N;
  f32x16 acc[VEC];
#pragma unroll
  for (int q = 0; q < VEC; ++q)
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[q][j] = 0.f;
  for (int kc = 0; kc < n3; kc += kKC) {
    const int rows = min(kKC, n3 - kc);
    __syncthreads();
    for (int e = threadIdx.x; e < (kKC + 2) * 32; e += WAVES * 64) {
      const int r = e >> 5, c = e & 31;
      Qs[e] = (r < rows && lc + c < p) ? Q[(int64_t)(kc + r) * p + lc + c] : 0.f;
    }
    __syncthreads();
    hat_accumulate<VEC, TIn>(A + (int64_t)kc * N + xl, N, active, rows, rows, Qs, 32, n, kh, acc);
  }
  if (!active) return;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int l = lc + 8 * (j >> 2) + 4 * kh + (j & 3);
    if (l < p) {
      float v[VEC];
#pragma unroll
      for (int q = 0; q < VEC; ++q) v[q] = acc[q][j];
      store_vec<VEC>(Ah + (int64_t)l * N + xl, v);
    }
  }
}

template <int VEC, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void unhat_f32_kernel(const float* __restrict__ Ah,
                                                               const float* __restrict__ Q,
                                                               float* __restrict__ C, int64_t N,
                                                               int n3, int p) {
  extern __shared__ float QsT[];  // [p_pad][32]: Q(t0 + tt, l) at l*32 + tt
  const int p_pad = (p + 1) & ~1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = lane & 31, kh = lane >> 5;
  const int64_t xl = ((int64_t)blockIdx.x * WAVES + wave) * (32 * VEC) + (int64_t)VEC * n;
  const bool active = xl < N;
  const int ntiles = (n3 + 31) / 32;
  const bool regB = p <= 32;
  float breg[16][VEC];
  if (regB) {
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int l = 2 * s + kh;
      if (active && l < p) {
        load_vec<VEC, float>(Ah + (int64_t)l * N + xl, breg[s]);
      } else {
#pragma unroll
        for (int q = 0; q < VEC; ++q) breg[s][q] = 0.f;
      }
    }
  }
  for (int tile = blockIdx.y; tile < ntiles; tile += gridDim.y) {
    const int t0 = tile * 32;
    __syncthreads();
    for (int e = threadIdx.x; e < p_pad * 32; e += WAVES * 64) {
      const int l = e >> 5, tt = e & 31;
      QsT[e] = (t0 + tt < n3 && l < p) ? Q[(int64_t)(t0 + tt) * p + l] : 0.f;
    }
    __syncthreads();
    f32x16 acc[VEC];
#pragma unroll
    for (int q = 0; q < VEC; ++q)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[q][j] = 0.f;
    if (regB) {
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        if (2 * s < p) {
          const float a = QsT[(2 * s + kh) * 32 + n];
#pragma unroll
          for (int q = 0; q < VEC; ++q)
            acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, breg[s][q], acc[q], 0, 0, 0);
        }
      }
    } else {
      for (int l0 = 0; l0 < p; l0 += 2) {
        const int l = l0 + kh;
        float b[VEC];
        if (active && l < p) {
          load_vec<VEC, float>(Ah + (int64_t)l * N + xl, b);
        } else {
#pragma unroll
          for (int q = 0; q < VEC; ++q) b[q] = 0.f;
        }
        const float a = QsT[l * 32 + n];
#pragma unroll
        for (int q = 0; q < VEC; ++q)
          acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b[q], acc[q], 0, 0, 0);
      }
    }
    if (active) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int t = t0 + 8 * (j >> 2) + 4 * kh + (j & 3);
        if (t < n3) {
          float v[VEC];
#pragma unroll
          for (int q = 0; q < VEC; ++q) v[q] = acc[q][j];
          store_vec<VEC>(C + (int64_t)t * N + xl, v);
        }
      }
    }
  }
}

// Fused projection, p <= 32: hat of the strip into the accumulators, then the
// accumulators feed the unhat MFMAs directly.  For unhat step j a lane
// supplies, as its B operand, its accumulator register j, which holds
// transform row l = 8*(j/4) + 4*kh + j%4 of its tube; the A operand it
// supplies is Q(t, l) for that same l, so each step contracts over the two
// rows held by the two half-waves and no data moves between lanes.
template <int VEC, int WAVES, typename TIn>
__global__ __launch_bounds__(WAVES * 64) void proj_f32_kernel(const TIn* __restrict__ A,
                                                              const float* __restrict__ Q,
                                                              float* __restrict__ out, int64_t N,
                                                              int n3, int p) {
  extern __shared__ float Qs[];  // [rows_pad][33]
  constexpr int ld = 33;
  const int ntiles = (n3 + 31) / 32;
  const int rows_pad = ntiles * 32 + 2;
  for (int e = threadIdx.x; e < rows_pad * ld; e += WAVES * 64) {
    const int r = e / ld, c = e - r * ld;
    Qs[e] = (r < n3 && c < p) ? Q[(int64_t)r * p + c] : 0.f;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = lane & 31, kh = lane >> 5;
  const int64_t xl = ((int64_t)blockIdx.x * WAVES + wave) * (32 * VEC) + (int64_t)VEC * n;
  const bool active = xl < N;
  f32x16 h[VEC];
#pragma unroll
  for (int q = 0; q < VEC; ++q)
#pragma unroll
    for (int j = 0; j < 16; ++j) h[q][j] = 0.f;
  hat_accumulate<VEC, TIn>(A + xl, N, active, n3, n3, Qs, ld, n, kh, h);
  for (int tile = 0; tile < ntiles; ++tile) {
    const int t0 = tile * 32;
    f32x16 acc[VEC];
#pragma unroll
    for (int q = 0; q < VEC; ++q)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[q][j] = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int lbase = 8 * (j >> 2) + (j & 3);
      if (lbase < p) {
        const float a = Qs[(t0 + n) * ld + lbase + 4 * kh];
#pragma unroll
        for (int q = 0; q < VEC; ++q)
          acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, h[q][j], acc[q], 0, 0, 0);
      }
    }
    if (active) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int t = t0 + 8 * (j >> 2) + 4 * kh + (j & 3);
        if (t < n3) {
          float v[VEC];
#pragma unroll
          for (int q = 0; q < VEC; ++q) v[q] = acc[q][j];
          store_vec<VEC>(out + (int64_t)t * N + xl, v);
        }
      }
    }
  }
}

// ---- float64 (plain VALU; the float64 path serves small problems) --------
template <typename T>
__global__ __launch_bounds__(256) void hat_generic_kernel(const T* __restrict__ A,
                                                          const T* __restrict__ Q,
                                                          T* __restrict__ Ah, int64_t N, int n3,
                                                          int p) {
  __shared__ T Qs[64][32];
  const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int lc = blockIdx.y * 32;
  T acc[32];
#pragma unroll
  for (int c = 0; c < 32; ++c) acc[c] = T(0);
  for (int kc = 0; kc < n3; kc += 64) {
    const int rows = min(64, n3 - kc);
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 32; e += 256) {
      const int r = e >> 5, c = e & 31;
      Qs[r][c] = (r < rows && lc + c < p) ? Q[(int64_t)(kc + r) * p + lc + c] : T(0);
    }
    __syncthreads();
    if (x < N) {
      for (int r = 0; r < rows; ++r) {
        const T a = A[(int64_t)(kc + r) * N + x];
#pragma unroll
        for (int c = 0; c < 32; ++c) acc[c] = fma(Qs[r][c], a, acc[c]);
      }
    }
  }
  if (x >= N) return;
  for (int c = 0; c < 32 && lc + c < p; ++c) Ah[(int64_t)(lc + c) * N + x] = acc[c];
}

template <typename T>
__global__ __launch_bounds__(256) void unhat_generic_kernel(const T* __restrict__ Ah,
                                                            const T* __restrict__ Q,
                                                            T* __restrict__ C, int64_t N, int n3,
                                                            int p) {
  const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int t = blockIdx.y;
  if (x >= N || t >= n3) return;
  T acc = T(0);
  for (int l = 0; l < p; ++l) acc = fma(Q[(int64_t)t * p + l], Ah[(int64_t)l * N + x], acc);
  C[(int64_t)t * N + x] = acc;
}

// Widest vector that divides N and the alignment of every base pointer.
int pick_vec(int64_t N, std::initializer_list<const void*> ptrs, int elem) {
  for (int v : {4, 2}) {
    if (N % v) continue;
    bool ok = true;
    for (const void* ptr : ptrs)
      if (reinterpret_cast<uintptr_t>(ptr) % (size_t)(v * elem)) ok = false;
    if (ok) return v;
  }
  return 1;
}

constexpr int kWaves = 4;

template <int VEC, typename TIn>
hipError_t hat_f32_vec(const TIn* A, const float* Q, float* Ah, int64_t N, int n3, int p,
                       hipStream_t s) {
  const int64_t strips = (N + 32 * VEC - 1) / (32 * VEC);
  dim3 grid((unsigned)((strips + kWaves - 1) / kWaves), (unsigned)((p + 31) / 32));
  hat_f32_kernel<VEC, kWaves, TIn><<<grid, kWaves * 64, 0, s>>>(A, Q, Ah, N, n3, p);
  return hipGetLastError();
}

template <int VEC>
hipError_t unhat_f32_vec(const float* Ah, const float* Q, float* C, int64_t N, int n3, int p,
                         hipStream_t s) {
  const int64_t strips = (N + 32 * VEC - 1) / (32 * VEC);
  const int64_t wgs = (strips + kWaves - 1) / kWaves;
  const int ntiles = (n3 + 31) / 32;
  // enough workgroups to fill 256 CUs several times over
  int ysplit = (int)std::min<int64_t>(ntiles, std::max<int64_t>(1, (2048 + wgs - 1) / wgs));
  const size_t lds = (size_t)((p + 1) & ~1) * 32 * sizeof(float);
  dim3 grid((unsigned)wgs, (unsigned)ysplit);
  unhat_f32_kernel<VEC, kWaves><<<grid, kWaves * 64, lds, s>>>(Ah, Q, C, N, n3, p);
  return hipGetLastError();
}

template <int VEC, typename TIn>
hipError_t proj_f32_vec(const TIn* A, const float* Q, float* out, int64_t N, int n3, int p,
                        hipStream_t s) {
  const int64_t strips = (N + 32 * VEC - 1) / (32 * VEC);
  const int ntiles = (n3 + 31) / 32;
  const size_t lds = (size_t)(ntiles * 32 + 2) * 33 * sizeof(float);
  dim3 grid((unsigned)((strips + kWaves - 1) / kWaves));
  proj_f32_kernel<VEC, kWaves, TIn><<<grid, kWaves * 64, lds, s>>>(A, Q, out, N, n3, p);
  return hipGetLastError();
}

}  // namespace

hipError_t hat_f32(const void* A, bool a_bf16, const float* Q, float* Ah, int64_t N, int n3, int p,
                   Prec prec, hipStream_t s) {
  if (prec != Prec::Default) return hipErrorNotSupported;
  if (a_bf16) {
    const uint16_t* a = static_cast<const uint16_t*>(A);
    switch (std::min(pick_vec(N, {A}, 2), pick_vec(N, {Ah}, 4))) {
      case 4: return hat_f32_vec<4>(a, Q, Ah, N, n3, p, s);
      case 2: return hat_f32_vec<2>(a, Q, Ah, N, n3, p, s);
      default: return hat_f32_vec<1>(a, Q, Ah, N, n3, p, s);
    }
  }
  const float* a = static_cast<const float*>(A);
  switch (pick_vec(N, {A, Ah}, 4)) {
    case 4: return hat_f32_vec<4>(a, Q, Ah, N, n3, p, s);
    case 2: return hat_f32_vec<2>(a, Q, Ah, N, n3, p, s);
    default: return hat_f32_vec<1>(a, Q, Ah, N, n3, p, s);
  }
}

hipError_t unhat_f32(const float* Ah, const float* Q, float* C, int64_t N, int n3, int p,
                     Prec prec, hipStream_t s) {
  if (prec != Prec::Default) return hipErrorNotSupported;
  switch (pick_vec(N, {Ah, C}, 4)) {
    case 4: return unhat_f32_vec<4>(Ah, Q, C, N, n3, p, s);
    case 2: return unhat_f32_vec<2>(Ah, Q, C, N, n3, p, s);
    default: return unhat_f32_vec<1>(Ah, Q, C, N, n3, p, s);
  }
}

bool proj_fused_ok(int n3, int p) { return p <= 32 && n3 <= 480; }

hipError_t proj_fused_f32(const void* A, bool a_bf16, const float* Q, float* out, int64_t N, int n3,
                          int p, Prec prec, hipStream_t s) {
  if (prec != Prec::Default) return hipErrorNotSupported;
  if (a_bf16) {
    const uint16_t* a = static_cast<const uint16_t*>(A);
    switch (std::min(pick_vec(N, {A}, 2), pick_vec(N, {out}, 4))) {
      case 4: return proj_f32_vec<4>(a, Q, out, N, n3, p, s);
      case 2: return proj_f32_vec<2>(a, Q, out, N, n3, p, s);
      default: return proj_f32_vec<1>(a, Q, out, N, n3, p, s);
    }
  }
  const float* a = static_cast<const float*>(A);
  switch (pick_vec(N, {A, out}, 4)) {
    case 4: return proj_f32_vec<4>(a, Q, out, N, n3, p, s);
    case 2: return proj_f32_vec<2>(a, Q, out, N, n3, p, s);
    default: return proj_f32_vec<1>(a, Q, out, N, n3, p, s);
  }
}

hipError_t hat_f64(const double* A, const double* Q, double* Ah, int64_t N, int n3, int p,
                   hipStream_t s) {
  dim3 grid((unsigned)((N + 255) / 256), (unsigned)((p + 31) / 32));
  hat_generic_kernel<double><<<grid, 256, 0, s>>>(A, Q, Ah, N, n3, p);
  return hipGetLastError();
}

hipError_t unhat_f64(const double* Ah, const double* Q, double* C, int64_t N, int n3, int p,
                     hipStream_t s) {
  dim3 grid((unsigned)((N + 255) / 256), (unsigned)n3);
  unhat_generic_kernel<double><<<grid, 256, 0, s>>>(Ah, Q, C, N, n3, p);
  return hipGetLastError();
}

}  // namespace pq
