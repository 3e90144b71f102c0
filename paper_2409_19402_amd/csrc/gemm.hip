// Batched dense GEMM for the facewise product (Def. 2.3) and the other
// contractions of the path (the transposed facewise products of the adjoint,
// the split-K reductions over the n1 n2 tubes that give dQ, the factor
// products of the truncated SVD).
//
// float32: a 64x64 output tile per 256-thread workgroup, K tiles of 32 or 128
// double-buffered in LDS, one 32x32 tile per wave on v_mfma_f32_32x32x2f32.
// The split-bfloat16 modes use the same pipeline on v_mfma_f32_32x32x16_bf16.
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace pq {
namespace {

constexpr int kTM = 64, kTN = 64, kLd = 68;

// One K-tile of KT rows: the 64 x KT block of A (as As[k][m]) or the KT x 64
// block of B (as Bs[k][n]), KT / 4 elements per thread, fetched into
// registers.  VEC = 4 reads float4 along the operand's contiguous dimension
// (the host guarantees that dimension, the leading dimension, the strides and
// the base are multiples of 4), VEC = 1 reads scalars.  Elements outside the
// matrix or past kend are 0.  CONT_ROW: the contiguous dimension is the
// tile's row index (m or n) rather than k.
template <int KT>
struct TileRegs {
  float v[KT / 4];
};

template <int KT, int VEC, bool CONT_ROW>
__device__ __forceinline__ void tile_fetch(const float* __restrict__ P, int64_t ld, int r0, int rmax, int k0,
                                           int kend, TileRegs<KT>& t) {
  const int tid = threadIdx.x;
  if constexpr (VEC == 4) {
#pragma unroll
    for (int h = 0; h < KT / 16; ++h) {
      const int idx = tid + 256 * h;
      int r, k;
      if (CONT_ROW) { k = idx >> 4; r = 4 * (idx & 15); } else { r = idx / (KT / 4); k = 4 * (idx % (KT / 4)); }
      const int gr = r0 + r, gk = k0 + k;
      const bool ok = gr < rmax && gk < kend;  // whole float4 in or out (sizes are multiples of 4)
      const int cr = ok ? gr : 0, ck = ok ? gk : 0;
      const float4 x = CONT_ROW ? *reinterpret_cast<const float4*>(P + cr + (int64_t)ck * ld)
                                : *reinterpret_cast<const float4*>(P + ck + (int64_t)cr * ld);
      t.v[4 * h + 0] = ok ? x.x : 0.f;
      t.v[4 * h + 1] = ok ? x.y : 0.f;
      t.v[4 * h + 2] = ok ? x.z : 0.f;
      t.v[4 * h + 3] = ok ? x.w : 0.f;
    }
  } else {
#pragma unroll
    for (int h = 0; h < KT / 4; ++h) {
      const int idx = tid + 256 * h;
      int r, k;
      if (CONT_ROW) { k = idx >> 6; r = idx & 63; } else { r = idx / KT; k = idx % KT; }
      const int gr = r0 + r, gk = k0 + k;
      const bool ok = gr < rmax && gk < kend;
      const int cr = ok ? gr : 0, ck = ok ? gk : 0;
      const float x = CONT_ROW ? P[cr + (int64_t)ck * ld] : P[ck + (int64_t)cr * ld];
      t.v[h] = ok ? x : 0.f;
    }
  }
}

template <int KT, int VEC, bool CONT_ROW>
__device__ __forceinline__ void tile_store(const TileRegs<KT>& t, float* S) {  // S: KT x kLd
  const int tid = threadIdx.x;
  if constexpr (VEC == 4) {
#pragma unroll
    for (int h = 0; h < KT / 16; ++h) {
      const int idx = tid + 256 * h;
      if (CONT_ROW) {
        const int k = idx >> 4, r = 4 * (idx & 15);
        *reinterpret_cast<float4*>(S + k * kLd + r) =
            make_float4(t.v[4 * h], t.v[4 * h + 1], t.v[4 * h + 2], t.v[4 * h + 3]);
      } else {
        const int r = idx / (KT / 4), k = 4 * (idx % (KT / 4));
#pragma unroll
        for (int i = 0; i < 4; ++i) S[(k + i) * kLd + r] = t.v[4 * h + i];
      }
    }
  } else {
#pragma unroll
    for (int h = 0; h < KT / 4; ++h) {
      const int idx = tid + 256 * h;
      int r, k;
      if (CONT_ROW) { k = idx >> 6; r = idx & 63; } else { r = idx / KT; k = idx % KT; }
      S[k * kLd + r] = t.v[h];
    }
  }
}

// C tile (64 x 64) = A (64 x K) B (K x 64) over K-tiles of KT, double
// buffered in LDS (dynamic: 4 KT kLd floats): the next tile's global loads
// are in flight while the MFMAs of the current one run.  The MFMA computes
// the transposed tile (rows = output columns), so the 32 lanes sharing an
// accumulator register hold 32 consecutive rows of the column-major output
// and stores coalesce.
template <bool TA, bool TB, int VA, int VB, int KT>
__global__ __launch_bounds__(256) void gemm_f32_kernel(Gemm g, int kchunk) {
  extern __shared__ __align__(16) float gsm[];
  // buffers: A at gsm + b * KT * kLd, B at gsm + (2 + b) * KT * kLd
  auto As = [&](int b) { return gsm + b * KT * kLd; };
  auto Bs = [&](int b) { return gsm + (2 + b) * KT * kLd; };
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
  // A(m, k) is contiguous in m unless transposed; B(k, n) is contiguous in k
  // unless transposed
  TileRegs<KT> ra, rb;
  int k0 = kbeg;
  if (k0 < kend) {
    tile_fetch<KT, VA, !TA>(A, g.lda, m0, g.M, k0, kend, ra);
    tile_fetch<KT, VB, TB>(B, g.ldb, n0, g.N, k0, kend, rb);
    tile_store<KT, VA, !TA>(ra, As(0));
    tile_store<KT, VB, TB>(rb, Bs(0));
  }
  __syncthreads();
  int buf = 0;
  for (; k0 < kend; k0 += KT) {
    const bool more = k0 + KT < kend;
    if (more) {
      tile_fetch<KT, VA, !TA>(A, g.lda, m0, g.M, k0 + KT, kend, ra);
      tile_fetch<KT, VB, TB>(B, g.ldb, n0, g.N, k0 + KT, kend, rb);
    }
    // the whole tile, unrolled (rows past kend were staged as zeros), so the
    // LDS reads run ahead of the MFMAs
    const float* as = As(buf) + kh * kLd + wm * 32 + nl;  // columns of the transposed tile: output rows
    const float* bs = Bs(buf) + kh * kLd + wn * 32 + nl;  // rows of the transposed tile: output columns
#pragma unroll 16
    for (int kk = 0; kk < KT; kk += 2)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(bs[kk * kLd], as[kk * kLd], acc, 0, 0, 0);
    if (more) {
      tile_store<KT, VA, !TA>(ra, As(buf ^ 1));
      tile_store<KT, VB, TB>(rb, Bs(buf ^ 1));
    }
    __syncthreads();
    buf ^= 1;
  }
  const int gm = m0 + wm * 32 + nl;
  if (gm >= g.M) return;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int gn = n0 + wn * 32 + 8 * (j >> 2) + 4 * kh + (j & 3);
    if (gn < g.N) C[gm + (int64_t)gn * g.ldc] = acc[j];
  }
}

// ---- split-bfloat16 facewise GEMM --------------------------------------------
// The same 64 x 64 tile and double-buffered K pipeline as the float32 kernel;
// the tile is fetched as float32 and split into NP bfloat16 parts on its way
// into LDS, stored row-major with k contiguous ([row][k], row stride KT + 8)
// so that a lane reads the 8 consecutive k of its row as one 16-byte operand
// of v_mfma_f32_32x32x16_bf16.  The part products of Split<NP, NP> are
// accumulated in float32.
constexpr int kPad16 = 8;  // bfloat16 elements of padding per LDS row

template <int KT, int VEC, bool CONT_ROW, int NP>
__device__ __forceinline__ void tile_store_split(const TileRegs<KT>& t, uint16_t* S) {
  // S: NP parts, each 64 rows x (KT + kPad16) bfloat16
  constexpr int ld = KT + kPad16;
  constexpr int part = 64 * ld;
  const int tid = threadIdx.x;
  auto put = [&](int r, int k, float x) {
    uint32_t w[NP];
    split_pack<NP>(x, 0.f, w);
#pragma unroll
    for (int i = 0; i < NP; ++i) S[i * part + r * ld + k] = (uint16_t)(w[i] & 0xffffu);
  };
  if constexpr (VEC == 4) {
#pragma unroll
    for (int h = 0; h < KT / 16; ++h) {
      const int idx = tid + 256 * h;
      if (CONT_ROW) {
        const int k = idx >> 4, r = 4 * (idx & 15);
#pragma unroll
        for (int i = 0; i < 4; ++i) put(r + i, k, t.v[4 * h + i]);
      } else {  // four consecutive k of one row: two packed words per part
        const int r = idx / (KT / 4), k = 4 * (idx % (KT / 4));
        uint32_t w0[NP], w1[NP];
        split_pack<NP>(t.v[4 * h + 0], t.v[4 * h + 1], w0);
        split_pack<NP>(t.v[4 * h + 2], t.v[4 * h + 3], w1);
#pragma unroll
        for (int i = 0; i < NP; ++i)
          *reinterpret_cast<uint2*>(S + i * part + r * ld + k) = make_uint2(w0[i], w1[i]);
      }
    }
  } else {
#pragma unroll
    for (int h = 0; h < KT / 4; ++h) {
      const int idx = tid + 256 * h;
      int r, k;
      if (CONT_ROW) { k = idx >> 6; r = idx & 63; } else { r = idx / KT; k = idx % KT; }
      put(r, k, t.v[h]);
    }
  }
}

template <bool TA, bool TB, int VA, int VB, int KT, int NP>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(Gemm g, int kchunk) {
  using SP = Split<NP, NP>;
  constexpr int ld = KT + kPad16;
  constexpr int part = 64 * ld;  // bfloat16 elements per part
  extern __shared__ __align__(16) uint16_t hsm[];
  // buffers: A parts at hsm + b * NP * part, B parts at hsm + (2 + b) * NP * part
  auto Ap = [&](int b) { return hsm + b * NP * part; };
  auto Bp = [&](int b) { return hsm + (2 + b) * NP * part; };
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
  TileRegs<KT> ra, rb;
  int k0 = kbeg;
  if (k0 < kend) {
    tile_fetch<KT, VA, !TA>(A, g.lda, m0, g.M, k0, kend, ra);
    tile_fetch<KT, VB, TB>(B, g.ldb, n0, g.N, k0, kend, rb);
    tile_store_split<KT, VA, !TA, NP>(ra, Ap(0));
    tile_store_split<KT, VB, TB, NP>(rb, Bp(0));
  }
  __syncthreads();
  int buf = 0;
  for (; k0 < kend; k0 += KT) {
    const bool more = k0 + KT < kend;
    if (more) {
      tile_fetch<KT, VA, !TA>(A, g.lda, m0, g.M, k0 + KT, kend, ra);
      tile_fetch<KT, VB, TB>(B, g.ldb, n0, g.N, k0 + KT, kend, rb);
    }
    // rows of the transposed tile are output columns (B's n), its columns
    // output rows (A's m)
    const uint16_t* ap = Ap(buf) + (wm * 32 + nl) * ld + 8 * kh;
    const uint16_t* bp = Bp(buf) + (wn * 32 + nl) * ld + 8 * kh;
#pragma unroll
    for (int ks = 0; ks < KT; ks += 16) {
      bf16x8 pa[NP], pb[NP];
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        pa[i] = *reinterpret_cast<const bf16x8*>(ap + i * part + ks);
        pb[i] = *reinterpret_cast<const bf16x8*>(bp + i * part + ks);
      }
#pragma unroll
      for (int pr = 0; pr < SP::n; ++pr)
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pb[SP::q[pr]], pa[SP::a[pr]], acc, 0, 0, 0);
    }
    if (more) {
      tile_store_split<KT, VA, !TA, NP>(ra, Ap(buf ^ 1));
      tile_store_split<KT, VB, TB, NP>(rb, Bp(buf ^ 1));
    }
    __syncthreads();
    buf ^= 1;
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

// float4 loads along an operand's contiguous dimension need that dimension,
// its leading dimension, the batch and split strides and the base to be
// multiples of 4 floats
bool vec4_ok(const void* P, int64_t cont, int64_t ld, int64_t stride) {
  return reinterpret_cast<uintptr_t>(P) % 16 == 0 && cont % 4 == 0 && ld % 4 == 0 && stride % 4 == 0;
}

template <bool TA, bool TB, int VA, int VB, int KT>
hipError_t gemm_f32_go(const Gemm& g, int kchunk, dim3 grid, hipStream_t s) {
  const size_t lds = sizeof(float) * 4 * KT * kLd;
  static hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_f32_kernel<TA, TB, VA, VB, KT>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return attr;
  gemm_f32_kernel<TA, TB, VA, VB, KT><<<grid, 256, lds, s>>>(g, kchunk);
  return hipGetLastError();
}

template <bool TA, bool TB, int KT>
hipError_t gemm_f32_launch(const Gemm& g, int kchunk, dim3 grid, hipStream_t s) {
  // contiguous dimension: A's is M (K when transposed), B's is K (N when transposed)
  const bool va = vec4_ok(g.A, TA ? g.K : g.M, g.lda, g.sA) && (!TA || kchunk % 4 == 0);
  const bool vb = vec4_ok(g.B, TB ? g.N : g.K, g.ldb, g.sB) && (TB || kchunk % 4 == 0);
  if (va && vb) return gemm_f32_go<TA, TB, 4, 4, KT>(g, kchunk, grid, s);
  if (va) return gemm_f32_go<TA, TB, 4, 1, KT>(g, kchunk, grid, s);
  if (vb) return gemm_f32_go<TA, TB, 1, 4, KT>(g, kchunk, grid, s);
  return gemm_f32_go<TA, TB, 1, 1, KT>(g, kchunk, grid, s);
}

template <bool TA, bool TB, int VA, int VB, int KT, int NP>
hipError_t gemm_bf16_go(const Gemm& g, int kchunk, dim3 grid, hipStream_t s) {
  const size_t lds = sizeof(uint16_t) * 4 * NP * 64 * (KT + kPad16);
  static hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_bf16_kernel<TA, TB, VA, VB, KT, NP>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return attr;
  gemm_bf16_kernel<TA, TB, VA, VB, KT, NP><<<grid, 256, lds, s>>>(g, kchunk);
  return hipGetLastError();
}

template <bool TA, bool TB, int KT, int NP>
hipError_t gemm_bf16_launch(const Gemm& g, int kchunk, dim3 grid, hipStream_t s) {
  const bool va = vec4_ok(g.A, TA ? g.K : g.M, g.lda, g.sA) && (!TA || kchunk % 4 == 0);
  const bool vb = vec4_ok(g.B, TB ? g.N : g.K, g.ldb, g.sB) && (TB || kchunk % 4 == 0);
  if (va && vb) return gemm_bf16_go<TA, TB, 4, 4, KT, NP>(g, kchunk, grid, s);
  if (va) return gemm_bf16_go<TA, TB, 4, 1, KT, NP>(g, kchunk, grid, s);
  if (vb) return gemm_bf16_go<TA, TB, 1, 4, KT, NP>(g, kchunk, grid, s);
  return gemm_bf16_go<TA, TB, 1, 1, KT, NP>(g, kchunk, grid, s);
}

template <bool TA, bool TB>
hipError_t gemm_launch(const Gemm& g, Prec prec, int kchunk, dim3 grid, hipStream_t s) {
  const bool deep = kchunk >= 96;
  switch (prec) {
    case Prec::BF16:
      return deep ? gemm_bf16_launch<TA, TB, 128, 1>(g, kchunk, grid, s)
                  : gemm_bf16_launch<TA, TB, 32, 1>(g, kchunk, grid, s);
    case Prec::BF16x3:
      return deep ? gemm_bf16_launch<TA, TB, 128, 2>(g, kchunk, grid, s)
                  : gemm_bf16_launch<TA, TB, 32, 2>(g, kchunk, grid, s);
    case Prec::BF16x6:
      return deep ? gemm_bf16_launch<TA, TB, 64, 3>(g, kchunk, grid, s)
                  : gemm_bf16_launch<TA, TB, 32, 3>(g, kchunk, grid, s);
    default:
      return deep ? gemm_f32_launch<TA, TB, 128>(g, kchunk, grid, s)
                  : gemm_f32_launch<TA, TB, 32>(g, kchunk, grid, s);
  }
}

hipError_t gemm_f32(const Gemm& g, Prec prec, hipStream_t s) {
  // deep K-tiles (one global round trip covers up to 128 of K) when a
  // workgroup has that much K
  const int kchunk = chunk_for(g, 32);
  dim3 grid((unsigned)((g.M + kTM - 1) / kTM), (unsigned)((g.N + kTN - 1) / kTN),
            (unsigned)(g.batch * std::max(1, g.ksplit)));
  if (!g.ta && !g.tb) return gemm_launch<false, false>(g, prec, kchunk, grid, s);
  if (!g.ta && g.tb) return gemm_launch<false, true>(g, prec, kchunk, grid, s);
  if (g.ta && !g.tb) return gemm_launch<true, false>(g, prec, kchunk, grid, s);
  return gemm_launch<true, true>(g, prec, kchunk, grid, s);
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
