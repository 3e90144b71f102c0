// Batched dense GEMM for the facewise product (Def. 2.3) and the other
// contractions of the path (the transposed facewise products of the adjoint,
// the split-K reductions over the n1 n2 tubes that give dQ, the factor
// products of the truncated SVD).
//
// float32: a 64x64 output tile per 256-thread workgroup, K tiles of 32 or 128
// double-buffered in LDS, one 32x32 tile per wave on v_mfma_f32_32x32x2f32.
// The split-bfloat16 modes use the same pipeline on v_mfma_f32_32x32x16_bf16.
// float64: 64x64 or 64x16 output tiles on v_mfma_f64_16x16x4f64.
#include <algorithm>
#include <cstdio>

#include "common.hpp"
#include "internal.hpp"

namespace pq {
namespace {

// Output tiles: 64 x 64, or 32 x 128 when the output has at most 32 rows
// (the dQ products, M = p), both four 32 x 32 wave tiles.
//
// LDS floats of one staged K-tile of R rows: k-major ([k][row], row stride
// R + 4) for an operand that is contiguous along its row index, row-major
// ([row][k], row stride KT + 4) for one that is contiguous along k, so that
// both the float4 stores and the MFMA operand reads avoid bank conflicts.
template <int R, int KT>
__host__ __device__ constexpr int tile_floats() {
  return KT * (R + 4) > R * (KT + 4) ? KT * (R + 4) : R * (KT + 4);
}

// One K-tile of KT rows: the R x KT block of A or the KT x R block of B,
// R KT / 256 elements per thread, fetched into registers.  VEC = 4 reads
// float4 along the operand's contiguous dimension (the host guarantees that
// dimension, the leading dimension, the strides and the base are multiples
// of 4), VEC = 1 reads scalars.  Elements outside the matrix or past kend
// are 0.  CONT_ROW: the contiguous dimension is the tile's row index (m or
// n) rather than k.
template <int R, int KT>
struct TileRegs {
  float v[R * KT / 256];
};

template <int R, int KT, int VEC, bool CONT_ROW>
__device__ __forceinline__ void tile_fetch(const float* __restrict__ P, int64_t ld, int r0, int rmax, int k0,
                                           int kend, TileRegs<R, KT>& t) {
  const int tid = threadIdx.x;
  if constexpr (VEC == 4) {
#pragma unroll
    for (int h = 0; h < R * KT / 1024; ++h) {
      const int idx = tid + 256 * h;
      int r, k;
      if (CONT_ROW) { k = idx / (R / 4); r = 4 * (idx % (R / 4)); } else { r = idx / (KT / 4); k = 4 * (idx % (KT / 4)); }
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
    for (int h = 0; h < R * KT / 256; ++h) {
      const int idx = tid + 256 * h;
      int r, k;
      if (CONT_ROW) { k = idx / R; r = idx % R; } else { r = idx / KT; k = idx % KT; }
      const int gr = r0 + r, gk = k0 + k;
      const bool ok = gr < rmax && gk < kend;
      const int cr = ok ? gr : 0, ck = ok ? gk : 0;
      const float x = CONT_ROW ? P[cr + (int64_t)ck * ld] : P[ck + (int64_t)cr * ld];
      t.v[h] = ok ? x : 0.f;
    }
  }
}

// S: the tile in the layout tile_floats describes (CONT_ROW: [k][row])
template <int R, int KT, int VEC, bool CONT_ROW>
__device__ __forceinline__ void tile_store(const TileRegs<R, KT>& t, float* S) {
  constexpr int ldr = R + 4, ldk = KT + 4;
  const int tid = threadIdx.x;
  if constexpr (VEC == 4) {
#pragma unroll
    for (int h = 0; h < R * KT / 1024; ++h) {
      const int idx = tid + 256 * h;
      const float4 x = make_float4(t.v[4 * h], t.v[4 * h + 1], t.v[4 * h + 2], t.v[4 * h + 3]);
      if (CONT_ROW) {
        *reinterpret_cast<float4*>(S + (idx / (R / 4)) * ldr + 4 * (idx % (R / 4))) = x;
      } else {
        *reinterpret_cast<float4*>(S + (idx / (KT / 4)) * ldk + 4 * (idx % (KT / 4))) = x;
      }
    }
  } else {
#pragma unroll
    for (int h = 0; h < R * KT / 256; ++h) {
      const int idx = tid + 256 * h;
      if (CONT_ROW) {
        S[(idx / R) * ldr + idx % R] = t.v[h];
      } else {
        S[(idx / KT) * ldk + idx % KT] = t.v[h];
      }
    }
  }
}

// Workgroups are dealt to the 8 XCDs round robin by their linear index, and
// each XCD has its own L2.  With grouped set the grid is one-dimensional and
// every tile of one slab z (a batch entry and K-slice, whose operand rows
// the tiles share) runs on the XCD z mod 8, so that the slab is fetched into
// one L2 instead of all eight.
constexpr int kXcds = 8;
constexpr int kCUs = 256;
struct TileIdx {
  int x, y, z;
};
__device__ __forceinline__ TileIdx tile_idx(bool grouped, int mt, int nt) {
  if (!grouped) return {(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z};
  const int b = blockIdx.x, m = b / kXcds, per = mt * nt;
  const int t = m % per;
  return {t % mt, t / mt, b % kXcds + kXcds * (m / per)};
}

// C tile (TM x TN) = A (TM x K) B (K x TN) over K-tiles of KT, double
// buffered in LDS (dynamic: 2 (tile_floats<TM, KT>() + tile_floats<TN, KT>())
// floats): the next tile's global loads are in flight while the MFMAs of the
// current one run.  The MFMA computes the transposed tile (rows = output
// columns), so the 32 lanes sharing an accumulator register hold 32
// consecutive rows of the column-major output and stores coalesce.  MFMA
// step j of a K-tile takes k = j in lanes 0-31 and k = KT/2 + j in lanes
// 32-63, so that a lane's k are consecutive and a row-major operand is read
// four steps at a time.
template <bool TA, bool TB, int VA, int VB, int KT, int TM>
__global__ __launch_bounds__(256) void gemm_f32_kernel(Gemm g, int kchunk, bool grouped) {
  constexpr int TN = 4096 / TM;
  constexpr int WM = TM / 32;  // wave grid WM x (4 / WM)
  extern __shared__ __align__(16) float gsm[];
  constexpr int FA = tile_floats<TM, KT>(), FB = tile_floats<TN, KT>();
  constexpr int H = KT / 2, ldk = KT + 4;
  // buffers: A at gsm + b FA, B at gsm + 2 FA + b FB
  auto As = [&](int b) { return gsm + b * FA; };
  auto Bs = [&](int b) { return gsm + 2 * FA + b * FB; };
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int nl = lane & 31, kh = lane >> 5;
  const int wm = wave % WM, wn = wave / WM;
  const TileIdx ti = tile_idx(grouped, (g.M + TM - 1) / TM, (g.N + TN - 1) / TN);
  if (ti.z >= g.batch * max(1, g.ksplit)) return;  // the grouped grid's last slots
  const int zb = ti.z % g.batch, zs = ti.z / g.batch;
  const int m0 = ti.x * TM, n0 = ti.y * TN;
  const int kbeg = zs * kchunk, kend = min(g.K, kbeg + kchunk);
  const float* A = static_cast<const float*>(g.A) + (int64_t)zb * g.sA;
  const float* B = static_cast<const float*>(g.B) + (int64_t)zb * g.sB;
  float* C = static_cast<float*>(g.C) + (int64_t)zb * g.sC + (int64_t)zs * g.sSplit;
  f32x16 acc;
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = 0.f;
  // A(m, k) is contiguous in m unless transposed; B(k, n) is contiguous in k
  // unless transposed
  TileRegs<TM, KT> ra;
  TileRegs<TN, KT> rb;
  int k0 = kbeg;
  if (k0 < kend) {
    tile_fetch<TM, KT, VA, !TA>(A, g.lda, m0, g.M, k0, kend, ra);
    tile_fetch<TN, KT, VB, TB>(B, g.ldb, n0, g.N, k0, kend, rb);
    tile_store<TM, KT, VA, !TA>(ra, As(0));
    tile_store<TN, KT, VB, TB>(rb, Bs(0));
  }
  __syncthreads();
  int buf = 0;
  for (; k0 < kend; k0 += KT) {
    const bool more = k0 + KT < kend;
    if (more) {
      tile_fetch<TM, KT, VA, !TA>(A, g.lda, m0, g.M, k0 + KT, kend, ra);
      tile_fetch<TN, KT, VB, TB>(B, g.ldb, n0, g.N, k0 + KT, kend, rb);
    }
    // the whole tile, unrolled (rows past kend were staged as zeros), so the
    // LDS reads run ahead of the MFMAs; A's rows are the output rows (the
    // columns of the transposed tile), B's the output columns
    const float* as = !TA ? As(buf) + kh * H * (TM + 4) + wm * 32 + nl : As(buf) + (wm * 32 + nl) * ldk + kh * H;
    const float* bs = TB ? Bs(buf) + kh * H * (TN + 4) + wn * 32 + nl : Bs(buf) + (wn * 32 + nl) * ldk + kh * H;
#pragma unroll
    for (int q = 0; q < H; q += 4) {
      float a[4], b[4];
      if constexpr (!TA) {
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = as[(q + i) * (TM + 4)];
      } else {
        const float4 v = *reinterpret_cast<const float4*>(as + q);
        a[0] = v.x; a[1] = v.y; a[2] = v.z; a[3] = v.w;
      }
      if constexpr (TB) {
#pragma unroll
        for (int i = 0; i < 4; ++i) b[i] = bs[(q + i) * (TN + 4)];
      } else {
        const float4 v = *reinterpret_cast<const float4*>(bs + q);
        b[0] = v.x; b[1] = v.y; b[2] = v.z; b[3] = v.w;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(b[i], a[i], acc, 0, 0, 0);
    }
    if (more) {
      tile_store<TM, KT, VA, !TA>(ra, As(buf ^ 1));
      tile_store<TN, KT, VB, TB>(rb, Bs(buf ^ 1));
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
__device__ __forceinline__ void tile_store_split(const TileRegs<64, KT>& t, uint16_t* S) {
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
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  const int kbeg = zs * kchunk, kend = min(g.K, kbeg + kchunk);
  const float* A = static_cast<const float*>(g.A) + (int64_t)zb * g.sA;
  const float* B = static_cast<const float*>(g.B) + (int64_t)zb * g.sB;
  float* C = static_cast<float*>(g.C) + (int64_t)zb * g.sC + (int64_t)zs * g.sSplit;
  f32x16 acc;
#pragma unroll
  for (int j = 0; j < 16; ++j) acc[j] = 0.f;
  TileRegs<64, KT> ra, rb;
  int k0 = kbeg;
  if (k0 < kend) {
    tile_fetch<64, KT, VA, !TA>(A, g.lda, m0, g.M, k0, kend, ra);
    tile_fetch<64, KT, VB, TB>(B, g.ldb, n0, g.N, k0, kend, rb);
    tile_store_split<KT, VA, !TA, NP>(ra, Ap(0));
    tile_store_split<KT, VB, TB, NP>(rb, Bp(0));
  }
  __syncthreads();
  int buf = 0;
  for (; k0 < kend; k0 += KT) {
    const bool more = k0 + KT < kend;
    if (more) {
      tile_fetch<64, KT, VA, !TA>(A, g.lda, m0, g.M, k0 + KT, kend, ra);
      tile_fetch<64, KT, VB, TB>(B, g.ldb, n0, g.N, k0 + KT, kend, rb);
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

// ---- float64 GEMM -------------------------------------------------------------
// A 64 x TN output tile (TN = 64, or 16 for outputs of at most 16 columns) per
// 256-thread workgroup on v_mfma_f64_16x16x4f64, K-tiles of 16 double
// buffered in LDS.  Both operands are staged k-major ([k][row], row stride
// R + 1 doubles: the odd stride keeps the transposing stores of a
// k-contiguous operand and the MFMA reads free of bank conflicts).  The MFMA
// takes B's columns as its first operand, so lane l holds output rows
// m = 16 i + l mod 16 and stores coalesce along the column-major output.
constexpr int kKT64 = 16;

template <int R>
struct Tile64 {
  double v[R * kKT64 / 256];
};

// elements (r, k) of an R x 16 operand tile, zero outside the matrix or past
// kend; CONT_ROW: the operand is contiguous along r
template <int R, bool CONT_ROW>
__device__ __forceinline__ void tile64_fetch(const double* __restrict__ P, int64_t ld, int r0, int rmax, int k0,
                                             int kend, Tile64<R>& t) {
#pragma unroll
  for (int h = 0; h < R * kKT64 / 256; ++h) {
    const int idx = threadIdx.x + 256 * h;
    const int r = CONT_ROW ? idx % R : idx / kKT64, k = CONT_ROW ? idx / R : idx % kKT64;
    const int gr = r0 + r, gk = k0 + k;
    const bool ok = gr < rmax && gk < kend;
    const int cr = ok ? gr : 0, ck = ok ? gk : 0;
    const double x = CONT_ROW ? P[cr + (int64_t)ck * ld] : P[ck + (int64_t)cr * ld];
    t.v[h] = ok ? x : 0.0;
  }
}

template <int R, bool CONT_ROW>
__device__ __forceinline__ void tile64_store(const Tile64<R>& t, double* S) {
#pragma unroll
  for (int h = 0; h < R * kKT64 / 256; ++h) {
    const int idx = threadIdx.x + 256 * h;
    const int r = CONT_ROW ? idx % R : idx / kKT64, k = CONT_ROW ? idx / R : idx % kKT64;
    S[k * (R + 1) + r] = t.v[h];
  }
}

template <bool TA, bool TB, int TN>
__global__ __launch_bounds__(256) void gemm_f64_kernel(Gemm g, int kchunk, bool grouped) {
  constexpr int TM = 64, KT = kKT64;
  constexpr int WN = TN >= 32 ? 2 : 1, WM = 4 / WN;  // wave grid
  constexpr int SM = TM / 16 / WM, SN = TN / 16 / WN;  // 16 x 16 blocks per wave
  static_assert(SM >= 1 && SN >= 1, "tile shape");
  __shared__ double As[2][KT * (TM + 1)];
  __shared__ double Bs[2][KT * (TN + 1)];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  const int wm = wave % WM, wn = wave / WM;
  const TileIdx ti = tile_idx(grouped, (g.M + TM - 1) / TM, (g.N + TN - 1) / TN);
  if (ti.z >= g.batch * max(1, g.ksplit)) return;  // the grouped grid's last slots
  const int zb = ti.z % g.batch, zs = ti.z / g.batch;
  const int m0 = ti.x * TM, n0 = ti.y * TN;
  const int kbeg = zs * kchunk, kend = min(g.K, kbeg + kchunk);
  const double* A = static_cast<const double*>(g.A) + (int64_t)zb * g.sA;
  const double* B = static_cast<const double*>(g.B) + (int64_t)zb * g.sB;
  double* C = static_cast<double*>(g.C) + (int64_t)zb * g.sC + (int64_t)zs * g.sSplit;
  f64x4 acc[SM][SN];
#pragma unroll
  for (int i = 0; i < SM; ++i)
#pragma unroll
    for (int j = 0; j < SN; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  // A(m, k) is contiguous in m unless transposed; B(k, n) is contiguous in k
  // unless transposed
  Tile64<TM> ra;
  Tile64<TN> rb;
  int k0 = kbeg;
  if (k0 < kend) {
    tile64_fetch<TM, !TA>(A, g.lda, m0, g.M, k0, kend, ra);
    tile64_fetch<TN, TB>(B, g.ldb, n0, g.N, k0, kend, rb);
    tile64_store<TM, !TA>(ra, As[0]);
    tile64_store<TN, TB>(rb, Bs[0]);
  }
  __syncthreads();
  int buf = 0;
  for (; k0 < kend; k0 += KT) {
    const bool more = k0 + KT < kend;
    if (more) {
      tile64_fetch<TM, !TA>(A, g.lda, m0, g.M, k0 + KT, kend, ra);
      tile64_fetch<TN, TB>(B, g.ldb, n0, g.N, k0 + KT, kend, rb);
    }
#pragma unroll
    for (int s4 = 0; s4 < KT; s4 += 4) {
      double a[SM], b[SN];
#pragma unroll
      for (int i = 0; i < SM; ++i) a[i] = As[buf][(s4 + kq) * (TM + 1) + (wm * SM + i) * 16 + l16];
#pragma unroll
      for (int j = 0; j < SN; ++j) b[j] = Bs[buf][(s4 + kq) * (TN + 1) + (wn * SN + j) * 16 + l16];
#pragma unroll
      for (int i = 0; i < SM; ++i)
#pragma unroll
        for (int j = 0; j < SN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(b[j], a[i], acc[i][j], 0, 0, 0);
    }
    if (more) {
      tile64_store<TM, !TA>(ra, As[buf ^ 1]);
      tile64_store<TN, TB>(rb, Bs[buf ^ 1]);
    }
    __syncthreads();
    buf ^= 1;
  }
  // lane l, value v of block (i, j): row m = 16 (wm SM + i) + l mod 16,
  // column n = 16 (wn SN + j) + l / 16 + 4 v
#pragma unroll
  for (int i = 0; i < SM; ++i) {
    const int gm = m0 + (wm * SM + i) * 16 + l16;
    if (gm >= g.M) continue;
#pragma unroll
    for (int j = 0; j < SN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gn = n0 + (wn * SN + j) * 16 + kq + 4 * v;
        if (gn < g.N) C[gm + (int64_t)gn * g.ldc] = acc[i][j][v];
      }
  }
}

// out[e] = sum over z of parts[z * stride + e]; 64 consecutive outputs per
// workgroup of 16 waves.  Wave w sums the slices z = w (mod 16) of its lane's
// output in four independent chains (z = w + 16 c (mod 64), c = 0..3), and
// the 16 wave sums are added in wave order: a fixed order for every call.
// Sums run in TO (float64 for float32 slices summed into float64).
constexpr int kSumWaves = 16;

template <typename TI, typename TO>
__global__ __launch_bounds__(64 * kSumWaves) void sum_partials_kernel(const TI* __restrict__ parts, int nparts,
                                                                      int64_t stride, int64_t count,
                                                                      TO* __restrict__ out) {
  __shared__ TO red[kSumWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * 64 + lane;
  TO acc[4] = {TO(0), TO(0), TO(0), TO(0)};
  if (e < count) {
    int z = w;
    for (; z + 3 * kSumWaves < nparts; z += 4 * kSumWaves) {
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] += (TO)parts[(int64_t)(z + c * kSumWaves) * stride + e];
    }
    // at most three slices remain (z + 48 >= nparts)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      if (z + c * kSumWaves < nparts) acc[c] += (TO)parts[(int64_t)(z + c * kSumWaves) * stride + e];
  }
  red[w][lane] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  if (w == 0 && e < count) {
    TO t = red[0][lane];
    for (int i = 1; i < kSumWaves; ++i) t += red[i][lane];
    out[e] = t;
  }
}

// ---- 128 x 128 output tiles ---------------------------------------------------
// For products big enough to be bound by the matrix cores (the facewise
// products of Def. 2.3 on faces of a few hundred rows and columns).  Four
// waves per workgroup, wave w owning the 64 x 64 quadrant (w mod 2, w / 2) as
// 2 x 2 blocks of 32 x 32: per MFMA step a lane reads one value of each of
// its two A blocks and two B blocks and feeds four independent accumulation
// chains, so that every LDS read serves two MFMAs and the matrix core never
// waits on one chain.  K-tiles of KT are double buffered in LDS (the next
// tile's global loads in flight during the current tile's MFMAs) in the same
// layouts as the 64 x 64 kernels (tile_floats); step j of a K-tile takes k =
// j in lanes 0-31 and k = KT/2 + j in lanes 32-63.
constexpr int kBig = 128;

// The MFMA operands of one 32-row block of a staged K-tile (rows rb .. rb +
// 31 of the tile; lane rl = lane mod 32 takes row rb + rl, lane half h the k
// half): v[j] = element (rb + rl, h KT/2 + j).
template <int R, int KT, bool CONT_ROW>
__device__ __forceinline__ void block_operands(const float* S, int rb, int rl, int h, float (&v)[KT / 2]) {
  constexpr int H = KT / 2;
  if constexpr (CONT_ROW) {  // [k][row], row stride R + 4
#pragma unroll
    for (int j = 0; j < H; ++j) v[j] = S[(h * H + j) * (R + 4) + rb + rl];
  } else {                   // [row][k], row stride KT + 4: four k per 16-byte read
#pragma unroll
    for (int j = 0; j < H; j += 4) {
      const float4 x = *reinterpret_cast<const float4*>(S + (rb + rl) * (KT + 4) + h * H + j);
      v[j] = x.x; v[j + 1] = x.y; v[j + 2] = x.z; v[j + 3] = x.w;
    }
  }
}

// One 128 x 128 output tile: C(m0.., n0..) = A(m0.., kbeg:kend) B(kbeg:kend,
// n0..), A, B, C already offset to the batch entry.  bsm: the dynamic LDS
// (4 tile_floats<128, KT>() floats).
template <bool TA, bool TB, int VA, int VB, int KT>
__device__ __forceinline__ void big_tile_f32(const float* __restrict__ A, int64_t lda, const float* __restrict__ B,
                                             int64_t ldb, float* __restrict__ C, int64_t ldc, int M, int N, int m0,
                                             int n0, int kbeg, int kend, float* bsm) {
  constexpr int H = KT / 2;
  constexpr int FA = tile_floats<kBig, KT>(), FB = FA;
  auto As = [&](int b) { return bsm + b * FA; };
  auto Bs = [&](int b) { return bsm + 2 * FA + b * FB; };
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rl = lane & 31, h = lane >> 5;
  const int wm = wave & 1, wn = wave >> 1;
  f32x16 acc[2][2];  // [B block][A block]
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;
  TileRegs<kBig, KT> ra, rb;
  int k0 = kbeg;
  if (k0 < kend) {
    tile_fetch<kBig, KT, VA, !TA>(A, lda, m0, M, k0, kend, ra);
    tile_fetch<kBig, KT, VB, TB>(B, ldb, n0, N, k0, kend, rb);
    tile_store<kBig, KT, VA, !TA>(ra, As(0));
    tile_store<kBig, KT, VB, TB>(rb, Bs(0));
  }
  __syncthreads();
  int buf = 0;
  for (; k0 < kend; k0 += KT) {
    const bool more = k0 + KT < kend;
    if (more) {
      tile_fetch<kBig, KT, VA, !TA>(A, lda, m0, M, k0 + KT, kend, ra);
      tile_fetch<kBig, KT, VB, TB>(B, ldb, n0, N, k0 + KT, kend, rb);
    }
    float a[2][H], b[2][H];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      block_operands<kBig, KT, !TA>(As(buf), wm * 64 + 32 * i, rl, h, a[i]);
      block_operands<kBig, KT, TB>(Bs(buf), wn * 64 + 32 * i, rl, h, b[i]);
    }
#pragma unroll
    for (int j = 0; j < H; ++j)
#pragma unroll
      for (int bn = 0; bn < 2; ++bn)
#pragma unroll
        for (int bm = 0; bm < 2; ++bm)
          acc[bn][bm] = __builtin_amdgcn_mfma_f32_32x32x2f32(b[bn][j], a[bm][j], acc[bn][bm], 0, 0, 0);
    if (more) {
      tile_store<kBig, KT, VA, !TA>(ra, As(buf ^ 1));
      tile_store<kBig, KT, VB, TB>(rb, Bs(buf ^ 1));
    }
    __syncthreads();
    buf ^= 1;
  }
  // lane (rl, h), value e of block (bn, bm): row m = m0 + 64 wm + 32 bm + rl,
  // column n = n0 + 64 wn + 32 bn + 8 (e / 4) + 4 h + e mod 4
#pragma unroll
  for (int bm = 0; bm < 2; ++bm) {
    const int gm = m0 + wm * 64 + 32 * bm + rl;
    if (gm >= M) continue;
#pragma unroll
    for (int bn = 0; bn < 2; ++bn)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int gn = n0 + wn * 64 + 32 * bn + 8 * (e >> 2) + 4 * h + (e & 3);
        if (gn < N) C[gm + (int64_t)gn * ldc] = acc[bn][bm][e];
      }
  }
}

template <bool TA, bool TB, int VA, int VB, int KT>
__global__ __launch_bounds__(256, 2) void gemm_f32_big_kernel(Gemm g, int kchunk, bool grouped) {
  extern __shared__ __align__(16) float bsm[];
  const TileIdx ti = tile_idx(grouped, (g.M + kBig - 1) / kBig, (g.N + kBig - 1) / kBig);
  if (ti.z >= g.batch * max(1, g.ksplit)) return;  // the grouped grid's last slots
  const int zb = ti.z % g.batch, zs = ti.z / g.batch;
  const int kbeg = zs * kchunk, kend = min(g.K, kbeg + kchunk);
  big_tile_f32<TA, TB, VA, VB, KT>(static_cast<const float*>(g.A) + (int64_t)zb * g.sA, g.lda,
                                   static_cast<const float*>(g.B) + (int64_t)zb * g.sB, g.ldb,
                                   static_cast<float*>(g.C) + (int64_t)zb * g.sC + (int64_t)zs * g.sSplit, g.ldc, g.M,
                                   g.N, ti.x * kBig, ti.y * kBig, kbeg, kend, bsm);
}

// Many independent facewise products (of different shapes) in one launch:
// workgroup w computes tile tiles[w] (a 128 x 128 output tile of one face of
// one product, the tiles ordered by the host, deepest K first).  Products
// whose operands allow 16-byte loads take them, the others scalar loads.
template <int KT>
__global__ __launch_bounds__(256, 2) void gemm_f32_grouped_kernel(const GemmDesc* __restrict__ descs,
                                                                 const GemmTile* __restrict__ tiles) {
  extern __shared__ __align__(16) float bsm[];
  const GemmTile t = tiles[blockIdx.x];
  const GemmDesc d = descs[t.desc];
  const float* A = d.A + (int64_t)t.z * d.sA;
  const float* B = d.B + (int64_t)t.z * d.sB;
  float* C = d.C + (int64_t)t.z * d.sC;
  if (d.vec4)
    big_tile_f32<false, false, 4, 4, KT>(A, d.lda, B, d.ldb, C, d.ldc, d.M, d.N, t.tx * kBig, t.ty * kBig, 0, d.K,
                                         bsm);
  else
    big_tile_f32<false, false, 1, 1, KT>(A, d.lda, B, d.ldb, C, d.ldc, d.M, d.N, t.tx * kBig, t.ty * kBig, 0, d.K,
                                         bsm);
}

// The split-bfloat16 form of the 128 x 128 kernel: the tiles are fetched as
// float32 and split into NP bfloat16 parts on their way into LDS ([row][k],
// row stride KT + 8 bfloat16, k contiguous), and a lane reads the 8
// consecutive k of its row as one 16-byte operand of
// v_mfma_f32_32x32x16_bf16 (k = 8 h + i of each 16-wide step).  The part
// products of Split<NP, NP> are accumulated in float32, smallest first.
template <int R, int KT, int VEC, bool CONT_ROW, int NP>
__device__ __forceinline__ void tile_store_split_r(const TileRegs<R, KT>& t, uint16_t* S) {
  constexpr int ld = KT + kPad16;
  constexpr int part = R * ld;
  const int tid = threadIdx.x;
  auto put = [&](int r, int k, float x) {
    uint32_t w[NP];
    split_pack<NP>(x, 0.f, w);
#pragma unroll
    for (int i = 0; i < NP; ++i) S[i * part + r * ld + k] = (uint16_t)(w[i] & 0xffffu);
  };
  if constexpr (VEC == 4) {
#pragma unroll
    for (int hh = 0; hh < R * KT / 1024; ++hh) {
      const int idx = tid + 256 * hh;
      if (CONT_ROW) {  // four consecutive rows of one k
        const int k = idx / (R / 4), r = 4 * (idx % (R / 4));
#pragma unroll
        for (int i = 0; i < 4; ++i) put(r + i, k, t.v[4 * hh + i]);
      } else {         // four consecutive k of one row: two packed words per part
        const int r = idx / (KT / 4), k = 4 * (idx % (KT / 4));
        uint32_t w0[NP], w1[NP];
        split_pack<NP>(t.v[4 * hh + 0], t.v[4 * hh + 1], w0);
        split_pack<NP>(t.v[4 * hh + 2], t.v[4 * hh + 3], w1);
#pragma unroll
        for (int i = 0; i < NP; ++i)
          *reinterpret_cast<uint2*>(S + i * part + r * ld + k) = make_uint2(w0[i], w1[i]);
      }
    }
  } else {
#pragma unroll
    for (int hh = 0; hh < R * KT / 256; ++hh) {
      const int idx = tid + 256 * hh;
      int r, k;
      if (CONT_ROW) { k = idx / R; r = idx % R; } else { r = idx / KT; k = idx % KT; }
      put(r, k, t.v[hh]);
    }
  }
}

// An operand contiguous along its rows (VEC = 4, CONT_ROW) is fetched for
// the split kernel as 4 x 4 blocks instead: thread t takes rows 4 (t mod
// (R / 4)) .. + 3 at the four consecutive k = 4 (t / (R / 4)) .. + 3 of a
// 16-k slab (R = 128: 32 row quads x 8 k quads = 256 threads per 32 k), so
// that after the split the four k of each row leave as one packed 8-byte LDS
// store per part.  The float4 loads of a wave still cover 512 contiguous
// bytes of one k.
template <int R, int KT>
__device__ __forceinline__ void tile_fetch_quads(const float* __restrict__ P, int64_t ld, int r0, int rmax, int k0,
                                                 int kend, TileRegs<R, KT>& t) {
  constexpr int RQ = R / 4, KQ = 256 / RQ;  // row quads, k quads per pass
  static_assert(RQ * KQ == 256 && KT % (4 * KQ) == 0, "quad tiling");
  const int rq = threadIdx.x % RQ, kq = threadIdx.x / RQ;
#pragma unroll
  for (int pass = 0; pass < KT / (4 * KQ); ++pass) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gr = r0 + 4 * rq, gk = k0 + 4 * (kq + KQ * pass) + j;
      const bool ok = gr < rmax && gk < kend;
      const float4 x = *reinterpret_cast<const float4*>(P + (ok ? gr : 0) + (int64_t)(ok ? gk : 0) * ld);
      float* v = t.v + 16 * pass + 4 * j;
      v[0] = ok ? x.x : 0.f;
      v[1] = ok ? x.y : 0.f;
      v[2] = ok ? x.z : 0.f;
      v[3] = ok ? x.w : 0.f;
    }
  }
}

// t.v[16 pass + 4 j + i] = element (row 4 rq + i, k = 4 (kq + KQ pass) + j)
template <int R, int KT, int NP>
__device__ __forceinline__ void tile_store_split_quads(const TileRegs<R, KT>& t, uint16_t* S) {
  constexpr int RQ = R / 4, KQ = 256 / RQ;
  constexpr int ld = KT + kPad16;
  constexpr int part = R * ld;
  const int rq = threadIdx.x % RQ, kq = threadIdx.x / RQ;
#pragma unroll
  for (int pass = 0; pass < KT / (4 * KQ); ++pass) {
    const float* v = t.v + 16 * pass;
    const int k = 4 * (kq + KQ * pass);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      uint32_t w0[NP], w1[NP];
      split_pack<NP>(v[i], v[4 + i], w0);
      split_pack<NP>(v[8 + i], v[12 + i], w1);
#pragma unroll
      for (int q = 0; q < NP; ++q)
        *reinterpret_cast<uint2*>(S + q * part + (4 * rq + i) * ld + k) = make_uint2(w0[q], w1[q]);
    }
  }
}

// operand fetch and split store of the split kernel: 4 x 4 blocks for an
// operand contiguous along its rows with 16-byte loads (when the K-tile
// holds whole passes of them), the 64 x 64 kernel's mapping otherwise
template <int R, int KT>
__host__ __device__ constexpr bool quads_fit() {
  return KT % (4 * (256 / (R / 4))) == 0;
}
template <int R, int KT, int VEC, bool CONT_ROW>
__device__ __forceinline__ void split_fetch(const float* __restrict__ P, int64_t ld, int r0, int rmax, int k0,
                                            int kend, TileRegs<R, KT>& t) {
  if constexpr (VEC == 4 && CONT_ROW && quads_fit<R, KT>()) tile_fetch_quads<R, KT>(P, ld, r0, rmax, k0, kend, t);
  else tile_fetch<R, KT, VEC, CONT_ROW>(P, ld, r0, rmax, k0, kend, t);
}
template <int R, int KT, int VEC, bool CONT_ROW, int NP>
__device__ __forceinline__ void split_store(const TileRegs<R, KT>& t, uint16_t* S) {
  if constexpr (VEC == 4 && CONT_ROW && quads_fit<R, KT>()) tile_store_split_quads<R, KT, NP>(t, S);
  else tile_store_split_r<R, KT, VEC, CONT_ROW, NP>(t, S);
}

template <bool TA, bool TB, int VA, int VB, int KT, int NP>
__global__ __launch_bounds__(256, 2) void gemm_bf16_big_kernel(Gemm g, int kchunk, bool grouped) {
  using SP = Split<NP, NP>;
  constexpr int ld = KT + kPad16;
  constexpr int part = kBig * ld;  // bfloat16 elements per part
  extern __shared__ __align__(16) uint16_t hbsm[];
  auto Ap = [&](int b) { return hbsm + b * NP * part; };
  auto Bp = [&](int b) { return hbsm + (2 + b) * NP * part; };
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rl = lane & 31, h = lane >> 5;
  const int wm = wave & 1, wn = wave >> 1;
  const TileIdx ti = tile_idx(grouped, (g.M + kBig - 1) / kBig, (g.N + kBig - 1) / kBig);
  if (ti.z >= g.batch * max(1, g.ksplit)) return;
  const int zb = ti.z % g.batch, zs = ti.z / g.batch;
  const int m0 = ti.x * kBig, n0 = ti.y * kBig;
  const int kbeg = zs * kchunk, kend = min(g.K, kbeg + kchunk);
  const float* A = static_cast<const float*>(g.A) + (int64_t)zb * g.sA;
  const float* B = static_cast<const float*>(g.B) + (int64_t)zb * g.sB;
  float* C = static_cast<float*>(g.C) + (int64_t)zb * g.sC + (int64_t)zs * g.sSplit;
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;
  TileRegs<kBig, KT> ra, rb;
  int k0 = kbeg;
  if (k0 < kend) {
    split_fetch<kBig, KT, VA, !TA>(A, g.lda, m0, g.M, k0, kend, ra);
    split_fetch<kBig, KT, VB, TB>(B, g.ldb, n0, g.N, k0, kend, rb);
    split_store<kBig, KT, VA, !TA, NP>(ra, Ap(0));
    split_store<kBig, KT, VB, TB, NP>(rb, Bp(0));
  }
  __syncthreads();
  int buf = 0;
  for (; k0 < kend; k0 += KT) {
    const bool more = k0 + KT < kend;
    if (more) {
      split_fetch<kBig, KT, VA, !TA>(A, g.lda, m0, g.M, k0 + KT, kend, ra);
      split_fetch<kBig, KT, VB, TB>(B, g.ldb, n0, g.N, k0 + KT, kend, rb);
    }
#pragma unroll
    for (int ks = 0; ks < KT; ks += 16) {
      bf16x8 pa[2][NP], pb[2][NP];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          pa[i][q] = *reinterpret_cast<const bf16x8*>(Ap(buf) + q * part + (wm * 64 + 32 * i + rl) * ld + ks + 8 * h);
          pb[i][q] = *reinterpret_cast<const bf16x8*>(Bp(buf) + q * part + (wn * 64 + 32 * i + rl) * ld + ks + 8 * h);
        }
#pragma unroll
      for (int pr = 0; pr < SP::n; ++pr)
#pragma unroll
        for (int bn = 0; bn < 2; ++bn)
#pragma unroll
          for (int bm = 0; bm < 2; ++bm)
            acc[bn][bm] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pb[bn][SP::q[pr]], pa[bm][SP::a[pr]], acc[bn][bm],
                                                                  0, 0, 0);
    }
    if (more) {
      split_store<kBig, KT, VA, !TA, NP>(ra, Ap(buf ^ 1));
      split_store<kBig, KT, VB, TB, NP>(rb, Bp(buf ^ 1));
    }
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int bm = 0; bm < 2; ++bm) {
    const int gm = m0 + wm * 64 + 32 * bm + rl;
    if (gm >= g.M) continue;
#pragma unroll
    for (int bn = 0; bn < 2; ++bn)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int gn = n0 + wn * 64 + 32 * bn + 8 * (e >> 2) + 4 * h + (e & 3);
        if (gn < g.N) C[gm + (int64_t)gn * g.ldc] = acc[bn][bm][e];
      }
  }
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

template <bool TA, bool TB, int VA, int VB, int KT, int TM>
hipError_t gemm_f32_go(const Gemm& g, int kchunk, hipStream_t s) {
  constexpr int TN = 4096 / TM;
  const size_t lds = sizeof(float) * 2 * (tile_floats<TM, KT>() + tile_floats<TN, KT>());
  static hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_f32_kernel<TA, TB, VA, VB, KT, TM>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return attr;
  const unsigned mt = (unsigned)((g.M + TM - 1) / TM), nt = (unsigned)((g.N + TN - 1) / TN);
  const unsigned nz = (unsigned)(g.batch * std::max(1, g.ksplit));
  // grouped when the slabs fill the XCDs evenly (a multiple of 8, or enough
  // that the last, partial pass over the XCDs costs little)
  const bool grouped = nz % kXcds == 0 || nz >= 8 * kXcds;
  const dim3 grid = grouped ? dim3(kXcds * mt * nt * ((nz + kXcds - 1) / kXcds)) : dim3(mt, nt, nz);
  gemm_f32_kernel<TA, TB, VA, VB, KT, TM><<<grid, 256, lds, s>>>(g, kchunk, grouped);
  return hipGetLastError();
}

template <bool TA, bool TB, int KT, int TM>
hipError_t gemm_f32_launch(const Gemm& g, int kchunk, hipStream_t s) {
  // contiguous dimension: A's is M (K when transposed), B's is K (N when transposed)
  const bool va = vec4_ok(g.A, TA ? g.K : g.M, g.lda, g.sA) && (!TA || kchunk % 4 == 0);
  const bool vb = vec4_ok(g.B, TB ? g.N : g.K, g.ldb, g.sB) && (TB || kchunk % 4 == 0);
  if (va && vb) return gemm_f32_go<TA, TB, 4, 4, KT, TM>(g, kchunk, s);
  if (va) return gemm_f32_go<TA, TB, 4, 1, KT, TM>(g, kchunk, s);
  if (vb) return gemm_f32_go<TA, TB, 1, 4, KT, TM>(g, kchunk, s);
  return gemm_f32_go<TA, TB, 1, 1, KT, TM>(g, kchunk, s);
}

template <bool TA, bool TB, int VA, int VB, int KT, int NP>
hipError_t gemm_bf16_go(const Gemm& g, int kchunk, hipStream_t s) {
  const size_t lds = sizeof(uint16_t) * 4 * NP * 64 * (KT + kPad16);
  static hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_bf16_kernel<TA, TB, VA, VB, KT, NP>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return attr;
  const dim3 grid((unsigned)((g.M + 63) / 64), (unsigned)((g.N + 63) / 64),
                  (unsigned)(g.batch * std::max(1, g.ksplit)));
  gemm_bf16_kernel<TA, TB, VA, VB, KT, NP><<<grid, 256, lds, s>>>(g, kchunk);
  return hipGetLastError();
}

template <bool TA, bool TB, int KT, int NP>
hipError_t gemm_bf16_launch(const Gemm& g, int kchunk, hipStream_t s) {
  const bool va = vec4_ok(g.A, TA ? g.K : g.M, g.lda, g.sA) && (!TA || kchunk % 4 == 0);
  const bool vb = vec4_ok(g.B, TB ? g.N : g.K, g.ldb, g.sB) && (TB || kchunk % 4 == 0);
  if (va && vb) return gemm_bf16_go<TA, TB, 4, 4, KT, NP>(g, kchunk, s);
  if (va) return gemm_bf16_go<TA, TB, 4, 1, KT, NP>(g, kchunk, s);
  if (vb) return gemm_bf16_go<TA, TB, 1, 4, KT, NP>(g, kchunk, s);
  return gemm_bf16_go<TA, TB, 1, 1, KT, NP>(g, kchunk, s);
}

// grid of the 128 x 128 kernels: grouped by slab on the XCDs under the same
// condition as the 64 x 64 float32 kernel
inline dim3 big_grid(const Gemm& g, bool& grouped) {
  const unsigned mt = (unsigned)((g.M + kBig - 1) / kBig), nt = (unsigned)((g.N + kBig - 1) / kBig);
  const unsigned nz = (unsigned)(g.batch * std::max(1, g.ksplit));
  grouped = nz % kXcds == 0 || nz >= 8 * kXcds;
  return grouped ? dim3(kXcds * mt * nt * ((nz + kXcds - 1) / kXcds)) : dim3(mt, nt, nz);
}

template <bool TA, bool TB, int VA, int VB, int KT>
hipError_t gemm_f32_big_go(const Gemm& g, int kchunk, hipStream_t s) {
  const size_t lds = sizeof(float) * 4 * tile_floats<kBig, KT>();
  static hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_f32_big_kernel<TA, TB, VA, VB, KT>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return attr;
  bool grouped = false;
  const dim3 grid = big_grid(g, grouped);
  gemm_f32_big_kernel<TA, TB, VA, VB, KT><<<grid, 256, lds, s>>>(g, kchunk, grouped);
  return hipGetLastError();
}

template <bool TA, bool TB, int VA, int VB, int KT, int NP>
hipError_t gemm_bf16_big_go(const Gemm& g, int kchunk, hipStream_t s) {
  const size_t lds = sizeof(uint16_t) * 4 * NP * kBig * (KT + kPad16);
  static hipError_t attr = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&gemm_bf16_big_kernel<TA, TB, VA, VB, KT, NP>),
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return attr;
  bool grouped = false;
  const dim3 grid = big_grid(g, grouped);
  gemm_bf16_big_kernel<TA, TB, VA, VB, KT, NP><<<grid, 256, lds, s>>>(g, kchunk, grouped);
  return hipGetLastError();
}

// NP = 0: float32 MFMA; otherwise NP bfloat16 parts
template <bool TA, bool TB, int KT, int NP>
hipError_t gemm_big_launch(const Gemm& g, int kchunk, hipStream_t s) {
  const bool va = vec4_ok(g.A, TA ? g.K : g.M, g.lda, g.sA) && (!TA || kchunk % 4 == 0);
  const bool vb = vec4_ok(g.B, TB ? g.N : g.K, g.ldb, g.sB) && (TB || kchunk % 4 == 0);
  if constexpr (NP == 0) {
    if (va && vb) return gemm_f32_big_go<TA, TB, 4, 4, KT>(g, kchunk, s);
    if (va) return gemm_f32_big_go<TA, TB, 4, 1, KT>(g, kchunk, s);
    if (vb) return gemm_f32_big_go<TA, TB, 1, 4, KT>(g, kchunk, s);
    return gemm_f32_big_go<TA, TB, 1, 1, KT>(g, kchunk, s);
  } else {
    if (va && vb) return gemm_bf16_big_go<TA, TB, 4, 4, KT, NP>(g, kchunk, s);
    if (va) return gemm_bf16_big_go<TA, TB, 4, 1, KT, NP>(g, kchunk, s);
    if (vb) return gemm_bf16_big_go<TA, TB, 1, 4, KT, NP>(g, kchunk, s);
    return gemm_bf16_big_go<TA, TB, 1, 1, KT, NP>(g, kchunk, s);
  }
}

// The 128 x 128 kernels take products without a K split whose output holds
// at least one whole 128 x 128 tile
inline bool big_tiles(const Gemm& g) { return g.ksplit <= 1 && g.M >= kBig && g.N >= kBig; }

template <bool TA, bool TB>
hipError_t gemm_small_launch(const Gemm& g, Prec prec, int kchunk, hipStream_t s);

template <bool TA, bool TB>
hipError_t gemm_launch(const Gemm& g, Prec prec, int kchunk, hipStream_t s) {
  if (big_tiles(g)) {
    // autotuned: 128 x 128 tiles with K-tiles of 32 (the default) or 16
    // (less LDS, more workgroups per CU), or the 64 x 64 kernel; the
    // compensated modes also time the same three in float32, which are at
    // least as accurate (and faster where few tiles leave the product bound
    // by latency rather than by matrix-core rate)
    char key[160];
    std::snprintf(key, sizeof key, "gemm:%d:%d%d:%dx%dx%dx%d", (int)prec, (int)TA, (int)TB, g.M, g.N, g.K, g.batch);
    const bool comp = prec == Prec::BF16x3 || prec == Prec::BF16x6;
    return tuned_launch(key, comp ? 6 : 3, 0, s, [&](int c) -> hipError_t {
      const Prec pc = c >= 3 ? Prec::Default : prec;
      c %= 3;
      if (c == 2) return gemm_small_launch<TA, TB>(g, pc, kchunk, s);
      switch (pc) {
        case Prec::BF16:
          return c ? gemm_big_launch<TA, TB, 16, 1>(g, kchunk, s) : gemm_big_launch<TA, TB, 32, 1>(g, kchunk, s);
        case Prec::BF16x3:
          return c ? gemm_big_launch<TA, TB, 16, 2>(g, kchunk, s) : gemm_big_launch<TA, TB, 32, 2>(g, kchunk, s);
        case Prec::BF16x6:
          return c ? gemm_big_launch<TA, TB, 16, 3>(g, kchunk, s) : gemm_big_launch<TA, TB, 32, 3>(g, kchunk, s);
        default:
          return c ? gemm_big_launch<TA, TB, 16, 0>(g, kchunk, s) : gemm_big_launch<TA, TB, 32, 0>(g, kchunk, s);
      }
    });
  }
  return gemm_small_launch<TA, TB>(g, prec, kchunk, s);
}

// the 64 x 64 (or 32 x 128) kernels
template <bool TA, bool TB>
hipError_t gemm_small_launch(const Gemm& g, Prec prec, int kchunk, hipStream_t s) {
  const bool deep = kchunk >= 96;
  switch (prec) {
    case Prec::BF16:
      return deep ? gemm_bf16_launch<TA, TB, 128, 1>(g, kchunk, s) : gemm_bf16_launch<TA, TB, 32, 1>(g, kchunk, s);
    case Prec::BF16x3:
      return deep ? gemm_bf16_launch<TA, TB, 128, 2>(g, kchunk, s) : gemm_bf16_launch<TA, TB, 32, 2>(g, kchunk, s);
    case Prec::BF16x6:
      return deep ? gemm_bf16_launch<TA, TB, 64, 3>(g, kchunk, s) : gemm_bf16_launch<TA, TB, 32, 3>(g, kchunk, s);
    default: {
      // outputs of at most 32 rows and more than 64 columns (the dQ
      // products) take the 32 x 128 tile, whose deep K-tile is 64 (LDS)
      const bool narrow = g.M <= 32 && g.N > 64;
      const int tm = narrow ? 32 : 64, tn = 4096 / tm;
      const int64_t wgs = (int64_t)((g.M + tm - 1) / tm) * ((g.N + tn - 1) / tn) * g.batch * std::max(1, g.ksplit);
      // a deep K-tile's LDS leaves one workgroup per CU: a split-K grid with
      // more workgroups than CUs takes the shallow one (several per CU)
      const bool d = deep && (g.ksplit <= 1 || wgs <= kCUs);
      if (narrow)
        return d ? gemm_f32_launch<TA, TB, 64, 32>(g, kchunk, s) : gemm_f32_launch<TA, TB, 32, 32>(g, kchunk, s);
      return d ? gemm_f32_launch<TA, TB, 128, 64>(g, kchunk, s) : gemm_f32_launch<TA, TB, 32, 64>(g, kchunk, s);
    }
  }
}

hipError_t gemm_f32(const Gemm& g, Prec prec, hipStream_t s) {
  // deep K-tiles (one global round trip covers up to 128 of K) when a
  // workgroup has that much K
  const int kchunk = chunk_for(g, 32);
  if (!g.ta && !g.tb) return gemm_launch<false, false>(g, prec, kchunk, s);
  if (!g.ta && g.tb) return gemm_launch<false, true>(g, prec, kchunk, s);
  if (g.ta && !g.tb) return gemm_launch<true, false>(g, prec, kchunk, s);
  return gemm_launch<true, true>(g, prec, kchunk, s);
}

template <bool TA, bool TB>
hipError_t gemm_f64_go(const Gemm& g, int kchunk, hipStream_t s) {
  const unsigned gz = (unsigned)(g.batch * std::max(1, g.ksplit));
  const unsigned mt = (unsigned)((g.M + 63) / 64), nt = g.N <= 16 ? 1u : (unsigned)((g.N + 63) / 64);
  // grouped by slab on the XCDs under the same condition as the float32 kernel
  const bool grouped = gz % kXcds == 0 || gz >= 8 * kXcds;
  const dim3 grid = grouped ? dim3(kXcds * mt * nt * ((gz + kXcds - 1) / kXcds)) : dim3(mt, nt, gz);
  if (g.N <= 16) {
    gemm_f64_kernel<TA, TB, 16><<<grid, 256, 0, s>>>(g, kchunk, grouped);
  } else {
    gemm_f64_kernel<TA, TB, 64><<<grid, 256, 0, s>>>(g, kchunk, grouped);
  }
  return hipGetLastError();
}

hipError_t gemm_f32_grouped(const GemmDesc* descs, const GemmTile* tiles, int ntiles, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  constexpr int KT = 32;
  const size_t lds = sizeof(float) * 4 * tile_floats<kBig, KT>();
  static hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_f32_grouped_kernel<KT>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return attr;
  gemm_f32_grouped_kernel<KT><<<(unsigned)ntiles, 256, lds, s>>>(descs, tiles);
  return hipGetLastError();
}

bool gemm_vec4_ok(const GemmDesc& d) {
  return vec4_ok(d.A, d.M, d.lda, d.sA) && vec4_ok(d.B, d.K, d.ldb, d.sB);
}

hipError_t gemm_f64(const Gemm& g, hipStream_t s) {
  const int kchunk = chunk_for(g, kKT64);
  if (!g.ta && !g.tb) return gemm_f64_go<false, false>(g, kchunk, s);
  if (!g.ta && g.tb) return gemm_f64_go<false, true>(g, kchunk, s);
  if (g.ta && !g.tb) return gemm_f64_go<true, false>(g, kchunk, s);
  return gemm_f64_go<true, true>(g, kchunk, s);
}

hipError_t sum_partials_f32(const float* parts, int nparts, int64_t stride, int64_t count,
                            float* out, hipStream_t s) {
  sum_partials_kernel<float, float><<<(unsigned)((count + 63) / 64), 64 * kSumWaves, 0, s>>>(parts, nparts, stride,
                                                                                            count, out);
  return hipGetLastError();
}

hipError_t sum_partials_f64(const double* parts, int nparts, int64_t stride, int64_t count,
                            double* out, hipStream_t s) {
  sum_partials_kernel<double, double><<<(unsigned)((count + 63) / 64), 64 * kSumWaves, 0, s>>>(parts, nparts, stride,
                                                                                              count, out);
  return hipGetLastError();
}

hipError_t sum_to_f64(const float* parts, int nparts, int64_t stride, int64_t count, double* out, hipStream_t s) {
  sum_partials_kernel<float, double><<<(unsigned)((count + 63) / 64), 64 * kSumWaves, 0, s>>>(parts, nparts, stride,
                                                                                             count, out);
  return hipGetLastError();
}

}  // namespace pq
