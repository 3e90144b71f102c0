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
#include <string>
#include <vector>

#include "common.hpp"
#include "internal.hpp"

namespace pq {
namespace {


// ---- float32 matrix-core transform -------------------------------------------
// Persistent strips with split-K inside the workgroup: a workgroup stages the
// rows of Q it needs in LDS once and then walks over several strips of tubes
// (strip = blockIdx.x + i * gridDim.x).  Its S waves share the current strip
// and take its 16-row blocks of the frontal-slice index in turn (block b goes
// to wave b mod S), so S x 16 rows of the strip are in flight even when the
// tensor has few tubes; a wave issues the loads of its next block before the
// MFMAs of its current one.  The S partial accumulators are summed through
// LDS.  Q rows are staged in chunks of at most kKC rows, zero-filled past n3
// and past p; with n3 > kKC the chunks are restaged for every strip.
constexpr int kKC = 256;

// Q(kc + r, lc + c) for r < kcr, c < 32 into Qs[r * ldq + c] (zero past n3 and
// past p), `nthr` threads, 8 loads in flight per thread before the LDS writes.
__device__ __forceinline__ void stage_q_rows(const float* __restrict__ Q, int p, int n3, int kc, int kcr,
                                             int lc, float* Qs, int ldq, int nthr) {
  const int total = kcr * 32;
  for (int e0 = threadIdx.x; e0 < total; e0 += 8 * nthr) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = min(e0 + u * nthr, total - 1);
      const int t = kc + (e >> 5), c = lc + (e & 31);
      v[u] = Q[(int64_t)min(t, n3 - 1) * p + min(c, p - 1)];
      v[u] = (t < n3 && c < p) ? v[u] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * nthr;
      if (e < total) Qs[(e >> 5) * ldq + (e & 31)] = v[u];
    }
  }
}

// Loads are unconditional, from a clamped in-bounds address, and values that
// lie outside the tensor are zeroed afterwards by a select: with no branch
// around them the compiler can keep a whole block of loads in flight.  Ap
// must point at a valid tube of row 0 for inactive lanes too.
template <int VEC, typename TIn>
__device__ __forceinline__ void load_block16(const TIn* __restrict__ Ap, int64_t N, bool active,
                                             int t0, int tmax, int kh, float (&b)[8][VEC]) {
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const int t = t0 + 2 * s + kh;
    const bool ok = active && t < tmax;
    load_vec<VEC>(Ap + (int64_t)min(t, tmax - 1) * N, b[s]);
#pragma unroll
    for (int q = 0; q < VEC; ++q) b[s][q] = ok ? b[s][q] : 0.f;
  }
}

template <int VEC>
__device__ __forceinline__ void mfma_block16(const float* Qs, int ldq, int r, int n, int kh,
                                             const float (&b)[8][VEC], f32x16 (&acc)[VEC]) {
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const float a = Qs[(r + 2 * s + kh) * ldq + n];
#pragma unroll
    for (int q = 0; q < VEC; ++q)
      acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b[s][q], acc[q], 0, 0, 0);
  }
}

// acc += Q(rows, chunk)^T A(rows, strip) over this wave's 16-row blocks of
// `rows` rows; Ap points at the first row, Qs at the staged rows (zero-filled
// to a multiple of 16).
template <int VEC, int S, typename TIn>
__device__ __forceinline__ void hat_accumulate(const TIn* __restrict__ Ap, int64_t N, bool active,
                                               int rows, const float* Qs, int ldq, int wave, int n,
                                               int kh, f32x16 (&acc)[VEC]) {
  const int nblk = (rows + 15) / 16;
  float b0[8][VEC], b1[8][VEC];
  int blk = wave;
  if (blk < nblk) load_block16<VEC, TIn>(Ap, N, active, 16 * blk, rows, kh, b0);
  for (; blk < nblk; blk += 2 * S) {
    if (blk + S < nblk) load_block16<VEC, TIn>(Ap, N, active, 16 * (blk + S), rows, kh, b1);
    mfma_block16<VEC>(Qs, ldq, 16 * blk, n, kh, b0, acc);
    if (blk + S >= nblk) break;
    if (blk + 2 * S < nblk) load_block16<VEC, TIn>(Ap, N, active, 16 * (blk + 2 * S), rows, kh, b0);
    mfma_block16<VEC>(Qs, ldq, 16 * (blk + S), n, kh, b1, acc);
  }
}

// Sum the S waves' accumulators into wave 0 through LDS (red holds
// (S - 1) * VEC * 16 * 64 floats).  Every wave of the workgroup must call it.
// Returns true in the wave that holds the sum.
template <int VEC, int S>
__device__ __forceinline__ bool reduce_waves(f32x16 (&acc)[VEC], float* red, int wave, int lane) {
  if constexpr (S == 1) {
    return true;
  } else {
    if (wave > 0) {
#pragma unroll
      for (int q = 0; q < VEC; ++q)
#pragma unroll
        for (int j = 0; j < 16; ++j) red[(((wave - 1) * VEC + q) * 16 + j) * 64 + lane] = acc[q][j];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int w = 1; w < S; ++w)
#pragma unroll
        for (int q = 0; q < VEC; ++q)
#pragma unroll
          for (int j = 0; j < 16; ++j) acc[q][j] += red[(((w - 1) * VEC + q) * 16 + j) * 64 + lane];
    }
    __syncthreads();
    return wave == 0;
  }
}

template <int VEC, int S, typename TIn>
__global__ __launch_bounds__(S * 64) void hat_f32_kernel(const TIn* __restrict__ A,
                                                         const float* __restrict__ Q,
                                                         float* __restrict__ Ah, int64_t N, int n3,
                                                         int p, int kcr, int64_t nstrips) {
  extern __shared__ float smem[];
  float* Qs = smem;              // kcr x 32
  float* red = smem + kcr * 32;  // (S - 1) * VEC * 16 * 64
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = lane & 31, kh = lane >> 5;
  const int lc = blockIdx.y * 32;
  const bool one_chunk = n3 <= kcr;
  auto stage = [&](int kc) { stage_q_rows(Q, p, n3, kc, kcr, lc, Qs, 32, S * 64); };
  if (one_chunk) {
    stage(0);
    __syncthreads();
  }
  for (int64_t strip = blockIdx.x; strip < nstrips; strip += gridDim.x) {
    const int64_t xl = strip * (32 * VEC) + (int64_t)VEC * n;
    const bool active = xl < N;
    const int64_t xs = active ? xl : N - VEC;  // a valid tube for address arithmetic
    f32x16 acc[VEC];
#pragma unroll
    for (int q = 0; q < VEC; ++q)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[q][j] = 0.f;
    for (int kc = 0; kc < n3; kc += kcr) {
      if (!one_chunk) {
        __syncthreads();
        stage(kc);
        __syncthreads();
      }
      hat_accumulate<VEC, S, TIn>(A + (int64_t)kc * N + xs, N, active, min(kcr, n3 - kc), Qs, 32,
                                  wave, n, kh, acc);
    }
    if (reduce_waves<VEC, S>(acc, red, wave, lane) && active) {
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
  }
}

// ---- float32 transform, one strip per workgroup ------------------------------
// A workgroup of S waves owns one strip of 32*VEC tubes; its waves take the
// pairs of frontal slices (t, t + 1) in turn, U pairs per batch.  A batch is
// the U slices of A a lane needs (VEC tubes each) and the matching U entries
// of Q (read through the cache: Q is a few KB).  The loads of the next batch
// are issued before the MFMAs of the current one (two register buffers), so
// every wave keeps a batch in flight while its MFMAs run; loads past the last
// slice read a clamped, in-bounds address and are masked at use.  Nothing is
// staged and nothing waits at a barrier until the S partial accumulators are
// summed through LDS at the end.
template <int VEC, int U, typename TIn>
__device__ __forceinline__ void strip_load(const TIn* __restrict__ A, const float* __restrict__ Q, int64_t N,
                                           int64_t xs, int n3, int p, int lq, int kh, int j0,
                                           float (&b)[U][VEC], float (&a)[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int tc = min(2 * (j0 + u) + kh, n3 - 1);
    load_vec<VEC>(A + (int64_t)tc * N + xs, b[u]);
    a[u] = Q[(int64_t)tc * p + lq];
  }
}

template <int VEC, int U>
__device__ __forceinline__ void strip_mma(int n3, int p, int l, bool active, int kh, int j0,
                                          const float (&b)[U][VEC], const float (&a)[U], f32x16 (&acc)[VEC]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int t = 2 * (j0 + u) + kh;
    const float av = (t < n3 && l < p) ? a[u] : 0.f;
    const bool okb = active && t < n3;
#pragma unroll
    for (int q = 0; q < VEC; ++q)
      acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, okb ? b[u][q] : 0.f, acc[q], 0, 0, 0);
  }
}

// One workgroup's strip `strip` of tubes and 32-row chunk `lc` of the
// transform (red: (S - 1) * VEC * 16 * 64 floats of LDS)
template <int VEC, int S, int U, typename TIn>
__device__ __forceinline__ void hat_strip_body(const TIn* __restrict__ A, const float* __restrict__ Q,
                                               float* __restrict__ Ah, int64_t N, int n3, int p, int64_t strip,
                                               int lc, float* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = lane & 31, kh = lane >> 5;
  const int64_t xl = strip * (32 * VEC) + (int64_t)VEC * n;
  const bool active = xl < N;
  const int64_t xs = active ? xl : N - VEC;  // a valid tube for address arithmetic
  const int l = lc + n;                      // this lane's column of Q (row of the MFMA's A operand)
  const int lq = min(l, p - 1);
  f32x16 acc[VEC];
#pragma unroll
  for (int q = 0; q < VEC; ++q)
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[q][j] = 0.f;
  const int npairs = (n3 + 1) >> 1;
  constexpr int step = S * U;
  float b0[U][VEC], a0[U], b1[U][VEC], a1[U];
  int j0 = wave * U;
  strip_load<VEC, U, TIn>(A, Q, N, xs, n3, p, lq, kh, j0, b0, a0);
  // the scheduling barriers keep each batch's loads ahead of the previous
  // batch's MFMAs (the compiler would otherwise interleave them and wait)
  while (j0 < npairs) {
    strip_load<VEC, U, TIn>(A, Q, N, xs, n3, p, lq, kh, j0 + step, b1, a1);
    __builtin_amdgcn_sched_barrier(0);
    strip_mma<VEC, U>(n3, p, l, active, kh, j0, b0, a0, acc);
    __builtin_amdgcn_sched_barrier(0);
    j0 += step;
    if (j0 >= npairs) break;
    strip_load<VEC, U, TIn>(A, Q, N, xs, n3, p, lq, kh, j0 + step, b0, a0);
    __builtin_amdgcn_sched_barrier(0);
    strip_mma<VEC, U>(n3, p, l, active, kh, j0, b1, a1, acc);
    __builtin_amdgcn_sched_barrier(0);
    j0 += step;
  }
  if (reduce_waves<VEC, S>(acc, red, wave, lane) && active) {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int lo = lc + 8 * (j >> 2) + 4 * kh + (j & 3);
      if (lo < p) {
        float v[VEC];
#pragma unroll
        for (int q = 0; q < VEC; ++q) v[q] = acc[q][j];
        store_vec<VEC>(Ah + (int64_t)lo * N + xl, v);
      }
    }
  }
}

// MW: minimum waves per SIMD the register allocation must allow (occupancy)
template <int VEC, int S, int U, int MW, typename TIn>
__global__ __launch_bounds__(S * 64, MW) void hat_strip_kernel(const TIn* __restrict__ A, const float* __restrict__ Q,
                                                               float* __restrict__ Ah, int64_t N, int n3, int p) {
  extern __shared__ float red[];  // (S - 1) * VEC * 16 * 64
  hat_strip_body<VEC, S, U, TIn>(A, Q, Ah, N, n3, p, blockIdx.x, blockIdx.y * 32, red);
}

// Many forward transforms of float32 tensors in one launch (the batched
// form): workgroup w takes tile tiles[w] (descriptor, strip, 32-row chunk).
template <int VEC, int S, int U, int MW>
__global__ __launch_bounds__(S * 64, MW) void hat_grouped_kernel(const XformDesc* __restrict__ descs,
                                                                 const XformTile* __restrict__ tiles) {
  extern __shared__ float red[];
  const XformTile t = tiles[blockIdx.x];
  const XformDesc d = descs[t.desc];
  hat_strip_body<VEC, S, U, float>(d.in, d.Q, d.out, d.N, d.n3, d.p, t.x, 32 * t.y, red);
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
  const int64_t xs = active ? xl : N - VEC;  // a valid tube for address arithmetic
  float breg[16][VEC];
  if (regB) {
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int l = 2 * s + kh;
      load_vec<VEC, float>(Ah + (int64_t)min(l, p - 1) * N + xs, breg[s]);
#pragma unroll
      for (int q = 0; q < VEC; ++q) breg[s][q] = (active && l < p) ? breg[s][q] : 0.f;
    }
  }
  for (int tile = blockIdx.y; tile < ntiles; tile += gridDim.y) {
    const int t0 = tile * 32;
    __syncthreads();
    for (int e = threadIdx.x; e < p_pad * 32; e += WAVES * 64) {
      const int l = e >> 5, tt = e & 31;
      const float v = Q[(int64_t)min(t0 + tt, n3 - 1) * p + min(l, p - 1)];
      QsT[e] = (t0 + tt < n3 && l < p) ? v : 0.f;
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
        load_vec<VEC, float>(Ah + (int64_t)min(l, p - 1) * N + xs, b);
#pragma unroll
        for (int q = 0; q < VEC; ++q) b[q] = (active && l < p) ? b[q] : 0.f;
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

// Fused projection, p <= 32: hat of the strip into the accumulators (split
// over the S waves as above), the sum broadcast back to every wave through
// LDS, then the accumulators feed the unhat MFMAs directly, each wave taking
// every S-th 32-row output tile.  For unhat step j a lane supplies, as its B
// operand, its accumulator register j, which holds transform row
// l = 8*(j/4) + 4*kh + j%4 of its tube; the A operand it supplies is Q(t, l)
// for that same l, so each step contracts over the two rows held by the two
// half-waves and no data moves between lanes.
template <int VEC, int S, typename TIn>
__global__ __launch_bounds__(S * 64) void proj_f32_kernel(const TIn* __restrict__ A,
                                                          const float* __restrict__ Q,
                                                          float* __restrict__ out, int64_t N,
                                                          int n3, int p) {
  extern __shared__ float smem[];
  constexpr int ld = 33;
  const int ntiles = (n3 + 31) / 32;
  const int rows_pad = ntiles * 32 + 16;
  float* Qs = smem;                            // [rows_pad][33]
  float* red = smem + rows_pad * ld;           // S * VEC * 16 * 64 floats
  for (int kc = 0; kc < rows_pad; kc += 32) stage_q_rows(Q, p, n3, kc, min(32, rows_pad - kc), 0, Qs + kc * ld, ld, S * 64);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = lane & 31, kh = lane >> 5;
  const int64_t xl = (int64_t)blockIdx.x * (32 * VEC) + (int64_t)VEC * n;
  const bool active = xl < N;
  const int64_t xs = active ? xl : N - VEC;  // a valid tube for address arithmetic
  f32x16 h[VEC];
#pragma unroll
  for (int q = 0; q < VEC; ++q)
#pragma unroll
    for (int j = 0; j < 16; ++j) h[q][j] = 0.f;
  hat_accumulate<VEC, S, TIn>(A + xs, N, active, n3, Qs, ld, wave, n, kh, h);
  if constexpr (S > 1) {
    const bool w0 = reduce_waves<VEC, S>(h, red, wave, lane);
    if (w0) {
#pragma unroll
      for (int q = 0; q < VEC; ++q)
#pragma unroll
        for (int j = 0; j < 16; ++j) red[((S - 1) * VEC + q) * 16 * 64 + j * 64 + lane] = h[q][j];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < VEC; ++q)
#pragma unroll
      for (int j = 0; j < 16; ++j) h[q][j] = red[((S - 1) * VEC + q) * 16 * 64 + j * 64 + lane];
  }
  for (int tile = wave; tile < ntiles; tile += S) {
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

// ---- bfloat16 matrix-core forms of the transform ---------------------------
// v_mfma_f32_32x32x16_bf16: D(32 x 32) += A(32 x 16) B(16 x 32); lane L holds
// A row L%32 and B column L%32, each over k = 8*(L/32) .. +7 (8 bfloat16 in 4
// dwords, k pairs packed low/high).  Here A = Q^T (rows: transform index l,
// k: the frontal-slice index t) and B = a 16-row slab of the tensor.
//
// A lane reads 8 consecutive rows t of TPL consecutive tubes (coalesced
// across the 32 lanes of a half-wave), packs rows 2q and 2q+1 of each tube
// into dword q of that tube's B operand (v_cvt_pk_bf16_f32 does the packing
// and the rounding at once), and issues one MFMA per tube and product; MFMA
// column n of tube slot c is tube 32*TPL*strip + TPL*n + c.
//
// Precision modes are sums of products of bfloat16 parts, x = x0 + x1 + x2
// with x0 = bf16(x), x1 = bf16(x - x0), x2 = bf16(x - x0 - x1):
//   plain: a0 q0;  split x3: a0 q0 + a0 q1 + a1 q0;
//   split x6: a0 q0 + a0 q1 + a1 q0 + a0 q2 + a1 q1 + a2 q0;
//   bfloat16 input, x3 or x6: a q0 + a q1 + a q2 (exact in float32: three
//   bfloat16 parts carry the full 24-bit significand of q).
template <typename TIn, int NA, int NQ, int TPL, int S>
__global__ __launch_bounds__(S * 64) void hat_bf16_kernel(const TIn* __restrict__ A,
                                                          const float* __restrict__ Q,
                                                          float* __restrict__ Ah, int64_t N, int n3,
                                                          int p, int kcr, int64_t nstrips) {
  using SP = Split<NA, NQ>;
  // Q parts in LDS as [part][t/8][l][8 bfloat16] (kcr rows): the 32 lanes of
  // a half-wave read 32 consecutive 16-byte rows.  Then the reduction buffer.
  extern __shared__ __align__(16) uint32_t smem_u[];
  auto qs = [&](int i, int t8, int l) -> uint32_t* {
    return smem_u + (((i * (kcr >> 3) + t8) * 32 + l) << 2);
  };
  float* red = reinterpret_cast<float*>(smem_u + NQ * kcr * 16);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = lane & 31, kh = lane >> 5;
  const int lc = blockIdx.y * 32;
  const bool one_chunk = n3 <= kcr;
  auto stage = [&](int kc) {
    const int rows = min(kcr, n3 - kc);
    const int total = (kcr / 2) * 32;
    for (int e0 = threadIdx.x; e0 < total; e0 += 4 * S * 64) {
      float qv[4][2];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = min(e0 + u * S * 64, total - 1);
        const int l = e & 31, t = 2 * (e >> 5);
        const int lcl = min(lc + l, p - 1);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const float v = Q[(int64_t)(kc + min(t + h, rows - 1)) * p + lcl];
          qv[u][h] = (t + h < rows && lc + l < p) ? v : 0.f;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * S * 64;
        if (e >= total) continue;
        const int l = e & 31, t = 2 * (e >> 5);
        uint32_t parts[NQ];
        split_pack<NQ>(qv[u][0], qv[u][1], parts);
#pragma unroll
        for (int i = 0; i < NQ; ++i) qs(i, t >> 3, l)[(t & 7) >> 1] = parts[i];
      }
    }
  };
  if (one_chunk) {
    stage(0);
    __syncthreads();
  }
  for (int64_t strip = blockIdx.x; strip < nstrips; strip += gridDim.x) {
    const int64_t xl = strip * (32 * TPL) + (int64_t)TPL * n;
    const bool active = xl < N;
    const int64_t xs = active ? xl : N - TPL;  // a valid tube for address arithmetic
    f32x16 acc[TPL];
#pragma unroll
    for (int c = 0; c < TPL; ++c)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[c][j] = 0.f;
    for (int kc = 0; kc < n3; kc += kcr) {
      if (!one_chunk) {
        __syncthreads();
        stage(kc);
        __syncthreads();
      }
      const int rows = min(kcr, n3 - kc);
      const int nsteps = (rows + 15) / 16;
      float x0[8][TPL], x1[8][TPL];
      auto load_step = [&](int st, float (&x)[8][TPL]) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int t = 16 * st + 8 * kh + r;
          const bool ok = active && t < rows;
          load_vec<TPL, TIn>(A + (int64_t)(kc + min(t, rows - 1)) * N + xs, x[r]);
#pragma unroll
          for (int c = 0; c < TPL; ++c) x[r][c] = ok ? x[r][c] : 0.f;
        }
      };
      auto mfma_step = [&](int st, const float (&x)[8][TPL]) {
        bf16x8 qop[NQ];
#pragma unroll
        for (int i = 0; i < NQ; ++i) qop[i] = *reinterpret_cast<const bf16x8*>(qs(i, 2 * st + kh, n));
#pragma unroll
        for (int c = 0; c < TPL; ++c) {
          uint32_t bw[NA][4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            uint32_t parts[NA];
            split_pack<NA>(x[2 * q][c], x[2 * q + 1][c], parts);
#pragma unroll
            for (int i = 0; i < NA; ++i) bw[i][q] = parts[i];
          }
#pragma unroll
          for (int pr = 0; pr < SP::n; ++pr) {
            const bf16x8 bop = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(bw[SP::a[pr]]));
            acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(qop[SP::q[pr]], bop, acc[c], 0, 0, 0);
          }
        }
      };
      // loads past the last step read clamped addresses and are masked; the
      // scheduling barriers keep each step's loads ahead of the previous
      // step's MFMAs
      int st = wave;
      load_step(st, x0);
      while (st < nsteps) {
        load_step(st + S, x1);
        __builtin_amdgcn_sched_barrier(0);
        mfma_step(st, x0);
        __builtin_amdgcn_sched_barrier(0);
        st += S;
        if (st >= nsteps) break;
        load_step(st + S, x0);
        __builtin_amdgcn_sched_barrier(0);
        mfma_step(st, x1);
        __builtin_amdgcn_sched_barrier(0);
        st += S;
      }
    }
    if (reduce_waves<TPL, S>(acc, red, wave, lane) && active) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int l = lc + 8 * (j >> 2) + 4 * kh + (j & 3);
        if (l < p) {
          float v[TPL];
#pragma unroll
          for (int c = 0; c < TPL; ++c) v[c] = acc[c][j];
          store_vec<TPL>(Ah + (int64_t)l * N + xl, v);
        }
      }
    }
  }
}

// ---- return transform, strip per wave -----------------------------------------
// Each wave owns a strip of 32*VEC tubes and keeps Chat(:, strip) (p <= 32) in
// registers; the workgroups along y take the 32-row tiles of the output in
// turn.  Per tile the 32 x p block of Q is read through the cache (the next
// tile's entries are loaded before the current tile's MFMAs), the tile is
// formed on the MFMA and written with VEC-wide stores.  No LDS, no barrier.
// float32: v_mfma_f32_32x32x2f32 over pairs of channels; split-bfloat16:
// v_mfma_f32_32x32x16_bf16 over 16 channels at a time, both operands split
// into parts (Split<NA, NQ>: Chat parts x Q parts).
// (workgroup bx of the strips; output tiles y0, y0 + ystep, ...)
// QL: the workgroup's copy of Q in LDS (row stride p | 1, so that the 32
// rows a half-wave reads fall in distinct banks).  Reading Q from memory
// inside the loop makes each tile wait for the previous tile's stores: the
// memory counter orders loads and stores together, and with stores under a
// branch the compiler's wait for the Q loads has to cover them all.  From
// LDS, the stores of one tile drain while the next tile's MFMAs run.
__host__ __device__ __forceinline__ int q_lds_stride(int p) { return p | 1; }

template <bool QL>
__device__ __forceinline__ void stage_q(const float* __restrict__ Q, int n3, int p, float* qs) {
  if constexpr (QL) {
    const int ps = q_lds_stride(p);
    for (int e = threadIdx.x; e < n3 * p; e += blockDim.x) qs[(e / p) * ps + e % p] = Q[e];
    __syncthreads();
  }
}

template <int VEC, int W, bool QL>
__device__ __forceinline__ void unhat_strip_body(const float* __restrict__ Ah, const float* __restrict__ Q,
                                                 float* __restrict__ C, int64_t N, int n3, int p, int64_t bx,
                                                 int y0, int ystep, const float* qs) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = lane & 31, kh = lane >> 5;
  const int64_t xl = (bx * W + wave) * (32 * VEC) + (int64_t)VEC * n;
  const bool active = xl < N;
  const int64_t xs = active ? xl : N - VEC;
  const int ntiles = (n3 + 31) >> 5;
  float b[16][VEC];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int l = 2 * s + kh;
    load_vec<VEC, float>(Ah + (int64_t)min(l, p - 1) * N + xs, b[s]);
#pragma unroll
    for (int q = 0; q < VEC; ++q) b[s][q] = (l < p) ? b[s][q] : 0.f;
  }
  auto qload = [&](int tile, float (&a)[16]) {
    const int t = min(tile * 32 + n, n3 - 1);
    if constexpr (QL) {
      const int ps = q_lds_stride(p);
#pragma unroll
      for (int s = 0; s < 16; ++s) a[s] = qs[t * ps + min(2 * s + kh, p - 1)];
    } else {
#pragma unroll
      for (int s = 0; s < 16; ++s) a[s] = Q[(int64_t)t * p + min(2 * s + kh, p - 1)];
    }
  };
  float a0[16], a1[16];
  int tile = y0;
  qload(min(tile, ntiles - 1), a0);
  while (tile < ntiles) {
    const int nxt = tile + ystep;
    qload(min(nxt, ntiles - 1), a1);
    __builtin_amdgcn_sched_barrier(0);
    f32x16 acc[VEC];
#pragma unroll
    for (int q = 0; q < VEC; ++q)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[q][j] = 0.f;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      if (2 * s < p) {
        const float av = (2 * s + kh < p) ? a0[s] : 0.f;
#pragma unroll
        for (int q = 0; q < VEC; ++q) acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, b[s][q], acc[q], 0, 0, 0);
      }
    }
    if (active) {
      const int t0 = tile * 32;
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
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < 16; ++s) a0[s] = a1[s];
    tile = nxt;
  }
}

template <int VEC, int W, int MW, bool QL>
__global__ __launch_bounds__(W * 64, MW) void unhat_strip_kernel(const float* __restrict__ Ah,
                                                                 const float* __restrict__ Q,
                                                                 float* __restrict__ C, int64_t N, int n3, int p) {
  extern __shared__ float qs[];  // QL: n3 rows of q_lds_stride(p)
  stage_q<QL>(Q, n3, p, qs);
  unhat_strip_body<VEC, W, QL>(Ah, Q, C, N, n3, p, blockIdx.x, blockIdx.y, gridDim.y, qs);
}

// Many return transforms in one launch (the batched form): workgroup w takes
// tile tiles[w] (descriptor, workgroup of strips, every output tile).
template <int VEC, int W, int MW, bool QL>
__global__ __launch_bounds__(W * 64, MW) void unhat_grouped_kernel(const XformDesc* __restrict__ descs,
                                                                   const XformTile* __restrict__ tiles) {
  extern __shared__ float qs[];
  const XformTile t = tiles[blockIdx.x];
  const XformDesc d = descs[t.desc];
  stage_q<QL>(d.Q, d.n3, d.p, qs);
  unhat_strip_body<VEC, W, QL>(d.in, d.Q, d.out, d.N, d.n3, d.p, t.x, t.y, 1, qs);
}


template <int VEC, int W, int MW, int NA, int NQ>
__global__ __launch_bounds__(W * 64, MW) void unhat_bstrip_kernel(const float* __restrict__ Ah,
                                                                  const float* __restrict__ Q,
                                                                  float* __restrict__ C, int64_t N, int n3, int p) {
  using SP = Split<NA, NQ>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = lane & 31, kh = lane >> 5;
  const int64_t xl = ((int64_t)blockIdx.x * W + wave) * (32 * VEC) + (int64_t)VEC * n;
  const bool active = xl < N;
  const int64_t xs = active ? xl : N - VEC;
  const int ntiles = (n3 + 31) >> 5;
  const int nsteps = (p + 15) >> 4;  // 16 channels per MFMA (p <= 32)
  // Chat(16 st + 8 kh + i, strip) split into NA parts, packed by pairs of i
  uint32_t bw[2][VEC][NA][4];
#pragma unroll
  for (int st = 0; st < 2; ++st)
#pragma unroll
    for (int q2 = 0; q2 < 4; ++q2) {
      float x0[VEC], x1[VEC];
      const int l0 = 16 * st + 8 * kh + 2 * q2;
      load_vec<VEC, float>(Ah + (int64_t)min(l0, p - 1) * N + xs, x0);
      load_vec<VEC, float>(Ah + (int64_t)min(l0 + 1, p - 1) * N + xs, x1);
#pragma unroll
      for (int c = 0; c < VEC; ++c) {
        uint32_t parts[NA];
        split_pack<NA>(l0 < p ? x0[c] : 0.f, l0 + 1 < p ? x1[c] : 0.f, parts);
#pragma unroll
        for (int i = 0; i < NA; ++i) bw[st][c][i][q2] = parts[i];
      }
    }
  auto qload = [&](int tile, float (&a)[2][8]) {
    const int t = min(tile * 32 + n, n3 - 1);
#pragma unroll
    for (int st = 0; st < 2; ++st)
#pragma unroll
      for (int i = 0; i < 8; ++i) a[st][i] = Q[(int64_t)t * p + min(16 * st + 8 * kh + i, p - 1)];
  };
  float a0[2][8], a1[2][8];
  int tile = blockIdx.y;
  qload(min(tile, ntiles - 1), a0);
  while (tile < ntiles) {
    const int nxt = tile + gridDim.y;
    qload(min(nxt, ntiles - 1), a1);
    __builtin_amdgcn_sched_barrier(0);
    f32x16 acc[VEC];
#pragma unroll
    for (int c = 0; c < VEC; ++c)
#pragma unroll
      for (int j = 0; j < 16; ++j) acc[c][j] = 0.f;
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      if (st < nsteps) {
        uint32_t qw[NQ][4];
#pragma unroll
        for (int q2 = 0; q2 < 4; ++q2) {
          const int l0 = 16 * st + 8 * kh + 2 * q2;
          uint32_t parts[NQ];
          split_pack<NQ>(l0 < p ? a0[st][2 * q2] : 0.f, l0 + 1 < p ? a0[st][2 * q2 + 1] : 0.f, parts);
#pragma unroll
          for (int i = 0; i < NQ; ++i) qw[i][q2] = parts[i];
        }
#pragma unroll
        for (int c = 0; c < VEC; ++c)
#pragma unroll
          for (int pr = 0; pr < SP::n; ++pr) {
            const bf16x8 aop = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(qw[SP::q[pr]]));
            const bf16x8 bop = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(bw[st][c][SP::a[pr]]));
            acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aop, bop, acc[c], 0, 0, 0);
          }
      }
    }
    if (active) {
      const int t0 = tile * 32;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int t = t0 + 8 * (j >> 2) + 4 * kh + (j & 3);
        if (t < n3) {
          float v[VEC];
#pragma unroll
          for (int c = 0; c < VEC; ++c) v[c] = acc[c][j];
          store_vec<VEC>(C + (int64_t)t * N + xl, v);
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int st = 0; st < 2; ++st)
#pragma unroll
      for (int i = 0; i < 8; ++i) a0[st][i] = a1[st][i];
    tile = nxt;
  }
}

// ---- split-bfloat16 transform, one strip per workgroup ------------------------
// The strip design of hat_strip_kernel for the bfloat16 MFMA
// (v_mfma_f32_32x32x16_bf16): a step is 16 frontal slices, the lanes of
// half-wave kh holding slices 8 kh .. 8 kh + 7 of it for their TPL tubes.
// Both operands are split into bfloat16 parts in registers as they arrive
// (Q's 8 entries per step come through the cache), the SP::n part products
// accumulate in float32, and the next step's loads are issued before the
// current step's MFMAs.
template <int TPL, typename TIn>
__device__ __forceinline__ void bstrip_load(const TIn* __restrict__ A, const float* __restrict__ Q, int64_t N,
                                            int64_t xs, int n3, int p, int lq, int kh, int st, float (&x)[8][TPL],
                                            float (&qv)[8]) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int tc = min(16 * st + 8 * kh + r, n3 - 1);
    load_vec<TPL, TIn>(A + (int64_t)tc * N + xs, x[r]);
    qv[r] = Q[(int64_t)tc * p + lq];
  }
}

template <int TPL, int NA, int NQ>
__device__ __forceinline__ void bstrip_mma(int n3, int p, int l, bool active, int kh, int st,
                                           const float (&x)[8][TPL], const float (&qv)[8], f32x16 (&acc)[TPL]) {
  using SP = Split<NA, NQ>;
  uint32_t qw[NQ][4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int t = 16 * st + 8 * kh + 2 * q;
    uint32_t parts[NQ];
    split_pack<NQ>((t < n3 && l < p) ? qv[2 * q] : 0.f, (t + 1 < n3 && l < p) ? qv[2 * q + 1] : 0.f, parts);
#pragma unroll
    for (int i = 0; i < NQ; ++i) qw[i][q] = parts[i];
  }
#pragma unroll
  for (int c = 0; c < TPL; ++c) {
    uint32_t bw[NA][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int t = 16 * st + 8 * kh + 2 * q;
      uint32_t parts[NA];
      split_pack<NA>((active && t < n3) ? x[2 * q][c] : 0.f, (active && t + 1 < n3) ? x[2 * q + 1][c] : 0.f, parts);
#pragma unroll
      for (int i = 0; i < NA; ++i) bw[i][q] = parts[i];
    }
#pragma unroll
    for (int pr = 0; pr < SP::n; ++pr) {
      const bf16x8 aop = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(qw[SP::q[pr]]));
      const bf16x8 bop = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(bw[SP::a[pr]]));
      acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aop, bop, acc[c], 0, 0, 0);
    }
  }
}

template <typename TIn, int NA, int NQ, int TPL, int S, int MW>
__global__ __launch_bounds__(S * 64, MW) void hat_bstrip_kernel(const TIn* __restrict__ A, const float* __restrict__ Q,
                                                                float* __restrict__ Ah, int64_t N, int n3, int p) {
  extern __shared__ float red[];  // (S - 1) * TPL * 16 * 64
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n = lane & 31, kh = lane >> 5;
  const int lc = blockIdx.y * 32;
  const int64_t xl = (int64_t)blockIdx.x * (32 * TPL) + (int64_t)TPL * n;
  const bool active = xl < N;
  const int64_t xs = active ? xl : N - TPL;  // a valid tube for address arithmetic
  const int l = lc + n, lq = min(l, p - 1);
  f32x16 acc[TPL];
#pragma unroll
  for (int c = 0; c < TPL; ++c)
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[c][j] = 0.f;
  const int nsteps = (n3 + 15) >> 4;
  float x0[8][TPL], q0[8], x1[8][TPL], q1[8];
  int st = wave;
  bstrip_load<TPL, TIn>(A, Q, N, xs, n3, p, lq, kh, st, x0, q0);
  while (st < nsteps) {
    bstrip_load<TPL, TIn>(A, Q, N, xs, n3, p, lq, kh, st + S, x1, q1);
    __builtin_amdgcn_sched_barrier(0);
    bstrip_mma<TPL, NA, NQ>(n3, p, l, active, kh, st, x0, q0, acc);
    __builtin_amdgcn_sched_barrier(0);
    st += S;
    if (st >= nsteps) break;
    bstrip_load<TPL, TIn>(A, Q, N, xs, n3, p, lq, kh, st + S, x0, q0);
    __builtin_amdgcn_sched_barrier(0);
    bstrip_mma<TPL, NA, NQ>(n3, p, l, active, kh, st, x1, q1, acc);
    __builtin_amdgcn_sched_barrier(0);
    st += S;
  }
  if (reduce_waves<TPL, S>(acc, red, wave, lane) && active) {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int lo = lc + 8 * (j >> 2) + 4 * kh + (j & 3);
      if (lo < p) {
        float v[TPL];
#pragma unroll
        for (int c = 0; c < TPL; ++c) v[c] = acc[c][j];
        store_vec<TPL>(Ah + (int64_t)lo * N + xl, v);
      }
    }
  }
}

// ---- float64 (plain VALU; the float64 path serves small problems) --------
// float64 forward transform Ah (p x N) = Q^T A for float32 A (widened on
// load, exactly) or float64 A: 64 tubes per workgroup of four waves and PC
// columns of Q per grid row.  Q is staged in LDS 64 rows at a time (zero past
// n3 and p; every lane of a wave reads the same entry, a broadcast); wave w
// accumulates the rows t = w (mod 4) of its lane's tube, and the four
// partial sums are added in wave order through LDS.
constexpr int kHat64Rows = 64;

template <typename TA, int PC>
__global__ __launch_bounds__(256) void hat64_kernel(const TA* __restrict__ A, const double* __restrict__ Q,
                                                    double* __restrict__ Ah, int64_t N, int n3, int p) {
  __shared__ __align__(16) double Qs[kHat64Rows][PC];
  __shared__ double part[3][PC][64];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t x = (int64_t)blockIdx.x * 64 + lane;
  const int64_t xc = x < N ? x : N - 1;
  const int lc = blockIdx.y * PC;
  double acc[PC];
#pragma unroll
  for (int c = 0; c < PC; ++c) acc[c] = 0.0;
  for (int kc = 0; kc < n3; kc += kHat64Rows) {
    __syncthreads();
    for (int e = threadIdx.x; e < kHat64Rows * PC; e += 256) {
      const int r = e / PC, c = e % PC;
      Qs[r][c] = (kc + r < n3 && lc + c < p) ? Q[(int64_t)(kc + r) * p + lc + c] : 0.0;
    }
    __syncthreads();
    const int rows = min(kHat64Rows, n3 - kc);
#pragma unroll 2
    for (int r = w; r < rows; r += 4) {
      const double a = (double)A[(int64_t)(kc + r) * N + xc];
#pragma unroll
      for (int c = 0; c < PC; ++c) acc[c] = fma(Qs[r][c], a, acc[c]);
    }
  }
  if (w > 0) {
#pragma unroll
    for (int c = 0; c < PC; ++c) part[w - 1][c][lane] = acc[c];
  }
  __syncthreads();
  if (w == 0 && x < N) {
#pragma unroll
    for (int c = 0; c < PC; ++c)
      if (lc + c < p)
        Ah[(int64_t)(lc + c) * N + x] = ((acc[c] + part[0][c][lane]) + part[1][c][lane]) + part[2][c][lane];
  }
}

// float64 return transform C (n3 x N) = Q Ah: one tube per thread and TR
// slices per grid row, the TR x 64 block of Q for the current 64 columns
// staged in LDS (every lane reads the same entry, a broadcast); each thread
// reads its tube's p transform-domain values once per grid row and keeps
// the TR outputs in registers.
constexpr int kUnhat64Rows = 32;

__global__ __launch_bounds__(256) void unhat64_kernel(const double* __restrict__ Ah, const double* __restrict__ Q,
                                                      double* __restrict__ C, int64_t N, int n3, int p) {
  constexpr int TR = kUnhat64Rows;
  __shared__ double Qs[64][TR];  // Qs[i][j] = Q[t0 + j][l0 + i]
  const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t xc = x < N ? x : N - 1;
  const int t0 = blockIdx.y * TR;
  double acc[TR];
#pragma unroll
  for (int j = 0; j < TR; ++j) acc[j] = 0.0;
  for (int l0 = 0; l0 < p; l0 += 64) {
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * TR; e += 256) {
      const int i = e / TR, j = e % TR;
      Qs[i][j] = (l0 + i < p && t0 + j < n3) ? Q[(int64_t)(t0 + j) * p + l0 + i] : 0.0;
    }
    __syncthreads();
    const int ln = min(64, p - l0);
#pragma unroll 2
    for (int i = 0; i < ln; ++i) {
      const double a = Ah[(int64_t)(l0 + i) * N + xc];
#pragma unroll
      for (int j = 0; j < TR; ++j) acc[j] = fma(Qs[i][j], a, acc[j]);
    }
  }
  if (x >= N) return;
#pragma unroll
  for (int j = 0; j < TR; ++j)
    if (t0 + j < n3) C[(int64_t)(t0 + j) * N + x] = acc[j];
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

// Candidate launch configurations of the transforms: vector width (tubes per
// lane) x waves per workgroup x strips per workgroup.  For the forward
// transform and the projection the waves of a workgroup split the rows of its
// current strip (split-K inside the workgroup) and the workgroup walks over
// `spw` strips; for the return transform each wave has its own strip.
struct Cfg {
  int vec, waves, spw;
  int strip = 0;  // > 0: hat_strip_kernel, `spw` slice pairs per load batch, `strip` min waves per SIMD
  bool f32 = false;  // a split-bfloat16 mode's candidate that runs the float32 kernel
  bool qlds = false;  // float32 return strip with Q staged in LDS
};

std::vector<Cfg> cands(int vmax, bool splitk) {
  std::vector<Cfg> v;
  for (int vec : {4, 2, 1})
    if (vec <= vmax)
      for (int w : {1, 2, 4, 8}) {
        if (!splitk) {
          if (w >= 2) v.push_back({vec, w, 1});
        } else if (vec * w <= 16) {
          for (int spw : {1, 4}) v.push_back({vec, w, spw});
        }
      }
  return v;
}

// untuned default for the split-K kernels: the widest vector whose strips,
// times up to 16 / vec waves each, still give about 2048+ waves; the waves
// per strip chosen to reach about 4096; one strip per workgroup
int default_splitk(const std::vector<Cfg>& c, int64_t N) {
  Cfg want{1, 8, 1};
  for (int vec : {4, 2, 1}) {
    const int64_t strips = (N + 32 * vec - 1) / (32 * vec);
    int w = 1;
    while (w < 8 && vec * w * 2 <= 16 && strips * w < 4096) w *= 2;
    if (strips * w >= 2048 || vec == 1) {
      want = {vec, w, 1};
      break;
    }
  }
  for (size_t i = 0; i < c.size(); ++i)
    if (c[i].vec == want.vec && c[i].waves == want.waves && c[i].spw == want.spw) return (int)i;
  return (int)c.size() - 1;
}

int default_strips(const std::vector<Cfg>& c, int64_t N) {
  int want = 1;
  for (int vec : {4, 2})
    if (want == 1 && N / (32 * vec) >= 2048) want = vec;
  for (size_t i = 0; i < c.size(); ++i)
    if (c[i].vec == want && c[i].waves == 4) return (int)i;
  return 0;
}

std::string key_of(const char* kind, int prec, int bf, int64_t N, int n3, int p, int vmax) {
  return std::string(kind) + "/prec" + std::to_string(prec) + "/bf" + std::to_string(bf) + "/N" +
         std::to_string(N) + "/n3_" + std::to_string(n3) + "/p" + std::to_string(p) + "/v" +
         std::to_string(vmax);
}

// dynamic LDS beyond the 64 KB default, set once per kernel instance
template <typename K>
hipError_t allow_lds(K kernel, size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

size_t red_bytes(int vec, int S) { return sizeof(float) * (size_t)(S - 1) * vec * 16 * 64; }

// rows of Q staged per chunk: n3 rounded up to 16, at most kKC
int chunk_rows(int n3) { return std::min(kKC, (n3 + 15) / 16 * 16); }

template <int VEC, int S, typename TIn>
hipError_t hat_f32_go(const TIn* A, const float* Q, float* Ah, int64_t N, int n3, int p, int spw,
                      hipStream_t s) {
  const int kcr = chunk_rows(n3);
  const size_t lds = sizeof(float) * (size_t)kcr * 32 + red_bytes(VEC, S);
  static hipError_t attr = allow_lds(&hat_f32_kernel<VEC, S, TIn>, 120 * 1024);
  if (attr != hipSuccess) return attr;
  const int64_t nstrips = (N + 32 * VEC - 1) / (32 * VEC);
  dim3 grid((unsigned)((nstrips + spw - 1) / spw), (unsigned)((p + 31) / 32));
  hat_f32_kernel<VEC, S, TIn><<<grid, S * 64, lds, s>>>(A, Q, Ah, N, n3, p, kcr, nstrips);
  return hipGetLastError();
}

template <typename TIn, int NA, int NQ, int TPL, int S>
hipError_t hat_bf16_go(const TIn* A, const float* Q, float* Ah, int64_t N, int n3, int p, int spw,
                       hipStream_t s) {
  const int kcr = chunk_rows(n3);
  const size_t lds = (size_t)NQ * kcr * 64 + red_bytes(TPL, S);
  static hipError_t attr = allow_lds(&hat_bf16_kernel<TIn, NA, NQ, TPL, S>, 120 * 1024);
  if (attr != hipSuccess) return attr;
  const int64_t nstrips = (N + 32 * TPL - 1) / (32 * TPL);
  dim3 grid((unsigned)((nstrips + spw - 1) / spw), (unsigned)((p + 31) / 32));
  hat_bf16_kernel<TIn, NA, NQ, TPL, S><<<grid, S * 64, lds, s>>>(A, Q, Ah, N, n3, p, kcr, nstrips);
  return hipGetLastError();
}

template <int VEC, int S, int U, int MW, typename TIn>
hipError_t hat_strip_go(const TIn* A, const float* Q, float* Ah, int64_t N, int n3, int p, hipStream_t s) {
  const size_t lds = red_bytes(VEC, S);
  dim3 grid((unsigned)((N + 32 * VEC - 1) / (32 * VEC)), (unsigned)((p + 31) / 32));
  hat_strip_kernel<VEC, S, U, MW, TIn><<<grid, S * 64, lds, s>>>(A, Q, Ah, N, n3, p);
  return hipGetLastError();
}

template <typename TIn>
hipError_t hat_strip_any(const TIn* A, const float* Q, float* Ah, int64_t N, int n3, int p, Cfg c,
                         hipStream_t s) {
#define PQ_S(V, W, U, MW)                                                                   \
  if (c.vec == V && c.waves == W && c.spw == U && c.strip == MW)                            \
    return hat_strip_go<V, W, U, MW, TIn>(A, Q, Ah, N, n3, p, s);
  PQ_S(4, 1, 4, 1) PQ_S(4, 2, 4, 1) PQ_S(4, 4, 4, 1) PQ_S(4, 2, 4, 2) PQ_S(4, 4, 4, 2) PQ_S(4, 2, 2, 4)
  PQ_S(4, 4, 2, 4) PQ_S(2, 2, 4, 1) PQ_S(2, 4, 4, 1) PQ_S(2, 2, 4, 4) PQ_S(2, 4, 4, 4) PQ_S(2, 4, 8, 2)
  PQ_S(1, 2, 4, 1) PQ_S(1, 4, 4, 1) PQ_S(1, 4, 8, 4) PQ_S(1, 8, 8, 4)
#undef PQ_S
  return hipErrorInvalidValue;
}

// strip-kernel candidates (vec, waves, pairs per batch, minimum waves per
// SIMD), widest vector first
void strip_cands(int vmax, std::vector<Cfg>& v) {
  static const int t[][4] = {{4, 1, 4, 1}, {4, 2, 4, 1}, {4, 4, 4, 1}, {4, 2, 4, 2}, {4, 4, 4, 2}, {4, 2, 2, 4},
                             {4, 4, 2, 4}, {2, 2, 4, 1}, {2, 4, 4, 1}, {2, 2, 4, 4}, {2, 4, 4, 4}, {2, 4, 8, 2},
                             {1, 2, 4, 1}, {1, 4, 4, 1}, {1, 4, 8, 4}, {1, 8, 8, 4}};
  for (const auto& r : t)
    if (r[0] <= vmax) {
      Cfg c{r[0], r[1], r[2]};
      c.strip = r[3];
      v.push_back(c);
    }
}

template <int VEC, int W, int MW, int NA, int NQ, bool QL = false>
hipError_t unhat_strip_go(const float* Ah, const float* Q, float* C, int64_t N, int n3, int p, hipStream_t s) {
  const int64_t strips = (N + 32 * VEC - 1) / (32 * VEC);
  const int64_t wgs = (strips + W - 1) / W;
  const int ntiles = (n3 + 31) / 32;
  // enough workgroups to fill 256 CUs several times over
  const int ysplit = (int)std::min<int64_t>(ntiles, std::max<int64_t>(1, (4096 + wgs - 1) / wgs));
  dim3 grid((unsigned)wgs, (unsigned)ysplit);
  if constexpr (NA == 0)
    unhat_strip_kernel<VEC, W, MW, QL>
        <<<grid, W * 64, QL ? sizeof(float) * (size_t)n3 * q_lds_stride(p) : 0, s>>>(Ah, Q, C, N, n3, p);
  else
    unhat_bstrip_kernel<VEC, W, MW, NA, NQ><<<grid, W * 64, 0, s>>>(Ah, Q, C, N, n3, p);
  return hipGetLastError();
}

// unhat strip candidates (vec, waves, min waves per SIMD); NA = 0: float32
template <int NA, int NQ>
hipError_t unhat_strip_any(const float* Ah, const float* Q, float* C, int64_t N, int n3, int p, Cfg c,
                           hipStream_t s) {
#define PQ_U(V, W, MW) \
  if (c.vec == V && c.waves == W && c.strip == MW) return unhat_strip_go<V, W, MW, NA, NQ>(Ah, Q, C, N, n3, p, s);
  if constexpr (NA == 0) {
    if (c.qlds) {
#define PQ_UL(V, W, MW) \
  if (c.vec == V && c.waves == W && c.strip == MW) return unhat_strip_go<V, W, MW, 0, 0, true>(Ah, Q, C, N, n3, p, s);
      PQ_UL(4, 4, 2) PQ_UL(4, 2, 2) PQ_UL(2, 4, 2) PQ_UL(2, 4, 4) PQ_UL(1, 8, 4)
#undef PQ_UL
      return hipErrorInvalidValue;
    }
  }
  PQ_U(4, 4, 2) PQ_U(4, 2, 2) PQ_U(2, 4, 4) PQ_U(2, 8, 4) PQ_U(2, 4, 2) PQ_U(2, 8, 2) PQ_U(1, 8, 4)
#undef PQ_U
  return hipErrorInvalidValue;
}

void unhat_strip_cands(int vmax, std::vector<Cfg>& v) {
  static const int t[][3] = {{4, 4, 2}, {4, 2, 2}, {2, 4, 4}, {2, 8, 4}, {2, 4, 2}, {2, 8, 2}, {1, 8, 4}};
  for (const auto& r : t)
    if (r[0] <= vmax) {
      Cfg c{r[0], r[1], 0};
      c.strip = r[2];
      v.push_back(c);
    }
}

// the float32 strip shapes with Q staged in LDS, when Q fits
constexpr size_t kQLdsMax = 64 * 1024;
void unhat_strip_ql_cands(int vmax, int n3, int p, std::vector<Cfg>& v) {
  if (sizeof(float) * (size_t)n3 * q_lds_stride(p) > kQLdsMax) return;
  static const int t[][3] = {{4, 4, 2}, {4, 2, 2}, {2, 4, 2}, {2, 4, 4}, {1, 8, 4}};
  for (const auto& r : t)
    if (r[0] <= vmax) {
      Cfg c{r[0], r[1], 0};
      c.strip = r[2];
      c.qlds = true;
      c.f32 = true;
      v.push_back(c);
    }
}

template <typename TIn, int NA, int NQ, int TPL, int S, int MW>
hipError_t hat_bstrip_go(const TIn* A, const float* Q, float* Ah, int64_t N, int n3, int p, hipStream_t s) {
  const size_t lds = red_bytes(TPL, S);
  dim3 grid((unsigned)((N + 32 * TPL - 1) / (32 * TPL)), (unsigned)((p + 31) / 32));
  hat_bstrip_kernel<TIn, NA, NQ, TPL, S, MW><<<grid, S * 64, lds, s>>>(A, Q, Ah, N, n3, p);
  return hipGetLastError();
}

template <typename TIn, int NA, int NQ>
hipError_t hat_bstrip_any(const TIn* A, const float* Q, float* Ah, int64_t N, int n3, int p, Cfg c,
                          hipStream_t s) {
#define PQ_B(V, W, MW)                                                                      \
  if (c.vec == V && c.waves == W && c.strip == MW)                                          \
    return hat_bstrip_go<TIn, NA, NQ, V, W, MW>(A, Q, Ah, N, n3, p, s);
  PQ_B(4, 2, 2) PQ_B(4, 4, 2) PQ_B(2, 2, 4) PQ_B(2, 4, 4) PQ_B(1, 4, 4) PQ_B(1, 8, 4)
#undef PQ_B
  return hipErrorInvalidValue;
}

// split-bfloat16 strip candidates (tubes per lane, waves, min waves per SIMD)
void bstrip_cands(int vmax, std::vector<Cfg>& v) {
  static const int t[][3] = {{4, 2, 2}, {4, 4, 2}, {2, 2, 4}, {2, 4, 4}, {1, 4, 4}, {1, 8, 4}};
  for (const auto& r : t)
    if (r[0] <= vmax) {
      Cfg c{r[0], r[1], 0};
      c.strip = r[2];
      v.push_back(c);
    }
}

template <int VEC, int S, typename TIn>
hipError_t proj_f32_go(const TIn* A, const float* Q, float* out, int64_t N, int n3, int p,
                       hipStream_t s) {
  const int ntiles = (n3 + 31) / 32;
  const size_t lds = (size_t)(ntiles * 32 + 16) * 33 * sizeof(float) + red_bytes(VEC, S + 1);
  static hipError_t attr = allow_lds(&proj_f32_kernel<VEC, S, TIn>, 160 * 1024);
  if (attr != hipSuccess) return attr;
  dim3 grid((unsigned)((N + 32 * VEC - 1) / (32 * VEC)));
  proj_f32_kernel<VEC, S, TIn><<<grid, S * 64, lds, s>>>(A, Q, out, N, n3, p);
  return hipGetLastError();
}

template <int VEC, int W>
hipError_t unhat_f32_go(const float* Ah, const float* Q, float* C, int64_t N, int n3, int p,
                        hipStream_t s) {
  const int64_t strips = (N + 32 * VEC - 1) / (32 * VEC);
  const int64_t wgs = (strips + W - 1) / W;
  const int ntiles = (n3 + 31) / 32;
  // enough workgroups to fill 256 CUs several times over
  int ysplit = (int)std::min<int64_t>(ntiles, std::max<int64_t>(1, (2048 + wgs - 1) / wgs));
  const size_t lds = (size_t)((p + 1) & ~1) * 32 * sizeof(float);
  dim3 grid((unsigned)wgs, (unsigned)ysplit);
  unhat_f32_kernel<VEC, W><<<grid, W * 64, lds, s>>>(Ah, Q, C, N, n3, p);
  return hipGetLastError();
}

// dispatch a (vec, waves) pair onto template instances
#define PQ_VW_DISPATCH(CFG, CALL)                                           \
  switch ((CFG).vec * 16 + (CFG).waves) {                                   \
    case 4 * 16 + 1: return CALL(4, 1);                                     \
    case 4 * 16 + 2: return CALL(4, 2);                                     \
    case 4 * 16 + 4: return CALL(4, 4);                                     \
    case 2 * 16 + 1: return CALL(2, 1);                                     \
    case 2 * 16 + 2: return CALL(2, 2);                                     \
    case 2 * 16 + 4: return CALL(2, 4);                                     \
    case 2 * 16 + 8: return CALL(2, 8);                                     \
    case 1 * 16 + 1: return CALL(1, 1);                                     \
    case 1 * 16 + 2: return CALL(1, 2);                                     \
    case 1 * 16 + 4: return CALL(1, 4);                                     \
    default: return CALL(1, 8);                                             \
  }

#define PQ_VW_DISPATCH_STRIPS(CFG, CALL)                                    \
  switch ((CFG).vec * 16 + (CFG).waves) {                                   \
    case 4 * 16 + 2: return CALL(4, 2);                                     \
    case 4 * 16 + 4: return CALL(4, 4);                                     \
    case 4 * 16 + 8: return CALL(4, 8);                                     \
    case 2 * 16 + 2: return CALL(2, 2);                                     \
    case 2 * 16 + 4: return CALL(2, 4);                                     \
    case 2 * 16 + 8: return CALL(2, 8);                                     \
    case 1 * 16 + 2: return CALL(1, 2);                                     \
    case 1 * 16 + 4: return CALL(1, 4);                                     \
    default: return CALL(1, 8);                                             \
  }

template <typename TIn, int NA, int NQ>
hipError_t hat_bf16_any(const TIn* A, const float* Q, float* Ah, int64_t N, int n3, int p, Cfg c,
                        hipStream_t s) {
#define PQ_CALL(V, W) hat_bf16_go<TIn, NA, NQ, V, W>(A, Q, Ah, N, n3, p, c.spw, s)
  PQ_VW_DISPATCH(c, PQ_CALL)
#undef PQ_CALL
}

template <typename TIn>
hipError_t hat_f32_any(const TIn* A, const float* Q, float* Ah, int64_t N, int n3, int p, Cfg c,
                       hipStream_t s) {
#define PQ_CALL(V, W) hat_f32_go<V, W, TIn>(A, Q, Ah, N, n3, p, c.spw, s)
  PQ_VW_DISPATCH(c, PQ_CALL)
#undef PQ_CALL
}

template <typename TIn>
hipError_t proj_f32_any(const TIn* A, const float* Q, float* out, int64_t N, int n3, int p, Cfg c,
                        hipStream_t s) {
#define PQ_CALL(V, W) proj_f32_go<V, W, TIn>(A, Q, out, N, n3, p, s)
  PQ_VW_DISPATCH(c, PQ_CALL)
#undef PQ_CALL
}

hipError_t unhat_f32_any(const float* Ah, const float* Q, float* C, int64_t N, int n3, int p, Cfg c,
                         hipStream_t s) {
#define PQ_CALL(V, W) unhat_f32_go<V, W>(Ah, Q, C, N, n3, p, s)
  PQ_VW_DISPATCH_STRIPS(c, PQ_CALL)
#undef PQ_CALL
}

}  // namespace

int xform_group_vec(const XformDesc& d) { return pick_vec(d.N, {d.in, d.out}, 4); }
int unhat_group_vec(const XformDesc& d) { return pick_vec(d.N, {d.in, d.out}, 4); }

void hat_group_tiles(const XformDesc& d, int desc, std::vector<XformTile>& tiles) {
  const int vec = xform_group_vec(d);
  const int64_t strips = (d.N + 32 * vec - 1) / (32 * vec);
  for (int y = 0; y < (d.p + 31) / 32; ++y)
    for (int64_t x = 0; x < strips; ++x) tiles.push_back(XformTile{x, desc, y});
}

void unhat_group_tiles(const XformDesc& d, int desc, std::vector<XformTile>& tiles) {
  const int vec = unhat_group_vec(d);
  const int64_t strips = (d.N + 32 * vec - 1) / (32 * vec);
  for (int64_t x = 0; x < (strips + 3) / 4; ++x) tiles.push_back(XformTile{x, desc, 0});
}

// the forward strip kernel's shapes that the autotuner picks most often for
// single transforms: four waves splitting the slices of a strip
hipError_t hat_grouped(const XformDesc* d, const XformTile* t, int ntiles, int vec, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (vec == 4)
    hat_grouped_kernel<4, 4, 2, 4><<<(unsigned)ntiles, 256, red_bytes(4, 4), s>>>(d, t);
  else if (vec == 2)
    hat_grouped_kernel<2, 4, 4, 4><<<(unsigned)ntiles, 256, red_bytes(2, 4), s>>>(d, t);
  else
    hat_grouped_kernel<1, 4, 4, 4><<<(unsigned)ntiles, 256, red_bytes(1, 4), s>>>(d, t);
  return hipGetLastError();
}

// The return transform's shapes per vector width, chosen by the autotuner
// per group (key: width and tile count): four waves with a strip each, at
// two or four waves per SIMD (the two-tube form needs more than 128
// registers with its Q entries double-buffered, and spills at four), with
// Q staged in LDS when the group's largest Q fits (q_bytes: its n3 rows of
// q_lds_stride(p) floats; 0: read from memory).
hipError_t unhat_grouped(const XformDesc* d, const XformTile* t, int ntiles, int vec, size_t q_bytes,
                         hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  const bool ql = q_bytes > 0 && q_bytes <= kQLdsMax;
  const std::string key = "unhatg/" + std::to_string(vec) + "/" + std::to_string(ntiles) + (ql ? "/q" : "");
  return tuned_launch(key, ql ? 4 : 2, ql ? 2 : 0, s, [&](int c) -> hipError_t {
    const unsigned g = (unsigned)ntiles;
    const size_t lds = c >= 2 ? q_bytes : 0;
    if (vec == 4) {
      if (c == 0) unhat_grouped_kernel<4, 4, 2, false><<<g, 256, 0, s>>>(d, t);
      else if (c == 1) unhat_grouped_kernel<4, 4, 1, false><<<g, 256, 0, s>>>(d, t);
      else if (c == 2) unhat_grouped_kernel<4, 4, 2, true><<<g, 256, lds, s>>>(d, t);
      else unhat_grouped_kernel<4, 4, 1, true><<<g, 256, lds, s>>>(d, t);
    } else if (vec == 2) {
      if (c == 0) unhat_grouped_kernel<2, 4, 2, false><<<g, 256, 0, s>>>(d, t);
      else if (c == 1) unhat_grouped_kernel<2, 4, 4, false><<<g, 256, 0, s>>>(d, t);
      else if (c == 2) unhat_grouped_kernel<2, 4, 2, true><<<g, 256, lds, s>>>(d, t);
      else unhat_grouped_kernel<2, 4, 4, true><<<g, 256, lds, s>>>(d, t);
    } else {
      if (c == 0) unhat_grouped_kernel<1, 4, 4, false><<<g, 256, 0, s>>>(d, t);
      else if (c == 1) unhat_grouped_kernel<1, 4, 2, false><<<g, 256, 0, s>>>(d, t);
      else if (c == 2) unhat_grouped_kernel<1, 4, 4, true><<<g, 256, lds, s>>>(d, t);
      else unhat_grouped_kernel<1, 4, 2, true><<<g, 256, lds, s>>>(d, t);
    }
    return hipGetLastError();
  });
}

size_t unhat_group_q_bytes(const XformDesc& d) { return sizeof(float) * (size_t)d.n3 * q_lds_stride(d.p); }

hipError_t hat_f32(const void* A, bool a_bf16, const float* Q, float* Ah, int64_t N, int n3, int p,
                   Prec prec, hipStream_t s) {
  const int vmax = a_bf16 ? std::min(pick_vec(N, {A}, 2), pick_vec(N, {Ah}, 4)) : pick_vec(N, {A, Ah}, 4);
  std::vector<Cfg> c;
  if (prec == Prec::Default) strip_cands(vmax, c);
  else bstrip_cands(vmax, c);
  const int nstrip = (int)c.size();
  for (const Cfg& g : cands(vmax, true)) c.push_back(g);
  const std::string key = key_of("hat", (int)prec, a_bf16, N, n3, p, vmax);
  const uint16_t* ab = static_cast<const uint16_t*>(A);
  const float* af = static_cast<const float*>(A);
  // untuned default: the strip kernel with two waves and four pairs per batch
  int dflt = nstrip;
  for (int i = 0; i < nstrip; ++i)
    if (c[i].vec == vmax && c[i].waves == (prec == Prec::Default ? 2 : 4) &&
        (prec != Prec::Default || c[i].spw == 4))
      dflt = i;
  if (dflt == nstrip) {
    std::vector<Cfg> rest(c.begin() + nstrip, c.end());
    dflt = nstrip + default_splitk(rest, N);
  }
  return tuned_launch(key, (int)c.size(), dflt, s, [&](int i) -> hipError_t {
    const Cfg g = c[i];
    if (g.strip) {
      if (prec == Prec::Default) {
        if (a_bf16) return hat_strip_any<uint16_t>(ab, Q, Ah, N, n3, p, g, s);
        return hat_strip_any<float>(af, Q, Ah, N, n3, p, g, s);
      }
      if (a_bf16) {
        if (prec == Prec::BF16) return hat_bstrip_any<uint16_t, 1, 1>(ab, Q, Ah, N, n3, p, g, s);
        return hat_bstrip_any<uint16_t, 1, 3>(ab, Q, Ah, N, n3, p, g, s);
      }
      switch (prec) {
        case Prec::BF16: return hat_bstrip_any<float, 1, 1>(af, Q, Ah, N, n3, p, g, s);
        case Prec::BF16x3: return hat_bstrip_any<float, 2, 2>(af, Q, Ah, N, n3, p, g, s);
        default: return hat_bstrip_any<float, 3, 3>(af, Q, Ah, N, n3, p, g, s);
      }
    }
    if (a_bf16) {
      switch (prec) {
        case Prec::Default: return hat_f32_any<uint16_t>(ab, Q, Ah, N, n3, p, g, s);
        case Prec::BF16: return hat_bf16_any<uint16_t, 1, 1>(ab, Q, Ah, N, n3, p, g, s);
        default: return hat_bf16_any<uint16_t, 1, 3>(ab, Q, Ah, N, n3, p, g, s);
      }
    }
    switch (prec) {
      case Prec::Default: return hat_f32_any<float>(af, Q, Ah, N, n3, p, g, s);
      case Prec::BF16: return hat_bf16_any<float, 1, 1>(af, Q, Ah, N, n3, p, g, s);
      case Prec::BF16x3: return hat_bf16_any<float, 2, 2>(af, Q, Ah, N, n3, p, g, s);
      default: return hat_bf16_any<float, 3, 3>(af, Q, Ah, N, n3, p, g, s);
    }
  });
}

hipError_t unhat_f32(const float* Ah, const float* Q, float* C, int64_t N, int n3, int p, Prec prec,
                     hipStream_t s) {
  const int vmax = pick_vec(N, {Ah, C}, 4);
  // strip kernels (p <= 32) in the requested precision, then the older
  // LDS-staged float32 kernels
  std::vector<Cfg> c;
  if (p <= 32) unhat_strip_cands(vmax, c);
  const int nstrip = (int)c.size();
  // the float32 strip shapes with Q in LDS (also timed by the compensated
  // modes, like the float32 strips below)
  std::vector<Cfg> ql;
  if (p <= 32 && (prec == Prec::Default || prec == Prec::BF16x3 || prec == Prec::BF16x6))
    unhat_strip_ql_cands(vmax, n3, p, ql);
  // the compensated modes also time the float32 kernels (strip and
  // LDS-staged): the return transform is bound by its float32 writes, and
  // float32 products are at least as accurate as the split ones
  const bool comp = prec == Prec::BF16x3 || prec == Prec::BF16x6;
  if (comp)
    for (int i = 0; i < nstrip; ++i) {
      Cfg g = c[(size_t)i];
      g.f32 = true;
      c.push_back(g);
    }
  for (const Cfg& g : ql) c.push_back(g);
  // (p > 32: the split forms are not built for this width)
  if (prec == Prec::Default || comp || nstrip == 0)
    for (const Cfg& g : cands(vmax, false)) c.push_back(g);
  int dflt = 0;
  if (nstrip == 0) dflt = default_strips(c, N);
  return tuned_launch(key_of("unhat", (int)prec, 0, N, n3, p, vmax), (int)c.size(), dflt, s,
                      [&](int i) -> hipError_t {
                        const Cfg& g = c[i];
                        if (!g.strip) return unhat_f32_any(Ah, Q, C, N, n3, p, g, s);
                        if (g.f32) return unhat_strip_any<0, 0>(Ah, Q, C, N, n3, p, g, s);
                        switch (prec) {
                          case Prec::BF16: return unhat_strip_any<1, 1>(Ah, Q, C, N, n3, p, g, s);
                          case Prec::BF16x3: return unhat_strip_any<2, 2>(Ah, Q, C, N, n3, p, g, s);
                          case Prec::BF16x6: return unhat_strip_any<3, 3>(Ah, Q, C, N, n3, p, g, s);
                          default: return unhat_strip_any<0, 0>(Ah, Q, C, N, n3, p, g, s);
                        }
                      });
}

bool proj_fused_ok(int n3, int p) { return p <= 32 && n3 <= 480; }

hipError_t proj_fused_f32(const void* A, bool a_bf16, const float* Q, float* out, int64_t N, int n3,
                          int p, Prec prec, hipStream_t s) {
  (void)prec;  // the fused projection runs on float32 MFMA in every mode
  const int vmax = a_bf16 ? std::min(pick_vec(N, {A}, 2), pick_vec(N, {out}, 4))
                          : pick_vec(N, {A, out}, 4);
  std::vector<Cfg> c;
  for (const Cfg& g : cands(vmax, true))
    if (g.spw == 1) c.push_back(g);  // the projection stages all of Q once per strip
  return tuned_launch(key_of("proj", 0, a_bf16, N, n3, p, vmax), (int)c.size(), default_splitk(c, N), s,
                      [&](int i) -> hipError_t {
                        if (a_bf16)
                          return proj_f32_any<uint16_t>(static_cast<const uint16_t*>(A), Q, out, N,
                                                        n3, p, c[i], s);
                        return proj_f32_any<float>(static_cast<const float*>(A), Q, out, N, n3, p,
                                                   c[i], s);
                      });
}

template <typename TA>
hipError_t hat64_launch(const TA* A, const double* Q, double* Ah, int64_t N, int n3, int p, hipStream_t s) {
  const unsigned gx = (unsigned)((N + 63) / 64);
  if (p <= 8) {
    hat64_kernel<TA, 8><<<dim3(gx, 1), 256, 0, s>>>(A, Q, Ah, N, n3, p);
  } else if (p <= 16) {
    hat64_kernel<TA, 16><<<dim3(gx, 1), 256, 0, s>>>(A, Q, Ah, N, n3, p);
  } else if (p <= 24) {
    hat64_kernel<TA, 24><<<dim3(gx, 1), 256, 0, s>>>(A, Q, Ah, N, n3, p);
  } else {
    hat64_kernel<TA, 32><<<dim3(gx, (unsigned)((p + 31) / 32)), 256, 0, s>>>(A, Q, Ah, N, n3, p);
  }
  return hipGetLastError();
}

hipError_t hat_f64(const double* A, const double* Q, double* Ah, int64_t N, int n3, int p,
                   hipStream_t s) {
  return hat64_launch(A, Q, Ah, N, n3, p, s);
}

hipError_t hat_f64_wide(const float* A, const double* Q, double* Ah, int64_t N, int n3, int p, hipStream_t s) {
  return hat64_launch(A, Q, Ah, N, n3, p, s);
}

hipError_t unhat_f64(const double* Ah, const double* Q, double* C, int64_t N, int n3, int p,
                     hipStream_t s) {
  const dim3 grid((unsigned)((N + 255) / 256), (unsigned)((n3 + kUnhat64Rows - 1) / kUnhat64Rows));
  unhat64_kernel<<<grid, 256, 0, s>>>(Ah, Q, C, N, n3, p);
  return hipGetLastError();
}

}  // namespace pq
