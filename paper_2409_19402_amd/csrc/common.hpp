// Device-side helpers shared by the projprod kernels (gfx950 / CDNA4).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace pq {

constexpr int kWave = 64;

// bfloat16 bit pattern -> float32 (exact).
__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

// float32 -> bfloat16 bit pattern, round to nearest, ties to even.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return static_cast<uint16_t>((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

template <typename T> struct Loader;
template <> struct Loader<float> {
  static __device__ __forceinline__ float ld(const float* p) { return *p; }
};
template <> struct Loader<double> {
  static __device__ __forceinline__ double ld(const double* p) { return *p; }
};
template <> struct Loader<uint16_t> {
  static __device__ __forceinline__ float ld(const uint16_t* p) { return bf16_to_f32(*p); }
};

// Load VEC consecutive elements (as float) starting at p; p is VEC-aligned.
template <int VEC, typename TIn>
__device__ __forceinline__ void load_vec(const TIn* __restrict__ p, float (&v)[VEC]);

template <>
__device__ __forceinline__ void load_vec<1, float>(const float* __restrict__ p, float (&v)[1]) { v[0] = *p; }
template <>
__device__ __forceinline__ void load_vec<2, float>(const float* __restrict__ p, float (&v)[2]) {
  float2 t = *reinterpret_cast<const float2*>(p);
  v[0] = t.x; v[1] = t.y;
}
template <>
__device__ __forceinline__ void load_vec<4, float>(const float* __restrict__ p, float (&v)[4]) {
  float4 t = *reinterpret_cast<const float4*>(p);
  v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
}
template <>
__device__ __forceinline__ void load_vec<1, uint16_t>(const uint16_t* __restrict__ p, float (&v)[1]) {
  v[0] = bf16_to_f32(*p);
}
template <>
__device__ __forceinline__ void load_vec<2, uint16_t>(const uint16_t* __restrict__ p, float (&v)[2]) {
  uint32_t u = *reinterpret_cast<const uint32_t*>(p);
  v[0] = __uint_as_float(u << 16); v[1] = __uint_as_float(u & 0xffff0000u);
}
template <>
__device__ __forceinline__ void load_vec<4, uint16_t>(const uint16_t* __restrict__ p, float (&v)[4]) {
  uint2 u = *reinterpret_cast<const uint2*>(p);
  v[0] = __uint_as_float(u.x << 16); v[1] = __uint_as_float(u.x & 0xffff0000u);
  v[2] = __uint_as_float(u.y << 16); v[3] = __uint_as_float(u.y & 0xffff0000u);
}

template <int VEC>
__device__ __forceinline__ void store_vec(float* __restrict__ p, const float (&v)[VEC]) {
  if constexpr (VEC == 1) { *p = v[0]; }
  else if constexpr (VEC == 2) { *reinterpret_cast<float2*>(p) = make_float2(v[0], v[1]); }
  else { *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]); }
}

// Sum over the 64 lanes of a wave (every lane gets the total).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
// Cross-lane move of a double with a DPP control (both 32-bit halves moved
// alike); lanes of rows left out of ROW_MASK get 0.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes on the VALU (DPP, no LDS traffic), returned as a
// wave-uniform value.  Lanes 0-15 form row 0 and so on:
//   quad_perm [1,0,3,2], [2,3,0,1]  -> every lane holds its quad's sum
//   row_half_mirror, row_mirror     -> every lane holds its row's sum
//   row_bcast:15 into rows 1 and 3  -> rows 1, 3 hold rows 0+1, 2+3
//   row_bcast:31 into rows 2 and 3  -> row 3 holds the total; read lane 63.
__device__ __forceinline__ double wave_total(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x141>(v);
  v += dpp_f64<0x140>(v);
  v += dpp_f64<0x142, 0xA>(v);
  v += dpp_f64<0x143, 0xC>(v);
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}

// ---- split-bfloat16 arithmetic ------------------------------------------------
// x = x0 + x1 (+ x2) with each part a bfloat16 (round to nearest even by the
// hardware pack conversion) and the products of parts accumulated in float32
// on the bfloat16 MFMA; Split<NA, NB> lists the part products of a mode,
// smallest terms first.
typedef float f32x2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  f32x2v v = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2v));
}
__device__ __forceinline__ float bf16_lo(uint32_t d) { return __uint_as_float(d << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t d) { return __uint_as_float(d & 0xffff0000u); }

template <int NA, int NQ>
struct Split;
// product list (a-part, q-part) per mode, smallest terms first
template <> struct Split<1, 1> { static constexpr int n = 1; static constexpr int a[1] = {0}; static constexpr int q[1] = {0}; };
template <> struct Split<2, 2> { static constexpr int n = 3; static constexpr int a[3] = {1, 0, 0}; static constexpr int q[3] = {0, 1, 0}; };
template <> struct Split<3, 3> { static constexpr int n = 6; static constexpr int a[6] = {2, 1, 0, 1, 0, 0}; static constexpr int q[6] = {0, 1, 2, 0, 1, 0}; };
template <> struct Split<1, 3> { static constexpr int n = 3; static constexpr int a[3] = {0, 0, 0}; static constexpr int q[3] = {2, 1, 0}; };

// split float pairs into NP bfloat16 parts, packed: out[i] holds part i
template <int NP>
__device__ __forceinline__ void split_pack(float x, float y, uint32_t (&out)[NP]) {
  out[0] = pack_bf16(x, y);
  if constexpr (NP > 1) {
    const float rx = x - bf16_lo(out[0]), ry = y - bf16_hi(out[0]);
    out[1] = pack_bf16(rx, ry);
    if constexpr (NP > 2) out[2] = pack_bf16(rx - bf16_lo(out[1]), ry - bf16_hi(out[1]));
  }
}

}  // namespace pq
