// Elementwise steps of the adjoint of the truncated tSVDQ (the map
// (A, Q) -> (A_k, s) of Alg. 4.1 and Thm. 4.2).  The products around them
// run on the facewise GEMM; these kernels form the resolvent coefficients and
// assemble the operands of those products.
//
// Per face, with the Jacobi side M_t (L x S: the face itself when n1 >= n2,
// its transpose otherwise), U (L x S) its left singular vectors in
// descending order of sigma, lambda = sigma^2, K the first k of them, D the
// rest, and Yall = M_t^T U (S x S, column j = sigma_j v_j, so that
// M_t = U Yall^T), Y its first k columns, H = G_t^T U_K:
//   Ra = G_t Y                                    L x k
//   Ba = U^T Ra,  Bb = Yall^T H                   S x k
//   E_jc  = -Ba_jc / lambda_c                                 j in K
//         = (Ba_jc lambda_j / lambda_c + Bb_jc) / (lambda_c - lambda_j)   j in D
//   Ep_jc = 0 (j in K),  (Ba_jc + Bb_jc) / (lambda_c - lambda_j) (j in D)
//   X  = Ra diag(1/lambda) + U E
//   N  = H + Yall Ep + Y diag(sbar / sigma)
//   dM_t = [U_K X] [N Y]^T.
// X is the resolvent (lambda_c I - M_t M_t^T)^+ applied to the part of
// G_t Y + M_t H outside span(U_K) (the derivative of the spectral
// projector); M_t H lies in span(U), so its coefficients come from Yall
// instead of a projection, and M_t^T X = Yall Ep exactly (M_t^T annihilates
// the complement of span(U)).  Neither step then divides rounding noise of
// size sigma_max by lambda_c.
#include "common.hpp"
#include "internal.hpp"

namespace pq {
namespace {

__global__ __launch_bounds__(256) void narrow_kernel(const double* __restrict__ x, float* __restrict__ y,
                                                     int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}

// one workgroup per face; cnt[face] = pairs (kept c, discarded j) whose
// relative gap |lambda_c - lambda_j| <= gap_tol lambda_c (coupling dropped)
template <typename T>
__global__ __launch_bounds__(256) void coef_kernel(const T* __restrict__ Ba, const T* __restrict__ Bb,
                                                   const double* __restrict__ sig, int nv, int k, double gap_tol,
                                                   T* __restrict__ E, T* __restrict__ Ep, int* __restrict__ cnt) {
  __shared__ int bad_total;
  const int face = blockIdx.x;
  if (threadIdx.x == 0) bad_total = 0;
  __syncthreads();
  const double* sg = sig + (int64_t)face * nv;
  const int64_t off = (int64_t)face * nv * k;
  int bad = 0;
  for (int idx = threadIdx.x; idx < nv * k; idx += 256) {
    const int j = idx % nv, c = idx / nv;
    const double lc = sg[c] * sg[c], lj = sg[j] * sg[j];
    const double ba = (double)Ba[off + idx], bb = (double)Bb[off + idx];
    double v = 0.0, vp = 0.0;
    if (lc > 0.0) {
      if (j < k) {
        v = -ba / lc;
      } else {
        const double d = lc - lj;
        if (fabs(d) <= gap_tol * lc) {
          ++bad;
          v = -ba / lc;  // the tied pair's coupling dropped
        } else {
          v = (ba * (lj / lc) + bb) / d;
          vp = (ba + bb) / d;
        }
      }
    }
    E[off + idx] = static_cast<T>(v);
    Ep[off + idx] = static_cast<T>(vp);
  }
  if (bad) atomicAdd(&bad_total, bad);
  __syncthreads();
  if (threadIdx.x == 0) cnt[face] = bad_total;
}

// LHS (L x 2k per face) = [U_K, R diag(1/lambda) + UE]; R == nullptr: X = 0
template <typename T>
__global__ __launch_bounds__(256) void xcombine_kernel(const T* __restrict__ R, const T* __restrict__ UE,
                                                       const T* __restrict__ U, const double* __restrict__ sig,
                                                       int L, int nv, int k, int64_t total, T* __restrict__ LHS) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= total) return;
  const int64_t per = (int64_t)L * 2 * k;
  const int face = (int)(idx / per);
  const int64_t r = idx - (int64_t)face * per;
  const int c2 = (int)(r / L), i = (int)(r - (int64_t)c2 * L);
  T v;
  if (c2 < k) {
    v = U[(int64_t)face * L * nv + (int64_t)c2 * L + i];
  } else {
    const int c = c2 - k;
    const double s = sig[(int64_t)face * nv + c];
    const double lc = s * s;
    const int64_t o = (int64_t)face * L * k + (int64_t)c * L + i;
    v = (R && lc > 0.0) ? static_cast<T>((double)R[o] / lc + (double)UE[o]) : T(0);
  }
  LHS[idx] = v;
}

// RHS (S x 2k per face) = [H + P1 + Y diag(sbar / sigma), Y]; null terms are
// 0; Y is the first k columns of Yall (S x S per face)
template <typename T, typename TS>
__global__ __launch_bounds__(256) void ncombine_kernel(const T* __restrict__ H, const T* __restrict__ P1,
                                                       const T* __restrict__ Y, const TS* __restrict__ sbar,
                                                       const double* __restrict__ sig, int S, int nv, int k,
                                                       int64_t total, T* __restrict__ RHS) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= total) return;
  const int64_t per = (int64_t)S * 2 * k;
  const int face = (int)(idx / per);
  const int64_t r = idx - (int64_t)face * per;
  const int c2 = (int)(r / S), i = (int)(r - (int64_t)c2 * S);
  const int c = c2 < k ? c2 : c2 - k;
  const int64_t o = (int64_t)face * S * k + (int64_t)c * S + i;
  const double y = (double)Y[(int64_t)face * S * S + (int64_t)c * S + i];
  double v;
  if (c2 >= k) {
    v = y;
  } else {
    v = 0.0;
    if (H) v += (double)H[o];
    if (P1) v += (double)P1[o];
    const double s = sig[(int64_t)face * nv + c];
    if (sbar && s > 0.0) v += y * (double)sbar[(int64_t)face * k + c] / s;
  }
  RHS[idx] = static_cast<T>(v);
}

__global__ void count_kernel(const int* __restrict__ cnt, int p, int* __restrict__ out) {
  if (threadIdx.x != 0) return;
  int t = 0;
  for (int f = 0; f < p; ++f) t += cnt[f];
  out[0] = t;
}

unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t grad_narrow(const double* x, float* y, int64_t n, hipStream_t s) {
  narrow_kernel<<<blocks(n), 256, 0, s>>>(x, y, n);
  return hipGetLastError();
}

hipError_t grad_coef(const void* Ba, const void* Bb, const double* sig, int p, int nv, int k, double gap_tol,
                     void* E, void* Ep, int* cnt, bool f64, hipStream_t s) {
  if (f64)
    coef_kernel<double><<<p, 256, 0, s>>>(static_cast<const double*>(Ba), static_cast<const double*>(Bb), sig, nv,
                                          k, gap_tol, static_cast<double*>(E), static_cast<double*>(Ep), cnt);
  else
    coef_kernel<float><<<p, 256, 0, s>>>(static_cast<const float*>(Ba), static_cast<const float*>(Bb), sig, nv, k,
                                         gap_tol, static_cast<float*>(E), static_cast<float*>(Ep), cnt);
  return hipGetLastError();
}

hipError_t grad_xcombine(const void* R, const void* UE, const void* U, const double* sig, int p, int L, int nv, int k,
                         void* LHS, bool f64, hipStream_t s) {
  const int64_t total = (int64_t)p * L * 2 * k;
  if (f64)
    xcombine_kernel<double><<<blocks(total), 256, 0, s>>>(static_cast<const double*>(R),
                                                          static_cast<const double*>(UE),
                                                          static_cast<const double*>(U), sig, L, nv, k, total,
                                                          static_cast<double*>(LHS));
  else
    xcombine_kernel<float><<<blocks(total), 256, 0, s>>>(static_cast<const float*>(R),
                                                         static_cast<const float*>(UE),
                                                         static_cast<const float*>(U), sig, L, nv, k, total,
                                                         static_cast<float*>(LHS));
  return hipGetLastError();
}

hipError_t grad_ncombine(const void* H, const void* P1, const void* Y, const void* sbar, const double* sig, int p,
                         int S, int nv, int k, void* RHS, bool f64, bool sbar_f32, hipStream_t s) {
  const int64_t total = (int64_t)p * S * 2 * k;
  if (f64 && sbar_f32)
    ncombine_kernel<double, float><<<blocks(total), 256, 0, s>>>(
        static_cast<const double*>(H), static_cast<const double*>(P1), static_cast<const double*>(Y),
        static_cast<const float*>(sbar), sig, S, nv, k, total, static_cast<double*>(RHS));
  else if (f64)
    ncombine_kernel<double, double><<<blocks(total), 256, 0, s>>>(
        static_cast<const double*>(H), static_cast<const double*>(P1), static_cast<const double*>(Y),
        static_cast<const double*>(sbar), sig, S, nv, k, total, static_cast<double*>(RHS));
  else
    ncombine_kernel<float, float><<<blocks(total), 256, 0, s>>>(
        static_cast<const float*>(H), static_cast<const float*>(P1), static_cast<const float*>(Y),
        static_cast<const float*>(sbar), sig, S, nv, k, total, static_cast<float*>(RHS));
  return hipGetLastError();
}

hipError_t grad_count(const int* cnt, int p, int* out, hipStream_t s) {
  count_kernel<<<1, 64, 0, s>>>(cnt, p, out);
  return hipGetLastError();
}

}  // namespace pq
