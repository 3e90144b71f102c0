// Facewise truncated SVD of the transform-domain faces (Alg. 4.1 step 3) by
// one-sided (Hestenes) Jacobi.
//
// Each face contributes nv = min(n1, n2) vectors of length L = max(n1, n2)
// (its columns when n1 >= n2, its rows otherwise).  A sweep visits every pair
// once in round-robin order: nv - 1 rounds of nv/2 disjoint pairs, so the
// pairs of a round rotate independently, one pair per wave.  For a pair the
// wave forms alpha = |a|^2, beta = |b|^2, gamma = a.b with float64
// accumulation and 64-lane shuffle reductions, computes the rotation that
// zeroes gamma in float64, and applies it.  A face has converged after a
// sweep in which no pair had |gamma| > tol sqrt(alpha beta).  Converged
// vectors are mutually orthogonal; their norms are the singular values and,
// normalised, they are the singular vectors of their side.
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace pq {
namespace {

constexpr int kJacobiThreads = 1024;

template <typename T>
__global__ __launch_bounds__(kJacobiThreads) void jacobi_kernel(T* __restrict__ W, int nv, int L,
                                                                int max_sweeps, double tol,
                                                                int* __restrict__ sweeps_used) {
  constexpr int NW = kJacobiThreads / 64;
  __shared__ int rotated;
  const int face = blockIdx.x;
  T* Wf = W + (int64_t)face * nv * L;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nvp = nv + (nv & 1);  // with nv odd, index nv is a bye
  const int npairs = nvp / 2;
  int sweep = 0;
  bool converged = false;
  while (sweep < max_sweeps) {
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < nvp - 1; ++round) {
      for (int pi = wave; pi < npairs; pi += NW) {
        int a, b;
        if (pi == 0) {
          a = nvp - 1;
          b = round;
        } else {
          a = (round + pi) % (nvp - 1);
          b = (round - pi + nvp - 1) % (nvp - 1);
        }
        if (a >= nv || b >= nv) continue;
        T* va = Wf + (int64_t)a * L;
        T* vb = Wf + (int64_t)b * L;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int e = lane; e < L; e += 64) {
          const double x = va[e], y = vb[e];
          al = fma(x, x, al);
          be = fma(y, y, be);
          ga = fma(x, y, ga);
        }
        al = wave_sum(al);
        be = wave_sum(be);
        ga = wave_sum(ga);
        if (ga != 0.0 && fabs(ga) > tol * sqrt(al) * sqrt(be)) {
          const double zeta = (be - al) / (2.0 * ga);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t);
          const double s = c * t;
          for (int e = lane; e < L; e += 64) {
            const double x = va[e], y = vb[e];
            va[e] = static_cast<T>(c * x - s * y);
            vb[e] = static_cast<T>(s * x + c * y);
          }
          if (lane == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    ++sweep;
    const int any = rotated;
    __syncthreads();
    if (!any) {
      converged = true;
      break;
    }
  }
  if (threadIdx.x == 0) sweeps_used[face] = converged ? sweep : max_sweeps + 1;
}

// W face l (nv x L, vector-major) <- transpose of Ah face l (n1 x n2 column
// major), i.e. vector i = row i.  32x32 tiles through LDS.
template <typename T>
__global__ __launch_bounds__(256) void transpose_faces_kernel(const T* __restrict__ Ah,
                                                              T* __restrict__ W, int n1, int n2) {
  __shared__ T tile[32][33];
  const int l = blockIdx.z;
  const int i0 = blockIdx.x * 32, j0 = blockIdx.y * 32;
  const T* src = Ah + (int64_t)l * n1 * n2;
  T* dst = W + (int64_t)l * n1 * n2;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int i = i0 + tx, j = j0 + r;
    if (i < n1 && j < n2) tile[r][tx] = src[i + (int64_t)j * n1];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = i0 + r, j = j0 + tx;
    if (i < n1 && j < n2) dst[j + (int64_t)i * n2] = tile[tx][r];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void finalize_kernel(const T* __restrict__ W, int nv, int L, int k,
                                                       T* __restrict__ F, T* __restrict__ s_out,
                                                       T* __restrict__ inv_s) {
  extern __shared__ double sig[];  // nv doubles, then k ints
  int* order = reinterpret_cast<int*>(sig + nv);
  const int face = blockIdx.x;
  const T* Wf = W + (int64_t)face * nv * L;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = wave; j < nv; j += 4) {
    double acc = 0.0;
    for (int e = lane; e < L; e += 64) {
      const double x = Wf[(int64_t)j * L + e];
      acc = fma(x, x, acc);
    }
    acc = wave_sum(acc);
    if (lane == 0) sig[j] = sqrt(acc);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < nv; j += 256) {
    const double v = sig[j];
    int r = 0;
    for (int i = 0; i < nv; ++i) r += (sig[i] > v) || (sig[i] == v && i < j);
    if (r < k) order[r] = j;
  }
  __syncthreads();
  for (int r = wave; r < k; r += 4) {
    const int j = order[r];
    const double v = sig[j];
    const double inv = v > 0.0 ? 1.0 / v : 0.0;
    if (lane == 0) {
      s_out[(int64_t)face * k + r] = static_cast<T>(v);
      inv_s[(int64_t)face * k + r] = static_cast<T>(inv);
    }
    T* dst = F + ((int64_t)face * k + r) * L;
    for (int e = lane; e < L; e += 64) dst[e] = static_cast<T>(inv * (double)Wf[(int64_t)j * L + e]);
  }
}

template <typename T>
hipError_t prep(const T* Ah, T* W, int n1, int n2, int p, hipStream_t s) {
  if (n1 >= n2) {
    return hipMemcpyAsync(W, Ah, sizeof(T) * (size_t)n1 * n2 * p, hipMemcpyDeviceToDevice, s);
  }
  dim3 grid((unsigned)((n1 + 31) / 32), (unsigned)((n2 + 31) / 32), (unsigned)p);
  transpose_faces_kernel<T><<<grid, 256, 0, s>>>(Ah, W, n1, n2);
  return hipGetLastError();
}

template <typename T>
hipError_t sweeps(T* W, int p, int nv, int L, int max_sweeps, double tol, int* used, hipStream_t s) {
  jacobi_kernel<T><<<p, kJacobiThreads, 0, s>>>(W, nv, L, max_sweeps, tol, used);
  return hipGetLastError();
}

template <typename T>
hipError_t finalize(const T* W, int p, int nv, int L, int k, T* F, T* s_out, T* inv_s,
                    hipStream_t s) {
  const size_t lds = sizeof(double) * (size_t)nv + sizeof(int) * (size_t)k;
  finalize_kernel<T><<<p, 256, lds, s>>>(W, nv, L, k, F, s_out, inv_s);
  return hipGetLastError();
}

__global__ void info_kernel(const int* __restrict__ used, int p, int max_sweeps, int* __restrict__ info) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int mx = 0, bad = 0;
  for (int l = 0; l < p; ++l) {
    const int u = used[l];
    if (u > max_sweeps) {
      ++bad;
      mx = max(mx, max_sweeps);
    } else {
      mx = max(mx, u);
    }
  }
  int total = 0;
  for (int l = 0; l < p; ++l) total += min(used[l], max_sweeps);
  info[0] = mx;
  info[1] = bad;
  info[2] = total;
}

}  // namespace

hipError_t jacobi_prep_f32(const float* Ah, float* W, int n1, int n2, int p, hipStream_t s) {
  return prep<float>(Ah, W, n1, n2, p, s);
}
hipError_t jacobi_prep_f64(const double* Ah, double* W, int n1, int n2, int p, hipStream_t s) {
  return prep<double>(Ah, W, n1, n2, p, s);
}
hipError_t jacobi_sweeps_f32(float* W, int p, int nv, int L, int max_sweeps, double tol, int* used,
                             hipStream_t s) {
  return sweeps<float>(W, p, nv, L, max_sweeps, tol, used, s);
}
hipError_t jacobi_sweeps_f64(double* W, int p, int nv, int L, int max_sweeps, double tol, int* used,
                             hipStream_t s) {
  return sweeps<double>(W, p, nv, L, max_sweeps, tol, used, s);
}
hipError_t jacobi_finalize_f32(const float* W, int p, int nv, int L, int k, float* F, float* s_out,
                               float* inv_s, hipStream_t s) {
  return finalize<float>(W, p, nv, L, k, F, s_out, inv_s, s);
}
hipError_t jacobi_finalize_f64(const double* W, int p, int nv, int L, int k, double* F,
                               double* s_out, double* inv_s, hipStream_t s) {
  return finalize<double>(W, p, nv, L, k, F, s_out, inv_s, s);
}
hipError_t jacobi_info(const int* used, int p, int max_sweeps, int* info, hipStream_t s) {
  info_kernel<<<1, 64, 0, s>>>(used, p, max_sweeps, info);
  return hipGetLastError();
}

}  // namespace pq
