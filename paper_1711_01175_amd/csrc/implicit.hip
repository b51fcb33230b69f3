// Locally implicit step (HIP, gfx950): the theta scheme of the DG operator
// solved by iHDG-II (Sec. 3, eq. iHDGlocal and iHDGtrace, Algorithm 1).
//
// The interface state is linear in both sides' traces, so the local equation
// of element k with the neighbours' previous iterate is the dense system
// B_k c_k = rhs_k, B_k = I - theta dt A_k (A_k: the operator restricted to
// the element's own 9 Np unknowns).  Written as an update of the previous
// iterate, one iHDG-II iteration over all elements is
//     q <- q + B_k^-1 (b + theta dt L(q) - q)
// with L(q) the full operator (neighbours at the previous iterate) and b the
// fixed part of the step.  Set-up probes A_k through the explicit operator
// kernels (one colour class of pairwise non-adjacent elements at a time) and
// inverts B_k in FP64; every iteration is one operator evaluation plus one
// batched matrix-vector product, an HBM stream of the stored inverses.
#include <hip/hip_runtime.h>

#include "dev.hpp"
#include "impdev.hpp"
#include "kcommon.hpp"

namespace ewdg {

template <int N>
struct ImpSz {
  static constexpr int Np = Sz<N>::Np;
  static constexpr int NV = 9 * Np;
  static constexpr int n = (NV + 15) / 16 * 16;
  // rows per thread of the matrix-vector product and threads per element
  static constexpr int RPT = (NV + 1023) / 1024;
  static constexpr int TPB = ((NV + RPT - 1) / RPT + 63) / 64 * 64;
};

__global__ void k_imp_identity(double* __restrict__ W, int64_t total, int n) {
  const int64_t nn = static_cast<int64_t>(n) * n;
  for (int64_t x = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; x < total;
       x += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t e = x % nn;
    W[x] = (e / n == e % n) ? 1.0 : 0.0;
  }
}

template <typename T>
__global__ void k_imp_zero(T* __restrict__ x, int64_t count) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < count;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    x[i] = T(0);
}

template <typename T>
__global__ void k_imp_probe(T* __restrict__ q, const int32_t* __restrict__ members, int cnt, int nv, int j_off,
                            int j_on) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= cnt) return;
  const int64_t base = static_cast<int64_t>(members[x]) * nv;
  if (j_off >= 0) q[base + j_off] = T(0);
  if (j_on >= 0) q[base + j_on] = T(1);
}

template <typename T>
__global__ void k_imp_gather(const T* __restrict__ L, double* __restrict__ W, const int32_t* __restrict__ members,
                             int nv, int n, int j, double thdt) {
  const int64_t k = members[blockIdx.x];
  double* row = W + (k * n + j) * n;
  const T* l = L + k * nv;
  for (int i = threadIdx.x; i < nv; i += blockDim.x)
    row[i] = (i == j ? 1.0 : 0.0) - thdt * static_cast<double>(l[i]);
}

// In-place block Gauss-Jordan inverse of one n x n FP64 matrix per
// workgroup.  For each 16-wide pivot block P:
//   D = A_PP^-1;  A_Pj <- D A_Pj (j not in P);  A_ij <- A_ij - A_iP A_Pj (i, j not in P);
//   A_iP <- -A_iP D (i not in P);  A_PP <- D.
// No row exchanges: B = I - theta dt A_k has a positive definite symmetric
// part in the energy inner product (the upwind operator is dissipative), so
// the pivots stay away from zero; a vanishing or non-finite pivot sets *flag.
template <int N>
__global__ __launch_bounds__(256) void k_imp_invert(double* __restrict__ W, int32_t* __restrict__ flag) {
  constexpr int n = ImpSz<N>::n, GB = 16;
  __shared__ double D[GB * GB];
  __shared__ double R[GB * n];
  double* A = W + static_cast<int64_t>(blockIdx.x) * n * n;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r = tid >> 4, c = tid & 15;
#pragma unroll 1
  for (int p = 0; p < n; p += GB) {
    D[tid] = A[static_cast<int64_t>(p + r) * n + p + c];
    __syncthreads();
#pragma unroll 1
    for (int m = 0; m < GB; ++m) {
      const double piv = D[m * GB + m];
      const double drm = D[r * GB + m], dmc = D[m * GB + c];
      double v = D[tid];
      if (r == m) v = (c == m) ? 1.0 / piv : v / piv;
      else v = (c == m) ? -drm / piv : v - drm * dmc / piv;
      if (tid == 0 && !(fabs(piv) > 1e-300 && fabs(piv) < 1e300)) flag[0] = 1;
      __syncthreads();
      D[tid] = v;
      __syncthreads();
    }
    // row panel through LDS
#pragma unroll 1
    for (int j = tid; j < n; j += 256) {
      // keeps the 256 values of D in LDS rather than hoisted into registers
      asm volatile("" ::: "memory");
      if (j >= p && j < p + GB) {
#pragma unroll
        for (int rr = 0; rr < GB; ++rr) R[rr * n + j] = D[rr * GB + (j - p)];
      } else {
        double a[GB];
#pragma unroll
        for (int m = 0; m < GB; ++m) a[m] = A[static_cast<int64_t>(p + m) * n + j];
#pragma unroll
        for (int rr = 0; rr < GB; ++rr) {
          double s = 0.0;
#pragma unroll
          for (int m = 0; m < GB; ++m) s += D[rr * GB + m] * a[m];
          R[rr * n + j] = s;
        }
      }
    }
    __syncthreads();
#pragma unroll 1
    for (int x = tid; x < GB * n; x += 256) A[static_cast<int64_t>(p + x / n) * n + x % n] = R[x];
    // the other rows: wave w takes rows w, w + 4, ...; lanes run along the row
#pragma unroll 1
    for (int i = w; i < n; i += 4) {
      if (i >= p && i < p + GB) continue;
      double* Ai = A + static_cast<int64_t>(i) * n;
      const double mine = lane < GB ? Ai[p + lane] : 0.0;
      double cm[GB];
#pragma unroll
      for (int m = 0; m < GB; ++m) cm[m] = __shfl(mine, m);
#pragma unroll 1
      for (int j = lane; j < n; j += 64) {
        double v;
        if (j >= p && j < p + GB) {
          v = 0.0;
#pragma unroll
          for (int m = 0; m < GB; ++m) v -= cm[m] * D[m * GB + (j - p)];
        } else {
          v = Ai[j];
#pragma unroll
          for (int m = 0; m < GB; ++m) v -= cm[m] * R[m * n + j];
        }
        Ai[j] = v;
      }
    }
    __syncthreads();
  }
}

__global__ void k_imp_to_float(const double* __restrict__ W, float* __restrict__ out, int64_t count) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < count;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    out[i] = static_cast<float>(W[i]);
}

template <typename T, int N>
__global__ __launch_bounds__(256) void k_imp_fixed(T* __restrict__ b, const T* __restrict__ q,
                                                   const T* __restrict__ L, T c1, int64_t K, int64_t src_elem,
                                                   T sv, T d0, T d1, T d2, const T* __restrict__ svec) {
  constexpr int Np = Sz<N>::Np, NV = 9 * Np;
  const int64_t total = K * NV;
  for (int64_t x = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; x < total;
       x += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    T v = q[x];
    if (L) v += c1 * L[x];
    const int64_t k = x / NV;
    const int rem = static_cast<int>(x - k * NV), comp = rem / Np, i = rem % Np;
    if (k == src_elem && comp < 3) v += sv * (comp == 0 ? d0 : comp == 1 ? d1 : d2) * svec[i];
    b[x] = v;
  }
}

// One iteration on one element per workgroup: r = b + thdt L - q (LDS),
// y = B^-1 r with one thread per row reading the column-major inverse
// (consecutive threads, consecutive addresses), q += y, and the element's
// J y^T M y for the stopping rule.
template <typename T, int N>
__global__ __launch_bounds__(ImpSz<N>::TPB) void k_imp_iterate(T* __restrict__ q, const T* __restrict__ b,
                                                                 const T* __restrict__ L,
                                                                 const T* __restrict__ inv, T thdt,
                                                                 const double* __restrict__ Mhat,
                                                                 const double* __restrict__ J,
                                                                 double* __restrict__ epart) {
  using S = ImpSz<N>;
  constexpr int Np = S::Np, NV = S::NV, n = S::n, TPB = S::TPB, RPT = S::RPT;
  __shared__ T r[NV];
  __shared__ double y[NV];
  __shared__ double red[TPB / 64];
  const int64_t k = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t base = k * NV;
  for (int x = tid; x < NV; x += TPB) r[x] = b[base + x] + thdt * L[base + x] - q[base + x];
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr < RPT; ++rr) {
    const int i = tid + rr * TPB;
    if (i < NV) {
      const T* col = inv + static_cast<int64_t>(k) * n * n + i;
      T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
      int j = 0;
#pragma unroll 4
      for (; j + 4 <= NV; j += 4) {
        a0 += col[static_cast<int64_t>(j) * n] * r[j];
        a1 += col[static_cast<int64_t>(j + 1) * n] * r[j + 1];
        a2 += col[static_cast<int64_t>(j + 2) * n] * r[j + 2];
        a3 += col[static_cast<int64_t>(j + 3) * n] * r[j + 3];
      }
      for (; j < NV; ++j) a0 += col[static_cast<int64_t>(j) * n] * r[j];
      const T yi = (a0 + a1) + (a2 + a3);
      q[base + i] += yi;
      y[i] = static_cast<double>(yi);
    }
  }
  __syncthreads();
  // squared L2 norm of the change: J sum_c y_c^T Mhat y_c
  double part = 0.0;
  for (int x = tid; x < NV; x += TPB) {
    const int comp = x / Np, a = x % Np;
    double z = 0.0;
    for (int bb = 0; bb < Np; ++bb) z += Mhat[a * Np + bb] * y[comp * Np + bb];
    part += y[x] * z;
  }
  for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off);
  if ((tid & 63) == 0) red[tid >> 6] = part;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int wv = 0; wv < TPB / 64; ++wv) s += red[wv];
    epart[k] = J[k] * s;
  }
}

__global__ __launch_bounds__(1024) void k_imp_sum(const double* __restrict__ x, int64_t n, double* __restrict__ out) {
  __shared__ double red[1024];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) acc += x[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// ------------------------------------------------------------------ launchers
static unsigned grid_for(int64_t count, int block) {
  const int64_t g = (count + block - 1) / block;
  return static_cast<unsigned>(g < 65536 ? (g > 0 ? g : 1) : 65536);
}

hipError_t launch_imp_identity(double* W, int64_t K, int n, hipStream_t st) {
  const int64_t total = K * n * n;
  hipLaunchKernelGGL(k_imp_identity, dim3(grid_for(total, 256)), dim3(256), 0, st, W, total, n);
  return hipGetLastError();
}

hipError_t launch_imp_zero(int prec, void* x, int64_t count, hipStream_t st) {
  if (prec == 32)
    hipLaunchKernelGGL(k_imp_zero<float>, dim3(grid_for(count, 256)), dim3(256), 0, st, static_cast<float*>(x), count);
  else
    hipLaunchKernelGGL(k_imp_zero<double>, dim3(grid_for(count, 256)), dim3(256), 0, st, static_cast<double*>(x),
                       count);
  return hipGetLastError();
}

hipError_t launch_imp_probe(int prec, void* q, const int32_t* members, int cnt, int nv, int j_off, int j_on,
                            hipStream_t st) {
  if (cnt <= 0) return hipSuccess;
  const dim3 grid((cnt + 255) / 256);
  if (prec == 32)
    hipLaunchKernelGGL(k_imp_probe<float>, grid, dim3(256), 0, st, static_cast<float*>(q), members, cnt, nv, j_off,
                       j_on);
  else
    hipLaunchKernelGGL(k_imp_probe<double>, grid, dim3(256), 0, st, static_cast<double*>(q), members, cnt, nv, j_off,
                       j_on);
  return hipGetLastError();
}

hipError_t launch_imp_gather(int prec, const void* L, double* W, const int32_t* members, int cnt, int nv, int n,
                             int j, double thdt, hipStream_t st) {
  if (cnt <= 0) return hipSuccess;
  if (prec == 32)
    hipLaunchKernelGGL(k_imp_gather<float>, dim3(cnt), dim3(256), 0, st, static_cast<const float*>(L), W, members, nv,
                       n, j, thdt);
  else
    hipLaunchKernelGGL(k_imp_gather<double>, dim3(cnt), dim3(256), 0, st, static_cast<const double*>(L), W, members,
                       nv, n, j, thdt);
  return hipGetLastError();
}

template <int N>
static hipError_t invert_impl(double* W, int64_t K, int n, int32_t* flag, hipStream_t st) {
  if (n != ImpSz<N>::n) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_imp_invert<N>), dim3(static_cast<unsigned>(K)), dim3(256), 0, st, W, flag);
  return hipGetLastError();
}

hipError_t launch_imp_invert(double* W, int64_t K, int n, int32_t* flag, hipStream_t st) {
  switch (n) {
    case ImpSz<1>::n: return invert_impl<1>(W, K, n, flag, st);
    case ImpSz<2>::n: return invert_impl<2>(W, K, n, flag, st);
    case ImpSz<3>::n: return invert_impl<3>(W, K, n, flag, st);
    case ImpSz<4>::n: return invert_impl<4>(W, K, n, flag, st);
    case ImpSz<5>::n: return invert_impl<5>(W, K, n, flag, st);
    case ImpSz<7>::n: return invert_impl<7>(W, K, n, flag, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_imp_to_float(const double* W, float* out, int64_t count, hipStream_t st) {
  hipLaunchKernelGGL(k_imp_to_float, dim3(grid_for(count, 256)), dim3(256), 0, st, W, out, count);
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t fixed_impl(const Dev& d, const ImpDev& m, const void* q, const void* L, double c1, int64_t src_elem,
                             double sv, const double dir[3], hipStream_t st) {
  const int64_t total = d.K * 9 * Sz<N>::Np;
  hipLaunchKernelGGL((k_imp_fixed<T, N>), dim3(grid_for(total, 256)), dim3(256), 0, st, static_cast<T*>(m.b),
                     static_cast<const T*>(q), static_cast<const T*>(L), static_cast<T>(c1), d.K, src_elem,
                     static_cast<T>(sv), static_cast<T>(dir[0]), static_cast<T>(dir[1]), static_cast<T>(dir[2]),
                     static_cast<const T*>(d.svec));
  return hipGetLastError();
}

hipError_t launch_imp_fixed(const Dev& d, const ImpDev& m, const void* q, const void* L, double c1, int64_t src_elem,
                            double sv, const double dir[3], hipStream_t st) {
  if (d.prec == 32) {
    EWDG_DISPATCH(d.N, return (fixed_impl<float, NN>(d, m, q, L, c1, src_elem, sv, dir, st)));
  }
  EWDG_DISPATCH(d.N, return (fixed_impl<double, NN>(d, m, q, L, c1, src_elem, sv, dir, st)));
}

template <typename T, int N>
static hipError_t iterate_impl(const Dev& d, const ImpDev& m, void* q, double thdt, hipStream_t st) {
  using S = ImpSz<N>;
  if (m.n != S::n || m.nv != S::NV) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_imp_iterate<T, N>), dim3(static_cast<unsigned>(d.K)), dim3(S::TPB), 0, st,
                     static_cast<T*>(q), static_cast<const T*>(m.b), static_cast<const T*>(m.L),
                     static_cast<const T*>(m.inv), static_cast<T>(thdt), d.Mhat64, d.J64, m.epart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_imp_sum, dim3(1), dim3(1024), 0, st, m.epart, d.K, m.norm2);
  return hipGetLastError();
}

hipError_t launch_imp_iterate(const Dev& d, const ImpDev& m, void* q, double thdt, hipStream_t st) {
  if (d.prec == 32) {
    EWDG_DISPATCH(d.N, return (iterate_impl<float, NN>(d, m, q, thdt, st)));
  }
  EWDG_DISPATCH(d.N, return (iterate_impl<double, NN>(d, m, q, thdt, st)));
}

}  // namespace ewdg
