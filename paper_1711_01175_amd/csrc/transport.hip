// Steady transport by upwind HDG on a structured grid, solved by iHDG-II
// (HIP, gfx950).  Sec. 4.1: each iteration solves every element's local
// equation with its own unknowns new and the exterior traces of its inflow
// faces from the previous iterate.  On a uniform grid with constant beta all
// elements share one local matrix A, so with c_e = A^-1 (load_e - boundary
// inflow_e) and G_a = -A^-1 (beta.n_a) C_a (C_a: the face coupling to the
// upwind neighbour along axis a) an iteration is
//     u_e^{k+1} = c_e + sum_a G_a u^k_{upwind neighbour of e along a}.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "tiles.hpp"
#include "trdev.hpp"

namespace ewdg {

template <int D, int P>
struct TrSz {
  static constexpr int Np = D == 2 ? (P + 1) * (P + 1) : (P + 1) * (P + 1) * (P + 1);
  static constexpr int EPB = Np >= 256 ? 1 : 256 / Np;      // elements per workgroup
  static constexpr int NT = (EPB * Np + 63) / 64 * 64;
};

// FP64, one workgroup per element: c = A^-1 ((f, phi) - boundary inflow),
// the exact solution's projection and the squared norms J ||u^e - Pi u^e||^2
// (a sum of squares of the projection residual, so that the error
// ||u - u^e||^2 = J ||u - Pi u^e||^2 + J ||u^e - Pi u^e||^2 keeps its digits
// when it is small) and J ||u^e||^2.
__global__ __launch_bounds__(256) void k_tr_load(TrDev t, int with_exact) {
  extern __shared__ double sh[];
  double* r = sh;                  // [Np]
  double* up = sh + t.Np;          // [Np]
  double* red = sh + 2 * t.Np;     // [256]
  const int64_t e = blockIdx.x;
  const int tid = threadIdx.x;
  for (int i = tid; i < t.Np; i += 256) {
    double F = 0.0, U = 0.0;
    for (int q = 0; q < t.Nq; ++q) {
      const double v = t.Vq[static_cast<int64_t>(q) * t.Np + i] * t.Wq[q];
      F += v * t.fq[e * t.Nq + q];
      if (with_exact) U += v * t.ueq[e * t.Nq + q];
    }
    F *= t.J;
    // boundary inflow faces: - beta.n <g, phi>_f
    int64_t stride = 1;
    for (int a = 0; a < t.d; ++a) {
      const int64_t ia = (e / stride) % t.n;
      const bool boundary = t.in_side[a] ? (ia == t.n - 1) : (ia == 0);
      if (boundary) {
        const int face = 2 * a + t.in_side[a];
        const double* g = t.gq + (e * 2 * t.d + face) * t.Nqf;
        const double* T = t.Tf + static_cast<int64_t>(face) * t.Nqf * t.Np;
        double s = 0.0;
        for (int q = 0; q < t.Nqf; ++q) s += t.Wf[q] * g[q] * T[static_cast<int64_t>(q) * t.Np + i];
        F -= t.bn[a] * t.Jf * s;
      }
      stride *= t.n;
    }
    r[i] = F;
    up[i] = U;
    if (with_exact) t.uep[e * t.Np + i] = U;
  }
  __syncthreads();
  for (int i = tid; i < t.Np; i += 256) {
    double s = 0.0;
    for (int j = 0; j < t.Np; ++j) s += t.Ainv[static_cast<int64_t>(i) * t.Np + j] * r[j];
    if (t.prec == 32) static_cast<float*>(t.c)[e * t.Np + i] = static_cast<float>(s);
    else static_cast<double*>(t.c)[e * t.Np + i] = s;
  }
  if (!with_exact) return;
  double res = 0.0, full = 0.0;
  for (int q = tid; q < t.Nq; q += 256) {
    const double ue = t.ueq[e * t.Nq + q];
    double pv = 0.0;
    for (int i = 0; i < t.Np; ++i) pv += t.Vq[static_cast<int64_t>(q) * t.Np + i] * up[i];
    res += t.Wq[q] * (ue - pv) * (ue - pv);
    full += t.Wq[q] * ue * ue;
  }
  red[tid] = res;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double rsum = red[0];
  __syncthreads();
  red[tid] = full;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  if (tid == 0) {
    t.rest[e] = t.J * rsum;
    t.rest[t.E + e] = t.J * red[0];
  }
}

template <typename T, int D, int P>
__global__ __launch_bounds__((TrSz<D, P>::NT)) void k_tr_sweep(TrDev t, int src, int to_exact) {
  using S = TrSz<D, P>;
  constexpr int Np = S::Np, EPB = S::EPB, NT = S::NT;
  __shared__ T nbv[EPB * D * Np];
  __shared__ double red[NT / 64];
  const T* uo = static_cast<const T*>(t.u[src]);
  T* un = static_cast<T*>(t.u[1 - src]);
  const T* c = static_cast<const T*>(t.c);
  const T* Gt = static_cast<const T*>(t.Gt);
  const int tid = threadIdx.x;
  const int64_t e0 = static_cast<int64_t>(blockIdx.x) * EPB;
  if (t.ctl->done) return;   // the solve has stopped: a queued iteration does nothing
  // the upwind neighbours' coefficients (zero across the boundary: the
  // boundary inflow is part of c)
  for (int x = tid; x < EPB * D * Np; x += NT) {
    const int el = x / (D * Np), rem = x % (D * Np), a = rem / Np, j = rem % Np;
    const int64_t e = e0 + el;
    T v = T(0);
    if (e < t.E) {
      int64_t stride = 1;
      for (int b = 0; b < a; ++b) stride *= t.n;
      const int64_t ia = (e / stride) % t.n;
      const int64_t nb = t.in_side[a] ? ia + 1 : ia - 1;
      if (nb >= 0 && nb < t.n) v = uo[(e + (nb - ia) * stride) * Np + j];
    }
    nbv[x] = v;
  }
  __syncthreads();
  const int el = tid / Np, i = tid % Np;
  const int64_t e = e0 + el;
  double part = 0.0;
  if (el < EPB && e < t.E) {
    T acc = c[e * Np + i];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const T* g = Gt + static_cast<int64_t>(a) * Np * Np + i;
      const T* v = nbv + (el * D + a) * Np;
#pragma unroll 5
      for (int j = 0; j < Np; ++j) acc += g[j * Np] * v[j];
    }
    un[e * Np + i] = acc;
    const double tg = to_exact ? t.uep[e * Np + i] : static_cast<double>(uo[e * Np + i]);
    const double dd = static_cast<double>(acc) - tg;
    part = dd * dd;
  }
  for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off);
  if ((tid & 63) == 0) red[tid >> 6] = part;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < NT / 64; ++w) s += red[w];
    t.epart[blockIdx.x] = t.J * s;
  }
}

// The same sweep on the matrix cores (Np > 16): a workgroup takes EC = 16 CT
// elements as matrix columns (64 in FP32, 32 in FP64); U_new = C + sum_a G_a
// V_a with V_a the upwind neighbours' coefficients (16x16x4 tiles: rows =
// output modes, k = input modes, zero padded to 16 / 4).  The 4 waves own the
// row tiles round-robin; each G_a fragment (one coalesced 64-lane load from
// L2) feeds CT products.  The axes are taken one at a time: V_a is staged in
// LDS in B-fragment order (a fragment read is 64 consecutive values), then
// multiplied; the result leaves through LDS in element-major rows.
template <typename T>
struct TrMmaShape {
  static constexpr int CT = sizeof(T) == 4 ? 4 : 2;   // column tiles
  static constexpr int EC = 16 * CT;                  // elements per workgroup
};

template <typename T, int D, int P>
__global__ __launch_bounds__(256) void k_tr_sweep_mma(TrDev t, int src, int to_exact) {
  using S = TrSz<D, P>;
  using M = Mfma<T>;
  using acc_t = typename M::acc_t;
  constexpr int Np = S::Np, CT = TrMmaShape<T>::CT, EC = TrMmaShape<T>::EC;
  constexpr int RT = (Np + 15) / 16, KS = (Np + 3) / 4, NpR = 16 * RT;
  constexpr int VSZ = KS * CT * 64;            // one axis, B-fragment ordered
  constexpr int OSZ = EC * NpR;                // element-major result rows
  __shared__ T V[VSZ > OSZ ? VSZ : OSZ];
  __shared__ double red[4];
  const T* uo = static_cast<const T*>(t.u[src]);
  T* un = static_cast<T*>(t.u[1 - src]);
  const T* c = static_cast<const T*>(t.c);
  const T* G = static_cast<const T*>(t.Gfrag);
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
  const int64_t e0 = static_cast<int64_t>(blockIdx.x) * EC;
  if (t.ctl->done) return;   // the solve has stopped: a queued iteration does nothing
  static_assert(D * EC <= 256, "one thread per neighbour offset");
  __shared__ int64_t nbe[D][EC];   // upwind neighbour of each column, -1 at the inflow boundary
  if (tid < D * EC) {
    const int a = tid / EC, col = tid % EC;
    const int64_t e = e0 + col;
    int64_t r = -1;
    if (e < t.E) {
      int64_t stride = 1;
      for (int b = 0; b < a; ++b) stride *= t.n;
      const int64_t ia = (e / stride) % t.n;
      const int64_t nb = t.in_side[a] ? ia + 1 : ia - 1;
      if (nb >= 0 && nb < t.n) r = e + (nb - ia) * stride;
    }
    nbe[a][col] = r;
  }
  acc_t acc[(RT + 3) / 4][CT];
#pragma unroll
  for (int rr = 0; rr < (RT + 3) / 4; ++rr)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) acc[rr][ct] = acc_t{0, 0, 0, 0};
  __syncthreads();
  // one axis at a time: the upwind neighbours' coefficients go to LDS, value
  // j of column col to fragment kk = j / 4, row j % 4, and within the row to
  // position (col + kk) mod 16 (a skew that spreads the stores, consecutive j,
  // over the banks); then the products.  The next axis's values are loaded
  // into registers before the current axis's products, so their latency
  // hides behind the matrix work.
  constexpr int RR = (RT + 3) / 4, TOT = EC * 4 * KS, NI = (TOT + 255) / 256;
  T vr[NI];
  auto gather = [&](int a) {
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int x = tid + 256 * i;
      if (TOT % 256 == 0 || x < TOT) {
        const int j = x % (4 * KS), col = x / (4 * KS);
        const int64_t s = nbe[a][col];
        vr[i] = (j < Np && s >= 0) ? uo[s * Np + j] : T(0);
      }
    }
  };
  gather(0);
#pragma unroll 1
  for (int a = 0; a < D; ++a) {
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int x = tid + 256 * i;
      if (TOT % 256 == 0 || x < TOT) {
        const int j = x % (4 * KS), col = x / (4 * KS), kk = j / 4;
        V[((kk * CT + col / 16) * 4 + j % 4) * 16 + ((col + kk) & 15)] = vr[i];
      }
    }
    __syncthreads();
    if (a + 1 < D) gather(a + 1);
#pragma unroll
    for (int rr = 0; rr < RR; ++rr) {
      const int R = w + 4 * rr;
      if (R < RT) {
        const T* g = G + (static_cast<int64_t>(a * RT + R) * KS) * 64 + l;
#pragma unroll 8
        for (int kk = 0; kk < KS; ++kk) {
          const T av = g[kk * 64];
          const T* vb = V + kk * CT * 64 + (l & 48) + ((l + kk) & 15);
#pragma unroll
          for (int ct = 0; ct < CT; ++ct) acc[rr][ct] = M::mma(av, vb[ct * 64], acc[rr][ct]);
        }
      }
    }
    __syncthreads();
  }
  // result rows to LDS: element col, mode i
  const int lg = l / 16;
#pragma unroll
  for (int rr = 0; rr < (RT + 3) / 4; ++rr) {
    const int R = w + 4 * rr;
    if (R < RT) {
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) V[(ct * 16 + l % 16) * NpR + 16 * R + M::row(lg, r)] = acc[rr][ct][r];
    }
  }
  __syncthreads();
  double part = 0.0;
  for (int x = tid; x < EC * Np; x += 256) {
    const int col = x / Np, i = x % Np;
    const int64_t e = e0 + col;
    if (e < t.E) {
      const T v = V[col * NpR + i] + c[e * Np + i];
      un[e * Np + i] = v;
      const double tg = to_exact ? t.uep[e * Np + i] : static_cast<double>(uo[e * Np + i]);
      const double dd = static_cast<double>(v) - tg;
      part += dd * dd;
    }
  }
  for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off);
  if (l == 0) red[w] = part;
  __syncthreads();
  if (tid == 0) t.epart[blockIdx.x] = t.J * (red[0] + red[1] + red[2] + red[3]);
}

__global__ __launch_bounds__(1024) void k_tr_sum(const double* __restrict__ x, int64_t n, double* __restrict__ out) {
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

// The stopping rule of iteration k (Sec. 6.1): sum the sweep's per-workgroup
// parts, record the norm and set done once the rule holds (or the norm is not
// finite).  Nothing happens once done is set.
__global__ __launch_bounds__(1024) void k_tr_check(const double* __restrict__ x, int64_t n, TrCtl* ctl, int64_t k) {
  __shared__ double red[1024];
  if (ctl->done) return;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) acc += x[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double s = red[0];
    const double v = ctl->exact ? sqrt(fmax(s + ctl->rest, 0.0)) : sqrt(fmax(s, 0.0));
    ctl->hist[k % kTrHist] = v;
    if (!isfinite(v)) {
      ctl->bad = 1;
      ctl->done = k;
    } else {
      const bool stop = ctl->exact ? fabs(v - ctl->prev) < ctl->tol : v < ctl->tol;
      ctl->prev = v;
      if (stop) ctl->done = k;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_tr_values(TrDev t, const T* __restrict__ u, double* __restrict__ out) {
  const int64_t e = blockIdx.x;
  for (int q = threadIdx.x; q < t.Nq; q += 256) {
    double s = 0.0;
    for (int i = 0; i < t.Np; ++i) s += t.Vq[static_cast<int64_t>(q) * t.Np + i] * static_cast<double>(u[e * t.Np + i]);
    out[e * t.Nq + q] = s;
  }
}

template <typename T>
__global__ void k_tr_zero(T* __restrict__ x, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    x[i] = T(0);
}

// ------------------------------------------------------------------ launchers
hipError_t launch_tr_load(const TrDev& t, bool with_exact, hipStream_t st) {
  const size_t lds = (2 * static_cast<size_t>(t.Np) + 256) * 8;
  hipLaunchKernelGGL(k_tr_load, dim3(static_cast<unsigned>(t.E)), dim3(256), lds, st, t, with_exact ? 1 : 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !with_exact) return e;
  hipLaunchKernelGGL(k_tr_sum, dim3(1), dim3(1024), 0, st, t.rest, t.E, t.scal + 6);
  hipLaunchKernelGGL(k_tr_sum, dim3(1), dim3(1024), 0, st, t.rest + t.E, t.E, t.scal + 7);
  return hipGetLastError();
}

template <typename T, int D, int P>
static hipError_t sweep_impl(const TrDev& t, int src, bool to_exact, int64_t k, hipStream_t st) {
  using S = TrSz<D, P>;
  unsigned blocks;
  if constexpr (S::Np > 16) {
    blocks = static_cast<unsigned>((t.E + TrMmaShape<T>::EC - 1) / TrMmaShape<T>::EC);
    hipLaunchKernelGGL((k_tr_sweep_mma<T, D, P>), dim3(blocks), dim3(256), 0, st, t, src, to_exact ? 1 : 0);
  } else {
    blocks = static_cast<unsigned>((t.E + S::EPB - 1) / S::EPB);
    hipLaunchKernelGGL((k_tr_sweep<T, D, P>), dim3(blocks), dim3(S::NT), 0, st, t, src, to_exact ? 1 : 0);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tr_check, dim3(1), dim3(1024), 0, st, t.epart, static_cast<int64_t>(blocks), t.ctl, k);
  return hipGetLastError();
}

template <typename T, int D>
static hipError_t sweep_p(const TrDev& t, int src, bool to_exact, int64_t k, hipStream_t st) {
  switch (t.p) {
    case 1: return sweep_impl<T, D, 1>(t, src, to_exact, k, st);
    case 2: return sweep_impl<T, D, 2>(t, src, to_exact, k, st);
    case 3: return sweep_impl<T, D, 3>(t, src, to_exact, k, st);
    case 4: return sweep_impl<T, D, 4>(t, src, to_exact, k, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tr_iterate(const TrDev& t, int src, bool to_exact, int64_t k, hipStream_t st) {
  if (t.prec == 32) return t.d == 2 ? sweep_p<float, 2>(t, src, to_exact, k, st)
                                    : sweep_p<float, 3>(t, src, to_exact, k, st);
  return t.d == 2 ? sweep_p<double, 2>(t, src, to_exact, k, st) : sweep_p<double, 3>(t, src, to_exact, k, st);
}

bool tr_uses_mma(int Np) { return Np > 16; }
int tr_row_tiles(int Np) { return (Np + 15) / 16; }
int tr_k_steps(int Np) { return (Np + 3) / 4; }

int tr_sweep_blocks(const TrDev& t) {
  const int Np = t.Np;
  const int epb = tr_uses_mma(Np) ? 32 : (Np >= 256 ? 1 : 256 / Np);   // the FP64 tile: the smaller count
  return static_cast<int>((t.E + epb - 1) / epb);
}

hipError_t launch_tr_values(const TrDev& t, int src, double* out, hipStream_t st) {
  if (t.prec == 32)
    hipLaunchKernelGGL(k_tr_values<float>, dim3(static_cast<unsigned>(t.E)), dim3(256), 0, st, t,
                       static_cast<const float*>(t.u[src]), out);
  else
    hipLaunchKernelGGL(k_tr_values<double>, dim3(static_cast<unsigned>(t.E)), dim3(256), 0, st, t,
                       static_cast<const double*>(t.u[src]), out);
  return hipGetLastError();
}

hipError_t launch_tr_zero(const TrDev& t, int which, hipStream_t st) {
  const int64_t n = t.E * t.Np;
  const unsigned g = static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 65536));
  if (t.prec == 32) hipLaunchKernelGGL(k_tr_zero<float>, dim3(g), dim3(256), 0, st, static_cast<float*>(t.u[which]), n);
  else hipLaunchKernelGGL(k_tr_zero<double>, dim3(g), dim3(256), 0, st, static_cast<double*>(t.u[which]), n);
  return hipGetLastError();
}

}  // namespace ewdg
