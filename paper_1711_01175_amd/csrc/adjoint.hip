// Discrete adjoint of the DG right-hand side (HIP, gfx950).
//
// For an adjoint vector y of a stage right-hand side, computes L^T y (the
// plain transpose of the nodal operator) and the parameter gradient
// y . d(L q + f)/d theta for per-element multipliers theta = (s_rho,
// s_lambda, s_mu) of the quadrature-sampled material, at the current
// material.  The face coupling is transposed as a gather: pass A stores, per
// face point, the sensitivities of the element's own face correction with
// respect to both sides' traces and impedances; pass B adds to each element
// its own-side terms and the neighbour-side terms computed by its
// neighbours, so every element writes only its own data (no atomics).
#include <hip/hip_runtime.h>

#include "adjdev.hpp"
#include "dev.hpp"
#include "kcommon.hpp"
#include "tiles.hpp"

// Tuning constants (measured on MI355X at N=4): EWDG_ADJ_LDS caps the LDS of
// one workgroup in KiB (fewer elements per workgroup, more workgroups per
// CU); EWDG_ADJ_UNROLL > 0 forces that unroll factor on the inner loops;
// EWDG_ADJ_QC32 / EWDG_ADJ_QC64 are the quadrature rows per projection chunk
// of the matrix-core pass B in FP32 / FP64 (in FP32, 32 rather than 64 halves
// the chunk registers and LDS: at N=4 3 waves per SIMD instead of 2, 7 % less
// gradient time; FP64 stays at one wave per SIMD either way and is 8 % faster
// with 64);
// EWDG_ADJ_OCC is its waves-per-SIMD target; EWDG_ADJ_MMA = 0 selects the
// LDS-staged pass B everywhere.
#ifndef EWDG_ADJ_LDS
#define EWDG_ADJ_LDS 20
#endif
#ifndef EWDG_ADJ_UNROLL
#define EWDG_ADJ_UNROLL 0
#endif
#ifndef EWDG_ADJ_MMA
#define EWDG_ADJ_MMA 1
#endif
#ifndef EWDG_ADJ_QC32
#define EWDG_ADJ_QC32 32
#endif
#ifndef EWDG_ADJ_QC64
#define EWDG_ADJ_QC64 64
#endif
#ifndef EWDG_ADJ_OCC
#define EWDG_ADJ_OCC 2
#endif
#define EWDG_PRAGMA(x) _Pragma(#x)
#if EWDG_ADJ_UNROLL > 0
#define EWDG_UNROLL_N(n) EWDG_PRAGMA(unroll n)
#else
#define EWDG_UNROLL_N(n)
#endif

namespace ewdg {

template <typename T>
struct AdjArgs {
  const T* y;          // [K][9][Np] adjoint of the stage right-hand side
  const T* q;          // forward stage input [K][9][Np] (null: no parameter gradient)
  const T* s;          // sigma_h(q) [K][6][Np]
  const T* rhs;        // velocity rows of L q + f, element stride rhs_es (density gradient)
  int rhs_es;
  T* ytil;             // [K][3][Np] W^T y_v
  T* fown;             // [K][4][Nfp][8] own-side sensitivities (v, T, Z_p, Z_s)
  T* fnbr;             // [K][4][Nfp][8] neighbour-side sensitivities
  T* qbar;             // [K][9][Np] += scale * L^T y
  double* g;           // [K][3] += scale * gradient (null: none)
  const T* W;
  const T* lm;
  const T* geo;
  const T* fgeo;
  const T* Z;
  const double* means;  // [K][3] element means of rho, lambda, mu
  const int32_t* conn;
  const int32_t* nbrnode;
  const int32_t* nbrface;
  const int32_t* fmask;
  const T* Dk;         // [3][Np][Np] row-major
  const T* LIFT;       // [Np][4Nfp]
  const T* Vq;         // [Nq][Np]
  const T* VqT;        // [Np][Nq]
  const T* Pq;         // [Np][Nq]
  // fragment-order operators for the matrix-core pass B
  const T* DTpad;      // D_k^T  [3][RT][NpK/4][64]
  const T* PqTpad;     // Pq^T   [QT][NpK/4][64]
  const T* VqTpad;     // Vq^T   [RT][NqK/4][64]
  const T* Vqpad;      // Vq     [QT][NpK/4][64]
  int64_t K;
  T scale;
  // if set (it is y itself): after qbar is updated, rupd = ra rupd + rb qbar
  // for the kernel's own elements (the scaling and the next axpy of the
  // reverse Runge-Kutta recurrence, fused)
  T* rupd;
  T ra, rb;
};

// rupd = ra rupd + rb qbar over the elements [e0, e0 + ne) of one workgroup;
// call after a barrier that follows every read of y and write of qbar.
template <typename T, int Np>
__device__ __forceinline__ void fused_recurrence(const AdjArgs<T>& a, int64_t e0, int ne, int tid, int nt) {
  for (int x = tid; x < ne * 9 * Np; x += nt) {
    const int64_t i = e0 * 9 * Np + x;
    a.rupd[i] = a.ra * a.rupd[i] + a.rb * a.qbar[i];
  }
}

template <typename T, int N>
struct AdjCfg {
  using S = Sz<N>;
  static constexpr int per_a = 12 * S::Np + 32;
  static constexpr int per_b = 27 * S::Np + 6 * S::Nq + 8 * S::Nfp + 2 * S::Nq + S::Np + 32;
  static constexpr int per = per_a > per_b ? per_a : per_b;
  static constexpr int e_lds = (EWDG_ADJ_LDS * 1024) / (per * static_cast<int>(sizeof(T)));
  static constexpr int e_thr = 256 / S::Np > 0 ? 256 / S::Np : 1;
  static constexpr int E = (e_lds < e_thr ? e_lds : e_thr) > 0 ? (e_lds < e_thr ? e_lds : e_thr) : 1;
  static constexpr int NT = ((E * S::Np + 63) / 64) * 64 > 64 ? ((E * S::Np + 63) / 64) * 64 : 64;
};

template <typename T>
__device__ __forceinline__ void load_geo(const AdjArgs<T>& a, int64_t e0, int ne, T* sg, int tid, int NT) {
  for (int x = tid; x < ne * 27; x += NT) {
    const int e = x / 27, m = x % 27;
    T v;
    if (m < 9) v = a.geo[(e0 + e) * 9 + m];
    else if (m < 25) v = a.fgeo[(e0 + e) * 16 + (m - 9)];
    else v = a.Z[(e0 + e) * kZS + (m - 25)];
    sg[e * 32 + m] = v;
  }
}

// Pass A: W^T y_v, LIFT^T at the face points and the transposed interface
// state.
template <typename T, int N>
__global__ __launch_bounds__((AdjCfg<T, N>::NT)) void k_adjA(AdjArgs<T> a) {
  using S = Sz<N>;
  using C = AdjCfg<T, N>;
  constexpr int Np = S::Np, Nfp = S::Nfp, NF = S::NF, E = C::E, NT = C::NT;
  __shared__ T Yv[E * 3 * Np];
  __shared__ T Yt[E * 9 * Np];
  __shared__ T sg[E * 32];
  const int tid = threadIdx.x;
  const int64_t e0 = static_cast<int64_t>(blockIdx.x) * E;
  const int ne = static_cast<int>((a.K - e0) < E ? (a.K - e0) : E);
  for (int x = tid; x < ne * 9 * Np; x += NT) {
    const int e = x / (9 * Np), c = (x / Np) % 9, j = x % Np;
    const T v = a.y[e0 * 9 * Np + x];
    if (c < 3) Yv[(e * 3 + c) * Np + j] = v;
    else Yt[(e * 9 + c) * Np + j] = v;
  }
  load_geo(a, e0, ne, sg, tid, NT);
  __syncthreads();
  for (int x = tid; x < ne * Np; x += NT) {
    const int e = x / Np, i = x % Np;
    const T* Wr = a.W + (e0 + e) * Np * Np + i * Np;   // W_ji over j
    T o[3] = {0, 0, 0};
    EWDG_UNROLL_N(EWDG_ADJ_UNROLL)
    for (int j = 0; j < Np; ++j) {
      const T wv = Wr[j];
#pragma unroll
      for (int c = 0; c < 3; ++c) o[c] += wv * Yv[(e * 3 + c) * Np + j];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Yt[(e * 9 + c) * Np + i] = o[c];
      a.ytil[(e0 + e) * 3 * Np + c * Np + i] = o[c];
    }
  }
  __syncthreads();
  for (int x = tid; x < ne * NF; x += NT) {
    const int e = x / NF, fj = x % NF, f = fj / Nfp, j = fj % Nfp;
    const T* gg = &sg[e * 32];
    const T n[3] = {gg[9 + f * 4], gg[9 + f * 4 + 1], gg[9 + f * 4 + 2]};
    const T fs = gg[9 + f * 4 + 3];
    const int32_t wd = a.conn[(e0 + e) * 4 + f];
    const int64_t nb = wd >> 5;
    const int code = wd & 31;
    const T zpm = gg[25], zsm = gg[26], zpp = a.Z[nb * kZS], zsp = a.Z[nb * kZS + 1];
    T D[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) D[c] = 0;
    EWDG_UNROLL_N(EWDG_ADJ_UNROLL)
    for (int i = 0; i < Np; ++i) {
      const T L = a.LIFT[i * NF + fj];
#pragma unroll
      for (int c = 0; c < 9; ++c) D[c] += L * Yt[(e * 9 + c) * Np + i];
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) D[c] *= fs;
    // adjoint of the strain correction sym(n (x) w) with respect to w
    const T wb[3] = {n[0] * D[3] + T(0.5) * (n[2] * D[7] + n[1] * D[8]),
                     n[1] * D[4] + T(0.5) * (n[2] * D[6] + n[0] * D[8]),
                     n[2] * D[5] + T(0.5) * (n[1] * D[6] + n[0] * D[7])};
    const T dTn = D[0] * n[0] + D[1] * n[1] + D[2] * n[2];
    const T wn = wb[0] * n[0] + wb[1] * n[1] + wb[2] * n[2];
    const T Sp = zpm + zpp, Ss = zsm + zsp;
    const T un = (zpm * dTn + wn) / Sp;
    T ut[3], dTt[3], wt[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      dTt[c] = D[c] - dTn * n[c];
      wt[c] = wb[c] - wn * n[c];
      ut[c] = (zsm * dTt[c] + wt[c]) / Ss;
    }
    T zpmb = 0, zppb = 0, zsmb = 0, zspb = 0;
    if (a.q) {
      const int il = a.fmask[f * Nfp + j];
      const int nn = a.nbrnode[((f * 4 + code / 6) * 6 + code % 6) * Nfp + j];
      T vm[3], vp[3], sm[6], sp[6];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        vm[c] = a.q[(e0 + e) * 9 * Np + c * Np + il];
        vp[c] = a.q[nb * 9 * Np + c * Np + nn];
      }
#pragma unroll
      for (int m = 0; m < 6; ++m) {
        sm[m] = a.s[(e0 + e) * 6 * Np + m * Np + il];
        sp[m] = a.s[nb * 6 * Np + m * Np + nn];
      }
      const T jT[3] = {(sp[0] - sm[0]) * n[0] + (sp[5] - sm[5]) * n[1] + (sp[4] - sm[4]) * n[2],
                       (sp[5] - sm[5]) * n[0] + (sp[1] - sm[1]) * n[1] + (sp[3] - sm[3]) * n[2],
                       (sp[4] - sm[4]) * n[0] + (sp[3] - sm[3]) * n[1] + (sp[2] - sm[2]) * n[2]};
      const T jv[3] = {vp[0] - vm[0], vp[1] - vm[1], vp[2] - vm[2]};
      const T jTn = jT[0] * n[0] + jT[1] * n[1] + jT[2] * n[2];
      const T jvn = jv[0] * n[0] + jv[1] * n[1] + jv[2] * n[2];
      const T u_n = jTn + zpp * jvn;
      zpmb = u_n * (zpp * dTn - wn) / (Sp * Sp);
      zppb = (jvn * Sp - u_n) * (zpm * dTn + wn) / (Sp * Sp);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T jTt = jT[c] - jTn * n[c], jvt = jv[c] - jvn * n[c];
        const T u_t = jTt + zsp * jvt;
        zsmb += u_t * (zsp * dTt[c] - wt[c]) / (Ss * Ss);
        zspb += (jvt * Ss - u_t) * (zsm * dTt[c] + wt[c]) / (Ss * Ss);
      }
    }
    T* fo = a.fown + (((e0 + e) * 4 + f) * Nfp + j) * 8;
    T* fn = a.fnbr + (((e0 + e) * 4 + f) * Nfp + j) * 8;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T Tp = un * n[c] + ut[c];                  // d/d T^+
      const T Vp = zpp * un * n[c] + zsp * ut[c];      // d/d v^+
      fo[c] = -Vp;
      fo[3 + c] = -Tp;
      fn[c] = Vp;
      fn[3 + c] = Tp;
    }
    fo[6] = zpmb;
    fo[7] = zsmb;
    fn[6] = zppb;
    fn[7] = zspb;
  }
}

// Pass B: gather of face sensitivities, transposed volume terms, transposed
// stress projection, update of qbar and of the parameter gradient.
template <typename T, int N>
__global__ __launch_bounds__((AdjCfg<T, N>::NT)) void k_adjB(AdjArgs<T> a) {
  using S = Sz<N>;
  using C = AdjCfg<T, N>;
  constexpr int Np = S::Np, Nfp = S::Nfp, Nq = S::Nq, E = C::E, NT = C::NT;
  __shared__ T Yt[E * 9 * Np];    // ytil (0..2), y strains (3..8)
  __shared__ T Zc[E * 9 * Np];    // strain adjoint folded with geometry; later own strains
  __shared__ T SB[E * 6 * Np];    // sigma-bar
  __shared__ T VB[E * 3 * Np];    // v-bar
  __shared__ T Qd[E * 6 * Nq];    // strain adjoint at the quadrature points
  __shared__ T zf[E * 8 * Nfp];   // impedance sensitivities per face point (2 each)
  __shared__ T pp[E * 2 * Nq];    // lambda / mu gradient partials per quadrature point
  __shared__ T pr[E * Np];        // density gradient partials per node
  __shared__ T sg[E * 32];
  const int tid = threadIdx.x;
  const int64_t e0 = static_cast<int64_t>(blockIdx.x) * E;
  const int ne = static_cast<int>((a.K - e0) < E ? (a.K - e0) : E);
  for (int x = tid; x < ne * 9 * Np; x += NT) {
    const int e = x / (9 * Np), c = (x / Np) % 9, j = x % Np;
    Yt[(e * 9 + c) * Np + j] = (c < 3) ? a.ytil[(e0 + e) * 3 * Np + c * Np + j] : a.y[e0 * 9 * Np + x];
  }
  load_geo(a, e0, ne, sg, tid, NT);
  __syncthreads();
  // z_c^k = sum_m (dr_k/dx_m) ybar_cm with ybar the strain adjoint as a
  // full tensor (off-diagonal halves)
  for (int x = tid; x < ne * Np; x += NT) {
    const int e = x / Np, r = x % Np;
    const T* y6 = &Yt[(e * 9 + 3) * Np + r];
    const T yb[3][3] = {{y6[0], T(0.5) * y6[5 * Np], T(0.5) * y6[4 * Np]},
                        {T(0.5) * y6[5 * Np], y6[Np], T(0.5) * y6[3 * Np]},
                        {T(0.5) * y6[4 * Np], T(0.5) * y6[3 * Np], y6[2 * Np]}};
    const T* g = &sg[e * 32];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        Zc[(e * 9 + c * 3 + k) * Np + r] = g[k * 3] * yb[c][0] + g[k * 3 + 1] * yb[c][1] + g[k * 3 + 2] * yb[c][2];
  }
  __syncthreads();
  for (int x = tid; x < ne * Np; x += NT) {
    const int e = x / Np, j = x % Np;
    T Gb[3][3], vb[3] = {0, 0, 0};
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int k = 0; k < 3; ++k) Gb[c][k] = 0;
    EWDG_UNROLL_N(EWDG_ADJ_UNROLL)
    for (int r = 0; r < Np; ++r) {
      T dk[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) dk[k] = a.Dk[(k * Np + r) * Np + j];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T yv = Yt[(e * 9 + c) * Np + r];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          Gb[c][k] += dk[k] * yv;
          vb[c] += dk[k] * Zc[(e * 9 + c * 3 + k) * Np + r];
        }
      }
    }
    const T* g = &sg[e * 32];
    T sb[6];
    sb[0] = g[0] * Gb[0][0] + g[3] * Gb[0][1] + g[6] * Gb[0][2];
    sb[1] = g[1] * Gb[1][0] + g[4] * Gb[1][1] + g[7] * Gb[1][2];
    sb[2] = g[2] * Gb[2][0] + g[5] * Gb[2][1] + g[8] * Gb[2][2];
    sb[3] = 0;
    sb[4] = 0;
    sb[5] = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      sb[3] += g[k * 3 + 2] * Gb[1][k] + g[k * 3 + 1] * Gb[2][k];   // yz
      sb[4] += g[k * 3 + 2] * Gb[0][k] + g[k * 3 + 0] * Gb[2][k];   // xz
      sb[5] += g[k * 3 + 1] * Gb[0][k] + g[k * 3 + 0] * Gb[1][k];   // xy
    }
#pragma unroll
    for (int m = 0; m < 6; ++m) SB[(e * 6 + m) * Np + j] = sb[m];
#pragma unroll
    for (int c = 0; c < 3; ++c) VB[(e * 3 + c) * Np + j] = vb[c];
  }
  __syncthreads();
  // own strains of the forward state for the lambda / mu gradient
  if (a.q) {
    for (int x = tid; x < ne * 6 * Np; x += NT) {
      const int e = x / (6 * Np), m = (x / Np) % 6, j = x % Np;
      Zc[(e * 6 + m) * Np + j] = a.q[(e0 + e) * 9 * Np + (3 + m) * Np + j];
    }
  }
  // face sensitivities, one face at a time (face nodes repeat across faces)
  for (int f = 0; f < 4; ++f) {
    for (int x = tid; x < ne * Nfp; x += NT) {
      const int e = x / Nfp, j = x % Nfp;
      const int il = a.fmask[f * Nfp + j];
      const T* gg = &sg[e * 32];
      const T n[3] = {gg[9 + f * 4], gg[9 + f * 4 + 1], gg[9 + f * 4 + 2]};
      const int32_t wd = a.conn[(e0 + e) * 4 + f];
      const int64_t nb = wd >> 5;
      const int code = wd & 31;
      const int jn = a.nbrface[((f * 4 + code / 6) * 6 + code % 6) * Nfp + j];
      const T* fo = a.fown + (((e0 + e) * 4 + f) * Nfp + j) * 8;
      const T* fn = a.fnbr + ((nb * 4 + code / 6) * Nfp + jn) * 8;
      // the neighbour's traction of this element's stress uses its normal -n
      T Te[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        VB[(e * 3 + c) * Np + il] += fo[c] + fn[c];
        Te[c] = fo[3 + c] - fn[3 + c];
      }
      SB[(e * 6 + 0) * Np + il] += Te[0] * n[0];
      SB[(e * 6 + 1) * Np + il] += Te[1] * n[1];
      SB[(e * 6 + 2) * Np + il] += Te[2] * n[2];
      SB[(e * 6 + 3) * Np + il] += Te[1] * n[2] + Te[2] * n[1];
      SB[(e * 6 + 4) * Np + il] += Te[0] * n[2] + Te[2] * n[0];
      SB[(e * 6 + 5) * Np + il] += Te[0] * n[1] + Te[1] * n[0];
      zf[(e * 4 * Nfp + f * Nfp + j) * 2] = fo[6] + fn[6];
      zf[(e * 4 * Nfp + f * Nfp + j) * 2 + 1] = fo[7] + fn[7];
    }
    __syncthreads();
  }
  // transposed projection: tau = Pq^T sigma-bar, then the elasticity adjoint
  for (int x = tid; x < ne * Nq; x += NT) {
    const int e = x / Nq, qp = x % Nq;
    T tau[6] = {0, 0, 0, 0, 0, 0};
    EWDG_UNROLL_N(EWDG_ADJ_UNROLL)
    for (int i = 0; i < Np; ++i) {
      const T p = a.Pq[i * Nq + qp];
#pragma unroll
      for (int m = 0; m < 6; ++m) tau[m] += p * SB[(e * 6 + m) * Np + i];
    }
    const T lam = a.lm[(e0 + e) * 2 * S::NqP + qp], mu = a.lm[(e0 + e) * 2 * S::NqP + S::NqP + qp];
    const T trt = tau[0] + tau[1] + tau[2];
#pragma unroll
    for (int m = 0; m < 6; ++m) Qd[(e * 6 + m) * Nq + qp] = T(2) * mu * tau[m] + (m < 3 ? lam * trt : T(0));
    if (a.q) {
      T ep[6] = {0, 0, 0, 0, 0, 0};
      EWDG_UNROLL_N(EWDG_ADJ_UNROLL)
      for (int j = 0; j < Np; ++j) {
        const T v = a.VqT[j * Nq + qp];
#pragma unroll
        for (int m = 0; m < 6; ++m) ep[m] += v * Zc[(e * 6 + m) * Np + j];
      }
      const T tr = ep[0] + ep[1] + ep[2];
      T pm = 0;
#pragma unroll
      for (int m = 0; m < 6; ++m) pm += tau[m] * T(2) * mu * ep[m];
      pp[(e * Nq + qp) * 2] = lam * tr * trt;
      pp[(e * Nq + qp) * 2 + 1] = pm;
    }
  }
  __syncthreads();
  for (int x = tid; x < ne * Np; x += NT) {
    const int e = x / Np, j = x % Np;
    T eb[6] = {0, 0, 0, 0, 0, 0};
    EWDG_UNROLL_N(EWDG_ADJ_UNROLL)
    for (int qp = 0; qp < Nq; ++qp) {
      const T v = a.Vq[qp * Np + j];
#pragma unroll
      for (int m = 0; m < 6; ++m) eb[m] += v * Qd[(e * 6 + m) * Nq + qp];
    }
    T* qb = a.qbar + (e0 + e) * 9 * Np + j;
#pragma unroll
    for (int c = 0; c < 3; ++c) qb[c * Np] += a.scale * VB[(e * 3 + c) * Np + j];
#pragma unroll
    for (int m = 0; m < 6; ++m) qb[(3 + m) * Np] += a.scale * eb[m];
    if (a.q) {
      T p = 0;
#pragma unroll
      for (int c = 0; c < 3; ++c)
        p += a.y[(e0 + e) * 9 * Np + c * Np + j] * a.rhs[(e0 + e) * a.rhs_es + c * Np + j];
      pr[e * Np + j] = -p;
    }
  }
  if (!a.q || !a.g) {
    if (a.rupd) {
      __syncthreads();
      fused_recurrence<T, Np>(a, e0, ne, tid, NT);
    }
    return;
  }
  __syncthreads();
  // per-element gradient in FP64, summed in a fixed order
  for (int e = tid; e < ne; e += NT) {
    double gr = 0, gl = 0, gm = 0, zp = 0, zs = 0;
    for (int j = 0; j < Np; ++j) gr += static_cast<double>(pr[e * Np + j]);
    EWDG_UNROLL_N(EWDG_ADJ_UNROLL)
    for (int qp = 0; qp < Nq; ++qp) {
      gl += static_cast<double>(pp[(e * Nq + qp) * 2]);
      gm += static_cast<double>(pp[(e * Nq + qp) * 2 + 1]);
    }
    for (int x = 0; x < 4 * Nfp; ++x) {
      zp += static_cast<double>(zf[(e * 4 * Nfp + x) * 2]);
      zs += static_cast<double>(zf[(e * 4 * Nfp + x) * 2 + 1]);
    }
    // chain rule through Z_p = sqrt(rho (lambda + 2 mu)), Z_s = sqrt(rho mu)
    const double* mn = a.means + (e0 + e) * 3;
    const double Zp = sqrt(mn[0] * (mn[1] + 2.0 * mn[2])), Zs = sqrt(mn[0] * mn[2]);
    gr += 0.5 * Zp * zp + 0.5 * Zs * zs;
    gl += mn[0] * mn[1] / (2.0 * Zp) * zp;
    gm += mn[0] * mn[2] / Zp * zp + 0.5 * Zs * zs;
    const double sc = static_cast<double>(a.scale);
    a.g[(e0 + e) * 3 + 0] += sc * gr;
    a.g[(e0 + e) * 3 + 1] += sc * gl;
    a.g[(e0 + e) * 3 + 2] += sc * gm;
  }
  if (a.rupd) fused_recurrence<T, Np>(a, e0, ne, tid, NT);   // y was last read before the barrier above
}

// Pass B on the matrix cores, for a tile of 16 elements (matrix columns are
// (field, element) pairs as in the stage kernel; the owner wave of node row
// tile R accumulates rows 16R..16R+15):
//  1. Gb_c^k = D_k^T ytil_c and vbar_c = sum_k D_k^T z_c^k, with z_c^k the
//     strain adjoint contracted with dr_k/dx; sigma-bar folds Gb with dr/dx;
//  2. face sensitivities from both sides are added at the face nodes;
//  3. tau = Pq^T sigma-bar at the quadrature points, the elasticity adjoint
//     2 mu tau + lambda tr(tau) I, and (for the gradient) eps_q = Vq eps;
//  4. epsbar = Vq^T (2 mu tau + lambda tr(tau) I), chunk by chunk;
//  5. qbar += scale (vbar, epsbar); per-element gradient in a fixed order.
template <typename T, int N>
struct AdjTile {
  using TL = Tile<N>;
  static constexpr int Np = TL::Np, Nfp = TL::Nfp, NpK = TL::NpK, E = TL::E, NW = TL::NW;
  static constexpr int SV = TL::SV, SE = TL::SE, SQ = TL::SQ;
  static constexpr int QCT = sizeof(T) == 4 ? EWDG_ADJ_QC32 : EWDG_ADJ_QC64;
  static constexpr int QC = TL::NqR < QCT ? TL::NqR : QCT;   // quadrature rows per chunk
  static constexpr int SB = 9 * 16 + 1;                       // sigma-bar (0..5) | v-bar (6..8)
  static constexpr int R1 = cmax2(2 * NpK * SV, NpK * SE);    // volume operands, own strains, epsbar
  static constexpr int R2 = NpK * SB;
  static constexpr int R3 = cmax2(cmax2(E * 4 * Nfp * 2, QC * SQ), E * Np);   // zf, then Qd, then rho partials
  static constexpr int RED = NW * 64 * 2;
  static constexpr int BYTES = (R1 + R2 + R3 + RED + E * 32) * static_cast<int>(sizeof(T)) + E * 2 * 8;
  static constexpr bool fits = BYTES <= 156 * 1024;
};

template <typename T, int N>
__global__ __launch_bounds__((Tile<N>::NT), EWDG_ADJ_OCC) void k_adjB_mma(AdjArgs<T> a) {
  using TL = Tile<N>;
  using AT = AdjTile<T, N>;
  using M = Mfma<T>;
  using acc_t = typename M::acc_t;
  constexpr int Np = TL::Np, Nfp = TL::Nfp, Nq = TL::Nq, NqP = TL::NqP, E = TL::E;
  constexpr int NpK = TL::NpK, NqK = TL::NqK, RT = TL::RT, QT = TL::QT, NW = TL::NW, NT = TL::NT;
  constexpr int SV = AT::SV, SE = AT::SE, SQ = AT::SQ, QC = AT::QC, SB = AT::SB;
  constexpr int KD = NpK / 4, KQ = QC / 4, NQC = (QT * 16 + QC - 1) / QC;
  __shared__ T r1[AT::R1];
  __shared__ T r2[AT::R2];
  __shared__ T r3[AT::R3];
  __shared__ T red[AT::RED];
  __shared__ T sgeo[E * 32];
  __shared__ double zsum[E * 2];
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, lr = l & 15, lg = l >> 4;
  const bool own = w < RT;
  const int R = w;
  const int64_t e0 = static_cast<int64_t>(blockIdx.x) * E;
  const int ne = static_cast<int>((a.K - e0) < E ? (a.K - e0) : E);
  const bool grad = a.q && a.g;

  for (int x = tid; x < E * 27; x += NT) {
    const int e = x / 27, m = x % 27;
    T v = T(0);
    if (e < ne) {
      if (m < 9) v = a.geo[(e0 + e) * 9 + m];
      else if (m < 25) v = a.fgeo[(e0 + e) * 16 + (m - 9)];
      else v = a.Z[(e0 + e) * kZS + (m - 25)];
    }
    sgeo[e * 32 + m] = v;
  }
  T* Sv = r1;               // [NpK][SV] ytil_c at column c*16+e
  T* SG = r1 + NpK * SV;    // [NpK][SV] z_c^k for the current direction
  // bank swizzle of the element slots of Sv and SG as in the stage kernel:
  // element e of row r sits in slot e ^ (r mod 16) (not at N = 7)
  auto sw = [](int r) { return N < 7 ? (r & 15) : 0; };
  for (int x = tid; x < E * 3 * NpK; x += NT) {
    const int e = x / (3 * NpK), rem = x % (3 * NpK), c = rem / NpK, j = rem % NpK;
    T v = T(0);
    if (e < ne && j < Np) v = a.ytil[(e0 + e) * 3 * Np + c * Np + j];
    Sv[j * SV + c * 16 + (e ^ sw(j))] = v;
    if (j >= Np) SG[j * SV + c * 16 + (e ^ sw(j))] = T(0);
  }
  __syncthreads();

  // ---- 1. transposed volume terms
  acc_t sb[6], vb[3];
#pragma unroll
  for (int m = 0; m < 6; ++m) sb[m] = acc_t{0, 0, 0, 0};
#pragma unroll
  for (int c = 0; c < 3; ++c) vb[c] = acc_t{0, 0, 0, 0};
  constexpr int NPT = (E * Np + NT - 1) / NT;
  // this thread's strain adjoints, loaded once for the three directions
  T yr[NPT][6];
#pragma unroll
  for (int p = 0; p < NPT; ++p) {
    const int x = tid + p * NT;
    const int e = x / Np, r = x % Np;
    const bool ok = x < E * Np && e < ne;
#pragma unroll
    for (int m = 0; m < 6; ++m) yr[p][m] = ok ? a.y[(e0 + e) * 9 * Np + (3 + m) * Np + r] : T(0);
  }
#pragma unroll 1
  for (int k = 0; k < 3; ++k) {
    T af[KD];
    if (own) {
      const T* D = a.DTpad + ((k * RT + R) * KD) * 64 + l;
#pragma unroll
      for (int kk = 0; kk < KD; ++kk) af[kk] = D[kk * 64];
    }
#pragma unroll
    for (int p = 0; p < NPT; ++p) {
      const int x = tid + p * NT;
      if (x < E * Np) {
        const int e = x / Np, r = x % Np;
        const T* y6 = yr[p];
        const T* g = &sgeo[e * 32 + k * 3];
        // z_c = sum_m g_m ybar_cm, ybar the strain adjoint as a tensor (off-diagonal halves)
        const int es = e ^ sw(r);
        SG[r * SV + 0 * 16 + es] = g[0] * y6[0] + T(0.5) * (g[1] * y6[5] + g[2] * y6[4]);
        SG[r * SV + 1 * 16 + es] = g[1] * y6[1] + T(0.5) * (g[0] * y6[5] + g[2] * y6[3]);
        SG[r * SV + 2 * 16 + es] = g[2] * y6[2] + T(0.5) * (g[0] * y6[4] + g[1] * y6[3]);
      }
    }
    __syncthreads();
    if (own) {
      acc_t gb[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) gb[c] = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < KD; ++kk) {
        const int rr = 4 * kk + lg;
        const int row = rr * SV + (lr ^ sw(rr));
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          gb[c] = M::mma(af[kk], Sv[row + c * 16], gb[c]);
          vb[c] = M::mma(af[kk], SG[row + c * 16], vb[c]);
        }
      }
      const T g0 = sgeo[lr * 32 + k * 3], g1 = sgeo[lr * 32 + k * 3 + 1], g2 = sgeo[lr * 32 + k * 3 + 2];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        sb[0][r] += g0 * gb[0][r];
        sb[1][r] += g1 * gb[1][r];
        sb[2][r] += g2 * gb[2][r];
        sb[3][r] += g2 * gb[1][r] + g1 * gb[2][r];
        sb[4][r] += g2 * gb[0][r] + g0 * gb[2][r];
        sb[5][r] += g1 * gb[0][r] + g0 * gb[1][r];
      }
    }
    __syncthreads();
  }
  T* SBV = r2;   // [NpK][SB]
  if (own) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = R * 16 + M::row(lg, r);
      if (i < NpK) {
#pragma unroll
        for (int m = 0; m < 6; ++m) SBV[i * SB + m * 16 + lr] = sb[m][r];
#pragma unroll
        for (int c = 0; c < 3; ++c) SBV[i * SB + (6 + c) * 16 + lr] = vb[c][r];
      }
    }
  }
  // own strains of the forward state (gradient), B operand of eps_q = Vq eps
  T* Sown = r1;  // [NpK][SE]
  if (grad) {
    for (int x = tid; x < E * 6 * NpK; x += NT) {
      const int e = x / (6 * NpK), rem = x % (6 * NpK), m = rem / NpK, j = rem % NpK;
      Sown[j * SE + m * 16 + e] = (e < ne && j < Np) ? a.q[(e0 + e) * 9 * Np + (3 + m) * Np + j] : T(0);
    }
  }
  __syncthreads();

  // ---- 2. face sensitivities of both sides, face by face
  T* zf = r3;    // [E][4][Nfp][2]
  constexpr int FPT = (E * Nfp + NT - 1) / NT;
  // own and neighbour-side sensitivities of all four faces, loads issued together
  T fsum[FPT][4][8];
#pragma unroll
  for (int p = 0; p < FPT; ++p) {
    const int x = tid + p * NT;
    const int e = x / Nfp, j = x % Nfp;
    const bool ok = x < E * Nfp && e < ne;
    const int ee = ok ? e : 0;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const int32_t wd = ok ? a.conn[(e0 + ee) * 4 + f] : static_cast<int32_t>((e0 * 4) << 5);
      const int64_t nb = wd >> 5;
      const int code = wd & 31;
      const int jn = a.nbrface[((f * 4 + code / 6) * 6 + code % 6) * Nfp + (ok ? j : 0)];
      const T* fo = a.fown + (((e0 + ee) * 4 + f) * Nfp + (ok ? j : 0)) * 8;
      const T* fn = a.fnbr + ((nb * 4 + code / 6) * Nfp + jn) * 8;
#pragma unroll
      for (int c = 0; c < 3; ++c) fsum[p][f][c] = fo[c] + fn[c];
#pragma unroll
      for (int c = 0; c < 3; ++c) fsum[p][f][3 + c] = fo[3 + c] - fn[3 + c];
      fsum[p][f][6] = fo[6] + fn[6];
      fsum[p][f][7] = fo[7] + fn[7];
    }
  }
#pragma unroll
  for (int f = 0; f < 4; ++f) {
#pragma unroll
    for (int p = 0; p < FPT; ++p) {
      const int x = tid + p * NT;
      const int e = x / Nfp, j = x % Nfp;
      if (x >= E * Nfp || e >= ne) continue;
      const int il = a.fmask[f * Nfp + j];
      const T* gg = &sgeo[e * 32];
      const T n[3] = {gg[9 + f * 4], gg[9 + f * 4 + 1], gg[9 + f * 4 + 2]};
      const T* fs = fsum[p][f];
      T* row = &SBV[il * SB + e];
      const T* Te = fs + 3;   // own traction sensitivity minus the neighbour's (its normal is -n)
#pragma unroll
      for (int c = 0; c < 3; ++c) row[(6 + c) * 16] += fs[c];
      row[0 * 16] += Te[0] * n[0];
      row[1 * 16] += Te[1] * n[1];
      row[2 * 16] += Te[2] * n[2];
      row[3 * 16] += Te[1] * n[2] + Te[2] * n[1];
      row[4 * 16] += Te[0] * n[2] + Te[2] * n[0];
      row[5 * 16] += Te[0] * n[1] + Te[1] * n[0];
      zf[(e * 4 * Nfp + f * Nfp + j) * 2] = fs[6];
      zf[(e * 4 * Nfp + f * Nfp + j) * 2 + 1] = fs[7];
    }
    __syncthreads();
  }
  if (grad) {
    for (int e = tid; e < ne; e += NT) {
      double zp = 0, zs = 0;
      for (int x = 0; x < 4 * Nfp; ++x) {
        zp += static_cast<double>(zf[(e * 4 * Nfp + x) * 2]);
        zs += static_cast<double>(zf[(e * 4 * Nfp + x) * 2 + 1]);
      }
      zsum[e * 2] = zp;
      zsum[e * 2 + 1] = zs;
    }
  }
  __syncthreads();

  // ---- 3./4. transposed projection, chunk by chunk
  T* Qd = r3;    // [QC][SQ]
  acc_t eb[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) eb[m] = acc_t{0, 0, 0, 0};
  T gl_acc = 0, gm_acc = 0;
  const int ec = lr < ne ? lr : ne - 1;
#pragma unroll 1
  for (int qc = 0; qc < NQC; ++qc) {
    const int q0 = qc * QC;
    const int rows = (NqK - q0) < QC ? (NqK - q0) : QC;
#pragma unroll 1
    for (int Rq = q0 / 16 + w; Rq < QT && Rq * 16 < q0 + QC; Rq += NW) {
      T pf[KD];
      const T* Pr = a.PqTpad + (Rq * KD) * 64 + l;
#pragma unroll
      for (int kk = 0; kk < KD; ++kk) pf[kk] = Pr[kk * 64];
      acc_t tau[6];
#pragma unroll
      for (int m = 0; m < 6; ++m) tau[m] = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < KD; ++kk) {
        const int row = (4 * kk + lg) * SB + lr;
#pragma unroll
        for (int m = 0; m < 6; ++m) tau[m] = M::mma(pf[kk], SBV[row + m * 16], tau[m]);
      }
      acc_t ep[6];
#pragma unroll
      for (int m = 0; m < 6; ++m) ep[m] = acc_t{0, 0, 0, 0};
      if (grad) {
        T vf[KD];
        const T* Vr = a.Vqpad + (Rq * KD) * 64 + l;
#pragma unroll
        for (int kk = 0; kk < KD; ++kk) vf[kk] = Vr[kk * 64];
#pragma unroll
        for (int kk = 0; kk < KD; ++kk) {
          const int row = (4 * kk + lg) * SE + lr;
#pragma unroll
          for (int m = 0; m < 6; ++m) ep[m] = M::mma(vf[kk], Sown[row + m * 16], ep[m]);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = Rq * 16 + M::row(lg, r);
        if (q >= NqK) continue;
        const bool ok = q < Nq && lr < ne;
        const int qq = q < Nq ? q : Nq - 1;
        const T lam = ok ? a.lm[(e0 + ec) * 2 * NqP + qq] : T(0);
        const T mu = ok ? a.lm[(e0 + ec) * 2 * NqP + NqP + qq] : T(0);
        const T trt = tau[0][r] + tau[1][r] + tau[2][r];
        T* o = &Qd[(q - q0) * SQ + lr];
#pragma unroll
        for (int m = 0; m < 6; ++m) o[m * 16] = T(2) * mu * tau[m][r] + (m < 3 ? lam * trt : T(0));
        if (grad) {
          const T tr = ep[0][r] + ep[1][r] + ep[2][r];
          T pm = 0;
#pragma unroll
          for (int m = 0; m < 6; ++m) pm += tau[m][r] * ep[m][r];
          gl_acc += lam * tr * trt;
          gm_acc += T(2) * mu * pm;
        }
      }
    }
    __syncthreads();
    if (own) {
      const T* Vt = a.VqTpad + (R * (NqK / 4) + q0 / 4) * 64 + l;
#pragma unroll
      for (int u = 0; u < KQ; ++u) {
        if (4 * u < rows) {
          const T vt = Vt[u * 64];
          const int row = (4 * u + lg) * SQ + lr;
#pragma unroll
          for (int m = 0; m < 6; ++m) eb[m] = M::mma(vt, Qd[row + m * 16], eb[m]);
        }
      }
    }
    __syncthreads();
  }

  // ---- 5. outputs
  T* Seb = r1;   // [NpK][SE] epsbar (the own strains are no longer needed)
  if (own) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = R * 16 + M::row(lg, r);
      if (i < Np) {
#pragma unroll
        for (int m = 0; m < 6; ++m) Seb[i * SE + m * 16 + lr] = eb[m][r];
      }
    }
  }
  red[(w * 64 + l) * 2] = gl_acc;
  red[(w * 64 + l) * 2 + 1] = gm_acc;
  __syncthreads();
  for (int x = tid; x < ne * 9 * Np; x += NT) {
    const int e = x / (9 * Np), c = (x / Np) % 9, j = x % Np;
    const T v = (c < 3) ? SBV[j * SB + (6 + c) * 16 + e] : Seb[j * SE + (c - 3) * 16 + e];
    a.qbar[e0 * 9 * Np + x] += a.scale * v;
  }
  if (!grad) {
    if (a.rupd) {
      __syncthreads();
      fused_recurrence<T, Np>(a, e0, ne, tid, NT);
    }
    return;
  }
  T* pr = r3;    // [E][Np] density partials (the chunk buffer is free)
  for (int x = tid; x < ne * Np; x += NT) {
    const int e = x / Np, j = x % Np;
    T p = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c)
      p += a.y[(e0 + e) * 9 * Np + c * Np + j] * a.rhs[(e0 + e) * a.rhs_es + c * Np + j];
    pr[e * Np + j] = -p;
  }
  __syncthreads();
  for (int e = tid; e < ne; e += NT) {
    double gr = 0, gl = 0, gm = 0;
    for (int j = 0; j < Np; ++j) gr += static_cast<double>(pr[e * Np + j]);
    for (int ww = 0; ww < NW; ++ww)
      for (int g4 = 0; g4 < 4; ++g4) {
        gl += static_cast<double>(red[(ww * 64 + g4 * 16 + e) * 2]);
        gm += static_cast<double>(red[(ww * 64 + g4 * 16 + e) * 2 + 1]);
      }
    const double zp = zsum[e * 2], zs = zsum[e * 2 + 1];
    // chain rule through Z_p = sqrt(rho (lambda + 2 mu)), Z_s = sqrt(rho mu)
    const double* mn = a.means + (e0 + e) * 3;
    const double Zp = sqrt(mn[0] * (mn[1] + 2.0 * mn[2])), Zs = sqrt(mn[0] * mn[2]);
    gr += 0.5 * Zp * zp + 0.5 * Zs * zs;
    gl += mn[0] * mn[1] / (2.0 * Zp) * zp;
    gm += mn[0] * mn[2] / Zp * zp + 0.5 * Zs * zs;
    const double sc = static_cast<double>(a.scale);
    a.g[(e0 + e) * 3 + 0] += sc * gr;
    a.g[(e0 + e) * 3 + 1] += sc * gl;
    a.g[(e0 + e) * 3 + 2] += sc * gm;
  }
  if (a.rupd) fused_recurrence<T, Np>(a, e0, ne, tid, NT);   // y was last read before the barrier above
}

// qbar_v(receiver element) += scale * l(x_r) resid_r, receivers in order.
template <typename T, int N>
__global__ __launch_bounds__(256) void k_adj_receivers(T* qbar, const double* rows, const int32_t* elem,
                                                       const double* resid, int nr, double scale) {
  constexpr int Np = Sz<N>::Np;
  for (int r = 0; r < nr; ++r) {
    const int64_t e = elem[r];
    for (int x = threadIdx.x; x < 3 * Np; x += blockDim.x) {
      const int c = x / Np, i = x % Np;
      qbar[e * 9 * Np + c * Np + i] += static_cast<T>(scale * rows[r * Np + i] * resid[r * 3 + c]);
    }
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_axpy(T* y, const T* x, T a, int64_t n) {
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += static_cast<int64_t>(gridDim.x) * 256)
    y[i] += a * x[i];
}

template <typename T>
static AdjArgs<T> adj_args(const Dev& d, const AdjDev& ad, const void* y, const void* q, const void* s,
                           const void* rhs, int rhs_es, void* qbar, double* g, double scale, void* rupd,
                           double ra, double rb) {
  AdjArgs<T> a;
  a.y = static_cast<const T*>(y);
  a.q = static_cast<const T*>(q);
  a.s = static_cast<const T*>(s);
  a.rhs = static_cast<const T*>(rhs);
  a.rhs_es = rhs_es;
  a.ytil = static_cast<T*>(ad.ytil);
  a.fown = static_cast<T*>(ad.fown);
  a.fnbr = static_cast<T*>(ad.fnbr);
  a.qbar = static_cast<T*>(qbar);
  a.g = g;
  a.W = static_cast<const T*>(d.W);
  a.lm = static_cast<const T*>(d.lm);
  a.geo = static_cast<const T*>(d.geo);
  a.fgeo = static_cast<const T*>(d.fgeo);
  a.Z = static_cast<const T*>(d.Z);
  a.means = d.means64;
  a.conn = d.conn;
  a.nbrnode = d.nbrnode;
  a.nbrface = d.nbrface;
  a.fmask = d.fmask;
  a.Dk = static_cast<const T*>(d.Dk);
  a.LIFT = static_cast<const T*>(d.LIFTr);
  a.Vq = static_cast<const T*>(d.Vqr);
  a.VqT = static_cast<const T*>(d.VqT);
  a.Pq = static_cast<const T*>(d.Pqr);
  a.DTpad = static_cast<const T*>(d.DTpad);
  a.PqTpad = static_cast<const T*>(d.PqTpad);
  a.VqTpad = static_cast<const T*>(d.VqTpad);
  a.Vqpad = static_cast<const T*>(d.Vqpad);
  a.K = d.K;
  a.scale = static_cast<T>(scale);
  a.rupd = static_cast<T*>(rupd);
  a.ra = static_cast<T>(ra);
  a.rb = static_cast<T>(rb);
  return a;
}

template <typename T, int N>
static hipError_t adjoint_impl(const Dev& d, const AdjDev& ad, const void* y, const void* q, const void* s,
                               const void* rhs, int rhs_es, void* qbar, double* g, double scale,
                               void* rupd, double ra, double rb, hipStream_t st) {
  using C = AdjCfg<T, N>;
  const AdjArgs<T> a = adj_args<T>(d, ad, y, q, s, rhs, rhs_es, qbar, g, scale, rupd, ra, rb);
  const unsigned grid = static_cast<unsigned>((d.K + C::E - 1) / C::E);
  hipLaunchKernelGGL((k_adjA<T, N>), dim3(grid), dim3(C::NT), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if constexpr (AdjTile<T, N>::fits && EWDG_ADJ_MMA) {
    const unsigned gridm = static_cast<unsigned>((d.K + Tile<N>::E - 1) / Tile<N>::E);
    hipLaunchKernelGGL((k_adjB_mma<T, N>), dim3(gridm), dim3(Tile<N>::NT), 0, st, a);
  } else {
    hipLaunchKernelGGL((k_adjB<T, N>), dim3(grid), dim3(C::NT), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_adjoint(const Dev& d, const AdjDev& ad, const void* y, const void* q, const void* s,
                          const void* rhs, int rhs_es, void* qbar, double* g, double scale, void* rupd, double ra,
                          double rb, hipStream_t st) {
  if (rupd && rupd != y) return hipErrorInvalidValue;   // the fused recurrence updates y itself
  if (d.prec == 32) {
    EWDG_DISPATCH(d.N,
                  return (adjoint_impl<float, NN>(d, ad, y, q, s, rhs, rhs_es, qbar, g, scale, rupd, ra, rb, st)));
  }
  EWDG_DISPATCH(d.N,
                return (adjoint_impl<double, NN>(d, ad, y, q, s, rhs, rhs_es, qbar, g, scale, rupd, ra, rb, st)));
}

hipError_t launch_adj_receivers(const Dev& d, void* qbar, const double* resid, int nr, double scale,
                                hipStream_t st) {
  if (nr <= 0) return hipSuccess;
  if (d.prec == 32) {
    EWDG_DISPATCH(d.N, hipLaunchKernelGGL((k_adj_receivers<float, NN>), dim3(1), dim3(256), 0, st,
                                          static_cast<float*>(qbar), d.rec_rows, d.rec_elem, resid, nr, scale);
                  return hipGetLastError());
  }
  EWDG_DISPATCH(d.N, hipLaunchKernelGGL((k_adj_receivers<double, NN>), dim3(1), dim3(256), 0, st,
                                        static_cast<double*>(qbar), d.rec_rows, d.rec_elem, resid, nr, scale);
                return hipGetLastError());
}

hipError_t launch_axpy(int prec, void* y, const void* x, double a, int64_t n, hipStream_t st) {
  const unsigned grid = static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 65536));
  if (prec == 32)
    hipLaunchKernelGGL((k_axpy<float>), dim3(grid), dim3(256), 0, st, static_cast<float*>(y),
                       static_cast<const float*>(x), static_cast<float>(a), n);
  else
    hipLaunchKernelGGL((k_axpy<double>), dim3(grid), dim3(256), 0, st, static_cast<double*>(y),
                       static_cast<const double*>(x), a, n);
  return hipGetLastError();
}

}  // namespace ewdg
