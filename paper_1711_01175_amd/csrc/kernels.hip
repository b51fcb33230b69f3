// HIP kernels for gfx950: material setup (FP64), the fused LSRK stage
// (volume derivatives, upwind interface flux, lift, density-weighted mass
// inverse, RK update and the stress projection of the new state), and the
// FP64 diagnostics (projection, evaluation, receivers, energy).
#include <hip/hip_runtime.h>

#include "dev.hpp"

namespace ewdg {

template <int N>
struct Sz {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;
  static constexpr int Nq = (N + 1) * (N + 1) * (N + 1);
  static constexpr int NF = 4 * Nfp;
  static constexpr int cmax(int a, int b) { return a > b ? a : b; }
  static constexpr int BUF = cmax(9 * Np, cmax(9 * NF, 6 * Nq));
};

// Elements per workgroup of the stage kernel: as many as fill ~256 node
// threads while the staged element data stays within 64 KiB of LDS.
template <typename T, int N>
struct StageCfg {
  using S = Sz<N>;
  static constexpr int per_elem = 18 * S::Np + S::BUF + 32;
  static constexpr int e_lds = (64 * 1024) / (per_elem * static_cast<int>(sizeof(T)));
  static constexpr int e_thr = 256 / S::Np > 0 ? 256 / S::Np : 1;
  static constexpr int E = (e_lds < e_thr ? e_lds : e_thr) > 0 ? (e_lds < e_thr ? e_lds : e_thr) : 1;
  static constexpr int NT = ((E * S::Np + 63) / 64) * 64;
};

template <typename T>
struct StageArgs {
  const T* qin;
  const T* sin;
  T* qout;
  T* sout;
  T* out;        // rhs (mode 0) or the LSRK register (mode 1)
  const T* W;
  const T* lm;
  const T* geo;
  const T* fgeo;
  const T* Z;
  const T* svec;
  const T* DrT;
  const T* DsT;
  const T* DtT;
  const T* LIFTT;
  const T* VqT;
  const T* PqT;
  const int32_t* conn;
  const int32_t* nbrnode;
  const int32_t* fmask;
  int64_t K;
  T a, b, dt, srcval;
  T dir0, dir1, dir2;
  int64_t src_elem;
};

// Exact Riemann state per wave mode at one face point (outward normal n of
// the own element).  Returns the velocity-equation correction T* - T^- and
// the velocity jump v* - v^- that drives the strain correction.
template <typename T>
__device__ __forceinline__ void interface_state(const T* n, const T* vm, const T* Tm, const T* vp,
                                                 const T* Tp, T zpm, T zpp, T zsm, T zsp,
                                                 T* dT, T* dv) {
  const T vmn = vm[0] * n[0] + vm[1] * n[1] + vm[2] * n[2];
  const T vpn = vp[0] * n[0] + vp[1] * n[1] + vp[2] * n[2];
  const T Tmn = Tm[0] * n[0] + Tm[1] * n[1] + Tm[2] * n[2];
  const T Tpn = Tp[0] * n[0] + Tp[1] * n[1] + Tp[2] * n[2];
  const T ip = T(1) / (zpm + zpp);
  const T is = T(1) / (zsm + zsp);
  // normal mode: T*_n - T^-_n and v*_n - v^-_n
  const T dTn = zpm * ((Tpn - Tmn) + zpp * (vpn - vmn)) * ip;
  const T dvn = ((Tpn - Tmn) + zpp * (vpn - vmn)) * ip;
  // tangential modes
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T vmt = vm[c] - vmn * n[c], vpt = vp[c] - vpn * n[c];
    const T Tmt = Tm[c] - Tmn * n[c], Tpt = Tp[c] - Tpn * n[c];
    const T jt = (Tpt - Tmt) + zsp * (vpt - vmt);
    dT[c] = zsm * jt * is + dTn * n[c];
    dv[c] = jt * is + dvn * n[c];
  }
}

template <typename T, int N, int MODE>
__global__ __launch_bounds__((StageCfg<T, N>::NT)) void k_stage(StageArgs<T> a) {
  using S = Sz<N>;
  using C = StageCfg<T, N>;
  constexpr int Np = S::Np, Nfp = S::Nfp, Nq = S::Nq, NF = S::NF, BUF = S::BUF;
  constexpr int E = C::E, NT = C::NT;
  __shared__ T sq[E * 9 * Np];
  __shared__ T ss[E * 6 * Np];
  __shared__ T sb[E * BUF];
  __shared__ T sr[E * 3 * Np];
  __shared__ T sg[E * 32];
  const int tid = threadIdx.x;
  const int64_t e0 = static_cast<int64_t>(blockIdx.x) * E;
  const int ne = static_cast<int>((a.K - e0) < E ? (a.K - e0) : E);

  for (int x = tid; x < ne * 9 * Np; x += NT) sq[x] = a.qin[e0 * 9 * Np + x];
  for (int x = tid; x < ne * 6 * Np; x += NT) ss[x] = a.sin[e0 * 6 * Np + x];
  for (int x = tid; x < ne * 27; x += NT) {
    const int e = x / 27, m = x % 27;
    T v;
    if (m < 9) v = a.geo[(e0 + e) * 9 + m];
    else if (m < 25) v = a.fgeo[(e0 + e) * 16 + (m - 9)];
    else v = a.Z[(e0 + e) * 2 + (m - 25)];
    sg[e * 32 + m] = v;
  }
  __syncthreads();

  // Contravariant stress components G_c^k = sum_m (dr_k/dx_m) sigma_cm.
  for (int x = tid; x < ne * Np; x += NT) {
    const int e = x / Np, j = x % Np;
    const T* sp = &ss[e * 6 * Np + j];
    const T sxx = sp[0], syy = sp[Np], szz = sp[2 * Np], syz = sp[3 * Np], sxz = sp[4 * Np],
            sxy = sp[5 * Np];
    const T row[3][3] = {{sxx, sxy, sxz}, {sxy, syy, syz}, {sxz, syz, szz}};
    const T* g = &sg[e * 32];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int k = 0; k < 3; ++k)
        sb[e * BUF + (c * 3 + k) * Np + j] =
            g[k * 3 + 0] * row[c][0] + g[k * 3 + 1] * row[c][1] + g[k * 3 + 2] * row[c][2];
  }
  __syncthreads();

  const bool act = tid < ne * Np;
  const int e = act ? tid / Np : 0, i = act ? tid % Np : 0;
  T rhs[9];
  if (act) {
    T div[3] = {0, 0, 0};
    T gv[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    const T* G = &sb[e * BUF];
    const T* v = &sq[e * 9 * Np];
    for (int j = 0; j < Np; ++j) {
      const T dr = a.DrT[j * Np + i], ds = a.DsT[j * Np + i], dt = a.DtT[j * Np + i];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        div[c] += dr * G[(c * 3 + 0) * Np + j] + ds * G[(c * 3 + 1) * Np + j] +
                  dt * G[(c * 3 + 2) * Np + j];
        const T vc = v[c * Np + j];
        gv[c][0] += dr * vc;
        gv[c][1] += ds * vc;
        gv[c][2] += dt * vc;
      }
    }
    const T* g = &sg[e * 32];
    T gr[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int m = 0; m < 3; ++m)
        gr[c][m] = g[0 * 3 + m] * gv[c][0] + g[1 * 3 + m] * gv[c][1] + g[2 * 3 + m] * gv[c][2];
    rhs[0] = div[0];
    rhs[1] = div[1];
    rhs[2] = div[2];
    rhs[3] = gr[0][0];
    rhs[4] = gr[1][1];
    rhs[5] = gr[2][2];
    rhs[6] = T(0.5) * (gr[1][2] + gr[2][1]);
    rhs[7] = T(0.5) * (gr[0][2] + gr[2][0]);
    rhs[8] = T(0.5) * (gr[0][1] + gr[1][0]);
  }
  __syncthreads();

  // Interface corrections at every face node, scaled by Fscale.
  for (int x = tid; x < ne * NF; x += NT) {
    const int ee = x / NF, fj = x % NF, f = fj / Nfp, j = fj % Nfp;
    const int il = a.fmask[f * Nfp + j];
    const T* gg = &sg[ee * 32];
    const T n[3] = {gg[9 + f * 4 + 0], gg[9 + f * 4 + 1], gg[9 + f * 4 + 2]};
    const T fs = gg[9 + f * 4 + 3];
    T vm[3], sm[6], vp[3], sp[6];
#pragma unroll
    for (int c = 0; c < 3; ++c) vm[c] = sq[ee * 9 * Np + c * Np + il];
#pragma unroll
    for (int m = 0; m < 6; ++m) sm[m] = ss[ee * 6 * Np + m * Np + il];
    const int32_t w = a.conn[(e0 + ee) * 4 + f];
    const int64_t nb = w >> 5;
    const int code = w & 31;
    const int nn = a.nbrnode[((f * 4 + code / 6) * 6 + code % 6) * Nfp + j];
#pragma unroll
    for (int c = 0; c < 3; ++c) vp[c] = a.qin[nb * 9 * Np + c * Np + nn];
#pragma unroll
    for (int m = 0; m < 6; ++m) sp[m] = a.sin[nb * 6 * Np + m * Np + nn];
    const T Tm[3] = {sm[0] * n[0] + sm[5] * n[1] + sm[4] * n[2],
                     sm[5] * n[0] + sm[1] * n[1] + sm[3] * n[2],
                     sm[4] * n[0] + sm[3] * n[1] + sm[2] * n[2]};
    const T Tp[3] = {sp[0] * n[0] + sp[5] * n[1] + sp[4] * n[2],
                     sp[5] * n[0] + sp[1] * n[1] + sp[3] * n[2],
                     sp[4] * n[0] + sp[3] * n[1] + sp[2] * n[2]};
    T dT[3], dv[3];
    interface_state(n, vm, Tm, vp, Tp, gg[25], a.Z[nb * 2], gg[26], a.Z[nb * 2 + 1], dT, dv);
    T* fl = &sb[ee * BUF + fj];
    fl[0 * NF] = fs * dT[0];
    fl[1 * NF] = fs * dT[1];
    fl[2 * NF] = fs * dT[2];
    fl[3 * NF] = fs * n[0] * dv[0];
    fl[4 * NF] = fs * n[1] * dv[1];
    fl[5 * NF] = fs * n[2] * dv[2];
    fl[6 * NF] = fs * T(0.5) * (n[1] * dv[2] + n[2] * dv[1]);
    fl[7 * NF] = fs * T(0.5) * (n[0] * dv[2] + n[2] * dv[0]);
    fl[8 * NF] = fs * T(0.5) * (n[0] * dv[1] + n[1] * dv[0]);
  }
  __syncthreads();

  if (act) {
    const T* fl = &sb[e * BUF];
    for (int m = 0; m < NF; ++m) {
      const T L = a.LIFTT[m * Np + i];
#pragma unroll
      for (int c = 0; c < 9; ++c) rhs[c] += L * fl[c * NF + m];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) sr[e * 3 * Np + c * Np + i] = rhs[c];
  }
  __syncthreads();

  if (act) {
    const int64_t ge = e0 + e;
    const T* W = a.W + ge * Np * Np;
    T o0 = 0, o1 = 0, o2 = 0;
    const T* r = &sr[e * 3 * Np];
    for (int j = 0; j < Np; ++j) {
      const T wv = W[j * Np + i];
      o0 += wv * r[j];
      o1 += wv * r[Np + j];
      o2 += wv * r[2 * Np + j];
    }
    if (ge == a.src_elem) {
      const T sv = a.srcval * a.svec[i];
      o0 += sv * a.dir0;
      o1 += sv * a.dir1;
      o2 += sv * a.dir2;
    }
    rhs[0] = o0;
    rhs[1] = o1;
    rhs[2] = o2;
    if (MODE == 0) {
#pragma unroll
      for (int c = 0; c < 9; ++c) a.out[ge * 9 * Np + c * Np + i] = rhs[c];
    } else {
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        const int64_t idx = ge * 9 * Np + c * Np + i;
        const T rr = a.a * a.out[idx] + a.dt * rhs[c];
        a.out[idx] = rr;
        const T qn = sq[e * 9 * Np + c * Np + i] + a.b * rr;
        a.qout[idx] = qn;
        sq[e * 9 * Np + c * Np + i] = qn;
      }
    }
  }
  if (MODE == 0) return;
  __syncthreads();

  // sigma_h of the new state: strains at the quadrature points, Hooke's law
  // with the sampled lambda, mu, and the L2_Q projection back to the nodes.
  for (int x = tid; x < ne * Nq; x += NT) {
    const int ee = x / Nq, qp = x % Nq;
    T ep[6] = {0, 0, 0, 0, 0, 0};
    const T* qq = &sq[ee * 9 * Np + 3 * Np];
    for (int j = 0; j < Np; ++j) {
      const T vv = a.VqT[j * Nq + qp];
#pragma unroll
      for (int m = 0; m < 6; ++m) ep[m] += vv * qq[m * Np + j];
    }
    const T lam = a.lm[(e0 + ee) * 2 * Nq + qp], mu = a.lm[(e0 + ee) * 2 * Nq + Nq + qp];
    const T ltr = lam * (ep[0] + ep[1] + ep[2]);
    T* o = &sb[ee * BUF + qp];
#pragma unroll
    for (int m = 0; m < 6; ++m) o[m * Nq] = T(2) * mu * ep[m] + (m < 3 ? ltr : T(0));
  }
  __syncthreads();
  if (act) {
    T sh[6] = {0, 0, 0, 0, 0, 0};
    const T* sqp = &sb[e * BUF];
    for (int qp = 0; qp < Nq; ++qp) {
      const T pv = a.PqT[qp * Np + i];
#pragma unroll
      for (int m = 0; m < 6; ++m) sh[m] += pv * sqp[m * Nq + qp];
    }
#pragma unroll
    for (int m = 0; m < 6; ++m) a.sout[(e0 + e) * 6 * Np + m * Np + i] = sh[m];
  }
}

// sigma_h = P_Q(lambda tr(e) I + 2 mu e) for a given state (no update).
template <typename T, int N>
__global__ __launch_bounds__(256) void k_sigma(const T* __restrict__ q, T* __restrict__ s,
                                               const T* __restrict__ lm, const T* __restrict__ VqT,
                                               const T* __restrict__ PqT, int64_t K) {
  using S = Sz<N>;
  constexpr int Np = S::Np, Nq = S::Nq;
  __shared__ T se[6 * Np];
  __shared__ T sg[6 * Nq];
  const int64_t e = blockIdx.x;
  for (int x = threadIdx.x; x < 6 * Np; x += 256) se[x] = q[e * 9 * Np + 3 * Np + x];
  __syncthreads();
  for (int qp = threadIdx.x; qp < Nq; qp += 256) {
    T ep[6] = {0, 0, 0, 0, 0, 0};
    for (int j = 0; j < Np; ++j) {
      const T vv = VqT[j * Nq + qp];
      for (int m = 0; m < 6; ++m) ep[m] += vv * se[m * Np + j];
    }
    const T lam = lm[e * 2 * Nq + qp], mu = lm[e * 2 * Nq + Nq + qp];
    const T ltr = lam * (ep[0] + ep[1] + ep[2]);
    for (int m = 0; m < 6; ++m) sg[m * Nq + qp] = T(2) * mu * ep[m] + (m < 3 ? ltr : T(0));
  }
  __syncthreads();
  for (int x = threadIdx.x; x < 6 * Np; x += 256) {
    const int m = x / Np, i = x % Np;
    T acc = 0;
    for (int qp = 0; qp < Nq; ++qp) acc += PqT[qp * Np + i] * sg[m * Nq + qp];
    s[e * 6 * Np + x] = acc;
  }
}

// In-place Gauss-Jordan inverse of an SPD matrix by one workgroup.
__device__ void gj_invert(double* M, int n) {
  for (int k = 0; k < n; ++k) {
    __syncthreads();
    const double p = 1.0 / M[k * n + k];
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += blockDim.x) M[k * n + j] = (j == k) ? p : M[k * n + j] * p;
    __syncthreads();
    for (int x = threadIdx.x; x < n * n; x += blockDim.x) {
      const int i = x / n, j = x % n;
      if (i != k && j != k) M[x] -= M[i * n + k] * M[k * n + j];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x)
      if (i != k) M[i * n + k] = -M[i * n + k] * p;
  }
  __syncthreads();
}

// M = Vq^T diag(w rho) Vq for one element (without the Jacobian).
template <int N>
__device__ void build_mass(const Dev& d, int64_t e, double* M, double* wr) {
  using S = Sz<N>;
  constexpr int Np = S::Np, Nq = S::Nq;
  for (int q = threadIdx.x; q < Nq; q += blockDim.x) wr[q] = d.wq64[q] * d.rho64[e * Nq + q];
  __syncthreads();
  for (int x = threadIdx.x; x < Np * Np; x += blockDim.x) {
    const int i = x / Np, j = x % Np;
    if (j < i) continue;
    double acc = 0.0;
    for (int q = 0; q < Nq; ++q) acc += d.Vq64T[i * Nq + q] * wr[q] * d.Vq64T[j * Nq + q];
    M[i * Np + j] = acc;
    M[j * Np + i] = acc;
  }
  __syncthreads();
}

template <typename T, int N, bool LDS>
__global__ __launch_bounds__(256) void k_material(Dev d, int64_t e_begin) {
  using S = Sz<N>;
  constexpr int Np = S::Np, Nq = S::Nq;
  constexpr int MS = LDS ? Np * Np : 1;
  __shared__ double sM[MS];
  __shared__ double wr[Nq];
  __shared__ double red[3 * 256];
  const int64_t e = e_begin + blockIdx.x;
  double* M = LDS ? sM : static_cast<double*>(d.scratch) + static_cast<int64_t>(blockIdx.x) * Np * Np;
  build_mass<N>(d, e, M, wr);
  gj_invert(M, Np);
  // W = (Vq^T diag(w rho) Vq)^-1 Mhat = M_rho^-1 M (the Jacobian cancels),
  // stored transposed per element: W[e][j][i] = W_ij.
  T* W = static_cast<T*>(d.W) + e * Np * Np;
  for (int x = threadIdx.x; x < Np * Np; x += blockDim.x) {
    const int i = x / Np, j = x % Np;
    double acc = 0.0;
    for (int k = 0; k < Np; ++k) acc += M[i * Np + k] * d.Mhat64[k * Np + j];
    W[j * Np + i] = static_cast<T>(acc);
  }
  // run-precision lambda, mu and the impedances from the element means
  T* lm = static_cast<T*>(d.lm) + e * 2 * Nq;
  double a0 = 0, a1 = 0, a2 = 0;
  for (int q = threadIdx.x; q < Nq; q += blockDim.x) {
    const double w = d.wq64[q];
    lm[q] = static_cast<T>(d.lam64[e * Nq + q]);
    lm[Nq + q] = static_cast<T>(d.mu64[e * Nq + q]);
    a0 += w * d.rho64[e * Nq + q];
    a1 += w * d.lam64[e * Nq + q];
    a2 += w * d.mu64[e * Nq + q];
  }
  red[threadIdx.x] = a0;
  red[256 + threadIdx.x] = a1;
  red[512 + threadIdx.x] = a2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0, l = 0, m = 0, ws = 0;
    for (int t = 0; t < static_cast<int>(blockDim.x); ++t) {
      r += red[t];
      l += red[256 + t];
      m += red[512 + t];
    }
    for (int q = 0; q < Nq; ++q) ws += d.wq64[q];
    r /= ws;
    l /= ws;
    m /= ws;
    T* Z = static_cast<T*>(d.Z) + e * 2;
    Z[0] = static_cast<T>(sqrt(r * (l + 2.0 * m)));
    Z[1] = static_cast<T>(sqrt(r * m));
  }
}

// Source vector M_rho^-1 phi(x_s) of the owning element.
template <typename T, int N>
__global__ __launch_bounds__(256) void k_source_vector(Dev d, int64_t e) {
  using S = Sz<N>;
  constexpr int Np = S::Np, Nq = S::Nq;
  __shared__ double wr[Nq];
  double* M = d.msmall;
  build_mass<N>(d, e, M, wr);
  gj_invert(M, Np);
  const double J = d.J64[e];
  for (int i = threadIdx.x; i < Np; i += blockDim.x) {
    double acc = 0.0;
    for (int k = 0; k < Np; ++k) acc += M[i * Np + k] * d.srcb[k];
    static_cast<T*>(d.svec)[i] = static_cast<T>(acc / J);
  }
}

// FP64 L2_Q projection of quadrature values to nodes: q = Pq fq.
template <typename T, int N>
__global__ __launch_bounds__(256) void k_project(Dev d, const double* __restrict__ fq, T* q) {
  using S = Sz<N>;
  constexpr int Np = S::Np, Nq = S::Nq;
  const int64_t e = blockIdx.x;
  for (int x = threadIdx.x; x < 9 * Np; x += 256) {
    const int c = x / Np, i = x % Np;
    const double* f = fq + (e * 9 + c) * Nq;
    double acc = 0.0;
    for (int qp = 0; qp < Nq; ++qp) acc += d.Pq64T[qp * Np + i] * f[qp];
    q[e * 9 * Np + x] = static_cast<T>(acc);
  }
}

// FP64 evaluation at the quadrature points: fq = Vq q.
template <typename T, int N>
__global__ __launch_bounds__(256) void k_evalq(Dev d, const T* __restrict__ q, double* fq) {
  using S = Sz<N>;
  constexpr int Np = S::Np, Nq = S::Nq;
  const int64_t e = blockIdx.x;
  __shared__ double sqv[9 * Np];
  for (int x = threadIdx.x; x < 9 * Np; x += 256) sqv[x] = static_cast<double>(q[e * 9 * Np + x]);
  __syncthreads();
  for (int x = threadIdx.x; x < 9 * Nq; x += 256) {
    const int c = x / Nq, qp = x % Nq;
    double acc = 0.0;
    for (int i = 0; i < Np; ++i) acc += d.Vq64T[i * Nq + qp] * sqv[c * Np + i];
    fq[e * 9 * Nq + x] = acc;
  }
}

// Receivers: v(x_r) = sum_i l_i(x_r) v_i accumulated in FP64.
template <typename T, int N>
__global__ __launch_bounds__(64) void k_receivers(Dev d, const T* __restrict__ q, int nr, int step) {
  using S = Sz<N>;
  constexpr int Np = S::Np;
  const int r = blockIdx.x;
  const int lane = threadIdx.x;
  const int64_t e = d.rec_elem[r];
  for (int c = 0; c < 3; ++c) {
    double acc = 0.0;
    for (int i = lane; i < Np; i += 64) acc += d.rec_rows[r * Np + i] * static_cast<double>(q[e * 9 * Np + c * Np + i]);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) d.rec_out[(static_cast<int64_t>(step) * nr + r) * 3 + c] = acc;
  }
}

// Per-element energy 1/2 J sum_q w (rho |v|^2 + e:sigma) in FP64.
template <typename T, int N>
__global__ __launch_bounds__(256) void k_energy(Dev d, const T* __restrict__ q) {
  using S = Sz<N>;
  constexpr int Np = S::Np, Nq = S::Nq;
  const int64_t e = blockIdx.x;
  __shared__ double sqv[9 * Np];
  __shared__ double red[256];
  for (int x = threadIdx.x; x < 9 * Np; x += 256) sqv[x] = static_cast<double>(q[e * 9 * Np + x]);
  __syncthreads();
  double acc = 0.0;
  for (int qp = threadIdx.x; qp < Nq; qp += 256) {
    double f[9];
    for (int c = 0; c < 9; ++c) f[c] = 0.0;
    for (int i = 0; i < Np; ++i) {
      const double v = d.Vq64T[i * Nq + qp];
      for (int c = 0; c < 9; ++c) f[c] += v * sqv[c * Np + i];
    }
    const double rho = d.rho64[e * Nq + qp], lam = d.lam64[e * Nq + qp], mu = d.mu64[e * Nq + qp];
    const double tr = f[3] + f[4] + f[5];
    double es = 0.0;
    for (int m = 0; m < 3; ++m) es += f[3 + m] * (lam * tr + 2.0 * mu * f[3 + m]);
    for (int m = 3; m < 6; ++m) es += 2.0 * f[3 + m] * (2.0 * mu * f[3 + m]);
    acc += d.wq64[qp] * (rho * (f[0] * f[0] + f[1] * f[1] + f[2] * f[2]) + es);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) d.epart[e] = 0.5 * d.J64[e] * red[0];
}

// Deterministic sum of n values by one workgroup (fixed order).
__global__ __launch_bounds__(1024) void k_sum(const double* __restrict__ x, int64_t n, double* out) {
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
template <typename T>
static StageArgs<T> stage_args(const Dev& d, const void* qin, const void* sin, void* qout,
                               void* sout, void* out, const StageCoef& c) {
  StageArgs<T> a;
  a.qin = static_cast<const T*>(qin);
  a.sin = static_cast<const T*>(sin);
  a.qout = static_cast<T*>(qout);
  a.sout = static_cast<T*>(sout);
  a.out = static_cast<T*>(out);
  a.W = static_cast<const T*>(d.W);
  a.lm = static_cast<const T*>(d.lm);
  a.geo = static_cast<const T*>(d.geo);
  a.fgeo = static_cast<const T*>(d.fgeo);
  a.Z = static_cast<const T*>(d.Z);
  a.svec = static_cast<const T*>(d.svec);
  a.DrT = static_cast<const T*>(d.DrT);
  a.DsT = static_cast<const T*>(d.DsT);
  a.DtT = static_cast<const T*>(d.DtT);
  a.LIFTT = static_cast<const T*>(d.LIFTT);
  a.VqT = static_cast<const T*>(d.VqT);
  a.PqT = static_cast<const T*>(d.PqT);
  a.conn = d.conn;
  a.nbrnode = d.nbrnode;
  a.fmask = d.fmask;
  a.K = d.K;
  a.a = static_cast<T>(c.a);
  a.b = static_cast<T>(c.b);
  a.dt = static_cast<T>(c.dt);
  a.srcval = static_cast<T>(c.srcval);
  a.dir0 = static_cast<T>(c.dir[0]);
  a.dir1 = static_cast<T>(c.dir[1]);
  a.dir2 = static_cast<T>(c.dir[2]);
  a.src_elem = c.src_elem;
  return a;
}

template <typename T, int N>
static hipError_t stage_impl(const Dev& d, int mode, const void* qin, const void* sin, void* qout,
                             void* sout, void* out, const StageCoef& c, hipStream_t st) {
  using C = StageCfg<T, N>;
  const StageArgs<T> a = stage_args<T>(d, qin, sin, qout, sout, out, c);
  const unsigned grid = static_cast<unsigned>((d.K + C::E - 1) / C::E);
  if (mode == 0)
    hipLaunchKernelGGL((k_stage<T, N, 0>), dim3(grid), dim3(C::NT), 0, st, a);
  else
    hipLaunchKernelGGL((k_stage<T, N, 1>), dim3(grid), dim3(C::NT), 0, st, a);
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t material_impl(const Dev& d, hipStream_t st) {
  using S = Sz<N>;
  constexpr bool lds = S::Np * S::Np * 8 <= 28 * 1024;
  if (lds) {
    hipLaunchKernelGGL((k_material<T, N, true>), dim3(static_cast<unsigned>(d.K)), dim3(256), 0, st, d,
                       int64_t(0));
    return hipGetLastError();
  }
  const int64_t per = static_cast<int64_t>(d.scratch_bytes / (sizeof(double) * S::Np * S::Np));
  if (per < 1) return hipErrorInvalidValue;
  for (int64_t b = 0; b < d.K; b += per) {
    const int64_t cnt = (d.K - b) < per ? (d.K - b) : per;
    hipLaunchKernelGGL((k_material<T, N, false>), dim3(static_cast<unsigned>(cnt)), dim3(256), 0, st,
                       d, b);
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  return hipSuccess;
}

#define EWDG_DISPATCH(NVAL, CALL)       \
  switch (NVAL) {                       \
    case 1: { constexpr int NN = 1; CALL; } \
    case 2: { constexpr int NN = 2; CALL; } \
    case 3: { constexpr int NN = 3; CALL; } \
    case 4: { constexpr int NN = 4; CALL; } \
    case 5: { constexpr int NN = 5; CALL; } \
    case 7: { constexpr int NN = 7; CALL; } \
    default: return hipErrorInvalidValue; \
  }

bool supported_degree(int N) { return N == 1 || N == 2 || N == 3 || N == 4 || N == 5 || N == 7; }

hipError_t launch_material(const Dev& d, hipStream_t st) {
  if (d.prec == 32) { EWDG_DISPATCH(d.N, return (material_impl<float, NN>(d, st))); }
  EWDG_DISPATCH(d.N, return (material_impl<double, NN>(d, st)));
}

hipError_t launch_source_vector(const Dev& d, int64_t elem, hipStream_t st) {
  if (d.prec == 32) {
    EWDG_DISPATCH(d.N, hipLaunchKernelGGL((k_source_vector<float, NN>), dim3(1), dim3(256), 0, st, d, elem);
                  return hipGetLastError());
  }
  EWDG_DISPATCH(d.N, hipLaunchKernelGGL((k_source_vector<double, NN>), dim3(1), dim3(256), 0, st, d, elem);
                return hipGetLastError());
}

hipError_t launch_sigma(const Dev& d, const void* q, void* s, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(d.K));
  if (d.prec == 32) {
    EWDG_DISPATCH(d.N, hipLaunchKernelGGL((k_sigma<float, NN>), grid, dim3(256), 0, st,
                                          static_cast<const float*>(q), static_cast<float*>(s),
                                          static_cast<const float*>(d.lm), static_cast<const float*>(d.VqT),
                                          static_cast<const float*>(d.PqT), d.K);
                  return hipGetLastError());
  }
  EWDG_DISPATCH(d.N, hipLaunchKernelGGL((k_sigma<double, NN>), grid, dim3(256), 0, st,
                                        static_cast<const double*>(q), static_cast<double*>(s),
                                        static_cast<const double*>(d.lm), static_cast<const double*>(d.VqT),
                                        static_cast<const double*>(d.PqT), d.K);
                return hipGetLastError());
}

hipError_t launch_stage(const Dev& d, int mode, const void* qin, const void* sin, void* qout, void* sout,
                        void* out, const StageCoef& c, hipStream_t st) {
  if (d.prec == 32) { EWDG_DISPATCH(d.N, return (stage_impl<float, NN>(d, mode, qin, sin, qout, sout, out, c, st))); }
  EWDG_DISPATCH(d.N, return (stage_impl<double, NN>(d, mode, qin, sin, qout, sout, out, c, st)));
}

hipError_t launch_project(const Dev& d, const double* fq, void* q, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(d.K));
  if (d.prec == 32) {
    EWDG_DISPATCH(d.N, hipLaunchKernelGGL((k_project<float, NN>), grid, dim3(256), 0, st, d, fq,
                                          static_cast<float*>(q));
                  return hipGetLastError());
  }
  EWDG_DISPATCH(d.N, hipLaunchKernelGGL((k_project<double, NN>), grid, dim3(256), 0, st, d, fq,
                                        static_cast<double*>(q));
                return hipGetLastError());
}

hipError_t launch_evalq(const Dev& d, const void* q, double* fq, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(d.K));
  if (d.prec == 32) {
    EWDG_DISPATCH(d.N, hipLaunchKernelGGL((k_evalq<float, NN>), grid, dim3(256), 0, st, d,
                                          static_cast<const float*>(q), fq);
                  return hipGetLastError());
  }
  EWDG_DISPATCH(d.N, hipLaunchKernelGGL((k_evalq<double, NN>), grid, dim3(256), 0, st, d,
                                        static_cast<const double*>(q), fq);
                return hipGetLastError());
}

hipError_t launch_receivers(const Dev& d, const void* q, int nr, int step, hipStream_t st) {
  if (nr <= 0) return hipSuccess;
  if (d.prec == 32) {
    EWDG_DISPATCH(d.N, hipLaunchKernelGGL((k_receivers<float, NN>), dim3(nr), dim3(64), 0, st, d,
                                          static_cast<const float*>(q), nr, step);
                  return hipGetLastError());
  }
  EWDG_DISPATCH(d.N, hipLaunchKernelGGL((k_receivers<double, NN>), dim3(nr), dim3(64), 0, st, d,
                                        static_cast<const double*>(q), nr, step);
                return hipGetLastError());
}

hipError_t launch_energy(const Dev& d, const void* q, double* out, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(d.K));
  hipError_t err;
  if (d.prec == 32) {
    EWDG_DISPATCH(d.N, hipLaunchKernelGGL((k_energy<float, NN>), grid, dim3(256), 0, st, d,
                                          static_cast<const float*>(q));
                  err = hipGetLastError(); break);
  } else {
    EWDG_DISPATCH(d.N, hipLaunchKernelGGL((k_energy<double, NN>), grid, dim3(256), 0, st, d,
                                          static_cast<const double*>(q));
                  err = hipGetLastError(); break);
  }
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, st, d.epart, d.K, out);
  return hipGetLastError();
}

}  // namespace ewdg
