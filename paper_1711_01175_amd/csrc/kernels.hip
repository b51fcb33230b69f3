// HIP kernels for gfx950: material setup (FP64), the fused LSRK stage
// (volume derivatives, upwind interface flux, lift, density-weighted mass
// inverse, RK update and the stress projection of the new state), and the
// FP64 diagnostics (projection, evaluation, receivers, energy).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dev.hpp"
#include "kcommon.hpp"
#include "tiles.hpp"

namespace ewdg {

template <typename T>
struct StageArgs {
  const T* qin;
  const T* sin;
  T* qout;
  T* sout;
  T* out;        // rhs (mode 0) or the LSRK register (modes 1, 2)
  T* rhsv;       // mode 2: the velocity rows of the right-hand side [K][3][Np]
  const T* W;
  const T* lm;
  const T* geo;
  const T* fgeo;
  const T* Z;
  const T* svec;
  // operators pre-arranged in matrix-core fragment order: for row tile R and
  // k-step kk, 64 consecutive values hold A[16R + l%16][4kk + l/16], l = lane
  const T* Dpad;     // [3][RT][NpK/4][64]
  const T* Lpad;     // [4 faces][RT][NfpK/4][64]
  const T* Vqpad;    // [QT][NpK/4][64]
  const T* Pqpad;    // [RT][NqK/4][64]
  const int32_t* conn;
  const int32_t* nbrnode;
  const int32_t* fmask;
  int64_t K;
  T a, b, dt, srcval;
  T dir0, dir1, dir2;
  int64_t src_elem;
  const int32_t* bcm;   // bounded meshes: per element, 2 bits per face (1 traction-free, 2 absorbing)
};

// Exact Riemann solution per wave mode at one face point (outward normal n
// of the own element): the normal (P) mode carries J_p = (dT.n + Z_p+ dv.n)
// / (Z_p- + Z_p+) and the tangential (S) mode j_t = ((dT + Z_s+ dv) minus
// its normal part) / (Z_s- + Z_s+), with the jumps dT = T+ - T- (tractions)
// and dv = v+ - v-.  Out, scaled by the face factor fs: fl[0..2] = fs (T* -
// T-) = fs (Z_s- j_t + Z_p- J_p n) (velocity equation) and fl[3..8] = the
// strain correction sym(n (x) (v* - v-)) with v* - v- = j_t + J_p n, as the
// rows xx, yy, zz, yz, xz, xy.
//
// FP32 forms the jumps first (about half the vector instructions of the
// per-state form, and the hardware reciprocal); FP64 projects each side's
// state onto the normal and tangential modes first, which measured faster
// there (the FP64 stage is register-bound at two waves per SIMD).
template <typename T>
__device__ __forceinline__ void interface_flux(const T* n, T fs, const T* vm, const T* sm, const T* vp,
                                               const T* sp, T zpm, T zpp, T zsm, T zsp, T* fl) {
  if constexpr (sizeof(T) == 4) {
    T ds[6], dv[3];
#pragma unroll
    for (int m = 0; m < 6; ++m) ds[m] = sp[m] - sm[m];
#pragma unroll
    for (int c = 0; c < 3; ++c) dv[c] = vp[c] - vm[c];
    const T dT[3] = {ds[0] * n[0] + ds[5] * n[1] + ds[4] * n[2], ds[5] * n[0] + ds[1] * n[1] + ds[3] * n[2],
                     ds[4] * n[0] + ds[3] * n[1] + ds[2] * n[2]};
    const T dTn = dT[0] * n[0] + dT[1] * n[1] + dT[2] * n[2];
    const T dvn = dv[0] * n[0] + dv[1] * n[1] + dv[2] * n[2];
    const T ip = fs * __builtin_amdgcn_rcpf(zpm + zpp), is = fs * __builtin_amdgcn_rcpf(zsm + zsp);
    const T jp = (dTn + zpp * dvn) * ip;      // fs J_p
    const T jsn = dTn + zsp * dvn;            // normal part of dT + Z_s+ dv
    const T tp = zpm * jp;
    T fv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T jt = (dT[c] + zsp * dv[c] - jsn * n[c]) * is;   // fs j_t
      fl[c] = zsm * jt + tp * n[c];
      fv[c] = jt + jp * n[c];
    }
    fl[3] = n[0] * fv[0];
    fl[4] = n[1] * fv[1];
    fl[5] = n[2] * fv[2];
    fl[6] = T(0.5) * (n[1] * fv[2] + n[2] * fv[1]);
    fl[7] = T(0.5) * (n[0] * fv[2] + n[2] * fv[0]);
    fl[8] = T(0.5) * (n[0] * fv[1] + n[1] * fv[0]);
  } else {
    const T Tm[3] = {sm[0] * n[0] + sm[5] * n[1] + sm[4] * n[2], sm[5] * n[0] + sm[1] * n[1] + sm[3] * n[2],
                     sm[4] * n[0] + sm[3] * n[1] + sm[2] * n[2]};
    const T Tp[3] = {sp[0] * n[0] + sp[5] * n[1] + sp[4] * n[2], sp[5] * n[0] + sp[1] * n[1] + sp[3] * n[2],
                     sp[4] * n[0] + sp[3] * n[1] + sp[2] * n[2]};
    const T vmn = vm[0] * n[0] + vm[1] * n[1] + vm[2] * n[2];
    const T vpn = vp[0] * n[0] + vp[1] * n[1] + vp[2] * n[2];
    const T Tmn = Tm[0] * n[0] + Tm[1] * n[1] + Tm[2] * n[2];
    const T Tpn = Tp[0] * n[0] + Tp[1] * n[1] + Tp[2] * n[2];
    const T ip = T(1) / (zpm + zpp);
    const T is = T(1) / (zsm + zsp);
    const T dTn = zpm * ((Tpn - Tmn) + zpp * (vpn - vmn)) * ip;   // Z_p- J_p
    const T dvn = ((Tpn - Tmn) + zpp * (vpn - vmn)) * ip;         // J_p
    T dT[3], dv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T vmt = vm[c] - vmn * n[c], vpt = vp[c] - vpn * n[c];
      const T Tmt = Tm[c] - Tmn * n[c], Tpt = Tp[c] - Tpn * n[c];
      const T jt = (Tpt - Tmt) + zsp * (vpt - vmt);
      dT[c] = zsm * jt * is + dTn * n[c];
      dv[c] = jt * is + dvn * n[c];
    }
    fl[0] = fs * dT[0];
    fl[1] = fs * dT[1];
    fl[2] = fs * dT[2];
    fl[3] = fs * n[0] * dv[0];
    fl[4] = fs * n[1] * dv[1];
    fl[5] = fs * n[2] * dv[2];
    fl[6] = fs * T(0.5) * (n[1] * dv[2] + n[2] * dv[1]);
    fl[7] = fs * T(0.5) * (n[0] * dv[2] + n[2] * dv[0]);
    fl[8] = fs * T(0.5) * (n[0] * dv[1] + n[1] * dv[0]);
  }
}

// Maps workgroups to element tiles so that each of the 8 XCDs (which own
// separate L2 caches and receive workgroups round-robin) works on a
// contiguous range of the mesh, keeping face neighbours in the same L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t bid, int64_t nblk) {
  if (nblk % 8 != 0) return bid;
  return (bid % 8) * (nblk / 8) + bid / 8;
}

// Face-point data gathered for one face ahead of its use: the neighbour's
// velocity and stresses at the matching node, and the own stresses where the
// tile does not keep them in LDS.
template <typename T>
struct FacePt {
  T sm[6], vp[3], sp[6];
};

template <typename T, int N, int MODE, bool BND = false, bool WADG = false>
__device__ __forceinline__ void stage_body(const StageArgs<T>& a, int tile) {
  using TL = Tile<N>;
  using M = Mfma<T>;
  using acc_t = typename M::acc_t;
  constexpr int Np = TL::Np, Nfp = TL::Nfp, Nq = TL::Nq, E = TL::E;
  constexpr int NpK = TL::NpK, NqK = TL::NqK, NfpK = TL::NfpK;
  constexpr int RT = TL::RT, QT = TL::QT, NW = TL::NW, NT = TL::NT;
  constexpr int SV = TL::SV, SE = TL::SE, SF = TL::SF, SQ = TL::SQ, GS = TL::GS;
  constexpr int KD = NpK / 4, KF = NfpK / 4;       // k-steps of the node / face contractions
  // Operator fragments of the node contractions are held in groups of GK
  // k-steps, two groups at a time, where all KD would crowd the registers
  // (N = 7: 30 k-steps).
  constexpr int GK = KD > 16 ? 10 : KD, NGK = (KD + GK - 1) / GK;
  constexpr int FPT = (Nfp * E + NT - 1) / NT;      // face points per thread and face
  __shared__ T sX[TL::X];
  __shared__ T sY[TL::Y];
  __shared__ T sgeo[TL::GEO];
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63;
  const int lr = l & 15, lg = l >> 4;  // A row / B column; K sub-index
  const int Ke = static_cast<int>(a.K);
  const int e0 = tile * E;
  const bool own = w < RT;             // this wave owns node row tile R = w
  const int R = w;
  // Bank swizzle of the 16-element column groups in the buffers of row
  // stride SV and SF (both 16 mod 32 values): the element slot of row r is
  // e ^ (r mod 16).  The matrix-core reads (lanes over the elements of a few
  // rows) stay conflict-free, and the element-wise accesses (lanes over
  // rows, one element) no longer fall into one or two banks.  FP32 at N = 7
  // keeps the plain layout: there the extra index arithmetic costs 10 % (the
  // registers are full); FP64 at N = 7 gains 3 % from the swizzle.
  auto sw = [](int r) { return (N < 7 || sizeof(T) == 8) ? (r & 15) : 0; };
  // own stresses [Np][SE] beside the face buffer, from the first volume
  // direction until the last flux, when they fit in the Y region
  constexpr bool SIGL = NfpK * SF + Np * SE <= TL::Y;
  T* Ssig = sY + NfpK * SF;

  // ---- face-point gathers, two faces ahead of use (buffers pa, pb in
  // turn): the neighbour's velocity and stresses at the matching node (and
  // the own stresses when they are not kept in LDS).
  // (one face ahead where the own stresses come from global memory too:
  // there the second buffer would not fit in the registers)
  constexpr bool G2 = SIGL;
  // Rounds of face points gathered ahead: all of them, except where the own
  // stresses come from global memory and a second round holds only a few
  // points (N = 7: 576 points on 512 threads); that round is gathered when
  // its flux needs it.
  constexpr int FPTP = (!SIGL && FPT > 1) ? 1 : FPT;
  FacePt<T> pa[FPTP], pb[G2 ? FPTP : 1];
  // The neighbour element and node of every face point of this thread,
  // looked up once per tile (connectivity, then the node table), packed as
  // nb * 256 + nn, so a face's gather issues its data loads with no
  // dependent address loads in between.
  // (Where the own stresses do not fit in LDS, N >= 5, the registers are
  // short: there each gather looks its neighbour up itself.)
  // The own volume node of each face point (four faces, one byte each) is
  // looked up at the same time: a face's flux then issues no table load,
  // which would otherwise wait behind the gathers already in flight.
  constexpr bool PRE = SIGL;
  int gofs[PRE ? FPT : 1][4];
  int ilp[PRE ? FPT : 1];
  if constexpr (PRE) {
#pragma unroll
    for (int p = 0; p < FPT; ++p) {
      const int x = tid + p * NT;
      const int xc = x < Nfp * E ? x : Nfp * E - 1;
      const int e = xc / Nfp, j = xc % Nfp;
      const int ge = e0 + e < Ke ? e0 + e : Ke - 1;
      const int4 wd = *reinterpret_cast<const int4*>(a.conn + ge * 4);
      const int w4[4] = {wd.x, wd.y, wd.z, wd.w};
      ilp[p] = 0;
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const int code = w4[f] & 31;
        const int nn = a.nbrnode[((f * 4 + code / 6) * 6 + code % 6) * Nfp + j];
        gofs[p][f] = (w4[f] >> 5) * 256 + nn;
        ilp[p] |= a.fmask[f * Nfp + j] << (8 * f);
      }
    }
  }
  auto gather_one = [&](int f, int p, FacePt<T>& pt) {
    {
      const int x = tid + p * NT;
      const int e = x / Nfp, j = x % Nfp;   // element-major: lanes share a neighbour's cache lines
      if (x < Nfp * E && e0 + e < Ke) {
        int nb, nn;
        if constexpr (PRE) {
          nb = gofs[p][f] >> 8;
          nn = gofs[p][f] & 255;
        } else {
          const int32_t wd = a.conn[(e0 + e) * 4 + f];
          const int code = wd & 31;
          nb = wd >> 5;
          nn = a.nbrnode[((f * 4 + code / 6) * 6 + code % 6) * Nfp + j];
        }
        const T* qn = a.qin + nb * 9 * Np + nn;
        const T* sn = a.sin + nb * 6 * Np + nn;
        if constexpr (!SIGL) {
          const int il = a.fmask[f * Nfp + j];
          const T* so = a.sin + (e0 + e) * 6 * Np + il;
#pragma unroll
          for (int m = 0; m < 6; ++m) pt.sm[m] = so[m * Np];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) pt.vp[c] = qn[c * Np];
#pragma unroll
        for (int m = 0; m < 6; ++m) pt.sp[m] = sn[m * Np];
      }
    }
  };
  auto gather = [&](int f, FacePt<T>* pf) {
#pragma unroll
    for (int p = 0; p < FPTP; ++p) gather_one(f, p, pf[p]);
  };

  // ---- element data: geometry, velocities (B layout) and, where they fit,
  // the own stresses, all loads issued before any is used (one memory
  // latency for the whole start-up); zero paddings
  T* Sv = sX;                // [NpK][SV]  v_c of element e at column c*16+e
  T* SG = sX + NpK * SV;     // [NpK][SV]  G^k_c for the current direction k
  {
    constexpr int NGV = 27;   // geometry and own impedances per element
    constexpr int NGL = (E * NGV + NT - 1) / NT;
    constexpr int NVL = (E * 3 * Np + NT - 1) / NT;
    constexpr int NSL = SIGL ? (E * 6 * Np + NT - 1) / NT : 1;
    T gv0[NGL], vv[NVL], sv[NSL];
#pragma unroll
    for (int p = 0; p < NGL; ++p) {
      const int x = tid + p * NT;
      const int e = x / NGV, m = x % NGV;
      const int ge = e0 + e < Ke ? e0 + e : Ke - 1;
      const T* src = m < 9 ? a.geo + ge * 9 + m : (m < 25 ? a.fgeo + ge * 16 + (m - 9) : a.Z + ge * kZS + (m - 25));
      gv0[p] = x < E * NGV ? *src : T(0);
    }
    // the neighbours' impedances across the four faces (8 values per element)
    static_assert(E * 8 <= NT, "one neighbour impedance per thread");
    const int ze = tid / 8, zm = tid % 8;
    const T znb = tid < E * 8 ? a.Z[(e0 + ze < Ke ? e0 + ze : Ke - 1) * kZS + 2 + zm] : T(0);
#pragma unroll
    for (int p = 0; p < NVL; ++p) {
      const int x = tid + p * NT;
      const int xc = x < E * 3 * Np ? x : E * 3 * Np - 1;
      const int e = xc / (3 * Np), rem = xc % (3 * Np);
      const int ge = e0 + e < Ke ? e0 + e : Ke - 1;
      vv[p] = a.qin[ge * 9 * Np + rem];
    }
    if constexpr (SIGL) {
#pragma unroll
      for (int p = 0; p < NSL; ++p) {
        const int x = tid + p * NT;
        const int xc = x < E * 6 * Np ? x : E * 6 * Np - 1;
        const int e = xc / (6 * Np), rem = xc % (6 * Np);
        const int ge = e0 + e < Ke ? e0 + e : Ke - 1;
        sv[p] = a.sin[ge * 6 * Np + rem];
      }
    }
    // the first faces' gathers stay in flight during the volume terms
    gather(0, pa);
    if constexpr (G2) gather(1, pb);
#pragma unroll
    for (int p = 0; p < NGL; ++p) {
      const int x = tid + p * NT;
      const int e = x / NGV, m = x % NGV;
      if (x < E * NGV) sgeo[e * GS + m] = e0 + e < Ke ? gv0[p] : T(0);
    }
    if (tid < E * 8) sgeo[ze * GS + NGV + zm] = znb;
#pragma unroll
    for (int p = 0; p < NVL; ++p) {
      const int x = tid + p * NT;
      const int e = x / (3 * Np), rem = x % (3 * Np), c = rem / Np, j = rem % Np;
      if (x < E * 3 * Np) Sv[j * SV + c * 16 + (e ^ sw(j))] = (e0 + e < Ke) ? vv[p] : T(0);
    }
    if constexpr (SIGL) {
#pragma unroll
      for (int p = 0; p < NSL; ++p) {
        const int x = tid + p * NT;
        const int e = x / (6 * Np), rem = x % (6 * Np), m = rem / Np, j = rem % Np;
        if (x < E * 6 * Np) Ssig[j * SE + m * 16 + e] = (e0 + e < Ke) ? sv[p] : T(0);
      }
    }
  }
  for (int x = tid; x < (NpK - Np) * SV; x += NT) {
    Sv[Np * SV + x] = T(0);
    SG[Np * SV + x] = T(0);
  }
  constexpr int NPT = (E * Np + NT - 1) / NT;
  __syncthreads();

  // ---- volume terms: div sigma = sum_k D_k G^k with the contravariant
  // stresses G^k_c = sum_m (dr_k/dx_m) sigma_cm, and sym grad v folded into
  // the strain rows direction by direction.
  acc_t rhs[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) rhs[c] = acc_t{0, 0, 0, 0};
  const T* gl = &sgeo[lr * GS];   // geometry of this lane's element
#pragma unroll 1
  for (int k = 0; k < 3; ++k) {
    T afA[GK], afB[GK];
    const T* D = a.Dpad + ((k * RT + R) * KD) * 64 + l;
    auto frag_load = [&](const T* src, int g, T* dst) {
#pragma unroll
      for (int u = 0; u < GK; ++u) dst[u] = (g * GK + u < KD) ? src[(g * GK + u) * 64] : T(0);
    };
    if (own) frag_load(D, 0, afA);
#pragma unroll
    for (int p = 0; p < NPT; ++p) {
      const int x = tid + p * NT;
      if (x < E * Np) {
        const int e = x / Np, j = x % Np;
        T sg[6];
        const int ge = e0 + e < Ke ? e0 + e : Ke - 1;
        if constexpr (!SIGL) {
#pragma unroll
          for (int m = 0; m < 6; ++m) sg[m] = a.sin[ge * 6 * Np + m * Np + j];
        } else {
#pragma unroll
          for (int m = 0; m < 6; ++m) sg[m] = Ssig[j * SE + m * 16 + e];
        }
        const T* g = &sgeo[e * GS + k * 3];
        // rows of sigma in Voigt order xx,yy,zz,yz,xz,xy
        const int es = e ^ sw(j);
        SG[j * SV + 0 * 16 + es] = g[0] * sg[0] + g[1] * sg[5] + g[2] * sg[4];
        SG[j * SV + 1 * 16 + es] = g[0] * sg[5] + g[1] * sg[1] + g[2] * sg[3];
        SG[j * SV + 2 * 16 + es] = g[0] * sg[4] + g[1] * sg[3] + g[2] * sg[2];
      }
    }
    __syncthreads();
    if (own) {
      acc_t gv[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) gv[c] = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int g = 0; g < NGK; ++g) {
        T* af = (g & 1) ? afB : afA;
        if (g + 1 < NGK) frag_load(D, g + 1, (g & 1) ? afA : afB);
#pragma unroll
        for (int u = 0; u < GK; ++u) {
          const int kk = g * GK + u;
          if (kk >= KD) break;
          const int rr = 4 * kk + lg;
          const int row = rr * SV + (lr ^ sw(rr));
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            rhs[c] = M::mma(af[u], SG[row + c * 16], rhs[c]);
            gv[c] = M::mma(af[u], Sv[row + c * 16], gv[c]);
          }
        }
      }
      // d v_c / d x_m += (dr_k/dx_m) D_k v_c, symmetrised into the strain rows
      const T g0 = gl[k * 3 + 0], g1 = gl[k * 3 + 1], g2 = gl[k * 3 + 2];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        rhs[3][r] += g0 * gv[0][r];
        rhs[4][r] += g1 * gv[1][r];
        rhs[5][r] += g2 * gv[2][r];
        rhs[6][r] += T(0.5) * (g2 * gv[1][r] + g1 * gv[2][r]);
        rhs[7][r] += T(0.5) * (g2 * gv[0][r] + g0 * gv[2][r]);
        rhs[8][r] += T(0.5) * (g1 * gv[0][r] + g0 * gv[1][r]);
      }
    }
    __syncthreads();
  }

  // ---- interface corrections, one face at a time, lifted on the matrix cores
  T* Sf = sY;  // [NfpK][SF]
  for (int x = tid; x < (NfpK - Nfp) * SF; x += NT) Sf[Nfp * SF + x] = T(0);
  // face f uses the gathers of buffer pf and refills it with face fn
  auto face = [&](const int f, FacePt<T>* pf, const int fn) {
    T lf[KF];
    if (own) {
      const T* Lr = a.Lpad + ((f * RT + R) * KF) * 64 + l;
#pragma unroll
      for (int kk = 0; kk < KF; ++kk) lf[kk] = Lr[kk * 64];
    }
#pragma unroll
    for (int p = 0; p < FPT; ++p) {
      const int x = tid + p * NT;
      if (x >= Nfp * E) continue;
      const int e = x / Nfp, j = x % Nfp;
      T* fl = &Sf[j * SF + (e ^ sw(j))];
      if (e0 + e >= Ke) {
#pragma unroll
        for (int c = 0; c < 9; ++c) fl[c * 16] = T(0);
        continue;
      }
      int il;
      if constexpr (PRE) il = (ilp[p] >> (8 * f)) & 255;
      else il = a.fmask[f * Nfp + j];
      const T* gg = &sgeo[e * GS];
      const T n[3] = {gg[9 + f * 4 + 0], gg[9 + f * 4 + 1], gg[9 + f * 4 + 2]};
      const T fs = gg[9 + f * 4 + 3];
      T vm[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) vm[c] = Sv[il * SV + c * 16 + (e ^ sw(il))];
      FacePt<T> late;
      if (p >= FPTP) gather_one(f, p, late);
      const FacePt<T>& pt = p < FPTP ? pf[p < FPTP ? p : 0] : late;
      T smv[6];
#pragma unroll
      for (int m = 0; m < 6; ++m) smv[m] = SIGL ? Ssig[il * SE + m * 16 + e] : pt.sm[m];
      const T* sm = smv;
      const T* sp = pt.sp;
      const T* vp = pt.vp;
      T spx[6], vpx[3];
      if constexpr (BND) {
        // a boundary face's gather read the element's own trace: the exterior
        // state is its mirror (traction-free: v+ = v-, T+ = -T-) or zero
        // (absorbing)
        const int bcode = (a.bcm[e0 + e] >> (2 * f)) & 3;
        const T cv = bcode == 2 ? T(0) : T(1);
        const T cs = bcode == 0 ? T(1) : (bcode == 1 ? T(-1) : T(0));
#pragma unroll
        for (int m = 0; m < 6; ++m) spx[m] = cs * pt.sp[m];
#pragma unroll
        for (int c = 0; c < 3; ++c) vpx[c] = cv * pt.vp[c];
        sp = spx;
        vp = vpx;
      }
      T flx[9];
      interface_flux(n, fs, vm, sm, vp, sp, gg[25], gg[27 + 2 * f], gg[26], gg[28 + 2 * f], flx);
#pragma unroll
      for (int c = 0; c < 9; ++c) fl[c * 16] = flx[c];
    }
    if (fn < 4) gather(fn, pf);   // in flight during the lift(s) before its flux
    __syncthreads();
    if (own) {
#pragma unroll
      for (int kk = 0; kk < KF; ++kk) {
        const int rr = 4 * kk + lg;
        const int row = rr * SF + (lr ^ sw(rr));
#pragma unroll
        for (int c = 0; c < 9; ++c) rhs[c] = M::mma(lf[kk], Sf[row + c * 16], rhs[c]);
      }
    }
    __syncthreads();
  };
  if constexpr (G2) {
    face(0, pa, 2);
    face(1, pb, 3);
    face(2, pa, 4);
    face(3, pb, 4);
  } else {
    face(0, pa, 1);
    face(1, pa, 2);
    face(2, pa, 3);
    face(3, pa, 4);
  }

  // ---- right-hand side to LDS: velocity rows [NpK][SV] for the mass
  // inverse and strain rows [NpK][SE].  When both fit in the Y region the
  // staged old velocities stay in place for the update (no second global
  // read of them) and the new strains go to the X region; otherwise the new
  // strains overwrite their right-hand side in place.
  constexpr bool VL = NpK * SV + NpK * SE <= TL::Y;
  T* Srv = sY;  // (the face buffer is free after the lift)
  T* Ser = VL ? sY + NpK * SV : sX;
  T* Se = sX;
  constexpr int NPU = (E * Np + NT - 1) / NT;
  T vold[NPU][3];
  if constexpr (VL) {
#pragma unroll
    for (int p = 0; p < NPU; ++p) {
      const int x = tid + p * NT;
      const int e = x / Np, i = x % Np;
#pragma unroll
      for (int c = 0; c < 3; ++c) vold[p][c] = x < E * Np ? Sv[i * SV + c * 16 + (e ^ sw(i))] : T(0);
    }
  }
  if (own) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = R * 16 + M::row(lg, r);
      if (i < NpK) {
#pragma unroll
        for (int c = 0; c < 3; ++c) Srv[i * SV + c * 16 + lr] = rhs[c][r];
#pragma unroll
        for (int m = 0; m < 6; ++m) Ser[i * SE + m * 16 + lr] = rhs[3 + m][r];
      }
    }
  }
  __syncthreads();
  if constexpr (VL) {
    // K-padding rows of the new strains (read by the V_Q products)
    for (int x = tid; x < (NpK - Np) * SE; x += NT) Se[Np * SE + x] = T(0);
  }

  // ---- per (element, node): density-weighted mass inverse on the velocity
  // rows, point source, LSRK update of all nine fields with coalesced
  // accesses; the new strains go to LDS for the projection.  Each thread
  // takes NPU (element, node) pairs in turn; the loads of pair p + 1 (its W
  // row, old residual and state) are issued before pair p is computed, from
  // clamped (valid) addresses, so one memory latency covers the whole step.
  constexpr int NQV = VL ? 6 : 9;        // state values read from global memory
  // o[0..2] += sum over j in [j0, j0 + n) of W_ij rhs_v[j]
  auto wdot = [&](int p, const T* w, int j0, int n, T* o) {
    const int x = tid + p * NT;
    const int e = (x < E * Np ? x : E * Np - 1) / Np;
    // (the velocity right-hand side is not swizzled: the lanes of a wave
    // read at most a few distinct addresses here, served as broadcasts)
#pragma unroll
    for (int u = 0; u < n; ++u) {
      const int j = j0 + u;
      o[0] += w[u] * Srv[j * SV + e];
      o[1] += w[u] * Srv[j * SV + 16 + e];
      o[2] += w[u] * Srv[j * SV + 32 + e];
    }
  };
  // source, LSRK update and stores of pair p, given o[0..2] = W rhs_v
  auto upd_finish = [&](int p, T* o, const T* rv, const T* qv) {
    const int x = tid + p * NT;
    const int e = x / Np, i = x % Np;
    const int ge = e0 + e;
    if (x >= E * Np || ge >= Ke) return;
    const int64_t base = static_cast<int64_t>(ge) * 9 * Np + i;
    if (!WADG && ge == a.src_elem) {
      const T sv = a.srcval * a.svec[i];
      o[0] += sv * a.dir0;
      o[1] += sv * a.dir1;
      o[2] += sv * a.dir2;
    }
    if (MODE == 2 || WADG) {
#pragma unroll
      for (int c = 0; c < 3; ++c) a.rhsv[static_cast<int64_t>(ge) * 3 * Np + c * Np + i] = o[c];
    }
#pragma unroll
    for (int m = 0; m < 6; ++m) o[3 + m] = Ser[i * SE + m * 16 + e];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      if (WADG && c < 3) continue;   // the velocity rows are k_wadg's
      if (MODE == 0) {
        a.out[base + c * Np] = o[c];
      } else {
        const T q0 = (VL && c < 3) ? vold[p][c < 3 ? c : 0] : qv[c - (9 - NQV) < 0 ? 0 : c - (9 - NQV)];
        const T rr = a.a * rv[c] + a.dt * o[c];
        const T qn = q0 + a.b * rr;
        a.out[base + c * Np] = rr;
        a.qout[base + c * Np] = qn;
        if (c >= 3) Se[i * SE + (c - 3) * 16 + e] = qn;
      }
    }
  };
  // one pair at a time, the W row in chunks of CW values whose loads issue
  // together (the rows of the larger degrees do not fit in the registers)
  constexpr int CWP = sizeof(T) == 8 ? (N <= 4 ? EWDG_CW64 : EWDG_CW) : (N <= 5 ? Np : EWDG_CW32);
  constexpr int CW = Np < CWP ? Np : CWP;
#pragma unroll
  for (int p = 0; p < NPU; ++p) {
    const int x = tid + p * NT;
    const int xc = x < E * Np ? x : E * Np - 1;
    const int e = xc / Np, i = xc % Np;
    const int ge = e0 + e < Ke ? e0 + e : Ke - 1;
    const int64_t base = static_cast<int64_t>(ge) * 9 * Np + i;
    T rv[9], qv[NQV];
    if constexpr (MODE != 0) {
#pragma unroll
      for (int c = 0; c < 9; ++c) rv[c] = (WADG && c < 3) ? T(0) : a.out[base + c * Np];
#pragma unroll
      for (int c = 0; c < NQV; ++c) qv[c] = (WADG && c + 9 - NQV < 3) ? T(0) : a.qin[base + (c + 9 - NQV) * Np];
    }
    T o[9] = {0, 0, 0};
    if constexpr (WADG) {
      // weight-adjusted mass inverse: the raw velocity right-hand side goes
      // to k_wadg, no W_rho stream
      o[0] = Srv[i * SV + e];
      o[1] = Srv[i * SV + 16 + e];
      o[2] = Srv[i * SV + 32 + e];
    } else {
      const T* Wm = a.W + static_cast<int64_t>(ge) * Np * Np + i;
#pragma unroll
      for (int j0 = 0; j0 < Np; j0 += CW) {
        constexpr int n0 = CW;
        T w[n0];
#pragma unroll
        for (int u = 0; u < n0; ++u) w[u] = (j0 + u < Np) ? Wm[(j0 + u) * Np] : T(0);
        wdot(p, w, j0, (Np - j0) < CW ? (Np - j0) : CW, o);
      }
    }
    upd_finish(p, o, rv, qv);
  }
  if (MODE == 0) return;

  // ---- sigma_h of the new state: strains at the quadrature points (matrix
  // cores), Hooke's law with the sampled lambda, mu, and the L2_Q projection
  // back to the nodes, in chunks of QC quadrature points with all six
  // components per chunk.  The owner wave of node row tile R accumulates the
  // projection of its rows for all six components, so each P_Q fragment is
  // loaded once per tile and feeds six independent products.
  T* Sq = sY;  // [QC][SQ]
  constexpr int QC = TL::QC, NQC = (QT * 16 + QC - 1) / QC, KQ = QC / 4;
  // each chunk has QC/16 <= NW quadrature row tiles, so a wave takes at most
  // one per chunk: row tile c QC/16 + w of chunk c, if w < QC/16.  In FP32
  // at N = 7 (8 waves, twice the row tiles of a chunk) each row tile is
  // split in two items, its diagonal stresses (with the trace) and its shear
  // stresses, so every wave has one: row tile c QC/16 + w/2, half w % 2.
  // (At N = 5 and in FP64 the split measured slower: the V_Q products of a
  // row tile are then formed twice for half the Hooke work each.)
  static_assert(QC / 16 <= NW, "one quadrature row tile per wave and chunk");
  constexpr bool SPLIT = NW >= 2 * (QC / 16) && N == 7 && sizeof(T) == 4;
  constexpr int MC = SPLIT ? 3 : 6;            // stress components per item
  const int slot = SPLIT ? (w >> 1) : w;
  const int half = SPLIT ? (w & 1) : 0;
  const bool qrow = slot < QC / 16;
  // lambda and 2 mu at this lane's four rows of quadrature row tile Rq
  // (clamped loads; rows past Nq and elements past K are zeroed after)
  auto lm_load = [&](int Rq, T* lam, T* mu2) {
    const int ge = e0 + lr;
    const int gc = ge < Ke ? ge : Ke - 1;
    constexpr int NqP = TL::NqP;
    const T* lmr = a.lm + static_cast<int64_t>(gc) * 2 * NqP;
    if constexpr (sizeof(T) == 4) {
      // rows 4 lg .. 4 lg + 3 of the tile are contiguous: one 16-byte load each
      const int q4 = Rq * 16 + 4 * lg;
      const int qs = q4 + 4 <= NqP ? q4 : NqP - 4;
      const float4 l4 = *reinterpret_cast<const float4*>(lmr + qs);
      const float4 m4 = *reinterpret_cast<const float4*>(lmr + NqP + qs);
      lam[0] = l4.x; lam[1] = l4.y; lam[2] = l4.z; lam[3] = l4.w;
      mu2[0] = m4.x; mu2[1] = m4.y; mu2[2] = m4.z; mu2[3] = m4.w;
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = Rq * 16 + M::row(lg, r);
        const int qq = q < Nq ? q : Nq - 1;
        lam[r] = lmr[qq];
        mu2[r] = lmr[NqP + qq];
      }
    }
  };
  // the first chunk's lambda, mu: issued before the barrier that ends the
  // update, in flight while the other waves finish it
  T lamN[4], muN[4];
  if (qrow && slot < QT) lm_load(slot, lamN, muN);
  __syncthreads();
  acc_t pq[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) pq[m] = acc_t{0, 0, 0, 0};
#pragma unroll 1
  for (int qc = 0; qc < NQC; ++qc) {
    const int q0 = qc * QC;
    const int rows = (NqK - q0) < QC ? (NqK - q0) : QC;   // K rows of this chunk
    // this chunk's P_Q fragments, in flight during the V_Q products
    T pf2[KQ];
    if (own) {
      const T* Pr = a.Pqpad + (R * (NqK / 4) + q0 / 4) * 64 + l;
#pragma unroll
      for (int u = 0; u < KQ; ++u) pf2[u] = (4 * u < rows) ? Pr[u * 64] : T(0);
    }
    const int Rq = q0 / 16 + slot;
    if (qrow && Rq < QT) {
      T vfA[GK], vfB[GK];
      const T* Vr = a.Vqpad + (Rq * KD) * 64 + l;
#pragma unroll
      for (int u = 0; u < GK; ++u) vfA[u] = (u < KD) ? Vr[u * 64] : T(0);
      T lam[4], mu2[4];
      const bool ge_ok = e0 + lr < Ke;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const bool ok = Rq * 16 + M::row(lg, r) < Nq && ge_ok;
        lam[r] = ok ? lamN[r] : T(0);
        mu2[r] = ok ? T(2) * muN[r] : T(0);
      }
      // the next chunk's lambda, mu, in flight during this chunk
      if (Rq + QC / 16 < QT) lm_load(Rq + QC / 16, lamN, muN);
      acc_t ac[MC];
#pragma unroll
      for (int m = 0; m < MC; ++m) ac[m] = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int g = 0; g < NGK; ++g) {
        T* vf = (g & 1) ? vfB : vfA;
        if (g + 1 < NGK) {
          T* nx = (g & 1) ? vfA : vfB;
#pragma unroll
          for (int u = 0; u < GK; ++u) nx[u] = ((g + 1) * GK + u < KD) ? Vr[((g + 1) * GK + u) * 64] : T(0);
        }
#pragma unroll
        for (int u = 0; u < GK; ++u) {
          const int kk = g * GK + u;
          if (kk >= KD) break;
          const int row = (4 * kk + lg) * SE + lr + 3 * half * 16;
#pragma unroll
          for (int m = 0; m < MC; ++m) ac[m] = M::mma(vf[u], Se[row + m * 16], ac[m]);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = Rq * 16 + M::row(lg, r);
        if (q >= NqK) continue;
        T* o = &Sq[(q - q0) * SQ + lr];
        if (!SPLIT || half == 0) {
          const T ltr = lam[r] * (ac[0][r] + ac[1][r] + ac[2][r]);
          o[0] = mu2[r] * ac[0][r] + ltr;
          o[16] = mu2[r] * ac[1][r] + ltr;
          o[32] = mu2[r] * ac[2][r] + ltr;
        }
        if constexpr (!SPLIT) {
          o[48] = mu2[r] * ac[3 % MC][r];
          o[64] = mu2[r] * ac[4 % MC][r];
          o[80] = mu2[r] * ac[5 % MC][r];
        } else if (half == 1) {
          o[48] = mu2[r] * ac[0][r];
          o[64] = mu2[r] * ac[1][r];
          o[80] = mu2[r] * ac[2][r];
        }
      }
    }
    __syncthreads();
    if (own) {
#pragma unroll
      for (int u = 0; u < KQ; ++u) {
        if (4 * u < rows) {
          const int row = (4 * u + lg) * SQ + lr;
#pragma unroll
          for (int m = 0; m < 6; ++m) pq[m] = M::mma(pf2[u], Sq[row + m * 16], pq[m]);
        }
      }
    }
    __syncthreads();
  }
  // new sigma_h through LDS (the strain buffer is free), stored coalesced
  T* Ss = sX;   // [NpK][SE]
  if (own) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = R * 16 + M::row(lg, r);
      if (i < Np) {
#pragma unroll
        for (int m = 0; m < 6; ++m) Ss[i * SE + m * 16 + lr] = pq[m][r];
      }
    }
  }
  __syncthreads();
#pragma unroll 2
  for (int x = tid; x < E * 6 * Np; x += NT) {
    const int e = x / (6 * Np), rem = x % (6 * Np), m = rem / Np, i = rem % Np;
    if (e0 + e < Ke) a.sout[static_cast<int64_t>(e0 + e) * 6 * Np + rem] = Ss[i * SE + m * 16 + e];
  }
}

// One mesh: workgroups map to element tiles, XCD-contiguous.  BND: the mesh
// has boundary faces.  WADG: the weight-adjusted mass inverse (k_wadg
// applies it and updates the velocity).
template <typename T, int N, int MODE, bool BND, bool WADG>
__global__ __launch_bounds__((Tile<N>::NT), (sizeof(T) == 4 ? EWDG_OCC32 : 2)) void k_stage(StageArgs<T> a) {
  const int nblk = static_cast<int>((a.K + Tile<N>::E - 1) / Tile<N>::E);
  stage_body<T, N, MODE, BND, WADG>(a, static_cast<int>(xcd_tile(blockIdx.x, nblk)));
}

template <typename T>
struct WadgArgs {
  const T* r;          // [K][3][Np] raw velocity right-hand side
  const T* rinv;       // [K][NqP] 1 / rho at the quadrature points
  const T* svw;        // [Np] M^-1 phi(x_s) of the source element
  const T* Vqpad;
  const T* Pqpad;
  T* out;              // mode 0: operator output [K][9][Np]; mode 1: LSRK register
  const T* qin;
  T* qout;
  int64_t K;
  T a, b, dt, srcval, dir0, dir1, dir2;
  int64_t src_elem;
};

// Weight-adjusted velocity update (the alternative to W_rho = M_rho^-1 M):
// u = P_Q diag(1/rho) V_Q r with r the velocity right-hand side plus the
// point source M^-1 phi(x_s) f, i.e. M^-1 M_{1/rho} M^-1 applied to the weak
// residual; then u into the velocity rows of the operator output (mode 0) or
// the LSRK update of the velocity (mode 1).  16 elements per workgroup, V_Q
// in chunks of 64 quadrature rows into LDS (scaled by 1/rho), P_Q
// accumulated across the chunks on the matrix cores.
template <typename T, int N, int MODE>
__global__ __launch_bounds__((Tile<N>::NT)) void k_wadg(WadgArgs<T> a) {
  using TL = Tile<N>;
  using M = Mfma<T>;
  using acc_t = typename M::acc_t;
  constexpr int Np = TL::Np, Nq = TL::Nq, NqP = TL::NqP, E = TL::E, NpK = TL::NpK, NqK = TL::NqK;
  constexpr int RT = TL::RT, QT = TL::QT, NT = TL::NT, KD = NpK / 4;
  constexpr int QCW = 64, NQC = (QT * 16 + QCW - 1) / QCW, SR = 48;
  __shared__ T Sr[NpK * SR];
  __shared__ T Sz[QCW * SR];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, lr = l & 15, lg = l >> 4;
  const int Ke = static_cast<int>(a.K);
  const int e0 = blockIdx.x * E;
  for (int x = tid; x < E * 3 * Np; x += NT) {
    const int e = x / (3 * Np), rem = x % (3 * Np), c = rem / Np, j = rem % Np;
    T v = T(0);
    if (e0 + e < Ke) {
      v = a.r[static_cast<int64_t>(e0 + e) * 3 * Np + rem];
      if (e0 + e == a.src_elem) v += a.srcval * (c == 0 ? a.dir0 : (c == 1 ? a.dir1 : a.dir2)) * a.svw[j];
    }
    Sr[j * SR + c * 16 + e] = v;
  }
  for (int x = tid; x < (NpK - Np) * SR; x += NT) Sr[Np * SR + x] = T(0);
  __syncthreads();
  acc_t u[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) u[c] = acc_t{0, 0, 0, 0};
  // per chunk, the loads that do not depend on the products (1/rho at this
  // lane's four quadrature rows and the V_Q fragments; in FP32 at N = 7 also
  // the P_Q fragments) are issued first, so their latency overlaps the V_Q
  // products.  Loading the P_Q fragments ahead costs registers: it measured
  // 6 % faster in FP32 at N = 7 and 3 % slower elsewhere (4 instead of 6
  // waves per SIMD in FP32 at N = 4).
  constexpr bool PQA = sizeof(T) == 4 && N >= 7;
#pragma unroll 1
  for (int qc = 0; qc < NQC; ++qc) {
    const int q0 = qc * QCW;
    const int Rq = q0 / 16 + w;
    const bool vq = w < QCW / 16 && Rq < QT;
    const int rows = (NqK - q0) < QCW ? (NqK - q0) : QCW;
    T ri[4], vf[KD], pf[PQA ? QCW / 4 : 1];
    if (vq) {
      const int ge = e0 + lr;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = Rq * 16 + M::row(lg, r);
        ri[r] = (q < Nq && ge < Ke) ? a.rinv[static_cast<int64_t>(ge) * NqP + q] : T(0);
      }
      const T* Vr = a.Vqpad + (Rq * KD) * 64 + l;
#pragma unroll
      for (int kk = 0; kk < KD; ++kk) vf[kk] = Vr[kk * 64];
    }
    if (PQA && w < RT) {
      const T* Pr = a.Pqpad + (w * (NqK / 4) + q0 / 4) * 64 + l;
#pragma unroll
      for (int kq = 0; kq < QCW / 4; ++kq) pf[PQA ? kq : 0] = 4 * kq < rows ? Pr[kq * 64] : T(0);
    }
    if (vq) {
      acc_t z[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) z[c] = acc_t{0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < KD; ++kk) {
        const int row = (4 * kk + lg) * SR + lr;
#pragma unroll
        for (int c = 0; c < 3; ++c) z[c] = M::mma(vf[kk], Sr[row + c * 16], z[c]);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = Rq * 16 + M::row(lg, r);
#pragma unroll
        for (int c = 0; c < 3; ++c) Sz[(q - q0) * SR + c * 16 + lr] = z[c][r] * ri[r];
      }
    }
    __syncthreads();
    if (w < RT) {
#pragma unroll
      for (int kq = 0; kq < QCW / 4; ++kq) {
        if (4 * kq < rows) {
          const int row = (4 * kq + lg) * SR + lr;
          const T pk = PQA ? pf[PQA ? kq : 0] : a.Pqpad[(w * (NqK / 4) + q0 / 4) * 64 + l + kq * 64];
#pragma unroll
          for (int c = 0; c < 3; ++c) u[c] = M::mma(pk, Sz[row + c * 16], u[c]);
        }
      }
    }
    __syncthreads();
  }
  if (w < RT) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = w * 16 + M::row(lg, r);
      if (i < Np) {
#pragma unroll
        for (int c = 0; c < 3; ++c) Sr[i * SR + c * 16 + lr] = u[c][r];
      }
    }
  }
  __syncthreads();
  for (int x = tid; x < E * 3 * Np; x += NT) {
    const int e = x / (3 * Np), rem = x % (3 * Np), c = rem / Np, i = rem % Np;
    if (e0 + e >= Ke) continue;
    const T uv = Sr[i * SR + c * 16 + e];
    const int64_t base = static_cast<int64_t>(e0 + e) * 9 * Np + rem;
    if (MODE == 0) {
      a.out[base] = uv;
    } else {
      const T rr = a.a * a.out[base] + a.dt * uv;
      a.out[base] = rr;
      a.qout[base] = a.qin[base] + a.b * rr;
    }
  }
}

// Many independent meshes of the same degree in one ragged launch: request r
// owns workgroups [tile_start[r], tile_start[r+1]); each request's arithmetic
// is exactly that of its own single-mesh launch.
template <typename T, int N>
__global__ __launch_bounds__((Tile<N>::NT), (sizeof(T) == 4 ? EWDG_OCC32 : 2)) void k_stage_batch(const char* __restrict__ table,
                                                                   int record_bytes,
                                                                   const int* __restrict__ tile_start,
                                                                   int nreq) {
  const int b = blockIdx.x;
  int lo = 0, hi = nreq;   // largest r with tile_start[r] <= b
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (tile_start[mid] <= b) lo = mid;
    else hi = mid;
  }
  // records are record_bytes apart (the host lays out both precisions alike)
  const StageArgs<T> a = *reinterpret_cast<const StageArgs<T>*>(table + static_cast<size_t>(lo) * record_bytes);
  stage_body<T, N, 1>(a, b - tile_start[lo]);
}

// sigma_h = P_Q(lambda tr(e) I + 2 mu e) for a given state (no update).
// sigma_h = P_Q (lambda tr(eps_Q) I + 2 mu eps_Q), eps_Q = V_Q eps, of a
// state q (the L2_Q projection of C eps, as in the stage kernel): 16
// elements per workgroup on the matrix cores.  The strains sit in LDS as B
// operands (node rows, element columns per component); V_Q runs in chunks of
// QC quadrature rows, Hooke's law is applied at the points, and P_Q
// accumulates across the chunks in the owner waves of the node row tiles.
template <typename T, int N>
__global__ __launch_bounds__((Tile<N>::NT)) void k_sigma(const T* __restrict__ q, T* __restrict__ s,
                                                         const T* __restrict__ lm, const T* __restrict__ Vqpad,
                                                         const T* __restrict__ Pqpad, int64_t K) {
  using TL = Tile<N>;
  using M = Mfma<T>;
  using acc_t = typename M::acc_t;
  constexpr int Np = TL::Np, Nq = TL::Nq, NqP = TL::NqP, E = TL::E, NpK = TL::NpK, NqK = TL::NqK;
  constexpr int RT = TL::RT, QT = TL::QT, NT = TL::NT, KD = NpK / 4;
  constexpr int SE = TL::SE, SQ = 96, QC = 64, NQC = (QT * 16 + QC - 1) / QC;
  __shared__ T Se[NpK * SE];   // strains, then the result
  __shared__ T Sq[QC * SQ];    // stresses at the chunk's quadrature points
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, lr = l & 15, lg = l >> 4;
  const int64_t e0 = static_cast<int64_t>(blockIdx.x) * E;
  for (int x = tid; x < E * 6 * Np; x += NT) {
    const int e = x / (6 * Np), rem = x % (6 * Np), m = rem / Np, j = rem % Np;
    Se[j * SE + m * 16 + e] = e0 + e < K ? q[(e0 + e) * 9 * Np + 3 * Np + rem] : T(0);
  }
  for (int x = tid; x < (NpK - Np) * SE; x += NT) Se[Np * SE + x] = T(0);
  __syncthreads();
  acc_t pq[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) pq[m] = acc_t{0, 0, 0, 0};
#pragma unroll 1
  for (int qc = 0; qc < NQC; ++qc) {
    const int q0 = qc * QC;
    const int rows = (NqK - q0) < QC ? (NqK - q0) : QC;
    const int Rq = q0 / 16 + w;
    if (w < QC / 16 && Rq < QT) {
      const int64_t ge = e0 + lr < K ? e0 + lr : K - 1;
      T lam[4], mu2[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int qp = Rq * 16 + M::row(lg, r);
        const bool ok = qp < Nq && e0 + lr < K;
        const int qq = qp < Nq ? qp : Nq - 1;
        lam[r] = ok ? lm[ge * 2 * NqP + qq] : T(0);
        mu2[r] = ok ? T(2) * lm[ge * 2 * NqP + NqP + qq] : T(0);
      }
      acc_t ac[6];
#pragma unroll
      for (int m = 0; m < 6; ++m) ac[m] = acc_t{0, 0, 0, 0};
      const T* Vr = Vqpad + (Rq * KD) * 64 + l;
#pragma unroll 4
      for (int kk = 0; kk < KD; ++kk) {
        const T vf = Vr[kk * 64];
        const int row = (4 * kk + lg) * SE + lr;
#pragma unroll
        for (int m = 0; m < 6; ++m) ac[m] = M::mma(vf, Se[row + m * 16], ac[m]);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int qp = Rq * 16 + M::row(lg, r);
        if (qp >= NqK) continue;
        T* o = &Sq[(qp - q0) * SQ + lr];
        const T ltr = lam[r] * (ac[0][r] + ac[1][r] + ac[2][r]);
#pragma unroll
        for (int m = 0; m < 6; ++m) o[m * 16] = mu2[r] * ac[m][r] + (m < 3 ? ltr : T(0));
      }
    }
    __syncthreads();
    if (w < RT) {
      const T* Pr = Pqpad + (w * (NqK / 4) + q0 / 4) * 64 + l;
#pragma unroll 4
      for (int u = 0; u < QC / 4; ++u) {
        if (4 * u < rows) {
          const T pf = Pr[u * 64];
          const int row = (4 * u + lg) * SQ + lr;
#pragma unroll
          for (int m = 0; m < 6; ++m) pq[m] = M::mma(pf, Sq[row + m * 16], pq[m]);
        }
      }
    }
    __syncthreads();
  }
  if (w < RT) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = w * 16 + M::row(lg, r);
      if (i < Np) {
#pragma unroll
        for (int m = 0; m < 6; ++m) Se[i * SE + m * 16 + lr] = pq[m][r];
      }
    }
  }
  __syncthreads();
  for (int x = tid; x < E * 6 * Np; x += NT) {
    const int e = x / (6 * Np), rem = x % (6 * Np), m = rem / Np, i = rem % Np;
    if (e0 + e < K) s[(e0 + e) * 6 * Np + rem] = Se[i * SE + m * 16 + e];
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
  constexpr int NqP = S::NqP;
  T* lm = static_cast<T*>(d.lm) + e * 2 * NqP;
  for (int q = Nq + threadIdx.x; q < NqP; q += blockDim.x) {
    lm[q] = T(0);
    lm[NqP + q] = T(0);
  }
  double a0 = 0, a1 = 0, a2 = 0;
  for (int q = threadIdx.x; q < Nq; q += blockDim.x) {
    const double w = d.wq64[q];
    lm[q] = static_cast<T>(d.lam64[e * Nq + q]);
    lm[NqP + q] = static_cast<T>(d.mu64[e * Nq + q]);
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
    T* Z = static_cast<T*>(d.Z) + e * kZS;
    Z[0] = static_cast<T>(sqrt(r * (l + 2.0 * m)));
    Z[1] = static_cast<T>(sqrt(r * m));
    d.means64[e * 3 + 0] = r;
    d.means64[e * 3 + 1] = l;
    d.means64[e * 3 + 2] = m;
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
                               void* sout, void* out, const StageCoef& c, void* rhsv = nullptr) {
  StageArgs<T> a;
  a.qin = static_cast<const T*>(qin);
  a.sin = static_cast<const T*>(sin);
  a.qout = static_cast<T*>(qout);
  a.sout = static_cast<T*>(sout);
  a.out = static_cast<T*>(out);
  a.rhsv = static_cast<T*>(rhsv);
  a.W = static_cast<const T*>(d.W);
  a.lm = static_cast<const T*>(d.lm);
  a.geo = static_cast<const T*>(d.geo);
  a.fgeo = static_cast<const T*>(d.fgeo);
  a.Z = static_cast<const T*>(d.Z);
  a.svec = static_cast<const T*>(d.svec);
  a.Dpad = static_cast<const T*>(d.Dpad);
  a.Lpad = static_cast<const T*>(d.Lpad);
  a.Vqpad = static_cast<const T*>(d.Vqpad);
  a.Pqpad = static_cast<const T*>(d.Pqpad);
  a.conn = d.conn;
  a.nbrnode = d.nbrnode;
  a.fmask = d.fmask;
  a.bcm = d.bcm;
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
                             void* sout, void* out, const StageCoef& c, void* rhsv, hipStream_t st) {
  using TL = Tile<N>;
  // the stage kernel indexes its arrays with 32-bit element offsets
  if (d.K * 9 * TL::Np >= (int64_t(1) << 31) || d.K * TL::Np * TL::Np >= (int64_t(1) << 31) ||
      d.K * 2 * TL::NqP >= (int64_t(1) << 31) || d.K >= (int64_t(1) << 23))
    return hipErrorInvalidValue;
  if (mode == 2 && !rhsv) return hipErrorInvalidValue;
  const StageArgs<T> a = stage_args<T>(d, qin, sin, qout, sout, out, c, rhsv);
  const unsigned grid = static_cast<unsigned>((d.K + TL::E - 1) / TL::E);
  if (d.wadg) {
    // weight-adjusted mass inverse (periodic meshes): the stage without the
    // velocity update, then k_wadg
    if (d.bcm || mode == 2 || !d.rhsw) return hipErrorInvalidValue;
    StageArgs<T> aw = a;
    aw.rhsv = static_cast<T*>(d.rhsw);
    if (mode == 0)
      hipLaunchKernelGGL((k_stage<T, N, 0, false, true>), dim3(grid), dim3(TL::NT), 0, st, aw);
    else
      hipLaunchKernelGGL((k_stage<T, N, 1, false, true>), dim3(grid), dim3(TL::NT), 0, st, aw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    WadgArgs<T> w;
    w.r = static_cast<const T*>(d.rhsw);
    w.rinv = static_cast<const T*>(d.rinv);
    w.svw = static_cast<const T*>(d.svw);
    w.Vqpad = static_cast<const T*>(d.Vqpad);
    w.Pqpad = static_cast<const T*>(d.Pqpad);
    w.out = static_cast<T*>(out);
    w.qin = static_cast<const T*>(qin);
    w.qout = static_cast<T*>(qout);
    w.K = d.K;
    w.a = a.a;
    w.b = a.b;
    w.dt = a.dt;
    w.srcval = a.srcval;
    w.dir0 = a.dir0;
    w.dir1 = a.dir1;
    w.dir2 = a.dir2;
    w.src_elem = a.src_elem;
    if (mode == 0)
      hipLaunchKernelGGL((k_wadg<T, N, 0>), dim3(grid), dim3(TL::NT), 0, st, w);
    else
      hipLaunchKernelGGL((k_wadg<T, N, 1>), dim3(grid), dim3(TL::NT), 0, st, w);
    return hipGetLastError();
  }
  if (d.bcm) {
    // bounded meshes: the forward stage and the operator (the adjoint and the
    // recording stage are periodic only)
    if (mode == 0)
      hipLaunchKernelGGL((k_stage<T, N, 0, true, false>), dim3(grid), dim3(TL::NT), 0, st, a);
    else if (mode == 1)
      hipLaunchKernelGGL((k_stage<T, N, 1, true, false>), dim3(grid), dim3(TL::NT), 0, st, a);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
  if (mode == 0)
    hipLaunchKernelGGL((k_stage<T, N, 0, false, false>), dim3(grid), dim3(TL::NT), 0, st, a);
  else if (mode == 1)
    hipLaunchKernelGGL((k_stage<T, N, 1, false, false>), dim3(grid), dim3(TL::NT), 0, st, a);
  else
    hipLaunchKernelGGL((k_stage<T, N, 2, false, false>), dim3(grid), dim3(TL::NT), 0, st, a);
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

template <typename T, int N>
static hipError_t stage_batch_impl(const void* table, int record_bytes, const int* tile_start, int nreq,
                                   int ntiles, hipStream_t st) {
  using TL = Tile<N>;
  if (ntiles <= 0) return hipSuccess;
  if (record_bytes < static_cast<int>(sizeof(StageArgs<T>)) || record_bytes % 16) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_stage_batch<T, N>), dim3(static_cast<unsigned>(ntiles)), dim3(TL::NT), 0, st,
                     static_cast<const char*>(table), record_bytes, tile_start, nreq);
  return hipGetLastError();
}

template <typename T>
static void fill_args(const Dev& d, const void* qin, const void* sin, void* qout, void* sout, void* out,
                      const StageCoef& c, void* dst) {
  *static_cast<StageArgs<T>*>(dst) = stage_args<T>(d, qin, sin, qout, sout, out, c);
}

bool supported_degree(int N) { return N == 1 || N == 2 || N == 3 || N == 4 || N == 5 || N == 7; }

// The neighbour's impedances across each face, next to the element's own
// (read by the face flux of the stage kernel from the tile's geometry block
// instead of being gathered per face point).  A boundary face's connectivity
// names the element itself.
template <typename T>
__global__ __launch_bounds__(256) void k_nbr_z(T* __restrict__ Z, const int32_t* __restrict__ conn, int64_t K) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= 4 * K) return;
  const int64_t e = i / 4, f = i % 4;
  const int64_t nb = conn[i] >> 5;
  Z[e * kZS + 2 + 2 * f] = Z[nb * kZS];
  Z[e * kZS + 3 + 2 * f] = Z[nb * kZS + 1];
}

hipError_t launch_material(const Dev& d, hipStream_t st) {
  hipError_t e;
  if (d.prec == 32) {
    EWDG_DISPATCH(d.N, e = (material_impl<float, NN>(d, st)); break);
  } else {
    EWDG_DISPATCH(d.N, e = (material_impl<double, NN>(d, st)); break);
  }
  if (e != hipSuccess) return e;
  const unsigned blocks = static_cast<unsigned>((4 * d.K + 255) / 256);
  if (d.prec == 32)
    hipLaunchKernelGGL(k_nbr_z<float>, dim3(blocks), dim3(256), 0, st, static_cast<float*>(d.Z), d.conn, d.K);
  else
    hipLaunchKernelGGL(k_nbr_z<double>, dim3(blocks), dim3(256), 0, st, static_cast<double*>(d.Z), d.conn, d.K);
  return hipGetLastError();
}

hipError_t launch_source_vector(const Dev& d, int64_t elem, hipStream_t st) {
  if (d.prec == 32) {
    EWDG_DISPATCH(d.N, hipLaunchKernelGGL((k_source_vector<float, NN>), dim3(1), dim3(256), 0, st, d, elem);
                  return hipGetLastError());
  }
  EWDG_DISPATCH(d.N, hipLaunchKernelGGL((k_source_vector<double, NN>), dim3(1), dim3(256), 0, st, d, elem);
                return hipGetLastError());
}

// 1 / rho at the quadrature points in the run precision, padded rows zero.
template <typename T>
__global__ void k_rinv(const double* __restrict__ rho, T* __restrict__ rinv, int64_t K, int Nq, int NqP) {
  const int64_t n = K * NqP;
  for (int64_t x = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; x < n;
       x += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t k = x / NqP;
    const int q = static_cast<int>(x - k * NqP);
    rinv[x] = q < Nq ? static_cast<T>(1.0 / rho[k * Nq + q]) : T(0);
  }
}

hipError_t launch_rinv(const Dev& d, hipStream_t st) {
  const int NqP = (d.Nq + 3) / 4 * 4;
  const int64_t n = d.K * NqP;
  const unsigned g = static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 65536));
  if (d.prec == 32)
    hipLaunchKernelGGL(k_rinv<float>, dim3(g), dim3(256), 0, st, d.rho64, static_cast<float*>(d.rinv), d.K, d.Nq, NqP);
  else
    hipLaunchKernelGGL(k_rinv<double>, dim3(g), dim3(256), 0, st, d.rho64, static_cast<double*>(d.rinv), d.K, d.Nq,
                       NqP);
  return hipGetLastError();
}

hipError_t launch_sigma(const Dev& d, const void* q, void* s, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>((d.K + 15) / 16));
  if (d.prec == 32) {
    EWDG_DISPATCH(d.N, hipLaunchKernelGGL((k_sigma<float, NN>), grid, dim3(Tile<NN>::NT), 0, st,
                                          static_cast<const float*>(q), static_cast<float*>(s),
                                          static_cast<const float*>(d.lm), static_cast<const float*>(d.Vqpad),
                                          static_cast<const float*>(d.Pqpad), d.K);
                  return hipGetLastError());
  }
  EWDG_DISPATCH(d.N, hipLaunchKernelGGL((k_sigma<double, NN>), grid, dim3(Tile<NN>::NT), 0, st,
                                        static_cast<const double*>(q), static_cast<double*>(s),
                                        static_cast<const double*>(d.lm), static_cast<const double*>(d.Vqpad),
                                        static_cast<const double*>(d.Pqpad), d.K);
                return hipGetLastError());
}

hipError_t launch_stage(const Dev& d, int mode, const void* qin, const void* sin, void* qout, void* sout,
                        void* out, const StageCoef& c, hipStream_t st, void* rhsv) {
  if (d.prec == 32) {
    EWDG_DISPATCH(d.N, return (stage_impl<float, NN>(d, mode, qin, sin, qout, sout, out, c, rhsv, st)));
  }
  EWDG_DISPATCH(d.N, return (stage_impl<double, NN>(d, mode, qin, sin, qout, sout, out, c, rhsv, st)));
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

namespace ewdg {
size_t stage_args_bytes(int prec) { return prec == 32 ? sizeof(StageArgs<float>) : sizeof(StageArgs<double>); }

void stage_args_fill(const Dev& d, const void* qin, const void* sin, void* qout, void* sout, void* out,
                     const StageCoef& c, void* dst) {
  if (d.prec == 32) fill_args<float>(d, qin, sin, qout, sout, out, c, dst);
  else fill_args<double>(d, qin, sin, qout, sout, out, c, dst);
}

int stage_tile_elems() { return 16; }

hipError_t launch_stage_batch(int N, int prec, const void* table, int record_bytes, const int* tile_start,
                              int nreq, int ntiles, hipStream_t st) {
  if (prec == 32) {
    EWDG_DISPATCH(N, return (stage_batch_impl<float, NN>(table, record_bytes, tile_start, nreq, ntiles, st)));
  }
  EWDG_DISPATCH(N, return (stage_batch_impl<double, NN>(table, record_bytes, tile_start, nreq, ntiles, st)));
}
}  // namespace ewdg
