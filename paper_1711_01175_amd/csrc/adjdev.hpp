// Device views of the adjoint workspace and the adjoint launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "dev.hpp"

namespace ewdg {

// Pointers into the caller's adjoint workspace ("run precision" as in Dev).
struct AdjDev {
  void* ytil = nullptr;      // [K][3][Np] W^T applied to the velocity adjoint
  void* fown = nullptr;      // [K][4][Nfp][8] own-side face sensitivities
  void* fnbr = nullptr;      // [K][4][Nfp][8] neighbour-side face sensitivities
  void* qbar = nullptr;      // [K][9][Np] adjoint of the state
  void* rbar = nullptr;      // [K][9][Np] adjoint of the LSRK register
  void* rhs = nullptr;       // [K][9][Np] L q + f (single right-hand-side adjoint)
  void* rhsv = nullptr;      // [5 C][K][3][Np] velocity rows of L q_i + f_i of one segment
  void* res = nullptr;       // [K][9][Np] LSRK register of the recomputation
  double* g = nullptr;       // [K][3] parameter gradient
  double* resid = nullptr;   // [nsteps][nr][3] receiver residuals
  // snapshots of (q, sigma_h(q)): checkpoints, and the stage inputs of every
  // stage of every step of one segment
  void* ck_q = nullptr;      // [nck][K][9][Np]
  void* ck_s = nullptr;      // [nck][K][6][Np]
  void* st_q = nullptr;      // [5 C + 1][K][9][Np]
  void* st_s = nullptr;      // [5 C + 1][K][6][Np]
  // second segment buffer of the overlapped layout (null otherwise)
  void* rhsv2 = nullptr;
  void* st_q2 = nullptr;
  void* st_s2 = nullptr;
};

// qbar += scale * L^T y; if q is given also g += scale * y . d(L q + f)/d theta
// (s = sigma_h(q); rhs holds the velocity rows of L q + f at element stride
// rhs_stride values, component c at offset c Np).  If rupd is given it must
// be y, and afterwards y = ra y + rb qbar (with the updated qbar).
hipError_t launch_adjoint(const Dev& d, const AdjDev& ad, const void* y, const void* q, const void* s,
                          const void* rhs, int rhs_stride, void* qbar, double* g, double scale, void* rupd,
                          double ra, double rb, hipStream_t st);
// qbar_v += scale * (receiver basis row)^T resid for every receiver
hipError_t launch_adj_receivers(const Dev& d, void* qbar, const double* resid, int nr, double scale,
                                hipStream_t st);
hipError_t launch_axpy(int prec, void* y, const void* x, double a, int64_t n, hipStream_t st);

}  // namespace ewdg
