// Device-side views and launchers of the locally implicit (iHDG-II) step.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "dev.hpp"

namespace ewdg {

// Pointers into the caller's implicit workspace.  nv = 9 Np unknowns per
// element; n = nv rounded up to 16 is the stride of one local matrix.
struct ImpDev {
  int nv = 0, n = 0;
  void* inv = nullptr;        // run precision [K][n][n]: inv[k][j][i] = (B_k^-1)_ij
  double* work = nullptr;     // FP64 [K][n][n]: B_k^T during set-up, (B_k^T)^-1 after (== inv in FP64)
  void* b = nullptr;          // [K][9][Np] fixed part of the local right-hand sides; probe state in set-up
  void* L = nullptr;          // [K][9][Np] operator output
  void* s = nullptr;          // [K][6][Np] sigma_h of the operator input
  int32_t* members = nullptr; // [K] elements ordered by colour class
  double* epart = nullptr;    // [K] per-element squared L2 norm of the iterate change
  double* norm2 = nullptr;    // [1] squared L2 norm of the iterate change
  int32_t* flag = nullptr;    // [1] set when a local matrix has a vanishing pivot
};

// Identity in each of the K n x n matrices of W.
hipError_t launch_imp_identity(double* W, int64_t K, int n, hipStream_t st);
// Zero a run-precision array of count values.
hipError_t launch_imp_zero(int prec, void* x, int64_t count, hipStream_t st);
// On the cnt elements listed in members: q[k][j_off] = 0 (j_off >= 0), q[k][j_on] = 1 (j_on >= 0).
hipError_t launch_imp_probe(int prec, void* q, const int32_t* members, int cnt, int nv, int j_off, int j_on,
                            hipStream_t st);
// On the listed elements: W[k][j][i] = delta_ij - thdt L[k][i] (row j of B_k^T).
hipError_t launch_imp_gather(int prec, const void* L, double* W, const int32_t* members, int cnt, int nv, int n,
                             int j, double thdt, hipStream_t st);
// In-place inverse of each n x n matrix (block Gauss-Jordan, 16-wide pivot blocks, no row exchange).
hipError_t launch_imp_invert(double* W, int64_t K, int n, int32_t* flag, hipStream_t st);
// out[i] = (float) W[i].
hipError_t launch_imp_to_float(const double* W, float* out, int64_t count, hipStream_t st);
// b = q + c1 L (L may be null when c1 == 0), plus sv dir (x) svec on the velocity rows of src_elem.
hipError_t launch_imp_fixed(const Dev& d, const ImpDev& m, const void* q, const void* L, double c1,
                            int64_t src_elem, double sv, const double dir[3], hipStream_t st);
// q += B^-1 (b + thdt L - q) on every element; m.norm2 = ||change||^2_{L2}.
hipError_t launch_imp_iterate(const Dev& d, const ImpDev& m, void* q, double thdt, hipStream_t st);

}  // namespace ewdg
