// Device-side views and launchers of the steady transport solver (iHDG-II on
// a structured grid of squares or cubes).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ewdg {

// Stopping-rule state of a solve, kept on the device so that iterations can
// be queued in batches: the check after each sweep records the norm and sets
// done once the rule holds, and the sweeps queued after that return at once.
constexpr int kTrHist = 64;              // ring of per-iteration norms (iteration k at k % kTrHist)
struct TrCtl {
  int64_t done = 0;                      // 0 while iterating, else the stopping iteration
  int64_t bad = 0;                       // 1 if that iteration's norm was not finite
  int64_t exact = 0;                     // 1: norm = ||u^k - u^e||, stop on its change; 0: ||u^k - u^{k-1}||
  double prev = 0;                       // the previous iteration's norm
  double rest = 0;                       // sum of J ||u^e - projection||^2 (exact mode)
  double tol = 0;
  double hist[kTrHist] = {};
};

// Elements are numbered e = i_0 + n i_1 + n^2 i_2.  Np = (p+1)^d modal
// coefficients per element (orthonormal Legendre tensor basis), Nq = (p+3)^d
// volume points and Nqf = (p+3)^(d-1) points per face.
struct TrDev {
  int d = 0, p = 0, n = 0, prec = 0, Np = 0, Nq = 0, Nqf = 0;
  int64_t E = 0;
  double J = 0, Jf = 0;                  // (h/2)^d, (h/2)^(d-1)
  double bn[3] = {0, 0, 0};              // beta . n on the inflow face of each axis (< 0)
  int in_side[3] = {0, 0, 0};            // inflow side of each axis (0: low, 1: high)
  void* u[2] = {nullptr, nullptr};       // run precision [E][Np] iterates
  void* c = nullptr;                     // run precision [E][Np] A^-1 (load - boundary inflow)
  void* Gt = nullptr;                    // run precision [d][Np j][Np i] = (G_a)_ij, G_a = -A^-1 bn_a Jf C_a
  void* Gfrag = nullptr;                 // run precision [d][RT][KS][64]: G_a in 16x16x4 A-fragment order
                                         // (lane l: row 16 R + l % 16, column 4 kk + l / 16; zero padded)
  double* uep = nullptr;                 // FP64 [E][Np] projection of the exact solution
  double* Ainv = nullptr;                // FP64 [Np][Np]
  double* Vq = nullptr;                  // FP64 [Nq][Np] basis at the volume points
  double* Wq = nullptr;                  // FP64 [Nq] reference weights
  double* Tf = nullptr;                  // FP64 [2d][Nqf][Np] basis on the face points (face 2a + side)
  double* Wf = nullptr;                  // FP64 [Nqf]
  double* fq = nullptr;                  // FP64 [E][Nq] staging of f
  double* gq = nullptr;                  // FP64 [E][2d][Nqf] staging of g
  double* ueq = nullptr;                 // FP64 [E][Nq] staging of the exact solution
  double* rest = nullptr;                // FP64 [2][E] J ||u^e - projection||^2_K, J ||u^e||^2_K
  double* epart = nullptr;               // FP64 [blocks] partial squared norms
  double* scal = nullptr;                // FP64 [8]
  TrCtl* ctl = nullptr;
};

hipError_t launch_tr_load(const TrDev& t, bool with_exact, hipStream_t st);
// Iteration k of a solve, skipped once ctl->done is set: u[dst] = c + sum
// over inflow axes of G_a u[src](neighbour), then the stopping rule on the sum
// over elements of J ||u[dst] - target||^2 with target = uep (to_exact) or
// u[src].
hipError_t launch_tr_iterate(const TrDev& t, int src, bool to_exact, int64_t k, hipStream_t st);
hipError_t launch_tr_values(const TrDev& t, int src, double* out, hipStream_t st);
hipError_t launch_tr_zero(const TrDev& t, int which, hipStream_t st);
int tr_sweep_blocks(const TrDev& t);
// matrix-core sweep for Np > 16: row tiles and k-steps of the padded G_a
int tr_row_tiles(int Np);
int tr_k_steps(int Np);
bool tr_uses_mma(int Np);

}  // namespace ewdg
