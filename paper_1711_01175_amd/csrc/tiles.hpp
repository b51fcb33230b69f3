// Matrix-core tiles and the padded tile shapes shared by the stage and
// adjoint kernels (HIP, gfx950).
#pragma once
#include <hip/hip_runtime.h>

#include "kcommon.hpp"

// Tuning constants of the stage kernel (compile time; values measured on
// MI355X at N=4):
//  EWDG_SV, EWDG_SE, EWDG_SF, EWDG_SQ: LDS row strides (values) of the 3-,
//    6-, 9- and 6-field operand buffers, 16 element columns per field;
//  EWDG_QC: quadrature points per projection chunk;
//  EWDG_CW, EWDG_CW64, EWDG_CW32: W_rho column values whose loads issue
//    together: FP64 at N >= 5 (40; 20 was 1 % slower at N = 7), FP64 up to
//    N = 4 (20; 12 to 24 alike, 1 % faster than 40), FP32 at N = 7 (16; 12 to
//    16 alike, 5 % faster than 40).  FP32 up to N = 5 takes the whole row
//    (N = 5: 56 values, 1.4 % faster than 40);
//  EWDG_OCC32: FP32 waves per SIMD asked of the register allocator.
#ifndef EWDG_SV
#define EWDG_SV 48
#endif
#ifndef EWDG_SE
#define EWDG_SE 97
#endif
#ifndef EWDG_SF
#define EWDG_SF 144
#endif
#ifndef EWDG_SQ
#define EWDG_SQ 96
#endif
#ifndef EWDG_QC
#define EWDG_QC 64
#endif
#ifndef EWDG_CW
#define EWDG_CW 40
#endif
#ifndef EWDG_CW64
#define EWDG_CW64 20
#endif
#ifndef EWDG_CW32
#define EWDG_CW32 16
#endif
#ifndef EWDG_OCC32
#define EWDG_OCC32 4
#endif

namespace ewdg {


// ---------------------------------------------------------------- MFMA tiles
// 16x16x4 matrix-core tiles: C[16x16] += A[16x4] B[4x16].  Lane l supplies
// A[l%16][l/16] and B[l/16][l%16].  Register r of the accumulator holds
// column l%16 and row row(l/16, r): 4(l/16)+r for FP32, 4r+(l/16) for FP64
// (measured with a layout probe on gfx950).
template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lg, int r) { return 4 * lg + r; }
};
template <>
struct Mfma<double> {
  typedef double acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lg, int r) { return 4 * r + lg; }
};

constexpr int ceil_to(int x, int m) { return (x + m - 1) / m * m; }
constexpr int cmax2(int a, int b) { return a > b ? a : b; }

// Padded shapes of the stage kernel.  A workgroup owns a tile of 16
// elements; matrix columns are (field, element) pairs, 16 per field.
template <int N>
struct Tile {
  using S = Sz<N>;
  static constexpr int Np = S::Np, Nfp = S::Nfp, Nq = S::Nq, NqP = S::NqP;
  static constexpr int E = 16;
  static constexpr int NpK = ceil_to(Np, 4);    // node index as the K dimension
  static constexpr int NpR = ceil_to(Np, 16);   // node index as the row dimension
  static constexpr int NqK = ceil_to(Nq, 4);
  static constexpr int NqR = ceil_to(Nq, 16);
  static constexpr int NfpK = ceil_to(Nfp, 4);  // face nodes of one face as K
  static constexpr int RT = NpR / 16;           // node row tiles
  static constexpr int QT = NqR / 16;           // quadrature row tiles
  // waves: 4 up to 3 node row tiles (N <= 4), else 8; waves beyond the row
  // tiles take part in the element-wise steps only.  8 waves at N = 5 (4 row
  // tiles) lower the per-thread arrays from 4 to 2 rounds and the registers
  // from 188 to 120 (FP32), doubling the waves per SIMD: 10 % faster stages.
  static constexpr int NW = RT > 3 ? 8 : 4;
  static constexpr int NT = 64 * NW;
  // LDS regions (in values): X holds v and the contravariant stresses, later
  // the strains (right-hand side, then new values) and the new sigma_h; Y
  // holds one face's interface corrections, then the velocity right-hand
  // side, later the stresses at the quadrature points.  Where they fit, Y
  // also keeps the element's own stresses beside the face buffer and the
  // strain right-hand side beside the velocity one (v then stays in X until
  // the update).
  // LDS row strides (values) of the B-operand buffers: 3, 6, 9 and 6 fields
  // of 16 element columns, padded against bank conflicts
  static constexpr int SV = EWDG_SV, SE = EWDG_SE, SF = EWDG_SF, SQ = EWDG_SQ;
  static constexpr int X = cmax2(2 * NpK * SV, NpK * SE);
  static constexpr int QC = NqR < EWDG_QC ? NqR : EWDG_QC;   // quadrature rows per chunk (whole tiles)
  static constexpr int Y = cmax2(cmax2(NfpK * SF, QC * SQ), NpK * SV);
  // per element in LDS: dr/dx (9), per face n and Fscale (16), own Z_p, Z_s
  // and the neighbour's across each face (10), padded to 36
  static constexpr int GS = 36;
  static constexpr int GEO = E * GS;
};

}  // namespace ewdg
