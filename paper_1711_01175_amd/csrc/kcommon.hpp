// Compile-time sizes shared by the HIP kernels.
#pragma once

namespace ewdg {

template <int N>
struct Sz {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;   // nodes
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;            // nodes of one face
  static constexpr int Nq = (N + 1) * (N + 1) * (N + 1);       // quadrature points
  static constexpr int NF = 4 * Nfp;
  static constexpr int NqP = (Nq + 3) / 4 * 4;                 // padded stride of lambda, mu
  static constexpr int cmax(int a, int b) { return a > b ? a : b; }
  static constexpr int BUF = cmax(9 * Np, cmax(9 * NF, 6 * Nq));
};

// Expands CALL with a compile-time NN for every supported degree.
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


}  // namespace ewdg
