// Connectivity from shared vertex triples and affine geometry (host, FP64).
#include "mesh.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <unordered_map>

#include "ewdg.h"

namespace ewdg {

namespace {
struct TripleHash {
  size_t operator()(const std::array<int64_t, 3>& a) const {
    uint64_t h = 1469598103934665603ull;
    for (int i = 0; i < 3; ++i) {
      h ^= static_cast<uint64_t>(a[i]) + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
    }
    return static_cast<size_t>(h);
  }
};
}  // namespace

int build_mesh(int64_t K, const int64_t* EToV, const double* VXYZ, MeshData& m,
               std::string& err, int bc) {
  if (K <= 0 || K >= (int64_t(1) << 26)) {
    err = "element count out of range";
    return EWDG_EINVAL;
  }
  m.K = K;
  m.conn.assign(K * 4, -1);
  m.geo.assign(K * 9, 0.0);
  m.fgeo.assign(K * 16, 0.0);
  m.J.assign(K, 0.0);
  m.X0.assign(K * 3, 0.0);
  m.A.assign(K * 9, 0.0);
  m.Ainv.assign(K * 9, 0.0);
  m.inradius.assign(K, 0.0);

  // Geometry.
  for (int64_t k = 0; k < K; ++k) {
    const double* X = VXYZ + k * 12;
    double A[9];
    for (int d = 0; d < 3; ++d)
      for (int c = 0; c < 3; ++c) A[d * 3 + c] = 0.5 * (X[(c + 1) * 3 + d] - X[d]);
    const double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                       A[2] * (A[3] * A[7] - A[4] * A[6]);
    if (!(det > 0.0)) {
      err = "element " + std::to_string(k) + " has non-positive Jacobian";
      return EWDG_EMESH;
    }
    double Ai[9];
    Ai[0] = (A[4] * A[8] - A[5] * A[7]) / det;
    Ai[1] = (A[2] * A[7] - A[1] * A[8]) / det;
    Ai[2] = (A[1] * A[5] - A[2] * A[4]) / det;
    Ai[3] = (A[5] * A[6] - A[3] * A[8]) / det;
    Ai[4] = (A[0] * A[8] - A[2] * A[6]) / det;
    Ai[5] = (A[2] * A[3] - A[0] * A[5]) / det;
    Ai[6] = (A[3] * A[7] - A[4] * A[6]) / det;
    Ai[7] = (A[1] * A[6] - A[0] * A[7]) / det;
    Ai[8] = (A[0] * A[4] - A[1] * A[3]) / det;
    m.J[k] = det;
    for (int i = 0; i < 9; ++i) {
      m.A[k * 9 + i] = A[i];
      m.Ainv[k * 9 + i] = Ai[i];
      m.geo[k * 9 + i] = Ai[i];   // row i: d r_i / d x_j
    }
    for (int d = 0; d < 3; ++d) m.X0[k * 3 + d] = X[d];
    double area_sum = 0.0;
    for (int f = 0; f < 4; ++f) {
      const int* fv = kFaceVerts[f];
      const int opp = 6 - fv[0] - fv[1] - fv[2];
      double e1[3], e2[3], cr[3], to[3];
      for (int d = 0; d < 3; ++d) {
        e1[d] = X[fv[1] * 3 + d] - X[fv[0] * 3 + d];
        e2[d] = X[fv[2] * 3 + d] - X[fv[0] * 3 + d];
        to[d] = X[opp * 3 + d] - X[fv[0] * 3 + d];
      }
      cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
      cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
      cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
      const double nrm = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
      double sgn = (cr[0] * to[0] + cr[1] * to[1] + cr[2] * to[2] > 0) ? -1.0 : 1.0;
      const double area = 0.5 * nrm;
      area_sum += area;
      for (int d = 0; d < 3; ++d) m.fgeo[k * 16 + f * 4 + d] = sgn * cr[d] / nrm;
      // surface Jacobian against the reference triangle of area 2
      m.fgeo[k * 16 + f * 4 + 3] = (area / 2.0) / det;
    }
    m.inradius[k] = 3.0 * (det * 4.0 / 3.0) / area_sum;
  }

  // Connectivity: faces are matched by their sorted vertex-id triples.
  std::unordered_map<std::array<int64_t, 3>, int64_t, TripleHash> table;
  table.reserve(static_cast<size_t>(K) * 3);
  for (int64_t k = 0; k < K; ++k)
    for (int f = 0; f < 4; ++f) {
      std::array<int64_t, 3> key = {EToV[k * 4 + kFaceVerts[f][0]], EToV[k * 4 + kFaceVerts[f][1]],
                                    EToV[k * 4 + kFaceVerts[f][2]]};
      if (key[0] == key[1] || key[1] == key[2] || key[0] == key[2]) {
        err = "degenerate face (repeated vertex id) in element " + std::to_string(k);
        return EWDG_EMESH;
      }
      std::sort(key.begin(), key.end());
      auto it = table.find(key);
      if (it == table.end()) {
        table.emplace(key, k * 4 + f);
        continue;
      }
      const int64_t other = it->second;
      if (other < 0) {
        err = "face shared by more than two elements";
        return EWDG_EMESH;
      }
      const int64_t k2 = other / 4;
      const int g = static_cast<int>(other % 4);
      // permutation: our vertex m sits at the neighbour's position img[m]
      int img[3], img2[3];
      for (int a = 0; a < 3; ++a) {
        img[a] = img2[a] = -1;
        for (int b = 0; b < 3; ++b) {
          if (EToV[k2 * 4 + kFaceVerts[g][b]] == EToV[k * 4 + kFaceVerts[f][a]]) img[a] = b;
          if (EToV[k * 4 + kFaceVerts[f][b]] == EToV[k2 * 4 + kFaceVerts[g][a]]) img2[a] = b;
        }
      }
      const int p = perm3_index(img), p2 = perm3_index(img2);
      if (p < 0 || p2 < 0) {
        err = "inconsistent face vertices";
        return EWDG_EMESH;
      }
      m.conn[k * 4 + f] = static_cast<int32_t>(k2 * 32 + g * 6 + p);
      m.conn[k2 * 4 + g] = static_cast<int32_t>(k * 32 + f * 6 + p2);
      it->second = -1;
    }
  m.bc = bc;
  m.bcm.assign(K, 0);
  for (int64_t i = 0; i < K * 4; ++i)
    if (m.conn[i] < 0) {
      if (bc == 0) {
        err = "face without a partner (a periodic mesh was asked for)";
        return EWDG_EMESH;
      }
      const int64_t k = i / 4;
      const int f = static_cast<int>(i % 4);
      m.conn[i] = static_cast<int32_t>(k * 32 + f * 6);   // itself, same face, identity permutation
      m.bcm[k] |= bc << (2 * f);
    }
  return EWDG_OK;
}

int64_t locate_point(const MeshData& m, const double* x, double* rhat) {
  const double tol = 1e-12;
  for (int64_t k = 0; k < m.K; ++k) {
    const double* Ai = &m.Ainv[k * 9];
    double d[3] = {x[0] - m.X0[k * 3], x[1] - m.X0[k * 3 + 1], x[2] - m.X0[k * 3 + 2]};
    double rh[3];
    for (int i = 0; i < 3; ++i) rh[i] = Ai[i * 3] * d[0] + Ai[i * 3 + 1] * d[1] + Ai[i * 3 + 2] * d[2] - 1.0;
    const double l0 = -0.5 * (1.0 + rh[0] + rh[1] + rh[2]);
    const double l1 = 0.5 * (1.0 + rh[0]), l2 = 0.5 * (1.0 + rh[1]), l3 = 0.5 * (1.0 + rh[2]);
    if (l0 >= -tol && l1 >= -tol && l2 >= -tol && l3 >= -tol) {
      for (int i = 0; i < 3; ++i) rhat[i] = rh[i];
      return k;
    }
  }
  return -1;
}

}  // namespace ewdg
