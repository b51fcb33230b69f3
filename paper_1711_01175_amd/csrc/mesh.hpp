// Connectivity and affine geometry of a periodic tetrahedral mesh (host).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "refelem.hpp"

namespace ewdg {

struct MeshData {
  int64_t K = 0;
  // conn[k*4+f] = nbr*32 + (g*6 + p): neighbour element, its face g and the
  // vertex permutation p mapping our face's vertex order to the neighbour's.
  std::vector<int32_t> conn;
  std::vector<double> geo;    // [K][9] dr/dx, dr/dy, dr/dz, ds/dx, ..., dt/dz
  std::vector<double> fgeo;   // [K][4][4] outward normal (3), Fscale = sJ/J
  std::vector<double> J;      // [K] Jacobian determinant of the affine map
  std::vector<double> X0;     // [K][3] image of reference vertex v0
  std::vector<double> A;      // [K][9] map matrix, x = X0 + A (rhat + 1)
  std::vector<double> Ainv;   // [K][9]
  std::vector<double> inradius;  // [K] 3|K| / |dK|
  // boundary faces (bounded meshes): bc of every face without a partner, 2
  // bits per face (1 traction-free, 2 absorbing); such a face's conn entry
  // points at the element itself, same face, identity vertex permutation
  std::vector<int32_t> bcm;
  int bc = 0;
};

// Returns 0 on success or an error code (EWDG_EMESH / EWDG_EINVAL) with a
// message in err.  bc = 0: every face must have a partner (periodic meshes);
// 1 or 2: faces without a partner are traction-free or absorbing boundary
// faces.
int build_mesh(int64_t K, const int64_t* EToV, const double* VXYZ, MeshData& m,
               std::string& err, int bc = 0);

// Owning element of a point (all barycentrics >= -tol, lowest index on
// ties) and its reference coordinates; returns -1 if no element contains it.
int64_t locate_point(const MeshData& m, const double* x, double* rhat);

}  // namespace ewdg
