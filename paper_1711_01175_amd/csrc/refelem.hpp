// Reference tetrahedron for the nodal DG discretisation: nodes, basis,
// quadrature and the dense reference operators, all built once in FP64 on
// the host.
#pragma once
#include <cstdint>
#include <vector>

namespace ewdg {

// Reference element T = {r,s,t >= -1, r+s+t <= -1}; vertices
// v0=(-1,-1,-1), v1=(1,-1,-1), v2=(-1,1,-1), v3=(-1,-1,1).
// Face f is the ordered vertex triple kFaceVerts[f].
extern const int kFaceVerts[4][3];

struct RefElem {
  int N = 0, Np = 0, Nfp = 0, Nq = 0;
  std::vector<double> r, s, t;            // nodes [Np]
  std::vector<double> V, Vinv;            // [Np][Np] row = node, col = mode
  std::vector<double> Dr, Ds, Dt;         // [Np][Np] nodal derivative matrices
  std::vector<double> Mhat;               // [Np][Np] reference mass (nodal)
  std::vector<double> LIFT;               // [Np][4*Nfp]
  std::vector<int> Fmask;                 // [4][Nfp] volume node of face node
  std::vector<double> fbary;              // [4][Nfp][3] face-node barycentrics
  // nbrnode[((f*4+g)*6+p)*Nfp + j]: volume node (in the neighbour) holding the
  // same point as face node j of face f, when the neighbour's face is g and
  // the vertex correspondence is permutation p (see perm3()).
  std::vector<int> nbrnode;
  std::vector<double> xq, wq;             // quadrature points [Nq][3], weights [Nq]
  std::vector<double> Vq;                 // [Nq][Np] nodal -> quadrature points
  std::vector<double> Pq;                 // [Np][Nq] L2_Q projection to nodal
};

// Builds the element; returns false if N is unsupported or a construction
// step fails (singular Vandermonde, missing face nodes).
bool build_refelem(int N, RefElem& re, char* err, int errlen);

// Orthonormal Dubiner basis of P_N on T (and its gradient) at one point.
void pkdo_eval(int N, double r, double s, double t, double* psi, double* dr,
               double* ds, double* dt);

// Gauss-Jacobi rule with weight (1-x)^alpha (1+x)^beta by Golub-Welsch.
void gauss_jacobi(int n, double alpha, double beta, double* x, double* w);

// The six permutations of {0,1,2}; perm3(p)[m] = image of m.
const int* perm3(int p);
int perm3_index(const int* img);

// Dense helpers (row-major).
bool invert(int n, std::vector<double>& A);   // in place, partial pivoting
}  // namespace ewdg
