// Reference tetrahedron: warp & blend nodes, Dubiner basis, Stroud
// quadrature and the dense reference operators (FP64, host).
//
// Published methods followed here, each written from its description:
//  * the orthonormal Jacobi polynomials by their three-term recurrence and
//    the orthonormal simplex (Proriol-Koornwinder-Dubiner) basis on the
//    tetrahedron in collapsed coordinates, with its gradients, as set out in
//    Hesthaven & Warburton, Nodal Discontinuous Galerkin Methods (Springer,
//    2008), chapters 3, 6 and 10;
//  * the warp & blend node set of Warburton, J. Eng. Math. 56 (2006);
//  * Gauss-Jacobi rules from the eigenvalues of the Jacobi matrix
//    (Golub & Welsch, Math. Comp. 23, 1969) and the conical product
//    (Stroud) rule built from them.
#include "refelem.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

namespace ewdg {

const int kFaceVerts[4][3] = {{0, 1, 2}, {0, 1, 3}, {1, 2, 3}, {0, 2, 3}};

static const int kPerm3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2},
                                 {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
const int* perm3(int p) { return kPerm3[p]; }
int perm3_index(const int* img) {
  for (int p = 0; p < 6; ++p)
    if (kPerm3[p][0] == img[0] && kPerm3[p][1] == img[1] && kPerm3[p][2] == img[2]) return p;
  return -1;
}

// ------------------------------------------------------------------ linear algebra
bool invert(int n, std::vector<double>& A) {
  std::vector<int> piv(n);
  std::vector<double> inv(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) inv[i * n + i] = 1.0;
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[i * n + k]) > std::fabs(A[p * n + k])) p = i;
    if (std::fabs(A[p * n + k]) < 1e-300) return false;
    if (p != k)
      for (int j = 0; j < n; ++j) {
        std::swap(A[k * n + j], A[p * n + j]);
        std::swap(inv[k * n + j], inv[p * n + j]);
      }
    const double d = 1.0 / A[k * n + k];
    for (int j = 0; j < n; ++j) {
      A[k * n + j] *= d;
      inv[k * n + j] *= d;
    }
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      const double f = A[i * n + k];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        A[i * n + j] -= f * A[k * n + j];
        inv[i * n + j] -= f * inv[k * n + j];
      }
    }
  }
  A.swap(inv);
  return true;
}

// Symmetric eigenproblem by cyclic Jacobi rotations: A (n x n, row-major) is
// overwritten by a diagonal matrix of eigenvalues, Q receives eigenvectors
// as columns.
static void sym_eig(int n, std::vector<double>& A, std::vector<double>& Q) {
  Q.assign(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) Q[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += A[i * n + j] * A[i * n + j];
        if (i != j) off += A[i * n + j] * A[i * n + j];
      }
    if (off <= 1e-32 * tot) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        const double tt = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(tt * tt + 1.0), s = tt * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double qkp = Q[k * n + p], qkq = Q[k * n + q];
          Q[k * n + p] = c * qkp - s * qkq;
          Q[k * n + q] = s * qkp + c * qkq;
        }
      }
  }
}

void gauss_jacobi(int n, double al, double be, double* x, double* w) {
  // Golub-Welsch: nodes are the eigenvalues of the Jacobi matrix of the
  // monic three-term recurrence; weights are mu0 times the squared first
  // eigenvector components.
  std::vector<double> J(static_cast<size_t>(n) * n, 0.0), Q;
  for (int k = 0; k < n; ++k) {
    const double s = 2.0 * k + al + be;
    J[k * n + k] = (k == 0) ? (be - al) / (al + be + 2.0) : (be * be - al * al) / (s * (s + 2.0));
    if (k + 1 < n) {
      const double m = k + 1.0, sm = 2.0 * m + al + be;
      const double b2 = 4.0 * m * (m + al) * (m + be) * (m + al + be) /
                        (sm * sm * (sm + 1.0) * (sm - 1.0));
      J[k * n + k + 1] = J[(k + 1) * n + k] = std::sqrt(b2);
    }
  }
  sym_eig(n, J, Q);
  const double mu0 = std::pow(2.0, al + be + 1.0) * std::tgamma(al + 1.0) * std::tgamma(be + 1.0) /
                     std::tgamma(al + be + 2.0);
  std::vector<std::pair<double, double>> xw(n);
  for (int i = 0; i < n; ++i) xw[i] = {J[i * n + i], mu0 * Q[i] * Q[i]};
  std::sort(xw.begin(), xw.end());
  for (int i = 0; i < n; ++i) {
    x[i] = xw[i].first;
    w[i] = xw[i].second;
  }
}

// ------------------------------------------------------------------ basis
// Orthonormal Jacobi polynomials P_0..P_n at x (weight (1-x)^a (1+x)^b).
static void jacobi_all(int n, double a, double b, double x, double* P) {
  const double g0 = std::pow(2.0, a + b + 1.0) / (a + b + 1.0) * std::tgamma(a + 1.0) *
                    std::tgamma(b + 1.0) / std::tgamma(a + b + 1.0);
  P[0] = 1.0 / std::sqrt(g0);
  if (n == 0) return;
  const double g1 = (a + 1.0) * (b + 1.0) / (a + b + 3.0) * g0;
  P[1] = ((a + b + 2.0) * x / 2.0 + (a - b) / 2.0) / std::sqrt(g1);
  if (n == 1) return;
  double aold = 2.0 / (2.0 + a + b) * std::sqrt((a + 1.0) * (b + 1.0) / (a + b + 3.0));
  for (int i = 1; i < n; ++i) {
    const double h1 = 2.0 * i + a + b;
    const double anew = 2.0 / (h1 + 2.0) *
                        std::sqrt((i + 1.0) * (i + 1.0 + a + b) * (i + 1.0 + a) * (i + 1.0 + b) /
                                  ((h1 + 1.0) * (h1 + 3.0)));
    const double bnew = -(a * a - b * b) / (h1 * (h1 + 2.0));
    P[i + 1] = ((x - bnew) * P[i] - aold * P[i - 1]) / anew;
    aold = anew;
  }
}

static double jac(int n, double a, double b, double x) {
  double P[32];
  jacobi_all(n, a, b, x, P);
  return P[n];
}

static double djac(int n, double a, double b, double x) {
  if (n == 0) return 0.0;
  return std::sqrt(n * (n + a + b + 1.0)) * jac(n - 1, a + 1.0, b + 1.0, x);
}

static inline double ipow(double x, int e) {
  double r = 1.0;
  for (int i = 0; i < e; ++i) r *= x;
  return r;
}

void pkdo_eval(int N, double r, double s, double t, double* psi, double* dr, double* ds,
               double* dt) {
  // Collapsed coordinates; on the singular edge/vertex any value of a (b)
  // gives the limit because the cancelled formulas below are polynomial
  // in (a, b, c).
  const double tol = 1e-12;
  const double a = (std::fabs(s + t) > tol) ? 2.0 * (1.0 + r) / (-s - t) - 1.0 : -1.0;
  const double b = (std::fabs(t - 1.0) > tol) ? 2.0 * (1.0 + s) / (1.0 - t) - 1.0 : -1.0;
  const double c = t;
  const double sq8 = std::sqrt(8.0);
  int m = 0;
  for (int i = 0; i <= N; ++i)
    for (int j = 0; j <= N - i; ++j)
      for (int k = 0; k <= N - i - j; ++k, ++m) {
        const double A = jac(i, 0, 0, a), dA = djac(i, 0, 0, a);
        const double B = jac(j, 2.0 * i + 1.0, 0, b), dB = djac(j, 2.0 * i + 1.0, 0, b);
        const double C = jac(k, 2.0 * (i + j) + 2.0, 0, c), dC = djac(k, 2.0 * (i + j) + 2.0, 0, c);
        psi[m] = sq8 * A * ipow(1.0 - b, i) * B * ipow(1.0 - c, i + j) * C;
        if (!dr) continue;
        // psi_r, and the pieces coming through b and c (negative powers only
        // ever multiply terms that vanish identically).
        const double Tr = (i > 0) ? 4.0 * sq8 * dA * ipow(1.0 - b, i - 1) * B * ipow(1.0 - c, i + j - 1) * C : 0.0;
        double Tb = 0.0;
        if (i + j > 0) {
          double br = ipow(1.0 - b, i) * dB;
          if (i > 0) br -= i * ipow(1.0 - b, i - 1) * B;
          Tb = 2.0 * sq8 * A * ipow(1.0 - c, i + j - 1) * C * br;
        }
        double cr = ipow(1.0 - c, i + j) * dC;
        if (i + j > 0) cr -= (i + j) * ipow(1.0 - c, i + j - 1) * C;
        const double Tc = sq8 * A * ipow(1.0 - b, i) * B * cr;
        dr[m] = Tr;
        ds[m] = 0.5 * (1.0 + a) * Tr + Tb;
        dt[m] = 0.5 * (1.0 + a) * Tr + 0.5 * (1.0 + b) * Tb + Tc;
      }
}

// Orthonormal basis on the triangle {u,v >= -1, u+v <= 0}.
static void pkd2_eval(int N, double u, double v, double* psi) {
  const double a = (std::fabs(v - 1.0) > 1e-12) ? 2.0 * (1.0 + u) / (1.0 - v) - 1.0 : -1.0;
  const double b = v;
  int m = 0;
  for (int i = 0; i <= N; ++i)
    for (int j = 0; j <= N - i; ++j, ++m)
      psi[m] = std::sqrt(2.0) * jac(i, 0, 0, a) * jac(j, 2.0 * i + 1.0, 0, b) * ipow(1.0 - b, i);
}

// ------------------------------------------------------------------ nodes
// Warp & blend nodes (Warburton 2006) with blending parameter alpha = 0:
// equispaced barycentric points on an equilateral tetrahedron are displaced
// along each edge by the 1-D Gauss-Lobatto warp, blended into the faces and
// from the faces into the volume.
static void warp_blend_nodes(int N, std::vector<double>& r, std::vector<double>& s,
                             std::vector<double>& t) {
  // 1-D warp: displacement of the Gauss-Lobatto points from equispaced ones,
  // interpolated on the equispaced points.
  std::vector<double> xg(N + 1), xe(N + 1);
  xg[0] = -1.0;
  xg[N] = 1.0;
  if (N > 1) {
    std::vector<double> w(N - 1);
    gauss_jacobi(N - 1, 1.0, 1.0, &xg[1], w.data());
  }
  for (int i = 0; i <= N; ++i) xe[i] = -1.0 + 2.0 * i / N;
  auto warp = [&](double x) {
    if (std::fabs(x) > 1.0 - 1e-10) return 0.0;
    double acc = 0.0;
    for (int i = 0; i <= N; ++i) {
      double l = 1.0;
      for (int j = 0; j <= N; ++j)
        if (j != i) l *= (x - xe[j]) / (xe[i] - xe[j]);
      acc += (xg[i] - xe[i]) * l;
    }
    return acc / (1.0 - x * x);
  };
  // Regular tetrahedron with edges of length 2.
  const double P[4][3] = {{-1.0, -1.0 / std::sqrt(3.0), -1.0 / std::sqrt(6.0)},
                          {1.0, -1.0 / std::sqrt(3.0), -1.0 / std::sqrt(6.0)},
                          {0.0, 2.0 / std::sqrt(3.0), -1.0 / std::sqrt(6.0)},
                          {0.0, 0.0, 3.0 / std::sqrt(6.0)}};
  const double tol = 1e-10;
  r.clear(); s.clear(); t.clear();
  for (int k = 0; k <= N; ++k)
    for (int j = 0; j <= N - k; ++j)
      for (int i = 0; i <= N - k - j; ++i) {
        double L[4] = {1.0 - double(i + j + k) / N, double(i) / N, double(j) / N, double(k) / N};
        double X[3] = {0, 0, 0}, shift[3] = {0, 0, 0}, over[3] = {0, 0, 0};
        bool overridden = false;
        for (int v = 0; v < 4; ++v)
          for (int d = 0; d < 3; ++d) X[d] += L[v] * P[v][d];
        for (int f = 0; f < 4; ++f) {
          const int* fv = kFaceVerts[f];
          const int a = 6 - fv[0] - fv[1] - fv[2];   // opposite vertex
          double D[3] = {0, 0, 0};
          for (int e = 0; e < 3; ++e) {
            const int p = fv[e], q = fv[(e + 1) % 3];
            const double g = 4.0 * L[p] * L[q] * warp(L[q] - L[p]);
            for (int d = 0; d < 3; ++d) D[d] += g * 0.5 * (P[q][d] - P[p][d]);
          }
          const double lb = L[fv[0]], lc = L[fv[1]], ld = L[fv[2]], la = L[a];
          if (la < tol) {
            const int pos = (lb > tol) + (lc > tol) + (ld > tol);
            if (pos < 3) {
              overridden = true;
              for (int d = 0; d < 3; ++d) over[d] = D[d];
            } else {
              for (int d = 0; d < 3; ++d) shift[d] += D[d];
            }
          } else {
            const double den = (lb + 0.5 * la) * (lc + 0.5 * la) * (ld + 0.5 * la);
            const double bl = lb * lc * ld / den;
            for (int d = 0; d < 3; ++d) shift[d] += bl * D[d];
          }
        }
        for (int d = 0; d < 3; ++d) X[d] += overridden ? over[d] : shift[d];
        // back to barycentrics: solve [P1-P0, P2-P0, P3-P0] mu = X - P0
        std::vector<double> M(9);
        for (int d = 0; d < 3; ++d)
          for (int c = 0; c < 3; ++c) M[d * 3 + c] = P[c + 1][d] - P[0][d];
        invert(3, M);
        double mu[3] = {0, 0, 0};
        for (int d = 0; d < 3; ++d)
          for (int c = 0; c < 3; ++c) mu[d] += M[d * 3 + c] * (X[c] - P[0][c]);
        // snap barycentrics that are zero by construction (boundary nodes)
        const double bary[4] = {1.0 - mu[0] - mu[1] - mu[2], mu[0], mu[1], mu[2]};
        double bb[4];
        for (int v = 0; v < 4; ++v) bb[v] = (L[v] < tol) ? 0.0 : bary[v];
        r.push_back(-1.0 + 2.0 * bb[1]);
        s.push_back(-1.0 + 2.0 * bb[2]);
        t.push_back(-1.0 + 2.0 * bb[3]);
      }
}

static void bary_of(double r, double s, double t, double* L) {
  L[1] = 0.5 * (1.0 + r);
  L[2] = 0.5 * (1.0 + s);
  L[3] = 0.5 * (1.0 + t);
  L[0] = -0.5 * (1.0 + r + s + t);
}

bool build_refelem(int N, RefElem& re, char* err, int errlen) {
  auto fail = [&](const char* m) {
    std::snprintf(err, errlen, "%s", m);
    return false;
  };
  if (N < 1 || N > 8) return fail("unsupported polynomial degree");
  re.N = N;
  re.Np = (N + 1) * (N + 2) * (N + 3) / 6;
  re.Nfp = (N + 1) * (N + 2) / 2;
  re.Nq = (N + 1) * (N + 1) * (N + 1);
  const int Np = re.Np, Nfp = re.Nfp, Nq = re.Nq;
  warp_blend_nodes(N, re.r, re.s, re.t);
  if (static_cast<int>(re.r.size()) != Np) return fail("node count mismatch");

  // Vandermonde and gradients.
  re.V.assign(Np * Np, 0.0);
  std::vector<double> Vr(Np * Np), Vs(Np * Np), Vt(Np * Np);
  for (int i = 0; i < Np; ++i)
    pkdo_eval(N, re.r[i], re.s[i], re.t[i], &re.V[i * Np], &Vr[i * Np], &Vs[i * Np], &Vt[i * Np]);
  re.Vinv = re.V;
  if (!invert(Np, re.Vinv)) return fail("singular Vandermonde");
  auto matmul = [](int n, int m, int l, const double* A, const double* B, double* C) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < l; ++j) {
        double acc = 0.0;
        for (int k = 0; k < m; ++k) acc += A[i * m + k] * B[k * l + j];
        C[i * l + j] = acc;
      }
  };
  re.Dr.assign(Np * Np, 0.0);
  re.Ds.assign(Np * Np, 0.0);
  re.Dt.assign(Np * Np, 0.0);
  matmul(Np, Np, Np, Vr.data(), re.Vinv.data(), re.Dr.data());
  matmul(Np, Np, Np, Vs.data(), re.Vinv.data(), re.Ds.data());
  matmul(Np, Np, Np, Vt.data(), re.Vinv.data(), re.Dt.data());
  // Mhat = Vinv^T Vinv ; Mhat^-1 = V V^T
  std::vector<double> VinvT(Np * Np), VT(Np * Np), MinvHat(Np * Np);
  for (int i = 0; i < Np; ++i)
    for (int j = 0; j < Np; ++j) {
      VinvT[i * Np + j] = re.Vinv[j * Np + i];
      VT[i * Np + j] = re.V[j * Np + i];
    }
  re.Mhat.assign(Np * Np, 0.0);
  matmul(Np, Np, Np, VinvT.data(), re.Vinv.data(), re.Mhat.data());
  matmul(Np, Np, Np, re.V.data(), VT.data(), MinvHat.data());

  // Faces: nodes whose barycentric coordinate opposite the face vanishes.
  re.Fmask.assign(4 * Nfp, -1);
  re.fbary.assign(4 * Nfp * 3, 0.0);
  for (int f = 0; f < 4; ++f) {
    const int* fv = kFaceVerts[f];
    const int opp = 6 - fv[0] - fv[1] - fv[2];
    int cnt = 0;
    for (int i = 0; i < Np; ++i) {
      double L[4];
      bary_of(re.r[i], re.s[i], re.t[i], L);
      if (std::fabs(L[opp]) < 1e-10) {
        if (cnt >= Nfp) return fail("too many face nodes");
        re.Fmask[f * Nfp + cnt] = i;
        for (int m = 0; m < 3; ++m) re.fbary[(f * Nfp + cnt) * 3 + m] = L[fv[m]];
        ++cnt;
      }
    }
    if (cnt != Nfp) return fail("face node count mismatch");
  }
  // Face mass matrices and LIFT = Mhat^-1 E.
  std::vector<double> Emat(Np * 4 * Nfp, 0.0);
  for (int f = 0; f < 4; ++f) {
    std::vector<double> V2(Nfp * Nfp);
    for (int j = 0; j < Nfp; ++j) {
      const double u = -1.0 + 2.0 * re.fbary[(f * Nfp + j) * 3 + 1];
      const double v = -1.0 + 2.0 * re.fbary[(f * Nfp + j) * 3 + 2];
      pkd2_eval(N, u, v, &V2[j * Nfp]);
    }
    std::vector<double> Mf(Nfp * Nfp), V2T(Nfp * Nfp);
    for (int i = 0; i < Nfp; ++i)
      for (int j = 0; j < Nfp; ++j) V2T[i * Nfp + j] = V2[j * Nfp + i];
    matmul(Nfp, Nfp, Nfp, V2.data(), V2T.data(), Mf.data());
    if (!invert(Nfp, Mf)) return fail("singular face Vandermonde");
    for (int i = 0; i < Nfp; ++i)
      for (int j = 0; j < Nfp; ++j)
        Emat[re.Fmask[f * Nfp + i] * (4 * Nfp) + f * Nfp + j] += Mf[i * Nfp + j];
  }
  re.LIFT.assign(Np * 4 * Nfp, 0.0);
  matmul(Np, Np, 4 * Nfp, MinvHat.data(), Emat.data(), re.LIFT.data());

  // Neighbour node tables for every (own face, neighbour face, vertex
  // permutation): same barycentric point with permuted vertex roles.
  re.nbrnode.assign(4 * 4 * 6 * Nfp, -1);
  for (int f = 0; f < 4; ++f)
    for (int g = 0; g < 4; ++g)
      for (int p = 0; p < 6; ++p) {
        const int* pm = perm3(p);
        for (int j = 0; j < Nfp; ++j) {
          const double* b = &re.fbary[(f * Nfp + j) * 3];
          int found = -1;
          for (int jj = 0; jj < Nfp; ++jj) {
            const double* bb = &re.fbary[(g * Nfp + jj) * 3];
            bool ok = true;
            for (int m = 0; m < 3; ++m)
              if (std::fabs(bb[pm[m]] - b[m]) > 1e-9) ok = false;
            if (ok) { found = jj; break; }
          }
          if (found < 0) return fail("face node set not symmetric");
          re.nbrnode[((f * 4 + g) * 6 + p) * Nfp + j] = re.Fmask[g * Nfp + found];
        }
      }

  // Stroud conical-product quadrature, first collapsed index fastest.
  const int m = N + 1;
  std::vector<double> a(m), wa(m), b(m), wb(m), c(m), wc(m);
  gauss_jacobi(m, 0.0, 0.0, a.data(), wa.data());
  gauss_jacobi(m, 1.0, 0.0, b.data(), wb.data());
  gauss_jacobi(m, 2.0, 0.0, c.data(), wc.data());
  re.xq.assign(Nq * 3, 0.0);
  re.wq.assign(Nq, 0.0);
  for (int k = 0; k < m; ++k)
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) {
        const int q = i + m * (j + m * k);
        re.xq[q * 3 + 0] = (1.0 + a[i]) * (1.0 - b[j]) * (1.0 - c[k]) / 4.0 - 1.0;
        re.xq[q * 3 + 1] = (1.0 + b[j]) * (1.0 - c[k]) / 2.0 - 1.0;
        re.xq[q * 3 + 2] = c[k];
        re.wq[q] = wa[i] * wb[j] * wc[k] / 8.0;
      }
  // Vq = Phi(xq) V^-1 ; Pq = Mhat^-1 Vq^T diag(w)
  std::vector<double> Phi(Nq * Np);
  for (int q = 0; q < Nq; ++q)
    pkdo_eval(N, re.xq[q * 3], re.xq[q * 3 + 1], re.xq[q * 3 + 2], &Phi[q * Np], nullptr,
              nullptr, nullptr);
  re.Vq.assign(Nq * Np, 0.0);
  matmul(Nq, Np, Np, Phi.data(), re.Vinv.data(), re.Vq.data());
  std::vector<double> VqTW(Np * Nq);
  for (int i = 0; i < Np; ++i)
    for (int q = 0; q < Nq; ++q) VqTW[i * Nq + q] = re.Vq[q * Np + i] * re.wq[q];
  re.Pq.assign(Np * Nq, 0.0);
  matmul(Np, Np, Nq, MinvHat.data(), VqTW.data(), re.Pq.data());
  return true;
}

}  // namespace ewdg
