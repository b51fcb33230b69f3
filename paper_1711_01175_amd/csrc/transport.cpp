// Host runtime of the steady transport solver: reference operators of the
// tensor-product Legendre basis (FP64), workspace layout, problem upload and
// the iHDG-II loop with the stopping rule of Sec. 6.1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "ewdg.h"
#include "refelem.hpp"
#include "trdev.hpp"

using namespace ewdg;

struct ewdg_tr {
  TrDev t;
  hipStream_t stream = nullptr;
  double beta[3] = {0, 0, 0};
  double h = 0;
  std::vector<double> Ainv, Vq, Wq, Tf, Wf, Gt;
  std::vector<double> xq1;               // fine 1-D points
  bool bound = false, has_problem = false, has_exact = false;
  double rest_total = 0.0, exact_norm2 = 0.0;
  int cur = 0;
  std::string err;
  int fail(int code, const std::string& m) {
    err = m;
    return code;
  }
  int hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return EWDG_OK;
    err = std::string(what) + ": " + hipGetErrorString(e);
    return EWDG_EHIP;
  }
  size_t tsz() const { return t.prec == 32 ? 4 : 8; }
};

namespace {

// Orthonormal Legendre polynomials sqrt((2k+1)/2) P_k and derivatives at x.
void legendre(int p, double x, double* v, double* dv) {
  std::vector<double> P(p + 2), D(p + 2);
  P[0] = 1.0;
  D[0] = 0.0;
  if (p >= 1) {
    P[1] = x;
    D[1] = 1.0;
  }
  for (int k = 1; k < p; ++k) {
    P[k + 1] = ((2 * k + 1) * x * P[k] - k * P[k - 1]) / (k + 1);
    D[k + 1] = D[k - 1] + (2 * k + 1) * P[k];
  }
  for (int k = 0; k <= p; ++k) {
    const double s = std::sqrt((2 * k + 1) / 2.0);
    v[k] = s * P[k];
    if (dv) dv[k] = s * D[k];
  }
}

int ipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// digit a (base m) of a multi-index number, first digit fastest
int digit(int idx, int a, int m) {
  for (int i = 0; i < a; ++i) idx /= m;
  return idx % m;
}

void build_operators(ewdg_tr* T) {
  TrDev& t = T->t;
  const int d = t.d, p = t.p, m = p + 1, mq = p + 3, Np = t.Np, Nq = t.Nq, Nqf = t.Nqf;
  std::vector<double> x(mq), w(mq);
  gauss_jacobi(mq, 0.0, 0.0, x.data(), w.data());
  T->xq1 = x;
  // 1-D basis at the fine points and at the ends
  std::vector<double> L(static_cast<size_t>(mq) * m), DL(static_cast<size_t>(mq) * m), E(2 * m);
  for (int q = 0; q < mq; ++q) legendre(p, x[q], &L[q * m], &DL[q * m]);
  legendre(p, -1.0, &E[0], nullptr);
  legendre(p, 1.0, &E[m], nullptr);
  // volume: phi_I(x_Q), d phi_I / d xi_a (x_Q), weights
  T->Vq.assign(static_cast<size_t>(Nq) * Np, 0.0);
  T->Wq.assign(Nq, 1.0);
  std::vector<double> dV(static_cast<size_t>(d) * Nq * Np, 0.0);
  for (int Q = 0; Q < Nq; ++Q) {
    for (int a = 0; a < d; ++a) T->Wq[Q] *= w[digit(Q, a, mq)];
    for (int I = 0; I < Np; ++I) {
      double v = 1.0;
      for (int a = 0; a < d; ++a) v *= L[digit(Q, a, mq) * m + digit(I, a, m)];
      T->Vq[static_cast<size_t>(Q) * Np + I] = v;
      for (int a = 0; a < d; ++a) {
        double g = 1.0;
        for (int b = 0; b < d; ++b) {
          const int qb = digit(Q, b, mq), ib = digit(I, b, m);
          g *= (b == a) ? DL[qb * m + ib] : L[qb * m + ib];
        }
        dV[(static_cast<size_t>(a) * Nq + Q) * Np + I] = g;
      }
    }
  }
  // face points: the free axes in increasing order, first fastest
  T->Wf.assign(Nqf, 1.0);
  T->Tf.assign(static_cast<size_t>(2 * d) * Nqf * Np, 0.0);
  for (int F = 0; F < Nqf; ++F)
    for (int k = 0; k < d - 1; ++k) T->Wf[F] *= w[digit(F, k, mq)];
  for (int a = 0; a < d; ++a)
    for (int side = 0; side < 2; ++side)
      for (int F = 0; F < Nqf; ++F)
        for (int I = 0; I < Np; ++I) {
          double v = E[side * m + digit(I, a, m)];
          int k = 0;
          for (int b = 0; b < d; ++b) {
            if (b == a) continue;
            v *= L[digit(F, k, mq) * m + digit(I, b, m)];
            ++k;
          }
          T->Tf[((static_cast<size_t>(2 * a + side)) * Nqf + F) * Np + I] = v;
        }
  // local matrix A = Jf (-sum_a beta_a S_a + sum over outflow faces beta.n M_f)
  std::vector<double> A(static_cast<size_t>(Np) * Np, 0.0);
  for (int I = 0; I < Np; ++I)
    for (int J = 0; J < Np; ++J) {
      double s = 0.0;
      for (int a = 0; a < d; ++a) {
        double v = 0.0;
        for (int Q = 0; Q < Nq; ++Q)
          v += T->Wq[Q] * T->Vq[static_cast<size_t>(Q) * Np + J] * dV[(static_cast<size_t>(a) * Nq + Q) * Np + I];
        s -= T->beta[a] * v;
      }
      A[static_cast<size_t>(I) * Np + J] = s;
    }
  auto face_form = [&](int fo, int fn, int I, int J) {
    // <phi_J on face fn of the element it belongs to, phi_I on face fo>
    double v = 0.0;
    for (int F = 0; F < Nqf; ++F)
      v += T->Wf[F] * T->Tf[(static_cast<size_t>(fo) * Nqf + F) * Np + I] *
           T->Tf[(static_cast<size_t>(fn) * Nqf + F) * Np + J];
    return v;
  };
  for (int a = 0; a < d; ++a)
    for (int side = 0; side < 2; ++side) {
      const double bn = T->beta[a] * (side ? 1.0 : -1.0);
      if (bn <= 0.0) continue;
      for (int I = 0; I < Np; ++I)
        for (int J = 0; J < Np; ++J) A[static_cast<size_t>(I) * Np + J] += bn * face_form(2 * a + side, 2 * a + side, I, J);
    }
  for (double& v : A) v *= t.Jf;
  T->Ainv = A;
  invert(Np, T->Ainv);
  // G_a = -A^-1 bn_a Jf C_a on the inflow face of axis a; stored transposed
  T->Gt.assign(static_cast<size_t>(d) * Np * Np, 0.0);
  for (int a = 0; a < d; ++a) {
    const int s_in = T->beta[a] > 0.0 ? 0 : 1;
    const double bn = T->beta[a] * (s_in ? 1.0 : -1.0);
    t.in_side[a] = s_in;
    t.bn[a] = bn;
    std::vector<double> C(static_cast<size_t>(Np) * Np);
    for (int I = 0; I < Np; ++I)
      for (int J = 0; J < Np; ++J) C[static_cast<size_t>(I) * Np + J] = bn * t.Jf * face_form(2 * a + s_in, 2 * a + 1 - s_in, I, J);
    for (int I = 0; I < Np; ++I)
      for (int J = 0; J < Np; ++J) {
        double s = 0.0;
        for (int K = 0; K < Np; ++K) s += T->Ainv[static_cast<size_t>(I) * Np + K] * C[static_cast<size_t>(K) * Np + J];
        T->Gt[(static_cast<size_t>(a) * Np + J) * Np + I] = -s;
      }
  }
}

size_t tr_layout(ewdg_tr* T, char* base) {
  TrDev& t = T->t;
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* q = base ? base + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return q;
  };
  const size_t E = static_cast<size_t>(t.E), ts = T->tsz();
  t.u[0] = take(E * t.Np * ts);
  t.u[1] = take(E * t.Np * ts);
  t.c = take(E * t.Np * ts);
  t.uep = reinterpret_cast<double*>(take(E * t.Np * 8));
  t.Gt = take(static_cast<size_t>(t.d) * t.Np * t.Np * ts);
  t.Gfrag = take(static_cast<size_t>(t.d) * tr_row_tiles(t.Np) * tr_k_steps(t.Np) * 64 * ts);
  t.Ainv = reinterpret_cast<double*>(take(static_cast<size_t>(t.Np) * t.Np * 8));
  t.Vq = reinterpret_cast<double*>(take(static_cast<size_t>(t.Nq) * t.Np * 8));
  t.Wq = reinterpret_cast<double*>(take(static_cast<size_t>(t.Nq) * 8));
  t.Tf = reinterpret_cast<double*>(take(static_cast<size_t>(2 * t.d) * t.Nqf * t.Np * 8));
  t.Wf = reinterpret_cast<double*>(take(static_cast<size_t>(t.Nqf) * 8));
  t.fq = reinterpret_cast<double*>(take(E * t.Nq * 8));
  t.gq = reinterpret_cast<double*>(take(E * 2 * t.d * t.Nqf * 8));
  t.ueq = reinterpret_cast<double*>(take(E * t.Nq * 8));
  t.rest = reinterpret_cast<double*>(take(2 * E * 8));
  t.epart = reinterpret_cast<double*>(take(static_cast<size_t>(tr_sweep_blocks(t)) * 8));
  t.scal = reinterpret_cast<double*>(take(8 * 8));
  t.ctl = reinterpret_cast<TrCtl*>(take(sizeof(TrCtl)));
  return off;
}

int up(ewdg_tr* T, void* dst, const void* src, size_t bytes) {
  return T->hip(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, T->stream), "upload");
}

}  // namespace

extern "C" {

int ewdg_transport_create(int dim, int p, int n, const double* beta, int precision_bits, void* hip_stream,
                          ewdg_tr** out) {
  if (!out || !beta) return EWDG_EINVAL;
  *out = nullptr;
  if ((dim != 2 && dim != 3) || p < 1 || p > 4 || n < 1 || (precision_bits != 32 && precision_bits != 64))
    return EWDG_EINVAL;
  for (int a = 0; a < dim; ++a)
    if (!(beta[a] != 0.0) || !std::isfinite(beta[a])) return EWDG_EINVAL;
  const int64_t E = dim == 2 ? int64_t(n) * n : int64_t(n) * n * n;
  const int Np = ipow(p + 1, dim), Nq = ipow(p + 3, dim), Nqf = ipow(p + 3, dim - 1);
  if (E * Nq >= (int64_t(1) << 40) || E >= (int64_t(1) << 31)) return EWDG_EINVAL;
  ewdg_tr* T = new ewdg_tr;
  T->stream = static_cast<hipStream_t>(hip_stream);
  T->h = 1.0 / n;
  for (int a = 0; a < dim; ++a) T->beta[a] = beta[a];
  TrDev& t = T->t;
  t.d = dim;
  t.p = p;
  t.n = n;
  t.prec = precision_bits;
  t.Np = Np;
  t.Nq = Nq;
  t.Nqf = Nqf;
  t.E = E;
  t.J = std::pow(T->h / 2.0, dim);
  t.Jf = std::pow(T->h / 2.0, dim - 1);
  build_operators(T);
  *out = T;
  return EWDG_OK;
}

int ewdg_transport_destroy(ewdg_tr* T) {
  if (!T) return EWDG_EINVAL;
  delete T;
  return EWDG_OK;
}

int ewdg_transport_sizes(const ewdg_tr* T, int64_t* E, int* Np, int* Nq, int* Nqf) {
  if (!T) return EWDG_EINVAL;
  if (E) *E = T->t.E;
  if (Np) *Np = T->t.Np;
  if (Nq) *Nq = T->t.Nq;
  if (Nqf) *Nqf = T->t.Nqf;
  return EWDG_OK;
}

int ewdg_transport_points(const ewdg_tr* T, double* xv, double* xf) {
  if (!T) return EWDG_EINVAL;
  const TrDev& t = T->t;
  const int d = t.d, mq = t.p + 3;
  for (int64_t e = 0; e < t.E; ++e) {
    int64_t idx[3] = {0, 0, 0};
    int64_t r = e;
    for (int a = 0; a < d; ++a) {
      idx[a] = r % t.n;
      r /= t.n;
    }
    if (xv)
      for (int Q = 0; Q < t.Nq; ++Q)
        for (int a = 0; a < d; ++a)
          xv[(e * t.Nq + Q) * d + a] = (idx[a] + (T->xq1[digit(Q, a, mq)] + 1.0) / 2.0) * T->h;
    if (xf)
      for (int a = 0; a < d; ++a)
        for (int side = 0; side < 2; ++side)
          for (int F = 0; F < t.Nqf; ++F) {
            double* o = xf + ((e * 2 * d + 2 * a + side) * t.Nqf + F) * d;
            int k = 0;
            for (int b = 0; b < d; ++b) {
              if (b == a) {
                o[b] = (idx[b] + side) * T->h;
              } else {
                o[b] = (idx[b] + (T->xq1[digit(F, k, mq)] + 1.0) / 2.0) * T->h;
                ++k;
              }
            }
          }
  }
  return EWDG_OK;
}

int ewdg_transport_workspace_bytes(const ewdg_tr* T, size_t* bytes) {
  if (!T || !bytes) return EWDG_EINVAL;
  ewdg_tr tmp;
  tmp.t = T->t;
  *bytes = tr_layout(&tmp, nullptr);
  return EWDG_OK;
}

int ewdg_transport_bind_workspace(ewdg_tr* T, void* ptr, size_t bytes) {
  if (!T) return EWDG_EINVAL;
  if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255u))
    return T->fail(EWDG_EINVAL, "workspace must be a non-null 256-byte aligned device pointer");
  if (bytes < tr_layout(T, nullptr)) return T->fail(EWDG_ENOMEM, "workspace smaller than ewdg_transport_workspace_bytes");
  tr_layout(T, static_cast<char*>(ptr));
  const TrDev& t = T->t;
  int rc;
  // G_a in matrix-core fragment order: lane l of block (a, R, kk) holds
  // G_a[16 R + l % 16][4 kk + l / 16]
  const int Np = t.Np, RT = tr_row_tiles(Np), KS = tr_k_steps(Np);
  std::vector<double> frag(static_cast<size_t>(t.d) * RT * KS * 64, 0.0);
  for (int a = 0; a < t.d; ++a)
    for (int R = 0; R < RT; ++R)
      for (int kk = 0; kk < KS; ++kk)
        for (int l = 0; l < 64; ++l) {
          const int i = 16 * R + l % 16, j = 4 * kk + l / 16;
          if (i < Np && j < Np)
            frag[((static_cast<size_t>(a) * RT + R) * KS + kk) * 64 + l] =
                T->Gt[(static_cast<size_t>(a) * Np + j) * Np + i];
        }
  if (T->t.prec == 32) {
    std::vector<float> g(T->Gt.begin(), T->Gt.end()), gf(frag.begin(), frag.end());
    if ((rc = up(T, t.Gt, g.data(), g.size() * 4))) return rc;
    if ((rc = up(T, t.Gfrag, gf.data(), gf.size() * 4))) return rc;
    if ((rc = T->hip(hipStreamSynchronize(T->stream), "upload sync"))) return rc;
  } else {
    if ((rc = up(T, t.Gt, T->Gt.data(), T->Gt.size() * 8))) return rc;
    if ((rc = up(T, t.Gfrag, frag.data(), frag.size() * 8))) return rc;
    if ((rc = T->hip(hipStreamSynchronize(T->stream), "upload sync"))) return rc;
  }
  if ((rc = up(T, t.Ainv, T->Ainv.data(), T->Ainv.size() * 8))) return rc;
  if ((rc = up(T, t.Vq, T->Vq.data(), T->Vq.size() * 8))) return rc;
  if ((rc = up(T, t.Wq, T->Wq.data(), T->Wq.size() * 8))) return rc;
  if ((rc = up(T, t.Tf, T->Tf.data(), T->Tf.size() * 8))) return rc;
  if ((rc = up(T, t.Wf, T->Wf.data(), T->Wf.size() * 8))) return rc;
  if ((rc = T->hip(hipStreamSynchronize(T->stream), "upload sync"))) return rc;
  T->bound = true;
  T->has_problem = false;
  return EWDG_OK;
}

int ewdg_transport_set_problem(ewdg_tr* T, const double* f, const double* g, const double* ue) {
  if (!T) return EWDG_EINVAL;
  if (!T->bound) return T->fail(EWDG_ESTATE, "bind the transport workspace first");
  if (!f || !g) return T->fail(EWDG_EINVAL, "f and g are required");
  const TrDev& t = T->t;
  const size_t E = static_cast<size_t>(t.E);
  int rc;
  if ((rc = up(T, t.fq, f, E * t.Nq * 8))) return rc;
  if ((rc = up(T, t.gq, g, E * 2 * t.d * t.Nqf * 8))) return rc;
  if (ue && (rc = up(T, t.ueq, ue, E * t.Nq * 8))) return rc;
  if ((rc = T->hip(launch_tr_load(t, ue != nullptr, T->stream), "load"))) return rc;
  double s[2] = {0, 0};
  if (ue && (rc = T->hip(hipMemcpyAsync(s, t.scal + 6, 16, hipMemcpyDeviceToHost, T->stream), "copy"))) return rc;
  if ((rc = T->hip(hipStreamSynchronize(T->stream), "load sync"))) return rc;
  T->rest_total = s[0];
  T->exact_norm2 = s[1];
  T->has_exact = ue != nullptr;
  T->has_problem = true;
  return EWDG_OK;
}

int ewdg_transport_solve(ewdg_tr* T, double tol, int max_iters, int* iters, double* history) {
  if (!T) return EWDG_EINVAL;
  if (!T->has_problem) return T->fail(EWDG_ESTATE, "set the problem first");
  if (!(tol >= 0.0) || max_iters < 1) return EWDG_EINVAL;
  const TrDev& t = T->t;
  int rc;
  T->cur = 0;
  if ((rc = T->hip(launch_tr_zero(t, 0, T->stream), "zero"))) return rc;
  // iterations are queued in batches (1, 2, 4, ... up to half the norm ring)
  // and the stopping state is read once per batch; the device skips the
  // iterations queued after the stop
  TrCtl h;
  h.exact = T->has_exact ? 1 : 0;
  h.prev = T->has_exact ? std::sqrt(T->exact_norm2) : 0.0;   // ||u^0 - u^e|| with u^0 = 0
  h.rest = T->rest_total;
  h.tol = tol;
  if ((rc = T->hip(hipMemcpyAsync(t.ctl, &h, sizeof(TrCtl), hipMemcpyHostToDevice, T->stream), "control upload")))
    return rc;
  if (history) history[0] = h.prev;
  TrCtl r;
  int64_t k = 1, kend = max_iters;
  while (k <= max_iters) {
    const int64_t batch = std::min<int64_t>({k, kTrHist / 2, static_cast<int64_t>(max_iters) - k + 1});
    for (int64_t i = 0; i < batch; ++i)
      if ((rc = T->hip(launch_tr_iterate(t, static_cast<int>((k + i - 1) & 1), T->has_exact, k + i, T->stream),
                       "sweep")))
        return rc;
    if ((rc = T->hip(hipMemcpyAsync(&r, t.ctl, sizeof(TrCtl), hipMemcpyDeviceToHost, T->stream), "norm copy")))
      return rc;
    if ((rc = T->hip(hipStreamSynchronize(T->stream), "norm sync"))) return rc;
    const int64_t last = r.done ? r.done : k + batch - 1;
    if (history)
      for (int64_t j = k; j <= last; ++j) history[j] = r.hist[j % kTrHist];
    if (r.bad) {
      T->cur = static_cast<int>(last & 1);
      return T->fail(EWDG_EINVAL, "non-finite iterate");
    }
    if (r.done) {
      kend = r.done;
      break;
    }
    k += batch;
  }
  T->cur = static_cast<int>(kend & 1);
  if (iters) *iters = static_cast<int>(kend);
  return EWDG_OK;
}

int ewdg_transport_values(ewdg_tr* T, double* u) {
  if (!T || !u) return EWDG_EINVAL;
  if (!T->bound) return T->fail(EWDG_ESTATE, "no workspace");
  const TrDev& t = T->t;
  int rc;
  // the f staging area holds the values on their way out (the load c it
  // produced stays, so solving again needs no new problem)
  if ((rc = T->hip(launch_tr_values(t, T->cur, t.fq, T->stream), "values"))) return rc;
  if ((rc = T->hip(hipMemcpyAsync(u, t.fq, static_cast<size_t>(t.E) * t.Nq * 8, hipMemcpyDeviceToHost, T->stream),
                   "values copy")))
    return rc;
  return T->hip(hipStreamSynchronize(T->stream), "values sync");
}

const char* ewdg_transport_last_error(const ewdg_tr* T) { return T ? T->err.c_str() : "null handle"; }

}  // extern "C"
