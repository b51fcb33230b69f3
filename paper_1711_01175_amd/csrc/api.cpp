// C-ABI entry points: context lifecycle, workspace layout, uploads and the
// LSRK(5,4) driver.  Device work is enqueued on the context's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "adjdev.hpp"
#include "dev.hpp"
#include "impdev.hpp"
#include "ewdg.h"
#include "mesh.hpp"
#include "refelem.hpp"

using namespace ewdg;

namespace {

// Carpenter-Kennedy (5,4) 2N-storage coefficients (NASA TM-109112).
const double kRkA[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                        -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
const double kRkB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                        1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                        2277821191437.0 / 14882151754819.0};
const double kRkC[5] = {0.0, 1432997174477.0 / 9575080441755.0, 2526269341429.0 / 6820363962896.0,
                        2006345519317.0 / 3224310063776.0, 2802321613138.0 / 2924317926251.0};

double ricker(double t, double f0, double t0) {
  const double a = (M_PI * f0 * (t - t0)) * (M_PI * f0 * (t - t0));
  return (1.0 - 2.0 * a) * std::exp(-a);
}

}  // namespace

struct ewdg_ctx {
  int N = 0, prec = 0;
  hipStream_t stream = nullptr;
  RefElem re;
  MeshData mesh;
  bool has_mesh = false, bound = false, has_material = false;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int max_rec = 0, max_steps = 0;
  Dev d;
  int cur = 0;
  double t = 0.0;
  std::vector<double> cpmax;  // per element max_q c_p
  bool has_source = false;
  int64_t src_elem = -1;
  double src_dir[3] = {0, 0, 0}, src_amp = 0, src_f0 = 0, src_t0 = 0;
  int nr = 0, rec_count = 0;
  // adjoint: workspace binding and the last recorded forward run
  AdjDev ad;
  bool adj_bound = false;
  int adj_max_steps = 0, adj_every = 0, adj_rec = 0;
  // overlapped reverse sweep: a second segment buffer, refilled on a second
  // stream while the current segment is reversed on the context's stream
  bool adj_overlap = false;
  hipStream_t adj_stream = nullptr;
  hipEvent_t ev_start = nullptr, ev_rec[2] = {nullptr, nullptr}, ev_rev[2] = {nullptr, nullptr};
  bool fwd_done = false;
  int fwd_steps = 0;
  double fwd_dt = 0.0;
  std::vector<double> step_t;  // time at the start of every recorded step
  // locally implicit (iHDG-II) step: its own workspace, the colour classes
  // of the face-adjacency graph and the step the local inverses were made for
  ImpDev im;
  bool imp_bound = false, imp_ready = false;
  double imp_dt = 0.0, imp_theta = 0.0;
  std::vector<int> imp_cstart;  // members[imp_cstart[c] .. imp_cstart[c+1]) have colour c
  std::string err;

  ~ewdg_ctx() {
    if (adj_stream) {
      (void)hipStreamSynchronize(adj_stream);
      (void)hipStreamDestroy(adj_stream);
    }
    for (hipEvent_t e : {ev_start, ev_rec[0], ev_rec[1], ev_rev[0], ev_rev[1]})
      if (e) (void)hipEventDestroy(e);
  }
  size_t tsz() const { return prec == 32 ? 4 : 8; }
  int fail(int code, const std::string& m) {
    err = m;
    return code;
  }
  int hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return EWDG_OK;
    err = std::string(what) + ": " + hipGetErrorString(e);
    return EWDG_EHIP;
  }
};

namespace {

size_t pad_to(size_t x, size_t m) { return (x + m - 1) / m * m; }

// Copy a row-major [rows][cols] block into a zero [R][C] array at (r0, c0).
void place(std::vector<double>& dst, size_t C, const std::vector<double>& src, int rows, int cols,
           size_t r0, size_t c0) {
  for (int i = 0; i < rows; ++i)
    for (int j = 0; j < cols; ++j) dst[(r0 + i) * C + c0 + j] = src[static_cast<size_t>(i) * cols + j];
}

// Sequential 256-byte aligned layout of the workspace.  With base == nullptr
// only the total size is computed.
size_t layout(ewdg_ctx* c, char* base) {
  const int64_t K = c->mesh.K;
  const size_t Np = c->re.Np, Nfp = c->re.Nfp, Nq = c->re.Nq, ts = c->tsz();
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return p;
  };
  Dev& d = c->d;
  d.q[0] = take(9 * Np * K * ts);
  d.s[0] = take(6 * Np * K * ts);
  char* scratch = base ? base + off : nullptr;
  const size_t scratch_begin = off;
  d.q[1] = take(9 * Np * K * ts);
  d.s[1] = take(6 * Np * K * ts);
  d.res = take(9 * Np * K * ts);
  d.scratch = scratch;
  d.scratch_bytes = off - scratch_begin;
  d.W = take(Np * Np * K * ts);
  d.lm = take(2 * ((Nq + 3) / 4 * 4) * K * ts);
  d.geo = take(9 * K * ts);
  d.fgeo = take(16 * K * ts);
  d.Z = take(kZS * K * ts);
  d.svec = take(Np * ts);
  const size_t NpR = pad_to(Np, 16), NpK = pad_to(Np, 4), NqR = pad_to(Nq, 16), NqK = pad_to(Nq, 4),
               NfpK = pad_to(Nfp, 4);
  // fragment-ordered operators: (row tiles) x (k-steps) x 64 values
  d.Dpad = take(3 * (NpR / 16) * (NpK / 4) * 64 * ts);
  d.Lpad = take(4 * (NpR / 16) * (NfpK / 4) * 64 * ts);
  d.Vqpad = take((NqR / 16) * (NpK / 4) * 64 * ts);
  d.Pqpad = take((NpR / 16) * (NqK / 4) * 64 * ts);
  d.DTpad = take(3 * (NpR / 16) * (NpK / 4) * 64 * ts);
  d.PqTpad = take((NqR / 16) * (NpK / 4) * 64 * ts);
  d.VqTpad = take((NpR / 16) * (NqK / 4) * 64 * ts);
  d.VqT = take(Nq * Np * ts);
  d.PqT = take(Nq * Np * ts);
  d.Dk = take(3 * Np * Np * ts);
  d.LIFTr = take(4 * Nfp * Np * ts);
  d.Vqr = take(Nq * Np * ts);
  d.Pqr = take(Nq * Np * ts);
  d.Vq64T = reinterpret_cast<double*>(take(Nq * Np * 8));
  d.Pq64T = reinterpret_cast<double*>(take(Nq * Np * 8));
  d.Mhat64 = reinterpret_cast<double*>(take(Np * Np * 8));
  d.wq64 = reinterpret_cast<double*>(take(Nq * 8));
  d.rho64 = reinterpret_cast<double*>(take(Nq * K * 8));
  d.lam64 = reinterpret_cast<double*>(take(Nq * K * 8));
  d.mu64 = reinterpret_cast<double*>(take(Nq * K * 8));
  d.J64 = reinterpret_cast<double*>(take(K * 8));
  d.means64 = reinterpret_cast<double*>(take(3 * K * 8));
  d.epart = reinterpret_cast<double*>(take(K * 8));
  d.scal = reinterpret_cast<double*>(take(64 * 8));
  d.srcb = reinterpret_cast<double*>(take(Np * 8));
  d.msmall = reinterpret_cast<double*>(take(Np * Np * 8));
  const size_t mr = c->max_rec > 0 ? c->max_rec : 1, ms = c->max_steps > 0 ? c->max_steps : 1;
  d.rec_rows = reinterpret_cast<double*>(take(mr * Np * 8));
  d.rec_elem = reinterpret_cast<int32_t*>(take(mr * 4));
  d.rec_out = reinterpret_cast<double*>(take(ms * mr * 3 * 8));
  d.conn = reinterpret_cast<int32_t*>(take(4 * K * 4));
  d.nbrnode = reinterpret_cast<int32_t*>(take(96 * Nfp * 4));
  d.nbrface = reinterpret_cast<int32_t*>(take(96 * Nfp * 4));
  d.fmask = reinterpret_cast<int32_t*>(take(4 * Nfp * 4));
  d.bcm_buf = reinterpret_cast<int32_t*>(take(K * 4));
  d.rinv = take(((Nq + 3) / 4 * 4) * K * ts);
  d.svw = take(Np * ts);
  d.rhsw = take(3 * Np * K * ts);
  d.bcm = (base && c->mesh.bc != 0) ? d.bcm_buf : nullptr;
  return off;
}

template <typename T>
std::vector<T> convert(const std::vector<double>& v) {
  std::vector<T> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = static_cast<T>(v[i]);
  return o;
}

std::vector<double> transpose(const std::vector<double>& A, int rows, int cols) {
  std::vector<double> B(A.size());
  for (int i = 0; i < rows; ++i)
    for (int j = 0; j < cols; ++j) B[static_cast<size_t>(j) * rows + i] = A[static_cast<size_t>(i) * cols + j];
  return B;
}

int upload_run(ewdg_ctx* c, void* dst, const std::vector<double>& src) {
  if (int rc = c->hip(hipStreamSynchronize(c->stream), "upload sync")) return rc;
  if (c->prec == 32) {
    const std::vector<float> f = convert<float>(src);
    return c->hip(hipMemcpy(dst, f.data(), f.size() * 4, hipMemcpyHostToDevice), "upload");
  }
  return c->hip(hipMemcpy(dst, src.data(), src.size() * 8, hipMemcpyHostToDevice), "upload");
}

int upload(ewdg_ctx* c, void* dst, const void* src, size_t bytes) {
  // device work already queued on the context stream may still read dst
  if (int rc = c->hip(hipStreamSynchronize(c->stream), "upload sync")) return rc;
  return c->hip(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice), "upload");
}

// Nodal basis values l_i(rhat) = sum_m psi_m(rhat) Vinv[m][i].
std::vector<double> nodal_row(const RefElem& re, const double* rh) {
  std::vector<double> psi(re.Np);
  pkdo_eval(re.N, rh[0], rh[1], rh[2], psi.data(), nullptr, nullptr, nullptr);
  std::vector<double> row(re.Np, 0.0);
  for (int i = 0; i < re.Np; ++i)
    for (int m = 0; m < re.Np; ++m) row[i] += psi[m] * re.Vinv[m * re.Np + i];
  return row;
}

int need(const ewdg_ctx* c, bool mesh, bool bound, bool material) {
  if (!c) return EWDG_EINVAL;
  if (mesh && !c->has_mesh) return EWDG_ESTATE;
  if (bound && !c->bound) return EWDG_ESTATE;
  if (material && !c->has_material) return EWDG_ESTATE;
  return EWDG_OK;
}

}  // namespace

extern "C" {

int ewdg_create(int N, int precision_bits, void* hip_stream, ewdg_ctx** out) {
  if (!out) return EWDG_EINVAL;
  *out = nullptr;
  if (!supported_degree(N) || (precision_bits != 32 && precision_bits != 64)) return EWDG_EINVAL;
  ewdg_ctx* c = new (std::nothrow) ewdg_ctx();
  if (!c) return EWDG_ENOMEM;
  c->N = N;
  c->prec = precision_bits;
  c->stream = static_cast<hipStream_t>(hip_stream);
  char msg[256] = {0};
  if (!build_refelem(N, c->re, msg, sizeof(msg))) {
    delete c;
    return EWDG_EINVAL;
  }
  c->d.N = N;
  c->d.prec = precision_bits;
  c->d.Np = c->re.Np;
  c->d.Nfp = c->re.Nfp;
  c->d.Nq = c->re.Nq;
  *out = c;
  return EWDG_OK;
}

int ewdg_destroy(ewdg_ctx* c) {
  delete c;
  return EWDG_OK;
}

int ewdg_set_stream(ewdg_ctx* c, void* s) {
  if (!c) return EWDG_EINVAL;
  c->stream = static_cast<hipStream_t>(s);
  return EWDG_OK;
}

const char* ewdg_last_error(const ewdg_ctx* c) { return c ? c->err.c_str() : "null context"; }

int ewdg_set_mesh(ewdg_ctx* c, int64_t K, const int64_t* EToV, const double* VXYZ) {
  return ewdg_set_mesh_bc(c, K, EToV, VXYZ, EWDG_BC_PERIODIC);
}

int ewdg_set_mesh_bc(ewdg_ctx* c, int64_t K, const int64_t* EToV, const double* VXYZ, int bc) {
  if (!c || !EToV || !VXYZ) return EWDG_EINVAL;
  if (bc != EWDG_BC_PERIODIC && bc != EWDG_BC_FREE && bc != EWDG_BC_ABSORBING)
    return c->fail(EWDG_EINVAL, "unknown boundary condition");
  // the kernels index element data with 32-bit offsets and pack a
  // neighbour index with a node index into 32 bits (nbr * 256 + node)
  {
    const int64_t Np = c->re.Np, NqP = (c->re.Nq + 3) / 4 * 4;
    const int64_t lim = int64_t(1) << 31;
    if (K >= (int64_t(1) << 23) || K * 9 * Np >= lim || K * Np * Np >= lim || K * 2 * NqP >= lim ||
        K * 32 * c->re.Nfp >= lim)
      return c->fail(EWDG_EINVAL, "mesh too large for the kernels' 32-bit element offsets");
  }
  MeshData m;
  std::string e;
  const int rc = build_mesh(K, EToV, VXYZ, m, e, bc);
  if (rc != EWDG_OK) return c->fail(rc, e);
  c->mesh = std::move(m);
  c->has_mesh = true;
  c->bound = false;
  c->has_material = false;
  c->adj_bound = false;
  c->fwd_done = false;
  c->imp_bound = false;
  c->imp_ready = false;
  c->d.wadg = false;
  c->d.K = K;
  return EWDG_OK;
}

int ewdg_sizes(const ewdg_ctx* c, int* Np, int* Nfp, int* Nq) {
  if (!c) return EWDG_EINVAL;
  if (Np) *Np = c->re.Np;
  if (Nfp) *Nfp = c->re.Nfp;
  if (Nq) *Nq = c->re.Nq;
  return EWDG_OK;
}

static void map_points(const ewdg_ctx* c, const double* ref, int n, double* xyz) {
  const MeshData& m = c->mesh;
  for (int64_t k = 0; k < m.K; ++k)
    for (int p = 0; p < n; ++p)
      for (int d = 0; d < 3; ++d) {
        double x = m.X0[k * 3 + d];
        for (int cc = 0; cc < 3; ++cc) x += m.A[k * 9 + d * 3 + cc] * (ref[p * 3 + cc] + 1.0);
        xyz[(k * n + p) * 3 + d] = x;
      }
}

int ewdg_node_points(const ewdg_ctx* c, double* xyz) {
  if (int rc = need(c, true, false, false)) return rc;
  if (!xyz) return EWDG_EINVAL;
  std::vector<double> ref(c->re.Np * 3);
  for (int i = 0; i < c->re.Np; ++i) {
    ref[i * 3] = c->re.r[i];
    ref[i * 3 + 1] = c->re.s[i];
    ref[i * 3 + 2] = c->re.t[i];
  }
  map_points(c, ref.data(), c->re.Np, xyz);
  return EWDG_OK;
}

int ewdg_quadrature_points(const ewdg_ctx* c, double* xyz) {
  if (int rc = need(c, true, false, false)) return rc;
  if (!xyz) return EWDG_EINVAL;
  map_points(c, c->re.xq.data(), c->re.Nq, xyz);
  return EWDG_OK;
}

int ewdg_reference_operator(const ewdg_ctx* c, int which, double* out) {
  if (!c || !out) return EWDG_EINVAL;
  const RefElem& re = c->re;
  const std::vector<double>* src = nullptr;
  switch (which) {
    case 0: src = &re.Dr; break;
    case 1: src = &re.Ds; break;
    case 2: src = &re.Dt; break;
    case 3: src = &re.LIFT; break;
    case 4: src = &re.Vq; break;
    case 5: src = &re.Pq; break;
    case 6: src = &re.Mhat; break;
    case 7:
      for (int i = 0; i < re.Np; ++i) {
        out[i * 3] = re.r[i];
        out[i * 3 + 1] = re.s[i];
        out[i * 3 + 2] = re.t[i];
      }
      return EWDG_OK;
    case 8: src = &re.wq; break;
    case 9:
      for (size_t i = 0; i < re.Fmask.size(); ++i) out[i] = re.Fmask[i];
      return EWDG_OK;
    case 10:
      for (size_t i = 0; i < re.nbrnode.size(); ++i) out[i] = re.nbrnode[i];
      return EWDG_OK;
    default: return EWDG_EINVAL;
  }
  std::memcpy(out, src->data(), src->size() * sizeof(double));
  return EWDG_OK;
}

int ewdg_connectivity(const ewdg_ctx* c, int32_t* conn) {
  if (int rc = need(c, true, false, false)) return rc;
  if (!conn) return EWDG_EINVAL;
  std::memcpy(conn, c->mesh.conn.data(), c->mesh.conn.size() * 4);
  return EWDG_OK;
}

int ewdg_workspace_bytes(const ewdg_ctx* c, int max_receivers, int max_record_steps, size_t* bytes) {
  if (int rc = need(c, true, false, false)) return rc;
  if (!bytes || max_receivers < 0 || max_record_steps < 0) return EWDG_EINVAL;
  ewdg_ctx tmp;
  tmp.N = c->N;
  tmp.prec = c->prec;
  tmp.re.Np = c->re.Np;
  tmp.re.Nfp = c->re.Nfp;
  tmp.re.Nq = c->re.Nq;
  tmp.mesh.K = c->mesh.K;
  tmp.max_rec = max_receivers;
  tmp.max_steps = max_record_steps;
  *bytes = layout(&tmp, nullptr);
  return EWDG_OK;
}

int ewdg_bind_workspace(ewdg_ctx* c, void* ptr, size_t bytes, int max_receivers, int max_record_steps) {
  if (int rc = need(c, true, false, false)) return rc;
  if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255u))
    return c->fail(EWDG_EINVAL, "workspace must be a non-null 256-byte aligned device pointer");
  if (max_receivers < 0 || max_record_steps < 0) return c->fail(EWDG_EINVAL, "negative receiver capacity");
  c->max_rec = max_receivers;
  c->max_steps = max_record_steps;
  const size_t need_bytes = layout(c, nullptr);
  if (bytes < need_bytes) return c->fail(EWDG_ENOMEM, "workspace smaller than ewdg_workspace_bytes");
  c->ws = static_cast<char*>(ptr);
  c->ws_bytes = bytes;
  layout(c, c->ws);
  const RefElem& re = c->re;
  const MeshData& m = c->mesh;
  const int Np = re.Np, Nfp = re.Nfp, Nq = re.Nq;
  int rc;
  {
    // matrix-core fragment order: block (row tile R, k-step kk) holds 64
    // values, lane l taking A[16R + l%16][4kk + l/16] (zero outside A)
    auto frag = [](const std::vector<double>& A, int rows, int cols, int RT, int KS, std::vector<double>& out,
                   size_t base) {
      for (int R = 0; R < RT; ++R)
        for (int kk = 0; kk < KS; ++kk)
          for (int l = 0; l < 64; ++l) {
            const int i = 16 * R + l % 16, j = 4 * kk + l / 16;
            out[base + (static_cast<size_t>(R) * KS + kk) * 64 + l] =
                (i < rows && j < cols) ? A[static_cast<size_t>(i) * cols + j] : 0.0;
          }
    };
    const int RT = static_cast<int>(pad_to(Np, 16) / 16), QT = static_cast<int>(pad_to(Nq, 16) / 16);
    const int KD = static_cast<int>(pad_to(Np, 4) / 4), KF = static_cast<int>(pad_to(Nfp, 4) / 4),
              KQ = static_cast<int>(pad_to(Nq, 4) / 4);
    std::vector<double> Dp(3 * RT * KD * 64), Lp(4 * RT * KF * 64), Vp(QT * KD * 64), Pp(RT * KQ * 64);
    frag(re.Dr, Np, Np, RT, KD, Dp, 0);
    frag(re.Ds, Np, Np, RT, KD, Dp, static_cast<size_t>(RT) * KD * 64);
    frag(re.Dt, Np, Np, RT, KD, Dp, 2 * static_cast<size_t>(RT) * KD * 64);
    for (int f = 0; f < 4; ++f) {
      std::vector<double> Lf(static_cast<size_t>(Np) * Nfp);
      for (int i = 0; i < Np; ++i)
        for (int j = 0; j < Nfp; ++j) Lf[i * Nfp + j] = re.LIFT[i * 4 * Nfp + f * Nfp + j];
      frag(Lf, Np, Nfp, RT, KF, Lp, static_cast<size_t>(f) * RT * KF * 64);
    }
    frag(re.Vq, Nq, Np, QT, KD, Vp, 0);
    frag(re.Pq, Np, Nq, RT, KQ, Pp, 0);
    if ((rc = upload_run(c, c->d.Dpad, Dp))) return rc;
    if ((rc = upload_run(c, c->d.Lpad, Lp))) return rc;
    if ((rc = upload_run(c, c->d.Vqpad, Vp))) return rc;
    if ((rc = upload_run(c, c->d.Pqpad, Pp))) return rc;
    // transposed operators for the adjoint kernels
    std::vector<double> DTp(3 * RT * KD * 64), PTp(QT * KD * 64), VTp(RT * KQ * 64);
    frag(transpose(re.Dr, Np, Np), Np, Np, RT, KD, DTp, 0);
    frag(transpose(re.Ds, Np, Np), Np, Np, RT, KD, DTp, static_cast<size_t>(RT) * KD * 64);
    frag(transpose(re.Dt, Np, Np), Np, Np, RT, KD, DTp, 2 * static_cast<size_t>(RT) * KD * 64);
    frag(transpose(re.Pq, Np, Nq), Nq, Np, QT, KD, PTp, 0);
    frag(transpose(re.Vq, Nq, Np), Np, Nq, RT, KQ, VTp, 0);
    if ((rc = upload_run(c, c->d.DTpad, DTp))) return rc;
    if ((rc = upload_run(c, c->d.PqTpad, PTp))) return rc;
    if ((rc = upload_run(c, c->d.VqTpad, VTp))) return rc;
  }
  if ((rc = upload_run(c, c->d.VqT, transpose(re.Vq, Nq, Np)))) return rc;
  if ((rc = upload_run(c, c->d.PqT, transpose(re.Pq, Np, Nq)))) return rc;
  {
    std::vector<double> Dk(re.Dr);
    Dk.insert(Dk.end(), re.Ds.begin(), re.Ds.end());
    Dk.insert(Dk.end(), re.Dt.begin(), re.Dt.end());
    if ((rc = upload_run(c, c->d.Dk, Dk))) return rc;
  }
  if ((rc = upload_run(c, c->d.LIFTr, re.LIFT))) return rc;
  if ((rc = upload_run(c, c->d.Vqr, re.Vq))) return rc;
  if ((rc = upload_run(c, c->d.Pqr, re.Pq))) return rc;
  const std::vector<double> Vq64T = transpose(re.Vq, Nq, Np), Pq64T = transpose(re.Pq, Np, Nq);
  if ((rc = upload(c, c->d.Vq64T, Vq64T.data(), Vq64T.size() * 8))) return rc;
  if ((rc = upload(c, c->d.Pq64T, Pq64T.data(), Pq64T.size() * 8))) return rc;
  if ((rc = upload(c, c->d.Mhat64, re.Mhat.data(), re.Mhat.size() * 8))) return rc;
  if ((rc = upload(c, c->d.wq64, re.wq.data(), re.wq.size() * 8))) return rc;
  if ((rc = upload_run(c, c->d.geo, m.geo))) return rc;
  if ((rc = upload_run(c, c->d.fgeo, m.fgeo))) return rc;
  if ((rc = upload(c, c->d.J64, m.J.data(), m.J.size() * 8))) return rc;
  if ((rc = upload(c, c->d.conn, m.conn.data(), m.conn.size() * 4))) return rc;
  std::vector<int32_t> nbn(re.nbrnode.begin(), re.nbrnode.end()), fm(re.Fmask.begin(), re.Fmask.end());
  if ((rc = upload(c, c->d.nbrnode, nbn.data(), nbn.size() * 4))) return rc;
  {
    // face-local index on the neighbour's face g of the node matching own
    // face point j: the inverse of Fmask on face g applied to nbrnode
    std::vector<int32_t> nbf(nbn.size(), -1);
    for (int f = 0; f < 4; ++f)
      for (int g = 0; g < 4; ++g)
        for (int p = 0; p < 6; ++p)
          for (int j = 0; j < Nfp; ++j) {
            const size_t at = ((static_cast<size_t>(f) * 4 + g) * 6 + p) * Nfp + j;
            for (int jj = 0; jj < Nfp; ++jj)
              if (re.Fmask[g * Nfp + jj] == re.nbrnode[at]) nbf[at] = jj;
            if (nbf[at] < 0) return c->fail(EWDG_EINVAL, "face node table is inconsistent");
          }
    if ((rc = upload(c, c->d.nbrface, nbf.data(), nbf.size() * 4))) return rc;
  }
  if ((rc = upload(c, c->d.fmask, fm.data(), fm.size() * 4))) return rc;
  if (m.bc != 0 && (rc = upload(c, c->d.bcm_buf, m.bcm.data(), m.bcm.size() * 4))) return rc;
  c->bound = true;
  c->adj_bound = false;
  c->fwd_done = false;
  c->has_material = false;
  c->imp_ready = false;
  c->has_source = false;
  c->nr = 0;
  c->rec_count = 0;
  return EWDG_OK;
}

int ewdg_set_material(ewdg_ctx* c, const double* rho, const double* lam, const double* mu) {
  if (int rc = need(c, true, true, false)) return c ? c->fail(rc, "set_material needs a bound workspace") : rc;
  if (!rho || !lam || !mu) return EWDG_EINVAL;
  const int64_t K = c->mesh.K;
  const int Nq = c->re.Nq;
  c->cpmax.assign(K, 0.0);
  for (int64_t k = 0; k < K; ++k)
    for (int q = 0; q < Nq; ++q) {
      const double r = rho[k * Nq + q], l = lam[k * Nq + q], u = mu[k * Nq + q];
      if (!(r > 0.0) || !(u > 0.0) || !(l >= 0.0) || !std::isfinite(r + l + u))
        return c->fail(EWDG_EINVAL, "material must satisfy rho > 0, mu > 0, lambda >= 0");
      const double cp = std::sqrt((l + 2.0 * u) / r);
      if (cp > c->cpmax[k]) c->cpmax[k] = cp;
    }
  int rc;
  const size_t bytes = static_cast<size_t>(K) * Nq * 8;
  if ((rc = upload(c, c->d.rho64, rho, bytes))) return rc;
  if ((rc = upload(c, c->d.lam64, lam, bytes))) return rc;
  if ((rc = upload(c, c->d.mu64, mu, bytes))) return rc;
  if ((rc = c->hip(launch_material(c->d, c->stream), "material setup"))) return rc;
  if (c->d.wadg && (rc = c->hip(launch_rinv(c->d, c->stream), "1/rho"))) return rc;
  // zero state at t = 0
  const size_t sb = static_cast<size_t>(K) * c->re.Np * c->tsz();
  if ((rc = c->hip(hipMemsetAsync(c->d.q[0], 0, 9 * sb, c->stream), "memset"))) return rc;
  if ((rc = c->hip(hipMemsetAsync(c->d.s[0], 0, 6 * sb, c->stream), "memset"))) return rc;
  if ((rc = c->hip(hipMemsetAsync(c->d.res, 0, 9 * sb, c->stream), "memset"))) return rc;
  c->cur = 0;
  c->t = 0.0;
  c->has_material = true;
  c->fwd_done = false;
  c->imp_ready = false;
  if (c->has_source) {
    if ((rc = c->hip(launch_source_vector(c->d, c->src_elem, c->stream), "source vector"))) return rc;
  }
  return c->hip(hipStreamSynchronize(c->stream), "material sync");
}

int ewdg_set_mass_inverse(ewdg_ctx* c, int mode) {
  if (int rc = need(c, true, true, false)) return c ? c->fail(rc, "set_mass_inverse needs a bound workspace") : rc;
  if (mode != EWDG_MASS_EXACT && mode != EWDG_MASS_WEIGHT_ADJUSTED) return c->fail(EWDG_EINVAL, "unknown mass inverse");
  if (mode == EWDG_MASS_WEIGHT_ADJUSTED && c->mesh.bc != 0)
    return c->fail(EWDG_EINVAL, "the weight-adjusted mass inverse needs a periodic mesh");
  if (c->adj_bound && mode != EWDG_MASS_EXACT)
    return c->fail(EWDG_ESTATE, "an adjoint workspace is bound (the adjoint needs the exact mass inverse)");
  c->d.wadg = mode == EWDG_MASS_WEIGHT_ADJUSTED;
  c->imp_ready = false;   // the local matrices depend on it
  c->fwd_done = false;
  int rc;
  if (c->d.wadg && c->has_material) {
    if ((rc = c->hip(launch_rinv(c->d, c->stream), "1/rho"))) return rc;
    return c->hip(hipStreamSynchronize(c->stream), "1/rho sync");
  }
  return EWDG_OK;
}

int ewdg_set_state(ewdg_ctx* c, const void* q, int on_device, double t) {
  if (int rc = need(c, true, true, true)) return c ? c->fail(rc, "set_state needs material") : rc;
  if (!q) return EWDG_EINVAL;
  const size_t bytes = static_cast<size_t>(c->mesh.K) * 9 * c->re.Np * c->tsz();
  int rc;
  c->cur = 0;
  if ((rc = c->hip(hipMemcpyAsync(c->d.q[0], q, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                  c->stream), "set_state copy")))
    return rc;
  if ((rc = c->hip(hipMemsetAsync(c->d.res, 0, bytes, c->stream), "memset"))) return rc;
  if ((rc = c->hip(launch_sigma(c->d, c->d.q[0], c->d.s[0], c->stream), "sigma"))) return rc;
  c->t = t;
  if (!on_device) return c->hip(hipStreamSynchronize(c->stream), "set_state sync");
  return EWDG_OK;
}

int ewdg_get_state(ewdg_ctx* c, void* q, int on_device, double* t) {
  if (int rc = need(c, true, true, true)) return rc;
  if (!q) return EWDG_EINVAL;
  const size_t bytes = static_cast<size_t>(c->mesh.K) * 9 * c->re.Np * c->tsz();
  int rc;
  if ((rc = c->hip(hipMemcpyAsync(q, c->d.q[c->cur], bytes,
                                  on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream),
                   "get_state copy")))
    return rc;
  if (t) *t = c->t;
  if (!on_device) return c->hip(hipStreamSynchronize(c->stream), "get_state sync");
  return EWDG_OK;
}

int ewdg_project_quadrature(ewdg_ctx* c, const double* fq, void* q) {
  if (int rc = need(c, true, true, false)) return rc;
  if (!fq || !q) return EWDG_EINVAL;
  return c->hip(launch_project(c->d, fq, q, c->stream), "project");
}

int ewdg_eval_quadrature(ewdg_ctx* c, const void* q, double* fq) {
  if (int rc = need(c, true, true, false)) return rc;
  if (!fq) return EWDG_EINVAL;
  if (!q) {
    if (!c->has_material) return EWDG_ESTATE;
    q = c->d.q[c->cur];
  }
  return c->hip(launch_evalq(c->d, q, fq, c->stream), "evalq");
}

int ewdg_set_source(ewdg_ctx* c, const double xs[3], const double dir[3], double amp, double f0, double t0) {
  if (int rc = need(c, true, true, false)) return rc;
  if (!xs || !dir) return EWDG_EINVAL;
  double rh[3];
  const int64_t e = locate_point(c->mesh, xs, rh);
  if (e < 0) return c->fail(EWDG_EPOINT, "source outside the mesh");
  const std::vector<double> row = nodal_row(c->re, rh);
  int rc;
  if ((rc = upload(c, c->d.srcb, row.data(), row.size() * 8))) return rc;
  {
    // M^-1 phi(x_s) (M = J Mhat) for the weight-adjusted mass inverse
    const int Np = c->re.Np;
    std::vector<double> Mi(c->re.Mhat);
    if (!invert(Np, Mi)) return c->fail(EWDG_EINVAL, "reference mass matrix is singular");
    std::vector<double> sw(Np, 0.0);
    for (int i = 0; i < Np; ++i)
      for (int j = 0; j < Np; ++j) sw[i] += Mi[static_cast<size_t>(i) * Np + j] * row[j] / c->mesh.J[e];
    if ((rc = upload_run(c, c->d.svw, sw))) return rc;
  }
  c->has_source = true;
  c->fwd_done = false;
  c->src_elem = e;
  for (int i = 0; i < 3; ++i) c->src_dir[i] = dir[i];
  c->src_amp = amp;
  c->src_f0 = f0;
  c->src_t0 = t0;
  if (c->has_material) {
    if ((rc = c->hip(launch_source_vector(c->d, e, c->stream), "source vector"))) return rc;
    return c->hip(hipStreamSynchronize(c->stream), "source sync");
  }
  return EWDG_OK;
}

int ewdg_clear_source(ewdg_ctx* c) {
  if (!c) return EWDG_EINVAL;
  c->has_source = false;
  c->fwd_done = false;
  c->src_elem = -1;
  return EWDG_OK;
}

int ewdg_set_receivers(ewdg_ctx* c, int nr, const double* xr) {
  if (int rc = need(c, true, true, false)) return rc;
  if (nr < 0 || (nr > 0 && !xr)) return EWDG_EINVAL;
  if (nr > c->max_rec) return c->fail(EWDG_ENOMEM, "more receivers than the workspace capacity");
  std::vector<double> rows(static_cast<size_t>(nr) * c->re.Np);
  std::vector<int32_t> el(nr);
  for (int r = 0; r < nr; ++r) {
    double rh[3];
    const int64_t e = locate_point(c->mesh, xr + 3 * r, rh);
    if (e < 0) return c->fail(EWDG_EPOINT, "receiver outside the mesh");
    el[r] = static_cast<int32_t>(e);
    const std::vector<double> row = nodal_row(c->re, rh);
    std::memcpy(&rows[static_cast<size_t>(r) * c->re.Np], row.data(), row.size() * 8);
  }
  int rc;
  if (nr > 0) {
    if ((rc = upload(c, c->d.rec_rows, rows.data(), rows.size() * 8))) return rc;
    if ((rc = upload(c, c->d.rec_elem, el.data(), el.size() * 4))) return rc;
  }
  c->nr = nr;
  c->rec_count = 0;
  c->fwd_done = false;
  return EWDG_OK;
}

int ewdg_receivers(ewdg_ctx* c, double* out, int* nsteps) {
  if (int rc = need(c, true, true, false)) return rc;
  if (nsteps) *nsteps = c->rec_count;
  if (!out || c->rec_count == 0 || c->nr == 0) return EWDG_OK;
  const size_t bytes = static_cast<size_t>(c->rec_count) * c->nr * 3 * 8;
  int rc;
  if ((rc = c->hip(hipMemcpyAsync(out, c->d.rec_out, bytes, hipMemcpyDeviceToHost, c->stream), "receivers copy")))
    return rc;
  return c->hip(hipStreamSynchronize(c->stream), "receivers sync");
}

int ewdg_cfl_dt(const ewdg_ctx* c, double cfl, double* dt) {
  if (!c || !dt || !(cfl > 0.0)) return EWDG_EINVAL;
  if (!c->has_mesh || c->cpmax.size() != static_cast<size_t>(c->mesh.K)) return EWDG_ESTATE;
  double mn = 1e300;
  for (int64_t k = 0; k < c->mesh.K; ++k) mn = std::fmin(mn, c->mesh.inradius[k] / c->cpmax[k]);
  *dt = cfl * mn / ((c->N + 1.0) * (c->N + 1.0));
  return EWDG_OK;
}

static StageCoef coef(const ewdg_ctx* c, double a, double b, double dt, double ts) {
  StageCoef sc;
  sc.a = a;
  sc.b = b;
  sc.dt = dt;
  if (c->has_source) {
    sc.src_elem = c->src_elem;
    sc.srcval = c->src_amp * ricker(ts, c->src_f0, c->src_t0);
    for (int i = 0; i < 3; ++i) sc.dir[i] = c->src_dir[i];
  }
  return sc;
}

int ewdg_rhs(ewdg_ctx* c, double t, const void* q, void* rhs) {
  if (int rc = need(c, true, true, true)) return c ? c->fail(rc, "rhs needs material") : rc;
  if (!q || !rhs) return EWDG_EINVAL;
  void* stmp = c->d.s[1 - c->cur];
  int rc;
  if ((rc = c->hip(launch_sigma(c->d, q, stmp, c->stream), "sigma"))) return rc;
  const StageCoef sc = coef(c, 0.0, 0.0, 0.0, t);
  return c->hip(launch_stage(c->d, 0, q, stmp, nullptr, nullptr, rhs, sc, c->stream), "rhs");
}

int ewdg_step(ewdg_ctx* c, double dt, int nsteps) {
  if (int rc = need(c, true, true, true)) return c ? c->fail(rc, "step needs material") : rc;
  if (nsteps < 0 || !(dt > 0.0)) return EWDG_EINVAL;
  if (c->nr > 0 && c->rec_count + nsteps > c->max_steps)
    return c->fail(EWDG_ENOMEM, "receiver record capacity exceeded");
  int rc;
  for (int n = 0; n < nsteps; ++n) {
    for (int i = 0; i < 5; ++i) {
      const int nx = 1 - c->cur;
      const StageCoef sc = coef(c, kRkA[i], kRkB[i], dt, c->t + kRkC[i] * dt);
      if ((rc = c->hip(launch_stage(c->d, 1, c->d.q[c->cur], c->d.s[c->cur], c->d.q[nx], c->d.s[nx], c->d.res,
                                    sc, c->stream),
                       "stage")))
        return rc;
      c->cur = nx;
    }
    c->t = c->t + dt;
    if (c->nr > 0) {
      if ((rc = c->hip(launch_receivers(c->d, c->d.q[c->cur], c->nr, c->rec_count, c->stream), "receivers")))
        return rc;
      ++c->rec_count;
    }
  }
  return EWDG_OK;
}

int ewdg_time(const ewdg_ctx* c, double* t) {
  if (!c || !t) return EWDG_EINVAL;
  *t = c->t;
  return EWDG_OK;
}

int ewdg_energy_device(ewdg_ctx* c, double* E_dev) {
  if (int rc = need(c, true, true, true)) return rc;
  if (!E_dev) return EWDG_EINVAL;
  return c->hip(launch_energy(c->d, c->d.q[c->cur], E_dev, c->stream), "energy");
}

int ewdg_energy(ewdg_ctx* c, double* E) {
  if (int rc = need(c, true, true, true)) return rc;
  if (!E) return EWDG_EINVAL;
  int rc;
  if ((rc = c->hip(launch_energy(c->d, c->d.q[c->cur], c->d.scal, c->stream), "energy"))) return rc;
  if ((rc = c->hip(hipMemcpyAsync(E, c->d.scal, 8, hipMemcpyDeviceToHost, c->stream), "energy copy"))) return rc;
  return c->hip(hipStreamSynchronize(c->stream), "energy sync");
}

}  // extern "C"

namespace {

// One stream per (degree, precision) group of ewdg_step_batch, created on
// first use (default priority) and kept for the life of the process (the
// runtime releases them at exit), with a completion event each.
struct GroupStream {
  hipStream_t s = nullptr;
  hipEvent_t done = nullptr;
};
// Two pinned host staging buffers for the whole-chunk tables, used in turn;
// a buffer is refilled only after its previous upload has executed, so the
// upload never blocks the host and the caller can queue the next chunk
// while the device still runs the previous one.
struct Staging {
  char* p = nullptr;
  size_t cap = 0;
  hipEvent_t copied = nullptr;
  bool pending = false;
};
struct BatchStreams {
  hipEvent_t fork = nullptr;
  std::map<std::pair<int, int>, GroupStream> g;
  Staging stage[2];
  int next = 0;
  GroupStream* get(int N, int prec) {
    GroupStream& x = g[{N, prec}];
    if (!x.s && hipStreamCreateWithFlags(&x.s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    if (!x.done && hipEventCreateWithFlags(&x.done, hipEventDisableTiming) != hipSuccess) return nullptr;
    return &x;
  }
  // a free staging buffer of at least bytes (waits for its last upload)
  Staging* staging(size_t bytes) {
    Staging& b = stage[next];
    next ^= 1;
    if (b.pending && hipEventSynchronize(b.copied) != hipSuccess) return nullptr;
    b.pending = false;
    if (!b.copied && hipEventCreateWithFlags(&b.copied, hipEventDisableTiming) != hipSuccess) return nullptr;
    if (b.cap < bytes) {
      if (b.p) (void)hipHostFree(b.p);
      b.p = nullptr;
      b.cap = 0;
      if (hipHostMalloc(reinterpret_cast<void**>(&b.p), bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
      b.cap = bytes;
    }
    return &b;
  }
};
BatchStreams& batch_streams() {
  static BatchStreams* b = [] {
    auto* p = new BatchStreams;
    (void)hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
    return p;
  }();
  return *b;
}

}  // namespace

extern "C" {

// Per step the table holds, for each of the 5 stages, n argument records
// followed by the groups' tile prefix arrays.
static size_t batch_record_bytes() {
  const size_t s = std::max(stage_args_bytes(32), stage_args_bytes(64));
  return (s + 15) / 16 * 16;
}

int ewdg_batch_table_bytes(int n, size_t* bytes) {
  if (n < 0 || !bytes) return EWDG_EINVAL;
  *bytes = 5 * (static_cast<size_t>(n) * batch_record_bytes() + 2 * static_cast<size_t>(n) * 4 + 256) + 256;
  return EWDG_OK;
}

int ewdg_step_batch(ewdg_ctx* const* ctxs, int n, const double* dts, int nsteps, void* table_dev,
                    size_t table_bytes, void* hip_stream) {
  if (n < 0 || nsteps < 0 || (n > 0 && (!ctxs || !dts || !table_dev))) return EWDG_EINVAL;
  if (n == 0 || nsteps == 0) return EWDG_OK;
  size_t need_b = 0;
  ewdg_batch_table_bytes(n, &need_b);
  if (table_bytes < need_b) return EWDG_ENOMEM;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  for (int i = 0; i < n; ++i)
    if (ctxs[i] && (ctxs[i]->mesh.bc != 0 || ctxs[i]->d.wadg))
      return ctxs[i]->fail(EWDG_EINVAL, "batched stepping needs periodic meshes and the exact mass inverse");
  for (int i = 0; i < n; ++i) {
    ewdg_ctx* c = ctxs[i];
    if (!c) return EWDG_EINVAL;
    if (int rc = need(c, true, true, true)) return c->fail(rc, "step_batch needs material");
    if (!(dts[i] > 0.0)) return c->fail(EWDG_EINVAL, "non-positive dt");
    if (c->nr > 0 && c->rec_count + nsteps > c->max_steps)
      return c->fail(EWDG_ENOMEM, "receiver record capacity exceeded");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == c) return c->fail(EWDG_EINVAL, "context repeated in a batch");
  }
  // groups of (degree, precision), in a fixed order
  std::map<std::pair<int, int>, std::vector<int>> groups;
  for (int i = 0; i < n; ++i) groups[{ctxs[i]->N, ctxs[i]->prec}].push_back(i);
  const size_t rec = batch_record_bytes();
  const int E = stage_tile_elems();
  // With room for every step's table (nsteps * stride bytes) all tables go
  // up in one copy and each group runs its steps on a stream of its own
  // (groups share no data, so their launches overlap on the device);
  // otherwise one table per step on hip_stream.
  const size_t stride = (need_b + 255) / 256 * 256;
  const bool whole = table_bytes / stride >= static_cast<size_t>(nsteps);
  struct Launch { int N, prec, nreq, ntiles, group; size_t args_off, tiles_off; };
  std::vector<char> host((whole ? static_cast<size_t>(nsteps) : 1) * stride, 0);
  char* dev = static_cast<char*>(table_dev);
  std::vector<int> cur(n);
  std::vector<double> tt(n);
  for (int i = 0; i < n; ++i) {
    cur[i] = ctxs[i]->cur;
    tt[i] = ctxs[i]->t;
  }
  // tables of the five stages of one step at host offset base; the
  // contexts' step state is taken from cur / tt
  auto build = [&](size_t base, std::vector<Launch>& launches) {
    size_t off = base;
    for (int i = 0; i < 5; ++i) {
      size_t rec_off = off, tiles_off = off + static_cast<size_t>(n) * rec;
      int gi = 0;
      for (auto& g : groups) {
        Launch L{g.first.first, g.first.second, static_cast<int>(g.second.size()), 0, gi++, rec_off, tiles_off};
        int32_t* ts = reinterpret_cast<int32_t*>(&host[tiles_off]);
        int tiles = 0;
        for (size_t m = 0; m < g.second.size(); ++m) {
          const int k = g.second[m];
          ewdg_ctx* c = ctxs[k];
          const double dt = dts[k];
          const int cs = (cur[k] + i) & 1;
          const StageCoef sc = coef(c, kRkA[i], kRkB[i], dt, tt[k] + kRkC[i] * dt);
          stage_args_fill(c->d, c->d.q[cs], c->d.s[cs], c->d.q[1 - cs], c->d.s[1 - cs], c->d.res, sc,
                          &host[rec_off]);
          rec_off += rec;
          ts[m] = tiles;
          tiles += static_cast<int>((c->mesh.K + E - 1) / E);
        }
        ts[g.second.size()] = tiles;
        L.ntiles = tiles;
        launches.push_back(L);
        tiles_off += (g.second.size() + 1) * 4;
      }
      off = base + (tiles_off - base + 255) / 256 * 256;
    }
  };
  auto advance = [&]() {
    for (int i = 0; i < n; ++i) {
      cur[i] = (cur[i] + 5) & 1;
      tt[i] = tt[i] + dts[i];
    }
  };
  auto commit = [&](int steps_done) {
    for (int i = 0; i < n; ++i) {
      ctxs[i]->cur = cur[i];
      ctxs[i]->t = tt[i];
      if (ctxs[i]->nr > 0) ctxs[i]->rec_count += steps_done;
    }
  };
  if (!whole) {
    for (int step = 0; step < nsteps; ++step) {
      std::vector<Launch> launches;
      build(0, launches);
      hipError_t e = hipMemcpyAsync(dev, host.data(), stride, hipMemcpyHostToDevice, st);
      if (e != hipSuccess) return ctxs[0]->hip(e, "batch table copy");
      for (const Launch& L : launches) {
        e = launch_stage_batch(L.N, L.prec, dev + L.args_off, static_cast<int>(rec),
                               reinterpret_cast<const int*>(dev + L.tiles_off), L.nreq, L.ntiles, st);
        if (e != hipSuccess) return ctxs[0]->hip(e, "batched stage");
      }
      advance();
      for (int i = 0; i < n; ++i) {
        ewdg_ctx* c = ctxs[i];
        if (c->nr > 0) {
          e = launch_receivers(c->d, c->d.q[cur[i]], c->nr, c->rec_count, st);
          if (e != hipSuccess) return c->hip(e, "receivers");
        }
      }
      commit(1);
    }
    return EWDG_OK;
  }
  std::vector<std::vector<Launch>> launches(nsteps);
  std::vector<std::vector<int>> cur_after(nsteps);
  for (int step = 0; step < nsteps; ++step) {
    build(static_cast<size_t>(step) * stride, launches[step]);
    advance();
    cur_after[step] = cur;
  }
  BatchStreams& bs = batch_streams();
  if (!bs.fork) return ctxs[0]->fail(EWDG_EHIP, "could not create the batch fork event");
  Staging* sb = bs.staging(host.size());
  if (!sb) return ctxs[0]->fail(EWDG_EHIP, "could not get a pinned staging buffer for the batch tables");
  std::memcpy(sb->p, host.data(), host.size());
  hipError_t e = hipMemcpyAsync(dev, sb->p, host.size(), hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return ctxs[0]->hip(e, "batch table copy");
  if ((e = hipEventRecord(sb->copied, st)) != hipSuccess) return ctxs[0]->hip(e, "event");
  sb->pending = true;
  if ((e = hipEventRecord(bs.fork, st)) != hipSuccess) return ctxs[0]->hip(e, "event");
  int gi = 0;
  for (auto& g : groups) {
    GroupStream* gs = bs.get(g.first.first, g.first.second);
    if (!gs) return ctxs[0]->fail(EWDG_EHIP, "could not create a batch stream");
    if ((e = hipStreamWaitEvent(gs->s, bs.fork, 0)) != hipSuccess) return ctxs[0]->hip(e, "event wait");
    for (int step = 0; step < nsteps; ++step) {
      for (const Launch& L : launches[step]) {
        if (L.group != gi) continue;
        e = launch_stage_batch(L.N, L.prec, dev + L.args_off, static_cast<int>(rec),
                               reinterpret_cast<const int*>(dev + L.tiles_off), L.nreq, L.ntiles, gs->s);
        if (e != hipSuccess) return ctxs[0]->hip(e, "batched stage");
      }
      for (int k : g.second) {
        ewdg_ctx* c = ctxs[k];
        if (c->nr > 0) {
          e = launch_receivers(c->d, c->d.q[cur_after[step][k]], c->nr, c->rec_count + step, gs->s);
          if (e != hipSuccess) return c->hip(e, "receivers");
        }
      }
    }
    if ((e = hipEventRecord(gs->done, gs->s)) != hipSuccess) return ctxs[0]->hip(e, "event");
    if ((e = hipStreamWaitEvent(st, gs->done, 0)) != hipSuccess) return ctxs[0]->hip(e, "event wait");
    ++gi;
  }
  commit(nsteps);
  return EWDG_OK;
}

}  // extern "C"

// ------------------------------------------- batched stepping, no allocation
// Launch tables of ewdg_step_batch_static live in this file-scope device
// array (one copy per GPU, held until the process ends) and are filled from a
// file-scope host array; nothing is allocated.  Host code never uses the
// array's name as an address: its device address is taken once per device
// with hipGetSymbolAddress and kept in scratch_dev.
namespace {

constexpr size_t kStaticTableBytes = 256 * 1024;
constexpr int kMaxDevices = 64;
__device__ __align__(256) char scratch[kStaticTableBytes];
alignas(256) char scratch_host[kStaticTableBytes];
void* scratch_dev[kMaxDevices] = {};

// Device address of this GPU's copy of the table array (looked up on first
// use, with the device current); nullptr on failure.
void* static_table(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    scratch_dev[dev] = p;
  }
  return scratch_dev[dev];
}

}  // namespace

extern "C" {

int ewdg_static_table_max_bytes(size_t* bytes) {
  if (!bytes) return EWDG_EINVAL;
  *bytes = kStaticTableBytes;
  return EWDG_OK;
}

int ewdg_step_batch_static(ewdg_ctx* const* ctxs, int n, const double* dts, int nsteps, void* hip_stream) {
  if (n < 0 || nsteps < 0 || (n > 0 && (!ctxs || !dts))) return EWDG_EINVAL;
  if (n == 0 || nsteps == 0) return EWDG_OK;
  if (!ctxs[0]) return EWDG_EINVAL;
  size_t need_b = 0;
  ewdg_batch_table_bytes(n, &need_b);
  if (need_b > kStaticTableBytes)
    return ctxs[0]->fail(EWDG_ENOMEM, "batch too large for the static launch table (ewdg_static_table_max_bytes)");
  for (int i = 0; i < n; ++i)
    if (ctxs[i] && (ctxs[i]->mesh.bc != 0 || ctxs[i]->d.wadg))
      return ctxs[i]->fail(EWDG_EINVAL, "batched stepping needs periodic meshes and the exact mass inverse");
  for (int i = 0; i < n; ++i) {
    ewdg_ctx* c = ctxs[i];
    if (!c) return EWDG_EINVAL;
    if (int rc = need(c, true, true, true)) return c->fail(rc, "step_batch_static needs material");
    if (!(dts[i] > 0.0)) return c->fail(EWDG_EINVAL, "non-positive dt");
    if (c->nr > 0 && c->rec_count + nsteps > c->max_steps)
      return c->fail(EWDG_ENOMEM, "receiver record capacity exceeded");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == c) return c->fail(EWDG_EINVAL, "context repeated in a batch");
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return ctxs[0]->fail(EWDG_EHIP, "hipGetDevice failed");
  char* table = static_cast<char*>(static_table(dev));
  if (!table) return ctxs[0]->fail(EWDG_EHIP, "could not find the static launch table on this device");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const size_t rec = batch_record_bytes();
  const int E = stage_tile_elems();
  // (degree, precision) groups in ascending order, as in ewdg_step_batch;
  // fixed-size bookkeeping only (no host or device allocation)
  static const int kDegrees[6] = {1, 2, 3, 4, 5, 7};
  struct Launch { int N, prec, nreq, ntiles; size_t args_off, tiles_off; };
  Launch launches[5 * 12];
  for (int step = 0; step < nsteps; ++step) {
    // the five stages' records and tile prefixes of this step, laid out as
    // in ewdg_step_batch, in the host array
    int nl = 0;
    size_t off = 0;
    for (int i = 0; i < 5; ++i) {
      size_t rec_off = off, tiles_off = off + static_cast<size_t>(n) * rec;
      for (int gN : kDegrees) {
        for (int gp : {32, 64}) {
          int32_t* ts = reinterpret_cast<int32_t*>(scratch_host + tiles_off);
          int tiles = 0, m = 0;
          for (int k = 0; k < n; ++k) {
            ewdg_ctx* c = ctxs[k];
            if (c->N != gN || c->prec != gp) continue;
            const double dt = dts[k];
            const int cs = (c->cur + i) & 1;
            const StageCoef sc = coef(c, kRkA[i], kRkB[i], dt, c->t + kRkC[i] * dt);
            stage_args_fill(c->d, c->d.q[cs], c->d.s[cs], c->d.q[1 - cs], c->d.s[1 - cs], c->d.res, sc,
                            scratch_host + rec_off + static_cast<size_t>(m) * rec);
            ts[m++] = tiles;
            tiles += static_cast<int>((c->mesh.K + E - 1) / E);
          }
          if (m == 0) continue;
          ts[m] = tiles;
          launches[nl++] = Launch{gN, gp, m, tiles, rec_off, tiles_off};
          rec_off += static_cast<size_t>(m) * rec;
          tiles_off += static_cast<size_t>(m + 1) * 4;
        }
      }
      off = (tiles_off + 255) / 256 * 256;
    }
    // pageable source: the copy has read the host array when it returns;
    // stream order puts it after the previous step's launches
    hipError_t e = hipMemcpyAsync(table, scratch_host, off, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return ctxs[0]->hip(e, "static batch table copy");
    for (int k = 0; k < nl; ++k) {
      const Launch& L = launches[k];
      e = launch_stage_batch(L.N, L.prec, table + L.args_off, static_cast<int>(rec),
                             reinterpret_cast<const int*>(table + L.tiles_off), L.nreq, L.ntiles, st);
      if (e != hipSuccess) return ctxs[0]->hip(e, "batched stage");
    }
    for (int i = 0; i < n; ++i) {
      ewdg_ctx* c = ctxs[i];
      c->cur = (c->cur + 5) & 1;
      c->t = c->t + dts[i];
      if (c->nr > 0) {
        e = launch_receivers(c->d, c->d.q[c->cur], c->nr, c->rec_count, st);
        if (e != hipSuccess) return c->hip(e, "receivers");
        ++c->rec_count;
      }
    }
  }
  return EWDG_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ adjoint
namespace {

// Layout of the adjoint workspace; with base == nullptr only the size.
size_t adj_layout(const ewdg_ctx* c, int max_steps, int every, int max_rec, char* base, AdjDev* ad,
                  bool overlap) {
  const size_t K = static_cast<size_t>(c->mesh.K), Np = c->re.Np, Nfp = c->re.Nfp, ts = c->tsz();
  const size_t nck = (static_cast<size_t>(max_steps) + every - 1) / every;
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return p;
  };
  AdjDev a;
  a.ytil = take(3 * Np * K * ts);
  a.fown = take(32 * Nfp * K * ts);
  a.fnbr = take(32 * Nfp * K * ts);
  a.qbar = take(9 * Np * K * ts);
  a.rbar = take(9 * Np * K * ts);
  a.rhs = take(9 * Np * K * ts);
  a.rhsv = take(static_cast<size_t>(every) * 5 * 3 * Np * K * ts);
  a.res = take(9 * Np * K * ts);
  a.g = reinterpret_cast<double*>(take(3 * K * 8));
  a.resid = reinterpret_cast<double*>(take(static_cast<size_t>(max_steps) * (max_rec > 0 ? max_rec : 1) * 3 * 8));
  a.ck_q = take(nck * 9 * Np * K * ts);
  a.ck_s = take(nck * 6 * Np * K * ts);
  // stage inputs (q_i, sigma_h(q_i)) of every stage of every step of one
  // segment, plus one slot for the last stage output
  const size_t nst = static_cast<size_t>(every) * 5 + 1;
  a.st_q = take(nst * 9 * Np * K * ts);
  a.st_s = take(nst * 6 * Np * K * ts);
  if (overlap) {   // the second segment buffer
    a.rhsv2 = take(static_cast<size_t>(every) * 5 * 3 * Np * K * ts);
    a.st_q2 = take(nst * 9 * Np * K * ts);
    a.st_s2 = take(nst * 6 * Np * K * ts);
  }
  if (ad) *ad = a;
  return off;
}

// Snapshot slot i of a [n][K][m][Np] array.
void* slot(void* base, const ewdg_ctx* c, int m, size_t i) {
  return static_cast<char*>(base) + i * m * c->re.Np * static_cast<size_t>(c->mesh.K) * c->tsz();
}

int copy_dev(ewdg_ctx* c, void* dst, const void* src, int m, hipStream_t st = nullptr) {
  const size_t bytes = static_cast<size_t>(m) * c->re.Np * c->mesh.K * c->tsz();
  return c->hip(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st ? st : c->stream), "snapshot copy");
}

// One LSRK stage on caller buffers (the context state is untouched); with
// rhsv the velocity rows of the stage's right-hand side are kept as well.
int stage_on(ewdg_ctx* c, int i, double dt, double tn, const void* qin, const void* sin, void* qout, void* sout,
             void* rhsv = nullptr, hipStream_t st = nullptr) {
  const StageCoef sc = coef(c, kRkA[i], kRkB[i], dt, tn + kRkC[i] * dt);
  return c->hip(launch_stage(c->d, rhsv ? 2 : 1, qin, sin, qout, sout, c->ad.res, sc, st ? st : c->stream, rhsv),
                "recompute stage");
}

int need_adj(ewdg_ctx* c) {
  if (int rc = need(c, true, true, true)) return c ? c->fail(rc, "adjoint needs a mesh, workspace and material") : rc;
  if (!c->adj_bound) return c->fail(EWDG_ESTATE, "no adjoint workspace bound");
  return EWDG_OK;
}

}  // namespace

extern "C" {

int ewdg_adjoint_workspace_bytes(const ewdg_ctx* c, int max_steps, int checkpoint_every, size_t* bytes) {
  if (int rc = need(c, true, true, false)) return rc;
  if (!bytes || max_steps < 1 || checkpoint_every < 1) return EWDG_EINVAL;
  *bytes = adj_layout(c, max_steps, checkpoint_every, c->max_rec, nullptr, nullptr, false);
  return EWDG_OK;
}

int ewdg_adjoint_workspace_bytes_overlapped(const ewdg_ctx* c, int max_steps, int checkpoint_every, size_t* bytes) {
  if (int rc = need(c, true, true, false)) return rc;
  if (!bytes || max_steps < 1 || checkpoint_every < 1) return EWDG_EINVAL;
  *bytes = adj_layout(c, max_steps, checkpoint_every, c->max_rec, nullptr, nullptr, true);
  return EWDG_OK;
}

int ewdg_bind_adjoint_workspace(ewdg_ctx* c, void* ptr, size_t bytes, int max_steps, int checkpoint_every) {
  if (int rc = need(c, true, true, false)) return c ? c->fail(rc, "bind the forward workspace first") : rc;
  if (c->mesh.bc != 0 || c->d.wadg)
    return c->fail(EWDG_EINVAL, "the adjoint needs a periodic mesh and the exact mass inverse");
  if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255u))
    return c->fail(EWDG_EINVAL, "adjoint workspace must be a non-null 256-byte aligned device pointer");
  if (max_steps < 1 || checkpoint_every < 1) return c->fail(EWDG_EINVAL, "max_steps and checkpoint_every must be >= 1");
  if (bytes < adj_layout(c, max_steps, checkpoint_every, c->max_rec, nullptr, nullptr, false))
    return c->fail(EWDG_ENOMEM, "adjoint workspace smaller than ewdg_adjoint_workspace_bytes");
  const bool overlap = bytes >= adj_layout(c, max_steps, checkpoint_every, c->max_rec, nullptr, nullptr, true);
  if (overlap && !c->adj_stream) {
    if (int rc = c->hip(hipStreamCreateWithFlags(&c->adj_stream, hipStreamNonBlocking), "adjoint stream")) return rc;
    for (hipEvent_t* e : {&c->ev_start, &c->ev_rec[0], &c->ev_rec[1], &c->ev_rev[0], &c->ev_rev[1]})
      if (int rc = c->hip(hipEventCreateWithFlags(e, hipEventDisableTiming), "adjoint event")) return rc;
  }
  c->adj_overlap = overlap;
  adj_layout(c, max_steps, checkpoint_every, c->max_rec, static_cast<char*>(ptr), &c->ad, overlap);
  // the recomputation register is scaled by a_1 = 0 at every step start, so
  // it only has to hold finite values
  if (int rc = c->hip(hipMemsetAsync(c->ad.res, 0, 9 * static_cast<size_t>(c->re.Np) * c->mesh.K * c->tsz(),
                                     c->stream), "memset"))
    return rc;
  c->adj_bound = true;
  c->adj_max_steps = max_steps;
  c->adj_every = checkpoint_every;
  c->adj_rec = c->max_rec;
  c->fwd_done = false;
  return c->hip(hipStreamSynchronize(c->stream), "adjoint bind sync");
}

int ewdg_rhs_adjoint(ewdg_ctx* c, double t, const void* q, const void* y, void* LTy, double* g) {
  if (int rc = need_adj(c)) return rc;
  if (!y || !LTy || (g && !q)) return c->fail(EWDG_EINVAL, "rhs_adjoint needs y, LTy, and q when g is requested");
  const size_t n = 9 * static_cast<size_t>(c->re.Np) * c->mesh.K;
  int rc;
  if ((rc = c->hip(hipMemsetAsync(LTy, 0, n * c->tsz(), c->stream), "memset"))) return rc;
  const void* s = nullptr;
  if (q) {
    s = c->ad.st_s;
    if ((rc = c->hip(launch_sigma(c->d, q, c->ad.st_s, c->stream), "sigma"))) return rc;
    const StageCoef sc = coef(c, 0.0, 0.0, 0.0, t);
    if ((rc = c->hip(launch_stage(c->d, 0, q, s, nullptr, nullptr, c->ad.rhs, sc, c->stream), "rhs"))) return rc;
  }
  if (g) {
    if ((rc = c->hip(hipMemsetAsync(g, 0, 3 * static_cast<size_t>(c->mesh.K) * 8, c->stream), "memset"))) return rc;
  }
  return c->hip(launch_adjoint(c->d, c->ad, y, q, s, c->ad.rhs, 9 * c->re.Np, LTy, g, 1.0, nullptr, 0.0, 0.0,
                               c->stream),
                "adjoint");
}

int ewdg_forward_misfit(ewdg_ctx* c, double dt, int nsteps, const double* data, double* J) {
  if (int rc = need_adj(c)) return rc;
  if (!(dt > 0.0) || nsteps < 1 || !J || (c->nr > 0 && !data)) return c->fail(EWDG_EINVAL, "bad forward_misfit arguments");
  if (nsteps > c->adj_max_steps) return c->fail(EWDG_ENOMEM, "more steps than the adjoint workspace holds");
  if (c->nr > c->adj_rec) return c->fail(EWDG_ENOMEM, "more receivers than the adjoint workspace holds");
  if (c->nr > 0 && nsteps > c->max_steps) return c->fail(EWDG_ENOMEM, "receiver record capacity exceeded");
  c->fwd_done = false;
  c->rec_count = 0;
  c->step_t.assign(nsteps, 0.0);
  const int C = c->adj_every;
  int rc;
  for (int n = 0; n < nsteps; ++n) {
    if (n % C == 0) {
      const size_t k = n / C;
      if ((rc = copy_dev(c, slot(c->ad.ck_q, c, 9, k), c->d.q[c->cur], 9))) return rc;
      if ((rc = copy_dev(c, slot(c->ad.ck_s, c, 6, k), c->d.s[c->cur], 6))) return rc;
    }
    c->step_t[n] = c->t;
    if ((rc = ewdg_step(c, dt, 1))) return rc;
  }
  double acc = 0.0;
  if (c->nr > 0) {
    const size_t m = static_cast<size_t>(nsteps) * c->nr * 3;
    std::vector<double> tr(m), r(m);
    int ns = 0;
    if ((rc = ewdg_receivers(c, tr.data(), &ns))) return rc;
    for (size_t i = 0; i < m; ++i) {
      r[i] = tr[i] - data[i];
      acc += r[i] * r[i];
    }
    if ((rc = c->hip(hipMemcpy(c->ad.resid, r.data(), m * 8, hipMemcpyHostToDevice), "residual upload"))) return rc;
  }
  if ((rc = c->hip(hipStreamSynchronize(c->stream), "forward sync"))) return rc;
  *J = 0.5 * dt * acc;
  c->fwd_steps = nsteps;
  c->fwd_dt = dt;
  c->fwd_done = true;
  return EWDG_OK;
}

int ewdg_adjoint_gradient(ewdg_ctx* c, double* g, void* qbar0) {
  if (int rc = need_adj(c)) return rc;
  if (!g) return c->fail(EWDG_EINVAL, "adjoint_gradient needs g");
  if (!c->fwd_done) return c->fail(EWDG_ESTATE, "no recorded forward run (ewdg_forward_misfit)");
  const int64_t K = c->mesh.K;
  const size_t n9 = 9 * static_cast<size_t>(c->re.Np) * K;
  const int C = c->adj_every, NS = c->fwd_steps;
  const double dt = c->fwd_dt;
  const AdjDev& a = c->ad;
  int rc;
  if ((rc = c->hip(hipMemsetAsync(a.qbar, 0, n9 * c->tsz(), c->stream), "memset"))) return rc;
  if ((rc = c->hip(hipMemsetAsync(a.rbar, 0, n9 * c->tsz(), c->stream), "memset"))) return rc;
  if ((rc = c->hip(hipMemsetAsync(a.g, 0, 3 * static_cast<size_t>(K) * 8, c->stream), "memset"))) return rc;
  const int nseg = (NS + C - 1) / C;
  // Segment buffers: with the overlapped layout segment seg uses buffer
  // seg & 1, and segment seg - 1 is recomputed on the second stream while
  // segment seg is reversed on the context's stream (events order the
  // hand-over of each buffer); otherwise one buffer, all on one stream.
  const bool ov = c->adj_overlap;
  hipStream_t rs = ov ? c->adj_stream : c->stream;
  auto buf_q = [&](int seg) { return (ov && (seg & 1)) ? a.st_q2 : a.st_q; };
  auto buf_s = [&](int seg) { return (ov && (seg & 1)) ? a.st_s2 : a.st_s; };
  auto buf_v = [&](int seg) { return (ov && (seg & 1)) ? a.rhsv2 : a.rhsv; };
  // every stage input of a segment and the velocity rows of every stage
  // right-hand side, recomputed from the segment's checkpoint; slot 5 m + i
  // holds the input of stage i of step m
  auto recompute = [&](int seg) -> int {
    const int s0 = seg * C, len = std::min(C, NS - s0);
    void *sq = buf_q(seg), *ss = buf_s(seg), *sv = buf_v(seg);
    if (int r = copy_dev(c, slot(sq, c, 9, 0), slot(a.ck_q, c, 9, seg), 9, rs)) return r;
    if (int r = copy_dev(c, slot(ss, c, 6, 0), slot(a.ck_s, c, 6, seg), 6, rs)) return r;
    for (int m = 0; m < len; ++m) {
      const double tn = c->step_t[s0 + m];
      for (int i = 0; i < 5; ++i) {
        const size_t k = 5 * static_cast<size_t>(m) + i;
        if (int r = stage_on(c, i, dt, tn, slot(sq, c, 9, k), slot(ss, c, 6, k), slot(sq, c, 9, k + 1),
                             slot(ss, c, 6, k + 1), slot(sv, c, 3, k), rs))
          return r;
      }
    }
    return EWDG_OK;
  };
  if (ov) {
    // the checkpoints and the cleared adjoint registers come from this stream
    if ((rc = c->hip(hipEventRecord(c->ev_start, c->stream), "event"))) return rc;
    if ((rc = c->hip(hipStreamWaitEvent(rs, c->ev_start, 0), "event wait"))) return rc;
    if ((rc = recompute(nseg - 1))) return rc;
    if ((rc = c->hip(hipEventRecord(c->ev_rec[(nseg - 1) & 1], rs), "event"))) return rc;
  }
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int s0 = seg * C, len = std::min(C, NS - s0);
    if (ov) {
      if (seg >= 1) {
        const int b = (seg - 1) & 1;
        // buffer b was last read by the reverse sweep of segment seg + 1
        if (seg + 1 <= nseg - 1 && (rc = c->hip(hipStreamWaitEvent(rs, c->ev_rev[b], 0), "event wait"))) return rc;
        if ((rc = recompute(seg - 1))) return rc;
        if ((rc = c->hip(hipEventRecord(c->ev_rec[b], rs), "event"))) return rc;
      }
      if ((rc = c->hip(hipStreamWaitEvent(c->stream, c->ev_rec[seg & 1], 0), "event wait"))) return rc;
    } else if ((rc = recompute(seg))) {
      return rc;
    }
    void *sq = buf_q(seg), *ss = buf_s(seg), *sv = buf_v(seg);
    for (int m = len - 1; m >= 0; --m) {
      const int n = s0 + m;
      // misfit term of the state after step n
      if (c->nr > 0) {
        if ((rc = c->hip(launch_adj_receivers(c->d, a.qbar, a.resid + static_cast<size_t>(n) * c->nr * 3, c->nr, dt,
                                              c->stream), "adjoint receivers")))
          return rc;
      }
      // reverse stage i: rbar += b_i qbar; qbar += dt L^T rbar (and the
      // gradient); rbar *= a_i.  The scaling and the next stage's axpy
      // (b_{i-1}; none after stage 1, whose a_1 = 0 clears rbar) run inside
      // the adjoint kernel; only the first axpy of a step, after the
      // misfit term, is a launch of its own.
      if ((rc = c->hip(launch_axpy(c->prec, a.rbar, a.qbar, kRkB[4], static_cast<int64_t>(n9), c->stream), "axpy")))
        return rc;
      for (int i = 4; i >= 0; --i) {
        const size_t k = 5 * static_cast<size_t>(m) + i;
        if ((rc = c->hip(launch_adjoint(c->d, a, a.rbar, slot(sq, c, 9, k), slot(ss, c, 6, k),
                                        slot(sv, c, 3, k), 3 * c->re.Np, a.qbar, a.g, dt, a.rbar, kRkA[i],
                                        i > 0 ? kRkB[i - 1] : 0.0, c->stream),
                         "adjoint")))
          return rc;
      }
    }
    // this segment's buffer may be refilled once its reverse sweep is done
    if (ov && (rc = c->hip(hipEventRecord(c->ev_rev[seg & 1], c->stream), "event"))) return rc;
  }
  if ((rc = c->hip(hipMemcpyAsync(g, a.g, 3 * static_cast<size_t>(K) * 8, hipMemcpyDefault, c->stream), "g copy")))
    return rc;
  if (qbar0) {
    if ((rc = c->hip(hipMemcpyAsync(qbar0, a.qbar, n9 * c->tsz(), hipMemcpyDefault, c->stream), "qbar copy")))
      return rc;
  }
  return c->hip(hipStreamSynchronize(c->stream), "adjoint sync");
}

}  // extern "C"

// ----------------------------------------------------------------------------
// Locally implicit step: the theta scheme solved by iHDG-II (Sec. 3,
// Algorithm 1; Sec. 4.3).
namespace {

size_t imp_layout(ewdg_ctx* c, char* base) {
  const int64_t K = c->mesh.K;
  const size_t Np = c->re.Np, ts = c->tsz();
  const int nv = 9 * static_cast<int>(Np);
  const int n = static_cast<int>(pad_to(nv, 16));
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return p;
  };
  ImpDev& m = c->im;
  m.nv = nv;
  m.n = n;
  const size_t mats = static_cast<size_t>(K) * n * n;
  m.inv = take(mats * ts);
  m.work = c->prec == 64 ? static_cast<double*>(m.inv) : reinterpret_cast<double*>(take(mats * 8));
  m.b = take(static_cast<size_t>(K) * nv * ts);
  m.L = take(static_cast<size_t>(K) * nv * ts);
  m.s = take(static_cast<size_t>(K) * 6 * Np * ts);
  m.members = reinterpret_cast<int32_t*>(take(static_cast<size_t>(K) * 4));
  m.epart = reinterpret_cast<double*>(take(static_cast<size_t>(K) * 8));
  m.norm2 = reinterpret_cast<double*>(take(8));
  m.flag = reinterpret_cast<int32_t*>(take(4));
  return off;
}

// Greedy colouring of the face-adjacency graph; members lists the elements
// colour by colour, cstart[c] the first position of colour c.
int colour_classes(const MeshData& m, std::vector<int32_t>& members, std::vector<int>& cstart) {
  const int64_t K = m.K;
  std::vector<int> col(K, -1);
  int ncol = 0;
  for (int64_t k = 0; k < K; ++k) {
    unsigned used = 0;
    for (int f = 0; f < 4; ++f) {
      if (m.bc != 0 && ((m.bcm[k] >> (2 * f)) & 3)) continue;   // boundary face
      const int64_t nb = m.conn[k * 4 + f] >> 5;
      if (nb == k) return EWDG_EMESH;
      if (col[nb] >= 0 && col[nb] < 32) used |= 1u << col[nb];
    }
    int cc = 0;
    while (used & (1u << cc)) ++cc;
    col[k] = cc;
    ncol = std::max(ncol, cc + 1);
  }
  cstart.assign(ncol + 1, 0);
  for (int64_t k = 0; k < K; ++k) ++cstart[col[k] + 1];
  for (int cc = 0; cc < ncol; ++cc) cstart[cc + 1] += cstart[cc];
  members.assign(K, 0);
  std::vector<int> at(cstart.begin(), cstart.end() - 1);
  for (int64_t k = 0; k < K; ++k) members[at[col[k]]++] = static_cast<int32_t>(k);
  return EWDG_OK;
}

}  // namespace

extern "C" {

int ewdg_implicit_workspace_bytes(const ewdg_ctx* c, size_t* bytes) {
  if (int rc = need(c, true, false, false)) return rc;
  if (!bytes) return EWDG_EINVAL;
  ewdg_ctx tmp;
  tmp.N = c->N;
  tmp.prec = c->prec;
  tmp.re.Np = c->re.Np;
  tmp.mesh.K = c->mesh.K;
  *bytes = imp_layout(&tmp, nullptr);
  return EWDG_OK;
}

int ewdg_bind_implicit_workspace(ewdg_ctx* c, void* ptr, size_t bytes) {
  if (int rc = need(c, true, true, false)) return c ? c->fail(rc, "bind the main workspace first") : rc;
  if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255u))
    return c->fail(EWDG_EINVAL, "workspace must be a non-null 256-byte aligned device pointer");
  if (bytes < imp_layout(c, nullptr)) return c->fail(EWDG_ENOMEM, "workspace smaller than ewdg_implicit_workspace_bytes");
  imp_layout(c, static_cast<char*>(ptr));
  std::vector<int32_t> members;
  if (colour_classes(c->mesh, members, c->imp_cstart) != EWDG_OK)
    return c->fail(EWDG_EMESH, "an element is its own face neighbour");
  int rc;
  if ((rc = upload(c, c->im.members, members.data(), members.size() * 4))) return rc;
  c->imp_bound = true;
  c->imp_ready = false;
  return EWDG_OK;
}

int ewdg_implicit_setup(ewdg_ctx* c, double dt, double theta) {
  if (int rc = need(c, true, true, true)) return c ? c->fail(rc, "implicit setup needs material") : rc;
  if (!c->imp_bound) return c->fail(EWDG_ESTATE, "implicit setup needs ewdg_bind_implicit_workspace");
  if (!(dt > 0.0) || !std::isfinite(dt) || !(theta > 0.0 && theta <= 1.0))
    return c->fail(EWDG_EINVAL, "need dt > 0 and 0 < theta <= 1");
  ImpDev& m = c->im;
  const int64_t K = c->mesh.K;
  const double thdt = theta * dt;
  int rc;
  c->imp_ready = false;
  if ((rc = c->hip(launch_imp_identity(m.work, K, m.n, c->stream), "identity"))) return rc;
  if ((rc = c->hip(launch_imp_zero(c->prec, m.b, K * m.nv, c->stream), "zero"))) return rc;
  // column j of A_k for every element k of one colour class: the operator
  // of the state that is the j-th unit value on every member of the class
  StageCoef none;   // no source
  for (size_t cc = 0; cc + 1 < c->imp_cstart.size(); ++cc) {
    const int32_t* mem = m.members + c->imp_cstart[cc];
    const int cnt = c->imp_cstart[cc + 1] - c->imp_cstart[cc];
    for (int j = 0; j < m.nv; ++j) {
      if ((rc = c->hip(launch_imp_probe(c->prec, m.b, mem, cnt, m.nv, j - 1, j, c->stream), "probe"))) return rc;
      if ((rc = c->hip(launch_sigma(c->d, m.b, m.s, c->stream), "sigma"))) return rc;
      if ((rc = c->hip(launch_stage(c->d, 0, m.b, m.s, nullptr, nullptr, m.L, none, c->stream), "operator")))
        return rc;
      if ((rc = c->hip(launch_imp_gather(c->prec, m.L, m.work, mem, cnt, m.nv, m.n, j, thdt, c->stream), "gather")))
        return rc;
    }
    if ((rc = c->hip(launch_imp_probe(c->prec, m.b, mem, cnt, m.nv, m.nv - 1, -1, c->stream), "probe"))) return rc;
  }
  const int32_t zero = 0;
  if ((rc = upload(c, m.flag, &zero, 4))) return rc;
  if ((rc = c->hip(launch_imp_invert(m.work, K, m.n, m.flag, c->stream), "invert"))) return rc;
  if (c->prec == 32) {
    if ((rc = c->hip(launch_imp_to_float(m.work, static_cast<float*>(m.inv), K * m.n * m.n, c->stream), "convert")))
      return rc;
  }
  int32_t flag = 0;
  if ((rc = c->hip(hipMemcpyAsync(&flag, m.flag, 4, hipMemcpyDeviceToHost, c->stream), "flag copy"))) return rc;
  if ((rc = c->hip(hipStreamSynchronize(c->stream), "implicit setup sync"))) return rc;
  if (flag) return c->fail(EWDG_EINVAL, "a local matrix I - theta dt A_k has a vanishing pivot");
  c->imp_dt = dt;
  c->imp_theta = theta;
  c->imp_ready = true;
  return EWDG_OK;
}

int ewdg_implicit_step(ewdg_ctx* c, int nsteps, double tol, int max_iters, int* iters, double* change) {
  if (int rc = need(c, true, true, true)) return rc;
  if (!c->imp_ready) return c->fail(EWDG_ESTATE, "implicit step needs ewdg_implicit_setup (again after new material)");
  if (nsteps < 0 || !(tol >= 0.0) || max_iters < 1) return EWDG_EINVAL;
  if (c->nr > 0 && c->rec_count + nsteps > c->max_steps)
    return c->fail(EWDG_ENOMEM, "receiver record capacity exceeded");
  ImpDev& m = c->im;
  const double dt = c->imp_dt, th = c->imp_theta;
  int rc;
  for (int n = 0; n < nsteps; ++n) {
    void* q = c->d.q[c->cur];
    // b = q^m + (1 - theta) dt (L q^m + s^m) + theta dt s^{m+1}
    const void* Lm = nullptr;
    if (th < 1.0) {
      const StageCoef sc = coef(c, 0.0, 0.0, 0.0, c->t);
      if ((rc = c->hip(launch_stage(c->d, 0, q, c->d.s[c->cur], nullptr, nullptr, m.L, sc, c->stream), "operator")))
        return rc;
      Lm = m.L;
    }
    const StageCoef next = coef(c, 0.0, 0.0, 0.0, c->t + dt);
    if ((rc = c->hip(launch_imp_fixed(c->d, m, q, Lm, (1.0 - th) * dt, next.src_elem, th * dt * next.srcval, next.dir,
                                      c->stream),
                     "fixed part")))
      return rc;
    int it = 0;
    double dq = 0.0;
    const StageCoef none;
    while (it < max_iters) {
      if ((rc = c->hip(launch_sigma(c->d, q, m.s, c->stream), "sigma"))) return rc;
      if ((rc = c->hip(launch_stage(c->d, 0, q, m.s, nullptr, nullptr, m.L, none, c->stream), "operator"))) return rc;
      if ((rc = c->hip(launch_imp_iterate(c->d, m, q, th * dt, c->stream), "iterate"))) return rc;
      double n2 = 0.0;
      if ((rc = c->hip(hipMemcpyAsync(&n2, m.norm2, 8, hipMemcpyDeviceToHost, c->stream), "norm copy"))) return rc;
      if ((rc = c->hip(hipStreamSynchronize(c->stream), "norm sync"))) return rc;
      ++it;
      dq = std::sqrt(std::max(n2, 0.0));
      if (!std::isfinite(dq)) return c->fail(EWDG_EINVAL, "iHDG-II iteration produced a non-finite change");
      if (dq < tol) break;
    }
    if (iters) iters[n] = it;
    if (change) change[n] = dq;
    // sigma_h of the new state, kept beside it for the explicit stepper
    if ((rc = c->hip(launch_sigma(c->d, q, c->d.s[c->cur], c->stream), "sigma"))) return rc;
    c->t = c->t + dt;
    if (c->nr > 0) {
      if ((rc = c->hip(launch_receivers(c->d, q, c->nr, c->rec_count, c->stream), "receivers"))) return rc;
      ++c->rec_count;
    }
  }
  return EWDG_OK;
}

int ewdg_implicit_dt(const ewdg_ctx* c, double* dt, double* theta) {
  if (!c || !dt || !theta) return EWDG_EINVAL;
  if (!c->imp_ready) return EWDG_ESTATE;
  *dt = c->imp_dt;
  *theta = c->imp_theta;
  return EWDG_OK;
}

}  // extern "C"
