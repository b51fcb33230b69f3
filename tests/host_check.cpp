// Host-only exercise of the C ABI for the sanitizer build (AddressSanitizer
// and UndefinedBehaviorSanitizer on the host code of the library): reference
// elements of every degree, mesh building and connectivity, geometry
// queries, workspace sizing and the argument and state error paths.  Makes
// no call that needs a GPU.
//
// usage: host_check MESH_DIR
//   MESH_DIR holds K.txt (one integer), EToV.bin (int64 [K][4]) and
//   VXYZ.bin (float64 [K][4][3]) of a periodic tetrahedral mesh.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <string>
#include <vector>

#include "ewdg.h"

static int failures = 0;

#define CHECK(cond)                                                         \
  do {                                                                      \
    if (!(cond)) {                                                          \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                           \
    }                                                                       \
  } while (0)

template <typename T>
static std::vector<T> read_all(const std::string& path, size_t count) {
  std::vector<T> v(count);
  std::ifstream f(path, std::ios::binary);
  f.read(reinterpret_cast<char*>(v.data()), static_cast<std::streamsize>(count * sizeof(T)));
  if (!f) {
    std::fprintf(stderr, "cannot read %s\n", path.c_str());
    std::exit(2);
  }
  return v;
}

int main(int argc, char** argv) {
  if (argc < 2) {
    std::fprintf(stderr, "usage: host_check MESH_DIR\n");
    return 2;
  }
  const std::string dir = argv[1];
  int64_t K = 0;
  {
    std::ifstream f(dir + "/K.txt");
    f >> K;
  }
  const std::vector<int64_t> EToV = read_all<int64_t>(dir + "/EToV.bin", static_cast<size_t>(K) * 4);
  const std::vector<double> VXYZ = read_all<double>(dir + "/VXYZ.bin", static_cast<size_t>(K) * 12);

  // unsupported degrees and precisions
  ewdg_ctx* bad = nullptr;
  CHECK(ewdg_create(6, 32, nullptr, &bad) == EWDG_EINVAL);
  CHECK(ewdg_create(4, 16, nullptr, &bad) == EWDG_EINVAL);
  CHECK(ewdg_create(4, 32, nullptr, nullptr) == EWDG_EINVAL);

  const int degrees[6] = {1, 2, 3, 4, 5, 7};
  for (int N : degrees) {
    for (int prec : {32, 64}) {
      ewdg_ctx* c = nullptr;
      CHECK(ewdg_create(N, prec, nullptr, &c) == EWDG_OK);
      if (!c) continue;
      int Np = 0, Nfp = 0, Nq = 0;
      CHECK(ewdg_sizes(c, &Np, &Nfp, &Nq) == EWDG_OK);
      CHECK(Np == (N + 1) * (N + 2) * (N + 3) / 6 && Nfp == (N + 1) * (N + 2) / 2 && Nq == (N + 1) * (N + 1) * (N + 1));
      // state errors before a mesh
      size_t bytes = 0;
      CHECK(ewdg_workspace_bytes(c, 0, 0, &bytes) == EWDG_ESTATE);
      CHECK(ewdg_implicit_workspace_bytes(c, &bytes) == EWDG_ESTATE);
      double dt = 0;
      CHECK(ewdg_cfl_dt(c, 0.5, &dt) == EWDG_ESTATE);
      CHECK(ewdg_step(c, 1e-3, 1) == EWDG_ESTATE);
      // reference operators: finite values
      const size_t sizes[11] = {size_t(Np) * Np, size_t(Np) * Np, size_t(Np) * Np, size_t(Np) * 4 * Nfp,
                                size_t(Nq) * Np, size_t(Np) * Nq, size_t(Np) * Np, size_t(Np) * 3,
                                size_t(Nq), size_t(4) * Nfp, size_t(4) * 4 * 6 * Nfp};
      for (int which = 0; which < 11; ++which) {
        std::vector<double> op(sizes[which], NAN);
        CHECK(ewdg_reference_operator(c, which, op.data()) == EWDG_OK);
        for (double x : op) CHECK(std::isfinite(x));
      }
      CHECK(ewdg_reference_operator(c, 11, nullptr) == EWDG_EINVAL);
      // mesh errors: null arrays, empty, a single unmatched element
      CHECK(ewdg_set_mesh(c, K, nullptr, VXYZ.data()) == EWDG_EINVAL);
      CHECK(ewdg_set_mesh(c, 0, EToV.data(), VXYZ.data()) == EWDG_EINVAL);
      CHECK(ewdg_set_mesh(c, 1, EToV.data(), VXYZ.data()) == EWDG_EMESH);
      // the periodic mesh
      CHECK(ewdg_set_mesh(c, K, EToV.data(), VXYZ.data()) == EWDG_OK);
      std::vector<double> xn(static_cast<size_t>(K) * Np * 3), xq(static_cast<size_t>(K) * Nq * 3);
      CHECK(ewdg_node_points(c, xn.data()) == EWDG_OK);
      CHECK(ewdg_quadrature_points(c, xq.data()) == EWDG_OK);
      for (double x : xn) CHECK(x >= -1.0 - 1e-12 && x <= 1.0 + 1e-12);
      for (double x : xq) CHECK(x > -1.0 && x < 1.0);
      std::vector<int32_t> conn(static_cast<size_t>(K) * 4, -1);
      CHECK(ewdg_connectivity(c, conn.data()) == EWDG_OK);
      for (int64_t k = 0; k < K; ++k)
        for (int f = 0; f < 4; ++f) {
          const int32_t w = conn[static_cast<size_t>(k) * 4 + f];
          const int64_t nb = w >> 5;
          const int g = (w & 31) / 6;
          CHECK(nb >= 0 && nb < K && nb != k && g < 4);
          // the neighbour's face g points back to (k, f)
          if (nb >= 0 && nb < K && g < 4) CHECK((conn[static_cast<size_t>(nb) * 4 + g] >> 5) == k);
        }
      CHECK(ewdg_workspace_bytes(c, 4, 100, &bytes) == EWDG_OK && bytes > 0);
      size_t ib = 0;
      CHECK(ewdg_implicit_workspace_bytes(c, &ib) == EWDG_OK && ib > bytes);
      CHECK(ewdg_implicit_setup(c, 1e-3, 1.0) == EWDG_ESTATE);       // nothing bound
      int its = 0;
      CHECK(ewdg_implicit_step(c, 1, 1e-10, 10, &its, nullptr) == EWDG_ESTATE);
      double idt = 0, ith = 0;
      CHECK(ewdg_implicit_dt(c, &idt, &ith) == EWDG_ESTATE);
      size_t ab = 0;
      CHECK(ewdg_adjoint_workspace_bytes(c, 100, 10, &ab) == EWDG_ESTATE);   // no workspace bound
      // calls that need the workspace or the material
      CHECK(ewdg_set_material(c, nullptr, nullptr, nullptr) != EWDG_OK);
      CHECK(ewdg_cfl_dt(c, 0.5, &dt) == EWDG_ESTATE);
      const double xs[3] = {0.1, 0.2, 0.3}, d[3] = {0, 0, 1};
      CHECK(ewdg_set_source(c, xs, d, 1.0, 5.0, 0.2) != EWDG_OK);
      CHECK(ewdg_set_receivers(c, 1, xs) != EWDG_OK);
      CHECK(ewdg_step(c, 1e-3, 1) == EWDG_ESTATE);
      double E = 0;
      CHECK(ewdg_energy(c, &E) != EWDG_OK);
      CHECK(ewdg_last_error(c) != nullptr);
      CHECK(ewdg_destroy(c) == EWDG_OK);
    }
  }
  size_t tb = 0;
  CHECK(ewdg_batch_table_bytes(-1, &tb) == EWDG_EINVAL);
  CHECK(ewdg_batch_table_bytes(8, &tb) == EWDG_OK && tb > 0);
  CHECK(ewdg_step_batch(nullptr, 0, nullptr, 1, nullptr, 0, nullptr) == EWDG_OK);
  CHECK(ewdg_step_batch_static(nullptr, 0, nullptr, 1, nullptr) == EWDG_OK);
  CHECK(ewdg_static_table_max_bytes(&tb) == EWDG_OK && tb == 256 * 1024);
  // transport: reference operators of every supported (dim, p), points, errors
  const double beta[3] = {1.0, -0.8, 0.6};
  ewdg_tr* tr = nullptr;
  CHECK(ewdg_transport_create(4, 2, 3, beta, 64, nullptr, &tr) == EWDG_EINVAL);
  CHECK(ewdg_transport_create(2, 5, 3, beta, 64, nullptr, &tr) == EWDG_EINVAL);
  for (int dim = 2; dim <= 3; ++dim)
    for (int p = 1; p <= 4; ++p) {
      tr = nullptr;
      CHECK(ewdg_transport_create(dim, p, 2, beta, 32, nullptr, &tr) == EWDG_OK);
      if (!tr) continue;
      int64_t E = 0;
      int Np = 0, Nq = 0, Nqf = 0;
      CHECK(ewdg_transport_sizes(tr, &E, &Np, &Nq, &Nqf) == EWDG_OK && E == (dim == 2 ? 4 : 8));
      std::vector<double> xv(static_cast<size_t>(E) * Nq * dim), xf(static_cast<size_t>(E) * 2 * dim * Nqf * dim);
      CHECK(ewdg_transport_points(tr, xv.data(), xf.data()) == EWDG_OK);
      for (double x : xv) CHECK(x > 0.0 && x < 1.0);
      for (double x : xf) CHECK(x >= 0.0 && x <= 1.0);
      size_t wb = 0;
      CHECK(ewdg_transport_workspace_bytes(tr, &wb) == EWDG_OK && wb > 0);
      int its = 0;
      CHECK(ewdg_transport_solve(tr, 1e-10, 10, &its, nullptr) == EWDG_ESTATE);
      CHECK(ewdg_transport_set_problem(tr, xv.data(), xv.data(), nullptr) == EWDG_ESTATE);
      CHECK(ewdg_transport_destroy(tr) == EWDG_OK);
    }
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("host_check: all checks passed (K = %lld)\n", static_cast<long long>(K));
  return 0;
}
