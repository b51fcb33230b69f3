// Device-side views shared by the host runtime and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ewdg {

// Impedances per element: own (Z_p, Z_s), then the neighbour's pair across
// each of the four faces (on a boundary face, the element's own pair).
constexpr int kZS = 10;

// All pointers live inside the caller's workspace.  "Run precision" arrays
// are float or double according to prec; the others are FP64 or int32.
struct Dev {
  int N = 0, prec = 0, Np = 0, Nfp = 0, Nq = 0;
  int64_t K = 0;
  // run precision
  void* q[2] = {nullptr, nullptr};   // [K][9][Np] ping-pong state
  void* s[2] = {nullptr, nullptr};   // [K][6][Np] sigma_h of q[i]
  void* res = nullptr;               // [K][9][Np] LSRK register
  void* W = nullptr;                 // [K][Np][Np], W[k][j][i] = (M_rho^-1 M)_ij
  void* lm = nullptr;                // [K][2][NqP] lambda, mu at quadrature points (NqP = Nq rounded up to 4, zero padded)
  void* geo = nullptr;               // [K][9] dr_i/dx_j
  void* fgeo = nullptr;              // [K][4][4] n_x, n_y, n_z, Fscale
  void* Z = nullptr;                 // [K][kZS]: own Z_p, Z_s, then the neighbour's Z_p, Z_s across faces 0..3
  void* svec = nullptr;              // [Np] source vector M_rho^-1 phi(x_s)
  // operators in matrix-core fragment order (see the stage kernel):
  // [row tile][k-step][64 lanes], zero padded
  void* Dpad = nullptr;              // Dr, Ds, Dt
  void* Lpad = nullptr;              // LIFT, one block per face
  void* Vqpad = nullptr;             // nodes -> quadrature points
  void* Pqpad = nullptr;             // quadrature points -> nodes (L2_Q projection)
  // transposed operators in fragment order for the adjoint
  void* DTpad = nullptr;             // Dr^T, Ds^T, Dt^T        [3][RT][NpK/4][64]
  void* PqTpad = nullptr;            // Pq^T (quadrature rows)  [QT][NpK/4][64]
  void* VqTpad = nullptr;            // Vq^T (node rows)        [RT][NqK/4][64]
  void* VqT = nullptr;               // [Np][Nq]
  void* PqT = nullptr;               // [Nq][Np]
  // row-major operators for the adjoint kernels
  void* Dk = nullptr;                // [3][Np][Np] Dr, Ds, Dt
  void* LIFTr = nullptr;             // [Np][4 Nfp]
  void* Vqr = nullptr;               // [Nq][Np]
  void* Pqr = nullptr;               // [Np][Nq]
  // FP64
  double* Vq64T = nullptr;           // [Np][Nq]
  double* Pq64T = nullptr;           // [Nq][Np]
  double* Mhat64 = nullptr;          // [Np][Np]
  double* wq64 = nullptr;            // [Nq]
  double* rho64 = nullptr;           // [K][Nq]
  double* lam64 = nullptr;
  double* mu64 = nullptr;
  double* J64 = nullptr;             // [K]
  double* means64 = nullptr;         // [K][3] element means of rho, lambda, mu
  double* epart = nullptr;           // [K] energy partials
  double* scal = nullptr;            // [64] small scalars (energy result, source basis)
  double* srcb = nullptr;            // [Np] nodal basis values at the source point
  double* msmall = nullptr;          // [Np][Np] scratch for one element's mass inverse
  double* rec_rows = nullptr;        // [max_rec][Np]
  int32_t* rec_elem = nullptr;       // [max_rec]
  double* rec_out = nullptr;         // [max_steps][max_rec][3]
  // int32
  int32_t* conn = nullptr;           // [K][4] nbr*32 + g*6 + p
  int32_t* nbrnode = nullptr;        // [4][4][6][Nfp] neighbour volume node
  int32_t* nbrface = nullptr;        // [4][4][6][Nfp] neighbour face-local node
  int32_t* fmask = nullptr;          // [4][Nfp]
  int32_t* bcm = nullptr;            // [K] boundary codes, 2 bits per face; null for periodic meshes
  int32_t* bcm_buf = nullptr;        // its storage in the workspace
  // weight-adjusted mass inverse (in place of W): 1/rho at the quadrature
  // points, the source's M^-1 phi(x_s), the raw velocity right-hand side
  bool wadg = false;
  void* rinv = nullptr;              // run precision [K][NqP]
  void* svw = nullptr;               // run precision [Np]
  void* rhsw = nullptr;              // run precision [K][3][Np]
  // scratch for setup (aliases q[1], s[1], res while no state exists)
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
};

struct StageCoef {
  double a = 0, b = 0, dt = 0;       // LSRK coefficients and step
  double srcval = 0;                 // amp * R(t_stage)
  double dir[3] = {0, 0, 0};
  int64_t src_elem = -1;
};

// Launchers (kernels.hip).  Each returns the launch status.
hipError_t launch_material(const Dev& d, hipStream_t st);
hipError_t launch_source_vector(const Dev& d, int64_t elem, hipStream_t st);
hipError_t launch_sigma(const Dev& d, const void* q, void* s, hipStream_t st);
// mode 0: rhs = L(qin) written to out; mode 1: LSRK stage, qin/sin -> qout/sout;
// mode 2: as mode 1, and the velocity rows of L(qin) + f go to rhsv [K][3][Np]
hipError_t launch_stage(const Dev& d, int mode, const void* qin, const void* sin, void* qout,
                        void* sout, void* out, const StageCoef& c, hipStream_t st, void* rhsv = nullptr);
hipError_t launch_project(const Dev& d, const double* fq, void* q, hipStream_t st);
hipError_t launch_evalq(const Dev& d, const void* q, double* fq, hipStream_t st);
hipError_t launch_receivers(const Dev& d, const void* q, int nr, int step, hipStream_t st);
hipError_t launch_energy(const Dev& d, const void* q, double* out, hipStream_t st);
hipError_t launch_rinv(const Dev& d, hipStream_t st);   // d.rinv = 1 / rho (weight-adjusted inverse)
bool supported_degree(int N);

// Batched stages over many meshes of one degree and precision: a device
// table of per-request stage arguments (filled on the host) and the first
// workgroup of each request.
size_t stage_args_bytes(int prec);
void stage_args_fill(const Dev& d, const void* qin, const void* sin, void* qout, void* sout, void* out,
                     const StageCoef& c, void* dst);
int stage_tile_elems();
// records in the table are record_bytes apart (a multiple of 16, at least
// stage_args_bytes(prec))
hipError_t launch_stage_batch(int N, int prec, const void* table, int record_bytes, const int* tile_start,
                              int nreq, int ntiles, hipStream_t st);

}  // namespace ewdg
