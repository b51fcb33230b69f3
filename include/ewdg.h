/*
 * ewdg -- explicit upwind nodal DG for the velocity-strain elastic wave
 * equation on periodic tetrahedral meshes, one AMD Instinct MI355X (gfx950).
 *
 * What is computed.  The semi-discrete operator L(q) of the first-order
 * system sum_k d_k(A_k u) + C u = f (Sec. 2, eq. LPDE) in its elastic
 * velocity-strain instance (C = 0):
 *     rho dv/dt = div(sigma) + f,  de/dt = sym(grad v),
 *     sigma = lambda tr(e) I + 2 mu e,
 * discretised element by element with the upwind HDG flux
 * F^.n = F(u).n + |A|(u - u^) (Sec. 2, eq. RiemannFluxBoth) whose trace u^
 * is eliminated through the single-valued flux condition (Sec. 2, eq.
 * HDGeqn; Sec. 3, eq. iHDGtrace with equal iterates).  With different
 * impedances on the two sides of a face the exact Riemann state per wave
 * mode is used; it reduces to that flux when the material is continuous.
 * Time stepping is the element-by-element explicit update of Sec. 4.3 with
 * forward Euler replaced by Carpenter-Kennedy LSRK(5,4).
 *
 * Discretisation details fixed by this interface:
 *  - unknowns per element: q = (v_x, v_y, v_z, e_xx, e_yy, e_zz, e_yz, e_xz,
 *    e_xy) with tensor shear strains; each field is a degree-N polynomial
 *    stored at Np = (N+1)(N+2)(N+3)/6 nodes (warp & blend nodes);
 *  - state layout q[K][9][Np], element-major, in the context's precision;
 *  - reference element T = {r,s,t >= -1, r+s+t <= -1} with vertices
 *    v0=(-1,-1,-1), v1=(1,-1,-1), v2=(-1,1,-1), v3=(-1,-1,1); element k is
 *    the affine image sending v_i to its i-th vertex;
 *  - quadrature Q_N: Stroud conical product, (N+1)^3 points, Gauss-Jacobi
 *    weights (1-x)^0,(1-x)^1,(1-x)^2 in the collapsed directions a, b, c
 *    with r = (1+a)(1-b)(1-c)/4 - 1, s = (1+b)(1-c)/2 - 1, t = c; point
 *    index q = i + (N+1)(j + (N+1)k) for (a_i, b_j, c_k).  Material fields
 *    are sampled at these points ([K][Nq]) and define the density-weighted
 *    mass and the stress projection sigma_h = P_Q(lambda tr(e) I + 2 mu e);
 *  - impedances Z_p = sqrt(rho(lambda+2mu)), Z_s = sqrt(rho mu) from the
 *    quadrature-weighted element means.
 *
 * Conventions.  Every function returns an int status (EWDG_OK = 0 or a
 * negative EWDG_E* code) and never throws.  ewdg_last_error(ctx) returns a
 * message owned by the context, valid until its next call.  A context is
 * not thread-safe; distinct contexts are independent.  All device work is
 * enqueued on the context's HIP stream (ewdg_step_batch and the overlapped
 * adjoint sweep also use streams of the library's own, forked from and
 * joined back into the caller's stream); functions returning host data
 * synchronise that stream.  Host input arrays are borrowed for the call and
 * copied.  Device memory is owned by the caller: the library works inside
 * caller-allocated workspaces (ewdg_workspace_bytes / ewdg_bind_workspace,
 * and the adjoint's) and never allocates device memory itself; it keeps two
 * pinned host staging buffers for the batch tables.
 */
#ifndef EWDG_H
#define EWDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  EWDG_OK = 0,
  EWDG_EINVAL = -1, /* bad argument, shape or unsupported degree            */
  EWDG_ESTATE = -2, /* call order (e.g. step before material)               */
  EWDG_ENOMEM = -3, /* workspace or receiver capacity too small             */
  EWDG_EHIP = -4,   /* HIP runtime error                                    */
  EWDG_EMESH = -5,  /* unmatched face, J <= 0, non-conforming mesh          */
  EWDG_EPOINT = -6  /* source or receiver outside the mesh                  */
};

typedef struct ewdg_ctx ewdg_ctx;

/* Create a context for degree N (1..5 or 7) and precision 32 or 64 bits.
 * hip_stream is a hipStream_t (NULL = default stream).  Builds the
 * reference element on the host; touches no GPU state. */
int ewdg_create(int N, int precision_bits, void* hip_stream, ewdg_ctx** out);
int ewdg_destroy(ewdg_ctx* ctx);
int ewdg_set_stream(ewdg_ctx* ctx, void* hip_stream);

/* Mesh (Sec. 2: elements, skeleton, outward normals).  EToV[K][4] holds
 * vertex ids with periodic images identified; VXYZ[K][4][3] holds each
 * element's own (unwrapped) vertex coordinates.  Every face must be shared
 * with exactly one other element (EWDG_EMESH otherwise), every element must
 * have positive orientation.  Host arrays.  The kernels use 32-bit element
 * offsets: K < 2^23 and K 9 Np, K Np^2, K 32 Nfp < 2^31 are required
 * (EWDG_EINVAL before any array is read otherwise), e.g. K < 6.8 M at
 * N = 4 and K < 1.99 M at N = 7. */
int ewdg_set_mesh(ewdg_ctx* ctx, int64_t K, const int64_t* EToV, const double* VXYZ);
/* Bounded meshes (the boundary faces of the skeleton, Sec. 2): as
 * ewdg_set_mesh, but faces without a partner are boundary faces with
 * condition bc: EWDG_BC_FREE (traction-free: the exterior state is the
 * mirror v+ = v-, T+ = -T-, so the interface state has zero traction) or
 * EWDG_BC_ABSORBING (zero exterior state: the upwind state keeps only the
 * outgoing characteristics).  EWDG_BC_PERIODIC is ewdg_set_mesh.  A boundary
 * face's ewdg_connectivity entry names the element itself.  The stage,
 * operator, energy, receivers and the implicit step support bounded meshes;
 * batched stepping and the adjoint refuse them (EWDG_EINVAL). */
enum { EWDG_BC_PERIODIC = 0, EWDG_BC_FREE = 1, EWDG_BC_ABSORBING = 2 };
int ewdg_set_mesh_bc(ewdg_ctx* ctx, int64_t K, const int64_t* EToV, const double* VXYZ, int bc);

/* Sizes of one element: nodes, face nodes, quadrature points. */
int ewdg_sizes(const ewdg_ctx* ctx, int* Np, int* Nfp, int* Nq);
/* Physical node and quadrature-point coordinates, host [K][Np][3] / [K][Nq][3]. */
int ewdg_node_points(const ewdg_ctx* ctx, double* xyz);
int ewdg_quadrature_points(const ewdg_ctx* ctx, double* xyz);
/* Reference-element operators (host, FP64, row-major) for inspection:
 * which = 0 Dr, 1 Ds, 2 Dt [Np][Np]; 3 LIFT [Np][4Nfp]; 4 Vq [Nq][Np];
 * 5 Pq [Np][Nq]; 6 reference mass [Np][Np]; 7 nodes (r,s,t) [Np][3];
 * 8 quadrature weights [Nq]; 9 face node list [4][Nfp] (volume node
 * indices); 10 neighbour node table [4][4][6][Nfp]: volume node, in the
 * neighbour, of face node j of face f when the neighbour's face is g and
 * the vertex correspondence is permutation p. */
int ewdg_reference_operator(const ewdg_ctx* ctx, int which, double* out);
/* Face connectivity, host int32 [K][4]: nbr*32 + g*6 + p (neighbour
 * element, its matching face g, vertex permutation p with our face vertex m
 * at the neighbour's face position perm_p(m), perm_0..5 = 012, 021, 102,
 * 120, 201, 210).  Requires the mesh. */
int ewdg_connectivity(const ewdg_ctx* ctx, int32_t* conn);

/* Device workspace needed for the mesh plus up to max_receivers receivers
 * recorded over up to max_record_steps steps.  Requires the mesh. */
int ewdg_workspace_bytes(const ewdg_ctx* ctx, int max_receivers, int max_record_steps,
                         size_t* bytes);
/* Bind caller-owned device memory of at least
 * ewdg_workspace_bytes(ctx, max_receivers, max_record_steps) bytes,
 * 256-byte aligned (EWDG_ENOMEM if too small).  Uploads the mesh tables and
 * reference operators; synchronises.  The memory must stay valid until the
 * context is destroyed or rebound. */
int ewdg_bind_workspace(ewdg_ctx* ctx, void* device_ptr, size_t bytes, int max_receivers,
                        int max_record_steps);

/* Material at the quadrature points, host FP64 [K][Nq] each; rho, mu > 0,
 * lambda >= 0.  Builds on the GPU, in FP64, the per-element density-
 * weighted mass inverse W_rho = M_rho^-1 M (stored in run precision), the
 * impedances, and run-precision copies of lambda and mu.  Resets the state
 * to zero at t = 0. */
int ewdg_set_material(ewdg_ctx* ctx, const double* rho_q, const double* lam_q,
                      const double* mu_q);
/* Mass inverse on the velocity rows (the element-local rho-weighted inverse
 * mass of the update, cf. the weighted norms of Sec. 2).  EWDG_MASS_EXACT
 * (default): W_rho = M_rho^-1 M from the quadrature mass with the sampled
 * density, a stored Np x Np matrix per element.  EWDG_MASS_WEIGHT_ADJUSTED:
 * M_rho^-1 ~ M^-1 M_{1/rho} M^-1, applied as the L2_Q projection of
 * (velocity right-hand side) / rho at the quadrature points (the point
 * source as M^-1 phi(x_s)): exact when rho is constant on every element,
 * otherwise a different (energy-stable) scheme; it reads Nq values of
 * 1/rho per element instead of Np^2.  Needs a bound workspace and a
 * periodic mesh; batched stepping and the adjoint refuse it (EWDG_EINVAL,
 * or EWDG_ESTATE while an adjoint workspace is bound).  The implicit step
 * must be set up again.  ewdg_energy keeps the physical energy (exact
 * M_rho). */
enum { EWDG_MASS_EXACT = 0, EWDG_MASS_WEIGHT_ADJUSTED = 1 };
int ewdg_set_mass_inverse(ewdg_ctx* ctx, int mode);

/* State in the public nodal layout q[K][9][Np] of the context precision;
 * on_device selects device (1) or host (0) memory. */
int ewdg_set_state(ewdg_ctx* ctx, const void* q, int on_device, double t);
int ewdg_get_state(ewdg_ctx* ctx, void* q, int on_device, double* t);
/* L2 projection under Q_N of values at the quadrature points:
 * fq_dev [K][9][Nq] FP64 (device) -> q_dev [K][9][Np] context precision. */
int ewdg_project_quadrature(ewdg_ctx* ctx, const double* fq_dev, void* q_dev);
/* Evaluate a nodal field at the quadrature points (FP64 arithmetic):
 * q_dev [K][9][Np] (NULL = current state) -> fq_dev [K][9][Nq] FP64. */
int ewdg_eval_quadrature(ewdg_ctx* ctx, const void* q_dev, double* fq_dev);

/* Point force amp * R(t) * dir at xs with the Ricker wavelet
 * R(t) = (1 - 2 pi^2 f0^2 (t-t0)^2) exp(-pi^2 f0^2 (t-t0)^2).  The owning
 * element is the lowest-index element containing xs (EWDG_EPOINT if none). */
int ewdg_set_source(ewdg_ctx* ctx, const double xs[3], const double dir[3], double amp,
                    double f0, double t0);
int ewdg_clear_source(ewdg_ctx* ctx);
/* Receivers: v at nr points (host [nr][3]) recorded in FP64 after every
 * full step; recording restarts at zero. */
int ewdg_set_receivers(ewdg_ctx* ctx, int nr, const double* xr);
/* Copy the recorded traces to host out[nsteps][nr][3]; *nsteps receives
 * the number of recorded steps (out may be NULL to query it). */
int ewdg_receivers(ewdg_ctx* ctx, double* out, int* nsteps);

/* dt = cfl * min_K (r_K / max_q c_p) / (N+1)^2 (explicit step scaling
 * h/(p^2 c) of Sec. 4.4); r_K the inradius. */
int ewdg_cfl_dt(const ewdg_ctx* ctx, double cfl, double* dt);

/* One evaluation rhs = L(q) + source at time t, device arrays [K][9][Np]
 * in the context precision.  Does not change the stored state. */
int ewdg_rhs(ewdg_ctx* ctx, double t, const void* q_dev, void* rhs_dev);
/* Advance the stored state by nsteps LSRK(5,4) steps of size dt,
 * recording receivers after each step. */
int ewdg_step(ewdg_ctx* ctx, double dt, int nsteps);
/* Current simulation time. */
int ewdg_time(const ewdg_ctx* ctx, double* t);
/* The energy of the stored state in the material-weighted norms of Sec. 2
 * (the (rho v, v) inner product and the elastic one of sigma = C e),
 * evaluated with the quadrature Q_N:
 *   E = 1/2 (rho v, v)_Q + 1/2 sum_K J sum_q w e:sigma,
 * the quantity the upwind flux makes non-increasing in time.  Accumulated
 * in FP64 with a deterministic reduction; synchronises. */
int ewdg_energy(ewdg_ctx* ctx, double* E);
/* The same energy written to E_dev (one FP64 value of caller-owned device
 * memory) by work enqueued on the context's stream, without synchronising:
 * for health checks that ride on a running stream (the serving loop's
 * per-request NaN and energy-growth guard). */
int ewdg_energy_device(ewdg_ctx* ctx, double* E_dev);

/* Batched stepping of many independent contexts (continuous-batching
 * serving).  Contexts are grouped by (degree, precision); every LSRK stage
 * issues one ragged launch per group covering all elements of all its
 * contexts, so the requests' work overlaps on the device while each
 * context's arithmetic stays exactly that of ewdg_step (results are
 * bitwise identical alone or in any mix).  dts[i] is context i's step; all
 * advance nsteps steps, recording their receivers.  table_dev is caller-
 * owned device memory of at least ewdg_batch_table_bytes(n) bytes holding
 * the per-request launch table.  With at least nsteps times that size
 * rounded up to 256 bytes, the tables of all steps are uploaded at once and
 * each (degree, precision) group runs on a HIP stream of its own (created by
 * the library at first use, default priority), forked from and joined back
 * into hip_stream, so that the groups' launches overlap; otherwise all work
 * is enqueued on hip_stream, one table upload per step.  Either way the
 * work is ordered after earlier work on hip_stream and before later work on
 * it (the contexts' own streams are not used).  A context may appear only
 * once.  Calls from several host threads must not overlap.
 * Errors are reported through the return code; the message of the failing
 * context is in its ewdg_last_error. */
int ewdg_batch_table_bytes(int n, size_t* bytes);
int ewdg_step_batch(ewdg_ctx* const* ctxs, int n, const double* dts, int nsteps, void* table_dev,
                    size_t table_bytes, void* hip_stream);

/* Batched stepping that allocates nothing, for callers that cannot allocate
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation).  Same arguments, arithmetic and results (bitwise) as
 * ewdg_step_batch with a one-step table, minus the caller's table buffer:
 * the launch table lives in a fixed device array of
 * ewdg_static_table_max_bytes bytes (256 KiB; one copy per GPU, held until
 * the process ends), filled from a fixed host array, and all work (one
 * table upload and the launches per step) is enqueued on hip_stream.  No
 * device or pinned memory, stream or event is created.  A batch whose
 * one-step table (ewdg_batch_table_bytes(n)) exceeds that size is rejected
 * with EWDG_ENOMEM before any work is queued.  Every call on a GPU shares
 * that GPU's table: calls that overlap on one GPU (from several host
 * threads, or on different streams whose work runs concurrently) race and
 * must be serialised by the caller.  Errors as ewdg_step_batch. */
int ewdg_static_table_max_bytes(size_t* bytes);
int ewdg_step_batch_static(ewdg_ctx* const* ctxs, int n, const double* dts, int nsteps, void* hip_stream);

/* ---------------------------------------------------------------- adjoint
 * Discrete adjoint of the fully discrete solve for the receiver misfit
 *     J = 1/2 dt sum_{n=1..nsteps} sum_r |v_h(x_r, t_n) - d_r(t_n)|^2
 * (traces after every step), with respect to per-element multipliers
 * theta_e = (s_rho, s_lambda, s_mu) of the quadrature-sampled fields at
 * theta = 1, i.e. g_e = dJ/d s applied to the current material (the
 * impedances follow the element means; dt is held fixed).  The adjoint is
 * the exact transpose of the discrete operator and of the LSRK(5,4)
 * recurrence, so g is the derivative of the computed J up to rounding.
 *
 * ewdg_adjoint_workspace_bytes: size of a second caller-owned workspace for
 * at most max_steps recorded steps with a checkpoint of (q, sigma_h) every
 * checkpoint_every = C steps; it holds ceil(max_steps/C) checkpoints and,
 * for the segment being reversed, the inputs of all 5 C stages with their
 * velocity right-hand sides: about (ceil(max_steps/C) + 6 C + 6) * 15 K Np
 * values in the run precision (memory is traded for recomputation: a
 * smaller C needs less).  Call
 * after ewdg_bind_workspace (the receiver capacity is taken from it);
 * binding the forward workspace again or a new mesh drops the binding.
 *
 * ewdg_adjoint_workspace_bytes_overlapped: the size of the same workspace
 * with a second segment buffer, about (ceil(max_steps/C) + 12 C + 7) * 15 K
 * Np values.  A workspace of at least this size, given to
 * ewdg_bind_adjoint_workspace, makes ewdg_adjoint_gradient recompute the next
 * segment on a second HIP stream (created by the library, default priority,
 * destroyed with the context) while the current one is reversed on the
 * context's stream; events order the two, and the result is bit-identical
 * to the single-buffer sweep.  Smaller workspaces run everything on the
 * context's stream. */
int ewdg_adjoint_workspace_bytes(const ewdg_ctx* ctx, int max_steps, int checkpoint_every, size_t* bytes);
int ewdg_adjoint_workspace_bytes_overlapped(const ewdg_ctx* ctx, int max_steps, int checkpoint_every,
                                            size_t* bytes);
int ewdg_bind_adjoint_workspace(ewdg_ctx* ctx, void* device_ptr, size_t bytes, int max_steps,
                                int checkpoint_every);
/* LTy_dev = L^T y (the transpose of ewdg_rhs's linear part in the plain
 * Euclidean product of nodal arrays [K][9][Np], context precision).  If
 * g_dev (FP64 [K][3], device) is given, q_dev is required and
 * g = y . d(L q + f(t))/d theta_e per element (rho, lambda, mu), computed
 * at the state q_dev.  Outputs are overwritten.  Needs the adjoint
 * workspace; does not change the stored state. */
int ewdg_rhs_adjoint(ewdg_ctx* ctx, double t, const void* q_dev, const void* y_dev, void* LTy_dev,
                     double* g_dev);
/* Run nsteps steps of size dt from the stored state exactly as ewdg_step
 * does, restarting the receiver record, checkpointing (q, sigma_h) every
 * checkpoint_every steps, and return J for data[nsteps][nr][3] (host,
 * FP64).  The stored state ends advanced by nsteps steps.  Changing the
 * material, the source or the receivers discards the recorded run. */
int ewdg_forward_misfit(ewdg_ctx* ctx, double dt, int nsteps, const double* data, double* J);
/* Reverse sweep over the run recorded by ewdg_forward_misfit: recomputes
 * each segment from its checkpoint, then applies the transposed stages
 * in reverse.  g receives dJ/dtheta as FP64 [K][3] (rho, lambda, mu);
 * qbar0, if not NULL, receives dJ/dq at the initial state ([K][9][Np],
 * context precision).  Either pointer may be host or device memory.
 * Synchronises. */
int ewdg_adjoint_gradient(ewdg_ctx* ctx, double* g, void* qbar0);

/* ---------------------------------------------------------- implicit step
 * Locally implicit time stepping (Sec. 4.3): the theta scheme
 *     (q^{m+1} - q^m)/dt = theta (L q^{m+1} + s^{m+1}) + (1 - theta)(L q^m + s^m)
 * of the same semi-discrete operator as ewdg_rhs (theta = 1: implicit Euler,
 * eq. implicitHDG of Sec. 4.3 written for this system; theta = 1/2:
 * Crank-Nicolson), solved by iHDG-II (Sec. 3, Algorithm 1).  Each iteration
 * solves every element's local equation (eq. iHDGlocal) with the interface
 * state (the weighted trace of eq. iHDGtrace) formed from the element's new
 * unknowns and its neighbours' previous iterate; elements are independent
 * within an iteration.  The initial guess is q^m; the loop stops at the
 * first iteration whose change ||q^k - q^{k-1}||_{L2(Omega)} (all nine
 * fields) is below tol (Sec. 6.1, the criterion without exact solution).
 *
 * ewdg_implicit_workspace_bytes: size of a third caller-owned workspace,
 * (K n^2 + 24 K Np) values of the run precision plus, in FP32, K n^2 FP64
 * values (n = 9 Np rounded up to 16: at N = 4, n = 320, 0.4 MB FP32 or
 * 0.8 MB FP64 per element for the stored local inverses) and 12 K bytes.
 * ewdg_bind_implicit_workspace: binds it (256-byte aligned device memory,
 * EWDG_ENOMEM if too small; after ewdg_bind_workspace; a new mesh or main
 * workspace drops the binding) and colours the face-adjacency graph.
 * ewdg_implicit_setup: forms B_k = I - theta dt A_k (A_k: the operator on the
 * element's own unknowns, probed column by column through the explicit
 * operator kernels) and inverts it in FP64 on the GPU; synchronises.  Needs
 * the material; setting material again requires a new set-up.  EWDG_EINVAL
 * if a pivot of the unpivoted elimination vanishes.
 * ewdg_implicit_step: nsteps steps of the dt and theta of the set-up from the
 * stored state and time (source and receivers as in ewdg_step), at most
 * max_iters iterations per step; iters[n] (host, may be NULL) receives the
 * iteration count of step n and change[n] (host, may be NULL) the final
 * change.  A step that reaches max_iters keeps its last iterate (compare
 * change with tol).  Synchronises once per iteration (the stopping test);
 * in FP32, tol must lie above the rounding level of the state (about
 * 1e-6 of its L2 norm).  ewdg_implicit_dt returns the set-up's dt and theta. */
int ewdg_implicit_workspace_bytes(const ewdg_ctx* ctx, size_t* bytes);
int ewdg_bind_implicit_workspace(ewdg_ctx* ctx, void* device_ptr, size_t bytes);
int ewdg_implicit_setup(ewdg_ctx* ctx, double dt, double theta);
int ewdg_implicit_step(ewdg_ctx* ctx, int nsteps, double tol, int max_iters, int* iters, double* change);
int ewdg_implicit_dt(const ewdg_ctx* ctx, double* dt, double* theta);

/* ------------------------------------------------------ steady transport
 * The paper's transport setting (Sec. 4.1, Sec. 6.1 Table 1): beta . grad u = f
 * on the unit square (dim 2) or cube (dim 3), u = g on the inflow boundary,
 * constant beta with nonzero components, a uniform grid of n^dim squares or
 * cubes, degree p in 1..4 (tensor-product space Q_p), upwind HDG (the trace
 * eliminated as in Sec. 4.1), solved by iHDG-II: each iteration solves every
 * element's local equation with its inflow faces' exterior traces from the
 * previous iterate (Theorem 1: the iteration marches the flow and is exact
 * after finitely many iterations).  u^0 = 0.
 *
 * Numbering: element e = i_0 + n i_1 + n^2 i_2 (grid indices along x, y, z);
 * volume points Q = q_0 + (p+3) q_1 + ... with q_a indexing the p+3 Gauss-
 * Legendre points along axis a; face 2a + side (side 0: x_a low, 1: high),
 * its points F indexing the Gauss points of the other axes in increasing
 * order, first fastest.
 *
 * ewdg_transport_create: EWDG_EINVAL for unsupported dim, p, n, precision or
 * a zero component of beta (dim values read).  Builds the reference
 * operators on the host (FP64).
 * ewdg_transport_sizes: E = n^dim elements, Np = (p+1)^dim coefficients,
 * Nq = (p+3)^dim volume and Nqf = (p+3)^(dim-1) face points per element.
 * ewdg_transport_points: physical points, host arrays xv [E][Nq][dim] and
 * xf [E][2 dim][Nqf][dim] (either may be NULL).
 * ewdg_transport_workspace_bytes / ewdg_transport_bind_workspace: caller-
 * owned device memory (256-byte aligned), about E (4 Np b + 2 Nq 8 + 2 dim
 * Nqf 8) bytes.
 * ewdg_transport_set_problem: host arrays f [E][Nq], g [E][2 dim][Nqf] (read
 * on the boundary inflow faces only) and, optionally, the exact solution ue
 * [E][Nq].  Forms c_e = A^-1 ((f, phi)_e - boundary inflow) in FP64 on the
 * GPU; synchronises.
 * ewdg_transport_solve: iterates from u^0 = 0 until the stopping rule of Sec.
 * 6.1 holds: with ue, | ||u^k - u^e|| - ||u^{k-1} - u^e|| | < tol (eq.
 * tolerancecriteria), without it ||u^k - u^{k-1}|| < tol (L2 norms over the
 * domain, the exact solution's by the volume-point rule), or max_iters.
 * iters (host) receives k; history (host, max_iters + 1 values, may be NULL)
 * the norm after every iteration, starting with ||u^0 - u^e|| (0 without
 * ue).  The stopping rule is evaluated on the GPU after every sweep;
 * iterations are queued in batches of 1, 2, 4, ... 32 with one
 * synchronisation per batch, and those queued after the stop do nothing.
 * EWDG_EINVAL (message "non-finite iterate") if a norm is not finite; the
 * history then ends with it.
 * ewdg_transport_values: the last iterate at the volume points, host
 * [E][Nq] FP64. */
typedef struct ewdg_tr ewdg_tr;
int ewdg_transport_create(int dim, int p, int n, const double* beta, int precision_bits, void* hip_stream,
                          ewdg_tr** out);
int ewdg_transport_destroy(ewdg_tr* tr);
int ewdg_transport_sizes(const ewdg_tr* tr, int64_t* E, int* Np, int* Nq, int* Nqf);
int ewdg_transport_points(const ewdg_tr* tr, double* xv, double* xf);
int ewdg_transport_workspace_bytes(const ewdg_tr* tr, size_t* bytes);
int ewdg_transport_bind_workspace(ewdg_tr* tr, void* device_ptr, size_t bytes);
int ewdg_transport_set_problem(ewdg_tr* tr, const double* f, const double* g, const double* ue);
int ewdg_transport_solve(ewdg_tr* tr, double tol, int max_iters, int* iters, double* history);
int ewdg_transport_values(ewdg_tr* tr, double* u);
const char* ewdg_transport_last_error(const ewdg_tr* tr);

const char* ewdg_last_error(const ewdg_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* EWDG_H */
