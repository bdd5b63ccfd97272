/*
 * ehdg.h -- C ABI of the MI355X (gfx950) eHDG solver library (libehdg.so).
 *
 * The method (Muralikrishnan, Tran, Bui-Thanh, "eHDG: an exponentially
 * convergent iterative solver for HDG discretizations of hyperbolic PDEs"):
 * every iteration solves one independent local problem per element, with the
 * face traces of the previous iterate as data (Algorithm 1, Section 3), and then
 * recomputes the traces from the new element solutions (eq. transportLocale for
 * transport; the trace formula below the shallow-water local solver for SWE).
 *
 * Supported problems (uniform axis-aligned meshes, constant coefficients unless set up
 * with ehdg_setup_variable, tensor Lagrange elements of degree p on Gauss-Lobatto-Legendre
 * nodes, Gauss-Legendre quadrature with p+2 points per direction):
 *   EHDG_TRANSPORT  beta . grad u + sigma u = f (steady) or its backward-Euler step
 *                   (Section 3, eq. transportLocal and the time-dependent paragraph)
 *   EHDG_SWE        linearized shallow water, backward Euler, 2D, Coriolis,
 *                   friction and wind stress zero (Section 3, linearizedShallow)
 *   EHDG_EULER      2D linearized Euler (rho', u', v', p') about a uniform state, backward
 *                   Euler: the same upwind HDG construction with the full |A_n|
 *                   (Section 3 notes the extension to other hyperbolic systems)
 *
 * Conventions shared by every entry point
 *   - Device pointers ("d_") are HIP device memory owned by the caller; host
 *     pointers are plain host memory.  The library never allocates device memory:
 *     all of its device state lives in the caller's workspace.
 *   - Element index e = i0 + n0 (i1 + n1 i2).  Node index a = a0 + (p+1) a1 +
 *     (p+1)^2 a2 over ascending GLL coordinates.  Faces 0..5 = x-, x+, y-, y+, z-, z+.
 *     Face nodes are ordered by the tangential node indices in increasing axis
 *     order, first tangential axis fastest.
 *   - External solution layout: double u[n_el][m][N_p] (m fields: transport 1;
 *     SWE 3 = phi, u, v; Euler 4 = rho', u', v', p').
 *   - Every function returns 0 (EHDG_OK) or one of the EHDG_ERR_* codes; no call
 *     aborts the process.  ehdg_last_error() gives a message for the handle.
 *   - All work is queued on the HIP stream given at setup.  Asynchronous calls
 *     report launch errors only; ehdg_solve / ehdg_step synchronize that stream.
 *   - Calls on one handle must not overlap; distinct handles are independent.
 */
#ifndef EHDG_H
#define EHDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  EHDG_OK = 0,
  EHDG_ERR_INVALID_ARG = 1,        /* bad pointer, size or descriptor field          */
  EHDG_ERR_UNSUPPORTED = 2,        /* valid problem this build does not implement    */
  EHDG_ERR_HIP = 3,                /* a HIP runtime call failed                      */
  EHDG_ERR_NOT_CONVERGED = 4,      /* iteration cap reached; outputs are valid       */
  EHDG_ERR_DIVERGED = 5,           /* residual became non-finite                     */
  EHDG_ERR_WORKSPACE_TOO_SMALL = 6 /* workspace smaller than ehdg_workspace_bytes()  */
};

enum { EHDG_TRANSPORT = 0, EHDG_SWE = 1, EHDG_EULER = 2 };

/* Arithmetic of the element sweeps.
 *   EHDG_FP64          every sweep in FP64.
 *   EHDG_FP32_REFINE   the local operator is applied in FP32 to a correction;
 *                      an FP64 residual of the fixed-point equation, its norm and
 *                      the update of the iterate stay in FP64 on the GPU.
 *   EHDG_BF16_REFINE   as above with BF16 operands on MFMA (FP32 accumulation).
 *   EHDG_FP32          plain sweeps in FP32: traces, g and the condensed operator in
 *                      FP32 (matrix cores, FP32 accumulation); only the increment norms
 *                      of the stopping test are accumulated in FP64.  The element
 *                      solution is recovered in FP64 from the FP32 traces.  Its result
 *                      differs from the FP64 fixed point by FP32 rounding of the operator,
 *                      data and traces (about 1e-6 relative): a rel_tol below about 1e-7
 *                      buys no accuracy (the rounded iteration stalls there, or reaches an
 *                      exact fixed point of the rounded map).  Not in batches.
 * With s inner sweeps per refinement and exact arithmetic, one refinement equals
 * s plain sweeps (the method is linear; Section 3, reduction to the homogeneous
 * problem). */
enum { EHDG_FP64 = 0, EHDG_FP32_REFINE = 1, EHDG_BF16_REFINE = 2, EHDG_FP32 = 3 };

typedef struct {
  int32_t pde;          /* EHDG_TRANSPORT, EHDG_SWE or EHDG_EULER                     */
  int32_t dim;          /* 2 or 3 (SWE, Euler: 2)                                    */
  int32_t n[3];         /* elements per axis (unused axes ignored), each >= 1        */
  double L[3];          /* domain [0, L_a] per axis, L_a > 0                          */
  int32_t periodic[3];  /* 1 = periodic axis; 0 = boundary: transport inflow data /
                           outflow; SWE reflecting wall; Euler no incoming waves     */
  int32_t degree;       /* p: transport 2D 1..6, 3D 1..4; SWE 1..6; Euler 1..5.
                           2D transport of degree 1 with both velocity components
                           non-zero returns UNSUPPORTED: its kernels are switched off
                           while a device failure recorded against them is unexplained */
  double beta[3];       /* transport velocity (components may be 0)                  */
  double sigma;         /* transport reaction coefficient, >= 0                       */
  double Phi;           /* SWE mean geopotential, > 0                                 */
  double U0[2];         /* Euler mean velocity; no face may see a zero wave speed:
                           U0_a != 0 and |U0_a| != c0 on every axis                   */
  double c0;            /* Euler sound speed, > 0                                     */
  double rho0;          /* Euler mean density, > 0                                    */
  double dt;            /* backward-Euler step; 0 = steady (transport only)           */
  int32_t precision;    /* EHDG_FP64 / EHDG_FP32_REFINE / EHDG_BF16_REFINE / EHDG_FP32 */
  int32_t inner_sweeps; /* low-precision sweeps per FP64 refinement (refine modes)    */
} ehdg_desc;

typedef struct ehdg_problem* ehdg_handle;

/* Reference points used by the discretization, for callers that sample data.
 * gll_nodes[p+1] (ascending, on [-1,1]); gauss_pts[p+2], gauss_wts[p+2]. Host memory.
 * Any pointer may be NULL.  Forcing is sampled at the tensor Gauss points of each
 * element, boundary data at the face GLL nodes, initial states at the GLL nodes. */
int ehdg_reference_points(int32_t degree, double* gll_nodes, double* gauss_pts, double* gauss_wts);

/* Device workspace (bytes) needed by ehdg_setup for this descriptor. */
int ehdg_workspace_bytes(const ehdg_desc* desc, size_t* bytes);

/* Builds the local operators on the host (FP64), uploads them into the caller's
 * workspace (aligned to 256 bytes, at least ehdg_workspace_bytes()) on `stream`
 * (a hipStream_t, NULL = default stream) and returns a handle.  The workspace must
 * stay valid until ehdg_destroy.  State after setup: zero forcing, zero boundary
 * data, zero initial state. */
int ehdg_setup(const ehdg_desc* desc, void* d_workspace, size_t workspace_bytes, void* stream,
               ehdg_handle* out);

/* Transport with a velocity field beta(x): the steady problems of Sections 4.1-4.3
 * (beta = (y, x); beta = (1 + sin(pi y / 2), 2) with discontinuous inflow data;
 * beta = (z, x, y)).  The local equation is the one of eq. transportLocal with beta
 * inside the integrals,
 *   A_e = -(psi_j, div(beta psi_i))_K + sum_f <(beta.n + |beta.n|) psi_j, psi_i>_f + sigma (psi_j, psi_i)_K,
 * lifts <|beta.n| mu_a, psi_i>_f, and the upwind trace of eq. transportLocale.  Every
 * element has its own operator: setup builds A_e, its inverse and T_e = Q A_e^{-1} L_e
 * per element on the host, all integrals by the p+2 point Gauss rule, and the sweep
 * streams T_e from the workspace.
 * Requirement: on the faces normal to axis a, beta_a has one strict sign at every face
 * Gauss point (or is 0 at all of them: the axis carries no transport); then the upwind
 * side of every face is fixed and the trace is the upwind element's face values, as
 * for a constant velocity.  Otherwise UNSUPPORTED.
 * desc: pde = EHDG_TRANSPORT, dt = 0, precision = EHDG_FP64 (else UNSUPPORTED); beta[]
 * is ignored.  Velocity samples, HOST memory, read during the call only:
 *   beta_q     double [n_el][dim][(p+2)^dim]: beta at the tensor Gauss points (point
 *              order as d_forcing_q of ehdg_set_forcing)
 *   div_beta_q double [n_el][(p+2)^dim]: div beta there, or NULL for 0
 *   beta_face  double [n_el][2 dim][(p+2)^(dim-1)]: on face f (order x-, x+, y-, ...),
 *              the component beta_(f/2) at the face's tensor Gauss points (tangential
 *              axes in increasing order, first fastest)
 * Boundary data (ehdg_set_forcing d_bc) are the nodal values of the inflow trace in the
 * face space (for non-polynomial g, e.g. its L2 projection on each face).
 * ehdg_variable_workspace_bytes gives a size that fits every velocity on the mesh.  The
 * handle takes every call of a steady FP64 handle; batches return UNSUPPORTED for it. */
int ehdg_variable_workspace_bytes(const ehdg_desc* desc, size_t* bytes);
int ehdg_setup_variable(const ehdg_desc* desc, const double* beta_q, const double* div_beta_q,
                        const double* beta_face, void* d_workspace, size_t workspace_bytes, void* stream,
                        ehdg_handle* out);

/* Problem data (Section 3 local equations' right-hand sides).
 *   d_forcing_q: right-hand side of each field's equation sampled at the tensor Gauss
 *                points, double [n_el][m][(p+2)^dim] with point q = q0 + (p+2) q1 +
 *                (p+2)^2 q2 (axis 0 fastest), or NULL for zero.  For SWE the momentum
 *                rows are the equations multiplied by Phi.
 *   d_bc:        transport inflow boundary data g at the boundary-face GLL nodes, or
 *                NULL for zero.  Layout: sides x-, x+, y-, y+, z-, z+ of the
 *                non-periodic axes concatenated; within a side, faces ordered by the
 *                tangential element indices (first tangential axis fastest), each face
 *                holding its (p+1)^(dim-1) nodes in face-node order.  Only inflow sides
 *                (beta . n < 0) are read.  Size: sum over non-periodic sides of
 *                (faces on the side) * (p+1)^(dim-1) doubles.
 * May be called again between steps; the current iterate is kept. */
int ehdg_set_forcing(ehdg_handle h, const double* d_forcing_q, const double* d_bc);

/* Initial state u^0 (external layout [n_el][m][N_p]) or NULL for zero.  Steady
 * problems: initial guess of Algorithm 1.  Backward Euler: the solution at the
 * current time level.  Recomputes the initial traces and resets the iteration count. */
int ehdg_set_initial(ehdg_handle h, const double* d_u0);

/* Asynchronous: exactly n_iters sweeps of Algorithm 1 (local solves + new traces),
 * with no stopping test.  Each sweep's relative trace increment
 * ||s^{k+1} - s^k||_2 / ||s^{k+1}||_2 is recorded (ehdg_get_residuals). */
int ehdg_iterate(ehdg_handle h, int32_t n_iters);

/* Synchronous: Algorithm 1 run to convergence.  Sweeps (step 2: the local equations
 * eq. transportLocalk1 / the shallow-water local solver; step 3: new traces by eq.
 * transportLocale / the shallow-water trace formula) until the convergence check of
 * step 4 holds: the relative trace increment ||s^{k+1} - s^k||_2 / ||s^{k+1}||_2 is
 * below rel_tol (the paper leaves the check's norm open; this one is evaluated on the
 * device after every sweep).  Then recovers the element solution from the last local
 * solve.  *iters = local solves performed in this call (the initial trace of the
 * algorithm's first line is not counted); *rel_res = the last increment.  Returns
 * EHDG_ERR_NOT_CONVERGED after max_iters sweeps (outputs valid), EHDG_ERR_DIVERGED if
 * the increment became non-finite.  Backward-Euler handles: solves the current step's
 * system (use ehdg_step to advance in time). */
int ehdg_solve(ehdg_handle h, double rel_tol, int32_t max_iters, int32_t* iters, double* rel_res);

/* Synchronous: n_steps backward-Euler steps.  Each step is the steady iteration with the
 * extra L2 term of the time-dependent paragraph of Section 3 (M/dt in the local operator,
 * M u^m / dt in the right-hand side), solved to rel_tol as in ehdg_solve, starting from
 * the previous step's traces: the warm start of Section 4.4, which keeps the count per
 * step small.  After a step converges its element solution becomes u^{m+1}.
 * iters_per_step: host int32_t[n_steps] or NULL; entries of steps not completed are 0.
 * Returns EHDG_ERR_NOT_CONVERGED if a step reached max_iters_per_step (the completed
 * steps stand), EHDG_ERR_DIVERGED on a non-finite increment.  Any n_steps >= 0 is
 * accepted (counts are read back batch by batch, so none is lost to the device ring). */
int ehdg_step(ehdg_handle h, int32_t n_steps, double rel_tol, int32_t max_iters_per_step,
              int32_t* iters_per_step);

/* Asynchronous: the element solution of the current iterate into d_u [n_el][m][N_p]:
 * u^{k+1} of Algorithm 1, i.e. the last local solve (eq. transportLocalk1 with the
 * traces it read), or the initial / current time level's state if no sweep ran since.
 * Recovering it costs one element-local solve; the sweeps themselves only carry traces. */
int ehdg_get_solution(ehdg_handle h, double* d_u);

/* Synchronous: residual history of sweeps [first, first+count) since the last
 * ehdg_set_initial or time step, into host memory.  Returns INVALID_ARG if out of range. */
int ehdg_get_residuals(ehdg_handle h, int32_t first, int32_t count, double* out);

/* Sizes of the handle's problem (host pointers, any may be NULL): element count,
 * fields m, nodes per element N_p, trace-state values per element S, gathered
 * inputs per element I, sweeps completed since the last reset. */
int ehdg_sizes(ehdg_handle h, int64_t* n_el, int32_t* m, int32_t* n_p, int32_t* s, int32_t* i,
               int32_t* iters);

/* Checkpoint / resume.  The state is the double-buffered traces, the iteration
 * count and the current time-level solution.  ehdg_state_bytes gives its size;
 * get/set copy it to/from caller device memory on the handle's stream. */
int ehdg_state_bytes(ehdg_handle h, size_t* bytes);
int ehdg_get_state(ehdg_handle h, void* d_dst, size_t bytes);
int ehdg_set_state(ehdg_handle h, const void* d_src, size_t bytes);

/* Launch shapes of the plain sweeps (EHDG_FP64, EHDG_FP32), for a tuner.  The sweep applies
 * the condensed operator to tiles of 16 elements; a launch gives each workgroup a range of
 * tiles.  ehdg_tune_set registers, for the problems with this (pde, dim, degree, precision)
 * set up afterwards in this process, the tiles per workgroup (0: as many as one round of
 * resident workgroups needs, the default; > 0: that many, rounded up to the tiling's step,
 * in as many rounds as it takes) and the order in which the workgroups take their ranges
 * (reverse_order != 0: reversed).  tiles_per_group = 0 with reverse_order = 0 removes the
 * entry; ehdg_tune_clear removes all.  The shape changes how the increment norms are summed
 * (per workgroup, then in a fixed order), not the iterates: each element's local solve is
 * the same arithmetic in any shape.  Batches use each member's shape.
 * ehdg_tune_set returns INVALID_ARG for tiles_per_group < 0 and for the refinement
 * precisions (their kernels keep their own shapes).  ehdg_launch_shape reports a handle's
 * shape; UNSUPPORTED for variable velocity. */
int ehdg_tune_set(int32_t pde, int32_t dim, int32_t degree, int32_t precision, int32_t tiles_per_group,
                  int32_t reverse_order);
int ehdg_tune_clear(void);
int ehdg_launch_shape(ehdg_handle h, int32_t* tiles_per_group, int32_t* groups, int32_t* reverse_order);

/* Releases the host-side handle (the workspace stays the caller's). */
int ehdg_destroy(ehdg_handle h);

/* ---- Batches of independent problems ------------------------------------------
 * Algorithm 1 treats every element independently, so a set of unrelated problems is
 * one bigger set of independent local solves.  A batch advances many problems (any
 * PDE, degree, mesh and coefficients, precision EHDG_FP64 or EHDG_FP32) together, and each
 * problem keeps its own control block, stopping test and residual history.  A round of
 * sweeps is one launch per operator family and precision over a (problem, tile range)
 * table, or (ehdg_batch_set_persistent) one persistent launch per precision for every 2D
 * transport and shallow-water member, a grid of resident workgroups striding over the
 * table and dispatching each entry to its family's sweep; backward-Euler step completions
 * are one launch per family.  The rounds are captured once into a HIP graph and replayed
 * (ehdg_batch_set_graph).  A problem's iterates, iteration counts and solution are bit for
 * bit those of the same handle advanced alone.
 *
 * handles: host array of n handles (from ehdg_setup, FP64 or FP32 precision), all distinct;
 * the batch keeps pointers to them, so they must outlive it, and no call on a member
 * handle may overlap a batch call.  The workspace (device memory, 256-byte aligned,
 * at least ehdg_batch_workspace_bytes) holds the problem table; it stays the caller's.
 * Work is queued on `stream` (NULL = default).  Returns UNSUPPORTED for a handle in a
 * refinement precision or with a variable velocity, INVALID_ARG for a repeated or null
 * handle. */
typedef struct ehdg_batch_s* ehdg_batch;
int ehdg_batch_workspace_bytes(const ehdg_handle* handles, int32_t n, size_t* bytes);
int ehdg_batch_create(const ehdg_handle* handles, int32_t n, void* d_workspace, size_t workspace_bytes,
                      void* stream, ehdg_batch* out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops that rebuild batches as members come and go, harnesses that forbid
 * hipMalloc): ehdg_batch_create without a workspace.  The batch's tables (problem
 * descriptors, workgroup table, control-block copies: what ehdg_batch_workspace_bytes
 * sizes) go into a static device array of the library, 8 MiB per GPU, held until the
 * process ends; the call allocates no device memory.  The array of the current device is
 * used (call with the members' device current).  Returns EHDG_ERR_WORKSPACE_TOO_SMALL if
 * the tables need more than 8 MiB (ehdg_batch_workspace_bytes > 8 MiB; use
 * ehdg_batch_create then), else as ehdg_batch_create.  One array per device means one
 * static batch per device at a time: creating a static batch replaces the tables of
 * the previous static batch on that device, whose later calls return
 * EHDG_ERR_INVALID_ARG (destroy it as usual).  Calls that overlap on one device race on
 * the array. */
int ehdg_batch_create_static(const ehdg_handle* handles, int32_t n, void* stream, ehdg_batch* out);

/* Synchronous: ehdg_solve for every member (each to rel_tol, at most max_iters sweeps,
 * then its recovery).  iters, rel_res: host arrays of n, or NULL.  Returns the first
 * non-OK member status in handle order (NOT_CONVERGED / DIVERGED), else OK. */
int ehdg_batch_solve(ehdg_batch b, double rel_tol, int32_t max_iters, int32_t* iters, double* rel_res);

/* Synchronous: ehdg_step(n_steps) for every member (all must be backward-Euler).
 * iters_per_step: host array [n][n_steps] (member-major), or NULL. */
int ehdg_batch_step(ehdg_batch b, int32_t n_steps, double rel_tol, int32_t max_iters_per_step,
                    int32_t* iters_per_step);

/* Asynchronous work, synchronous report: `rounds` rounds for every member, each one
 * sweep (stopping test at rel_tol) and, for backward-Euler members, a step completion.
 * Steady members stop at convergence.  Backward-Euler member i stops once it has
 * completed step_targets[i] steps since its last ehdg_set_initial (NULL: one more step
 * than it had completed when the call started).  Meant for serving loops that change the
 * batch between calls: a member's state lives in its own workspace, so it continues
 * where it stopped.  state: host array of n, 0 running, 1 finished (converged / took its
 * steps), 2 non-finite increment.  ehdg_get_solution then gives a finished member's
 * result. */
int ehdg_batch_advance(ehdg_batch b, int32_t rounds, double rel_tol, const int32_t* step_targets, int32_t* state);

/* Asynchronous rounds with a report per launch, for serving loops that keep the GPU busy
 * while they admit and retire problems.
 *
 * ehdg_batch_launch queues `rounds` rounds (as ehdg_batch_advance; step_targets is
 * required when the batch has backward-Euler members), then a copy of every member's
 * control block into h_report, and returns without waiting.  h_report: host memory of at
 * least ehdg_batch_report_bytes, pinned (hipHostMalloc; pageable memory makes the copy,
 * and so the call, wait for the rounds), owned by the caller, left untouched until the
 * launch's report is read, and not shared with another pending launch.  At most four
 * launches may be pending; INVALID_ARG beyond that.
 *
 * ehdg_batch_poll reads the oldest pending launch's report if its work has completed:
 * *ready = 1, state[] (host array of n, or NULL) as ehdg_batch_advance gives it, and
 * the members' host-side control-block copies refreshed; else *ready = 0 without waiting.
 * INVALID_ARG when no launch is pending.
 *
 * ehdg_batch_get_solution queues on the batch's stream the solution of a member that the
 * last report read showed finished (state 1; INVALID_ARG otherwise) into d_u (device,
 * layout as ehdg_get_solution); later rounds leave a finished member unchanged, so this
 * may follow pending launches.  Asynchronous.
 *
 * Ordering: every batch call queues its work after what the members' own streams hold at
 * the call (the batch stream waits on an event recorded there; static batches wait on the
 * host).  ehdg_batch_solve, _step and _advance return INVALID_ARG while launches are
 * pending.  ehdg_batch_destroy waits for the batch's own queued work. */
int ehdg_batch_report_bytes(ehdg_batch b, size_t* bytes);
int ehdg_batch_launch(ehdg_batch b, int32_t rounds, double rel_tol, const int32_t* step_targets, void* h_report,
                      size_t report_bytes);
int ehdg_batch_poll(ehdg_batch b, int32_t* state, int32_t* ready);
int ehdg_batch_get_solution(ehdg_batch b, int32_t member, double* d_u);

/* Rounds as a captured HIP graph (enabled != 0, the default for ehdg_batch_create) or as
 * launches queued one by one (0).  The graph is captured on a private stream of the batch
 * and replayed on the batch's stream; a caller's stream that is itself being captured gets
 * plain launches.  Static batches (ehdg_batch_create_static) have no graphs (enabling
 * returns UNSUPPORTED): instantiating a graph allocates. */
int ehdg_batch_set_graph(ehdg_batch b, int32_t enabled);

/* Sweeps of the 2D transport and shallow-water members in the persistent launch (enabled
 * != 0) or in one launch per family like the other families (0, the default, faster on
 * mixed batches: each family's kernel keeps its own register budget and occupancy).
 * Every member gets the same work either way, so the results are bitwise the same.
 * INVALID_ARG while launches are pending. */
int ehdg_batch_set_persistent(ehdg_batch b, int32_t enabled);

int ehdg_batch_destroy(ehdg_batch b);
const char* ehdg_batch_last_error(ehdg_batch b);

const char* ehdg_error_string(int code);
const char* ehdg_last_error(ehdg_handle h);

#ifdef __cplusplus
}
#endif

#endif /* EHDG_H */
