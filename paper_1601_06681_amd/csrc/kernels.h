// Device-side data of one eHDG problem and the kernel entry points (host view).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace ehdg {

// Elements per workgroup (one per lane of a wavefront) and wavefronts per
// workgroup; each wavefront applies a block of ceil(rows / kRowGroups) operator rows,
// so operators are stored with their row count padded to a multiple of kRowGroups.
constexpr int kElemsPerGroup = 64;
constexpr int kRowGroups = 4;
inline int padded_rows(int rows) { return (rows + kRowGroups - 1) / kRowGroups * kRowGroups; }

// FP64 sweeps run on the matrix cores (v_mfma_f64_16x16x4f64): the S x I operator is
// cut into 16 x 4 fragments held in registers, stored fragment-major so that a
// wavefront loads fragment (mt, kt) as one contiguous 512-byte run:
//   Tf[(mt * KT + kt) * 64 + lane] = T[16 mt + lane % 16][4 kt + lane / 16]  (0 outside S x I).
// Elements are processed in tiles of 16 (one per matrix column).
constexpr int kMfmaTileElems = 16;
inline int mfma_row_tiles(int rows) { return (rows + 15) / 16; }
inline int mfma_k_tiles(int cols) { return (cols + 3) / 4; }

// Arrival counters of the last-workgroup reductions: two sets (sweep reduction, step
// completion) of kCounterGroups group counters plus one counter of finished groups,
// each on its own 256 bytes so that concurrent arrivals do not queue on one line.
// (Measured on the 256^2 shallow-water sweep: 8 groups 12.1 us, 32 groups 11.5 us,
// 128 groups 13.1 us; 4 KB apart instead of 256 bytes, 11.8 us.)
constexpr int kCounterGroups = 32;
constexpr int kCounterStride = 64;  // unsigned ints
constexpr int kCounterSet = (kCounterGroups + 1) * kCounterStride;
constexpr size_t kCounterBytes = 2 * (size_t)kCounterSet * sizeof(unsigned);

// Device-resident iteration control, one per handle.  Kernels choose their
// buffers from it, so work can be queued ahead of the host knowing when a solve
// converges: the trace state after k sweeps (or refinements) of the current
// segment is in s[(base + k) & 1]; the current time level's solution is u[ucur].
struct Ctrl {
  // the first four fields are read together by every sweep (one 16-byte load)
  int done;           // set once the stopping test holds (or the increment is non-finite)
  int iters;          // sweeps (or refinements) of the current segment whose increment is known
  int base;           // state buffer holding s^0 of the current segment
  int status;         // 0 running, 1 converged, 2 non-finite increment
  unsigned seg_seq;   // FP64 sweeps: launch number of the sweep before the segment's first
  int ucur;           // solution buffer holding the current time level
  int steps_done;     // backward-Euler steps completed since the last initial state
  unsigned applied;   // refinement forms: stamp of the last correction sweep that also
                      // stored s' = s + correction (the next refinement finds it in place)
  double last_res;    // last relative increment
  double pad[3];
};
static_assert(sizeof(Ctrl) == 64, "Ctrl is one 64-byte block");

// Mesh indexing shared by every kernel.
struct MeshDev {
  int nel;
  int n[3];
  int periodic[3];
  int ax[3];   // transport: active axes
  int dir[3];  // transport: +1 if beta_ax > 0 (upwind neighbour at i-1), -1 otherwise
  int order;   // plain sweeps: 1 = workgroups take their tile ranges in reverse order (tuning)
};

// All device pointers of a problem (SoA: component k of element e at [k * nel + e]).
struct DevProblem {
  MeshDev mesh;
  int pde, dim, nf, S, I, n, m, Np, na;
  bool be;
  const double* T64;       // S x I
  const double* Tf64;      // fragment-major T for the matrix-core sweep
  const float* Tf32;       // the same in FP32
  const float* T32;        // S x I
  const uint16_t* T16;     // S x I (bf16 bits)
  const double* R;         // n x I
  const double* P;         // n x n (BE)
  const double* G;         // S x n (BE)
  const double* Mvol;      // recovery: steady R (n x I); BE [[P, R], [G P, G R]]; rows padded
  const double* Mf64;      // fragment-major Mvol for the matrix-core step completion
  double* gbe;             // BE source part of the next g: g_src + G w_src  (S)
  bool has_src;            // forcing or boundary data present (w_src, g_src nonzero)
  double* s[2];            // trace state, double buffered
  double* g;               // S
  float* g32;              // S: g in FP32 (plain FP32 precision only)
  double* g_src;           // S
  double* w_src;           // n
  double* u2[2];           // n: solution buffers; u2[ucur] is the current time level
  int* step_iters;         // sweeps per completed backward-Euler step (ring)
  int step_cap;
  void* lo[2];             // low-precision correction, double buffered (S)
  void* rlo[2];            // low-precision residual, double buffered (S)
  double* partials;        // per workgroup (d2, n2); FP64 sweeps: two sets, partial_stride apart
  int partial_stride;      // doubles between the two sets
  int nb_sweep;            // workgroups of one plain sweep launch
  int sweep_tpg;           // tiles per workgroup of the plain sweeps (0: one round of resident
                           // workgroups; > 0: the tuned value, rounded to the tiling's step)
  Ctrl* ctrl;
  unsigned* counters;      // kCounterBytes: arrival counters (zero between launches)
  double* hist;            // residual ring
  int hist_cap;
  // variable velocity: per-element operators.  T_e tile-major (element e = 16 t + j:
  // Tv[((t * I + c) * S + r) * 16 + j], tiles padded with zeros), R_e entry-major with
  // the element index fastest (Rv[(c * N_p + r) * nel + e]), and room for the gathered
  // inputs of every element (I x nel)
  const double* Tv;
  const double* Rv;
  double* in_scratch;
};

// One problem of a batch as the batched kernels see it (device memory, one per problem).
struct BatchProblem {
  MeshDev mesh;
  int steps_target;        // the batched step stops a problem after this many completed steps
  int hist_cap, step_cap;
  const double* Tf64;      // fragment-major operators
  const double* Mf64;
  const float* Tf32;       // plain FP32 members: FP32 fragments, g in FP32 (the state buffers
  float* g32;              // s0, s1 then hold floats); null for FP64 members
  const double* g;
  double* s0;
  double* s1;
  double* u0;
  double* u1;
  const double* w_src;     // null: no forcing / boundary data
  const double* gbe;       // null: no forcing / boundary data
  Ctrl* ctrl;
  unsigned* counters;
  double* partials;
  double* hist;
  int* step_iters;
};

// One workgroup of a batched launch: its problem, its index among that problem's
// workgroups, their number, and the 16-element tiles each of them takes.
struct BatchEntry {
  int problem, block, nblocks, tiles_per_group;
  int family;  // persistent batched sweeps: the family's code (KernelSet::persist)
};

// The persistent batched sweep: one launch per precision covers every entry of every
// family whose code is >= 0; a grid of resident workgroups strides over the n entries
// (entry i on workgroup i mod grid), each entry doing the work of one workgroup of that
// family's own batched sweep (so results are bitwise those of the per-family launch).
void launch_sweep_persist(const BatchEntry* table, int n, const BatchProblem* probs, double tol, int fp32,
                          hipStream_t st);

// Kernels of one (pde, dim, active axes, face nodes) family.
struct KernelSet {
  // one FP64 sweep s^{k+1} = g + T in(s^k), launch number seq (the host numbers every
  // sweep of a handle), buffers from the control block and seq.  The stopping test of
  // the previous sweep is taken at the start (tol < 0: record only, never stop); this
  // sweep's own increment is left as partial sums for the next launch (or
  // launch_reduce_lagged)
  void (*sweep64)(const DevProblem&, double tol, unsigned seq, hipStream_t);
  // element solution u_out = w_src + R in(s_prev) (+ P u_old for BE); no control change
  void (*volume)(const DevProblem&, const double* s_prev, const double* u_old, double* u_out, hipStream_t);
  // backward-Euler step completion, queued after a step's sweeps: if the step has
  // converged, u[ucur^1] = solution of the last local solve (lag 1: it read
  // s^{K-1}; lag 0: refinement, it reads s^K), next g, and the control block
  // advances to the next step; otherwise nothing happens.  lagged (FP64 sweeps): the
  // last sweep's increment is still pending and is tested here against tol; seq_next
  // is the launch number the next sweep will get
  void (*step)(const DevProblem&, int lag, unsigned seq_next, double tol, int lagged, hipStream_t);
  // mixed precision outer step: s' = s^k + lo_in (lo_in ignored on the segment's
  // first refinement); r = g + T in(s') - s' in FP64 into r_out (low precision);
  // s' stored as s^{k+1}; reduction of ||r|| / ||s' + r||.  stamp != 0: if the control
  // block's `applied` equals it, s' is already in place (the previous correction sweep
  // stored it) and only r and the reduction remain
  void (*refine32)(const DevProblem&, const void* lo_in, void* r_out, double tol, unsigned stamp, hipStream_t);
  // inner sweep on the correction: lo_out = r_lo + T_lo in(lo_in).  stamp != 0 (the last
  // sweep of a refinement): where the family's refinement applies the correction in a
  // pass of its own, this sweep stores s' = s + lo_out in its place (not lo_out) and sets
  // the control block's `applied` to stamp; elsewhere stamp is ignored
  void (*inner32)(const DevProblem&, const void* r_lo, const void* lo_in, void* lo_out, unsigned stamp,
                  hipStream_t);
  void (*refine16)(const DevProblem&, const void* lo_in, void* r_out, double tol, unsigned stamp, hipStream_t);
  void (*inner16)(const DevProblem&, const void* r_lo, const void* lo_in, void* lo_out, unsigned stamp,
                  hipStream_t);
  // workgroups of the FP64 sweep / step completion for n_el elements (the same shape a
  // single problem launches with, so batched and single results agree bit for bit);
  // sweep_groups takes a tuned tiles-per-workgroup in *tiles_per_group (0: default)
  void (*sweep_groups)(int nel, int* tiles_per_group, int* groups);
  void (*step_groups)(int nel, int* tiles_per_group, int* groups);
  // one FP64 sweep / one step completion of every problem of a batch that uses this
  // family: n entries of table, problems in probs (device memory)
  void (*sweep64_batch)(const BatchEntry* table, int n, const BatchProblem* probs, double tol, hipStream_t);
  void (*step_batch)(const BatchEntry* table, int n, const BatchProblem* probs, int lag, hipStream_t);
  // plain FP32 form: the sweep s^{k+1} = g + T in(s^k) on FP32 state and g (FP32
  // matrix cores), with the FP64 increment norms and the lagged stopping test of the
  // FP64 sweep (same partial sets and launch numbering; the state buffers s[0], s[1]
  // hold floats); recovery and step completion read the FP32 state (FP64 arithmetic,
  // the next g written in FP32 to g32)
  void (*sweep32)(const DevProblem&, double tol, unsigned seq, hipStream_t);
  void (*volume32)(const DevProblem&, const float* s_prev, const double* u_old, double* u_out, hipStream_t);
  void (*step32)(const DevProblem&, int lag, unsigned seq_next, double tol, int lagged, hipStream_t);
  void (*sweep32_groups)(int nel, int* tiles_per_group, int* groups);
  // batches of plain FP32 members: the FP32 sweep (arrival-based test) and step completion
  void (*sweep32_batch)(const BatchEntry* table, int n, const BatchProblem* probs, double tol, hipStream_t);
  void (*step32_batch)(const BatchEntry* table, int n, const BatchProblem* probs, int lag, hipStream_t);
  // code of the family in the persistent batched sweep, -1 if it is not covered there
  int persist;
};

const KernelSet* find_kernels(int pde, int dim, int na, int nf);

// Variable-velocity transport sweep: a wavefront takes 16 elements and a block of
// 4 * var_rows_per_lane(S) operator rows (lane l: element l % 16, rows l / 16 + 4 k);
// workgroups of 4 wavefronts.
inline constexpr int var_row_blocks(int S) { return (S + 11) / 12; }
inline constexpr int var_rows_per_lane(int S) {
  return (S + 4 * var_row_blocks(S) - 1) / (4 * var_row_blocks(S));
}
inline long long var_sweep_groups(long long nel, int S) {
  return ((nel + kMfmaTileElems - 1) / kMfmaTileElems * var_row_blocks(S) + 3) / 4;
}
// Kernels of variable-velocity transport (sweep64 and volume; the rest null).
const KernelSet* find_var_kernels(int dim, int na, int p);

// Generic setup-time kernels (FP64, runtime sizes).
// y[r][e] = (accumulate ? y[r][e] : 0) + sum_c M[r][c] x[c][e]
void launch_matvec(const double* M, int rows, int cols, const double* x, double* y, int nel, bool accumulate,
                   hipStream_t st);
// per-element operators: y[r][e] = (accumulate ? y[r][e] : 0) + sum_c M[(c * rows + r) * nel + e] x[c][e]
void launch_matvec_pe(const double* M, int rows, int cols, const double* x, double* y, int nel, bool accumulate,
                      hipStream_t st);
// SoA [K][nel] <-> external [nel][K]
void launch_ext_to_soa(const double* ext, double* soa, int K, int nel, hipStream_t st);
void launch_soa_to_ext(const double* soa, double* ext, int K, int nel, hipStream_t st);
void launch_fill(double* p, double v, size_t count, hipStream_t st);
void launch_fill_bytes(void* p, size_t bytes, hipStream_t st);
// transport boundary inputs: in_bc[c][e] (I rows) from the compact side layout
void launch_bc_inputs(const DevProblem& dp, const double* bc, double* in_bc, hipStream_t st);
// full = 1: everything (new initial state); full = 0: start a new segment from the
// latest state; full = 2: the same, but only if the current segment has finished.
// seq_next: the launch number of the next FP64 sweep
void launch_ctrl_reset(Ctrl* c, int full, unsigned seq_next, hipStream_t st);
// the stopping test of the last FP64 sweep before launch number seq (its increment
// pending as partial sums), as the sweep launched as seq would take it
void launch_reduce_lagged(const DevProblem& dp, double tol, unsigned seq, hipStream_t st);
void launch_counters_reset(unsigned* counters, hipStream_t st);
// the same reset for every problem of a batch, and a copy of their control blocks into out[n]
void launch_ctrl_reset_batch(const BatchProblem* probs, int n, int full, hipStream_t st);
void launch_ctrl_gather(const BatchProblem* probs, int n, Ctrl* out, hipStream_t st);
void launch_cast(const double* src, void* dst, size_t count, int to_bf16, hipStream_t st);

}  // namespace ehdg
