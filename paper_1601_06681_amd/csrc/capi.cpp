// C ABI of the eHDG library: handles, workspace layout and the iteration drivers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <tuple>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/ehdg.h"
#include "kernels.h"
#include "ring.h"
#include "setup.h"

using namespace ehdg;

struct ehdg_problem {
  ehdg_desc desc;
  Operators ops;
  DevProblem dp;
  const KernelSet* ks = nullptr;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  // workspace regions used only at setup / data time
  double* Q = nullptr;
  double* W = nullptr;
  double* Bfull = nullptr;  // n x (m * nq_el), block diagonal load matrix
  double* scratch = nullptr;
  // variable velocity: per-element operators (T_e, R_e in dp; W_e = A_e^{-1} here)
  bool var = false;
  double* Wv = nullptr;
  // host mirror of the device control block, valid after every synchronizing call
  Ctrl mirror{};
  int recovered = -1;     // 1 when u2[ucur ^ 1] holds the solution of the current iterate
  int predict = 4;        // sweeps the next solve / step is expected to need
  int predict_outer = 2;  // refinements the next mixed-precision solve / step is expected to need
  unsigned seq = 0;       // launch number of the last FP64 sweep queued (the sweeps' lagged tests)
  unsigned stamp = 0;     // last stamp given to a refinement's last correction sweep (never 0)
  std::string err;
};

namespace {

constexpr int kHistCap = 1 << 16;
constexpr int kStepCap = 1 << 16;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int fail(ehdg_problem* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  return code;
}

#define HIP_TRY(h, call)                                                                    \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) return fail((h), EHDG_ERR_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

Desc to_desc(const ehdg_desc* d) {
  Desc o;
  o.pde = d->pde;
  o.dim = d->dim;
  for (int a = 0; a < 3; ++a) {
    o.n[a] = (a < d->dim) ? d->n[a] : 1;
    o.L[a] = (a < d->dim) ? d->L[a] : 1.0;
    o.periodic[a] = (a < d->dim) ? (d->periodic[a] ? 1 : 0) : 0;
    o.beta[a] = (a < d->dim) ? d->beta[a] : 0.0;
  }
  o.degree = d->degree;
  o.sigma = d->sigma;
  o.Phi = d->Phi;
  o.dt = d->dt;
  o.U0[0] = d->U0[0];
  o.U0[1] = d->U0[1];
  o.c0 = d->c0;
  o.rho0 = d->rho0;
  return o;
}

struct Layout {
  size_t off_ctrl, off_counters, off_Mf64, off_Tf32, off_partials, off_hist, off_steps, off_T64, off_Tf64, off_T32, off_T16, off_R, off_Q, off_W, off_P,
      off_G,
      off_B, off_Mv, off_gbe;
  size_t off_s0, off_s1, off_g, off_g32, off_gsrc, off_wsrc, off_u0, off_u1, off_lo0, off_lo1, off_rlo0, off_rlo1,
      off_scratch;
  size_t off_Tv, off_Rv, off_Wv;
  size_t total;
};

// lowp: room for the correction and residual of the refinement forms; plain32: g in FP32
// (the FP32 state lives in the first half of the FP64 state buffers); var: room for the
// per-element operators of a variable velocity
Layout layout_for(const Operators& o, long long nel, bool lowp, bool plain32 = false, bool var = false) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += align256(bytes);
    return at;
  };
  // one partial pair per workgroup: at most one workgroup per 16-element tile
  size_t nb = (size_t)((nel + kMfmaTileElems - 1) / kMfmaTileElems);
  if (var) nb = std::max(nb, (size_t)var_sweep_groups(nel, o.S));
  const size_t S = o.S, I = o.I, n = o.n, ne = (size_t)nel;
  const size_t Sp = (size_t)padded_rows(o.S);
  L.off_ctrl = take(sizeof(Ctrl));
  L.off_counters = take(kCounterBytes);
  // two sets of one (d2, n2) pair per workgroup (FP64 sweeps alternate between them)
  L.off_partials = take(2 * 2 * nb * sizeof(double));
  L.off_hist = take(kHistCap * sizeof(double));
  L.off_steps = take(kStepCap * sizeof(int));
  L.off_T64 = take(Sp * I * 8);
  L.off_Tf64 = take((size_t)mfma_row_tiles(o.S) * mfma_k_tiles(o.I) * 64 * 8);
  L.off_Mf64 = take((size_t)mfma_row_tiles(o.Mvol.r) * mfma_k_tiles(o.Mvol.c) * 64 * 8);
  L.off_Tf32 = take((size_t)mfma_row_tiles(o.S) * mfma_k_tiles(o.I) * 64 * 4);
  L.off_T32 = take(Sp * I * 4);
  L.off_T16 = take(Sp * I * 2);
  L.off_Mv = take((size_t)padded_rows(o.Mvol.r) * o.Mvol.c * 8);
  L.off_gbe = take(o.be ? S * ne * 8 : 8);
  L.off_R = take(n * I * 8);
  L.off_Q = take(S * n * 8);
  L.off_W = take(n * n * 8);
  L.off_P = take(o.be ? n * n * 8 : 8);
  L.off_G = take(o.be ? S * n * 8 : 8);
  L.off_B = take(n * (size_t)o.m * o.nq_el * 8);
  L.off_s0 = take(S * ne * 8);
  L.off_s1 = take(S * ne * 8);
  L.off_g = take(S * ne * 8);
  L.off_g32 = take(plain32 ? S * ne * 4 : 8);
  L.off_gsrc = take(S * ne * 8);
  L.off_wsrc = take(n * ne * 8);
  L.off_u0 = take(n * ne * 8);
  L.off_u1 = take(n * ne * 8);
  L.off_lo0 = take(lowp ? S * ne * 4 : 8);
  L.off_lo1 = take(lowp ? S * ne * 4 : 8);
  L.off_rlo0 = take(lowp ? S * ne * 4 : 8);
  L.off_rlo1 = take(lowp ? S * ne * 4 : 8);
  const size_t scr = std::max((size_t)o.m * o.nq_el, I);
  L.off_scratch = take(scr * ne * 8);
  L.off_Tv = take(var ? S * I * ((ne + 15) / 16 * 16) * 8 : 8);
  L.off_Rv = take(var ? n * I * ne * 8 : 8);
  L.off_Wv = take(var ? n * n * ne * 8 : 8);
  L.total = off;
  return L;
}

// Launch shapes of the plain sweeps chosen by a tuner, keyed by (pde, dim, degree,
// precision): tiles per workgroup (0 = one round of resident workgroups) and workgroup
// order.  Read when a handle is set up; the shape is fixed for the handle's life (the
// lagged stopping test reads the previous launch's per-workgroup partial sums).
struct TuneTable {
  std::mutex mu;
  std::map<std::tuple<int, int, int, int>, std::pair<int, int>> shape;
};
TuneTable& tune_table() {
  static TuneTable t;
  return t;
}
std::pair<int, int> tuned_shape(const ehdg_desc* d) {
  TuneTable& t = tune_table();
  std::lock_guard<std::mutex> lk(t.mu);
  const auto it = t.shape.find(std::make_tuple(d->pde, d->dim, d->degree, d->precision));
  return it == t.shape.end() ? std::make_pair(0, 0) : it->second;
}

long long nel_of(const ehdg_desc* d) {
  long long n = 1;
  for (int a = 0; a < d->dim; ++a) n *= d->n[a];
  return n;
}

// Degree-1 2D transport with both velocity components non-zero (constant or variable
// velocity) is refused: its kernels were running when a GPU run ended with the device
// faulted, and the case stays switched off until that failure has a known cause.
bool held_family(const ehdg_desc* d, int na) { return d->pde == EHDG_TRANSPORT && d->dim == 2 && d->degree == 1 && na == 2; }

std::string validate(const ehdg_desc* d) {
  if (!d) return "null descriptor";
  if (d->dim != 2 && d->dim != 3) return "dim must be 2 or 3";
  for (int a = 0; a < d->dim; ++a)
    if (d->n[a] < 1) return "n[a] must be >= 1";
  if (nel_of(d) > (1LL << 31) - 1024) return "too many elements";
  if (d->precision < EHDG_FP64 || d->precision > EHDG_FP32) return "unknown precision";
  if ((d->precision == EHDG_FP32_REFINE || d->precision == EHDG_BF16_REFINE) && d->inner_sweeps < 1)
    return "inner_sweeps must be >= 1";
  return "";
}

// Operator A (rows x cols) cut into the 16 x 4 fragments of the FP64 matrix-core
// instruction: F[(mt * KT + kt) * 64 + l] = A[16 mt + l % 16][4 kt + l / 16], zero outside A.
std::vector<double> fragments(const Mat& A) {
  const int MT = mfma_row_tiles(A.r), KT = mfma_k_tiles(A.c);
  std::vector<double> F((size_t)MT * KT * 64, 0.0);
  for (int mt = 0; mt < MT; ++mt)
    for (int kt = 0; kt < KT; ++kt)
      for (int l = 0; l < 64; ++l) {
        const int r = 16 * mt + l % 16, c = 4 * kt + l / 16;
        if (r < A.r && c < A.c) F[((size_t)mt * KT + kt) * 64 + l] = A(r, c);
      }
  return F;
}

int upload(ehdg_problem* h, void* dst, const void* src, size_t bytes) {
  HIP_TRY(h, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->stream));
  return EHDG_OK;
}

// Sweep counts of the completed steps [first, first + count) from the device ring
// (count <= kStepCap: the caller reads them back before the ring can wrap onto them).
int read_step_counts(ehdg_problem* h, const int* ring, int first, int count, int* out) {
  const RingSpan sp = ring_span(first, count, kStepCap);
  if (sp.n0) HIP_TRY(h, hipMemcpy(out, ring + sp.off0, sp.n0 * sizeof(int), hipMemcpyDeviceToHost));
  if (sp.n1) HIP_TRY(h, hipMemcpy(out + sp.n0, ring + sp.off1, sp.n1 * sizeof(int), hipMemcpyDeviceToHost));
  return EHDG_OK;
}

int check_launch(ehdg_problem* h) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(h, EHDG_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return EHDG_OK;
}

// synchronizes the stream and refreshes the host mirror of the control block
int sync_ctrl(ehdg_problem* h) {
  HIP_TRY(h, hipMemcpyAsync(&h->mirror, h->dp.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return EHDG_OK;
}

double* u_cur(ehdg_problem* h) { return h->dp.u2[h->mirror.ucur & 1]; }
double* u_other(ehdg_problem* h) { return h->dp.u2[(h->mirror.ucur & 1) ^ 1]; }

// g for the current time level: steady g = g_src; backward Euler g = g_src + G u (and
// its FP32 copy in the plain FP32 form)
void rebuild_g(ehdg_problem* h) {
  DevProblem& dp = h->dp;
  const size_t cnt = (size_t)dp.S * dp.mesh.nel;
  hipMemcpyAsync(dp.g, dp.g_src, cnt * 8, hipMemcpyDeviceToDevice, h->stream);
  if (dp.be) launch_matvec(dp.G, dp.S, dp.n, u_cur(h), dp.g, dp.mesh.nel, true, h->stream);
  if (dp.g32) launch_cast(dp.g, dp.g32, cnt, 0, h->stream);
}

// refinement forms (low-precision correction sweeps inside FP64 refinements)
bool mixed(const ehdg_problem* h) {
  return h->desc.precision == EHDG_FP32_REFINE || h->desc.precision == EHDG_BF16_REFINE;
}
// plain FP32 form: FP32 state, g and sweeps, FP64 stopping test and recovery
bool plain32(const ehdg_problem* h) { return h->desc.precision == EHDG_FP32; }

// element solution of the local solve that read state buffer `buf` into u_other (on the
// handle's stream, or on `st`)
void recover(ehdg_problem* h, int buf, hipStream_t st = nullptr) {
  DevProblem& dp = h->dp;
  if (!st) st = h->stream;
  if (plain32(h))
    h->ks->volume32(dp, (const float*)dp.s[buf & 1], u_cur(h), u_other(h), st);
  else
    h->ks->volume(dp, dp.s[buf & 1], u_cur(h), u_other(h), st);
}

// queues one outer iteration: a plain sweep, or a refinement with its inner sweeps
struct Outer {
  ehdg_problem* h;
  const void* lo_prev = nullptr;
  unsigned applied = 0;  // stamp of the last correction sweep queued (0: none)
  int k = 0;             // refinements queued (selects the residual buffer)
  void queue(double tol) {
    DevProblem& dp = h->dp;
    if (!mixed(h)) {
      (plain32(h) ? h->ks->sweep32 : h->ks->sweep64)(dp, tol, ++h->seq, h->stream);
      return;
    }
    const bool bf = h->desc.precision == EHDG_BF16_REFINE;
    auto refine = bf ? h->ks->refine16 : h->ks->refine32;
    auto inner = bf ? h->ks->inner16 : h->ks->inner32;
    // refinement k writes residual buffer rlo[k & 1]; the correction it reads is
    // the previous refinement's last inner iterate, never that buffer
    void* r = dp.rlo[k & 1];
    refine(dp, lo_prev, r, tol, applied, h->stream);
    applied = 0;
    const void* cur = r;
    for (int q = 1; q < h->desc.inner_sweeps; ++q) {
      void* out = dp.lo[q & 1];
      // the last correction sweep may store s' for the next refinement (stamped)
      if (q + 1 == h->desc.inner_sweeps) {
        if (++h->stamp == 0u) ++h->stamp;
        applied = h->stamp;
      }
      inner(dp, r, cur, out, applied, h->stream);
      cur = out;
    }
    lo_prev = cur;
    ++k;
  }
};

// Runs outer iterations of the current segment until the device flag is raised or
// max_outer have been queued.  The first batch is the predicted count (a warm
// start needs about as many as the previous solve); later batches grow.  Queued
// iterations after convergence exit at once on the device flag.
int run_segment(ehdg_problem* h, double tol, int max_outer) {
  Outer o{h};
  int& pred = mixed(h) ? h->predict_outer : h->predict;
  int launched = 0, chunk = std::max(1, pred), next = 2;
  for (;;) {
    const int n = std::min(chunk, max_outer - launched);
    for (int j = 0; j < n; ++j) o.queue(tol);
    launched += n;
    // plain sweeps leave their own stopping test to the next launch: take the last one
    if (!mixed(h)) launch_reduce_lagged(h->dp, tol, h->seq + 1, h->stream);
    int rc = check_launch(h);
    if (rc) return rc;
    rc = sync_ctrl(h);
    if (rc) return rc;
    if (h->mirror.done || launched >= max_outer) {
      if (h->mirror.status == 1) pred = h->mirror.iters;
      return EHDG_OK;
    }
    chunk = next;
    next = std::min(next * 2, 64);
  }
}

int status_code(ehdg_problem* h) {
  if (h->mirror.status == 2) return fail(h, EHDG_ERR_DIVERGED, "relative trace increment became non-finite");
  if (h->mirror.status != 1) return fail(h, EHDG_ERR_NOT_CONVERGED, "iteration cap reached");
  return EHDG_OK;
}

}  // namespace

extern "C" {

int ehdg_reference_points(int32_t degree, double* gll_nodes, double* gauss_pts, double* gauss_wts) {
  if (degree < 1 || degree > 16) return EHDG_ERR_INVALID_ARG;
  Basis1D b = make_basis(degree);
  if (gll_nodes) std::memcpy(gll_nodes, b.x.data(), b.x.size() * sizeof(double));
  if (gauss_pts) std::memcpy(gauss_pts, b.xq.data(), b.xq.size() * sizeof(double));
  if (gauss_wts) std::memcpy(gauss_wts, b.wq.data(), b.wq.size() * sizeof(double));
  return EHDG_OK;
}

int ehdg_workspace_bytes(const ehdg_desc* desc, size_t* bytes) {
  if (!bytes) return EHDG_ERR_INVALID_ARG;
  std::string v = validate(desc);
  if (!v.empty()) return EHDG_ERR_INVALID_ARG;
  Operators ops;
  std::string e = build_operators(to_desc(desc), ops);
  if (!e.empty() || held_family(desc, ops.na)) return EHDG_ERR_UNSUPPORTED;
  const bool lowp = desc->precision == EHDG_FP32_REFINE || desc->precision == EHDG_BF16_REFINE;
  *bytes = layout_for(ops, nel_of(desc), lowp, desc->precision == EHDG_FP32).total;
  return EHDG_OK;
}

// smp: velocity samples of a variable-velocity transport problem, else null
static int setup_impl(const ehdg_desc* desc, const VarSamples* smp, void* d_workspace, size_t workspace_bytes,
                      void* stream, ehdg_handle* out) {
  if (!out || !desc) return EHDG_ERR_INVALID_ARG;
  *out = nullptr;
  std::string v = validate(desc);
  if (!v.empty()) return EHDG_ERR_INVALID_ARG;
  if (!d_workspace || ((uintptr_t)d_workspace & 255)) return EHDG_ERR_INVALID_ARG;
  if (smp && desc->precision != EHDG_FP64) return EHDG_ERR_UNSUPPORTED;
  ehdg_problem* h = new (std::nothrow) ehdg_problem();
  if (!h) return EHDG_ERR_INVALID_ARG;
  h->desc = *desc;
  h->stream = (hipStream_t)stream;
  h->var = smp != nullptr;
  VarOperators vo;
  std::string e = smp ? build_variable_operators(to_desc(desc), smp, h->ops, &vo) : build_operators(to_desc(desc), h->ops);
  if (!e.empty() || held_family(desc, h->ops.na)) {
    delete h;
    return EHDG_ERR_UNSUPPORTED;
  }
  const Operators& o = h->ops;
  h->ks = smp ? find_var_kernels(desc->dim, o.na, desc->degree)
              : find_kernels(desc->pde, desc->dim, desc->pde == 0 ? o.na : 0, desc->degree);
  const bool lowp = desc->precision == EHDG_FP32_REFINE || desc->precision == EHDG_BF16_REFINE;
  if (!h->ks || (desc->precision == EHDG_BF16_REFINE && !h->ks->refine16) ||
      (desc->precision == EHDG_FP32_REFINE && !h->ks->refine32) || (desc->precision == EHDG_FP32 && !h->ks->sweep32)) {
    delete h;
    return EHDG_ERR_UNSUPPORTED;
  }
  const long long nel = nel_of(desc);
  Layout L = layout_for(o, nel, lowp, desc->precision == EHDG_FP32, h->var);
  if (workspace_bytes < L.total) {
    delete h;
    return EHDG_ERR_WORKSPACE_TOO_SMALL;
  }
  char* ws = (char*)d_workspace;
  h->ws = ws;
  h->ws_bytes = workspace_bytes;
  DevProblem& dp = h->dp;
  std::memset(&dp, 0, sizeof(dp));
  dp.mesh.nel = (int)nel;
  for (int a = 0; a < 3; ++a) {
    dp.mesh.n[a] = (a < desc->dim) ? desc->n[a] : 1;
    dp.mesh.periodic[a] = (a < desc->dim) ? (desc->periodic[a] ? 1 : 0) : 0;
    dp.mesh.ax[a] = o.ax[a];
    dp.mesh.dir[a] = o.dir[a];
  }
  dp.pde = desc->pde;
  dp.dim = desc->dim;
  dp.nf = o.nf;
  dp.S = o.S;
  dp.I = o.I;
  dp.n = o.n;
  dp.m = o.m;
  dp.Np = o.Np;
  dp.na = o.na;
  dp.be = o.be;
  dp.ctrl = (Ctrl*)(ws + L.off_ctrl);
  dp.counters = (unsigned*)(ws + L.off_counters);
  dp.partials = (double*)(ws + L.off_partials);
  dp.partial_stride = (int)((L.off_hist - L.off_partials) / sizeof(double) / 2);
  if (h->ks->sweep_groups) {
    const std::pair<int, int> shape = tuned_shape(desc);
    dp.mesh.order = shape.second ? 1 : 0;
    int tpg = shape.first, groups = 0;
    (desc->precision == EHDG_FP32 ? h->ks->sweep32_groups : h->ks->sweep_groups)((int)nel, &tpg, &groups);
    dp.sweep_tpg = shape.first > 0 ? tpg : 0;
    dp.nb_sweep = groups;
  } else {
    dp.nb_sweep = (int)var_sweep_groups(nel, o.S);
  }
  if (2 * (long long)dp.nb_sweep > dp.partial_stride) {
    delete h;
    return EHDG_ERR_INVALID_ARG;
  }
  dp.hist = (double*)(ws + L.off_hist);
  dp.hist_cap = kHistCap;
  dp.step_iters = (int*)(ws + L.off_steps);
  dp.step_cap = kStepCap;
  dp.T64 = (const double*)(ws + L.off_T64);
  dp.Tf64 = (const double*)(ws + L.off_Tf64);
  dp.Mf64 = (const double*)(ws + L.off_Mf64);
  dp.Tf32 = (const float*)(ws + L.off_Tf32);
  dp.T32 = (const float*)(ws + L.off_T32);
  dp.T16 = (const uint16_t*)(ws + L.off_T16);
  dp.R = (const double*)(ws + L.off_R);
  dp.Mvol = (const double*)(ws + L.off_Mv);
  dp.gbe = (double*)(ws + L.off_gbe);
  dp.has_src = false;
  dp.P = (const double*)(ws + L.off_P);
  dp.G = (const double*)(ws + L.off_G);
  dp.s[0] = (double*)(ws + L.off_s0);
  dp.s[1] = (double*)(ws + L.off_s1);
  dp.g = (double*)(ws + L.off_g);
  dp.g32 = desc->precision == EHDG_FP32 ? (float*)(ws + L.off_g32) : nullptr;
  dp.g_src = (double*)(ws + L.off_gsrc);
  dp.w_src = (double*)(ws + L.off_wsrc);
  dp.u2[0] = (double*)(ws + L.off_u0);
  dp.u2[1] = (double*)(ws + L.off_u1);
  dp.lo[0] = ws + L.off_lo0;
  dp.lo[1] = ws + L.off_lo1;
  dp.rlo[0] = ws + L.off_rlo0;
  dp.rlo[1] = ws + L.off_rlo1;
  h->Q = (double*)(ws + L.off_Q);
  h->W = (double*)(ws + L.off_W);
  h->Bfull = (double*)(ws + L.off_B);
  h->scratch = (double*)(ws + L.off_scratch);
  dp.in_scratch = h->scratch;
  dp.Tv = (const double*)(ws + L.off_Tv);
  dp.Rv = (const double*)(ws + L.off_Rv);
  h->Wv = (double*)(ws + L.off_Wv);
  int rc = 0;
  const size_t SI = (size_t)padded_rows(o.S) * o.I;
  // operators (FP64 host -> device, rows zero-padded to whole row groups) and the
  // low-precision copies of T
  std::vector<double> Tpad(SI, 0.0), Mvpad((size_t)padded_rows(o.Mvol.r) * o.Mvol.c, 0.0);
  std::copy(o.T.a.begin(), o.T.a.end(), Tpad.begin());
  std::copy(o.Mvol.a.begin(), o.Mvol.a.end(), Mvpad.begin());
  // fragment-major copies of T and of the recovery operator for the matrix-core kernels
  const std::vector<double> Tf = fragments(o.T), Mf = fragments(o.Mvol);
  std::vector<double> B;
  {
    const int cols = o.m * o.nq_el;
    B.assign((size_t)o.n * cols, 0.0);
    for (int f = 0; f < o.m; ++f)
      for (int i = 0; i < o.Np; ++i)
        for (int q = 0; q < o.nq_el; ++q) B[(size_t)(f * o.Np + i) * cols + f * o.nq_el + q] = o.Bload(i, q);
  }
  if ((rc = upload(h, (void*)dp.T64, Tpad.data(), SI * 8)) ||
      (rc = upload(h, (void*)dp.Tf64, Tf.data(), Tf.size() * 8)) ||
      (rc = upload(h, (void*)dp.Mf64, Mf.data(), Mf.size() * 8)) ||
      (rc = upload(h, (void*)dp.Mvol, Mvpad.data(), Mvpad.size() * 8)) ||
      (rc = upload(h, (void*)dp.R, o.R.a.data(), (size_t)o.n * o.I * 8)) ||
      (rc = upload(h, h->Q, o.Q.a.data(), (size_t)o.S * o.n * 8)) ||
      (rc = upload(h, h->W, o.W.a.data(), (size_t)o.n * o.n * 8)) ||
      (rc = upload(h, h->Bfull, B.data(), B.size() * 8)) ||
      (o.be && (rc = upload(h, (void*)dp.P, o.P.a.data(), (size_t)o.n * o.n * 8))) ||
      (o.be && (rc = upload(h, (void*)dp.G, o.G.a.data(), (size_t)o.S * o.n * 8))) ||
      (h->var && ((rc = upload(h, (void*)dp.Tv, vo.T.data(), vo.T.size() * 8)) ||
                  (rc = upload(h, (void*)dp.Rv, vo.R.data(), vo.R.size() * 8)) ||
                  (rc = upload(h, h->Wv, vo.W.data(), vo.W.size() * 8))))) {
    delete h;
    return rc;
  }
  launch_cast(dp.T64, (void*)dp.T32, SI, 0, h->stream);
  launch_cast(dp.T64, (void*)dp.T16, SI, 1, h->stream);
  launch_cast(dp.Tf64, (void*)dp.Tf32, Tf.size(), 0, h->stream);
  launch_fill_bytes(dp.counters, kCounterBytes, h->stream);
  launch_fill_bytes(dp.partials, L.off_hist - L.off_partials, h->stream);
  launch_fill(dp.hist, 0.0, kHistCap, h->stream);
  launch_fill_bytes(dp.step_iters, kStepCap * sizeof(int), h->stream);
  launch_ctrl_reset(dp.ctrl, 1, h->seq + 1, h->stream);
  // the host buffers above are pageable: the copies complete before this returns
  rc = sync_ctrl(h);
  if (!rc) rc = ehdg_set_forcing(h, nullptr, nullptr);
  if (!rc) rc = ehdg_set_initial(h, nullptr);
  if (rc) {
    delete h;
    return rc;
  }
  *out = h;
  return EHDG_OK;
}

int ehdg_setup(const ehdg_desc* desc, void* d_workspace, size_t workspace_bytes, void* stream, ehdg_handle* out) {
  return setup_impl(desc, nullptr, d_workspace, workspace_bytes, stream, out);
}

int ehdg_variable_workspace_bytes(const ehdg_desc* desc, size_t* bytes) {
  if (!bytes) return EHDG_ERR_INVALID_ARG;
  std::string v = validate(desc);
  if (!v.empty()) return EHDG_ERR_INVALID_ARG;
  if (desc->precision != EHDG_FP64) return EHDG_ERR_UNSUPPORTED;
  Operators ops;
  std::string e = build_variable_operators(to_desc(desc), nullptr, ops, nullptr);
  if (!e.empty() || held_family(desc, ops.na)) return EHDG_ERR_UNSUPPORTED;
  *bytes = layout_for(ops, nel_of(desc), false, false, true).total;
  return EHDG_OK;
}

int ehdg_setup_variable(const ehdg_desc* desc, const double* beta_q, const double* div_beta_q,
                        const double* beta_face, void* d_workspace, size_t workspace_bytes, void* stream,
                        ehdg_handle* out) {
  if (!beta_q || !beta_face) return EHDG_ERR_INVALID_ARG;
  const VarSamples smp{beta_q, div_beta_q, beta_face};
  return setup_impl(desc, &smp, d_workspace, workspace_bytes, stream, out);
}

int ehdg_set_forcing(ehdg_handle h, const double* d_forcing_q, const double* d_bc) {
  if (!h) return EHDG_ERR_INVALID_ARG;
  DevProblem& dp = h->dp;
  const int nel = dp.mesh.nel;
  hipStream_t st = h->stream;
  const Operators& o = h->ops;
  if (d_bc && dp.pde != 0) return fail(h, EHDG_ERR_INVALID_ARG, "boundary data applies to transport only");
  if (d_forcing_q) {
    // F = (f, psi) per field (u_other is free here), then w_src = A^{-1} F
    launch_ext_to_soa(d_forcing_q, h->scratch, o.m * o.nq_el, nel, st);
    launch_matvec(h->Bfull, o.n, o.m * o.nq_el, h->scratch, u_other(h), nel, false, st);
    if (h->var)
      launch_matvec_pe(h->Wv, o.n, o.n, u_other(h), dp.w_src, nel, false, st);
    else
      launch_matvec(h->W, o.n, o.n, u_other(h), dp.w_src, nel, false, st);
  } else {
    launch_fill(dp.w_src, 0.0, (size_t)o.n * nel, st);
  }
  if (d_bc) {
    launch_bc_inputs(dp, d_bc, h->scratch, st);
    if (h->var)
      launch_matvec_pe(dp.Rv, o.n, o.I, h->scratch, dp.w_src, nel, true, st);
    else
      launch_matvec(dp.R, o.n, o.I, h->scratch, dp.w_src, nel, true, st);
  }
  launch_matvec(h->Q, o.S, o.n, dp.w_src, dp.g_src, nel, false, st);
  dp.has_src = d_forcing_q != nullptr || d_bc != nullptr;
  if (dp.be) {
    // source part of the next step's g: Q A^{-1} (F_src + Mbt A^{-1} F_src)
    hipMemcpyAsync(dp.gbe, dp.g_src, (size_t)o.S * nel * 8, hipMemcpyDeviceToDevice, st);
    launch_matvec(dp.G, o.S, o.n, dp.w_src, dp.gbe, nel, true, st);
  }
  rebuild_g(h);
  h->recovered = -1;
  return check_launch(h);
}

int ehdg_set_initial(ehdg_handle h, const double* d_u0) {
  if (!h) return EHDG_ERR_INVALID_ARG;
  DevProblem& dp = h->dp;
  const int nel = dp.mesh.nel;
  launch_ctrl_reset(dp.ctrl, 1, h->seq + 1, h->stream);
  h->mirror.base = 0;
  h->mirror.ucur = 0;
  h->mirror.iters = 0;
  h->mirror.done = 0;
  h->mirror.steps_done = 0;
  if (d_u0)
    launch_ext_to_soa(d_u0, dp.u2[0], dp.n, nel, h->stream);
  else
    launch_fill(dp.u2[0], 0.0, (size_t)dp.n * nel, h->stream);
  if (dp.g32) {
    // plain FP32 form: the initial trace in FP32, in the first half of state buffer 0
    launch_matvec(h->Q, dp.S, dp.n, dp.u2[0], h->scratch, nel, false, h->stream);
    launch_cast(h->scratch, (float*)dp.s[0], (size_t)dp.S * nel, 0, h->stream);
  } else {
    launch_matvec(h->Q, dp.S, dp.n, dp.u2[0], dp.s[0], nel, false, h->stream);
  }
  rebuild_g(h);
  h->recovered = -1;
  return check_launch(h);
}

int ehdg_iterate(ehdg_handle h, int32_t n_iters) {
  if (!h || n_iters < 0) return EHDG_ERR_INVALID_ARG;
  if (mixed(h)) return fail(h, EHDG_ERR_UNSUPPORTED, "iterate runs the plain (FP64 or FP32) sweep");
  // a finished solve is continued in a new segment from its last iterate (on the device)
  launch_ctrl_reset(h->dp.ctrl, 2, h->seq + 1, h->stream);
  auto sweep = plain32(h) ? h->ks->sweep32 : h->ks->sweep64;
  for (int j = 0; j < n_iters; ++j) sweep(h->dp, -1.0, ++h->seq, h->stream);
  // the last sweep's increment is recorded by the next launch: take it now
  if (n_iters > 0) launch_reduce_lagged(h->dp, -1.0, h->seq + 1, h->stream);
  h->recovered = -1;
  return check_launch(h);
}

int ehdg_solve(ehdg_handle h, double rel_tol, int32_t max_iters, int32_t* iters, double* rel_res) {
  if (!h || max_iters < 1 || !(rel_tol >= 0.0)) return EHDG_ERR_INVALID_ARG;
  DevProblem& dp = h->dp;
  launch_ctrl_reset(dp.ctrl, 0, h->seq + 1, h->stream);  // a new segment from the latest state
  const int s = mixed(h) ? h->desc.inner_sweeps : 1;
  const int max_outer = std::max(1, (max_iters + s - 1) / s);
  int rc = run_segment(h, rel_tol, max_outer);
  if (rc) return rc;
  const Ctrl& c = h->mirror;
  if (iters) *iters = c.iters * s;
  if (rel_res) *rel_res = c.last_res;
  rc = status_code(h);
  h->recovered = -1;
  if (c.iters > 0 && c.status != 2) {
    // plain: u^K is the local solve that read s^{K-1}; refinement: the refined iterate s^K
    const int lag = mixed(h) ? 0 : 1;
    recover(h, (c.base + c.iters - lag) & 1);
    int rc2 = check_launch(h);
    if (rc2) return rc2;
    h->recovered = 1;
  }
  return rc;
}

int ehdg_step(ehdg_handle h, int32_t n_steps, double rel_tol, int32_t max_iters_per_step, int32_t* iters_per_step) {
  if (!h || n_steps < 0 || max_iters_per_step < 1 || !(rel_tol >= 0.0)) return EHDG_ERR_INVALID_ARG;
  if (!h->dp.be) return fail(h, EHDG_ERR_INVALID_ARG, "ehdg_step needs a backward-Euler problem (dt > 0)");
  if (n_steps == 0) return EHDG_OK;
  DevProblem& dp = h->dp;
  const int s = mixed(h) ? h->desc.inner_sweeps : 1;
  const int lag = mixed(h) ? 0 : 1;
  const int max_outer = std::max(1, (max_iters_per_step + s - 1) / s);
  int& pred = mixed(h) ? h->predict_outer : h->predict;
  // the first step continues from the latest state of whatever ran before
  launch_ctrl_reset(dp.ctrl, 0, h->seq + 1, h->stream);
  int rc = sync_ctrl(h);
  if (rc) return rc;
  const int first = h->mirror.steps_done, target = first + n_steps;
  Outer o{h};
  int max_seen = 0;
  std::vector<int> counts;  // sweeps of the steps completed in this call
  counts.reserve(n_steps);
  // Every step is queued as (predicted outer iterations + a margin) followed by the
  // step kernel.  A step that converges early leaves no-op launches; one that needs more
  // borrows the next step's iterations (its step kernel finds it unconverged and does
  // nothing), which leaves the rest of that step's slot as no-ops and usually costs
  // another batch.  Counts grow slowly along a run, so the margin (1 + pred / 8) keeps
  // borrowing rare at the cost of a few no-ops per step.  The host synchronizes once per
  // batch and reads that batch's counts back; a batch queues at most kStepCap steps, so
  // the ring never wraps onto counts not yet read.
  while (h->mirror.steps_done < target) {
    const int remaining = std::min(target - h->mirror.steps_done, kStepCap);
    const int before = h->mirror.steps_done;
    const int p = std::max(1, pred);
    const int per = std::min(p + 1 + (p + 7) / 8, max_outer);
    for (int r = 0; r < remaining; ++r) {
      for (int j = 0; j < per; ++j) o.queue(rel_tol);
      (plain32(h) ? h->ks->step32 : h->ks->step)(dp, lag, h->seq + 1, rel_tol, mixed(h) ? 0 : 1, h->stream);
    }
    rc = check_launch(h);
    if (rc) return rc;
    rc = sync_ctrl(h);
    if (rc) return rc;
    if (h->mirror.status == 2) return status_code(h);
    const int fresh = h->mirror.steps_done - before;
    if (fresh > 0) {
      counts.resize(counts.size() + fresh);
      rc = read_step_counts(h, dp.step_iters, before, fresh, counts.data() + counts.size() - fresh);
      if (rc) return rc;
      for (size_t i = counts.size() - fresh; i < counts.size(); ++i) max_seen = std::max(max_seen, counts[i]);
      pred = max_seen;
    }
    if (h->mirror.steps_done < target && h->mirror.iters >= max_outer) {
      status_code(h);
      break;
    }
  }
  const int done = h->mirror.steps_done - first;
  if (iters_per_step)
    for (int i = 0; i < done && i < (int)counts.size(); ++i) iters_per_step[i] = counts[i] * s;
  for (int i = done; iters_per_step && i < n_steps; ++i) iters_per_step[i] = 0;
  h->recovered = -1;
  if (done < n_steps) return fail(h, EHDG_ERR_NOT_CONVERGED, "iteration cap reached within a time step");
  return EHDG_OK;
}

}  // extern "C"

namespace {
// Queues on st the element solution of the state the host mirror describes into d_u
// (external layout): the recovery from the latest sweep's traces, unless it is there
// already or no sweep ran since the current time level was set.
void queue_solution(ehdg_problem* h, double* d_u, hipStream_t st) {
  DevProblem& dp = h->dp;
  const Ctrl& c = h->mirror;
  const double* src = u_cur(h);
  if (h->recovered == 1) {
    src = u_other(h);
  } else if (c.iters > 0 && !mixed(h)) {
    recover(h, (c.base + c.iters - 1) & 1, st);
    h->recovered = 1;
    src = u_other(h);
  }
  launch_soa_to_ext(src, d_u, dp.n, dp.mesh.nel, st);
}
}  // namespace

extern "C" {

int ehdg_get_solution(ehdg_handle h, double* d_u) {
  if (!h || !d_u) return EHDG_ERR_INVALID_ARG;
  int rc = sync_ctrl(h);
  if (rc) return rc;
  queue_solution(h, d_u, h->stream);
  return check_launch(h);
}

int ehdg_get_residuals(ehdg_handle h, int32_t first, int32_t count, double* out) {
  if (!h || first < 0 || count < 0 || (count > 0 && !out)) return EHDG_ERR_INVALID_ARG;
  int rc = sync_ctrl(h);
  if (rc) return rc;
  const Ctrl& c = h->mirror;
  if ((long long)first + count > c.iters || count > kHistCap || c.iters - first > kHistCap)
    return fail(h, EHDG_ERR_INVALID_ARG, "residual range not recorded");
  std::vector<double> ring(kHistCap);
  HIP_TRY(h, hipMemcpyAsync(ring.data(), h->dp.hist, kHistCap * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  for (int i = 0; i < count; ++i) out[i] = ring[(first + i) % kHistCap];
  return EHDG_OK;
}

int ehdg_sizes(ehdg_handle h, int64_t* n_el, int32_t* m, int32_t* n_p, int32_t* s, int32_t* i, int32_t* iters) {
  if (!h) return EHDG_ERR_INVALID_ARG;
  if (n_el) *n_el = h->dp.mesh.nel;
  if (m) *m = h->dp.m;
  if (n_p) *n_p = h->dp.Np;
  if (s) *s = h->dp.S;
  if (i) *i = h->dp.I;
  if (iters) {
    int rc = sync_ctrl(h);
    if (rc) return rc;
    *iters = h->mirror.iters;
  }
  return EHDG_OK;
}

// state blob: [Ctrl (256 B)][s0][s1][u of the current time level]
int ehdg_state_bytes(ehdg_handle h, size_t* bytes) {
  if (!h || !bytes) return EHDG_ERR_INVALID_ARG;
  const size_t ne = (size_t)h->dp.mesh.nel;
  *bytes = 256 + align256(h->dp.S * ne * 8) * 2 + align256(h->dp.n * ne * 8);
  return EHDG_OK;
}

int ehdg_get_state(ehdg_handle h, void* d_dst, size_t bytes) {
  size_t need = 0;
  if (!h || !d_dst || ehdg_state_bytes(h, &need) || bytes < need) return EHDG_ERR_INVALID_ARG;
  DevProblem& dp = h->dp;
  const size_t ne = (size_t)dp.mesh.nel;
  char* d = (char*)d_dst;
  const size_t sb = align256(dp.S * ne * 8);
  int rc = sync_ctrl(h);
  if (rc) return rc;
  HIP_TRY(h, hipMemcpyAsync(d, dp.ctrl, sizeof(Ctrl), hipMemcpyDeviceToDevice, h->stream));
  HIP_TRY(h, hipMemcpyAsync(d + 256, dp.s[0], dp.S * ne * 8, hipMemcpyDeviceToDevice, h->stream));
  HIP_TRY(h, hipMemcpyAsync(d + 256 + sb, dp.s[1], dp.S * ne * 8, hipMemcpyDeviceToDevice, h->stream));
  HIP_TRY(h, hipMemcpyAsync(d + 256 + 2 * sb, u_cur(h), dp.n * ne * 8, hipMemcpyDeviceToDevice, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return EHDG_OK;
}

int ehdg_set_state(ehdg_handle h, const void* d_src, size_t bytes) {
  size_t need = 0;
  if (!h || !d_src || ehdg_state_bytes(h, &need) || bytes < need) return EHDG_ERR_INVALID_ARG;
  DevProblem& dp = h->dp;
  const size_t ne = (size_t)dp.mesh.nel;
  const char* d = (const char*)d_src;
  const size_t sb = align256(dp.S * ne * 8);
  HIP_TRY(h, hipMemcpyAsync(dp.ctrl, d, sizeof(Ctrl), hipMemcpyDeviceToDevice, h->stream));
  int rc = sync_ctrl(h);
  if (rc) return rc;
  const Ctrl& c = h->mirror;
  if ((c.base & ~1) || (c.ucur & ~1) || c.iters < 0) return fail(h, EHDG_ERR_INVALID_ARG, "corrupt state blob");
  HIP_TRY(h, hipMemcpyAsync(dp.s[0], d + 256, dp.S * ne * 8, hipMemcpyDeviceToDevice, h->stream));
  HIP_TRY(h, hipMemcpyAsync(dp.s[1], d + 256 + sb, dp.S * ne * 8, hipMemcpyDeviceToDevice, h->stream));
  HIP_TRY(h, hipMemcpyAsync(u_cur(h), d + 256 + 2 * sb, dp.n * ne * 8, hipMemcpyDeviceToDevice, h->stream));
  rebuild_g(h);
  h->recovered = -1;
  return check_launch(h);
}

int ehdg_tune_set(int32_t pde, int32_t dim, int32_t degree, int32_t precision, int32_t tiles_per_group,
                  int32_t reverse_order) {
  if (tiles_per_group < 0 || (precision != EHDG_FP64 && precision != EHDG_FP32)) return EHDG_ERR_INVALID_ARG;
  TuneTable& t = tune_table();
  std::lock_guard<std::mutex> lk(t.mu);
  const auto key = std::make_tuple((int)pde, (int)dim, (int)degree, (int)precision);
  if (tiles_per_group == 0 && !reverse_order)
    t.shape.erase(key);
  else
    t.shape[key] = std::make_pair((int)tiles_per_group, reverse_order ? 1 : 0);
  return EHDG_OK;
}

int ehdg_tune_clear(void) {
  TuneTable& t = tune_table();
  std::lock_guard<std::mutex> lk(t.mu);
  t.shape.clear();
  return EHDG_OK;
}

int ehdg_launch_shape(ehdg_handle h, int32_t* tiles_per_group, int32_t* groups, int32_t* reverse_order) {
  if (!h) return EHDG_ERR_INVALID_ARG;
  if (h->var) return fail(h, EHDG_ERR_UNSUPPORTED, "variable-velocity sweeps have a fixed shape");
  int tpg = h->dp.sweep_tpg, ng = 0;
  (plain32(h) ? h->ks->sweep32_groups : h->ks->sweep_groups)(h->dp.mesh.nel, &tpg, &ng);
  if (tiles_per_group) *tiles_per_group = tpg;
  if (groups) *groups = ng;
  if (reverse_order) *reverse_order = h->dp.mesh.order;
  return EHDG_OK;
}

int ehdg_destroy(ehdg_handle h) {
  if (!h) return EHDG_ERR_INVALID_ARG;
  delete h;
  return EHDG_OK;
}

// ---------------------------------------------------------------------------- batches
}  // extern "C"

struct ehdg_batch_s {
  // members of one kernel family and precision: their own sweep entries (families the
  // persistent sweep does not cover) and step-completion entries
  struct Group {
    const KernelSet* ks;
    bool fp32;
    int sweep_first, sweep_n, step_first, step_n;
  };
  // the persistent sweep's entries, per precision
  int persist_first[2] = {0, 0}, persist_n[2] = {0, 0};
  // rounds queued as a HIP graph (captured on a private stream, replayed on `stream`)
  bool use_graph = true;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  int graph_rounds = 0;
  int graph_steps = 0;
  double graph_tol = 0.0;
  // tables in the device's static scratch array (ehdg_batch_create_static): valid while
  // no later static batch was created on the same device (generation check)
  bool is_static = false;
  int dev = 0;
  unsigned gen = 0;
  std::vector<ehdg_problem*> h;
  hipStream_t stream = nullptr;
  std::vector<Group> groups;
  BatchProblem* d_probs = nullptr;
  BatchEntry* d_table = nullptr;
  Ctrl* d_ctrl = nullptr;
  std::vector<BatchProblem> probs;
  std::vector<Ctrl> ctrl;
  std::string err;
  // the workgroup table as uploaded (the upload is asynchronous: kept until destroy) and
  // whether d_probs holds `probs` already
  std::vector<BatchEntry> table_host;
  bool probs_valid = false;
  // asynchronous rounds (ehdg_batch_launch / ehdg_batch_poll): launches whose report has
  // not been read, oldest first, each with the event recorded after its report copy
  static constexpr int kMaxPending = 4;
  struct Pending {
    int slot;
    const Ctrl* report;
    std::vector<int> target;
  };
  hipEvent_t ev[kMaxPending] = {};
  std::deque<Pending> pending;
  unsigned launches = 0;
  std::vector<int> polled;        // per member: state in the last report read (-1: none)
  hipEvent_t join_ev = nullptr;   // orders the batch stream after the members' own streams
  hipEvent_t last_ev = nullptr;   // after the batch's latest asynchronous work
  bool last_ev_set = false;
  hipEvent_t probs_ev = nullptr;  // after the latest upload of `probs`
};

// Device scratch of ehdg_batch_create_static: the batch's problem descriptors, workgroup
// table and control-block copies (see batch_layout), at most kStaticBatchBytes (8 MiB)
// per device, held until the process ends.
constexpr size_t kStaticBatchBytes = (size_t)8 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticBatchBytes];

namespace {

// ---- batch tables in a static device array, for callers that cannot allocate
// One array per GPU (each device holds its own copy of a __device__ variable), found
// with hipGetSymbolAddress the first time a static batch is created on that device.
// In host code the array's name is not a device address: only the pointer returned by
// hipGetSymbolAddress is passed to kernels and copies.
constexpr int kMaxDevices = 64;

struct StaticScratch {
  std::mutex mu;
  void* ptr[kMaxDevices] = {};
  unsigned gen[kMaxDevices] = {};
};
StaticScratch& static_scratch() {
  static StaticScratch s;
  return s;
}

int bfail(ehdg_batch_s* b, int code, const std::string& msg) {
  if (b) b->err = msg;
  return code;
}

#define HIP_TRY_B(b, call)                                                                   \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) return bfail((b), EHDG_ERR_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

// The workgroup table: first the persistent sweep's entries (FP64 members, then FP32
// members, each member's entries contiguous), then per (family, precision) group in order
// of first appearance its own sweep entries (families the persistent sweep does not cover)
// and its step-completion entries.  A member's entries are those of its own launch shape,
// so batched results are bitwise those of the member alone.
void batch_plan(const std::vector<ehdg_problem*>& hs, std::vector<ehdg_batch_s::Group>& groups,
                std::vector<BatchEntry>& table, int* persist_first, int* persist_n, bool use_persist = true) {
  auto fp32 = [&](size_t i) { return hs[i]->desc.precision == EHDG_FP32; };
  auto persist = [&](size_t i) { return use_persist ? hs[i]->ks->persist : -1; };
  auto sweep_entries = [&](size_t i) {
    const KernelSet* ks = hs[i]->ks;
    int tpg = hs[i]->dp.sweep_tpg, ng = 0;
    (fp32(i) ? ks->sweep32_groups : ks->sweep_groups)(hs[i]->dp.mesh.nel, &tpg, &ng);
    for (int b = 0; b < ng; ++b) table.push_back({(int)i, b, ng, tpg, persist(i)});
  };
  for (int prec = 0; prec < 2; ++prec) {
    persist_first[prec] = (int)table.size();
    for (size_t i = 0; i < hs.size(); ++i)
      if (persist(i) >= 0 && fp32(i) == (prec == 1)) sweep_entries(i);
    persist_n[prec] = (int)table.size() - persist_first[prec];
  }
  std::vector<std::pair<const KernelSet*, bool>> fams;
  for (size_t i = 0; i < hs.size(); ++i) {
    const auto key = std::make_pair(hs[i]->ks, fp32(i));
    if (std::find(fams.begin(), fams.end(), key) == fams.end()) fams.push_back(key);
  }
  for (const auto& key : fams) {
    const KernelSet* ks = key.first;
    ehdg_batch_s::Group g{ks, key.second, (int)table.size(), 0, 0, 0};
    for (size_t i = 0; i < hs.size(); ++i)
      if (hs[i]->ks == ks && fp32(i) == key.second && persist(i) < 0) sweep_entries(i);
    g.sweep_n = (int)table.size() - g.sweep_first;
    g.step_first = (int)table.size();
    for (size_t i = 0; i < hs.size(); ++i) {
      if (hs[i]->ks != ks || fp32(i) != key.second || !hs[i]->dp.be) continue;
      int tpg = 0, ng = 0;
      ks->step_groups(hs[i]->dp.mesh.nel, &tpg, &ng);
      for (int b = 0; b < ng; ++b) table.push_back({(int)i, b, ng, tpg, -1});
    }
    g.step_n = (int)table.size() - g.step_first;
    groups.push_back(g);
  }
}

struct BatchLayout {
  size_t off_probs, off_table, off_ctrl, total;
};

BatchLayout batch_layout(size_t n, size_t entries) {
  BatchLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off += align256(bytes);
    return at;
  };
  L.off_probs = take(n * sizeof(BatchProblem));
  L.off_table = take(entries * sizeof(BatchEntry));
  L.off_ctrl = take(n * sizeof(Ctrl));
  L.total = off;
  return L;
}

int batch_check(const ehdg_handle* handles, int32_t n, std::vector<ehdg_problem*>& hs) {
  if (!handles || n < 1) return EHDG_ERR_INVALID_ARG;
  for (int i = 0; i < n; ++i) {
    if (!handles[i]) return EHDG_ERR_INVALID_ARG;
    if (std::find(hs.begin(), hs.end(), handles[i]) != hs.end()) return EHDG_ERR_INVALID_ARG;
    const int prec = handles[i]->desc.precision;
    if ((prec != EHDG_FP64 && prec != EHDG_FP32) || handles[i]->var) return EHDG_ERR_UNSUPPORTED;
    hs.push_back(handles[i]);
  }
  return EHDG_OK;
}

// Device copies of the members' current state pointers (forcing may have changed since
// the batch was made) with each member's step limit, and uploads them.
int batch_upload(ehdg_batch_s* b, const std::vector<int>& steps_target) {
  std::vector<BatchProblem> np(b->h.size(), BatchProblem{});
  for (size_t i = 0; i < b->h.size(); ++i) {
    const DevProblem& dp = b->h[i]->dp;
    BatchProblem& P = np[i];
    P.mesh = dp.mesh;
    P.steps_target = steps_target[i];
    P.hist_cap = dp.hist_cap;
    P.step_cap = dp.step_cap;
    P.Tf64 = dp.Tf64;
    P.Mf64 = dp.Mf64;
    P.Tf32 = dp.g32 ? dp.Tf32 : nullptr;
    P.g32 = dp.g32;
    P.g = dp.g;
    P.s0 = dp.s[0];
    P.s1 = dp.s[1];
    P.u0 = dp.u2[0];
    P.u1 = dp.u2[1];
    P.w_src = dp.has_src ? dp.w_src : nullptr;
    P.gbe = dp.has_src ? dp.gbe : nullptr;
    P.ctrl = dp.ctrl;
    P.counters = dp.counters;
    P.partials = dp.partials;
    P.hist = dp.hist;
    P.step_iters = dp.step_iters;
  }
  // the kernels only read the descriptors: skip an upload of what d_probs holds already
  if (b->probs_valid && std::memcmp(np.data(), b->probs.data(), np.size() * sizeof(BatchProblem)) == 0)
    return EHDG_OK;
  // the host copy is the source of an asynchronous upload: an earlier upload from it must
  // have completed before it is rewritten
  if (b->probs_valid) {
    if (b->probs_ev)
      HIP_TRY_B(b, hipEventSynchronize(b->probs_ev));
    else
      HIP_TRY_B(b, hipStreamSynchronize(b->stream));
  }
  b->probs.swap(np);
  HIP_TRY_B(b, hipMemcpyAsync(b->d_probs, b->probs.data(), b->probs.size() * sizeof(BatchProblem),
                              hipMemcpyHostToDevice, b->stream));
  if (!b->is_static) {  // static batches create no events
    if (!b->probs_ev) HIP_TRY_B(b, hipEventCreateWithFlags(&b->probs_ev, hipEventDisableTiming));
    HIP_TRY_B(b, hipEventRecord(b->probs_ev, b->stream));
  }
  b->probs_valid = true;
  return EHDG_OK;
}

// waits for the members' own streams, so no earlier work on a member is still queued;
// refuses a static batch whose tables a later static batch on its device has replaced
int batch_quiesce(ehdg_batch_s* b) {
  if (b->is_static) {
    {
      StaticScratch& ss = static_scratch();
      std::lock_guard<std::mutex> lk(ss.mu);
      if (ss.gen[b->dev] != b->gen)
        return bfail(b, EHDG_ERR_INVALID_ARG, "static batch replaced by a later ehdg_batch_create_static on its device");
    }
    for (auto* h : b->h) HIP_TRY_B(b, hipStreamSynchronize(h->stream));
    return EHDG_OK;
  }
  // the batch stream waits for what is queued on each other member stream (no host wait)
  std::vector<hipStream_t> seen;
  for (auto* h : b->h) {
    if (h->stream == b->stream || std::find(seen.begin(), seen.end(), h->stream) != seen.end()) continue;
    seen.push_back(h->stream);
    if (!b->join_ev) HIP_TRY_B(b, hipEventCreateWithFlags(&b->join_ev, hipEventDisableTiming));
    HIP_TRY_B(b, hipEventRecord(b->join_ev, h->stream));
    HIP_TRY_B(b, hipStreamWaitEvent(b->stream, b->join_ev, 0));
  }
  return EHDG_OK;
}

// records the batch's latest asynchronous work (the event destroy and uploads wait for)
int mark_last(ehdg_batch_s* b) {
  if (!b->last_ev) HIP_TRY_B(b, hipEventCreateWithFlags(&b->last_ev, hipEventDisableTiming));
  HIP_TRY_B(b, hipEventRecord(b->last_ev, b->stream));
  b->last_ev_set = true;
  return EHDG_OK;
}

int no_pending(ehdg_batch_s* b) {
  if (!b->pending.empty())
    return bfail(b, EHDG_ERR_INVALID_ARG, "launches of ehdg_batch_launch are pending: read them with ehdg_batch_poll");
  return EHDG_OK;
}

int batch_sync_ctrl(ehdg_batch_s* b) {
  launch_ctrl_gather(b->d_probs, (int)b->h.size(), b->d_ctrl, b->stream);
  HIP_TRY_B(b, hipMemcpyAsync(b->ctrl.data(), b->d_ctrl, b->ctrl.size() * sizeof(Ctrl), hipMemcpyDeviceToHost,
                              b->stream));
  HIP_TRY_B(b, hipStreamSynchronize(b->stream));
  return EHDG_OK;
}

// One round of the batch on stream st: a sweep of every member (the persistent sweep per
// precision, then the families it does not cover), then, if steps, the step completions.
void queue_round(ehdg_batch_s* b, double tol, bool steps, hipStream_t st) {
  for (int prec = 0; prec < 2; ++prec)
    launch_sweep_persist(b->d_table + b->persist_first[prec], b->persist_n[prec], b->d_probs, tol, prec, st);
  for (const auto& g : b->groups)
    if (g.sweep_n) (g.fp32 ? g.ks->sweep32_batch : g.ks->sweep64_batch)(b->d_table + g.sweep_first, g.sweep_n, b->d_probs, tol, st);
  if (steps)
    for (const auto& g : b->groups)
      if (g.step_n) (g.fp32 ? g.ks->step32_batch : g.ks->step_batch)(b->d_table + g.step_first, g.step_n, b->d_probs, 1, st);
}

void drop_graph(ehdg_batch_s* b) {
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  b->graph = nullptr;
  b->graph_rounds = 0;
}

// `rounds` rounds on the batch's stream, with the step completions after every round
// (steps = 1) or after the last one only (steps = 2), or none (0).  Graph mode: the rounds
// are captured once into a HIP graph (kernels only: every counter the kernels use is reset
// by the kernels themselves) and the graph is replayed `repeat` times, and again by later
// calls while the round count, the step mode and the tolerance stay the same.  Otherwise
// (static batches, a caller's stream that is being captured, or graphs switched off) the
// launches are queued one by one.
int run_rounds(ehdg_batch_s* b, int rounds, double tol, int steps, int repeat = 1) {
  if (rounds <= 0 || repeat <= 0) return EHDG_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (b->stream) (void)hipStreamIsCapturing(b->stream, &cs);
  if (!b->use_graph || cs != hipStreamCaptureStatusNone) {
    for (int q = 0; q < repeat; ++q)
      for (int r = 0; r < rounds; ++r) queue_round(b, tol, steps == 1 || (steps == 2 && r == rounds - 1), b->stream);
    return EHDG_OK;
  }
  if (!(b->graph && b->graph_rounds == rounds && b->graph_steps == steps && b->graph_tol == tol)) {
    drop_graph(b);
    if (!b->cap_stream) HIP_TRY_B(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    HIP_TRY_B(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int r = 0; r < rounds; ++r)
      queue_round(b, tol, steps == 1 || (steps == 2 && r == rounds - 1), b->cap_stream);
    hipGraph_t g = nullptr;
    HIP_TRY_B(b, hipStreamEndCapture(b->cap_stream, &g));
    const hipError_t e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      b->graph = nullptr;
      return bfail(b, EHDG_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    b->graph_rounds = rounds;
    b->graph_steps = steps;
    b->graph_tol = tol;
  }
  for (int q = 0; q < repeat; ++q) HIP_TRY_B(b, hipGraphLaunch(b->graph, b->stream));
  return EHDG_OK;
}

int batch_check_launch(ehdg_batch_s* b) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return bfail(b, EHDG_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return EHDG_OK;
}

}  // namespace

extern "C" {

int ehdg_batch_workspace_bytes(const ehdg_handle* handles, int32_t n, size_t* bytes) {
  if (!bytes) return EHDG_ERR_INVALID_ARG;
  std::vector<ehdg_problem*> hs;
  int rc = batch_check(handles, n, hs);
  if (rc) return rc;
  std::vector<ehdg_batch_s::Group> groups;
  std::vector<BatchEntry> table;
  int pf[2], pn[2];
  batch_plan(hs, groups, table, pf, pn);
  *bytes = batch_layout(hs.size(), table.size()).total;
  return EHDG_OK;
}

}  // extern "C"

namespace {

// ehdg_batch_create's work with the tables at d_workspace (256-byte aligned, bytes long)
int batch_create_in(std::vector<ehdg_problem*>& hs, void* d_workspace, size_t workspace_bytes, void* stream,
                    ehdg_batch_s** out, bool in_static) {
  ehdg_batch_s* b = new (std::nothrow) ehdg_batch_s();
  if (!b) return EHDG_ERR_INVALID_ARG;
  b->h = hs;
  b->stream = (hipStream_t)stream;
  std::vector<BatchEntry> table;
  batch_plan(hs, b->groups, table, b->persist_first, b->persist_n, false);  // per-family launches by default
  const BatchLayout L = batch_layout(hs.size(), table.size());
  if (workspace_bytes < L.total) {
    delete b;
    return EHDG_ERR_WORKSPACE_TOO_SMALL;
  }
  char* ws = (char*)d_workspace;
  b->d_probs = (BatchProblem*)(ws + L.off_probs);
  b->d_table = (BatchEntry*)(ws + L.off_table);
  b->d_ctrl = (Ctrl*)(ws + L.off_ctrl);
  b->probs.assign(hs.size(), BatchProblem{});
  b->ctrl.assign(hs.size(), Ctrl{});
  b->polled.assign(hs.size(), -1);
  b->table_host.swap(table);
  // asynchronous upload from table_host, which lives until destroy (destroy waits for it);
  // static batches create no events: their upload completes here
  if (hipMemcpyAsync(b->d_table, b->table_host.data(), b->table_host.size() * sizeof(BatchEntry),
                     hipMemcpyHostToDevice, b->stream) != hipSuccess ||
      (in_static ? hipStreamSynchronize(b->stream) != hipSuccess : mark_last(b) != EHDG_OK)) {
    if (b->last_ev) (void)hipEventDestroy(b->last_ev);
    delete b;
    return EHDG_ERR_HIP;
  }
  *out = b;
  return EHDG_OK;
}

}  // namespace

extern "C" {

int ehdg_batch_create(const ehdg_handle* handles, int32_t n, void* d_workspace, size_t workspace_bytes, void* stream,
                      ehdg_batch* out) {
  if (!out) return EHDG_ERR_INVALID_ARG;
  *out = nullptr;
  std::vector<ehdg_problem*> hs;
  int rc = batch_check(handles, n, hs);
  if (rc) return rc;
  if (!d_workspace || ((uintptr_t)d_workspace & 255)) return EHDG_ERR_INVALID_ARG;
  return batch_create_in(hs, d_workspace, workspace_bytes, stream, out, false);
}

int ehdg_batch_create_static(const ehdg_handle* handles, int32_t n, void* stream, ehdg_batch* out) {
  if (!out) return EHDG_ERR_INVALID_ARG;
  *out = nullptr;
  std::vector<ehdg_problem*> hs;
  int rc = batch_check(handles, n, hs);
  if (rc) return rc;
  {
    std::vector<ehdg_batch_s::Group> groups;
    std::vector<BatchEntry> table;
    int pf[2], pn[2];
    batch_plan(hs, groups, table, pf, pn);
    if (batch_layout(hs.size(), table.size()).total > kStaticBatchBytes) return EHDG_ERR_WORKSPACE_TOO_SMALL;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return EHDG_ERR_HIP;
  StaticScratch& ss = static_scratch();
  void* ptr = nullptr;
  unsigned gen = 0;
  {
    std::lock_guard<std::mutex> lk(ss.mu);
    if (!ss.ptr[dev]) {
      // once per device, with that device current: the device address of its copy
      void* p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return EHDG_ERR_HIP;
      ss.ptr[dev] = p;
    }
    ptr = ss.ptr[dev];
    gen = ++ss.gen[dev];  // any earlier static batch on this device is now replaced
  }
  rc = batch_create_in(hs, ptr, kStaticBatchBytes, stream, out, true);
  if (rc) return rc;
  (*out)->is_static = true;
  (*out)->use_graph = false;  // graph instantiation allocates: static batches launch eagerly
  (*out)->dev = dev;
  (*out)->gen = gen;
  return EHDG_OK;
}

int ehdg_batch_solve(ehdg_batch b, double rel_tol, int32_t max_iters, int32_t* iters, double* rel_res) {
  if (!b || max_iters < 1 || !(rel_tol >= 0.0)) return EHDG_ERR_INVALID_ARG;
  const size_t n = b->h.size();
  int rc = no_pending(b);
  if (!rc) rc = batch_quiesce(b);
  if (!rc) rc = batch_upload(b, std::vector<int>(n, INT32_MAX));
  if (rc) return rc;
  launch_ctrl_reset_batch(b->d_probs, (int)n, 0, b->stream);
  int pred = 1;
  for (auto* h : b->h) pred = std::max(pred, h->predict);
  int launched = 0, chunk = pred, next = 2;
  for (;;) {
    const int nq = std::min(chunk, max_iters - launched);
    if ((rc = run_rounds(b, nq, rel_tol, 0))) return rc;
    launched += nq;
    if ((rc = batch_check_launch(b)) || (rc = batch_sync_ctrl(b))) return rc;
    bool all = true;
    for (const Ctrl& c : b->ctrl) all = all && c.done;
    if (all || launched >= max_iters) break;
    chunk = next;
    next = std::min(next * 2, 64);
  }
  int first_bad = EHDG_OK;
  for (size_t i = 0; i < n; ++i) {
    ehdg_problem* h = b->h[i];
    h->mirror = b->ctrl[i];
    const Ctrl& c = h->mirror;
    if (iters) iters[i] = c.iters;
    if (rel_res) rel_res[i] = c.last_res;
    if (c.status == 1) h->predict = c.iters;
    const int st = c.status == 2 ? EHDG_ERR_DIVERGED : (c.status == 1 ? EHDG_OK : EHDG_ERR_NOT_CONVERGED);
    if (st && !first_bad) first_bad = st;
    h->recovered = -1;
    if (c.iters > 0 && c.status != 2) {
      recover(h, (c.base + c.iters - 1) & 1, b->stream);
      h->recovered = 1;
    }
  }
  if ((rc = batch_check_launch(b))) return rc;
  HIP_TRY_B(b, hipStreamSynchronize(b->stream));
  if (first_bad) b->err = first_bad == EHDG_ERR_DIVERGED ? "a member diverged" : "a member reached the cap";
  return first_bad;
}

int ehdg_batch_step(ehdg_batch b, int32_t n_steps, double rel_tol, int32_t max_iters_per_step,
                    int32_t* iters_per_step) {
  if (!b || n_steps < 0 || max_iters_per_step < 1 || !(rel_tol >= 0.0)) return EHDG_ERR_INVALID_ARG;
  for (auto* h : b->h)
    if (!h->dp.be) return bfail(b, EHDG_ERR_INVALID_ARG, "ehdg_batch_step needs backward-Euler members");
  if (n_steps == 0) return EHDG_OK;
  const size_t n = b->h.size();
  int rc = no_pending(b);
  if (!rc) rc = batch_quiesce(b);
  if (rc) return rc;
  // the first step of each member continues from its latest state
  if ((rc = batch_upload(b, std::vector<int>(n, INT32_MAX)))) return rc;
  launch_ctrl_reset_batch(b->d_probs, (int)n, 0, b->stream);
  if ((rc = batch_sync_ctrl(b))) return rc;
  std::vector<int> first(n), target(n);
  for (size_t i = 0; i < n; ++i) {
    first[i] = b->ctrl[i].steps_done;
    target[i] = first[i] + n_steps;
  }
  if ((rc = batch_upload(b, target))) return rc;
  int pred = 1;
  for (auto* h : b->h) pred = std::max(pred, h->predict);
  const int max_outer = max_iters_per_step;
  int status = EHDG_OK;
  // per member, the sweep counts of its steps completed in this call, read back after
  // every round (a round queues at most kStepCap steps, so no ring wraps onto unread counts)
  std::vector<std::vector<int>> counts(n);
  for (;;) {
    int remaining = 0;
    for (size_t i = 0; i < n; ++i) remaining = std::max(remaining, target[i] - b->ctrl[i].steps_done);
    if (remaining <= 0) break;
    remaining = std::min(remaining, kStepCap);
    std::vector<int> before(n);
    for (size_t i = 0; i < n; ++i) before[i] = b->ctrl[i].steps_done;
    const int per = std::min(pred + 1, max_outer);
    if ((rc = run_rounds(b, per, rel_tol, 2, remaining))) return rc;
    if ((rc = batch_check_launch(b)) || (rc = batch_sync_ctrl(b))) return rc;
    for (size_t i = 0; i < n; ++i) {
      const int fresh = b->ctrl[i].steps_done - before[i];
      if (fresh <= 0) continue;
      counts[i].resize(counts[i].size() + fresh);
      if ((rc = read_step_counts(b->h[i], b->h[i]->dp.step_iters, before[i], fresh,
                                 counts[i].data() + counts[i].size() - fresh)))
        return bfail(b, rc, b->h[i]->err);
    }
    bool stuck = false;
    for (size_t i = 0; i < n; ++i) {
      const Ctrl& c = b->ctrl[i];
      if (c.status == 2) status = EHDG_ERR_DIVERGED;
      if (c.steps_done < target[i] && c.iters >= max_outer) stuck = true;
    }
    if (status) break;
    if (stuck) {
      status = EHDG_ERR_NOT_CONVERGED;
      break;
    }
    pred = std::min(2 * pred, max_outer);  // a round that left steps undone queued too few sweeps
  }
  for (size_t i = 0; i < n; ++i) {
    ehdg_problem* h = b->h[i];
    h->mirror = b->ctrl[i];
    h->recovered = -1;
    const int done = h->mirror.steps_done - first[i];
    const std::vector<int>& its = counts[i];
    int mx = 1;
    for (int v : its) mx = std::max(mx, v);
    h->predict = mx;
    if (iters_per_step)
      for (int k = 0; k < n_steps; ++k) iters_per_step[i * n_steps + k] = k < (int)its.size() ? its[k] : 0;
    if (!status && done < n_steps) status = EHDG_ERR_NOT_CONVERGED;
  }
  if (status) b->err = status == EHDG_ERR_DIVERGED ? "a member diverged" : "a member did not finish its steps";
  return status;
}

int ehdg_batch_advance(ehdg_batch b, int32_t rounds, double rel_tol, const int32_t* step_targets, int32_t* state) {
  if (!b || rounds < 0 || !(rel_tol >= 0.0) || !state) return EHDG_ERR_INVALID_ARG;
  const size_t n = b->h.size();
  int rc = no_pending(b);
  if (!rc) rc = batch_quiesce(b);
  if (rc) return rc;
  std::vector<int> target(n, INT32_MAX);
  bool any_be = false;
  for (size_t i = 0; i < n; ++i) {
    if (!b->h[i]->dp.be) continue;
    any_be = true;
    target[i] = step_targets ? step_targets[i] : b->h[i]->mirror.steps_done + 1;
  }
  if ((rc = batch_upload(b, target))) return rc;
  if ((rc = run_rounds(b, rounds, rel_tol, any_be ? 1 : 0))) return rc;
  if ((rc = batch_check_launch(b)) || (rc = batch_sync_ctrl(b))) return rc;
  for (size_t i = 0; i < n; ++i) {
    ehdg_problem* h = b->h[i];
    h->mirror = b->ctrl[i];
    h->recovered = -1;
    const Ctrl& c = h->mirror;
    if (c.status == 2)
      state[i] = 2;
    else if (h->dp.be)
      state[i] = c.steps_done >= target[i] ? 1 : 0;
    else
      state[i] = c.status == 1 ? 1 : 0;
    b->polled[i] = state[i];
  }
  return EHDG_OK;
}

}  // extern "C"

namespace {
// state of member i in a control block: 2 non-finite increment, 1 finished (converged, or
// took `target` steps for a backward-Euler member), 0 running
int member_state(const ehdg_problem* h, const Ctrl& c, int target) {
  if (c.status == 2) return 2;
  if (h->dp.be) return c.steps_done >= target ? 1 : 0;
  return c.status == 1 ? 1 : 0;
}
}  // namespace

extern "C" {

int ehdg_batch_report_bytes(ehdg_batch b, size_t* bytes) {
  if (!b || !bytes) return EHDG_ERR_INVALID_ARG;
  *bytes = b->h.size() * sizeof(Ctrl);
  return EHDG_OK;
}

int ehdg_batch_launch(ehdg_batch b, int32_t rounds, double rel_tol, const int32_t* step_targets, void* h_report,
                      size_t report_bytes) {
  if (!b || rounds < 1 || !(rel_tol >= 0.0) || !h_report) return EHDG_ERR_INVALID_ARG;
  const size_t n = b->h.size();
  if (report_bytes < n * sizeof(Ctrl)) return bfail(b, EHDG_ERR_INVALID_ARG, "report buffer smaller than ehdg_batch_report_bytes");
  if ((int)b->pending.size() >= ehdg_batch_s::kMaxPending)
    return bfail(b, EHDG_ERR_INVALID_ARG, "four launches pending: read one with ehdg_batch_poll first");
  for (const auto& p : b->pending)
    if ((const void*)p.report == h_report)
      return bfail(b, EHDG_ERR_INVALID_ARG, "report buffer in use by a pending launch");
  std::vector<int> target(n, INT32_MAX);
  bool any_be = false;
  for (size_t i = 0; i < n; ++i) {
    if (!b->h[i]->dp.be) continue;
    if (!step_targets) return bfail(b, EHDG_ERR_INVALID_ARG, "backward-Euler members need step targets");
    any_be = true;
    target[i] = step_targets[i];
  }
  int rc = batch_quiesce(b);
  if (!rc) rc = batch_upload(b, target);
  if (!rc) rc = run_rounds(b, rounds, rel_tol, any_be ? 1 : 0);
  if (rc) return rc;
  const int slot = (int)(b->launches % ehdg_batch_s::kMaxPending);
  if (!b->ev[slot]) HIP_TRY_B(b, hipEventCreateWithFlags(&b->ev[slot], hipEventDisableTiming));
  launch_ctrl_gather(b->d_probs, (int)n, b->d_ctrl, b->stream);
  HIP_TRY_B(b, hipMemcpyAsync(h_report, b->d_ctrl, n * sizeof(Ctrl), hipMemcpyDeviceToHost, b->stream));
  HIP_TRY_B(b, hipEventRecord(b->ev[slot], b->stream));
  if ((rc = mark_last(b)) || (rc = batch_check_launch(b))) return rc;
  b->pending.push_back({slot, (const Ctrl*)h_report, std::move(target)});
  ++b->launches;
  return EHDG_OK;
}

int ehdg_batch_poll(ehdg_batch b, int32_t* state, int32_t* ready) {
  if (!b || !ready) return EHDG_ERR_INVALID_ARG;
  *ready = 0;
  if (b->pending.empty()) return bfail(b, EHDG_ERR_INVALID_ARG, "no launch pending");
  const ehdg_batch_s::Pending& p = b->pending.front();
  const hipError_t e = hipEventQuery(b->ev[p.slot]);
  if (e == hipErrorNotReady) {
    (void)hipGetLastError();  // not an error: leave no trace for later launch checks
    return EHDG_OK;
  }
  if (e != hipSuccess) return bfail(b, EHDG_ERR_HIP, std::string("hipEventQuery: ") + hipGetErrorString(e));
  for (size_t i = 0; i < b->h.size(); ++i) {
    ehdg_problem* h = b->h[i];
    const int st = member_state(h, p.report[i], p.target[i]);
    // a finished member keeps its state (later rounds leave it), and with it its recovery
    if (!(b->polled[i] == 1 && st == 1)) h->recovered = -1;
    h->mirror = p.report[i];
    b->polled[i] = st;
    if (state) state[i] = st;
  }
  b->pending.pop_front();
  *ready = 1;
  return EHDG_OK;
}

int ehdg_batch_get_solution(ehdg_batch b, int32_t member, double* d_u) {
  if (!b || !d_u || member < 0 || member >= (int32_t)b->h.size()) return EHDG_ERR_INVALID_ARG;
  if (b->polled[member] != 1)
    return bfail(b, EHDG_ERR_INVALID_ARG, "member not reported finished by the last report read");
  queue_solution(b->h[member], d_u, b->stream);
  int rc = batch_check_launch(b);
  if (!rc && !b->is_static) rc = mark_last(b);
  return rc;
}

int ehdg_batch_set_graph(ehdg_batch b, int32_t enabled) {
  if (!b) return EHDG_ERR_INVALID_ARG;
  if (enabled && b->is_static) return bfail(b, EHDG_ERR_UNSUPPORTED, "static batches launch without graphs");
  b->use_graph = enabled != 0;
  if (!b->use_graph) drop_graph(b);
  return EHDG_OK;
}

int ehdg_batch_set_persistent(ehdg_batch b, int32_t enabled) {
  if (!b) return EHDG_ERR_INVALID_ARG;
  int rc = no_pending(b);
  if (rc) return rc;
  std::vector<ehdg_batch_s::Group> groups;
  std::vector<BatchEntry> table;
  int pf[2], pn[2];
  batch_plan(b->h, groups, table, pf, pn, enabled != 0);
  if (table.size() != b->table_host.size()) return bfail(b, EHDG_ERR_INVALID_ARG, "table size changed");
  // the table's host copy may be the source of a pending upload
  if (b->last_ev_set)
    HIP_TRY_B(b, hipEventSynchronize(b->last_ev));
  else
    HIP_TRY_B(b, hipStreamSynchronize(b->stream));
  b->table_host.swap(table);
  b->groups.swap(groups);
  for (int q = 0; q < 2; ++q) {
    b->persist_first[q] = pf[q];
    b->persist_n[q] = pn[q];
  }
  HIP_TRY_B(b, hipMemcpyAsync(b->d_table, b->table_host.data(), b->table_host.size() * sizeof(BatchEntry),
                              hipMemcpyHostToDevice, b->stream));
  if (b->is_static)
    HIP_TRY_B(b, hipStreamSynchronize(b->stream));
  else if ((rc = mark_last(b)))
    return rc;
  drop_graph(b);
  return EHDG_OK;
}

int ehdg_batch_destroy(ehdg_batch b) {
  if (!b) return EHDG_ERR_INVALID_ARG;
  // the batch's own queued work (launches, uploads from its host copies) ends first
  if (b->last_ev_set) (void)hipEventSynchronize(b->last_ev);
  drop_graph(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  for (auto& e : b->ev)
    if (e) (void)hipEventDestroy(e);
  if (b->join_ev) (void)hipEventDestroy(b->join_ev);
  if (b->probs_ev) (void)hipEventDestroy(b->probs_ev);
  if (b->last_ev) (void)hipEventDestroy(b->last_ev);
  delete b;
  return EHDG_OK;
}

const char* ehdg_batch_last_error(ehdg_batch b) { return b ? b->err.c_str() : "null batch"; }

const char* ehdg_error_string(int code) {
  switch (code) {
    case EHDG_OK: return "ok";
    case EHDG_ERR_INVALID_ARG: return "invalid argument";
    case EHDG_ERR_UNSUPPORTED: return "unsupported problem";
    case EHDG_ERR_HIP: return "HIP runtime error";
    case EHDG_ERR_NOT_CONVERGED: return "not converged within the iteration cap";
    case EHDG_ERR_DIVERGED: return "iteration diverged";
    case EHDG_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
  }
  return "unknown error";
}

const char* ehdg_last_error(ehdg_handle h) { return h ? h->err.c_str() : "null handle"; }

}  // extern "C"
