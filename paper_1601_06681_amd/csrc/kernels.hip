// HIP kernels of the eHDG iteration for gfx950 (MI355X).
//
// One eHDG sweep (Algorithm 1: independent local solves with the previous traces, then
// new traces) is, in trace form, per element e
//     s_out[e] = g[e] + T in_e(s_in),
// where in_e gathers the element's own and its face neighbours' trace data and T is the
// condensed local operator shared by every element of a uniform mesh (Sec. 3).
//   * Layout.  State arrays are component-major (SoA): component k of element e at
//     [k * n_el + e], so 16 consecutive elements read and write 128 contiguous bytes per
//     component, and face neighbours (e +- 1, e +- n0, e +- n0 n1) are contiguous runs.
//   * Matrix cores.  Elements are taken in tiles of 16: the tile's gathered inputs are
//     the B operand and T the A operand of v_mfma_f64_16x16x4f64 (FP64) or
//     v_mfma_f32_16x16x4f32 (FP32 forms).  Each wavefront keeps its row block of T in
//     registers for the whole launch (fragment-major copy made at set-up), so T is read
//     once per wavefront, not per element.  Large operators split the rows over the
//     waves of a workgroup and share the gathered tile through LDS, double-buffered so
//     the next tile's gather overlaps the current tile's products.
//   * Launch shape.  One round of resident workgroups, each over a contiguous range of
//     tiles (or a tuned tiles-per-workgroup count and order); workgroup ids are remapped
//     so each of the 8 XCDs sweeps a contiguous slab and neighbour re-reads hit its own
//     L2.
//   * Stopping test.  Single-problem sweeps take a lagged test: each sweep leaves
//     per-workgroup partial sums of its increment and takes the previous sweep's test
//     from the other partial set, summed in a canonical order, so no workgroup waits for
//     another; batched sweeps reduce with the last workgroup to arrive.  Either raises a
//     device-side done flag that makes queued sweeps exit at once.
//   * Batches.  Problems of one family share a launch through a (problem, tile range)
//     table; a persistent kernel strides over the table of every 2D transport and
//     shallow-water member, dispatching each entry to its family's sweep.
//   * Also here: the step completion of backward Euler (stacked recovery and next
//     right-hand side), the refinement forms (FP64 residual on s', FP32 / BF16
//     corrections), the variable-velocity sweep (per-element operators streamed from
//     HBM), and the set-up kernels (per-element products with a shared matrix staged
//     through LDS, tiled layout transposes).
#include "kernels.h"

#include <algorithm>
#include <cmath>
#include <type_traits>

namespace ehdg {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int remap_block(int b, int nb) {
  // blocks are dispatched round-robin over the 8 XCDs (block i -> XCD i % 8);
  // give XCD x the contiguous logical range it would own in a blocked split
  const int xcd = b & 7, idx = b >> 3;
  const int per = nb >> 3, rem = nb & 7;
  return xcd * per + min(xcd, rem) + idx;
}

// element coordinates (i0, i1, i2) of e
struct Ijk {
  int c0, c1, c2;
};

__device__ __forceinline__ Ijk coords(const MeshDev& m, int e) {
  Ijk c;
  c.c0 = e % m.n[0];
  const int r = e / m.n[0];
  c.c1 = r % m.n[1];
  c.c2 = r / m.n[1];
  return c;
}

__device__ __forceinline__ int sel3(int a0, int a1, int a2, int i) {
  return a0 * (int)(i == 0) + a1 * (int)(i == 1) + a2 * (int)(i == 2);
}

// neighbour of e one step along `axis` (wrapping on periodic axes), -1 outside.
// Written with selects: indexing a register array by a runtime axis would move it to scratch.
__device__ __forceinline__ int neighbour(const MeshDev& m, int e, const Ijk& c, int axis, int step) {
  const int ci = sel3(c.c0, c.c1, c.c2, axis);
  const int ni = sel3(m.n[0], m.n[1], m.n[2], axis);
  const int per = sel3(m.periodic[0], m.periodic[1], m.periodic[2], axis);
  const int stride = sel3(1, m.n[0], m.n[0] * m.n[1], axis);
  const int v = ci + step;
  const bool out = v < 0 || v >= ni;
  const int vw = v < 0 ? v + ni : (v >= ni ? v - ni : v);  // wrapped on a periodic axis
  const int n = e + (vw - ci) * stride;
  return (out && !per) ? -1 : n;
}

// Index of the wavefront within the workgroup.
__device__ __forceinline__ int wave_id() { return (int)(threadIdx.x >> 6); }

// A wave-uniform value as an SGPR: operator rows addressed through it are fetched
// with scalar loads (applied where the value is used, since a value that is merely
// known to be uniform may still be kept in a vector register).
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// done, iters, base and status of the control block in one 16-byte load
struct CtrlHead {
  int done, iters, base, status;
};
__device__ __forceinline__ CtrlHead ctrl_head(const Ctrl* c) {
  const int4 v = *reinterpret_cast<const int4*>(c);
  return {v.x, v.y, v.z, v.w};
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);                                             // round to nearest even
  return (uint16_t)(u >> 16);
}

// loaders: value of state row r of element e, per storage layout and precision
struct Ld64 {  // FP64, component-major
  const double* p;
  size_t nel;
  __device__ __forceinline__ double operator()(int r, int e) const { return p[(size_t)r * nel + e]; }
};
struct Ld32 {  // FP32, component-major
  const float* p;
  size_t nel;
  __device__ __forceinline__ float operator()(int r, int e) const { return p[(size_t)r * nel + e]; }
};
template <int S>
struct Ld16Aos {  // BF16, element-major: the S values of an element are contiguous
  const uint16_t* p;
  __device__ __forceinline__ float operator()(int r, int e) const { return bf16_to_f32(p[(size_t)e * S + r]); }
};
template <int S>
struct Ld32Aos {  // FP32, element-major
  const float* p;
  __device__ __forceinline__ float operator()(int r, int e) const { return p[(size_t)e * S + r]; }
};
// loader of a component-major state of element type ST (double or float)
template <typename ST>
using LdOf = std::conditional_t<std::is_same_v<ST, float>, Ld32, Ld64>;

// FP64 iterate plus a low-precision correction: s + delta (delta ignored unless use)
template <class LD>
struct LdSum {
  Ld64 s;
  LD d;
  int use;
  __device__ __forceinline__ double operator()(int r, int e) const {
    const double v = s(r, e);
    return use ? v + (double)d(r, e) : v;
  }
};

// point a loader's FP64 state at the buffer chosen on the device
__device__ __forceinline__ void set_state(Ld64& l, const double* p, int) { l.p = p; }
template <class LD>
__device__ __forceinline__ void set_state(LdSum<LD>& l, const double* p, int use) {
  l.s.p = p;
  l.use = use;
}

template <typename T>
__device__ __forceinline__ T fmadd(T a, T b, T c) { return fma(a, b, c); }

// ---------------------------------------------------------------------------
// gathers: in_e(s) for each problem family, one input row at a time
// ---------------------------------------------------------------------------
// A workgroup owns kLanes consecutive elements (one per lane).  Input row c of all
// its elements is read by one wavefront, so every row read is a contiguous run of
// the component-major state (coalesced), then staged in LDS for the contraction.
constexpr int kLanes = kElemsPerGroup;
constexpr int kWaves = kRowGroups;
constexpr int kThreads = kLanes * kWaves;

// neighbour indices of one element, kept in named registers.  get() selects by a
// mask-weighted sum: a select chain over the fields may be folded into an indexed
// load from a stack copy, which would live in scratch memory.
struct Nb {
  int n0 = -1, n1 = -1, n2 = -1, n3 = -1;
  __device__ __forceinline__ int get(int i) const {
    return n0 * (int)(i == 0) + n1 * (int)(i == 1) + n2 * (int)(i == 2) + n3 * (int)(i == 3);
  }
};

// Transport, NA active axes, P1 = p + 1.  State per element: the outflow-face
// values of each active axis (row t*NF + k).  Inputs: rows [0, NA*NF) are the
// inflow faces, i.e. the upwind neighbour's state rows (0 on an inflow boundary,
// whose data is folded into g); rows [NA*NF, 2*NA*NF) are the element's own state.
// The upwind trace (eq. transportLocale) is the upwind element's value, so the
// gather is pure data movement.
template <int DIM, int NA, int P1>
struct TransportFam {
  static constexpr int NF = DIM == 2 ? P1 : P1 * P1;
  static constexpr int NP = DIM == 2 ? P1 * P1 : P1 * P1 * P1;
  static constexpr int S = NA * NF, I = 2 * NA * NF, N = NP;
  __device__ __forceinline__ static void neighbours(const MeshDev& m, int e, Nb& nb) {
    const Ijk c = coords(m, e);
    if (NA > 0) nb.n0 = neighbour(m, e, c, m.ax[0], -m.dir[0]);
    if (NA > 1) nb.n1 = neighbour(m, e, c, m.ax[1], -m.dir[1]);
    if (NA > 2) nb.n2 = neighbour(m, e, c, m.ax[2], -m.dir[2]);
  }
  // e must be a valid element index (callers pass a stand-in for idle lanes): the
  // load is unconditional, so the loads of all rows of a wavefront can be in flight
  // together, and only the value is selected
  template <class LD>
  __device__ __forceinline__ static auto row(const MeshDev& m, int e, const Nb& nb, const LD& ld, int c)
      -> decltype(ld(0, 0)) {
    using V = decltype(ld(0, 0));
    const bool up = c < NA * NF;
    const int n = nb.get(c / NF);
    const bool inflow_bc = up && n < 0;
    const V v = ld(up ? c : c - NA * NF, (up && n >= 0) ? n : e);
    return inflow_bc ? V(0) : v;
  }
  // row() in two parts: the loads, and the combination (which needs only indices), so
  // that a caller can keep the loads in flight across other work
  template <class LD>
  __device__ __forceinline__ static void row_load(const MeshDev&, int e, const Nb& nb, const LD& ld, int c,
                                                  decltype(ld(0, 0))& x, decltype(ld(0, 0))& y) {
    const bool up = c < NA * NF;
    const int n = nb.get(c / NF);
    x = ld(up ? c : c - NA * NF, (up && n >= 0) ? n : e);
    y = x;
  }
  template <class V>
  __device__ __forceinline__ static V row_combine(const Nb& nb, int c, V x, V) {
    const bool inflow_bc = c < NA * NF && nb.get(c / NF) < 0;
    return inflow_bc ? V(0) : x;
  }
  // (state row, element) of row_load's two loads
  __device__ __forceinline__ static void row_index(const Nb& nb, int e, int c, int& rx, int& ex, int& ry, int& ey) {
    const bool up = c < NA * NF;
    const int n = nb.get(c / NF);
    rx = up ? c : c - NA * NF;
    ex = (up && n >= 0) ? n : e;
    ry = rx;
    ey = ex;
  }
  // input column of the element's own state row 0 (row r is column kOwnCol + r; row_load's
  // x is its raw value); kOwnRaw: the combined input of such a column is that raw value
  static constexpr int kOwnCol = NA * NF;
  static constexpr bool kOwnRaw = true;
};

// Shallow water, P1 = p + 1.  State per element side f: c_f = (phi + sqrt(Phi)
// vel.n_f) / 2 at the face nodes (row f*NF + k).  Input row f*NF + k: the trace
// phihat = c_own + c_neighbour (the trace formula below the local solver in
// Section 3); on a wall phihat = phi + sqrt(Phi) vel.n = 2 c_own.
template <int P1>
struct SweFam {
  static constexpr int NF = P1, NP = P1 * P1;
  static constexpr int S = 4 * NF, I = 4 * NF, N = 3 * NP;
  __device__ __forceinline__ static void neighbours(const MeshDev& m, int e, Nb& nb) {
    const Ijk c = coords(m, e);
    nb.n0 = neighbour(m, e, c, 0, -1);
    nb.n1 = neighbour(m, e, c, 0, 1);
    nb.n2 = neighbour(m, e, c, 1, -1);
    nb.n3 = neighbour(m, e, c, 1, 1);
  }
  template <class LD>
  __device__ __forceinline__ static auto row(const MeshDev& m, int e, const Nb& nb, const LD& ld, int c)
      -> decltype(ld(0, 0)) {
    decltype(ld(0, 0)) own;
    return row_parts(m, e, nb, ld, c, own);
  }
  // input row c and, separately, the element's own state row c (S == I)
  template <class LD>
  __device__ __forceinline__ static auto row_parts(const MeshDev& m, int e, const Nb& nb, const LD& ld, int c,
                                                   decltype(ld(0, 0))& own) -> decltype(ld(0, 0)) {
    const int f = c / NF, k = c - f * NF;
    const int n = nb.get(f);
    own = ld(c, e);
    const auto other = ld((f ^ 1) * NF + k, n >= 0 ? n : e);  // unconditional, in bounds
    return own + (n >= 0 ? other : own);
  }
  template <class LD>
  __device__ __forceinline__ static void row_load(const MeshDev&, int e, const Nb& nb, const LD& ld, int c,
                                                  decltype(ld(0, 0))& x, decltype(ld(0, 0))& y) {
    const int f = c / NF, k = c - f * NF;
    const int n = nb.get(f);
    x = ld(c, e);
    y = ld((f ^ 1) * NF + k, n >= 0 ? n : e);
  }
  template <class V>
  __device__ __forceinline__ static V row_combine(const Nb& nb, int c, V own, V other) {
    return own + (nb.get(c / NF) >= 0 ? other : own);
  }
  __device__ __forceinline__ static void row_index(const Nb& nb, int e, int c, int& rx, int& ex, int& ry, int& ey) {
    const int f = c / NF, k = c - f * NF;
    const int n = nb.get(f);
    rx = c;
    ex = e;
    ry = (f ^ 1) * NF + k;
    ey = n >= 0 ? n : e;
  }
  static constexpr int kOwnCol = 0;
  static constexpr bool kOwnRaw = false;  // the input is the trace c_own + c_neighbour
};

// Linearized Euler, P1 = p + 1.  State per element side f: the outgoing part
// c_f = (I + S_f)/2 w of the 4-vector w = (rho', u', v', p') at the face nodes,
// row (4 f + field) NF + k.  Input row of face f: the trace what = c_own +
// c_neighbour (the conservation condition of the upwind flux); on a boundary
// without incoming waves what = c_own.
template <int P1>
struct EulerFam {
  static constexpr int NF = P1, NP = P1 * P1;
  static constexpr int S = 16 * NF, I = 16 * NF, N = 4 * NP;
  __device__ __forceinline__ static void neighbours(const MeshDev& m, int e, Nb& nb) {
    const Ijk c = coords(m, e);
    nb.n0 = neighbour(m, e, c, 0, -1);
    nb.n1 = neighbour(m, e, c, 0, 1);
    nb.n2 = neighbour(m, e, c, 1, -1);
    nb.n3 = neighbour(m, e, c, 1, 1);
  }
  template <class LD>
  __device__ __forceinline__ static auto row(const MeshDev& m, int e, const Nb& nb, const LD& ld, int c)
      -> decltype(ld(0, 0)) {
    decltype(ld(0, 0)) own;
    return row_parts(m, e, nb, ld, c, own);
  }
  template <class LD>
  __device__ __forceinline__ static auto row_parts(const MeshDev& m, int e, const Nb& nb, const LD& ld, int c,
                                                   decltype(ld(0, 0))& own) -> decltype(ld(0, 0)) {
    using V = decltype(ld(0, 0));
    const int f = c / (4 * NF), rem = c - f * 4 * NF;
    const int n = nb.get(f);
    own = ld(c, e);
    const V other = ld((f ^ 1) * 4 * NF + rem, n >= 0 ? n : e);  // unconditional, in bounds
    return own + (n >= 0 ? other : V(0));
  }
  template <class LD>
  __device__ __forceinline__ static void row_load(const MeshDev&, int e, const Nb& nb, const LD& ld, int c,
                                                  decltype(ld(0, 0))& x, decltype(ld(0, 0))& y) {
    const int f = c / (4 * NF), rem = c - f * 4 * NF;
    const int n = nb.get(f);
    x = ld(c, e);
    y = ld((f ^ 1) * 4 * NF + rem, n >= 0 ? n : e);
  }
  template <class V>
  __device__ __forceinline__ static V row_combine(const Nb& nb, int c, V own, V other) {
    return own + (nb.get(c / (4 * NF)) >= 0 ? other : V(0));
  }
  __device__ __forceinline__ static void row_index(const Nb& nb, int e, int c, int& rx, int& ex, int& ry, int& ey) {
    const int f = c / (4 * NF), rem = c - f * 4 * NF;
    const int n = nb.get(f);
    rx = c;
    ex = e;
    ry = (f ^ 1) * 4 * NF + rem;
    ey = n >= 0 ? n : e;
  }
  static constexpr int kOwnCol = 0;
  static constexpr bool kOwnRaw = false;  // the input is the trace c_own + c_neighbour
};

// ---------------------------------------------------------------------------
// residual reduction (FP64, deterministic)
// ---------------------------------------------------------------------------
struct ResidArgs {
  Ctrl* ctrl;
  unsigned* cnt;  // arrival counter set
  double* partials;
  double* hist;
  int hist_cap;
  double tol;
  int stop;  // 1: set done on tol or non-finite; 0: record only
};

// Two-level arrival count of workgroup b of nb: the workgroups are split into G =
// kCounterGroups groups (b mod G; with G a multiple of 8 each group's workgroups run on
// one XCD) counting on their own counter; the last arrival of each group then counts on
// the counter of finished groups.  Returns true for the last workgroup overall, which
// resets the counters.  The caller completes (waits for) every store the last
// workgroup must see before arriving.
__device__ bool arrive_last(unsigned* cnt, int b, int nb) {
  constexpr int G = kCounterGroups;
  const int grp = b % G;
  const int size = nb / G + (grp < nb % G ? 1 : 0);
  const unsigned prev =
      __hip_atomic_fetch_add(cnt + grp * kCounterStride, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (prev != (unsigned)(size - 1)) return false;
  const unsigned groups = nb < G ? (unsigned)nb : (unsigned)G;
  const unsigned done =
      __hip_atomic_fetch_add(cnt + G * kCounterStride, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (done != groups - 1) return false;
  for (int i = 0; i <= G; ++i) __hip_atomic_store(cnt + i * kCounterStride, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return true;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// The sum of nb partial pairs (d2, n2) at p in one canonical order, independent of the
// kernel and of its workgroup size: virtual lane v (0..255) adds pairs v, v + 256, v +
// 512, ... in turn; the lanes of virtual wavefront q (lanes 64q .. 64q + 63) are summed by
// a shuffle tree (lane 0's result); the four wavefront sums are added in order q = 0..3.
// Wavefront w of an NW-wavefront workgroup takes virtual wavefronts w, w + NW, ... and
// leaves their sums in sq[q]; after a barrier, canonical_total() gives every thread the
// same bits.  ATOMIC: agent-scope loads (partials of the same launch).
constexpr int kVirtLanes = 256;
template <int NW, bool ATOMIC>
__device__ __forceinline__ void canonical_sums(const double* __restrict__ p, int nb, double (*sq)[2]) {
  const int lane = threadIdx.x & 63, w = wave_id();
  constexpr int kU = 4;
#pragma unroll
  for (int q = w; q < kVirtLanes / 64; q += NW) {
    const int v = 64 * q + lane;
    double a = 0.0, b = 0.0;
    for (int i0 = v; i0 < nb; i0 += kVirtLanes * kU) {
      double pa[kU], pb[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int i = i0 + kVirtLanes * u;
        const int ic = i < nb ? i : nb - 1;
        if constexpr (ATOMIC) {
          pa[u] = __hip_atomic_load(&p[2 * ic], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          pb[u] = __hip_atomic_load(&p[2 * ic + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
          pa[u] = p[2 * ic];
          pb[u] = p[2 * ic + 1];
        }
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const bool in = i0 + kVirtLanes * u < nb;
        a += in ? pa[u] : 0.0;
        b += in ? pb[u] : 0.0;
      }
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane == 0) {
      sq[q][0] = a;
      sq[q][1] = b;
    }
  }
}
__device__ __forceinline__ double canonical_total(const double (*sq)[2], double& b) {
  b = ((sq[0][1] + sq[1][1]) + sq[2][1]) + sq[3][1];
  return ((sq[0][0] + sq[1][0]) + sq[2][0]) + sq[3][0];
}
__device__ __forceinline__ double relative_increment(double a, double b) { return b > 0.0 ? sqrt(a / b) : sqrt(a); }

// Control block update for the stopping test of sweep number `it` (1-based) of the
// segment with relative increment res.  Returns whether the segment stops.
__device__ __forceinline__ bool stop_test(double res, double tol, int stop) {
  return isfinite(res) ? (stop && res < tol) : (stop != 0);
}
__device__ __forceinline__ void record_test(Ctrl* c, double* hist, int hist_cap, int it, double res, double tol,
                                            int stop) {
  hist[(it - 1) % hist_cap] = res;
  c->iters = it;
  c->last_res = res;
  if (!isfinite(res)) {
    c->status = 2;
    if (stop) c->done = 1;
  } else if (stop && res < tol) {
    c->status = 1;
    c->done = 1;
  }
}

// Block sum of (d2, n2) over an NW-wavefront workgroup (lane 0 of each wavefront, then
// the wavefronts in order): the value every reduction of this library stores as the
// workgroup's partial.  Valid in thread 0 after the call (which contains a barrier).
template <int NW>
__device__ __forceinline__ void block_pair(double& d2, double& n2) {
  __shared__ double sd[NW][2];
  const int lane = threadIdx.x & 63, w = wave_id();
  d2 = wave_sum(d2);
  n2 = wave_sum(n2);
  if (lane == 0) {
    sd[w][0] = d2;
    sd[w][1] = n2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int i = 0; i < NW; ++i) {
      a += sd[i][0];
      b += sd[i][1];
    }
    d2 = a;
    n2 = b;
  }
}

// NW: wavefronts per workgroup; (bid, nb): this workgroup's index among the nb
// workgroups that share the reduction (a whole launch, or one problem of a batch).
// First half: the workgroup's partial sums are stored and it arrives; returns (to every
// thread) whether it arrived last.  Stores issued after this call do not delay the
// arrival, so a caller may keep its outputs in registers and store them afterwards.
template <int NW = kWaves>
__device__ bool residual_arrive(double d2, double n2, const ResidArgs& ra, int bid, int nb) {
  __shared__ int is_last;
  block_pair<NW>(d2, n2);
  if (threadIdx.x == 0) {
    const double a = d2, b = n2;
    // The partials are agent-scope atomic stores (written through to the level where
    // all XCDs see them).  Waiting for their completion before the arrival is counted
    // orders them before it, without a device-wide release fence: such a fence writes
    // back this XCD's whole L2 and, once per workgroup, costs more than the sweep.
    __hip_atomic_store(&ra.partials[2 * bid], a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&ra.partials[2 * bid + 1], b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_s_waitcnt(0);
    is_last = arrive_last(ra.cnt, bid, nb) ? 1 : 0;
  }
  __syncthreads();
  return is_last != 0;
}

// Second half, run by every thread of the last workgroup: the sum of all partials in the
// canonical order (every partial has arrived; the agent-scope loads read them where they
// were written), the history entry and the control block update.  iters: the control
// block's iteration count as read at the start of the launch (only this workgroup
// changes it, so passing it in saves a memory round trip at the end of the launch).
template <int NW = kWaves>
__device__ void residual_final(const ResidArgs& ra, int nb, int iters) {
  __shared__ double sq[kVirtLanes / 64][2];
  canonical_sums<NW, true>(ra.partials, nb, sq);
  __syncthreads();
  if (threadIdx.x == 0) {
    double b;
    const double a = canonical_total(sq, b);
    record_test(ra.ctrl, ra.hist, ra.hist_cap, iters + 1, relative_increment(a, b), ra.tol, ra.stop);
  }
}

template <int NW = kWaves>
__device__ void finish_residual(double d2, double n2, const ResidArgs& ra, int bid, int nb, int iters) {
  if (residual_arrive<NW>(d2, n2, ra, bid, nb)) residual_final<NW>(ra, nb, iters);
}

template <int NW = kWaves>
__device__ __forceinline__ void finish_residual(double d2, double n2, const ResidArgs& ra, int iters) {
  finish_residual<NW>(d2, n2, ra, (int)blockIdx.x, (int)gridDim.x, iters);
}

// ---------------------------------------------------------------------------
// the sweep
// ---------------------------------------------------------------------------
// Rows of the (zero-padded) operator handled by one wavefront.
template <int ROWS>
struct RowSplit {
  static constexpr int RW = (ROWS + kWaves - 1) / kWaves;
  static constexpr int PAD = RW * kWaves;
};

extern __shared__ __align__(16) unsigned char g_smem[];

// Gathers input rows [c_begin, c_end) of the workgroup's elements into LDS rows
// starting at lds_row (wavefront w takes rows w, w + kWaves, ...).
// es is the lane's element, or element 0 for a lane past the end (valid = false).
template <class F, typename T, class LD>
__device__ __forceinline__ void stage_inputs(const MeshDev& m, int es, bool valid, const Nb& nb, const LD& ld,
                                             T* x, int lds_row) {
  const int lane = threadIdx.x & 63, w = wave_id();
  // unrolled with a compile-time trip count and unconditional loads, so every load
  // is in flight before the first LDS write waits for one
  constexpr int J = (F::I + kWaves - 1) / kWaves;
  T v[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int c = w + j * kWaves;
    const T r = (T)F::row(m, es, nb, ld, c < F::I ? c : F::I - 1);
    v[j] = valid ? r : T(0);
  }
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int c = w + j * kWaves;
    if (c < F::I) x[(lds_row + c) * kLanes + lane] = v[j];
  }
}

// ---------------------------------------------------------------------------
// the FP64 sweep on the matrix cores
// ---------------------------------------------------------------------------
// out = g + T in(s) for tiles of 16 elements as D(S x 16) = T(S x I) B(I x 16) + G with
// v_mfma_f64_16x16x4f64.  Lane l of a wavefront holds A[l % 16][l / 16] of each 16 x 4
// operator fragment (kept in registers for the whole launch), B[l / 16][l % 16] = input
// row 4 kt + l / 16 of element 16 t + l % 16 (gathered straight from the component-
// major state: 16 lanes read 128 contiguous bytes), and D[l / 16 + 4 r][l % 16] (rows
// interleaved by 4 in the FP64 variant; checked on gfx950 with a one-wavefront probe).
// A workgroup of WPG wavefronts shares each element tile, wavefront w applying row
// tiles [w MTW, (w + 1) MTW); it sweeps a contiguous range of tiles.
typedef double doublex4_t __attribute__((ext_vector_type(4)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

constexpr int kMfmaMaxA = 48;  // operator doubles per lane a wavefront keeps in registers

template <int ROWS, int COLS, int MAXA = kMfmaMaxA>
struct Tiling64 {
  static constexpr int MT = (ROWS + 15) / 16, KT = (COLS + 3) / 4;
  static constexpr int pick(int d) { return d <= 1 ? 1 : ((MT % d == 0 && d * KT <= MAXA) ? d : pick(d - 1)); }
  static constexpr int MTW = pick(MT);              // row tiles per wavefront
  static constexpr int WPG = MT / MTW;              // wavefronts per element tile
  static constexpr int TS = WPG > 1 ? 1 : 4;          // element tiles in flight per workgroup
  static constexpr int NW = WPG * TS;               // wavefronts per workgroup
};

// Matrix-core engine for a workgroup of WPG (> 1) wavefronts that share every element
// tile: the B tile (COLS x 16 elements) is gathered once per workgroup into LDS (wave-
// front w loads k tiles w, w + WPG, ...), double-buffered, with the next tile's loads
// in flight while the current tile's MFMAs run; wavefront w then applies row tiles
// [w MTW, (w + 1) MTW) with its register-resident operator fragments a.
//   colload(c, es, nb, x, y): issue the loads of input column c (< COLS) of element es (a
//                      valid element index) into x, y, without using their values
//   colcombine(c, nb, x, y): the column's value from those loads
//   init(row, es, aux, keep): C entry of output row (< ROWS), used if keep (else 0); may
//                      also set aux (a value the epilogue needs, loaded together with
//                      the C entries)
//   epi(row, e, v, aux): result of output row for element e (valid lanes only)
//   OWN_LDS: aux is instead the staged input column F::kOwnCol + row of the element (the
//                      element's own state row, where F::kOwnRaw: the gather stages it
//                      unchanged), read from the LDS tile; init then need not load it
// Loads complete in order and any use of a loaded value (even a select) waits for it, so
// the combination and the masking of the prefetched columns happen when they are staged,
// after this tile's MFMAs, and the C entries are masked after the prefetch is issued.
template <class F, int ROWS, int COLS, int MTW, int WPG, bool OWN_LDS = false, class ColLoad, class ColCombine,
          class Init, class Epi>
__device__ __forceinline__ void mfma64_shared_b(const MeshDev& m, const double (&a)[MTW][(COLS + 3) / 4], int t0,
                                                int t1, double* lds, ColLoad colload, ColCombine colcombine,
                                                Init init, Epi epi) {
  constexpr int KT = (COLS + 3) / 4, KTW = (KT + WPG - 1) / WPG, BT = KT * 4 * 16;
  const int lane = threadIdx.x & 63, w = wave_id();
  // the workgroup is WPG wavefronts: with w bounded, the compiler resolves which k tiles
  // hold which kind of column, and drops loads that a column kind does not need
  __builtin_assume(w >= 0 && w < WPG);
  const int j = lane & 15, kq = lane >> 4;
  double vx[KTW], vy[KTW];
  Nb gnb;
  bool gvalid = false;
  auto gather = [&](int t) {
    const int e = t * 16 + j;
    gvalid = e < m.nel;
    const int es = gvalid ? e : 0;
    F::neighbours(m, es, gnb);
#pragma unroll
    for (int i = 0; i < KTW; ++i) {
      const int kt = w + i * WPG, c = 4 * kt + kq;
      colload(c < COLS ? c : COLS - 1, es, gnb, vx[i], vy[i]);
    }
  };
  auto stage = [&](double* buf) {
#pragma unroll
    for (int i = 0; i < KTW; ++i) {
      const int kt = w + i * WPG, c = 4 * kt + kq;
      if (kt < KT) {
        const double x = colcombine(c < COLS ? c : COLS - 1, gnb, vx[i], vy[i]);
        buf[(4 * kt + kq) * 16 + j] = (gvalid && c < COLS) ? x : 0.0;
      }
    }
  };
  if (t0 < t1) {
    gather(t0);
    stage(lds);
  }
  __syncthreads();
  for (int t = t0; t < t1; ++t) {
    const int cur = (t - t0) & 1;
    const double* bcur = lds + cur * BT;
    const int e = t * 16 + j;
    const bool valid = e < m.nel;
    const int es = valid ? e : 0;
    // C entries of this tile first (their loads are waited for before the prefetch's)
    double c0[MTW][4], aux[MTW][4];
    bool keep[MTW][4];
#pragma unroll
    for (int u = 0; u < MTW; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * (w * MTW + u) + kq + 4 * r;
        c0[u][r] = init(row < ROWS ? row : ROWS - 1, es, aux[u][r], keep[u][r]);
      }
    // unconditional, so that the count of loads in flight is the same on every path (the
    // last tile gathers itself again, and does not stage it)
    gather(t + 1 < t1 ? t + 1 : t);
    __builtin_amdgcn_sched_barrier(0);  // the prefetch is issued before the MFMAs
    // With one row tile per wavefront the products start from zero and the C entries are
    // added after them, so the C entries' loads are in flight during the MFMAs instead of
    // ahead of them (with more row tiles the registers this holds would cost occupancy)
    constexpr bool kAddAfter = MTW == 1;
    doublex4_t acc[MTW];
#pragma unroll
    for (int u = 0; u < MTW; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * (w * MTW + u) + kq + 4 * r;
        acc[u][r] = (!kAddAfter && valid && row < ROWS && keep[u][r]) ? c0[u][r] : 0.0;
      }
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      const double b = bcur[(4 * kt + kq) * 16 + j];
#pragma unroll
      for (int u = 0; u < MTW; ++u) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][kt], b, acc[u], 0, 0, 0);
    }
    if (valid) {
#pragma unroll
      for (int u = 0; u < MTW; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * (w * MTW + u) + kq + 4 * r;
          if (row < ROWS) {
            const double v = kAddAfter ? (double)acc[u][r] + (keep[u][r] ? c0[u][r] : 0.0) : (double)acc[u][r];
            double own;
            if constexpr (OWN_LDS) {
              static_assert(F::kOwnRaw && F::kOwnCol + ROWS <= COLS, "own rows must be staged unchanged");
              own = bcur[(F::kOwnCol + row) * 16 + j];
            } else {
              own = aux[u][r];
            }
            epi(row, e, v, own);
          }
        }
    }
    if (t + 1 < t1) stage(lds + (cur ^ 1) * BT);
    __syncthreads();
  }
}

// Matrix-core engine with the whole operator in LDS, for contractions whose operator
// fits there (the step completion of the smaller families): the workgroup has copied the
// fragment-major operator Mf (MT row tiles x KT k tiles x 64 lanes) into LDS (lds_a_copy,
// at the start of the kernel, so that the copy overlaps the kernel's set-up).  Each
// wavefront owns TPW element tiles (t0 + w + i NW below t1): gather() loads the B
// fragments of all of them straight into registers at once, and apply() runs all MT row
// tiles over each in turn as independent accumulator chains, reading the operator
// fragments from LDS: the later tiles' loads are in flight during the first tile's
// products, and each tile's stores during the next one's.  (A fixed count of tiles, not
// a loop over tiles: in a loop the compiler keeps every column's address across
// iterations, beyond the register budget.)  Each row tile takes its k tiles in order,
// from the C entries (C_FIRST) or from zero with the C entries added after the products,
// whichever the other engine does for the same family, so that the two give bitwise the
// same results.
//   colload / colcombine / epi as for mfma64_shared_b; init(row, es, aux, keep) as there
template <int ROWS, int COLS, int NW>
__device__ __forceinline__ void lds_a_copy(const double* __restrict__ Mf, double* la) {
  constexpr int kTotal = ((ROWS + 15) / 16) * ((COLS + 3) / 4) * 64;
#pragma unroll
  for (int i0 = 0; i0 < kTotal; i0 += 64 * NW) {
    const int i = i0 + (int)threadIdx.x;
    if (i < kTotal) la[i] = Mf[i];
  }
}
template <class F, int ROWS, int COLS, int NW, int TPW, int MH, bool C_FIRST>
struct LdsAEngine {
  static constexpr int MT = (ROWS + 15) / 16, KT = (COLS + 3) / 4;
  double b[TPW][KT];
  int ev[TPW];
  // the B fragments of this wavefront's tiles (zero past t1 and past the last element)
  template <class ColLoad, class ColCombine>
  __device__ __forceinline__ void gather(const MeshDev& m, int t0, int t1, ColLoad colload, ColCombine colcombine) {
    const int lane = threadIdx.x & 63, w = wave_id();
    const int j = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int t = t0 + w + i * NW;
      const int e = t * 16 + j;
      const bool valid = t < t1 && e < m.nel;
      const int es = valid ? e : 0;
      ev[i] = valid ? e : -1;
      Nb nb;
      F::neighbours(m, es, nb);
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) {
        const int c = 4 * kt + kq, cc = c < COLS ? c : COLS - 1;
        double x, y;
        colload(cc, es, nb, x, y);
        const double v = colcombine(cc, nb, x, y);
        b[i][kt] = (valid && c < COLS) ? v : 0.0;
      }
    }
  }
  // the products and the epilogue (la: the operator in LDS, copied by every thread of the
  // workgroup before this call)
  template <class Init, class Epi>
  __device__ __forceinline__ void apply(const double* la, int t0, int t1, Init init, Epi epi) {
    __syncthreads();  // the operator copy is complete
    const int lane = threadIdx.x & 63, w = wave_id();
    const int kq = lane >> 4;
    if (t0 + w >= t1) return;
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      if (t0 + w + i * NW >= t1) break;  // wavefront-uniform
      const int e = ev[i];
      const bool valid = e >= 0;
      const int es = valid ? e : 0;
      // the row tiles in passes of MH (the accumulators of a pass and the B fragments within
      // the register budget); the next k tile's operator fragments are read from LDS while
      // this k tile's products run
#pragma unroll
      for (int h = 0; h < MT; h += MH) {
        doublex4_t acc[MH];
        double ac[MH], an[MH], aux[MH][4];
#pragma unroll
        for (int u = 0; u < MH; ++u) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 16 * (h + u) + kq + 4 * r;
            bool keep = false;
            double c0 = 0.0;
            if constexpr (C_FIRST) c0 = init(row < ROWS ? row : ROWS - 1, es, aux[u][r], keep);
            acc[u][r] = (C_FIRST && valid && h + u < MT && row < ROWS && keep) ? c0 : 0.0;
          }
          ac[u] = h + u < MT ? la[((h + u) * KT) * 64 + lane] : 0.0;
        }
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) {
#pragma unroll
          for (int u = 0; u < MH; ++u)
            an[u] = (kt + 1 < KT && h + u < MT) ? la[((h + u) * KT + kt + 1) * 64 + lane] : 0.0;
#pragma unroll
          for (int u = 0; u < MH; ++u)
            if (h + u < MT) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ac[u], b[i][kt], acc[u], 0, 0, 0);
#pragma unroll
          for (int u = 0; u < MH; ++u) ac[u] = an[u];
          // the LDS reads ahead of the products (the compiler would otherwise issue them
          // after the products and wait for them at once)
          __builtin_amdgcn_sched_group_barrier(0x100, MH, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, MH, 0);
          __builtin_amdgcn_sched_barrier(0);
        }
        if (valid) {
#pragma unroll
          for (int u = 0; u < MH; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = 16 * (h + u) + kq + 4 * r;
              if (h + u < MT && row < ROWS) {
                if constexpr (C_FIRST) {
                  epi(row, e, (double)acc[u][r], aux[u][r]);
                } else {
                  double a1;
                  bool keep;
                  const double c0 = init(row, es, a1, keep);
                  epi(row, e, (double)acc[u][r] + (keep ? c0 : 0.0), a1);
                }
              }
            }
        }
      }
    }
  }
};

template <class F>
struct SweepWaves {  // wavefronts per workgroup of the matrix-core sweep
  static constexpr int value = Tiling64<F::S, F::I>::NW;
};

// Lagged stopping test (LAGGED; single-problem FP64 sweeps).  The host numbers the
// sweeps of a handle (seq); the control block holds the number of the sweep before the
// segment's first (seg_seq), so this sweep is number k = seq - seg_seq of its segment.
// It leaves its own increment as per-workgroup partial sums in set seq & 1 and takes
// the stopping test of sweep k - 1 from set (seq - 1) & 1 before it writes anything:
// every workgroup sums the partials in the canonical order and reaches the same
// decision; workgroup 0 records it.  No workgroup waits for another, so the launch has
// no arrival and no last-workgroup tail.  Without LAGGED (batched launches) the last
// workgroup to arrive takes the test of this sweep, as before.
struct LagArgs {
  unsigned seq;     // this launch's sweep number
  int stride;       // doubles between the two partial sets
};

// The first kU pairs of each of a wavefront's virtual lanes (the canonical order of
// canonical_sums), loaded into registers ahead of their use; pairs beyond
// kVirtLanes * kU are read when consumed.
template <int NW>
struct PartialPrefetch {
  static constexpr int kQ = (kVirtLanes / 64 + NW - 1) / NW;  // virtual wavefronts per wavefront
  static constexpr int kU = 4;
  double pa[kQ][kU], pb[kQ][kU];
  __device__ __forceinline__ void issue(const double* __restrict__ p, int nb) {
    const int lane = threadIdx.x & 63, w = wave_id();
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const int q = w + i * NW, v = 64 * (q < kVirtLanes / 64 ? q : 0) + lane;
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int j = v + kVirtLanes * u;
        const int jc = j < nb ? j : nb - 1;
        pa[i][u] = p[2 * jc];
        pb[i][u] = p[2 * jc + 1];
      }
    }
  }
  __device__ __forceinline__ void consume(const double* __restrict__ p, int nb, double (*sq)[2]) const {
    const int lane = threadIdx.x & 63, w = wave_id();
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const int q = w + i * NW;
      if (q >= kVirtLanes / 64) break;
      const int v = 64 * q + lane;
      double a = 0.0, b = 0.0;
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const bool in = v + kVirtLanes * u < nb;
        a += in ? pa[i][u] : 0.0;
        b += in ? pb[i][u] : 0.0;
      }
      for (int j = v + kVirtLanes * kU; j < nb; j += kVirtLanes) {
        a += p[2 * j];
        b += p[2 * j + 1];
      }
      a = wave_sum(a);
      b = wave_sum(b);
      if (lane == 0) {
        sq[q][0] = a;
        sq[q][1] = b;
      }
    }
  }
};

// Start of a lagged sweep, all threads: the previous sweep's partials are loaded with the
// control block, the control block's done flag is made uniform across the workgroup (a
// launch queued past convergence leaves here, without waiting for the partials), the
// partials are summed in the canonical order, and the stopping test of sweep k - 1 is
// taken.  Returns k (> 0), or 0 if the segment has stopped (then the caller writes nothing).
// The previous sweep's partial set.
__device__ __forceinline__ const double* lagged_parts(const ResidArgs& ra, const LagArgs& lag) {
  return ra.partials + (size_t)((lag.seq - 1u) & 1u) * lag.stride;
}

// The control block's done flag as workgroup 0's first wavefront read it, the same for
// every wavefront of the workgroup (a launch queued past convergence leaves on it).
__device__ __forceinline__ int uniform_done(const CtrlHead& ch) {
  __shared__ int s_done;
  if (threadIdx.x == 0) s_done = ch.done;
  __syncthreads();
  return s_done;
}

// The stopping test of the previous sweep once its partials' loads are issued (pf) and the
// segment is known to be running: callers may issue other loads in between, whose latency
// then overlaps the sum.  Returns k (> 0), or 0 if the test stops the segment.
template <int NW>
__device__ __forceinline__ int lagged_test(const ResidArgs& ra, const LagArgs& lag, int nb, int bid, unsigned seg,
                                           const PartialPrefetch<NW>& pf, const double* parts) {
  __shared__ double sq[kVirtLanes / 64][2];
  pf.consume(parts, nb, sq);
  __syncthreads();
  const int k = (int)(lag.seq - seg);
  if (k >= 2) {
    double b;
    const double res = relative_increment(canonical_total(sq, b), b);
    if (bid == 0 && threadIdx.x == 0) record_test(ra.ctrl, ra.hist, ra.hist_cap, k - 1, res, ra.tol, ra.stop);
    if (stop_test(res, ra.tol, ra.stop)) return 0;
  }
  return k;
}

template <int NW>
__device__ __forceinline__ int lagged_begin(const ResidArgs& ra, const LagArgs& lag, int nb, int bid,
                                            const CtrlHead& ch, unsigned seg) {
  const double* parts = lagged_parts(ra, lag);
  PartialPrefetch<NW> pf;
  pf.issue(parts, nb);
  if (uniform_done(ch)) return 0;
  return lagged_test<NW>(ra, lag, nb, bid, seg, pf, parts);
}

// End of a lagged sweep, all threads: the workgroup's partial sums into set seq & 1.
template <int NW>
__device__ __forceinline__ void lagged_end(double d2, double n2, const ResidArgs& ra, const LagArgs& lag, int bid) {
  block_pair<NW>(d2, n2);
  if (threadIdx.x == 0) {
    double* p = ra.partials + (size_t)(lag.seq & 1u) * lag.stride;
    p[2 * bid] = d2;
    p[2 * bid + 1] = n2;
  }
}

template <class F, bool DEVPAR, bool LAGGED>
__device__ __forceinline__ void sweep_mfma_body(MeshDev m, Ld64 ld, const double* __restrict__ g,
                                                const double* __restrict__ Tf, double* out, const ResidArgs& ra,
                                                double* s0, double* s1, int tiles_per_group, int bid, int nbk,
                                                LagArgs lag) {
  using TL = Tiling64<F::S, F::I>;
  constexpr int MTW = TL::MTW, KT = TL::KT;
  const CtrlHead ch = ctrl_head(ra.ctrl);
  const unsigned seg = LAGGED ? ra.ctrl->seg_seq : 0u;
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int w = wave % TL::WPG, slot = wave / TL::WPG;  // row-tile group, tile slot
  const int j = lane & 15, kq = lane >> 4;
  // this wavefront's operator fragments (loaded while the control block read is in flight)
  double a[MTW][KT];
#pragma unroll
  for (int u = 0; u < MTW; ++u)
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) a[u][kt] = Tf[((w * MTW + u) * KT + kt) * 64 + lane];
  // the sweep number of the segment, and with it the input buffer, follow from the
  // control block head alone (the lagged test below only decides whether to go on)
  const int kpre = LAGGED ? (int)(lag.seq - seg) : ch.iters + 1;
  if constexpr (DEVPAR) {
    const int parity = (ch.base + kpre - 1) & 1;  // s^(k-1) of the segment
    ld.p = parity ? s1 : s0;
    out = parity ? s0 : s1;
  }
  const size_t nel = (size_t)m.nel;
  const int ntiles = (m.nel + 15) >> 4;
  const int t0 = remap_block(m.order ? nbk - 1 - bid : bid, nbk) * tiles_per_group;
  const int t1 = min(t0 + tiles_per_group, ntiles);
  double d2 = 0.0, n2 = 0.0;
  if constexpr (TL::WPG > 1) {
    if constexpr (LAGGED) {
      if (lagged_begin<TL::NW>(ra, lag, nbk, bid, ch, seg) == 0) return;
    } else {
      if (ch.done) return;
    }
    __shared__ double bt[2 * KT * 4 * 16];
    // the previous state rows, for the increment, from the staged tile where the family
    // stages them unchanged
    constexpr bool kOwnLds = F::kOwnRaw;
    mfma64_shared_b<F, F::S, F::I, MTW, TL::WPG, kOwnLds>(
        m, a, t0, t1, bt,
        [&](int c, int es, const Nb& nb, double& x, double& y) { F::row_load(m, es, nb, ld, c, x, y); },
        [&](int c, const Nb& nb, double x, double y) { return F::row_combine(nb, c, x, y); },
        [&](int row, int es, double& old, bool& keep) {
          if constexpr (kOwnLds)
            old = 0.0;
          else
            old = ld(row, es);
          keep = true;
          return g[(size_t)row * nel + es];
        },
        [&](int row, int e, double v, double old) {
          out[(size_t)row * nel + e] = v;
          const double dd = v - old;
          d2 += dd * dd;
          n2 += v * v;
        });
    if constexpr (LAGGED)
      lagged_end<TL::NW>(d2, n2, ra, lag, bid);
    else
      finish_residual<TL::NW>(d2, n2, ra, bid, nbk, ch.iters);
    return;
  }
  // WPG == 1: each wavefront gathers and applies its own tiles.  The first tile's inputs
  // (gathered traces, g, the element's own state) are loaded before the previous sweep's
  // stopping test is summed, so their latency overlaps it; a launch that stops discards
  // them (they are only read).
  // (only loads here: every use of a loaded value, even a select, waits for it)
  // The element's previous state rows, for the increment, from the gathered registers: in
  // the FP64 result layout a lane's output rows are kq + 4 r of its row tiles; with
  // o = kOwnCol mod 4 and k0 = kOwnCol / 4, output row r of row tile u is own column
  // kOwnCol + 16 u + kq + 4 r, held by 16-lane row (kq + o) mod 4 in register
  // k0 + 4 u + r + (kq + o >= 4).  For o = 0 that is the lane itself; otherwise each lane
  // offers register k0 + 4 u + r + (its row < o) and reads it from the lane 16 o further
  // on (a shuffle over the whole wavefront).  (This path runs only with WPG == 1: wider
  // tiles took the shared-tile engine above.)
  constexpr bool kOwnRegs = TL::WPG == 1;
  struct TileIn {
    double x[KT], y[KT];
    double g0[MTW][4];
    double old[kOwnRegs ? 1 : MTW][4];
    Nb nb;
  };
  auto load_tile = [&](int t, bool active, TileIn& in) {
    const int e = t * 16 + j;
    const int es = (active && e < m.nel) ? e : 0;
    F::neighbours(m, es, in.nb);
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      const int c = 4 * kt + kq;
      F::row_load(m, es, in.nb, ld, c < F::I ? c : F::I - 1, in.x[kt], in.y[kt]);
    }
#pragma unroll
    for (int u = 0; u < MTW; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * (w * MTW + u) + kq + 4 * r;
        const int rc = row < F::S ? row : F::S - 1;
        in.g0[u][r] = g[(size_t)rc * nel + es];
        if constexpr (!kOwnRegs) in.old[u][r] = ld(rc, es);
      }
  };
  // issue order: the partials (addresses from the launch's arguments), then the tile
  // (addresses from the control block head); loads complete in order, so the partials can
  // be waited for and summed while the tile's loads are still in flight
  const double* parts = nullptr;
  PartialPrefetch<TL::NW> pf;
  if constexpr (LAGGED) {
    parts = lagged_parts(ra, lag);
    pf.issue(parts, nbk);
    __builtin_amdgcn_sched_barrier(0);  // keep the partials' loads ahead of the tile's
  }
  // a launch past convergence leaves before any tile load (the same decision for the whole
  // workgroup); the loads are then unconditional (a branch around them would make the
  // compiler wait for them before the sum): a wavefront without a tile reads element 0
  if constexpr (LAGGED) {
    if (uniform_done(ch)) return;
  } else {
    if (ch.done) return;
  }
  TileIn cur;
  const int tf = t0 + slot;
  load_tile(tf, tf < t1, cur);
  if constexpr (LAGGED) {
    if (lagged_test<TL::NW>(ra, lag, nbk, bid, seg, pf, parts) == 0) return;
  }
  doublex4_t pend[MTW];
  int pend_e = -1;
  for (int t = tf; t < t1; t += TL::TS) {
    if (t != tf) load_tile(t, true, cur);
    const int e = t * 16 + j;
    const bool valid = e < m.nel;
    double b[KT];
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      const int c = 4 * kt + kq;
      const double v = F::row_combine(cur.nb, c < F::I ? c : F::I - 1, cur.x[kt], cur.y[kt]);
      b[kt] = (valid && c < F::I) ? v : 0.0;
    }
    doublex4_t acc[MTW];
#pragma unroll
    for (int u = 0; u < MTW; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * (w * MTW + u) + kq + 4 * r;
        acc[u][r] = (valid && row < F::S) ? cur.g0[u][r] : 0.0;
      }
#pragma unroll
    for (int kt = 0; kt < KT; ++kt)
#pragma unroll
      for (int u = 0; u < MTW; ++u) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][kt], b[kt], acc[u], 0, 0, 0);
    // the increment against the element's own previous state
    double prev[MTW][4];
#pragma unroll
    for (int u = 0; u < MTW; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if constexpr (kOwnRegs) {
          constexpr int k0 = F::kOwnCol / 4, o = F::kOwnCol % 4;
          const int ka = k0 + 4 * u + r;  // WPG == 1: the wavefront's row tiles are 0 .. MTW - 1
          const double xa = cur.x[ka < KT ? ka : KT - 1];
          if constexpr (o == 0) {
            prev[u][r] = xa;
          } else {
            const double xb = cur.x[ka + 1 < KT ? ka + 1 : KT - 1];
            prev[u][r] = __shfl(kq < o ? xb : xa, (lane + 16 * o) & 63);
          }
        } else {
          prev[u][r] = cur.old[u][r];
        }
      }
#pragma unroll
    for (int u = 0; u < MTW; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * (w * MTW + u) + kq + 4 * r;
        if (valid && row < F::S) {
          const double v = acc[u][r];
          const double dd = v - prev[u][r];
          d2 += dd * dd;
          n2 += v * v;
        }
      }
    // the wavefront's last tile is stored after the arrival below; earlier ones now
    if (t + TL::TS < t1) {
      if (valid)
#pragma unroll
        for (int u = 0; u < MTW; ++u)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 16 * (w * MTW + u) + kq + 4 * r;
            if (row < F::S) out[(size_t)row * nel + e] = acc[u][r];
          }
    } else {
      pend_e = valid ? e : -1;
#pragma unroll
      for (int u = 0; u < MTW; ++u) pend[u] = acc[u];
    }
  }
  // the arrival (without LAGGED) goes first; the last tile's stores follow it
  bool last = false;
  if constexpr (!LAGGED) last = residual_arrive<TL::NW>(d2, n2, ra, bid, nbk);
  if (pend_e >= 0)
#pragma unroll
    for (int u = 0; u < MTW; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * (w * MTW + u) + kq + 4 * r;
        if (row < F::S) out[(size_t)row * nel + pend_e] = pend[u][r];
      }
  if constexpr (LAGGED)
    lagged_end<TL::NW>(d2, n2, ra, lag, bid);
  else if (last)
    residual_final<TL::NW>(ra, nbk, ch.iters);
}

template <class F, bool DEVPAR>
__global__ __launch_bounds__(64 * SweepWaves<F>::value) void k_sweep_mfma(
    MeshDev m, Ld64 ld, const double* __restrict__ g, const double* __restrict__ Tf, double* out, ResidArgs ra,
    double* s0, double* s1, int tiles_per_group, LagArgs lag) {
  sweep_mfma_body<F, DEVPAR, true>(m, ld, g, Tf, out, ra, s0, s1, tiles_per_group, (int)blockIdx.x,
                                   (int)gridDim.x, lag);
}

// mixed precision outer step: s_out = s_in (+ lo_in); r = g + T in(s_out) - s_out (FP64);
// r_lo = r in the low precision; norms of r and of s_out + r.
struct StSoa32 {  // FP32, component-major
  float* p;
  size_t nel;
  __device__ __forceinline__ void operator()(int r, int e, double v) const { p[(size_t)r * nel + e] = (float)v; }
};
template <int S>
struct StAos32 {  // FP32, element-major
  float* p;
  __device__ __forceinline__ void operator()(int r, int e, double v) const { p[(size_t)e * S + r] = (float)v; }
};
template <int S>
struct StAos16 {  // BF16, element-major
  uint16_t* p;
  __device__ __forceinline__ void operator()(int r, int e, double v) const {
    p[(size_t)e * S + r] = f32_to_bf16((float)v);
  }
};

// Element solution from the traces of the last local solve, as one stacked contraction
//   steady:          u_new = w_src + R in(s_prev)
//   backward Euler:  [u_new; g_next] = [w_src; gbe] + [[P, R], [G P, G R]] [u_old; in(s_prev)]
// (u_new = A^{-1}(F_src + Mbt u_old + L in) and g_next = Q A^{-1}(F_src + Mbt u_new)).
template <class F, bool BE, typename ST = double>
__device__ __forceinline__ void volume_body(const MeshDev& m, const ST* __restrict__ s_prev,
                                            const double* __restrict__ Mv, const double* __restrict__ u_old,
                                            const double* __restrict__ w_src, const double* __restrict__ gbe,
                                            double* __restrict__ u_new, double* __restrict__ g_out) {
  constexpr int COLS = (BE ? F::N : 0) + F::I;
  constexpr int ROWS = F::N + (BE ? F::S : 0);
  constexpr int RW = RowSplit<ROWS>::RW;
  double* x = reinterpret_cast<double*>(g_smem);
  const int lane = threadIdx.x & 63, w = wave_id();
  const int e = remap_block(blockIdx.x, gridDim.x) * kLanes + lane;
  const bool valid = e < m.nel;
  const size_t nel = (size_t)m.nel;
  const int es = valid ? e : 0;
  Nb nb;
  F::neighbours(m, es, nb);
  if constexpr (BE) {
    constexpr int J = (F::N + kWaves - 1) / kWaves;
    double v[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int c = w + j * kWaves;
      const double u = u_old[(size_t)(c < F::N ? c : F::N - 1) * nel + es];
      v[j] = valid ? u : 0.0;
    }
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int c = w + j * kWaves;
      if (c < F::N) x[c * kLanes + lane] = v[j];
    }
  }
  stage_inputs<F, double>(m, es, valid, nb, LdOf<ST>{s_prev, nel}, x, BE ? F::N : 0);
  __syncthreads();
  const int r0 = w * RW;
  double acc[RW];
#pragma unroll
  for (int i = 0; i < RW; ++i) acc[i] = 0.0;
  const double* __restrict__ Mrow = Mv + (size_t)uniform(r0 * COLS);
#pragma unroll 4
  for (int c = 0; c < COLS; ++c) {
    const double xc = x[c * kLanes + lane];
#pragma unroll
    for (int i = 0; i < RW; ++i) acc[i] = fma(Mrow[i * COLS + c], xc, acc[i]);
  }
#pragma unroll
  for (int i = 0; i < RW; ++i) {
    const int q = r0 + i;
    if (!valid) break;
    if (q < F::N) {
      u_new[(size_t)q * nel + e] = acc[i] + (w_src ? w_src[(size_t)q * nel + e] : 0.0);
    } else if (BE && q < ROWS && g_out) {
      const int r = q - F::N;
      g_out[(size_t)r * nel + e] = acc[i] + (gbe ? gbe[(size_t)r * nel + e] : 0.0);
    }
  }
}

template <class F, bool BE, typename ST = double>
__global__ __launch_bounds__(kThreads) void k_volume(MeshDev m, const ST* __restrict__ s_prev,
                                                      const double* __restrict__ Mv,
                                                      const double* __restrict__ u_old,
                                                      const double* __restrict__ w_src,
                                                      const double* __restrict__ gbe, double* __restrict__ u_new) {
  volume_body<F, BE, ST>(m, s_prev, Mv, u_old, w_src, gbe, u_new, nullptr);
}

// s' = s^k + the low-precision correction (from the segment's second refinement on;
// before that a copy of s^k), written to the buffer the refinement writes s^{k+1} to.
// One thread per element: the FP64 state is component-major (coalesced per row), the
// correction either component-major (FP32) or element-major (BF16, S values per element).
template <class F, class LDD>
__global__ __launch_bounds__(256) void k_apply_correction(const Ctrl* ctrl, double* s0, double* s1, LDD d, int nel,
                                                          unsigned stamp) {
  const CtrlHead ch = ctrl_head(ctrl);
  if (ch.done || (stamp != 0u && ctrl->applied == stamp)) return;  // s' already stored
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nel) return;
  const int parity = (ch.base + ch.iters) & 1;
  const double* __restrict__ s = parity ? s1 : s0;
  double* __restrict__ out = parity ? s0 : s1;
  const bool use = ch.iters > 0;
  if constexpr (std::is_same_v<LDD, Ld16Aos<F::S>> && F::S % 8 == 0) {
    // the element's S BF16 values are contiguous and 16-byte aligned (S * 2 bytes per
    // element, 256-byte aligned buffer): 16-byte loads of 8 values each
    const uint4* __restrict__ q = reinterpret_cast<const uint4*>(d.p + (size_t)e * F::S);
#pragma unroll 2
    for (int c = 0; c < F::S / 8; ++c) {
      const uint4 v4 = q[c];
      const uint32_t wd[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
      for (int h = 0; h < 8; ++h) {
        const size_t i = (size_t)(8 * c + h) * nel + e;
        const double v = s[i];
        const uint16_t b = (uint16_t)(wd[h >> 1] >> (16 * (h & 1)));
        out[i] = use ? v + (double)bf16_to_f32(b) : v;
      }
    }
  } else {
#pragma unroll 8
    for (int r = 0; r < F::S; ++r) {
      const size_t i = (size_t)r * nel + e;
      const double v = s[i];
      out[i] = use ? v + (double)d(r, e) : v;
    }
  }
}

// Mixed-precision refinement on the matrix cores: s' = s^k (+ the low-precision
// correction from the segment's second refinement on); r = g + T in(s') - s' in FP64,
// stored in the low precision (r_lo); s' stored as s^{k+1}; the stopping test on
// ||r|| / ||s' + r|| (the increment of the refined iterate).
// With APPLIED (LD = Ld64) s' is already in the buffer s^{k+1} goes to (k_apply_correction
// wrote it): the gather reads one FP64 value per input instead of a state value and a
// correction value, and s' is not stored again.
template <class F, class LD, class ST, bool APPLIED = false>
__global__ __launch_bounds__(64 * SweepWaves<F>::value) void k_refine_mfma(
    MeshDev m, LD ld, const double* __restrict__ g, const double* __restrict__ Tf, double* s0, double* s1, ST r_lo,
    ResidArgs ra, int tiles_per_group) {
  using TL = Tiling64<F::S, F::I>;
  constexpr int MTW = TL::MTW, KT = TL::KT;
  const CtrlHead ch = ctrl_head(ra.ctrl);
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int w = wave % TL::WPG, slot = wave / TL::WPG;
  const int j = lane & 15, kq = lane >> 4;
  double a[MTW][KT];
#pragma unroll
  for (int u = 0; u < MTW; ++u)
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) a[u][kt] = Tf[((w * MTW + u) * KT + kt) * 64 + lane];
  if (ch.done) return;
  const int parity = (ch.base + ch.iters) & 1;
  if constexpr (APPLIED)
    ld.p = parity ? s0 : s1;
  else
    set_state(ld, parity ? s1 : s0, ch.iters > 0 ? 1 : 0);
  double* s_out = parity ? s0 : s1;
  const size_t nel = (size_t)m.nel;
  const int ntiles = (m.nel + 15) >> 4;
  const int t0 = remap_block(blockIdx.x, gridDim.x) * tiles_per_group;
  const int t1 = min(t0 + tiles_per_group, ntiles);
  double d2 = 0.0, n2 = 0.0;
  if constexpr (TL::WPG > 1) {
    __shared__ double bt[2 * KT * 4 * 16];
    // the own state rows (the residual's s') from the staged tile where the family stages
    // them unchanged
    constexpr bool kOwnLds = F::kOwnRaw;
    mfma64_shared_b<F, F::S, F::I, MTW, TL::WPG, kOwnLds>(
        m, a, t0, t1, bt,
        [&](int c, int es, const Nb& nb, double& x, double& y) {
          if constexpr (APPLIED) {
            F::row_load(m, es, nb, ld, c, x, y);
          } else {
            x = (double)F::row(m, es, nb, ld, c);
            y = 0.0;
          }
        },
        [&](int c, const Nb& nb, double x, double y) {
          if constexpr (APPLIED)
            return F::row_combine(nb, c, x, y);
          else
            return x;
        },
        [&](int row, int es, double& own, bool& keep) {
          if constexpr (kOwnLds)
            own = 0.0;
          else
            own = ld(row, es);
          keep = true;
          return g[(size_t)row * nel + es];
        },
        [&](int row, int e, double v, double own) {
          const double res = v - own;
          if constexpr (!APPLIED) s_out[(size_t)row * nel + e] = own;
          r_lo(row, e, res);
          d2 += res * res;
          n2 += v * v;
        });
    finish_residual<TL::NW>(d2, n2, ra, ch.iters);
    return;
  }
  for (int t = t0 + slot; t < t1; t += TL::TS) {
    const int e = t * 16 + j;
    const bool valid = e < m.nel;
    const int es = valid ? e : 0;
    Nb nb;
    F::neighbours(m, es, nb);
    double b[KT];
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      const int c = 4 * kt + kq;
      const double v = F::row(m, es, nb, ld, c < F::I ? c : F::I - 1);
      b[kt] = (valid && c < F::I) ? v : 0.0;
    }
    doublex4_t acc[MTW];
    double own[MTW][4];
#pragma unroll
    for (int u = 0; u < MTW; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * (w * MTW + u) + kq + 4 * r;
        const int rc = row < F::S ? row : F::S - 1;
        const double gv = g[(size_t)rc * nel + es];
        own[u][r] = ld(rc, es);
        acc[u][r] = (valid && row < F::S) ? gv : 0.0;
      }
#pragma unroll
    for (int kt = 0; kt < KT; ++kt)
#pragma unroll
      for (int u = 0; u < MTW; ++u) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][kt], b[kt], acc[u], 0, 0, 0);
#pragma unroll
    for (int u = 0; u < MTW; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * (w * MTW + u) + kq + 4 * r;
        if (valid && row < F::S) {
          const double v = acc[u][r], res = v - own[u][r];
          if constexpr (!APPLIED) s_out[(size_t)row * nel + e] = own[u][r];
          r_lo(row, e, res);
          d2 += res * res;
          n2 += v * v;
        }
      }
  }
  finish_residual<TL::NW>(d2, n2, ra, ch.iters);
}

// The last correction sweep of a refinement, where the refinement applies the correction
// in a pass of its own (k_apply_correction): the sweep stores s' = s + correction (the
// FP64 value that pass would store, from the same low-precision correction value) in
// place of the correction, and stamps the control block, so that the pass finds s' in
// place and returns at once.  The correction itself is not stored: a later pass reads it
// only when the stamp does not match, which happens only once the control block has
// moved on (a new step or segment: iteration count 0, so that pass copies s unchanged).
struct FusedApply {
  double* s0;
  double* s1;
  unsigned stamp;
  // i: index of value (row, element) in the component-major state
  __device__ __forceinline__ double load(const CtrlHead& ch, size_t i) const {
    return ((ch.base + ch.iters) & 1 ? s1 : s0)[i];
  }
  __device__ __forceinline__ void put(const CtrlHead& ch, size_t i, double v, double corr) const {
    ((ch.base + ch.iters) & 1 ? s0 : s1)[i] = ch.iters > 0 ? v + corr : v;
  }
  __device__ __forceinline__ void store(const CtrlHead& ch, size_t i, double corr) const {
    put(ch, i, load(ch, i), corr);
  }
  // the stamp lies outside the control block head the other workgroups read, so writing
  // it while they run changes nothing they see
  __device__ __forceinline__ void mark(Ctrl* ctrl) const {
    if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->applied = stamp;
  }
};

// FP32 correction sweep on the matrix cores: lo_out = r_lo + T in(lo_in) with
// v_mfma_f32_16x16x4f32 (same fragments as the FP64 sweep, in FP32; the FP32 result
// fragment holds D[4 (l / 16) + r][l % 16]).
// The FP32 correction sweep's tiling: FP32 fragments take half the registers of FP64
// ones, so the same register budget holds twice as many (96 per lane), and a wavefront
// can take every row tile of an element tile itself.  (With the FP64 budget the 64^3
// transport family split its 3 row tiles over 3 wavefronts, each gathering the whole
// B tile again.)
constexpr int kMfmaMaxA32 = 2 * kMfmaMaxA;
template <class F>
struct Inner32Tiling {
  using TL = Tiling64<F::S, F::I, kMfmaMaxA32>;
  static constexpr int value = TL::NW;
};

template <class F, bool PIPE, bool FUSE = false>
__global__ __launch_bounds__(64 * Inner32Tiling<F>::value) void k_inner32_mfma(
    MeshDev m, Ld32 ld, const float* __restrict__ r_lo, const float* __restrict__ Tf, float* __restrict__ out,
    Ctrl* ctrl, int tiles_per_group, FusedApply fa) {
  using TL = typename Inner32Tiling<F>::TL;
  constexpr int MTW = TL::MTW, KT = TL::KT;
  const CtrlHead ch = ctrl_head(ctrl);
  const int done = ch.done;
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int w = wave % TL::WPG, slot = wave / TL::WPG;
  const int j = lane & 15, kq = lane >> 4;
  float a[MTW][KT];
#pragma unroll
  for (int u = 0; u < MTW; ++u)
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) a[u][kt] = Tf[((w * MTW + u) * KT + kt) * 64 + lane];
  if (done) return;
  const size_t nel = (size_t)m.nel;
  const int ntiles = (m.nel + 15) >> 4;
  const int t0 = remap_block(blockIdx.x, gridDim.x) * tiles_per_group;
  const int t1 = min(t0 + tiles_per_group, ntiles);
  // PIPE: software-pipelined over the wavefront's tiles: the next tile's loads (gather
  // parts and C entries, values unused until its turn) are issued before this tile's
  // MFMAs; they are unconditional (the last tile loads itself again), so that the count
  // of loads in flight is the same on every path.  Without PIPE each tile loads at its
  // turn.  Either way the C entries are added after the products, so their loads overlap
  // the MFMAs.  (PIPE pays while the FP32 state is served from the Infinity Cache and
  // costs when it streams from HBM; the launcher chooses by the state's size.)
  struct In32 {
    float x[KT], y[KT];
    float c[MTW][4];
    Nb nb;
  };
  auto load = [&](int t, In32& in) {
    const int e = t * 16 + j;
    const int es = e < m.nel ? e : 0;
    F::neighbours(m, es, in.nb);
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      const int c = 4 * kt + kq;
      F::row_load(m, es, in.nb, ld, c < F::I ? c : F::I - 1, in.x[kt], in.y[kt]);
    }
#pragma unroll
    for (int u = 0; u < MTW; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * (w * MTW + u) + 4 * kq + r;
        in.c[u][r] = r_lo[(size_t)(row < F::S ? row : F::S - 1) * nel + es];
      }
  };
  const int tf = t0 + slot;
  In32 cur, nxt;
  if constexpr (PIPE) load(tf < t1 ? tf : t0, cur);
  for (int t = tf; t < t1; t += TL::TS) {
    if constexpr (PIPE)
      load(t + TL::TS < t1 ? t + TL::TS : t, nxt);
    else
      load(t, cur);
    const int e = t * 16 + j;
    const bool valid = e < m.nel;
    // FUSE with PIPE: the state values s' is formed from, loaded (unconditionally, in
    // bounds) ahead of the products so that they arrive during them; without PIPE they are
    // loaded in the epilogue (ahead, their registers would cost a wavefront per SIMD)
    constexpr bool kEarly = FUSE && PIPE;
    double sv[kEarly ? MTW : 1][4];
    if constexpr (kEarly) {
#pragma unroll
      for (int u = 0; u < MTW; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * (w * MTW + u) + 4 * kq + r;
          sv[u][r] = fa.load(ch, (size_t)(row < F::S ? row : F::S - 1) * nel + (valid ? e : 0));
        }
    }
    float b[KT];
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      const int c = 4 * kt + kq;
      const float v = F::row_combine(cur.nb, c < F::I ? c : F::I - 1, cur.x[kt], cur.y[kt]);
      b[kt] = (valid && c < F::I) ? v : 0.0f;
    }
    floatx4_t acc[MTW];
#pragma unroll
    for (int u = 0; u < MTW; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[u][r] = 0.0f;
#pragma unroll
    for (int kt = 0; kt < KT; ++kt)
#pragma unroll
      for (int u = 0; u < MTW; ++u) acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][kt], b[kt], acc[u], 0, 0, 0);
    if (valid) {
#pragma unroll
      for (int u = 0; u < MTW; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * (w * MTW + u) + 4 * kq + r;
          if (row < F::S) {
            const float v = acc[u][r] + cur.c[u][r];
            if constexpr (kEarly)
              fa.put(ch, (size_t)row * nel + e, sv[u][r], (double)v);
            else if constexpr (FUSE)
              fa.store(ch, (size_t)row * nel + e, (double)v);
            else
              out[(size_t)row * nel + e] = v;
          }
        }
    }
    if constexpr (PIPE) cur = nxt;
  }
  if constexpr (FUSE) fa.mark(ctrl);
}

// 4 x 4 transpose across a wavefront's four 16-lane rows: on entry v[k] of row q (lanes
// 16 q .. 16 q + 15) is element (q, k); on return v[r] of row q is element (r, q), each lane
// keeping its column l % 16.  Two stages of register-pair swaps: lanes 32 apart
// (v_permlane32_swap), then lanes 16 apart (v_permlane16_swap).
__device__ __forceinline__ void transpose_rows4(float (&v)[4]) {
  unsigned r0 = __float_as_uint(v[0]), r1 = __float_as_uint(v[1]);
  unsigned r2 = __float_as_uint(v[2]), r3 = __float_as_uint(v[3]);
  const auto s02 = __builtin_amdgcn_permlane32_swap(r0, r2, false, false);
  const auto s13 = __builtin_amdgcn_permlane32_swap(r1, r3, false, false);
  r0 = s02[0];
  r2 = s02[1];
  r1 = s13[0];
  r3 = s13[1];
  const auto s01 = __builtin_amdgcn_permlane16_swap(r0, r1, false, false);
  const auto s23 = __builtin_amdgcn_permlane16_swap(r2, r3, false, false);
  v[0] = __uint_as_float(s01[0]);
  v[1] = __uint_as_float(s01[1]);
  v[2] = __uint_as_float(s23[0]);
  v[3] = __uint_as_float(s23[1]);
}

// Plain FP32 sweep on the matrix cores: s_out = g + T in(s_in) with FP32 state, g and
// operator fragments (v_mfma_f32_16x16x4f32, the correction sweep's tiling), and the
// stopping test of the FP64 sweep: the increment norms ||s_out - s_in||^2 and
// ||s_out||^2 are accumulated in FP64 from the FP32 values, left as per-workgroup
// partial sums for the next launch (lagged test, canonical order), and the previous
// sweep's test is taken at the start.  Buffers come from the control block and the
// launch number, as in the FP64 sweep.
// LAGGED: single-problem launches (the lagged test, as in the FP64 sweep); otherwise the
// last workgroup of the problem to arrive takes this sweep's test (batched launches).
template <class F, bool LAGGED>
__device__ __forceinline__ void sweep32_body(const MeshDev& m, const float* __restrict__ g,
                                             const float* __restrict__ Tf, const ResidArgs& ra, float* s0, float* s1,
                                             int tiles_per_group, int bid, int nbk, const LagArgs& lag) {
  using TL = typename Inner32Tiling<F>::TL;
  constexpr int MTW = TL::MTW, KT = TL::KT;
  const CtrlHead ch = ctrl_head(ra.ctrl);
  const unsigned seg = LAGGED ? ra.ctrl->seg_seq : 0u;
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int w = wave % TL::WPG, slot = wave / TL::WPG;
  const int j = lane & 15, kq = lane >> 4;
  float a[MTW][KT];
#pragma unroll
  for (int u = 0; u < MTW; ++u)
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) a[u][kt] = Tf[((w * MTW + u) * KT + kt) * 64 + lane];
  // as in the FP64 sweep: the input buffer follows from the control block head; the
  // previous sweep's partials are loaded first and the first tile's loads overlap their sum
  const int kpre = LAGGED ? (int)(lag.seq - seg) : ch.iters + 1;
  const int parity = (ch.base + kpre - 1) & 1;  // s^(k-1) of the segment
  const size_t nel = (size_t)m.nel;
  const Ld32 ld{parity ? s1 : s0, nel};
  float* __restrict__ out = parity ? s0 : s1;
  const int ntiles = (m.nel + 15) >> 4;
  const int t0 = remap_block(m.order ? nbk - 1 - bid : bid, nbk) * tiles_per_group;
  const int t1 = min(t0 + tiles_per_group, ntiles);
  double d2 = 0.0, n2 = 0.0;
  // Tile inputs as loads only (gather parts, g, the element's own state); the values are
  // combined and masked at the tile's turn.  g is added after the products, so its loads
  // overlap the MFMAs.
  // The element's previous state rows, for the increment: the lane's output rows are
  // 4 kq + r of its row tiles, and the own-state columns it gathered are those of its
  // 16-lane row, kq mod 4.  Where a wavefront takes all row tiles of its element tile (so
  // that the register index is fixed), each row tile's values come from gathered registers
  // by 4 x 4 transposes across the wavefront's four 16-lane rows (transpose_rows4): with
  // o = kOwnCol mod 4, output row r of the tile is own column kOwnCol + 16 u + 4 kq + r, in
  // row (o + r) mod 4 of the transpose of registers k0 + 4 u + (o + r) / 4 + (0 .. 3)
  // (k0 = kOwnCol / 4): one transpose if o = 0, two otherwise.  Elsewhere they are loaded.
  constexpr bool kOwnRegs = TL::WPG == 1;
  struct In32 {
    float x[KT], y[KT];
    float g0[MTW][4], old[kOwnRegs ? 1 : MTW][4];
    Nb nb;
  };
  auto load = [&](int t, bool active, In32& in) {
    const int e = t * 16 + j;
    const int es = (active && e < m.nel) ? e : 0;
    F::neighbours(m, es, in.nb);
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      const int c = 4 * kt + kq;
      F::row_load(m, es, in.nb, ld, c < F::I ? c : F::I - 1, in.x[kt], in.y[kt]);
    }
#pragma unroll
    for (int u = 0; u < MTW; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * (w * MTW + u) + 4 * kq + r;
        const int rc = row < F::S ? row : F::S - 1;
        in.g0[u][r] = g[(size_t)rc * nel + es];
        if constexpr (!kOwnRegs) in.old[u][r] = ld(rc, es);
      }
  };
  const double* parts = nullptr;
  PartialPrefetch<TL::NW> pf;
  if constexpr (LAGGED) {
    parts = lagged_parts(ra, lag);
    pf.issue(parts, nbk);
    __builtin_amdgcn_sched_barrier(0);  // keep the partials' loads ahead of the tile's
    if (uniform_done(ch)) return;
  } else {
    if (ch.done) return;
  }
  const int tf = t0 + slot;
  In32 cur;
  load(tf, tf < t1, cur);
  if constexpr (LAGGED) {
    if (lagged_test<TL::NW>(ra, lag, nbk, bid, seg, pf, parts) == 0) return;
  }
  for (int t = tf; t < t1; t += TL::TS) {
    if (t != tf) load(t, true, cur);
    const int e = t * 16 + j;
    const bool valid = e < m.nel;
    float b[KT];
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      const int c = 4 * kt + kq;
      const float v = F::row_combine(cur.nb, c < F::I ? c : F::I - 1, cur.x[kt], cur.y[kt]);
      b[kt] = (valid && c < F::I) ? v : 0.0f;
    }
    float old[MTW][4];
#pragma unroll
    for (int u = 0; u < MTW; ++u) {
      if constexpr (kOwnRegs) {
        constexpr int k0 = F::kOwnCol / 4, o = F::kOwnCol % 4;
        const int kb = k0 + 4 * u;  // WPG == 1: the wavefront's row tiles are 0 .. MTW - 1
        float t0[4], t1[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) t0[q] = cur.x[kb + q < KT ? kb + q : KT - 1];
        transpose_rows4(t0);
        if constexpr (o != 0) {
#pragma unroll
          for (int q = 0; q < 4; ++q) t1[q] = cur.x[kb + 1 + q < KT ? kb + 1 + q : KT - 1];
          transpose_rows4(t1);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) old[u][r] = (o + r) < 4 ? t0[(o + r) & 3] : t1[(o + r) & 3];
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) old[u][r] = cur.old[u][r];
      }
    }
    floatx4_t acc[MTW];
#pragma unroll
    for (int u = 0; u < MTW; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[u][r] = 0.0f;
#pragma unroll
    for (int kt = 0; kt < KT; ++kt)
#pragma unroll
      for (int u = 0; u < MTW; ++u) acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][kt], b[kt], acc[u], 0, 0, 0);
#pragma unroll
    for (int u = 0; u < MTW; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * (w * MTW + u) + 4 * kq + r;
        if (valid && row < F::S) {
          const float v = acc[u][r] + cur.g0[u][r];
          const double dd = (double)v - (double)old[u][r];
          d2 += dd * dd;
          n2 += (double)v * (double)v;
          out[(size_t)row * nel + e] = v;
        }
      }
  }
  if constexpr (LAGGED)
    lagged_end<TL::NW>(d2, n2, ra, lag, bid);
  else
    finish_residual<TL::NW>(d2, n2, ra, bid, nbk, ch.iters);
}

template <class F>
__global__ __launch_bounds__(64 * Inner32Tiling<F>::value) void k_sweep32_mfma(
    MeshDev m, const float* __restrict__ g, const float* __restrict__ Tf, ResidArgs ra, float* s0, float* s1,
    int tiles_per_group, LagArgs lag) {
  sweep32_body<F, true>(m, g, Tf, ra, s0, s1, tiles_per_group, (int)blockIdx.x, (int)gridDim.x, lag);
}

// The same step completion on the matrix cores: [u_new; g_next] = [w_src; gbe] + M
// [u_old; in(s_prev)] with the stacked operator M of (N + S) x (N + I) held as
// fragments (fragment-major copy Mf, laid out like the sweep operator's).
// The step completion keeps half the sweep's operator registers per wavefront (one
// row tile of the stacked operator for the shallow-water family instead of two): at
// 48 doubles its wavefronts needed 244 VGPRs, so only two fitted per SIMD and the
// matrix cores were busy a third of the time; at 24 they need about 120, and twice as
// many wavefronts share each element tile.
constexpr int kStepMaxA = 24;
template <class F>
struct StepTiling {
  using TL = Tiling64<F::N + F::S, F::N + F::I, kStepMaxA>;
  static constexpr int value = TL::NW;
};
// The step completion with the stacked operator in LDS (LdsAEngine): workgroups of
// kStepLdsWaves wavefronts, kStepLdsTiles element tiles per wavefront, for families whose
// operator fits in 96 KB and whose B fragments (all tiles) and the accumulators of half
// the row tiles fit well within half of the register file (two wavefronts per SIMD).
constexpr int kStepLdsWaves = 8, kStepLdsTiles = 2;
template <class F>
struct StepLdsA {
  static constexpr int MT = (F::N + F::S + 15) / 16, KT = (F::N + F::I + 3) / 4, MH = (MT + 1) / 2;
  static constexpr size_t bytes = (size_t)MT * KT * 64 * 8;
  static constexpr bool ok = bytes <= 96 * 1024 && 2 * KT * kStepLdsTiles + 8 * MH <= 160;
};

// Lagged stopping test of a step's last sweep (lagged FP64 sweeps leave it pending).
struct StepLag {
  int lagged;             // 0: the sweeps took their own tests (batched or refinement)
  unsigned seq_next;      // number the next sweep launch will get
  double tol;
  const double* partials; // the sweeps' partial sets, stride apart, nb pairs each
  int stride, nb;
  double* hist;
  int hist_cap;
};

// ST: element type of the trace state and of g (FP64, or FP32 in the plain FP32 form;
// the contraction itself is FP64 either way).
template <class F, typename ST = double, bool LDSA = false>
__device__ __forceinline__ void step_mfma_body(MeshDev m, ST* s0, ST* s1, const double* __restrict__ Mf,
                                               double* u0, double* u1, const double* __restrict__ w_src,
                                               const double* __restrict__ gbe, ST* __restrict__ g_out,
                                               Ctrl* ctrl, unsigned* cnt, int* step_iters, int step_cap, int lag,
                                               int tiles_per_group, int bid, int nbk, const StepLag& sl) {
  using TL = typename StepTiling<F>::TL;
  constexpr int MTW = TL::MTW, KT = TL::KT, N = F::N, ROWS = F::N + F::S, COLS = F::N + F::I;
  constexpr int NW = LDSA ? kStepLdsWaves : TL::NW;
  const CtrlHead ch = ctrl_head(ctrl);
  const unsigned seg = ctrl->seg_seq;
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int w = wave % TL::WPG, slot = wave / TL::WPG;
  const int j = lane & 15, kq = lane >> 4;
  double a[MTW][KT];
  if constexpr (LDSA) {
    // the operator into LDS while the control block and the partial sums are read
    lds_a_copy<ROWS, COLS, NW>(Mf, reinterpret_cast<double*>(g_smem));
  } else {
#pragma unroll
    for (int u = 0; u < MTW; ++u)
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) a[u][kt] = Mf[((w * MTW + u) * KT + kt) * 64 + lane];
  }
  // K: sweeps of this step (its last local solve read s^(K-1)); conv: the step converged
  int K = ch.iters;
  bool conv = ch.status == 1, reduced = false;
  double res = 0.0;
  if (sl.lagged) {
    __shared__ double sq[kVirtLanes / 64][2];
    __shared__ int s_done, s_status;
    canonical_sums<NW, false>(sl.partials + (size_t)((sl.seq_next - 1u) & 1u) * sl.stride, sl.nb, sq);
    if (threadIdx.x == 0) {
      s_done = ch.done;
      s_status = ch.status;
    }
    __syncthreads();
    if (s_done) {
      conv = s_status == 1;
    } else {
      K = (int)(sl.seq_next - seg) - 1;
      conv = false;
      if (K >= 1) {
        double b;
        res = relative_increment(canonical_total(sq, b), b);
        reduced = true;
        conv = isfinite(res) && res < sl.tol;
      }
    }
  }
  if (!conv) {
    if (reduced && bid == 0 && threadIdx.x == 0) record_test(ctrl, sl.hist, sl.hist_cap, K, res, sl.tol, 1);
    return;
  }
  const int iters = K, base = ch.base, uc = ctrl->ucur;
  const size_t nel = (size_t)m.nel;
  const LdOf<ST> ld{((base + iters - lag) & 1) ? s1 : s0, nel};
  const double* __restrict__ u_old = uc ? u1 : u0;
  double* __restrict__ u_new = uc ? u0 : u1;
  const int ntiles = (m.nel + 15) >> 4;
  const int t0 = remap_block(bid, nbk) * tiles_per_group;
  const int t1 = min(t0 + tiles_per_group, ntiles);
  auto colval = [&](int c, int es, const Nb& nb) {
    // inputs: u_old rows, then the gathered trace rows (the branch is uniform across a
    // wavefront except in the one k tile that straddles the two blocks)
    double v;
    if (c < N)
      v = u_old[(size_t)c * nel + es];
    else
      v = F::row(m, es, nb, ld, c - N);
    return v;
  };
  // the same split into loads and combination for the shared-tile engine
  // FP64 state: no branch, two loads per column whatever its kind (a u row loads its value
  // twice, from one cache line), so the count of loads in flight is the same on every path
  auto colload = [&](int c, int es, const Nb& nb, double& x, double& y) {
    if constexpr (std::is_same_v<ST, double>) {
      const bool uc = c < N;
      int rx, ex, ry, ey;
      F::row_index(nb, es, uc ? 0 : c - N, rx, ex, ry, ey);
      const double* px = uc ? u_old + (size_t)c * nel + es : ld.p + (size_t)rx * nel + ex;
      const double* py = uc ? px : ld.p + (size_t)ry * nel + ey;
      x = *px;
      y = *py;
    } else {
      if (c < N)
        x = u_old[(size_t)c * nel + es];
      else
        x = (double)F::row(m, es, nb, ld, c - N);
      y = 0.0;
    }
  };
  auto colcombine = [&](int c, const Nb& nb, double x, double y) {
    if constexpr (std::is_same_v<ST, double>)
      return c < N ? x : F::row_combine(nb, c - N, x, y);
    else
      return x;
  };
  auto init = [&](int q, int es, double&, bool& keep) {
    double c0 = 0.0;
    if (q < N) {
      if (w_src) c0 = w_src[(size_t)q * nel + es];
    } else if (gbe) {
      c0 = gbe[(size_t)(q - N) * nel + es];
    }
    keep = true;
    return c0;
  };
  // for the shared-tile engine: one load per entry on every path (without a source, a u
  // row already in the caches), the source's absence applied as a mask
  auto init_flat = [&](int q, int es, double&, bool& keep) {
    const bool uq = q < N;
    const double* src = uq ? w_src : gbe;
    keep = src != nullptr;
    const double* base = keep ? src : u_old;
    return base[(size_t)(uq ? q : q - N) * nel + es];
  };
  auto epi = [&](int q, int e, double v, double) {
    if (q < N)
      u_new[(size_t)q * nel + e] = v;
    else if (g_out)
      g_out[(size_t)(q - N) * nel + e] = (ST)v;
  };
  if constexpr (LDSA) {
    // the shared-tile engine adds the C entries after the products where a wavefront has one
    // row tile; it and the one-tile-per-wavefront path start from them otherwise
    constexpr bool kCFirst = !(TL::WPG > 1 && TL::MTW == 1);
    LdsAEngine<F, ROWS, COLS, NW, kStepLdsTiles, StepLdsA<F>::MH, kCFirst> eng;
    eng.gather(m, t0, t1, colload, colcombine);
    eng.apply(reinterpret_cast<const double*>(g_smem), t0, t1, init, epi);
  } else if constexpr (TL::WPG > 1) {
    __shared__ double bt[2 * KT * 4 * 16];
    mfma64_shared_b<F, ROWS, COLS, MTW, TL::WPG>(m, a, t0, t1, bt, colload, colcombine, init_flat, epi);
  } else {
    for (int t = t0 + slot; t < t1; t += TL::TS) {
      const int e = t * 16 + j;
      const bool valid = e < m.nel;
      const int es = valid ? e : 0;
      Nb nb;
      F::neighbours(m, es, nb);
      double b[KT];
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) {
        const int c = 4 * kt + kq;
        const double v = colval(c < COLS ? c : COLS - 1, es, nb);
        b[kt] = (valid && c < COLS) ? v : 0.0;
      }
      doublex4_t acc[MTW];
      double unused;
#pragma unroll
      for (int u = 0; u < MTW; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q = 16 * (w * MTW + u) + kq + 4 * r;
          bool keep;
          const double c0 = init(q < ROWS ? q : ROWS - 1, es, unused, keep);
          acc[u][r] = (valid && q < ROWS) ? c0 : 0.0;
        }
#pragma unroll
      for (int kt = 0; kt < KT; ++kt)
#pragma unroll
        for (int u = 0; u < MTW; ++u) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][kt], b[kt], acc[u], 0, 0, 0);
      if (valid) {
#pragma unroll
        for (int u = 0; u < MTW; ++u)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int q = 16 * (w * MTW + u) + kq + 4 * r;
            if (q < ROWS) epi(q, e, (double)acc[u][r], 0.0);
          }
      }
    }
  }
  // The arrival only elects the workgroup that advances the control block: every
  // workgroup has used its read of the block by now, and the next launch sees all
  // stores of this one, so the stores above need not complete first.
  __shared__ int is_last;
  __syncthreads();
  if (threadIdx.x == 0) is_last = arrive_last(cnt, bid, nbk) ? 1 : 0;
  __syncthreads();
  if (is_last && threadIdx.x == 0) {
    if (reduced) {
      sl.hist[(iters - 1) % sl.hist_cap] = res;
      ctrl->last_res = res;
    }
    step_iters[ctrl->steps_done % step_cap] = iters;
    ctrl->steps_done += 1;
    ctrl->base = (base + iters) & 1;
    ctrl->ucur = uc ^ 1;
    ctrl->iters = 0;
    ctrl->done = 0;
    ctrl->status = 0;
    ctrl->seg_seq = sl.seq_next - 1u;
  }
}

template <class F, typename ST = double>
__global__ __launch_bounds__(64 * StepTiling<F>::value) void k_step_mfma(
    MeshDev m, ST* s0, ST* s1, const double* __restrict__ Mf, double* u0, double* u1,
    const double* __restrict__ w_src, const double* __restrict__ gbe, ST* __restrict__ g_out, Ctrl* ctrl,
    unsigned* cnt, int* step_iters, int step_cap, int lag, int tiles_per_group, StepLag sl) {
  step_mfma_body<F, ST>(m, s0, s1, Mf, u0, u1, w_src, gbe, g_out, ctrl, cnt, step_iters, step_cap, lag,
                        tiles_per_group, (int)blockIdx.x, (int)gridDim.x, sl);
}
// The same with the stacked operator in LDS (dynamic LDS of StepLdsA<F>::bytes).
template <class F, typename ST = double>
__global__ __launch_bounds__(64 * kStepLdsWaves) void k_step_lds(
    MeshDev m, ST* s0, ST* s1, const double* __restrict__ Mf, double* u0, double* u1,
    const double* __restrict__ w_src, const double* __restrict__ gbe, ST* __restrict__ g_out, Ctrl* ctrl,
    unsigned* cnt, int* step_iters, int step_cap, int lag, int tiles_per_group, StepLag sl) {
  step_mfma_body<F, ST, true>(m, s0, s1, Mf, u0, u1, w_src, gbe, g_out, ctrl, cnt, step_iters, step_cap, lag,
                              tiles_per_group, (int)blockIdx.x, (int)gridDim.x, sl);
}

// ---------------------------------------------------------------------------
// batched launches: every problem of a batch that shares this family in one launch
// ---------------------------------------------------------------------------
// Each workgroup looks up its problem and its place among that problem's workgroups in a
// table; the work per workgroup is exactly what a single-problem launch gives it.
template <class F>
__global__ __launch_bounds__(64 * SweepWaves<F>::value) void k_sweep_mfma_batch(
    const BatchEntry* __restrict__ table, const BatchProblem* __restrict__ probs, double tol, int stop) {
  const BatchEntry be = table[blockIdx.x];
  const BatchProblem& P = probs[be.problem];
  if (P.ctrl->steps_done >= P.steps_target) return;  // this problem has taken its steps
  ResidArgs ra;
  ra.ctrl = P.ctrl;
  ra.cnt = P.counters;
  ra.partials = P.partials;
  ra.hist = P.hist;
  ra.hist_cap = P.hist_cap;
  ra.tol = tol;
  ra.stop = stop;
  sweep_mfma_body<F, true, false>(P.mesh, Ld64{P.s0, (size_t)P.mesh.nel}, P.g, P.Tf64, nullptr, ra, P.s0, P.s1,
                                  be.tiles_per_group, be.block, be.nblocks, LagArgs{0u, 0});
}

template <class F, typename ST = double>
__global__ __launch_bounds__(64 * StepTiling<F>::value) void k_step_mfma_batch(
    const BatchEntry* __restrict__ table, const BatchProblem* __restrict__ probs, int lag) {
  const BatchEntry be = table[blockIdx.x];
  const BatchProblem& P = probs[be.problem];
  if (P.ctrl->steps_done >= P.steps_target) return;
  ST* g_out;
  if constexpr (std::is_same_v<ST, float>)
    g_out = P.g32;
  else
    g_out = const_cast<double*>(P.g);
  step_mfma_body<F, ST>(P.mesh, (ST*)P.s0, (ST*)P.s1, P.Mf64, P.u0, P.u1, P.w_src, P.gbe, g_out, P.ctrl,
                        P.counters + kCounterSet, P.step_iters, P.step_cap, lag, be.tiles_per_group, be.block,
                        be.nblocks, StepLag{0, 0u, 0.0, nullptr, 0, 0, nullptr, 1});
}

// One entry of a batched sweep (the work of one workgroup of the family's batched launch),
// FP64 or plain FP32.
template <class F, bool FP32>
__device__ __forceinline__ void batch_sweep_item(const BatchEntry& be, const BatchProblem& P, double tol, int stop) {
  ResidArgs ra;
  ra.ctrl = P.ctrl;
  ra.cnt = P.counters;
  ra.partials = P.partials;
  ra.hist = P.hist;
  ra.hist_cap = P.hist_cap;
  ra.tol = tol;
  ra.stop = stop;
  if constexpr (FP32)
    sweep32_body<F, false>(P.mesh, P.g32, P.Tf32, ra, (float*)P.s0, (float*)P.s1, be.tiles_per_group, be.block,
                           be.nblocks, LagArgs{0u, 0});
  else
    sweep_mfma_body<F, true, false>(P.mesh, Ld64{P.s0, (size_t)P.mesh.nel}, P.g, P.Tf64, nullptr, ra, P.s0, P.s1,
                                    be.tiles_per_group, be.block, be.nblocks, LagArgs{0u, 0});
}

template <class F>
__global__ __launch_bounds__(64 * Inner32Tiling<F>::value) void k_sweep32_batch(
    const BatchEntry* __restrict__ table, const BatchProblem* __restrict__ probs, double tol, int stop) {
  const BatchEntry be = table[blockIdx.x];
  const BatchProblem& P = probs[be.problem];
  if (P.ctrl->steps_done >= P.steps_target) return;
  batch_sweep_item<F, true>(be, P, tol, stop);
}

// ---------------------------------------------------------------------------
// the persistent batched sweep
// ---------------------------------------------------------------------------
// The families it covers: 2D transport (one or two active axes; degree 1 with two axes is
// refused at set-up) and shallow water, every degree the library builds.  Each is swept
// by four wavefronts per workgroup in FP64 and in FP32, so one kernel of 256 threads can
// run any of their entries.
template <class... Fs>
struct FamList {};
using PersistFams =
    FamList<TransportFam<2, 1, 2>, TransportFam<2, 1, 3>, TransportFam<2, 1, 4>, TransportFam<2, 1, 5>,
            TransportFam<2, 1, 6>, TransportFam<2, 1, 7>, TransportFam<2, 2, 3>, TransportFam<2, 2, 4>,
            TransportFam<2, 2, 5>, TransportFam<2, 2, 6>, TransportFam<2, 2, 7>, SweFam<2>, SweFam<3>, SweFam<4>,
            SweFam<5>, SweFam<6>, SweFam<7>>;

template <class F, class... Fs>
struct IndexOf {
  static constexpr int value = -1;
};
template <class F, class G, class... Fs>
struct IndexOf<F, G, Fs...> {
  static constexpr int rest = IndexOf<F, Fs...>::value;
  static constexpr int value = std::is_same_v<F, G> ? 0 : (rest < 0 ? -1 : 1 + rest);
};
template <class F, class L>
struct FamIndex;
template <class F, class... Fs>
struct FamIndex<F, FamList<Fs...>> {
  static constexpr int value = IndexOf<F, Fs...>::value;
};

// Each family's entry body is a function of its own (not inlined), so the persistent kernel
// needs the registers of its largest body, not of all bodies inlined into one function.
template <class F, bool FP32>
__device__ __noinline__ void persist_item(const BatchEntry& be, const BatchProblem& P, double tol, int stop) {
  batch_sweep_item<F, FP32>(be, P, tol, stop);
}

template <bool FP32, class L>
struct PersistDispatch;
template <bool FP32, class... Fs>
struct PersistDispatch<FP32, FamList<Fs...>> {
  __device__ __forceinline__ static void run(int code, const BatchEntry& be, const BatchProblem& P, double tol,
                                             int stop) {
    static_assert(((Tiling64<Fs::S, Fs::I>::NW == 4 && Inner32Tiling<Fs>::value == 4) && ...),
                  "every family of the persistent sweep runs on four wavefronts");
    int i = 0;
    ((code == i++ ? (persist_item<Fs, FP32>(be, P, tol, stop), 0) : 0), ...);
  }
};

// Workgroup g takes entries g, g + G, g + 2 G, ... (G = grid).  Most entries of a late
// round belong to problems that have already converged, and finding that out is a chain of
// three dependent loads (entry, problem, control block), so the workgroup first checks 256
// of its entries at once (one per thread), keeps the live ones in LDS in entry order, and
// then runs only those.  A problem's done flag changes only when the last entry of its
// sweep has arrived, so an entry found live is still live when it runs.
template <bool FP32>
__global__ __launch_bounds__(256, 3) void k_sweep_persist(const BatchEntry* __restrict__ table, int n,
                                                       const BatchProblem* __restrict__ probs, double tol, int stop) {
  __shared__ int live_at[256];
  __shared__ int wave_count[4];
  const int G = (int)gridDim.x, lane = threadIdx.x & 63, w = wave_id();
  for (int base = (int)blockIdx.x; base < n; base += 256 * G) {
    const int it = base + (int)threadIdx.x * G;
    bool live = false;
    if (it < n) {
      const BatchEntry be = table[it];
      const BatchProblem& P = probs[be.problem];
      const CtrlHead ch = ctrl_head(P.ctrl);
      live = !ch.done && P.ctrl->steps_done < P.steps_target;
    }
    // compaction in entry order: per-wavefront ballot, then the wavefronts' counts in order
    const unsigned long long ball = __ballot(live);
    if (lane == 0) wave_count[w] = __popcll(ball);
    __syncthreads();
    int before = 0, total = 0;
    for (int q = 0; q < 4; ++q) {
      before += q < w ? wave_count[q] : 0;
      total += wave_count[q];
    }
    if (live) live_at[before + __popcll(ball & ((1ull << lane) - 1ull))] = it;
    __syncthreads();
    for (int k = 0; k < total; ++k) {
      const BatchEntry be = table[live_at[k]];
      const BatchProblem& P = probs[be.problem];
      PersistDispatch<FP32, PersistFams>::run(be.family, be, P, tol, stop);
    }
    __syncthreads();  // live_at and wave_count are rewritten for the next chunk
  }
}

template <bool FP32>
static int persist_resident();

void launch_sweep_persist(const BatchEntry* table, int n, const BatchProblem* probs, double tol, int fp32,
                          hipStream_t st) {
  if (n <= 0) return;
  const int groups = std::max(1, std::min(n, fp32 ? persist_resident<true>() : persist_resident<false>()));
  if (fp32)
    hipLaunchKernelGGL(k_sweep_persist<true>, dim3(groups), dim3(256), 0, st, table, n, probs, tol, tol >= 0.0 ? 1 : 0);
  else
    hipLaunchKernelGGL(k_sweep_persist<false>, dim3(groups), dim3(256), 0, st, table, n, probs, tol,
                       tol >= 0.0 ? 1 : 0);
}

// ---------------------------------------------------------------------------
// host launchers of one family
// ---------------------------------------------------------------------------
static inline int nblocks(int nel) { return (nel + kBlock - 1) / kBlock; }
static inline int ngroups(int nel) { return (nel + kLanes - 1) / kLanes; }

// Workgroups of a kernel that the device holds at once (its occupancy by registers,
// LDS and wave slots, times the compute units).
template <typename K>
static int resident_groups(K kernel, int threads, size_t lds = 0) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess || per_cu < 1)
    per_cu = 1;
  return per_cu * cus;
}

template <bool FP32>
static int persist_resident() {
  static const int r = resident_groups(k_sweep_persist<FP32>, 256);
  return r;
}

// Matrix-core launches: one round of resident workgroups (resident = how many the
// device holds at once), each taking a contiguous range of 16-element tiles, a
// multiple of ts (tiles in flight per workgroup).  A second, partial round would
// leave most of the chip idle while it runs.  groups <= number of tiles.
static inline void mfma_groups(int nel, int ts, int resident, int& tiles_per_group, int& groups) {
  const int ntiles = (nel + kMfmaTileElems - 1) / kMfmaTileElems;
  resident = std::max(1, resident);
  tiles_per_group = std::max(ts, (ntiles + resident - 1) / resident);
  tiles_per_group = (tiles_per_group + ts - 1) / ts * ts;
  groups = (ntiles + tiles_per_group - 1) / tiles_per_group;
}
// The same with a tuned tiles-per-workgroup (tuned > 0, rounded up to a multiple of ts):
// as many workgroups as that takes, in as many rounds as needed.
static inline void tuned_groups(int nel, int ts, int resident, int tuned, int& tiles_per_group, int& groups) {
  if (tuned <= 0) {
    mfma_groups(nel, ts, resident, tiles_per_group, groups);
    return;
  }
  const int ntiles = (nel + kMfmaTileElems - 1) / kMfmaTileElems;
  tiles_per_group = (std::max(tuned, ts) + ts - 1) / ts * ts;
  groups = std::max(1, (ntiles + tiles_per_group - 1) / tiles_per_group);
}

static inline ResidArgs resid_args(const DevProblem& dp, double tol, int stop) {
  ResidArgs ra;
  ra.ctrl = dp.ctrl;
  ra.cnt = dp.counters;
  ra.partials = dp.partials;
  ra.hist = dp.hist;
  ra.hist_cap = dp.hist_cap;
  ra.tol = tol;
  ra.stop = stop;
  return ra;
}

// dynamic LDS above 64 KB must be enabled per kernel
template <typename K>
static void allow_lds(K kernel, size_t bytes) {
  if (bytes > 65536) (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <class F>
struct Family {
  static constexpr size_t lds_in64 = (size_t)F::I * kLanes * 8;
  static constexpr size_t lds_in32 = (size_t)F::I * kLanes * 4;
  // resident workgroups of each matrix-core kernel (queried once)
  static int res_sweep() {
    static const int r = resident_groups(k_sweep_mfma<F, true>, 64 * Tiling64<F::S, F::I>::NW);
    return r;
  }
  static int res_step() {
    static const int r = resident_groups(k_step_mfma<F>, 64 * StepTiling<F>::value);
    return r;
  }
  // The operator-in-LDS step completion, where the family's operator fits and the mesh
  // fills at least half of a round of its workgroups; else the shared-tile one.  The two
  // give bitwise the same results.
  template <typename ST>
  static int res_step_lds() {
    static const int r = [] {
      allow_lds(k_step_lds<F, ST>, StepLdsA<F>::bytes);
      return resident_groups(k_step_lds<F, ST>, 64 * kStepLdsWaves, StepLdsA<F>::bytes);
    }();
    return r;
  }
  template <typename ST>
  static bool step_lds(int nel) {
    if constexpr (StepLdsA<F>::ok) {
      const long ntiles = (nel + kMfmaTileElems - 1) / kMfmaTileElems;
      return ntiles >= (long)kStepLdsWaves * kStepLdsTiles / 2 * res_step_lds<ST>();
    } else {
      return false;
    }
  }
  template <typename ST>
  static void step_lds_launch(const DevProblem& dp, ST* g_out, const StepLag& sl, int lag, hipStream_t st) {
    if constexpr (StepLdsA<F>::ok) {
      const int ntiles = (dp.mesh.nel + kMfmaTileElems - 1) / kMfmaTileElems;
      const int tpg = kStepLdsWaves * kStepLdsTiles, groups = (ntiles + tpg - 1) / tpg;
      hipLaunchKernelGGL((k_step_lds<F, ST>), dim3(groups), dim3(64 * kStepLdsWaves), StepLdsA<F>::bytes, st,
                         dp.mesh, (ST*)dp.s[0], (ST*)dp.s[1], dp.Mf64, dp.u2[0], dp.u2[1],
                         (const double*)(dp.has_src ? dp.w_src : nullptr),
                         (const double*)(dp.has_src ? dp.gbe : nullptr), g_out, dp.ctrl, dp.counters + kCounterSet,
                         dp.step_iters, dp.step_cap, lag, tpg, sl);
    }
  }
  template <bool PIPE, bool FUSE = false>
  static int res_inner32() {
    static const int r = resident_groups(k_inner32_mfma<F, PIPE, FUSE>, 64 * Inner32Tiling<F>::value);
    return r;
  }
  static int res_sweep32() {
    static const int r = resident_groups(k_sweep32_mfma<F>, 64 * Inner32Tiling<F>::value);
    return r;
  }
  static int res_step32() {
    static const int r = resident_groups(k_step_mfma<F, float>, 64 * StepTiling<F>::value);
    return r;
  }
  template <class LD, class ST, bool APPLIED = false>
  static int res_refine() {
    static const int r = resident_groups(k_refine_mfma<F, LD, ST, APPLIED>, 64 * Tiling64<F::S, F::I>::NW);
    return r;
  }
  static void sweep64(const DevProblem& dp, double tol, unsigned seq, hipStream_t st) {
    using TL = Tiling64<F::S, F::I>;
    const ResidArgs ra = resid_args(dp, tol, tol >= 0.0 ? 1 : 0);
    int tpg, groups;
    tuned_groups(dp.mesh.nel, TL::TS, res_sweep(), dp.sweep_tpg, tpg, groups);
    hipLaunchKernelGGL((k_sweep_mfma<F, true>), dim3(groups), dim3(64 * TL::NW), 0, st, dp.mesh,
                       Ld64{dp.s[0], (size_t)dp.mesh.nel}, (const double*)dp.g, dp.Tf64, (double*)nullptr, ra,
                       dp.s[0], dp.s[1], tpg, LagArgs{seq, dp.partial_stride});
  }
  template <typename ST>
  static void volume_t(const DevProblem& dp, const ST* s_prev, const double* u_old, double* u_out, hipStream_t st) {
    const dim3 grid(ngroups(dp.mesh.nel)), block(kThreads);
    const double* wsrc = dp.has_src ? dp.w_src : nullptr;
    if (dp.be) {
      const size_t lds = (size_t)(F::N + F::I) * kLanes * 8;
      auto kern = k_volume<F, true, ST>;
      allow_lds(kern, lds);
      hipLaunchKernelGGL(kern, grid, block, lds, st, dp.mesh, s_prev, dp.Mvol, u_old, wsrc, (const double*)nullptr,
                         u_out);
    } else {
      auto kern = k_volume<F, false, ST>;
      allow_lds(kern, lds_in64);
      hipLaunchKernelGGL(kern, grid, block, lds_in64, st, dp.mesh, s_prev, dp.Mvol, (const double*)nullptr, wsrc,
                         (const double*)nullptr, u_out);
    }
  }
  static void volume(const DevProblem& dp, const double* s_prev, const double* u_old, double* u_out,
                     hipStream_t st) {
    volume_t<double>(dp, s_prev, u_old, u_out, st);
  }
  static void volume32(const DevProblem& dp, const float* s_prev, const double* u_old, double* u_out,
                       hipStream_t st) {
    volume_t<float>(dp, s_prev, u_old, u_out, st);
  }
  static void sweep32(const DevProblem& dp, double tol, unsigned seq, hipStream_t st) {
    using TL = typename Inner32Tiling<F>::TL;
    const ResidArgs ra = resid_args(dp, tol, tol >= 0.0 ? 1 : 0);
    int tpg, groups;
    tuned_groups(dp.mesh.nel, TL::TS, res_sweep32(), dp.sweep_tpg, tpg, groups);
    hipLaunchKernelGGL((k_sweep32_mfma<F>), dim3(groups), dim3(64 * TL::NW), 0, st, dp.mesh,
                       (const float*)dp.g32, dp.Tf32, ra, (float*)dp.s[0], (float*)dp.s[1], tpg,
                       LagArgs{seq, dp.partial_stride});
  }
  static void sweep32_groups(int nel, int* tpg, int* groups) {
    using TL = typename Inner32Tiling<F>::TL;
    tuned_groups(nel, TL::TS, res_sweep32(), *tpg, *tpg, *groups);
  }
  static void sweep32_batch(const BatchEntry* table, int n, const BatchProblem* probs, double tol, hipStream_t st) {
    using TL = typename Inner32Tiling<F>::TL;
    if (n <= 0) return;
    hipLaunchKernelGGL((k_sweep32_batch<F>), dim3(n), dim3(64 * TL::NW), 0, st, table, probs, tol, tol >= 0.0 ? 1 : 0);
  }
  static void step32_batch(const BatchEntry* table, int n, const BatchProblem* probs, int lag, hipStream_t st) {
    using TL = typename StepTiling<F>::TL;
    if (n <= 0) return;
    hipLaunchKernelGGL((k_step_mfma_batch<F, float>), dim3(n), dim3(64 * TL::NW), 0, st, table, probs, lag);
  }
  static void step32(const DevProblem& dp, int lag, unsigned seq_next, double tol, int lagged, hipStream_t st) {
    using TL = typename StepTiling<F>::TL;
    const StepLag sl{lagged, seq_next, tol, dp.partials, dp.partial_stride, dp.nb_sweep, dp.hist, dp.hist_cap};
    if (step_lds<float>(dp.mesh.nel)) {
      step_lds_launch<float>(dp, dp.g32, sl, lag, st);
      return;
    }
    int tpg, groups;
    mfma_groups(dp.mesh.nel, TL::TS, res_step32(), tpg, groups);
    hipLaunchKernelGGL((k_step_mfma<F, float>), dim3(groups), dim3(64 * TL::NW), 0, st, dp.mesh, (float*)dp.s[0],
                       (float*)dp.s[1], dp.Mf64, dp.u2[0], dp.u2[1], (const double*)(dp.has_src ? dp.w_src : nullptr),
                       (const double*)(dp.has_src ? dp.gbe : nullptr), dp.g32, dp.ctrl, dp.counters + kCounterSet,
                       dp.step_iters, dp.step_cap, lag, tpg, sl);
  }
  static void sweep_groups(int nel, int* tpg, int* groups) {
    using TL = Tiling64<F::S, F::I>;
    tuned_groups(nel, TL::TS, res_sweep(), *tpg, *tpg, *groups);
  }
  static void step_groups(int nel, int* tpg, int* groups) {
    using TL = typename StepTiling<F>::TL;
    mfma_groups(nel, TL::TS, res_step(), *tpg, *groups);
  }
  static void sweep64_batch(const BatchEntry* table, int n, const BatchProblem* probs, double tol, hipStream_t st) {
    using TL = Tiling64<F::S, F::I>;
    if (n <= 0) return;
    hipLaunchKernelGGL((k_sweep_mfma_batch<F>), dim3(n), dim3(64 * TL::NW), 0, st, table, probs, tol,
                       tol >= 0.0 ? 1 : 0);
  }
  static void step_batch(const BatchEntry* table, int n, const BatchProblem* probs, int lag, hipStream_t st) {
    using TL = typename StepTiling<F>::TL;
    if (n <= 0) return;
    hipLaunchKernelGGL((k_step_mfma_batch<F>), dim3(n), dim3(64 * TL::NW), 0, st, table, probs, lag);
  }
  static void step(const DevProblem& dp, int lag, unsigned seq_next, double tol, int lagged, hipStream_t st) {
    using TL = typename StepTiling<F>::TL;
    const StepLag sl{lagged, seq_next, tol, dp.partials, dp.partial_stride, dp.nb_sweep, dp.hist, dp.hist_cap};
    if (step_lds<double>(dp.mesh.nel)) {
      step_lds_launch<double>(dp, dp.g, sl, lag, st);
      return;
    }
    int tpg, groups;
    mfma_groups(dp.mesh.nel, TL::TS, res_step(), tpg, groups);
    hipLaunchKernelGGL((k_step_mfma<F>), dim3(groups), dim3(64 * TL::NW), 0, st, dp.mesh, dp.s[0], dp.s[1],
                       dp.Mf64, dp.u2[0], dp.u2[1], (const double*)(dp.has_src ? dp.w_src : nullptr),
                       (const double*)(dp.has_src ? dp.gbe : nullptr), dp.g, dp.ctrl, dp.counters + kCounterSet,
                       dp.step_iters, dp.step_cap, lag, tpg, sl);
  }
  static void refine32(const DevProblem& dp, const void* lo_in, void* r_out, double tol, unsigned stamp,
                       hipStream_t st) {
    const size_t ne = (size_t)dp.mesh.nel;
    const StSoa32 store{(float*)r_out, ne};
    if (lo_in)
      refine_corrected(dp, Ld32{(const float*)lo_in, ne}, store, tol, stamp, st);
    else
      refine_mfma(dp, Ld64{dp.s[0], ne}, store, tol, st);
  }
  template <class LD, class ST, bool APPLIED = false>
  static void refine_mfma(const DevProblem& dp, const LD& ld, const ST& store, double tol, hipStream_t st) {
    using TL = Tiling64<F::S, F::I>;
    const ResidArgs ra = resid_args(dp, tol, 1);
    int tpg, groups;
    mfma_groups(dp.mesh.nel, TL::TS, res_refine<LD, ST, APPLIED>(), tpg, groups);
    hipLaunchKernelGGL((k_refine_mfma<F, LD, ST, APPLIED>), dim3(groups), dim3(64 * TL::NW), 0, st, dp.mesh, ld,
                       (const double*)dp.g, dp.Tf64, dp.s[0], dp.s[1], store, ra, tpg);
  }
  // A refinement after the segment's first: where the refinement shares element tiles
  // among wavefronts (the wide families), s' = s + correction is applied by a streaming
  // kernel first (which returns at once where the last correction sweep already stored
  // s', stamp) and the refinement gathers s' alone; elsewhere the refinement gathers
  // both and adds them itself.
  template <class LDD, class ST>
  static void refine_corrected(const DevProblem& dp, const LDD& d, const ST& store, double tol, unsigned stamp,
                               hipStream_t st) {
    const size_t ne = (size_t)dp.mesh.nel;
    if constexpr (Tiling64<F::S, F::I>::WPG > 1) {
      hipLaunchKernelGGL((k_apply_correction<F, LDD>), dim3((dp.mesh.nel + 255) / 256), dim3(256), 0, st,
                         (const Ctrl*)dp.ctrl, dp.s[0], dp.s[1], d, dp.mesh.nel, stamp);
      refine_mfma<Ld64, ST, true>(dp, Ld64{dp.s[0], ne}, store, tol, st);
    } else {
      refine_mfma(dp, LdSum<LDD>{Ld64{dp.s[0], ne}, d, 1}, store, tol, st);
    }
  }
  // the pipelined correction sweep while the FP32 state (S values per element) is at most
  // 64 MB, a quarter of the Infinity Cache, and each wavefront has two or more tiles
  static constexpr size_t kPipeBytes = (size_t)64 << 20;
  template <bool PIPE, bool FUSE = false>
  static void inner32_as(const DevProblem& dp, const void* r_lo, const void* lo_in, void* lo_out, unsigned stamp,
                         hipStream_t st) {
    using TL = typename Inner32Tiling<F>::TL;
    int tpg, groups;
    mfma_groups(dp.mesh.nel, TL::TS, res_inner32<PIPE, FUSE>(), tpg, groups);
    hipLaunchKernelGGL((k_inner32_mfma<F, PIPE, FUSE>), dim3(groups), dim3(64 * TL::NW), 0, st, dp.mesh,
                       Ld32{(const float*)lo_in, (size_t)dp.mesh.nel}, (const float*)r_lo, dp.Tf32,
                       (float*)lo_out, dp.ctrl, tpg, FusedApply{dp.s[0], dp.s[1], stamp});
  }
  static void inner32(const DevProblem& dp, const void* r_lo, const void* lo_in, void* lo_out, unsigned stamp,
                      hipStream_t st) {
    using TL = typename Inner32Tiling<F>::TL;
    int tpg, groups;
    mfma_groups(dp.mesh.nel, TL::TS, res_inner32<true>(), tpg, groups);
    // pipelined with two or more tiles per wavefront (one would only load itself again)
    const bool pipe = tpg >= 2 * TL::TS && (size_t)F::S * dp.mesh.nel * sizeof(float) <= kPipeBytes;
    // the last sweep of a refinement stores s' itself where the refinement would apply
    // the correction in a pass of its own
    if constexpr (Tiling64<F::S, F::I>::WPG > 1) {
      if (stamp) {
        if (pipe)
          inner32_as<true, true>(dp, r_lo, lo_in, lo_out, stamp, st);
        else
          inner32_as<false, true>(dp, r_lo, lo_in, lo_out, stamp, st);
        return;
      }
    }
    if (pipe)
      inner32_as<true>(dp, r_lo, lo_in, lo_out, 0u, st);
    else
      inner32_as<false>(dp, r_lo, lo_in, lo_out, 0u, st);
  }
};

// ---------------------------------------------------------------------------
// BF16 correction sweep on MFMA (3D transport, degree 3: S = 48, I = 96)
// ---------------------------------------------------------------------------
// lo_out = r + T in(lo_in) with T, in and r in BF16 and FP32 accumulation, as
// D(48 x 16 elements) = T(48 x 96) B(96 x 16) per tile of 16 elements: 3 x 3
// v_mfma_f32_16x16x32_bf16.  Fragment layout (16x16x32): lane l holds A[l%16][8(l/16)+0..7],
// B[8(l/16)+0..7][l%16] and D[4(l/16)+0..3][l%16].  The correction is element-major
// (48 BF16 per element), so each B fragment is one 16-byte load: 8 consecutive
// state rows of the lane's element or of its upwind neighbour.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned short ushort4_t __attribute__((ext_vector_type(4)));

template <class F, bool FUSE = false>
__global__ __launch_bounds__(kThreads) void k_inner_mfma(MeshDev m, const uint16_t* __restrict__ lo_in,
                                                          const uint16_t* __restrict__ r_lo,
                                                          const uint16_t* __restrict__ T16,
                                                          uint16_t* __restrict__ lo_out, Ctrl* ctrl,
                                                          int tiles_per_wave, FusedApply fa) {
  static_assert(F::S == 48 && F::I == 96 && F::NF == 16, "tiling assumes S = 48, I = 96");
  const CtrlHead ch = ctrl_head(ctrl);
  if (ch.done) return;
  const int lane = threadIdx.x & 63, w = wave_id();
  const int j = lane & 15, kg = lane >> 4;
  // A fragments of T (3 row tiles x 3 k tiles), held for the whole wave
  bf16x8_t a[3][3];
#pragma unroll
  for (int mt = 0; mt < 3; ++mt)
#pragma unroll
    for (int kt = 0; kt < 3; ++kt)
      a[mt][kt] = *reinterpret_cast<const bf16x8_t*>(T16 + (size_t)(mt * 16 + j) * 96 + kt * 32 + 8 * kg);
  const int ntiles = (m.nel + 15) >> 4;
  const int t0 = (remap_block(blockIdx.x, gridDim.x) * kWaves + w) * tiles_per_wave;
  const int t1 = min(t0 + tiles_per_wave, ntiles);
  // A tile's inputs as loads only: the B fragments (inputs 8q .. 8q+7, q = 4 kt + kg:
  // q < 6 -> the upwind neighbour of face q/2, its state rows 8q..; q >= 6 -> the own
  // state rows 8q - 48 ..) and the r entries of the lane's result rows.  Every load is
  // unconditional, at an in-bounds element (the lane's own for an inflow boundary or an
  // idle lane), and the zero of an inflow boundary is selected at the tile's turn.  r is
  // added after the products, so its loads overlap the MFMAs, and the next tile's loads
  // are issued before this tile's MFMAs (the last tile loads itself again).
  struct In16 {
    bf16x8_t b[3];
    ushort4_t r[3];
    bool up[3];
  };
  auto load = [&](int t, In16& in) {
    const int e = t * 16 + j;
    const int es = e < m.nel ? e : 0;
    Nb nb;
    F::neighbours(m, es, nb);
#pragma unroll
    for (int kt = 0; kt < 3; ++kt) {
      const int q = 4 * kt + kg;
      const int src = q < 6 ? nb.get(q >> 1) : es;
      const int row = q < 6 ? 8 * q : 8 * q - 48;
      in.up[kt] = src >= 0;
      in.b[kt] = *reinterpret_cast<const bf16x8_t*>(lo_in + (size_t)(src >= 0 ? src : es) * 48 + row);
    }
#pragma unroll
    for (int mt = 0; mt < 3; ++mt)
      in.r[mt] = *reinterpret_cast<const ushort4_t*>(r_lo + (size_t)es * 48 + mt * 16 + 4 * kg);
  };
  In16 cur, nxt;
  load(t0 < t1 ? t0 : 0, cur);
  for (int t = t0; t < t1; ++t) {
    load(t + 1 < t1 ? t + 1 : t, nxt);
    const int e = t * 16 + j;
    const bool valid = e < m.nel;
    floatx4_t acc[3];
#pragma unroll
    for (int mt = 0; mt < 3; ++mt) acc[mt] = floatx4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 3; ++kt) {
      const bf16x8_t b = (valid && cur.up[kt]) ? cur.b[kt] : bf16x8_t{};
#pragma unroll
      for (int mt = 0; mt < 3; ++mt) acc[mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt][kt], b, acc[mt], 0, 0, 0);
    }
    if (valid) {
#pragma unroll
      for (int mt = 0; mt < 3; ++mt) {
        const ushort4_t rr = cur.r[mt];
        ushort4_t o;
        o.x = f32_to_bf16(acc[mt].x + bf16_to_f32(rr.x));
        o.y = f32_to_bf16(acc[mt].y + bf16_to_f32(rr.y));
        o.z = f32_to_bf16(acc[mt].z + bf16_to_f32(rr.z));
        o.w = f32_to_bf16(acc[mt].w + bf16_to_f32(rr.w));
        if constexpr (FUSE) {
          // s' in the component-major FP64 state: rows mt * 16 + 4 kg + 0..3 of element e
          const size_t i0 = (size_t)(mt * 16 + 4 * kg) * m.nel + e, st = (size_t)m.nel;
          fa.store(ch, i0, (double)bf16_to_f32(o.x));
          fa.store(ch, i0 + st, (double)bf16_to_f32(o.y));
          fa.store(ch, i0 + 2 * st, (double)bf16_to_f32(o.z));
          fa.store(ch, i0 + 3 * st, (double)bf16_to_f32(o.w));
        } else {
          *reinterpret_cast<ushort4_t*>(lo_out + (size_t)e * 48 + mt * 16 + 4 * kg) = o;
        }
      }
    }
    cur = nxt;
  }
  if constexpr (FUSE) fa.mark(ctrl);
}

// BF16-MFMA refinement launchers (only where the tiling applies)
template <class F, bool ENABLE>
struct Bf16Ops {
  static constexpr auto refine = nullptr;
  static constexpr auto inner = nullptr;
};

template <class F>
struct Bf16Ops<F, true> {
  static void refine(const DevProblem& dp, const void* lo_in, void* r_out, double tol, unsigned stamp,
                     hipStream_t st) {
    const size_t ne = (size_t)dp.mesh.nel;
    const StAos16<F::S> store{(uint16_t*)r_out};
    if (lo_in)
      Family<F>::refine_corrected(dp, Ld16Aos<F::S>{(const uint16_t*)lo_in}, store, tol, stamp, st);
    else
      Family<F>::refine_mfma(dp, Ld64{dp.s[0], ne}, store, tol, st);
  }
  static void inner(const DevProblem& dp, const void* r_lo, const void* lo_in, void* lo_out, unsigned stamp,
                    hipStream_t st) {
    // tiles per wavefront: 4 while that fits the grid in one round of resident
    // workgroups, else 8 (longer pipelines over fewer waves)
    static const int resident = resident_groups(k_inner_mfma<F>, kThreads);
    const int tiles = (dp.mesh.nel + 15) / 16;
    const int tpw = tiles <= (long long)resident * kWaves * 4 ? 4 : 8;
    const int per_group = kWaves * tpw;
    const dim3 grid((tiles + per_group - 1) / per_group), block(kThreads);
    const FusedApply fa{dp.s[0], dp.s[1], stamp};
    // this family's refinement applies the correction in a pass of its own (wide tiles)
    static_assert(Tiling64<F::S, F::I>::WPG > 1, "fused application assumes the separate pass");
    if (stamp)
      hipLaunchKernelGGL((k_inner_mfma<F, true>), grid, block, 0, st, dp.mesh, (const uint16_t*)lo_in,
                         (const uint16_t*)r_lo, dp.T16, (uint16_t*)lo_out, dp.ctrl, tpw, fa);
    else
      hipLaunchKernelGGL((k_inner_mfma<F, false>), grid, block, 0, st, dp.mesh, (const uint16_t*)lo_in,
                         (const uint16_t*)r_lo, dp.T16, (uint16_t*)lo_out, dp.ctrl, tpw, fa);
  }
};

// FP32 correction sweep with element-major correction and residual (3D transport, degree 3:
// S = 48, I = 96): lo_out = r + T in(lo_in) with v_mfma_f32_16x16x4f32 as in k_inner32_mfma,
// but with the contraction's columns taken in a permuted order, so that a lane's inputs
// are consecutive state rows: k tile 4 b + s gives lane (j, kq) input column
// 16 b + 4 kq + s, so the four k tiles 4 b .. 4 b + 3 of a lane are one 16-byte load of rows
// 16 b + 4 kq .. + 3 of one element (b < 3: the upwind neighbour across face b, whose
// state rows 16 b .. are that face's inflow; b >= 3: the element's own rows).  The operator
// fragments are read in the same permuted order from the FP32 fragment array.  The result
// rows 4 kq + 0..3 of a row tile are consecutive too: the residual is one 16-byte load and
// the correction one 16-byte store per row tile.  Tiles and pipelining as in k_inner_mfma;
// FUSE as in k_inner32_mfma, unpipelined, with the FP64 state values s' is formed from
// loaded in the epilogue (the next tile's loads, or those values, held over the products
// would cost a wavefront per SIMD).
typedef float floatx4v_t __attribute__((ext_vector_type(4)));

template <class F, bool FUSE = false>
__global__ __launch_bounds__(kThreads) void k_inner32_aos(MeshDev m, const float* __restrict__ lo_in,
                                                           const float* __restrict__ r_lo,
                                                           const float* __restrict__ Tf,
                                                           float* __restrict__ lo_out, Ctrl* ctrl,
                                                           int tiles_per_wave, FusedApply fa) {
  static_assert(F::S == 48 && F::I == 96 && F::NF == 16, "tiling assumes S = 48, I = 96");
  constexpr int KT = 24;  // the FP32 fragment array's k tiles (96 columns)
  const CtrlHead ch = ctrl_head(ctrl);
  if (ch.done) return;
  const int lane = threadIdx.x & 63, w = wave_id();
  const int j = lane & 15, kq = lane >> 4;
  // A[16 mt + j][16 b + 4 kq + s] for k tile 4 b + s; the fragment array holds A[16 mt +
  // l % 16][4 k + l / 16] of k tile k at lane l
  float a[3][KT];
#pragma unroll
  for (int mt = 0; mt < 3; ++mt)
#pragma unroll
    for (int b = 0; b < 6; ++b)
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) a[mt][4 * b + s4] = Tf[(mt * KT + 4 * b + kq) * 64 + 16 * s4 + j];
  const int ntiles = (m.nel + 15) >> 4;
  const int t0 = (remap_block(blockIdx.x, gridDim.x) * kWaves + w) * tiles_per_wave;
  const int t1 = min(t0 + tiles_per_wave, ntiles);
  // a tile's inputs as loads only (unconditional, at an in-bounds element: the lane's own
  // for an inflow boundary or an idle lane; the zero of an inflow boundary is selected at
  // the tile's turn), and the next tile's loads in flight over this tile's MFMAs
  struct In32a {
    floatx4v_t b[6];
    floatx4v_t r[3];
    bool up[3];
  };
  auto load = [&](int t, In32a& in) {
    const int e = t * 16 + j;
    const int es = e < m.nel ? e : 0;
    Nb nb;
    F::neighbours(m, es, nb);
#pragma unroll
    for (int b = 0; b < 6; ++b) {
      const int src = b < 3 ? nb.get(b) : es;
      if (b < 3) in.up[b] = src >= 0;
      const int row = 16 * (b < 3 ? b : b - 3) + 4 * kq;
      in.b[b] = *reinterpret_cast<const floatx4v_t*>(lo_in + (size_t)(src >= 0 ? src : es) * 48 + row);
    }
#pragma unroll
    for (int mt = 0; mt < 3; ++mt)
      in.r[mt] = *reinterpret_cast<const floatx4v_t*>(r_lo + (size_t)es * 48 + 16 * mt + 4 * kq);
  };
  In32a cur, nxt;
  if constexpr (!FUSE) load(t0 < t1 ? t0 : 0, cur);
  for (int t = t0; t < t1; ++t) {
    const int e = t * 16 + j;
    const bool valid = e < m.nel;
    if constexpr (FUSE)
      load(t, cur);
    else
      load(t + 1 < t1 ? t + 1 : t, nxt);
    floatx4_t acc[3];
#pragma unroll
    for (int mt = 0; mt < 3; ++mt) acc[mt] = floatx4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int b = 0; b < 6; ++b) {
      const bool use = valid && (b >= 3 || cur.up[b < 3 ? b : 0]);
      const floatx4v_t bv = use ? cur.b[b] : floatx4v_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
        for (int mt = 0; mt < 3; ++mt)
          acc[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[mt][4 * b + s4], bv[s4], acc[mt], 0, 0, 0);
    }
    if (valid) {
#pragma unroll
      for (int mt = 0; mt < 3; ++mt) {
        floatx4v_t o;
#pragma unroll
        for (int r = 0; r < 4; ++r) o[r] = acc[mt][r] + cur.r[mt][r];
        if constexpr (FUSE) {
          // s' in the component-major FP64 state: rows 16 mt + 4 kq + 0..3 of element e
          const size_t i0 = (size_t)(16 * mt + 4 * kq) * m.nel + e, st = (size_t)m.nel;
#pragma unroll
          for (int r = 0; r < 4; ++r) fa.store(ch, i0 + r * st, (double)o[r]);
        } else {
          *reinterpret_cast<floatx4v_t*>(lo_out + (size_t)e * 48 + 16 * mt + 4 * kq) = o;
        }
      }
    }
    if constexpr (!FUSE) cur = nxt;
  }
  if constexpr (FUSE) fa.mark(ctrl);
}

template <class F>
struct HasMfmaTiling {
  static constexpr bool value = false;
};
template <>
struct HasMfmaTiling<TransportFam<3, 3, 4>> {
  static constexpr bool value = true;
};

// The FP32 correction form's refinement and correction sweep: element-major correction
// and residual where the family has the tiling of k_inner32_aos and the FP32 state is
// larger than a quarter of the Infinity Cache (64 MB; below that the component-major
// state is served from that cache and its pipelined sweep measured as fast), else the
// component-major form of Family<F>.  The choice is a function of the element count, so
// a problem's refinement, correction sweeps and correction application all take the same
// layout.
template <class F, bool AOS>
struct Fp32Ops {
  static void refine(const DevProblem& dp, const void* lo_in, void* r_out, double tol, unsigned stamp,
                     hipStream_t st) {
    Family<F>::refine32(dp, lo_in, r_out, tol, stamp, st);
  }
  static void inner(const DevProblem& dp, const void* r_lo, const void* lo_in, void* lo_out, unsigned stamp,
                    hipStream_t st) {
    Family<F>::inner32(dp, r_lo, lo_in, lo_out, stamp, st);
  }
};

template <class F>
struct Fp32Ops<F, true> {
  static bool aos(const DevProblem& dp) { return (size_t)F::S * dp.mesh.nel * sizeof(float) > Family<F>::kPipeBytes; }
  static void refine(const DevProblem& dp, const void* lo_in, void* r_out, double tol, unsigned stamp,
                     hipStream_t st) {
    if (!aos(dp)) {
      Family<F>::refine32(dp, lo_in, r_out, tol, stamp, st);
      return;
    }
    const size_t ne = (size_t)dp.mesh.nel;
    const StAos32<F::S> store{(float*)r_out};
    if (lo_in)
      Family<F>::refine_corrected(dp, Ld32Aos<F::S>{(const float*)lo_in}, store, tol, stamp, st);
    else
      Family<F>::refine_mfma(dp, Ld64{dp.s[0], ne}, store, tol, st);
  }
  static void inner(const DevProblem& dp, const void* r_lo, const void* lo_in, void* lo_out, unsigned stamp,
                    hipStream_t st) {
    if (!aos(dp)) {
      Family<F>::inner32(dp, r_lo, lo_in, lo_out, stamp, st);
      return;
    }
    // tiles per wavefront as in the BF16 correction sweep
    static const int resident = resident_groups(k_inner32_aos<F>, kThreads);
    const int tiles = (dp.mesh.nel + 15) / 16;
    const int tpw = tiles <= (long long)resident * kWaves * 4 ? 4 : 8;
    const int per_group = kWaves * tpw;
    const dim3 grid((tiles + per_group - 1) / per_group), block(kThreads);
    const FusedApply fa{dp.s[0], dp.s[1], stamp};
    static_assert(Tiling64<F::S, F::I>::WPG > 1, "fused application assumes the separate pass");
    if (stamp)
      hipLaunchKernelGGL((k_inner32_aos<F, true>), grid, block, 0, st, dp.mesh, (const float*)lo_in,
                         (const float*)r_lo, dp.Tf32, (float*)lo_out, dp.ctrl, tpw, fa);
    else
      hipLaunchKernelGGL((k_inner32_aos<F, false>), grid, block, 0, st, dp.mesh, (const float*)lo_in,
                         (const float*)r_lo, dp.Tf32, (float*)lo_out, dp.ctrl, tpw, fa);
  }
};

// ---------------------------------------------------------------------------
// registry
// ---------------------------------------------------------------------------
template <class F>
static const KernelSet* set_of() {
  static const KernelSet ks = {&Family<F>::sweep64,       &Family<F>::volume,
                               &Family<F>::step,          &Fp32Ops<F, HasMfmaTiling<F>::value>::refine,
                               &Fp32Ops<F, HasMfmaTiling<F>::value>::inner, Bf16Ops<F, HasMfmaTiling<F>::value>::refine,
                               Bf16Ops<F, HasMfmaTiling<F>::value>::inner,
                               &Family<F>::sweep_groups,  &Family<F>::step_groups,
                               &Family<F>::sweep64_batch, &Family<F>::step_batch,
                               &Family<F>::sweep32,       &Family<F>::volume32,
                               &Family<F>::step32,        &Family<F>::sweep32_groups,
                               &Family<F>::sweep32_batch, &Family<F>::step32_batch,
                               FamIndex<F, PersistFams>::value};
  return &ks;
}

template <int DIM, int NA>
static const KernelSet* transport_p(int p) {
  if constexpr (DIM == 2) {
    switch (p) {
      case 1: return set_of<TransportFam<2, NA, 2>>();
      case 2: return set_of<TransportFam<2, NA, 3>>();
      case 3: return set_of<TransportFam<2, NA, 4>>();
      case 4: return set_of<TransportFam<2, NA, 5>>();
      case 5: return set_of<TransportFam<2, NA, 6>>();
      case 6: return set_of<TransportFam<2, NA, 7>>();
    }
  } else {
    switch (p) {
      case 1: return set_of<TransportFam<3, NA, 2>>();
      case 2: return set_of<TransportFam<3, NA, 3>>();
      case 3: return set_of<TransportFam<3, NA, 4>>();
      case 4: return set_of<TransportFam<3, NA, 5>>();
    }
  }
  return nullptr;
}

const KernelSet* find_kernels(int pde, int dim, int na, int p) {
  if (pde == 0) {
    if (dim == 2) {
      if (na == 1) return transport_p<2, 1>(p);
      if (na == 2) return transport_p<2, 2>(p);
    } else if (dim == 3) {
      if (na == 1) return transport_p<3, 1>(p);
      if (na == 2) return transport_p<3, 2>(p);
      if (na == 3) return transport_p<3, 3>(p);
    }
    return nullptr;
  }
  if (pde == 1 && dim == 2) {
    switch (p) {
      case 1: return set_of<SweFam<2>>();
      case 2: return set_of<SweFam<3>>();
      case 3: return set_of<SweFam<4>>();
      case 4: return set_of<SweFam<5>>();
      case 5: return set_of<SweFam<6>>();
      case 6: return set_of<SweFam<7>>();
    }
  }
  if (pde == 2 && dim == 2) {
    switch (p) {
      case 1: return set_of<EulerFam<2>>();
      case 2: return set_of<EulerFam<3>>();
      case 3: return set_of<EulerFam<4>>();
      case 4: return set_of<EulerFam<5>>();
      case 5: return set_of<EulerFam<6>>();
    }
  }
  return nullptr;
}

// ---------------------------------------------------------------------------
// variable velocity: per-element operators streamed from HBM
// ---------------------------------------------------------------------------
// s^{k+1}_e = g_e + T_e in_e(s^k) with a different T_e (S x I) for every element.  No
// operator entry is used by two elements, so the sweep is a stream of the T_e from
// HBM (matrix cores would only help with reuse).  T is stored tile-major: the
// operators of a tile of 16 elements are one contiguous block, entry (c, r) of its
// elements 16 consecutive doubles.  Lane l of a wavefront takes element 16 t + l % 16
// of tile t and rows 4 RPL rb + l / 16 + 4 k (k < RPL) of row block rb, so every
// operator load of a wavefront is one contiguous 512-byte run and a wavefront streams
// one contiguous range per input column.  The same lanes gather the inputs in_e(c)
// (the four lanes of an element read one address).
template <class F>
__global__ __launch_bounds__(256) void k_sweep_var(MeshDev m, const double* __restrict__ g,
                                                    const double* __restrict__ Tv, ResidArgs ra, double* s0,
                                                    double* s1, LagArgs lag) {
  constexpr int NRB = var_row_blocks(F::S), RPL = var_rows_per_lane(F::S);
  const CtrlHead ch = ctrl_head(ra.ctrl);
  const unsigned seg = ra.ctrl->seg_seq;
  const int lane = threadIdx.x & 63, w = wave_id();
  const int item = remap_block(blockIdx.x, gridDim.x) * 4 + w;  // (tile, row block) of this wavefront
  const int tile = item / NRB, rb = item - tile * NRB;
  const int e = tile * 16 + (lane & 15);
  const bool valid = e < m.nel;
  const int es = valid ? e : 0;  // stand-in element for lanes past the end: loads stay in bounds
  const size_t nel = (size_t)m.nel;
  int row[RPL];
  bool live[RPL];
  double acc[RPL];
#pragma unroll
  for (int k = 0; k < RPL; ++k) {
    const int r = rb * 4 * RPL + (lane >> 4) + 4 * k;
    live[k] = valid && r < F::S;
    row[k] = r < F::S ? r : F::S - 1;
    acc[k] = g[(size_t)row[k] * nel + es];
  }
  // the stopping test of the previous sweep (lagged, like the matrix-core sweep)
  const int ks = lagged_begin<4>(ra, lag, (int)gridDim.x, (int)blockIdx.x, ch, seg);
  if (ks == 0) return;
  const int parity = (ch.base + ks - 1) & 1;
  const Ld64 ld{parity ? s1 : s0, nel};
  double* out = parity ? s0 : s1;
  Nb nb;
  F::neighbours(m, es, nb);
  const int ntiles = (m.nel + 15) >> 4;
  const double* __restrict__ Te =
      Tv + (size_t)(tile < ntiles ? tile : 0) * (F::I * F::S * 16) + (lane & 15);  // in bounds for idle lanes
#pragma unroll 8
  for (int c = 0; c < F::I; ++c) {
    const double x = F::row(m, es, nb, ld, c);
#pragma unroll
    for (int k = 0; k < RPL; ++k) acc[k] = fma(Te[(c * F::S + row[k]) * 16], x, acc[k]);
  }
  double d2 = 0.0, n2 = 0.0;
#pragma unroll
  for (int k = 0; k < RPL; ++k) {
    const double old = ld(row[k], es);
    if (live[k]) {
      const double dd = acc[k] - old;
      d2 += dd * dd;
      n2 += acc[k] * acc[k];
    }
  }
#pragma unroll
  for (int k = 0; k < RPL; ++k)
    if (live[k]) out[(size_t)row[k] * nel + e] = acc[k];
  lagged_end<4>(d2, n2, ra, lag, (int)blockIdx.x);
}

// in(s) of every element into in[c][e] (recovery of the element solutions)
template <class F>
__global__ __launch_bounds__(kBlock) void k_gather_var(MeshDev m, const double* __restrict__ s, double* __restrict__ in) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.nel) return;
  Nb nb;
  F::neighbours(m, e, nb);
  const Ld64 ld{s, (size_t)m.nel};
#pragma unroll 4
  for (int c = 0; c < F::I; ++c) in[(size_t)c * m.nel + e] = F::row(m, e, nb, ld, c);
}

template <class F>
struct VarFamily {
  static void sweep64(const DevProblem& dp, double tol, unsigned seq, hipStream_t st) {
    const ResidArgs ra = resid_args(dp, tol, tol >= 0.0 ? 1 : 0);
    const long long groups = var_sweep_groups(dp.mesh.nel, F::S);
    hipLaunchKernelGGL((k_sweep_var<F>), dim3((unsigned)groups), dim3(256), 0, st, dp.mesh, (const double*)dp.g,
                       dp.Tv, ra, dp.s[0], dp.s[1], LagArgs{seq, dp.partial_stride});
  }
  // u_out = w_src + R_e in(s_prev)  (steady only)
  static void volume(const DevProblem& dp, const double* s_prev, const double*, double* u_out, hipStream_t st) {
    const int nel = dp.mesh.nel;
    hipLaunchKernelGGL((k_gather_var<F>), dim3(nblocks(nel)), dim3(kBlock), 0, st, dp.mesh, s_prev, dp.in_scratch);
    if (dp.has_src) (void)hipMemcpyAsync(u_out, dp.w_src, (size_t)F::N * nel * 8, hipMemcpyDeviceToDevice, st);
    launch_matvec_pe(dp.Rv, F::N, F::I, dp.in_scratch, u_out, nel, dp.has_src, st);
  }
};

template <class F>
static const KernelSet* var_set_of() {
  static const KernelSet ks = [] {
    KernelSet k{};
    k.sweep64 = &VarFamily<F>::sweep64;
    k.volume = &VarFamily<F>::volume;
    k.persist = -1;
    return k;
  }();
  return &ks;
}

template <int DIM, int NA>
static const KernelSet* var_transport_p(int p) {
  if constexpr (DIM == 2) {
    switch (p) {
      case 1: return var_set_of<TransportFam<2, NA, 2>>();
      case 2: return var_set_of<TransportFam<2, NA, 3>>();
      case 3: return var_set_of<TransportFam<2, NA, 4>>();
      case 4: return var_set_of<TransportFam<2, NA, 5>>();
      case 5: return var_set_of<TransportFam<2, NA, 6>>();
      case 6: return var_set_of<TransportFam<2, NA, 7>>();
    }
  } else {
    switch (p) {
      case 1: return var_set_of<TransportFam<3, NA, 2>>();
      case 2: return var_set_of<TransportFam<3, NA, 3>>();
      case 3: return var_set_of<TransportFam<3, NA, 4>>();
      case 4: return var_set_of<TransportFam<3, NA, 5>>();
    }
  }
  return nullptr;
}

const KernelSet* find_var_kernels(int dim, int na, int p) {
  if (dim == 2) {
    if (na == 1) return var_transport_p<2, 1>(p);
    if (na == 2) return var_transport_p<2, 2>(p);
  } else if (dim == 3) {
    if (na == 1) return var_transport_p<3, 1>(p);
    if (na == 2) return var_transport_p<3, 2>(p);
    if (na == 3) return var_transport_p<3, 3>(p);
  }
  return nullptr;
}

// ---------------------------------------------------------------------------
// setup-time kernels (FP64, runtime sizes)
// ---------------------------------------------------------------------------
__global__ void k_matvec(const double* __restrict__ M, int rows, int cols, const double* __restrict__ x,
                         double* __restrict__ y, int nel, int accumulate) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nel) return;
  const size_t n = (size_t)nel;
  for (int r = 0; r < rows; ++r) {
    double acc = accumulate ? y[r * n + e] : 0.0;
    for (int c = 0; c < cols; ++c) acc = fma(M[(size_t)r * cols + c], x[c * n + e], acc);
    y[r * n + e] = acc;
  }
}

// y (+)= M x for EB elements per workgroup (M: rows x cols, row-major, shared by every
// element; x, y: SoA).  The workgroup stages its elements' x columns in LDS once; thread t
// takes element t % EB and every (256 / EB)-th block of four rows, so each x value read
// from LDS feeds four FMAs and no x value is read from memory twice.  Every output is one
// FMA chain over c in ascending order from the old value (or 0): the same arithmetic as
// k_matvec, so the results are bitwise those of k_matvec.
template <int EB>
__global__ __launch_bounds__(256) void k_matvec_lds(const double* __restrict__ M, int rows, int cols,
                                                    const double* __restrict__ x, double* __restrict__ y, int nel,
                                                    int accumulate) {
  extern __shared__ double xs[];  // [cols][EB]
  constexpr int kStreams = 256 / EB, kR = 4;
  const int t = threadIdx.x, el = t % EB, stream = t / EB;
  const int e0 = blockIdx.x * EB;
  const size_t n = (size_t)nel;
  for (int i = t; i < cols * EB; i += 256) {
    const int c = i / EB, l = i % EB;
    xs[i] = e0 + l < nel ? x[(size_t)c * n + e0 + l] : 0.0;
  }
  __syncthreads();
  const int e = e0 + el;
  if (e >= nel) return;
  for (int r0 = stream * kR; r0 < rows; r0 += kStreams * kR) {
    // rows past the end compute on row rows-1 and are not stored
    const double* Mr[kR];
    double acc[kR];
#pragma unroll
    for (int k = 0; k < kR; ++k) {
      const int r = min(r0 + k, rows - 1);
      Mr[k] = M + (size_t)r * cols;
      acc[k] = accumulate ? y[(size_t)r * n + e] : 0.0;
    }
#pragma unroll 2
    for (int c = 0; c < cols; ++c) {
      const double xv = xs[c * EB + el];
#pragma unroll
      for (int k = 0; k < kR; ++k) acc[k] = fma(Mr[k][c], xv, acc[k]);
    }
#pragma unroll
    for (int k = 0; k < kR; ++k)
      if (r0 + k < rows) y[(size_t)(r0 + k) * n + e] = acc[k];
  }
}

void launch_matvec(const double* M, int rows, int cols, const double* x, double* y, int nel, bool accumulate,
                   hipStream_t st) {
  if (nel <= 0 || rows <= 0) return;
  constexpr size_t kLds = 64 * 1024;
  if ((size_t)cols * 64 * sizeof(double) <= kLds) {
    hipLaunchKernelGGL(k_matvec_lds<64>, dim3((nel + 63) / 64), dim3(256), (size_t)cols * 64 * sizeof(double), st, M,
                       rows, cols, x, y, nel, accumulate ? 1 : 0);
  } else if ((size_t)cols * 32 * sizeof(double) <= kLds) {
    hipLaunchKernelGGL(k_matvec_lds<32>, dim3((nel + 31) / 32), dim3(256), (size_t)cols * 32 * sizeof(double), st, M,
                       rows, cols, x, y, nel, accumulate ? 1 : 0);
  } else {
    hipLaunchKernelGGL(k_matvec, dim3(nblocks(nel)), dim3(kBlock), 0, st, M, rows, cols, x, y, nel,
                       accumulate ? 1 : 0);
  }
}

__global__ void k_matvec_pe(const double* __restrict__ M, int rows, int cols, const double* __restrict__ x,
                            double* __restrict__ y, int nel, int accumulate) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;  // = r * nel + e
  if (t >= (size_t)rows * nel) return;
  const size_t n = (size_t)nel;
  const size_t r = t / n, e = t - r * n;
  double acc = accumulate ? y[t] : 0.0;
  for (int c = 0; c < cols; ++c) acc = fma(M[((size_t)c * rows + r) * n + e], x[c * n + e], acc);
  y[t] = acc;
}

void launch_matvec_pe(const double* M, int rows, int cols, const double* x, double* y, int nel, bool accumulate,
                      hipStream_t st) {
  const size_t total = (size_t)rows * nel;
  hipLaunchKernelGGL(k_matvec_pe, dim3((unsigned)((total + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, M, rows,
                     cols, x, y, nel, accumulate ? 1 : 0);
}

// ext [nel][K] <-> SoA [K][nel] through a 64-element x 32-value LDS tile, so that both the
// reads and the writes are runs of consecutive addresses.
constexpr int kTrE = 64, kTrK = 32;
__global__ __launch_bounds__(256) void k_transpose_tiled(const double* __restrict__ src, double* __restrict__ dst,
                                                         int K, int nel, int to_soa) {
  __shared__ double tile[kTrE][kTrK + 1];
  const int e0 = blockIdx.x * kTrE, k0 = blockIdx.y * kTrK;
  const int ne = min(kTrE, nel - e0), nk = min(kTrK, K - k0);
  const size_t n = (size_t)nel;
  if (to_soa) {
    for (int i = threadIdx.x; i < kTrE * kTrK; i += 256) {
      const int el = i / kTrK, kl = i % kTrK;
      if (el < ne && kl < nk) tile[el][kl] = src[(size_t)(e0 + el) * K + k0 + kl];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kTrE * kTrK; i += 256) {
      const int kl = i / kTrE, el = i % kTrE;
      if (el < ne && kl < nk) dst[(size_t)(k0 + kl) * n + e0 + el] = tile[el][kl];
    }
  } else {
    for (int i = threadIdx.x; i < kTrE * kTrK; i += 256) {
      const int kl = i / kTrE, el = i % kTrE;
      if (el < ne && kl < nk) tile[el][kl] = src[(size_t)(k0 + kl) * n + e0 + el];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kTrE * kTrK; i += 256) {
      const int el = i / kTrK, kl = i % kTrK;
      if (el < ne && kl < nk) dst[(size_t)(e0 + el) * K + k0 + kl] = tile[el][kl];
    }
  }
}

static void launch_transpose(const double* src, double* dst, int K, int nel, int to_soa, hipStream_t st) {
  if (K <= 0 || nel <= 0) return;
  const dim3 grid((unsigned)((nel + kTrE - 1) / kTrE), (unsigned)((K + kTrK - 1) / kTrK));
  hipLaunchKernelGGL(k_transpose_tiled, grid, dim3(256), 0, st, src, dst, K, nel, to_soa);
}

void launch_ext_to_soa(const double* ext, double* soa, int K, int nel, hipStream_t st) {
  launch_transpose(ext, soa, K, nel, 1, st);
}

void launch_soa_to_ext(const double* soa, double* ext, int K, int nel, hipStream_t st) {
  launch_transpose(soa, ext, K, nel, 0, st);
}

__global__ void k_fill(double* p, double v, size_t count) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

void launch_fill(double* p, double v, size_t count, hipStream_t st) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((count + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, p, v, count);
}

__global__ void k_fill_bytes(uint32_t* p, size_t words) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < words) p[i] = 0u;
}

void launch_fill_bytes(void* p, size_t bytes, hipStream_t st) {
  const size_t words = bytes / 4;
  if (words == 0) return;
  hipLaunchKernelGGL(k_fill_bytes, dim3((unsigned)((words + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                     (uint32_t*)p, words);
}

__device__ void ctrl_reset(Ctrl* c, int full, unsigned seq_next) {
  if (full == 1) {
    c->base = 0;
    c->ucur = 0;
    c->steps_done = 0;
    c->last_res = 0.0;
  } else {
    if (full == 2 && !c->done) {
      // the current segment is still running: continue it (the next sweep is number iters + 1)
      c->seg_seq = seq_next - 1u - (unsigned)c->iters;
      return;
    }
    c->base = (c->base + c->iters) & 1;  // the new segment starts from the latest state
  }
  c->done = 0;
  c->iters = 0;
  c->status = 0;
  c->seg_seq = seq_next - 1u;
}

__global__ void k_ctrl_reset(Ctrl* c, int full, unsigned seq_next) {
  if (threadIdx.x == 0) ctrl_reset(c, full, seq_next);
}

__global__ void k_ctrl_reset_batch(const BatchProblem* probs, int n, int full) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) ctrl_reset(probs[i].ctrl, full, 0u);  // batched sweeps take their own tests
}

__global__ void k_ctrl_gather(const BatchProblem* probs, int n, Ctrl* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = *probs[i].ctrl;
}

void launch_ctrl_reset_batch(const BatchProblem* probs, int n, int full, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_ctrl_reset_batch, dim3((n + 63) / 64), dim3(64), 0, st, probs, n, full);
}

void launch_ctrl_gather(const BatchProblem* probs, int n, Ctrl* out, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(k_ctrl_gather, dim3((n + 63) / 64), dim3(64), 0, st, probs, n, out);
}

__global__ void k_counters_reset(unsigned* cnt) {
  for (int i = threadIdx.x; i < 2 * (kCounterGroups + 1); i += blockDim.x) cnt[i * kCounterStride] = 0u;
}

void launch_counters_reset(unsigned* counters, hipStream_t st) {
  hipLaunchKernelGGL(k_counters_reset, dim3(1), dim3(64), 0, st, counters);
}

void launch_ctrl_reset(Ctrl* c, int full, unsigned seq_next, hipStream_t st) {
  hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, st, c, full, seq_next);
}

// The stopping test of the sweep before launch number seq, as that launch would take it
// (one workgroup of four wavefronts: the canonical order needs no particular size).
__global__ __launch_bounds__(256) void k_reduce_lagged(Ctrl* c, const double* __restrict__ partials, int stride,
                                                       int nb, double* hist, int hist_cap, double tol, int stop,
                                                       unsigned seq) {
  __shared__ double sq[kVirtLanes / 64][2];
  const CtrlHead ch = ctrl_head(c);
  const unsigned seg = c->seg_seq;
  canonical_sums<4, false>(partials + (size_t)((seq - 1u) & 1u) * stride, nb, sq);
  __syncthreads();
  if (threadIdx.x != 0 || ch.done) return;
  const int k = (int)(seq - seg);
  if (k < 2) return;
  double b;
  const double res = relative_increment(canonical_total(sq, b), b);
  record_test(c, hist, hist_cap, k - 1, res, tol, stop);
}

void launch_reduce_lagged(const DevProblem& dp, double tol, unsigned seq, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_lagged, dim3(1), dim3(256), 0, st, dp.ctrl, (const double*)dp.partials,
                     dp.partial_stride, dp.nb_sweep, dp.hist, dp.hist_cap, tol, tol >= 0.0 ? 1 : 0, seq);
}

__global__ void k_cast(const double* __restrict__ src, void* __restrict__ dst, size_t count, int to_bf16) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  if (to_bf16)
    ((uint16_t*)dst)[i] = f32_to_bf16((float)src[i]);
  else
    ((float*)dst)[i] = (float)src[i];
}

void launch_cast(const double* src, void* dst, size_t count, int to_bf16, hipStream_t st) {
  if (count == 0) return;
  hipLaunchKernelGGL(k_cast, dim3((unsigned)((count + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, src, dst, count,
                     to_bf16);
}

// Transport inflow-boundary inputs.  For every active axis whose upwind neighbour
// lies outside the (non-periodic) domain, the inflow-face inputs are the boundary
// data of that face; everything else is zero.
struct BcArgs {
  MeshDev mesh;
  int dim, na, nf, I;
  long long side_off[6];
};

__global__ void k_bc_inputs(BcArgs a, const double* __restrict__ bc, double* __restrict__ in_bc) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const MeshDev& m = a.mesh;
  if (e >= m.nel) return;
  const size_t nel = (size_t)m.nel;
  const Ijk ijk = coords(m, e);
  const int c[3] = {ijk.c0, ijk.c1, ijk.c2};
  for (int r = 0; r < a.I; ++r) in_bc[r * nel + e] = 0.0;
  for (int t = 0; t < a.na; ++t) {
    const int ax = m.ax[t];
    if (neighbour(m, e, ijk, ax, -m.dir[t]) >= 0) continue;
    const int side = 2 * ax + (m.dir[t] > 0 ? 0 : 1);
    long long fi = 0, stride = 1;
    for (int q = 0; q < a.dim; ++q)
      if (q != ax) {
        fi += c[q] * stride;
        stride *= m.n[q];
      }
    const double* src = bc + a.side_off[side] + fi * a.nf;
    for (int k = 0; k < a.nf; ++k) in_bc[(size_t)(t * a.nf + k) * nel + e] = src[k];
  }
}

void launch_bc_inputs(const DevProblem& dp, const double* bc, double* in_bc, hipStream_t st) {
  BcArgs a;
  a.mesh = dp.mesh;
  a.dim = dp.dim;
  a.na = dp.na;
  a.nf = dp.nf;
  a.I = dp.I;
  long long off = 0;
  for (int s = 0; s < 6; ++s) {
    a.side_off[s] = off;
    const int ax = s / 2;
    if (ax >= dp.dim || dp.mesh.periodic[ax]) continue;
    long long faces = 1;
    for (int q = 0; q < dp.dim; ++q)
      if (q != ax) faces *= dp.mesh.n[q];
    off += faces * dp.nf;
  }
  hipLaunchKernelGGL(k_bc_inputs, dim3(nblocks(dp.mesh.nel)), dim3(kBlock), 0, st, a, bc, in_bc);
}

}  // namespace ehdg
