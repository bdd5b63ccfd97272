// HIP kernels of the eHDG iteration for gfx950 (MI355X).
//
// One eHDG sweep (Algorithm 1: independent local solves with the previous traces,
// then new traces) is, in trace form, per element e
//     s_out[e] = g[e] + T in_e(s_in),
// where in_e gathers the element's own and its face neighbours' trace data and T is
// the condensed local operator shared by every element of a uniform mesh.  The
// sweep is HBM-bound, so the design is about bytes:
//   * state arrays are component-major (SoA): component k of element e at
//     [k * n_el + e], so a wavefront of 64 consecutive elements reads and writes
//     512 contiguous bytes per component, and the face neighbours (e +- 1,
//     e +- n0, e +- n0 n1) are contiguous runs too;
//   * T is addressed uniformly across the wavefront, so it is fetched with scalar
//     loads and used as an SGPR operand of the FMAs (no LDS traffic);
//   * workgroups are remapped so each of the 8 XCDs sweeps a contiguous slab of
//     elements and the neighbour re-reads hit its own L2;
//   * the FP64 relative-increment norms are reduced per wavefront, per block, and
//     then by the last block to finish, in a fixed order (deterministic), which
//     also raises a device-side "done" flag that makes later sweeps exit at once.
#include "kernels.h"

#include <cmath>

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

__device__ __forceinline__ void coords(const MeshDev& m, int e, int c[3]) {
  c[0] = e % m.n[0];
  const int r = e / m.n[0];
  c[1] = r % m.n[1];
  c[2] = r / m.n[1];
}

// neighbour of e one step along `axis` (wrapping on periodic axes), -1 outside
__device__ __forceinline__ int neighbour(const MeshDev& m, int e, const int c[3], int axis, int step) {
  int v = c[axis] + step;
  const int stride = axis == 0 ? 1 : (axis == 1 ? m.n[0] : m.n[0] * m.n[1]);
  if (v < 0 || v >= m.n[axis]) {
    if (!m.periodic[axis]) return -1;
    v = v < 0 ? v + m.n[axis] : v - m.n[axis];
  }
  return e + (v - c[axis]) * stride;
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);                                             // round to nearest even
  return (uint16_t)(u >> 16);
}

// loaders: component-major arrays, value type per precision
struct Ld64 {
  const double* p;
  __device__ __forceinline__ double operator()(size_t i) const { return p[i]; }
};
struct Ld32 {
  const float* p;
  __device__ __forceinline__ float operator()(size_t i) const { return p[i]; }
};
struct Ld16 {
  const uint16_t* p;
  __device__ __forceinline__ float operator()(size_t i) const { return bf16_to_f32(p[i]); }
};
// FP64 iterate plus a low-precision correction: s + delta
template <class LD>
struct LdSum {
  const double* s;
  LD d;
  __device__ __forceinline__ double operator()(size_t i) const { return s[i] + (double)d(i); }
};

template <typename T>
__device__ __forceinline__ T fmadd(T a, T b, T c) { return fma(a, b, c); }

// ---------------------------------------------------------------------------
// gathers: in_e(s) for each problem family
// ---------------------------------------------------------------------------
// Transport, NA active axes, P1 = p + 1.  State per element: the outflow-face
// values of each active axis.  Inputs: [inflow face of each active axis (the
// upwind neighbour's outflow values; 0 on an inflow boundary, whose data is folded
// into g) | own outflow values].  The upwind trace (eq. transportLocale) is the
// upwind element's value, so no arithmetic is needed in the gather.
template <int DIM, int NA, int P1>
struct TransportFam {
  static constexpr int NF = DIM == 2 ? P1 : P1 * P1;
  static constexpr int NP = DIM == 2 ? P1 * P1 : P1 * P1 * P1;
  static constexpr int S = NA * NF, I = 2 * NA * NF, N = NP;
  template <class LD, typename T>
  __device__ __forceinline__ static void gather(const MeshDev& m, int e, const LD& ld, T* in) {
    int c[3];
    coords(m, e, c);
    const size_t nel = (size_t)m.nel;
#pragma unroll
    for (int t = 0; t < NA; ++t) {
      const int nb = neighbour(m, e, c, m.ax[t], -m.dir[t]);
      const int src = nb >= 0 ? nb : e;
      const T keep = nb >= 0 ? T(1) : T(0);
#pragma unroll
      for (int k = 0; k < NF; ++k) {
        const size_t row = (size_t)(t * NF + k) * nel;
        in[(NA + t) * NF + k] = (T)ld(row + e);
        in[t * NF + k] = keep * (T)ld(row + src);
      }
    }
  }
};

// Shallow water, P1 = p + 1.  State per element side f: c_f = (phi + sqrt(Phi)
// vel.n_f) / 2 at the face nodes.  Input on face f: the trace
// phihat = c_own + c_neighbour (the trace formula below the local solver in
// Section 3); on a wall phihat = phi + sqrt(Phi) vel.n = 2 c_own.
template <int P1>
struct SweFam {
  static constexpr int NF = P1, NP = P1 * P1;
  static constexpr int S = 4 * NF, I = 4 * NF, N = 3 * NP;
  template <class LD, typename T>
  __device__ __forceinline__ static void gather(const MeshDev& m, int e, const LD& ld, T* in) {
    int c[3];
    coords(m, e, c);
    const size_t nel = (size_t)m.nel;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const int nb = neighbour(m, e, c, f >> 1, (f & 1) ? 1 : -1);
      const bool wall = nb < 0;
      const int src = wall ? e : nb;
      const int fs = wall ? f : (f ^ 1);
#pragma unroll
      for (int k = 0; k < NF; ++k) {
        const T own = (T)ld((size_t)(f * NF + k) * nel + e);
        const T oth = (T)ld((size_t)(fs * NF + k) * nel + src);
        in[f * NF + k] = own + oth;
      }
    }
  }
};

// ---------------------------------------------------------------------------
// residual reduction (FP64, deterministic)
// ---------------------------------------------------------------------------
struct ResidArgs {
  Ctrl* ctrl;
  double* partials;
  double* hist;
  int hist_cap;
  double tol;
  int stop;  // 1: set done on tol or non-finite; 0: record only
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ void finish_residual(double d2, double n2, const ResidArgs& ra) {
  __shared__ double sd[kBlock / 64][2];
  __shared__ int is_last;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  d2 = wave_sum(d2);
  n2 = wave_sum(n2);
  if (lane == 0) {
    sd[w][0] = d2;
    sd[w][1] = n2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int i = 0; i < kBlock / 64; ++i) {
      a += sd[i][0];
      b += sd[i][1];
    }
    __hip_atomic_store(&ra.partials[2 * blockIdx.x], a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&ra.partials[2 * blockIdx.x + 1], b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const unsigned prev = atomicAdd(&ra.ctrl->counter, 1u);
    is_last = (prev == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < (int)gridDim.x; i += kBlock) {
    a += __hip_atomic_load(&ra.partials[2 * i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    b += __hip_atomic_load(&ra.partials[2 * i + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  a = wave_sum(a);
  b = wave_sum(b);
  __syncthreads();
  if (lane == 0) {
    sd[w][0] = a;
    sd[w][1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = 0.0;
    b = 0.0;
    for (int i = 0; i < kBlock / 64; ++i) {
      a += sd[i][0];
      b += sd[i][1];
    }
    const double res = b > 0.0 ? sqrt(a / b) : sqrt(a);
    Ctrl* c = ra.ctrl;
    const int it = c->iters;
    ra.hist[it % ra.hist_cap] = res;
    c->iters = it + 1;
    c->last_res = res;
    if (!isfinite(res)) {
      c->status = 2;
      if (ra.stop) c->done = 1;
    } else if (ra.stop && res < ra.tol) {
      c->status = 1;
      c->done = 1;
    }
    c->counter = 0u;
  }
}

// ---------------------------------------------------------------------------
// the sweep
// ---------------------------------------------------------------------------
// out[r][e] = g[r][e] + sum_c T[r][c] in_e[c]   (r < S, c < I)
template <class F, typename T, class LD, bool RESID>
__global__ __launch_bounds__(kBlock) void k_sweep(MeshDev m, LD ld, const T* __restrict__ g,
                                                   const T* __restrict__ Tm, T* __restrict__ out,
                                                   ResidArgs ra) {
  if (ra.ctrl->done) return;
  const int e = remap_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  double d2 = 0.0, n2 = 0.0;
  if (e < m.nel) {
    T in[F::I];
    F::gather(m, e, ld, in);
    const size_t nel = (size_t)m.nel;
#pragma unroll 2
    for (int r = 0; r < F::S; ++r) {
      T acc = g[(size_t)r * nel + e];
#pragma unroll
      for (int c = 0; c < F::I; ++c) acc = fmadd(Tm[r * F::I + c], in[c], acc);
      out[(size_t)r * nel + e] = acc;
      if (RESID) {
        const double dd = (double)acc - (double)ld((size_t)r * nel + e);
        d2 += dd * dd;
        n2 += (double)acc * (double)acc;
      }
    }
  }
  if (RESID) finish_residual(d2, n2, ra);
}

// mixed precision outer step: s_out = s_in (+ lo_in); r = g + T in(s_out) - s_out (FP64);
// r_lo = r in the low precision; norms of r and of s_out + r.
template <class F, class LD, typename Lo>
__global__ __launch_bounds__(kBlock) void k_refine(MeshDev m, LD ld, const double* __restrict__ g,
                                                    const double* __restrict__ Tm, double* __restrict__ s_out,
                                                    Lo* __restrict__ r_lo, ResidArgs ra) {
  if (ra.ctrl->done) return;
  const int e = remap_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  double d2 = 0.0, n2 = 0.0;
  if (e < m.nel) {
    double in[F::I];
    F::gather(m, e, ld, in);
    const size_t nel = (size_t)m.nel;
#pragma unroll 2
    for (int r = 0; r < F::S; ++r) {
      double acc = g[(size_t)r * nel + e];
#pragma unroll
      for (int c = 0; c < F::I; ++c) acc = fma(Tm[r * F::I + c], in[c], acc);
      const double s1 = ld((size_t)r * nel + e);
      const double res = acc - s1;
      s_out[(size_t)r * nel + e] = s1;
      if constexpr (sizeof(Lo) == 4)
        r_lo[(size_t)r * nel + e] = (float)res;
      else
        r_lo[(size_t)r * nel + e] = f32_to_bf16((float)res);
      d2 += res * res;
      n2 += acc * acc;
    }
  }
  finish_residual(d2, n2, ra);
}

// element solution from the traces of the last sweep's input:
//   u_new = w_src + R in(s_prev) (+ P u for backward Euler);
//   backward Euler, next step: g = g_src + G u_new
template <class F, bool BE>
__global__ __launch_bounds__(kBlock) void k_volume(MeshDev m, const double* __restrict__ s_prev,
                                                    const double* __restrict__ R, const double* __restrict__ P,
                                                    const double* __restrict__ Gm,
                                                    const double* __restrict__ w_src,
                                                    const double* __restrict__ u_old, double* __restrict__ u_new,
                                                    const double* __restrict__ g_src, double* __restrict__ g_out,
                                                    int update_g) {
  const int e = remap_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (e >= m.nel) return;
  const size_t nel = (size_t)m.nel;
  double in[F::I];
  F::gather(m, e, Ld64{s_prev}, in);
  double uo[BE ? F::N : 1];
  double gacc[BE ? F::S : 1];
  if constexpr (BE) {
#pragma unroll
    for (int c = 0; c < F::N; ++c) uo[c] = u_old[(size_t)c * nel + e];
#pragma unroll
    for (int i = 0; i < F::S; ++i) gacc[i] = g_src ? g_src[(size_t)i * nel + e] : 0.0;
  }
  for (int r = 0; r < F::N; ++r) {
    double acc = w_src ? w_src[(size_t)r * nel + e] : 0.0;
#pragma unroll
    for (int c = 0; c < F::I; ++c) acc = fma(R[r * F::I + c], in[c], acc);
    if constexpr (BE) {
#pragma unroll
      for (int c = 0; c < F::N; ++c) acc = fma(P[r * F::N + c], uo[c], acc);
#pragma unroll
      for (int i = 0; i < F::S; ++i) gacc[i] = fma(Gm[i * F::N + r], acc, gacc[i]);
    }
    u_new[(size_t)r * nel + e] = acc;
  }
  if constexpr (BE) {
    if (update_g) {
#pragma unroll
      for (int i = 0; i < F::S; ++i) g_out[(size_t)i * nel + e] = gacc[i];
    }
  }
}

// ---------------------------------------------------------------------------
// host launchers of one family
// ---------------------------------------------------------------------------
static inline int nblocks(int nel) { return (nel + kBlock - 1) / kBlock; }

static inline ResidArgs resid_args(const DevProblem& dp, double tol, int stop) {
  ResidArgs ra;
  ra.ctrl = dp.ctrl;
  ra.partials = dp.partials;
  ra.hist = dp.hist;
  ra.hist_cap = dp.hist_cap;
  ra.tol = tol;
  ra.stop = stop;
  return ra;
}

template <class F>
struct Family {
  static void sweep64(const DevProblem& dp, int k, bool resid, double tol, hipStream_t st) {
    const ResidArgs ra = resid_args(dp, tol, tol >= 0.0 ? 1 : 0);
    const Ld64 ld{dp.s[k & 1]};
    if (resid)
      hipLaunchKernelGGL((k_sweep<F, double, Ld64, true>), dim3(nblocks(dp.mesh.nel)), dim3(kBlock), 0, st, dp.mesh,
                         ld, (const double*)dp.g, dp.T64, dp.s[(k + 1) & 1], ra);
    else
      hipLaunchKernelGGL((k_sweep<F, double, Ld64, false>), dim3(nblocks(dp.mesh.nel)), dim3(kBlock), 0, st,
                         dp.mesh, ld, (const double*)dp.g, dp.T64, dp.s[(k + 1) & 1], ra);
  }
  static void volume(const DevProblem& dp, const double* s_prev, bool update_g, hipStream_t st) {
    if (dp.be)
      hipLaunchKernelGGL((k_volume<F, true>), dim3(nblocks(dp.mesh.nel)), dim3(kBlock), 0, st, dp.mesh, s_prev, dp.R,
                         dp.P, dp.G, (const double*)dp.w_src, (const double*)dp.u, dp.u_new,
                         (const double*)dp.g_src, dp.g, update_g ? 1 : 0);
    else
      hipLaunchKernelGGL((k_volume<F, false>), dim3(nblocks(dp.mesh.nel)), dim3(kBlock), 0, st, dp.mesh, s_prev,
                         dp.R, dp.P, dp.G, (const double*)dp.w_src, (const double*)dp.u, dp.u_new,
                         (const double*)dp.g_src, dp.g, 0);
  }
  static void refine32(const DevProblem& dp, const double* s_in, const void* lo_in, double* s_out, void* r_out,
                       double tol, hipStream_t st) {
    const ResidArgs ra = resid_args(dp, tol, 1);
    if (lo_in) {
      const LdSum<Ld32> ld{s_in, Ld32{(const float*)lo_in}};
      hipLaunchKernelGGL((k_refine<F, LdSum<Ld32>, float>), dim3(nblocks(dp.mesh.nel)), dim3(kBlock), 0, st, dp.mesh,
                         ld, (const double*)dp.g, dp.T64, s_out, (float*)r_out, ra);
    } else {
      hipLaunchKernelGGL((k_refine<F, Ld64, float>), dim3(nblocks(dp.mesh.nel)), dim3(kBlock), 0, st, dp.mesh,
                         Ld64{s_in}, (const double*)dp.g, dp.T64, s_out, (float*)r_out, ra);
    }
  }
  static void inner32(const DevProblem& dp, const void* r_lo, const void* lo_in, void* lo_out, hipStream_t st) {
    const ResidArgs ra = resid_args(dp, -1.0, 0);
    hipLaunchKernelGGL((k_sweep<F, float, Ld32, false>), dim3(nblocks(dp.mesh.nel)), dim3(kBlock), 0, st, dp.mesh,
                       Ld32{(const float*)lo_in}, (const float*)r_lo, dp.T32, (float*)lo_out, ra);
  }
};

// ---------------------------------------------------------------------------
// registry
// ---------------------------------------------------------------------------
template <class F>
static const KernelSet* set_of() {
  static const KernelSet ks = {&Family<F>::sweep64, &Family<F>::volume, &Family<F>::refine32,
                               &Family<F>::inner32, nullptr, nullptr};
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

void launch_matvec(const double* M, int rows, int cols, const double* x, double* y, int nel, bool accumulate,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_matvec, dim3(nblocks(nel)), dim3(kBlock), 0, st, M, rows, cols, x, y, nel,
                     accumulate ? 1 : 0);
}

__global__ void k_transpose(const double* __restrict__ src, double* __restrict__ dst, int K, int nel, int to_soa) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)K * nel;
  if (i >= total) return;
  // i indexes the destination
  if (to_soa) {
    const size_t k = i / nel, e = i % nel;
    dst[i] = src[e * K + k];
  } else {
    const size_t e = i / K, k = i % K;
    dst[i] = src[k * nel + e];
  }
}

void launch_ext_to_soa(const double* ext, double* soa, int K, int nel, hipStream_t st) {
  const size_t total = (size_t)K * nel;
  hipLaunchKernelGGL(k_transpose, dim3((unsigned)((total + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, ext, soa,
                     K, nel, 1);
}

void launch_soa_to_ext(const double* soa, double* ext, int K, int nel, hipStream_t st) {
  const size_t total = (size_t)K * nel;
  hipLaunchKernelGGL(k_transpose, dim3((unsigned)((total + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, soa, ext,
                     K, nel, 0);
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

__global__ void k_ctrl_reset(Ctrl* c) {
  if (threadIdx.x == 0) {
    c->done = 0;
    c->iters = 0;
    c->status = 0;
    c->counter = 0u;
    c->last_res = 0.0;
  }
}

void launch_ctrl_reset(Ctrl* c, hipStream_t st) { hipLaunchKernelGGL(k_ctrl_reset, dim3(1), dim3(64), 0, st, c); }

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
  int c[3];
  coords(m, e, c);
  for (int r = 0; r < a.I; ++r) in_bc[r * nel + e] = 0.0;
  for (int t = 0; t < a.na; ++t) {
    const int ax = m.ax[t];
    if (neighbour(m, e, c, ax, -m.dir[t]) >= 0) continue;
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
