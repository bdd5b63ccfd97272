// Host-side (FP64) construction of the eHDG element operators; see setup.h.
//
// The discretization (tensor Lagrange elements on GLL nodes, Gauss quadrature with
// p+2 points per direction) is assembled from 1D factors: on an axis-aligned box
// every volume and face integral of products of basis functions factors into 1D
// mass matrices M1 and 1D convection matrices K1, scaled by the half-widths h/2.
#include "setup.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <thread>

namespace ehdg {

namespace {

// Legendre P_n and P_n' at x by the three-term recurrence (derivative recurrence
// P_k' = P_{k-2}' + (2k-1) P_{k-1}).
void legendre(int n, double x, double& P, double& dP) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (n == 0) { P = 1.0; dP = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    double d2 = d0 + (2.0 * k - 1.0) * p1;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  P = p1; dP = d1;
}

// Barycentric weights of the Lagrange basis on nodes x.
std::vector<double> bary_weights(const std::vector<double>& x) {
  size_t n = x.size();
  std::vector<double> lam(n, 1.0);
  for (size_t j = 0; j < n; ++j)
    for (size_t k = 0; k < n; ++k)
      if (k != j) lam[j] /= (x[j] - x[k]);
  return lam;
}

// l_j(t) for all j (barycentric form), exact at the nodes.
void lagrange_at(const std::vector<double>& x, const std::vector<double>& lam, double t, double* out) {
  size_t n = x.size();
  for (size_t j = 0; j < n; ++j)
    if (t == x[j]) {
      for (size_t k = 0; k < n; ++k) out[k] = (k == j) ? 1.0 : 0.0;
      return;
    }
  double den = 0.0;
  for (size_t j = 0; j < n; ++j) {
    out[j] = lam[j] / (t - x[j]);
    den += out[j];
  }
  for (size_t j = 0; j < n; ++j) out[j] /= den;
}

}  // namespace

Basis1D make_basis(int p) {
  Basis1D b;
  b.p = p;
  const int n = p + 1;
  // GLL nodes: +-1 and the roots of P_p' (Newton on P_p' with P_p'' from the
  // Legendre equation (1-x^2) P'' = 2x P' - p(p+1) P).
  b.x.assign(n, 0.0);
  b.w.assign(n, 0.0);
  b.x[0] = -1.0;
  b.x[p] = 1.0;
  for (int i = 1; i < p; ++i) {
    double x = -std::cos(M_PI * i / p);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(p, x, P, dP);
      double d2P = (2.0 * x * dP - p * (p + 1.0) * P) / (1.0 - x * x);
      double step = dP / d2P;
      x -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    b.x[i] = x;
  }
  for (int i = 0; i < n; ++i) {
    double P, dP;
    legendre(p, b.x[i], P, dP);
    b.w[i] = 2.0 / (p * (p + 1.0) * P * P);
  }
  // Gauss points: roots of P_nq by Newton from the Chebyshev guess.
  const int nq = p + 2;
  b.nq = nq;
  b.xq.assign(nq, 0.0);
  b.wq.assign(nq, 0.0);
  for (int i = 0; i < nq; ++i) {
    double x = -std::cos(M_PI * (i + 0.75) / (nq + 0.5));
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(nq, x, P, dP);
      double step = P / dP;
      x -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    double P, dP;
    legendre(nq, x, P, dP);
    b.xq[i] = x;
    b.wq[i] = 2.0 / ((1.0 - x * x) * dP * dP);
  }
  // basis and derivatives at the Gauss points; derivative via the nodal
  // differentiation matrix D_ij = l_j'(x_i) (exact: l_j' has degree p-1)
  std::vector<double> lam = bary_weights(b.x);
  std::vector<double> D((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    double diag = 0.0;
    for (int j = 0; j < n; ++j)
      if (j != i) {
        D[(size_t)i * n + j] = (lam[j] / lam[i]) / (b.x[i] - b.x[j]);
        diag -= D[(size_t)i * n + j];
      }
    D[(size_t)i * n + i] = diag;
  }
  b.B.assign((size_t)nq * n, 0.0);
  b.dB.assign((size_t)nq * n, 0.0);
  std::vector<double>& dB = b.dB;
  for (int q = 0; q < nq; ++q) {
    lagrange_at(b.x, lam, b.xq[q], &b.B[(size_t)q * n]);
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int i = 0; i < n; ++i) s += b.B[(size_t)q * n + i] * D[(size_t)i * n + j];
      dB[(size_t)q * n + j] = s;
    }
  }
  b.M1.assign((size_t)n * n, 0.0);
  b.K1.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double m = 0.0, k = 0.0;
      for (int q = 0; q < nq; ++q) {
        m += b.wq[q] * b.B[(size_t)q * n + i] * b.B[(size_t)q * n + j];
        k += b.wq[q] * b.B[(size_t)q * n + j] * dB[(size_t)q * n + i];
      }
      b.M1[(size_t)i * n + j] = m;
      b.K1[(size_t)i * n + j] = k;
    }
  return b;
}

Mat matmul(const Mat& A, const Mat& B) {
  Mat C(A.r, B.c);
  for (int i = 0; i < A.r; ++i)
    for (int k = 0; k < A.c; ++k) {
      double a = A(i, k);
      if (a == 0.0) continue;
      for (int j = 0; j < B.c; ++j) C(i, j) += a * B(k, j);
    }
  return C;
}

bool invert(const Mat& A, Mat& Ainv) {
  const int n = A.r;
  Mat LU = A;
  std::vector<int> piv(n);
  for (int k = 0; k < n; ++k) {
    int pr = k;
    double best = std::fabs(LU(k, k));
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(LU(i, k)) > best) { best = std::fabs(LU(i, k)); pr = i; }
    if (best == 0.0) return false;
    piv[k] = pr;
    if (pr != k)
      for (int j = 0; j < n; ++j) std::swap(LU(k, j), LU(pr, j));
    for (int i = k + 1; i < n; ++i) {
      double l = LU(i, k) / LU(k, k);
      LU(i, k) = l;
      for (int j = k + 1; j < n; ++j) LU(i, j) -= l * LU(k, j);
    }
  }
  Ainv = Mat(n, n);
  std::vector<double> col(n);
  for (int c = 0; c < n; ++c) {
    for (int i = 0; i < n; ++i) col[i] = (i == c) ? 1.0 : 0.0;
    for (int k = 0; k < n; ++k) std::swap(col[k], col[piv[k]]);
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < i; ++k) col[i] -= LU(i, k) * col[k];
    for (int i = n - 1; i >= 0; --i) {
      for (int k = i + 1; k < n; ++k) col[i] -= LU(i, k) * col[k];
      col[i] /= LU(i, i);
    }
    for (int i = 0; i < n; ++i) Ainv(i, c) = col[i];
  }
  return true;
}

namespace {

// sign(A) by the Newton iteration X <- (X + X^{-1}) / 2 from X = A (converges for
// any A without eigenvalues on the imaginary axis); |A| = sign(A) A.
bool matrix_sign(const Mat& A, Mat& S) {
  S = A;
  Mat Xi;
  for (int it = 0; it < 100; ++it) {
    if (!invert(S, Xi)) return false;
    double diff = 0.0, nrm = 0.0;
    for (size_t k = 0; k < S.a.size(); ++k) {
      const double nx = 0.5 * (S.a[k] + Xi.a[k]);
      diff = std::max(diff, std::fabs(nx - S.a[k]));
      nrm = std::max(nrm, std::fabs(nx));
      S.a[k] = nx;
    }
    if (diff <= 1e-15 * nrm) return true;
  }
  return true;
}

// Element-level tensor operators on a box with half-widths hh[d].
struct ElementOps {
  int d, p, n1, Np, nf;
  std::vector<std::vector<int>> nodeidx;  // Np x d
  std::vector<std::vector<int>> fn;       // 2d x nf: volume node of each face node
  Mat M;                                  // Np x Np
  Mat K[3];                               // K[a](i,j) = (psi_j, d psi_i / dx_a)
  Mat Lf[6];                              // Np x nf: <mu_c, psi_i>_f
  Mat E[6];                               // Np x Np: <psi_j, psi_i>_f
};

ElementOps element_ops(const Basis1D& b, int d, const double* hh) {
  ElementOps E;
  E.d = d;
  E.p = b.p;
  E.n1 = b.p + 1;
  const int n1 = E.n1;
  E.Np = 1;
  for (int a = 0; a < d; ++a) E.Np *= n1;
  E.nf = E.Np / n1;
  E.nodeidx.assign(E.Np, std::vector<int>(3, 0));
  for (int i = 0; i < E.Np; ++i) {
    int r = i;
    for (int a = 0; a < d; ++a) { E.nodeidx[i][a] = r % n1; r /= n1; }
  }
  auto M1 = [&](int i, int j) { return b.M1[(size_t)i * n1 + j]; };
  auto K1 = [&](int i, int j) { return b.K1[(size_t)i * n1 + j]; };
  E.M = Mat(E.Np, E.Np);
  for (int a = 0; a < d; ++a) E.K[a] = Mat(E.Np, E.Np);
  for (int i = 0; i < E.Np; ++i)
    for (int j = 0; j < E.Np; ++j) {
      double m = 1.0;
      for (int t = 0; t < d; ++t) m *= hh[t] * M1(E.nodeidx[i][t], E.nodeidx[j][t]);
      E.M(i, j) = m;
      for (int a = 0; a < d; ++a) {
        // (psi_j, d psi_i / dx_a): the 2/h of the derivative cancels the h/2 of axis a
        double k = K1(E.nodeidx[i][a], E.nodeidx[j][a]);
        for (int t = 0; t < d; ++t)
          if (t != a) k *= hh[t] * M1(E.nodeidx[i][t], E.nodeidx[j][t]);
        E.K[a](i, j) = k;
      }
    }
  E.fn.assign(2 * d, std::vector<int>(E.nf, 0));
  for (int f = 0; f < 2 * d; ++f) {
    const int ax = f / 2, end = (f % 2) ? b.p : 0;
    int tang[2] = {0, 0}, nt = 0;
    for (int t = 0; t < d; ++t)
      if (t != ax) tang[nt++] = t;
    // face node c <-> tangential multi-index (c0, c1), first tangential axis fastest
    for (int c = 0; c < E.nf; ++c) {
      int ct[2] = {c % n1, (c / n1) % n1};
      int idx[3] = {0, 0, 0};
      idx[ax] = end;
      for (int t = 0; t < nt; ++t) idx[tang[t]] = ct[t];
      int node = 0, stride = 1;
      for (int t = 0; t < d; ++t) { node += idx[t] * stride; stride *= n1; }
      E.fn[f][c] = node;
    }
    E.Lf[f] = Mat(E.Np, E.nf);
    for (int i = 0; i < E.Np; ++i) {
      if (E.nodeidx[i][ax] != end) continue;
      for (int c = 0; c < E.nf; ++c) {
        int ct[2] = {c % n1, (c / n1) % n1};
        double v = 1.0;
        for (int t = 0; t < nt; ++t) v *= hh[tang[t]] * M1(E.nodeidx[i][tang[t]], ct[t]);
        E.Lf[f](i, c) = v;
      }
    }
    // E_f(i, j) = sum_c Lf(i, c) psi_j(face node c) = Lf(i, c_j) for face nodes j
    E.E[f] = Mat(E.Np, E.Np);
    for (int i = 0; i < E.Np; ++i)
      for (int c = 0; c < E.nf; ++c) E.E[f](i, E.fn[f][c]) = E.Lf[f](i, c);
  }
  return E;
}

}  // namespace

std::string build_operators(const Desc& d, Operators& ops) {
  char msg[256];
  if (d.dim != 2 && d.dim != 3) return "dim must be 2 or 3";
  for (int a = 0; a < d.dim; ++a) {
    if (d.n[a] < 1) return "n[a] must be >= 1";
    if (!(d.L[a] > 0.0)) return "L[a] must be > 0";
  }
  const int p = d.degree;
  ops.dim = d.dim;
  ops.p = p;
  double hh[3] = {1, 1, 1};
  for (int a = 0; a < d.dim; ++a) hh[a] = 0.5 * d.L[a] / d.n[a];
  if (d.pde == 0) {
    ops.pde = Pde::Transport;
    int pmax = (d.dim == 2) ? 6 : 4;
    if (p < 1 || p > pmax) {
      snprintf(msg, sizeof msg, "transport %dD supports degree 1..%d (got %d)", d.dim, pmax, p);
      return msg;
    }
    if (d.sigma < 0.0 || d.dt < 0.0) return "sigma and dt must be >= 0";
    if (!std::isfinite(d.sigma) || !std::isfinite(d.dt)) return "sigma and dt must be finite";
  } else if (d.pde == 1) {
    ops.pde = Pde::Swe;
    if (d.dim != 2) return "shallow water is 2D";
    if (p < 1 || p > 6) return "shallow water supports degree 1..6";
    if (!(d.Phi > 0.0) || !std::isfinite(d.Phi)) return "Phi must be > 0";
    if (!(d.dt > 0.0) || !std::isfinite(d.dt)) return "shallow water needs dt > 0";
  } else if (d.pde == 2) {
    ops.pde = Pde::Euler;
    if (d.dim != 2) return "linearized Euler is 2D";
    if (p < 1 || p > 5) return "linearized Euler supports degree 1..5";
    if (!(d.dt > 0.0) || !std::isfinite(d.dt)) return "linearized Euler needs dt > 0";
    if (!(d.c0 > 0.0) || !(d.rho0 > 0.0)) return "c0 and rho0 must be > 0";
    for (int a = 0; a < 2; ++a)
      if (d.U0[a] == 0.0 || std::fabs(d.U0[a]) == d.c0 || !std::isfinite(d.U0[a]))
        return "a face normal sees a zero wave speed (U0_a = 0 or |U0_a| = c0)";
  } else {
    return "unknown pde";
  }
  Basis1D b = make_basis(p);
  ElementOps E = element_ops(b, d.dim, hh);
  const int Np = E.Np, nf = E.nf;
  ops.Np = Np;
  ops.nf = nf;
  ops.be = d.dt > 0.0;
  ops.nq_el = 1;
  for (int a = 0; a < d.dim; ++a) ops.nq_el *= b.nq;
  Mat A, L, Mbt;
  if (ops.pde == Pde::Transport) {
    ops.m = 1;
    ops.n = Np;
    ops.na = 0;
    for (int a = 0; a < d.dim; ++a)
      if (d.beta[a] != 0.0) {
        if (!std::isfinite(d.beta[a])) return "beta must be finite";
        ops.ax[ops.na] = a;
        ops.dir[ops.na] = d.beta[a] > 0.0 ? 1 : -1;
        ops.na++;
      }
    if (ops.na == 0) return "beta = 0: no transport";
    ops.S = ops.na * nf;
    ops.I = 2 * ops.na * nf;
    const double react = d.sigma + (ops.be ? 1.0 / d.dt : 0.0);
    A = Mat(Np, Np);
    for (int i = 0; i < Np; ++i)
      for (int j = 0; j < Np; ++j) {
        double v = react * E.M(i, j);
        for (int a = 0; a < d.dim; ++a) v -= d.beta[a] * E.K[a](i, j);
        A(i, j) = v;
      }
    for (int f = 0; f < 2 * d.dim; ++f) {
      double bn = (f % 2 ? 1.0 : -1.0) * d.beta[f / 2];
      double wgt = bn + std::fabs(bn);
      if (wgt == 0.0) continue;
      for (int i = 0; i < Np; ++i)
        for (int j = 0; j < Np; ++j) A(i, j) += wgt * E.E[f](i, j);
    }
    // gathered inputs: [inflow face of each active axis | own outflow face of each]
    L = Mat(Np, ops.I);
    ops.Q = Mat(ops.S, Np);
    for (int t = 0; t < ops.na; ++t) {
      const int a = ops.ax[t];
      const int f_in = 2 * a + (ops.dir[t] > 0 ? 0 : 1), f_out = f_in ^ 1;
      const double w = std::fabs(d.beta[a]);
      for (int i = 0; i < Np; ++i)
        for (int c = 0; c < nf; ++c) {
          L(i, t * nf + c) = w * E.Lf[f_in](i, c);
          L(i, (ops.na + t) * nf + c) = w * E.Lf[f_out](i, c);
        }
      for (int c = 0; c < nf; ++c) ops.Q(t * nf + c, E.fn[f_out][c]) = 1.0;
    }
    if (ops.be) {
      Mbt = Mat(Np, Np);
      for (size_t k = 0; k < Mbt.a.size(); ++k) Mbt.a[k] = E.M.a[k] / d.dt;
    }
  } else if (ops.pde == Pde::Swe) {
    ops.m = 3;
    const int n = 3 * Np;
    ops.n = n;
    ops.S = 4 * nf;
    ops.I = 4 * nf;
    const double Phi = d.Phi, sq = std::sqrt(d.Phi), idt = 1.0 / d.dt;
    A = Mat(n, n);
    auto blk = [&](int bi, int bj, int i, int j) -> double& { return A(bi * Np + i, bj * Np + j); };
    for (int i = 0; i < Np; ++i)
      for (int j = 0; j < Np; ++j) {
        blk(0, 0, i, j) = idt * E.M(i, j);
        blk(0, 1, i, j) = -Phi * E.K[0](i, j);
        blk(0, 2, i, j) = -Phi * E.K[1](i, j);
        blk(1, 0, i, j) = -Phi * E.K[0](i, j);
        blk(1, 1, i, j) = Phi * idt * E.M(i, j);
        blk(2, 0, i, j) = -Phi * E.K[1](i, j);
        blk(2, 2, i, j) = Phi * idt * E.M(i, j);
      }
    L = Mat(n, ops.I);
    ops.Q = Mat(ops.S, n);
    for (int f = 0; f < 4; ++f) {
      const double n1 = (f / 2 == 0) ? (f % 2 ? 1.0 : -1.0) : 0.0;
      const double n2 = (f / 2 == 1) ? (f % 2 ? 1.0 : -1.0) : 0.0;
      for (int i = 0; i < Np; ++i)
        for (int j = 0; j < Np; ++j) {
          double e = E.E[f](i, j);
          if (e == 0.0) continue;
          blk(0, 0, i, j) += sq * e;
          blk(0, 1, i, j) += Phi * n1 * e;
          blk(0, 2, i, j) += Phi * n2 * e;
        }
      for (int i = 0; i < Np; ++i)
        for (int c = 0; c < nf; ++c) {
          double l = E.Lf[f](i, c);
          L(i, f * nf + c) = sq * l;
          L(Np + i, f * nf + c) = -Phi * n1 * l;
          L(2 * Np + i, f * nf + c) = -Phi * n2 * l;
        }
      for (int c = 0; c < nf; ++c) {
        const int node = E.fn[f][c];
        ops.Q(f * nf + c, node) = 0.5;
        ops.Q(f * nf + c, Np + node) = 0.5 * sq * n1;
        ops.Q(f * nf + c, 2 * Np + node) = 0.5 * sq * n2;
      }
    }
    Mbt = Mat(n, n);
    for (int i = 0; i < Np; ++i)
      for (int j = 0; j < Np; ++j) {
        Mbt(i, j) = idt * E.M(i, j);
        Mbt(Np + i, Np + j) = Phi * idt * E.M(i, j);
        Mbt(2 * Np + i, 2 * Np + j) = Phi * idt * E.M(i, j);
      }
  }
  if (ops.pde == Pde::Euler) {
    // w = (rho', u', v', p'); flux A_x w, A_y w; upwind HDG with |A_n| (see ehdg.h)
    const int n = 4 * Np;
    ops.m = 4;
    ops.n = n;
    ops.S = 16 * nf;
    ops.I = 16 * nf;
    const double U = d.U0[0], V = d.U0[1], r0 = d.rho0, k0 = d.rho0 * d.c0 * d.c0, idt = 1.0 / d.dt;
    Mat Ax(4, 4), Ay(4, 4);
    const double ax[16] = {U, r0, 0, 0, 0, U, 0, 1 / r0, 0, 0, U, 0, 0, k0, 0, U};
    const double ay[16] = {V, 0, r0, 0, 0, V, 0, 0, 0, 0, V, 1 / r0, 0, 0, k0, V};
    std::copy(ax, ax + 16, Ax.a.begin());
    std::copy(ay, ay + 16, Ay.a.begin());
    A = Mat(n, n);
    for (int fa = 0; fa < 4; ++fa)
      for (int fb = 0; fb < 4; ++fb)
        for (int i = 0; i < Np; ++i)
          for (int j = 0; j < Np; ++j)
            A(fa * Np + i, fb * Np + j) =
                (fa == fb ? idt * E.M(i, j) : 0.0) - Ax(fa, fb) * E.K[0](i, j) - Ay(fa, fb) * E.K[1](i, j);
    L = Mat(n, ops.I);
    ops.Q = Mat(ops.S, n);
    for (int f = 0; f < 4; ++f) {
      const double n1 = (f / 2 == 0) ? (f % 2 ? 1.0 : -1.0) : 0.0;
      const double n2 = (f / 2 == 1) ? (f % 2 ? 1.0 : -1.0) : 0.0;
      Mat An(4, 4), Sg, Ab;
      for (int k = 0; k < 16; ++k) An.a[k] = n1 * Ax.a[k] + n2 * Ay.a[k];
      if (!matrix_sign(An, Sg)) return "a face normal sees a zero wave speed";
      Ab = matmul(Sg, An);
      for (int fa = 0; fa < 4; ++fa)
        for (int fb = 0; fb < 4; ++fb) {
          const double w = An(fa, fb) + Ab(fa, fb);
          for (int i = 0; i < Np; ++i)
            for (int j = 0; j < Np; ++j) {
              const double e = E.E[f](i, j);
              if (e != 0.0) A(fa * Np + i, fb * Np + j) += w * e;
            }
          for (int i = 0; i < Np; ++i)
            for (int c = 0; c < nf; ++c) L(fa * Np + i, (f * 4 + fb) * nf + c) = Ab(fa, fb) * E.Lf[f](i, c);
          // outgoing part of the own state on this side: (I + S) / 2 w at the face nodes
          const double q = 0.5 * ((fa == fb ? 1.0 : 0.0) + Sg(fa, fb));
          for (int c = 0; c < nf; ++c) ops.Q((f * 4 + fa) * nf + c, fb * Np + E.fn[f][c]) = q;
        }
    }
    Mbt = Mat(n, n);
    for (int fa = 0; fa < 4; ++fa)
      for (int i = 0; i < Np; ++i)
        for (int j = 0; j < Np; ++j) Mbt(fa * Np + i, fa * Np + j) = idt * E.M(i, j);
  }
  if (!invert(A, ops.W)) return "local operator is singular";
  ops.R = matmul(ops.W, L);
  ops.T = matmul(ops.Q, ops.R);
  if (ops.be) {
    ops.P = matmul(ops.W, Mbt);
    ops.G = matmul(ops.Q, ops.P);
    const Mat GP = matmul(ops.G, ops.P), GR = matmul(ops.G, ops.R);
    const int n = ops.n;
    ops.Mvol = Mat(n + ops.S, n + ops.I);
    for (int i = 0; i < n; ++i) {
      for (int j = 0; j < n; ++j) ops.Mvol(i, j) = ops.P(i, j);
      for (int j = 0; j < ops.I; ++j) ops.Mvol(i, n + j) = ops.R(i, j);
    }
    for (int i = 0; i < ops.S; ++i) {
      for (int j = 0; j < n; ++j) ops.Mvol(n + i, j) = GP(i, j);
      for (int j = 0; j < ops.I; ++j) ops.Mvol(n + i, n + j) = GR(i, j);
    }
  } else {
    ops.Mvol = ops.R;
  }
  // load matrix: F_i = (f, psi_i) = sum_q J w_q psi_i(x_q) f(x_q)
  const int nq = b.nq, n1 = p + 1;
  double J = 1.0;
  for (int a = 0; a < d.dim; ++a) J *= hh[a];
  ops.Bload = Mat(Np, ops.nq_el);
  for (int i = 0; i < Np; ++i)
    for (int q = 0; q < ops.nq_el; ++q) {
      int r = q;
      double v = J;
      for (int a = 0; a < d.dim; ++a) {
        int qa = r % nq;
        r /= nq;
        v *= b.wq[qa] * b.B[(size_t)qa * n1 + E.nodeidx[i][a]];
      }
      ops.Bload(i, q) = v;
    }
  return "";
}


std::string build_variable_operators(const Desc& d, const VarSamples* smp, Operators& ops, VarOperators* vo) {
  if (d.pde != 0) return "a velocity field applies to transport";
  if (d.dt != 0.0) return "variable-velocity transport is steady (dt = 0)";
  if (d.dim != 2 && d.dim != 3) return "dim must be 2 or 3";
  const int dim = d.dim, p = d.degree;
  if (p < 1 || p > (dim == 2 ? 6 : 4)) return "degree out of range for transport";
  long long nel = 1;
  for (int a = 0; a < dim; ++a) {
    if (d.n[a] < 1) return "n[a] must be >= 1";
    nel *= d.n[a];
  }
  const int n1 = p + 1, nq = p + 2;
  int nqf = 1, Nq = 1;
  for (int a = 0; a < dim; ++a) Nq *= nq;
  for (int a = 1; a < dim; ++a) nqf *= nq;
  // upwind direction of each axis from the signs of beta_a on the faces normal to it
  Desc dc = d;
  for (int a = 0; a < 3; ++a) dc.beta[a] = a < dim ? 1.0 : 0.0;
  if (smp) {
    if (!smp->beta_q || !smp->beta_face) return "velocity samples missing";
    for (int a = 0; a < dim; ++a) {
      bool pos = false, neg = false, zero = false;
      for (long long e = 0; e < nel; ++e)
        for (int side = 0; side < 2; ++side) {
          const double* v = smp->beta_face + ((size_t)e * 2 * dim + 2 * a + side) * nqf;
          for (int q = 0; q < nqf; ++q) {
            if (!std::isfinite(v[q])) return "velocity samples must be finite";
            pos |= v[q] > 0.0;
            neg |= v[q] < 0.0;
            zero |= v[q] == 0.0;
          }
        }
      if ((pos && neg) || (zero && (pos || neg)))
        return "a velocity component changes sign or vanishes on the faces normal to its axis";
      dc.beta[a] = pos ? 1.0 : (neg ? -1.0 : 0.0);
    }
    const size_t nvq = (size_t)nel * dim * Nq;
    for (size_t k = 0; k < nvq; ++k)
      if (!std::isfinite(smp->beta_q[k])) return "velocity samples must be finite";
    if (smp->div_q)
      for (size_t k = 0; k < (size_t)nel * Nq; ++k)
        if (!std::isfinite(smp->div_q[k])) return "velocity samples must be finite";
  }
  // shape, Q and the load matrix are those of a constant velocity with the same signs
  std::string err = build_operators(dc, ops);
  if (!err.empty()) return err;
  if (!vo) return "";

  const Basis1D b = make_basis(p);
  double hh[3] = {1, 1, 1};
  for (int a = 0; a < dim; ++a) hh[a] = 0.5 * d.L[a] / d.n[a];
  const ElementOps E = element_ops(b, dim, hh);
  const int Np = E.Np, nf = E.nf, S = ops.S, I = ops.I, na = ops.na;
  double J = 1.0;
  for (int a = 0; a < dim; ++a) J *= hh[a];
  // reference tables at the tensor Gauss points (axis 0 fastest): psi_i, d psi_i / d xi_a, weights
  std::vector<double> Psi((size_t)Nq * Np), G((size_t)dim * Nq * Np), wvol(Nq);
  for (int q = 0; q < Nq; ++q) {
    int qa[3] = {0, 0, 0}, r = q;
    for (int a = 0; a < dim; ++a) { qa[a] = r % nq; r /= nq; }
    double w = J;
    for (int a = 0; a < dim; ++a) w *= b.wq[qa[a]];
    wvol[q] = w;
    for (int i = 0; i < Np; ++i) {
      double v = 1.0;
      for (int a = 0; a < dim; ++a) v *= b.B[(size_t)qa[a] * n1 + E.nodeidx[i][a]];
      Psi[(size_t)q * Np + i] = v;
      for (int a = 0; a < dim; ++a) {
        double g = b.dB[(size_t)qa[a] * n1 + E.nodeidx[i][a]];
        for (int t = 0; t < dim; ++t)
          if (t != a) g *= b.B[(size_t)qa[t] * n1 + E.nodeidx[i][t]];
        G[((size_t)a * Nq + q) * Np + i] = g;
      }
    }
  }
  // face tables: trace basis mu_c at the face Gauss points (first tangential axis
  // fastest, as the face nodes) and the face weights with the face Jacobian
  std::vector<double> mu((size_t)nqf * nf), wfc((size_t)2 * dim * nqf);
  for (int qf = 0; qf < nqf; ++qf)
    for (int c = 0; c < nf; ++c) {
      int rq = qf, rc = c;
      double v = 1.0;
      for (int t = 0; t < dim - 1; ++t) {
        v *= b.B[(size_t)(rq % nq) * n1 + rc % n1];
        rq /= nq;
        rc /= n1;
      }
      mu[(size_t)qf * nf + c] = v;
    }
  for (int f = 0; f < 2 * dim; ++f) {
    int tang[2] = {0, 0}, nt = 0;
    for (int t = 0; t < dim; ++t)
      if (t != f / 2) tang[nt++] = t;
    for (int qf = 0; qf < nqf; ++qf) {
      int rq = qf;
      double w = 1.0;
      for (int t = 0; t < nt; ++t) {
        w *= b.wq[rq % nq] * hh[tang[t]];
        rq /= nq;
      }
      wfc[(size_t)f * nqf + qf] = w;
    }
  }
  const size_t ne = (size_t)nel;
  const size_t ntiles = (ne + 15) / 16;
  vo->T.assign((size_t)S * I * ntiles * 16, 0.0);
  vo->R.assign((size_t)Np * I * ne, 0.0);
  vo->W.assign((size_t)Np * Np * ne, 0.0);
  std::atomic<long long> singular(-1);
  auto work = [&](long long e0, long long e1) {
    Mat A(Np, Np), L(Np, I), Ainv;
    std::vector<double> H((size_t)Nq * Np), Mw((size_t)nf * nf);
    for (long long e = e0; e < e1; ++e) {
      // volume: A(i, j) = sigma M(i, j) - sum_q w_q psi_j (beta . grad psi_i + div(beta) psi_i)
      const double* bq = smp->beta_q + (size_t)e * dim * Nq;
      const double* dq = smp->div_q ? smp->div_q + (size_t)e * Nq : nullptr;
      for (int q = 0; q < Nq; ++q) {
        double ca[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) ca[a] = wvol[q] * bq[(size_t)a * Nq + q] / hh[a];
        const double cd = dq ? wvol[q] * dq[q] : 0.0;
        for (int i = 0; i < Np; ++i) {
          double v = cd * Psi[(size_t)q * Np + i];
          for (int a = 0; a < dim; ++a) v += ca[a] * G[((size_t)a * Nq + q) * Np + i];
          H[(size_t)q * Np + i] = v;
        }
      }
      for (int i = 0; i < Np; ++i)
        for (int j = 0; j < Np; ++j) A(i, j) = d.sigma * E.M(i, j);
      for (int q = 0; q < Nq; ++q)
        for (int i = 0; i < Np; ++i) {
          const double h = H[(size_t)q * Np + i];
          if (h == 0.0) continue;
          for (int j = 0; j < Np; ++j) A(i, j) -= h * Psi[(size_t)q * Np + j];
        }
      // faces of the active axes: weighted face mass Mw = <|beta.n| mu_c, mu_a>_f
      std::fill(L.a.begin(), L.a.end(), 0.0);
      for (int t = 0; t < na; ++t) {
        const int ax = ops.ax[t];
        const int f_in = 2 * ax + (ops.dir[t] > 0 ? 0 : 1), f_out = f_in ^ 1;
        for (int side = 0; side < 2; ++side) {
          const int f = side ? f_out : f_in;
          const double* bf = smp->beta_face + ((size_t)e * 2 * dim + f) * nqf;
          std::fill(Mw.begin(), Mw.end(), 0.0);
          for (int qf = 0; qf < nqf; ++qf) {
            const double w = wfc[(size_t)f * nqf + qf] * std::fabs(bf[qf]);
            for (int c = 0; c < nf; ++c) {
              const double wc = w * mu[(size_t)qf * nf + c];
              for (int k = 0; k < nf; ++k) Mw[(size_t)c * nf + k] += wc * mu[(size_t)qf * nf + k];
            }
          }
          const int col0 = (side ? na + t : t) * nf;
          for (int c = 0; c < nf; ++c)
            for (int k = 0; k < nf; ++k) {
              L(E.fn[f][c], col0 + k) = Mw[(size_t)c * nf + k];
              // beta.n + |beta.n| = 2 |beta.n| on the outflow face, 0 on the inflow face
              if (side) A(E.fn[f][c], E.fn[f][k]) += 2.0 * Mw[(size_t)c * nf + k];
            }
        }
      }
      if (!invert(A, Ainv)) {
        singular.store(e);
        continue;
      }
      const Mat R = matmul(Ainv, L);
      for (int col = 0; col < I; ++col) {
        for (int r = 0; r < Np; ++r) vo->R[((size_t)col * Np + r) * ne + e] = R(r, col);
        for (int t = 0; t < na; ++t) {
          const int ax = ops.ax[t];
          const int f_out = (2 * ax + (ops.dir[t] > 0 ? 0 : 1)) ^ 1;
          for (int c = 0; c < nf; ++c)
            vo->T[(((size_t)(e / 16) * I + col) * S + t * nf + c) * 16 + e % 16] = R(E.fn[f_out][c], col);
        }
      }
      for (int col = 0; col < Np; ++col)
        for (int r = 0; r < Np; ++r) vo->W[((size_t)col * Np + r) * ne + e] = Ainv(r, col);
    }
  };
  unsigned nt = std::thread::hardware_concurrency();
  nt = std::max(1u, std::min(nt, 16u));
  if ((long long)nt > nel) nt = (unsigned)nel;
  std::vector<std::thread> pool;
  const long long chunk = (nel + nt - 1) / nt;
  for (unsigned k = 0; k < nt; ++k) {
    const long long e0 = k * chunk, e1 = std::min(nel, e0 + chunk);
    if (e0 < e1) pool.emplace_back(work, e0, e1);
  }
  for (auto& th : pool) th.join();
  if (singular.load() >= 0) return "the local operator of an element is singular";
  return "";
}

}  // namespace ehdg
