// Host-side (FP64) construction of the eHDG element operators.
//
// For a uniform mesh with constant coefficients every element has the same local
// operator, so the iteration is written in "trace form": with s the per-element
// trace state and in(s) the gathered inputs of one element (its own and its
// neighbours' face data),
//     u^{k+1} = A^{-1} (F + L in(s^k))                 (local solve, Algorithm 1)
//     s^{k+1} = Q u^{k+1} = g + T in(s^k),  T = Q A^{-1} L,  g = Q A^{-1} F.
// Only T (S x I) and g are needed per sweep; u is recovered at the end with
// R = A^{-1} L.  For backward Euler, F = F_src + Mbt u^m and the next step's
// g = g_src + G u^{m+1} with G = Q A^{-1} Mbt, u^{m+1} = w_src + P u^m + R in,
// P = A^{-1} Mbt.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace ehdg {

struct Basis1D {
  int p = 0, nq = 0;
  std::vector<double> x, w;    // GLL nodes and weights (p+1)
  std::vector<double> xq, wq;  // Gauss points and weights (p+2)
  std::vector<double> B;       // nq x (p+1): l_j(xq_i)
  std::vector<double> dB;      // nq x (p+1): l_j'(xq_i)
  std::vector<double> M1;      // (p+1)^2: int l_i l_j
  std::vector<double> K1;      // (p+1)^2: K1[i][j] = int l_j l_i'
};

Basis1D make_basis(int p);

// Dense row-major matrix helpers.
struct Mat {
  int r = 0, c = 0;
  std::vector<double> a;
  Mat() = default;
  Mat(int r_, int c_) : r(r_), c(c_), a((size_t)r_ * c_, 0.0) {}
  double& operator()(int i, int j) { return a[(size_t)i * c + j]; }
  double operator()(int i, int j) const { return a[(size_t)i * c + j]; }
};
Mat matmul(const Mat& A, const Mat& B);
// Inverse by LU with partial pivoting; returns false if singular.
bool invert(const Mat& A, Mat& Ainv);

enum class Pde { Transport = 0, Swe = 1, Euler = 2 };

// Everything the device needs for one problem.
struct Operators {
  Pde pde;
  int dim = 2, p = 1, m = 1, Np = 0, nf = 0, n = 0;  // n = m * Np
  int S = 0, I = 0;                                   // trace state / gathered inputs per element
  int nq_el = 0;                                      // Gauss points per element
  // transport: active axes (beta component nonzero), their upwind step (+1 when
  // beta > 0: the inflow face is the minus face and the upwind neighbour is i-1)
  int na = 0, ax[3] = {0, 0, 0}, dir[3] = {0, 0, 0};
  bool be = false;  // backward Euler (dt > 0)
  Mat T;            // S x I
  Mat R;            // n x I
  Mat Q;            // S x n
  Mat W;            // n x n  (A^{-1}: source part of the local solve)
  Mat P;            // n x n  (A^{-1} Mbt), BE only
  Mat G;            // S x n  (Q A^{-1} Mbt), BE only
  Mat Bload;        // Np x nq_el: F_i = sum_q Bload(i,q) f_q for one field
  // recovery as one contraction: steady u = w + R in; BE [u; g_next] = [w; gbe] +
  // [[P, R], [G P, G R]] [u_old; in]
  Mat Mvol;
};

struct Desc {
  int pde, dim, n[3];
  double L[3];
  int periodic[3];
  int degree;
  double beta[3], sigma, Phi, dt;
  double U0[2], c0, rho0;
};

// Builds the operators; returns an empty string on success, else an error message.
std::string build_operators(const Desc& d, Operators& ops);

// Transport with a velocity field beta(x) (the steady problems of Sections 4.1-4.3).
// Every element has its own local operator
//   A_e = -(psi_j, div(beta psi_i)) + sum_f <(beta.n + |beta.n|) psi_j, psi_i>_f + sigma (psi_j, psi_i)
// with the lifts L_e = <|beta.n| mu_a, psi_i>_f of the inflow and own outflow faces, so
// the trace form keeps per element T_e = Q A_e^{-1} L_e, R_e = A_e^{-1} L_e and
// W_e = A_e^{-1}.  T is tile-major for the sweep (element e = 16 t + j:
// T[((t * I + col) * S + row) * 16 + j], the last tile padded with zeros); R and W are
// entry-major with the element index fastest: X[(col * rows + row) * nel + e].
// The trace keeps the constant-velocity structure
// when every velocity component is one-signed on the faces normal to its axis (no
// face quadrature point with beta.n = 0 or of the other sign); that is checked.
struct VarSamples {
  const double* beta_q;     // [nel][dim][nq^dim]   velocity at the tensor Gauss points
  const double* div_q;      // [nel][nq^dim]        div beta there, or null (zero)
  const double* beta_face;  // [nel][2 dim][nq^(dim-1)]  beta_(f/2) at the face Gauss points
};
struct VarOperators {
  std::vector<double> T, R, W;
};
// ops gets the shape, Q and the load matrix (the element-independent parts); with
// vo == null only the shape for the maximum number of active axes (workspace sizing).
std::string build_variable_operators(const Desc& d, const VarSamples* smp, Operators& ops, VarOperators* vo);

}  // namespace ehdg
