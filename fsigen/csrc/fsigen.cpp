// Synthetic linearised ALE-FSI Jacobian generator (seeded input only).
//
// Assembles, on a structured channel of Q2 (velocity, displacement) / Q1
// (pressure) quads or hexes, the Newton matrix and right-hand side of the
// monolithic ALE fluid-structure system written as the sum of the variational
// equations in the paper's Section 3 (the semi-linear form A(U)(Phi) minus the
// linear form F(Phi), Backward Euler theta = 1).  The derivative of every
// quadrature-point integrand with respect to the local field values
// (v, grad v, u, grad u, p) is taken by forward-mode dual numbers, which gives
// exactly the shape derivatives of the FSI-related derivative theorem
// (dF, dJ, dF^{-1}, dF^{-T}) without expanding them by hand.
//
// Two quantities are held frozen at the linearisation state (they are inputs,
// not unknowns): the advecting velocity in the convective term (Oseen-type
// linearisation) and 1/J in the harmonic mesh-motion equation
// (Jacobian-scaled stiffness).  With those held fixed the matrix is the exact
// derivative of the residual this file evaluates, which is what the
// finite-difference tests check.
//
// This module holds no part of the linear solver: it only writes the blocks
// M, C_ms, C_sm, S, C_sf, C_fm, C_fs, F of the 3x3 block system (Section 3.4,
// the block matrix A_h) and the Newton right-hand side.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <string>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {
typedef struct {
  int32_t dim;
  int32_t nc[3];
  double L[3];
  int32_t solid_lo[3], solid_hi[3];
  double rho_f, nu_f, rho_s, mu_s, lambda_s, dt, theta;
  double v_peak, u_peak, p_amp;
  uint64_t seed;
  double t_phase;      // pseudo-time phase angle (radians): a cos + a' sin
  int32_t newton_mesh; // 1: differentiate 1/J in the mesh equation too
  int32_t pad;
} fsigen_cfg;
}

namespace {

// ---------------------------------------------------------------- dual numbers
template <int N> struct Dual {
  double v;
  double d[N];
};
template <int N> inline Dual<N> dconst(double c) {
  Dual<N> r;
  r.v = c;
  for (int i = 0; i < N; ++i) r.d[i] = 0.0;
  return r;
}
template <int N> inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v + b.v;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <int N> inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v - b.v;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <int N> inline Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r; r.v = -a.v;
  for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
  return r;
}
template <int N> inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v * b.v;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <int N> inline Dual<N> operator*(double s, const Dual<N>& a) {
  Dual<N> r; r.v = s * a.v;
  for (int i = 0; i < N; ++i) r.d[i] = s * a.d[i];
  return r;
}
template <int N> inline Dual<N> operator*(const Dual<N>& a, double s) { return s * a; }
template <int N> inline Dual<N> operator+(const Dual<N>& a, double s) {
  Dual<N> r = a; r.v += s; return r;
}
template <int N> inline Dual<N> operator-(const Dual<N>& a, double s) {
  Dual<N> r = a; r.v -= s; return r;
}
template <int N> inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v / b.v;
  const double ib = 1.0 / b.v;
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib;
  return r;
}
template <int N> inline Dual<N> operator/(double s, const Dual<N>& b) {
  return dconst<N>(s) / b;
}

inline double dconst_like(double, double c) { return c; }
template <int N> inline Dual<N> dconst_like(const Dual<N>&, double c) { return dconst<N>(c); }

// -------------------------------------------------------- small tensor algebra
template <class T, int D> struct Mat { T a[D][D]; };

template <class T> inline T det2(const Mat<T, 2>& F) { return F.a[0][0] * F.a[1][1] - F.a[0][1] * F.a[1][0]; }
template <class T> inline T det3(const Mat<T, 3>& F) {
  return F.a[0][0] * (F.a[1][1] * F.a[2][2] - F.a[1][2] * F.a[2][1]) -
         F.a[0][1] * (F.a[1][0] * F.a[2][2] - F.a[1][2] * F.a[2][0]) +
         F.a[0][2] * (F.a[1][0] * F.a[2][1] - F.a[1][1] * F.a[2][0]);
}
template <class T> inline T detD(const Mat<T, 2>& F) { return det2(F); }
template <class T> inline T detD(const Mat<T, 3>& F) { return det3(F); }

template <class T> inline Mat<T, 2> invD(const Mat<T, 2>& F, const T& J) {
  Mat<T, 2> r;
  r.a[0][0] = F.a[1][1] / J; r.a[0][1] = -F.a[0][1] / J;
  r.a[1][0] = -F.a[1][0] / J; r.a[1][1] = F.a[0][0] / J;
  return r;
}
template <class T> inline Mat<T, 3> invD(const Mat<T, 3>& F, const T& J) {
  Mat<T, 3> r;
  r.a[0][0] = (F.a[1][1] * F.a[2][2] - F.a[1][2] * F.a[2][1]) / J;
  r.a[0][1] = (F.a[0][2] * F.a[2][1] - F.a[0][1] * F.a[2][2]) / J;
  r.a[0][2] = (F.a[0][1] * F.a[1][2] - F.a[0][2] * F.a[1][1]) / J;
  r.a[1][0] = (F.a[1][2] * F.a[2][0] - F.a[1][0] * F.a[2][2]) / J;
  r.a[1][1] = (F.a[0][0] * F.a[2][2] - F.a[0][2] * F.a[2][0]) / J;
  r.a[1][2] = (F.a[0][2] * F.a[1][0] - F.a[0][0] * F.a[1][2]) / J;
  r.a[2][0] = (F.a[1][0] * F.a[2][1] - F.a[1][1] * F.a[2][0]) / J;
  r.a[2][1] = (F.a[0][1] * F.a[2][0] - F.a[0][0] * F.a[2][1]) / J;
  r.a[2][2] = (F.a[0][0] * F.a[1][1] - F.a[0][1] * F.a[1][0]) / J;
  return r;
}

// --------------------------------------------------------------- parameters
struct Phys {
  double rho_f, nu_f, rho_s, mu_s, lambda_s, dtth;
  int newton_mesh;
};

// Index layout of the quadrature-point unknowns q and of the integrand outputs.
// Inputs:  v[c] | grad v[c][k] | u[c] | grad u[c][k] | p
// Outputs: f_v[c] | g_v[c][k] | f_u[c] | g_u[c][k] | f_p
// A residual contribution to test function phi (field X, component c) is
//   f_X[c] * phi + sum_k g_X[c][k] * d_k phi.
template <int D> struct Lay {
  static constexpr int V = 0, GV = D, U = D + D * D, GU = 2 * D + D * D, P = 2 * D + 2 * D * D;
  static constexpr int NQ = 2 * D + 2 * D * D + 1;
};

template <int D> struct Frozen {
  double a[D];      // advecting velocity (Oseen)
  double vold[D], uold[D];
  double Jbar;      // 1/J frozen in the mesh equation
};

// Fluid cell integrand (momentum in ALE form, incompressibility, harmonic mesh
// motion with Jacobian-scaled stiffness), Section 3.3 sum of the equations.
template <int D, class T>
void fluid_integrand(const T* q, const Frozen<D>& fz, const Phys& ph, T* out) {
  using L = Lay<D>;
  Mat<T, D> F, GVm;
  for (int c = 0; c < D; ++c)
    for (int k = 0; k < D; ++k) {
      F.a[c][k] = q[L::GU + c * D + k] + (c == k ? 1.0 : 0.0);
      GVm.a[c][k] = q[L::GV + c * D + k];
    }
  T J = detD(F);
  Mat<T, D> Fi = invD(F, J);
  // GF = grad v F^{-1}
  Mat<T, D> GF;
  for (int c = 0; c < D; ++c)
    for (int k = 0; k < D; ++k) {
      T s = GVm.a[c][0] * Fi.a[0][k];
      for (int m = 1; m < D; ++m) s = s + GVm.a[c][m] * Fi.a[m][k];
      GF.a[c][k] = s;
    }
  const double rho = ph.rho_f, mu = ph.rho_f * ph.nu_f, dtth = ph.dtth;
  for (int c = 0; c < D; ++c) {
    T adv = GF.a[c][0] * fz.a[0];
    T mv = GF.a[c][0] * (q[L::U + 0] - fz.uold[0]);
    for (int k = 1; k < D; ++k) {
      adv = adv + GF.a[c][k] * fz.a[k];
      mv = mv + GF.a[c][k] * (q[L::U + k] - fz.uold[k]);
    }
    out[L::V + c] = rho * (J * (q[L::V + c] - fz.vold[c])) + (dtth * rho) * (J * adv) - rho * (J * mv);
  }
  // g_v = dt theta J sigma_v F^{-T} - J p F^{-T},  sigma_v = rho nu (GF + GF^T)
  for (int c = 0; c < D; ++c)
    for (int k = 0; k < D; ++k) {
      T s = (GF.a[c][0] + GF.a[0][c]) * Fi.a[k][0];
      for (int m = 1; m < D; ++m) s = s + (GF.a[c][m] + GF.a[m][c]) * Fi.a[k][m];
      out[L::GV + c * D + k] = (dtth * mu) * (J * s) - J * (q[L::P] * Fi.a[k][c]);
    }
  T tr = GF.a[0][0];
  for (int c = 1; c < D; ++c) tr = tr + GF.a[c][c];
  out[L::P] = J * tr;
  for (int c = 0; c < D; ++c) out[L::U + c] = dconst_like(q[0], 0.0);
  if (ph.newton_mesh) {
    for (int c = 0; c < D; ++c)
      for (int k = 0; k < D; ++k) out[L::GU + c * D + k] = q[L::GU + c * D + k] / J;
  } else {
    const double iJ = 1.0 / fz.Jbar;
    for (int c = 0; c < D; ++c)
      for (int k = 0; k < D; ++k) out[L::GU + c * D + k] = iJ * q[L::GU + c * D + k];
  }
}

// Outflow boundary correction of the symmetric fluid stress on x = L (normal e_x):
//   -dt theta rho nu < J F^{-T} grad v^T F^{-T} n , phi >.
template <int D, class T>
void outflow_integrand(const T* q, const Phys& ph, T* out) {
  using L = Lay<D>;
  Mat<T, D> F;
  for (int c = 0; c < D; ++c)
    for (int k = 0; k < D; ++k) F.a[c][k] = q[L::GU + c * D + k] + (c == k ? 1.0 : 0.0);
  T J = detD(F);
  Mat<T, D> Fi = invD(F, J);
  T w[D], z[D];
  for (int m = 0; m < D; ++m) w[m] = Fi.a[0][m];  // F^{-T} e_x
  for (int k = 0; k < D; ++k) {
    T s = q[L::GV + 0 * D + k] * w[0];
    for (int m = 1; m < D; ++m) s = s + q[L::GV + m * D + k] * w[m];
    z[k] = s;  // grad v^T w
  }
  const double coef = -ph.dtth * ph.rho_f * ph.nu_f;
  for (int c = 0; c < D; ++c) {
    T y = Fi.a[0][c] * z[0];
    for (int k = 1; k < D; ++k) y = y + Fi.a[k][c] * z[k];
    out[L::V + c] = coef * (J * y);
  }
}

// Solid cell integrand (St. Venant-Kirchhoff elastodynamics and kinematics).
template <int D, class T>
void solid_integrand(const T* q, const Frozen<D>& fz, const Phys& ph, T* out) {
  using L = Lay<D>;
  Mat<T, D> F;
  for (int c = 0; c < D; ++c)
    for (int k = 0; k < D; ++k) F.a[c][k] = q[L::GU + c * D + k] + (c == k ? 1.0 : 0.0);
  Mat<T, D> E;
  for (int c = 0; c < D; ++c)
    for (int k = 0; k < D; ++k) {
      T s = F.a[0][c] * F.a[0][k];
      for (int m = 1; m < D; ++m) s = s + F.a[m][c] * F.a[m][k];
      E.a[c][k] = 0.5 * (s - (c == k ? 1.0 : 0.0));
    }
  T trE = E.a[0][0];
  for (int c = 1; c < D; ++c) trE = trE + E.a[c][c];
  Mat<T, D> S;
  for (int c = 0; c < D; ++c)
    for (int k = 0; k < D; ++k) {
      S.a[c][k] = (2.0 * ph.mu_s) * E.a[c][k];
      if (c == k) S.a[c][k] = S.a[c][k] + ph.lambda_s * trE;
    }
  for (int c = 0; c < D; ++c)
    for (int k = 0; k < D; ++k) {
      T s = F.a[c][0] * S.a[0][k];
      for (int m = 1; m < D; ++m) s = s + F.a[c][m] * S.a[m][k];
      out[L::GV + c * D + k] = ph.dtth * s;
    }
  for (int c = 0; c < D; ++c) {
    out[L::V + c] = ph.rho_s * (q[L::V + c] - fz.vold[c]);
    out[L::U + c] = (q[L::U + c] - fz.uold[c]) - ph.dtth * q[L::V + c];
    for (int k = 0; k < D; ++k) out[L::GU + c * D + k] = dconst_like(q[0], 0.0);
  }
  out[L::P] = dconst_like(q[0], 0.0);
}


// ------------------------------------------------------------- 1D shape data
// Q2 Lagrange basis on [0,1] with nodes 0, 1/2, 1 and Q1 basis with nodes 0, 1.
inline void q2_1d(double x, double* N, double* dN) {
  N[0] = (2.0 * x - 1.0) * (x - 1.0);
  N[1] = 4.0 * x * (1.0 - x);
  N[2] = x * (2.0 * x - 1.0);
  dN[0] = 4.0 * x - 3.0;
  dN[1] = 4.0 - 8.0 * x;
  dN[2] = 4.0 * x - 1.0;
}
inline void q1_1d(double x, double* M) {
  M[0] = 1.0 - x;
  M[1] = x;
}
const double kGx[3] = {0.5 - 0.38729833462074168852, 0.5, 0.5 + 0.38729833462074168852};
const double kGw[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};

// -------------------------------------------------------------- smooth fields
// f(x) = sum_{k in {1,2,3}^d} a_k |k|^-2 prod_i sin(k_i pi (x_i - xmin_i) / L_i)
// with a_k = cos(t) a_k^0 + sin(t) a_k^1, a^0, a^1 uniform on [-1,1] drawn from
// mt19937_64 as ((x >> 11) * 2^-53) * 2 - 1.  Every component of every field
// draws its own two coefficient sets, in the order v_0..v_{d-1}, u_0..u_{d-1}, p.
struct Smooth {
  int D;
  double L[3];
  std::vector<double> coef;  // 3^D coefficients
  double eval(const double* x) const {
    double s = 0.0;
    int nk = 1;
    for (int a = 0; a < D; ++a) nk *= 3;
    for (int id = 0; id < nk; ++id) {
      int k[3] = {1, 1, 1};
      int r = id;
      for (int a = D - 1; a >= 0; --a) { k[a] = 1 + r % 3; r /= 3; }
      double kk = 0.0, prod = 1.0;
      for (int a = 0; a < D; ++a) {
        kk += double(k[a]) * double(k[a]);
        prod *= std::sin(double(k[a]) * M_PI * x[a] / L[a]);
      }
      s += coef[id] * prod / kk;
    }
    return s;
  }
};

struct Gen {
  fsigen_cfg cfg;
  int D;
  int nc[3];
  int NN[3];
  double h[3];
  int64_t nnodes, ncells;
  std::vector<uint8_t> cell_solid;
  std::vector<uint8_t> node_flags;  // bit0 solid, bit1 fluid, bit2 v-dirichlet, bit3 u-dirichlet
  std::vector<int64_t> vdof, udof, pdof;  // base dof (component 0) or -1
  int64_t n_m = 0, n_vs = 0, n_vf = 0, n_p = 0, N = 0;
  // fields at Q2 nodes (component-interleaved) and p at nodes (used at vertices)
  std::vector<double> vbar, ubar, pbar;
  // global CSR pattern / values
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<double> val;
  std::vector<double> res;
  std::string err;
  bool bad_pattern = false;
  double min_J = 1e300, max_J = -1e300;

  int64_t node_id(const int* I) const {
    int64_t id = I[0];
    for (int a = 1; a < D; ++a) id = id * NN[a] + I[a];
    return id;
  }
  void node_ijk(int64_t id, int* I) const {
    for (int a = D - 1; a >= 0; --a) { I[a] = int(id % NN[a]); id /= NN[a]; }
  }
  int64_t cell_id(const int* C) const {
    int64_t id = C[0];
    for (int a = 1; a < D; ++a) id = id * nc[a] + C[a];
    return id;
  }
  void cell_ijk(int64_t id, int* C) const {
    for (int a = D - 1; a >= 0; --a) { C[a] = int(id % nc[a]); id /= nc[a]; }
  }
  int nq2() const { return D == 2 ? 9 : 27; }
  int nq1() const { return D == 2 ? 4 : 8; }
  // Local Q2 node l -> global node id of cell C.
  int64_t cell_node(const int* C, int l) const {
    int I[3] = {0, 0, 0};
    int r = l;
    for (int a = D - 1; a >= 0; --a) { I[a] = 2 * C[a] + r % 3; r /= 3; }
    return node_id(I);
  }
  int64_t cell_vertex(const int* C, int l) const {
    int I[3] = {0, 0, 0};
    int r = l;
    for (int a = D - 1; a >= 0; --a) { I[a] = 2 * C[a] + 2 * (r % 2); r /= 2; }
    return node_id(I);
  }
  // Cells containing node I (at most 2^D).
  int node_cells(const int* I, int64_t* out) const {
    int lo[3], hi[3];
    for (int a = 0; a < D; ++a) {
      if (I[a] % 2 == 0) { lo[a] = I[a] / 2 - 1; hi[a] = I[a] / 2; }
      else { lo[a] = hi[a] = (I[a] - 1) / 2; }
      lo[a] = std::max(lo[a], 0);
      hi[a] = std::min(hi[a], nc[a] - 1);
    }
    int n = 0;
    int C[3] = {0, 0, 0};
    if (D == 2) {
      for (C[0] = lo[0]; C[0] <= hi[0]; ++C[0])
        for (C[1] = lo[1]; C[1] <= hi[1]; ++C[1]) out[n++] = cell_id(C);
    } else {
      for (C[0] = lo[0]; C[0] <= hi[0]; ++C[0])
        for (C[1] = lo[1]; C[1] <= hi[1]; ++C[1])
          for (C[2] = lo[2]; C[2] <= hi[2]; ++C[2]) out[n++] = cell_id(C);
    }
    return n;
  }

  bool setup() {
    D = cfg.dim;
    if (D != 2 && D != 3) { err = "dim must be 2 or 3"; return false; }
    if (cfg.theta != 1.0) { err = "only theta = 1 (Backward Euler) is generated"; return false; }
    nnodes = 1; ncells = 1;
    for (int a = 0; a < 3; ++a) {
      nc[a] = a < D ? cfg.nc[a] : 1;
      NN[a] = a < D ? 2 * nc[a] + 1 : 1;
      h[a] = a < D ? cfg.L[a] / nc[a] : 1.0;
      if (a < D) { nnodes *= NN[a]; ncells *= nc[a]; }
      if (a < D && nc[a] < 1) { err = "bad cell count"; return false; }
    }
    cell_solid.assign(ncells, 0);
    for (int64_t c = 0; c < ncells; ++c) {
      int C[3] = {0, 0, 0};
      cell_ijk(c, C);
      bool s = true;
      for (int a = 0; a < D; ++a) s = s && C[a] >= cfg.solid_lo[a] && C[a] < cfg.solid_hi[a];
      cell_solid[c] = s;
    }
    node_flags.assign(nnodes, 0);
    for (int64_t n = 0; n < nnodes; ++n) {
      int I[3] = {0, 0, 0};
      node_ijk(n, I);
      int64_t cs[8];
      int k = node_cells(I, cs);
      uint8_t f = 0;
      for (int i = 0; i < k; ++i) f |= cell_solid[cs[i]] ? 1 : 2;
      bool x0 = I[0] == 0, x1 = I[0] == NN[0] - 1;
      bool wall = I[1] == 0 || I[1] == NN[1] - 1;
      if (D == 3) wall = wall || I[2] == 0 || I[2] == NN[2] - 1;
      if (x0 || wall) f |= 4;          // v: inflow and walls (outflow is do-nothing)
      if (x0 || x1 || wall) f |= 8;    // u: whole outer boundary
      node_flags[n] = f;
    }
    // dof numbering in block order: mesh | solid v | solid u | fluid v | p
    vdof.assign(nnodes, -1); udof.assign(nnodes, -1); pdof.assign(nnodes, -1);
    int64_t off = 0;
    for (int64_t n = 0; n < nnodes; ++n) {
      uint8_t f = node_flags[n];
      if ((f & 2) && !(f & 1) && !(f & 8)) { udof[n] = off; off += D; }
    }
    n_m = off;
    for (int64_t n = 0; n < nnodes; ++n) {
      uint8_t f = node_flags[n];
      if ((f & 1) && !(f & 4)) { vdof[n] = off; off += D; }
    }
    n_vs = off - n_m;
    for (int64_t n = 0; n < nnodes; ++n) {
      uint8_t f = node_flags[n];
      if ((f & 1) && !(f & 8)) { udof[n] = off; off += D; }
      if ((f & 1) && (((f & 4) != 0) != ((f & 8) != 0))) {
        err = "solid velocity and displacement Dirichlet sets differ";
        return false;
      }
    }
    if (off - n_m - n_vs != n_vs) { err = "solid v/u dof counts differ"; return false; }
    for (int64_t n = 0; n < nnodes; ++n) {
      uint8_t f = node_flags[n];
      if ((f & 2) && !(f & 1) && !(f & 4)) { vdof[n] = off; off += D; }
    }
    n_vf = off - n_m - 2 * n_vs;
    for (int64_t c = 0; c < ncells; ++c) {
      if (cell_solid[c]) continue;
      int C[3] = {0, 0, 0};
      cell_ijk(c, C);
      for (int l = 0; l < nq1(); ++l) {
        int64_t n = cell_vertex(C, l);
        if (pdof[n] < 0) pdof[n] = 1;  // mark; numbered below in node order
      }
    }
    for (int64_t n = 0; n < nnodes; ++n)
      if (pdof[n] >= 0) { pdof[n] = off; off += 1; }
    n_p = off - n_m - 2 * n_vs - n_vf;
    N = off;
    if (N >= (int64_t(1) << 31)) { err = "too many dofs for int32 columns"; return false; }
    return true;
  }

  void make_fields() {
    std::mt19937_64 rng(cfg.seed);
    auto draw = [&]() { return (double(rng() >> 11) * 0x1.0p-53) * 2.0 - 1.0; };
    int nk = D == 2 ? 9 : 27;
    auto make = [&]() {
      Smooth s;
      s.D = D;
      for (int a = 0; a < 3; ++a) s.L[a] = cfg.L[a];
      std::vector<double> a0(nk), a1(nk);
      for (int i = 0; i < nk; ++i) a0[i] = draw();
      for (int i = 0; i < nk; ++i) a1[i] = draw();
      s.coef.resize(nk);
      for (int i = 0; i < nk; ++i) s.coef[i] = std::cos(cfg.t_phase) * a0[i] + std::sin(cfg.t_phase) * a1[i];
      return s;
    };
    std::vector<Smooth> fv, fu;
    for (int c = 0; c < D; ++c) fv.push_back(make());
    for (int c = 0; c < D; ++c) fu.push_back(make());
    Smooth fp = make();
    vbar.assign(nnodes * D, 0.0); ubar.assign(nnodes * D, 0.0); pbar.assign(nnodes, 0.0);
    double vmax = 0.0, umax = 0.0, pmax = 0.0;
#pragma omp parallel for reduction(max : vmax, umax, pmax) schedule(static)
    for (int64_t n = 0; n < nnodes; ++n) {
      int I[3] = {0, 0, 0};
      node_ijk(n, I);
      double x[3] = {0, 0, 0};
      for (int a = 0; a < D; ++a) x[a] = 0.5 * h[a] * I[a];
      double vv = 0.0, uu = 0.0;
      for (int c = 0; c < D; ++c) {
        vbar[n * D + c] = fv[c].eval(x);
        ubar[n * D + c] = fu[c].eval(x);
        vv += vbar[n * D + c] * vbar[n * D + c];
        uu += ubar[n * D + c] * ubar[n * D + c];
      }
      pbar[n] = fp.eval(x);
      vmax = std::max(vmax, std::sqrt(vv));
      umax = std::max(umax, std::sqrt(uu));
      pmax = std::max(pmax, std::fabs(pbar[n]));
    }
    for (auto& x : vbar) x *= cfg.v_peak / vmax;
    for (auto& x : ubar) x *= cfg.u_peak / umax;
    for (auto& x : pbar) x *= cfg.p_amp / pmax;
  }

  // Column rule: which local dofs of a cell a row couples to, given the
  // structure of the integrands (mass terms are component-diagonal, the frozen
  // mesh Laplacian is component-diagonal).
  void build_pattern() {
    rowptr.assign(N + 1, 0);
    std::vector<std::vector<int32_t>> rows(N);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t n = 0; n < nnodes; ++n) {
      int I[3] = {0, 0, 0};
      node_ijk(n, I);
      int64_t cs[8];
      int kc = node_cells(I, cs);
      uint8_t f = node_flags[n];
      // v rows
      if (vdof[n] >= 0) {
        for (int c = 0; c < D; ++c) {
          auto& r = rows[vdof[n] + c];
          for (int i = 0; i < kc; ++i) {
            int C[3] = {0, 0, 0};
            cell_ijk(cs[i], C);
            bool solid = cell_solid[cs[i]];
            for (int l = 0; l < nq2(); ++l) {
              int64_t m = cell_node(C, l);
              if (vdof[m] >= 0) {
                if (solid) r.push_back(int32_t(vdof[m] + c));
                else for (int e = 0; e < D; ++e) r.push_back(int32_t(vdof[m] + e));
              }
              if (udof[m] >= 0) for (int e = 0; e < D; ++e) r.push_back(int32_t(udof[m] + e));
            }
            if (!solid)
              for (int l = 0; l < nq1(); ++l) {
                int64_t m = cell_vertex(C, l);
                if (pdof[m] >= 0) r.push_back(int32_t(pdof[m]));
              }
          }
        }
      }
      // u rows: solid kinematics on solid nodes, mesh motion on fluid-only nodes
      if (udof[n] >= 0) {
        for (int c = 0; c < D; ++c) {
          auto& r = rows[udof[n] + c];
          for (int i = 0; i < kc; ++i) {
            bool solid = cell_solid[cs[i]];
            if ((f & 1) != solid) continue;
            int C[3] = {0, 0, 0};
            cell_ijk(cs[i], C);
            for (int l = 0; l < nq2(); ++l) {
              int64_t m = cell_node(C, l);
              if (solid) {
                if (udof[m] >= 0) r.push_back(int32_t(udof[m] + c));
                if (vdof[m] >= 0) r.push_back(int32_t(vdof[m] + c));
              } else if (udof[m] >= 0) {
                if (cfg.newton_mesh) for (int e = 0; e < D; ++e) r.push_back(int32_t(udof[m] + e));
                else r.push_back(int32_t(udof[m] + c));
              }
            }
          }
        }
      }
      // p rows
      if (pdof[n] >= 0) {
        auto& r = rows[pdof[n]];
        for (int i = 0; i < kc; ++i) {
          if (cell_solid[cs[i]]) continue;
          int C[3] = {0, 0, 0};
          cell_ijk(cs[i], C);
          for (int l = 0; l < nq2(); ++l) {
            int64_t m = cell_node(C, l);
            if (vdof[m] >= 0) for (int e = 0; e < D; ++e) r.push_back(int32_t(vdof[m] + e));
            if (udof[m] >= 0) for (int e = 0; e < D; ++e) r.push_back(int32_t(udof[m] + e));
          }
        }
      }
    }
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < N; ++i) {
      auto& r = rows[i];
      std::sort(r.begin(), r.end());
      r.erase(std::unique(r.begin(), r.end()), r.end());
    }
    for (int64_t i = 0; i < N; ++i) rowptr[i + 1] = rowptr[i] + int64_t(rows[i].size());
    col.resize(rowptr[N]);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
      std::copy(rows[i].begin(), rows[i].end(), col.begin() + rowptr[i]);
      std::vector<int32_t>().swap(rows[i]);
    }
    val.assign(rowptr[N], 0.0);
    res.assign(N, 0.0);
  }

  inline void add_entry(int64_t r, int32_t c, double v) {
    const int32_t* b = col.data() + rowptr[r];
    const int32_t* e = col.data() + rowptr[r + 1];
    const int32_t* p = std::lower_bound(b, e, c);
    if (p == e || *p != c) {
      if (v != 0.0) bad_pattern = true;
      return;
    }
    val[p - col.data()] += v;
  }

  // Element routine.  Local dof layout: v (node-major, comp) | u | p (vertices).
  template <int DD>
  void element(int64_t cell, const std::vector<double>* dU, double eps, std::vector<double>& Ke,
               std::vector<double>& Re, std::vector<int64_t>& gd, std::vector<uint8_t>& test_on,
               double& jmin, double& jmax, bool want_matrix) {
    using L = Lay<DD>;
    constexpr int NQ = L::NQ;
    constexpr int NQ2 = DD == 2 ? 9 : 27, NQ1 = DD == 2 ? 4 : 8;
    constexpr int NV = NQ2 * DD;
    int C[3] = {0, 0, 0};
    cell_ijk(cell, C);
    const bool solid = cell_solid[cell];
    const int nloc = 2 * NV + (solid ? 0 : NQ1);
    Ke.assign(size_t(nloc) * nloc, 0.0);
    Re.assign(nloc, 0.0);
    gd.assign(nloc, -1);
    test_on.assign(nloc, 0);
    int64_t nodes[NQ2], verts[NQ1];
    for (int l = 0; l < NQ2; ++l) nodes[l] = cell_node(C, l);
    for (int l = 0; l < NQ1; ++l) verts[l] = cell_vertex(C, l);
    // local state values: state = bar + eps * dU at free dofs
    double lv[NV], lu[NV], lvb[NV], lub[NV], lp[NQ1];
    for (int l = 0; l < NQ2; ++l) {
      int64_t n = nodes[l];
      for (int c = 0; c < DD; ++c) {
        lvb[l * DD + c] = vbar[n * DD + c];
        lub[l * DD + c] = ubar[n * DD + c];
        lv[l * DD + c] = lvb[l * DD + c];
        lu[l * DD + c] = lub[l * DD + c];
        if (vdof[n] >= 0) {
          gd[l * DD + c] = vdof[n] + c;
          if (dU) lv[l * DD + c] += eps * (*dU)[vdof[n] + c];
        }
        if (udof[n] >= 0) {
          gd[NV + l * DD + c] = udof[n] + c;
          if (dU) lu[l * DD + c] += eps * (*dU)[udof[n] + c];
        }
        test_on[l * DD + c] = vdof[n] >= 0;
        // mesh equation is not tested at interface nodes; solid kinematics is
        bool utest = solid ? true : !(node_flags[n] & 1);
        test_on[NV + l * DD + c] = (udof[n] >= 0) && utest;
      }
    }
    if (!solid)
      for (int l = 0; l < NQ1; ++l) {
        int64_t n = verts[l];
        lp[l] = pbar[n];
        gd[2 * NV + l] = pdof[n];
        if (dU && pdof[n] >= 0) lp[l] += eps * (*dU)[pdof[n]];
        test_on[2 * NV + l] = pdof[n] >= 0;
      }
    Phys ph{cfg.rho_f, cfg.nu_f, cfg.rho_s, cfg.mu_s, cfg.lambda_s, cfg.dt * cfg.theta, cfg.newton_mesh};
    double detJ = 1.0;
    for (int a = 0; a < DD; ++a) detJ *= h[a];

    // quadrature: volume (3^D points) then the outflow face when present
    const bool outflow = !solid && C[0] == nc[0] - 1;
    const int nvol = DD == 2 ? 9 : 27, nface = DD == 2 ? 3 : 9;
    const int npts = nvol + (outflow ? nface : 0);
    std::vector<double> DB(size_t(nloc) * NQ);
    for (int ip = 0; ip < npts; ++ip) {
      const bool face = ip >= nvol;
      double xi[3], w;
      if (!face) {
        int r = ip;
        w = detJ;
        for (int a = DD - 1; a >= 0; --a) { xi[a] = kGx[r % 3]; w *= kGw[r % 3]; r /= 3; }
      } else {
        int r = ip - nvol;
        w = 1.0;
        xi[0] = 1.0;
        for (int a = DD - 1; a >= 1; --a) { xi[a] = kGx[r % 3]; w *= kGw[r % 3] * h[a]; r /= 3; }
      }
      double n1[3][3], d1[3][3], m1[3][2];
      for (int a = 0; a < DD; ++a) { q2_1d(xi[a], n1[a], d1[a]); q1_1d(xi[a], m1[a]); }
      double N[NQ2], dN[NQ2][DD], M[NQ1];
      for (int l = 0; l < NQ2; ++l) {
        int ia[3];
        int r = l;
        for (int a = DD - 1; a >= 0; --a) { ia[a] = r % 3; r /= 3; }
        double prod = 1.0;
        for (int a = 0; a < DD; ++a) prod *= n1[a][ia[a]];
        N[l] = prod;
        for (int k = 0; k < DD; ++k) {
          double g = d1[k][ia[k]] / h[k];
          for (int a = 0; a < DD; ++a) if (a != k) g *= n1[a][ia[a]];
          dN[l][k] = g;
        }
      }
      for (int l = 0; l < NQ1; ++l) {
        int ia[3];
        int r = l;
        for (int a = DD - 1; a >= 0; --a) { ia[a] = r % 2; r /= 2; }
        double prod = 1.0;
        for (int a = 0; a < DD; ++a) prod *= m1[a][ia[a]];
        M[l] = prod;
      }
      // interpolate state and frozen fields
      double qv[NQ];
      for (int i = 0; i < NQ; ++i) qv[i] = 0.0;
      Frozen<DD> fz;
      double gub[DD][DD];
      for (int c = 0; c < DD; ++c) {
        fz.a[c] = fz.vold[c] = fz.uold[c] = 0.0;
        for (int k = 0; k < DD; ++k) gub[c][k] = 0.0;
      }
      for (int l = 0; l < NQ2; ++l)
        for (int c = 0; c < DD; ++c) {
          qv[L::V + c] += N[l] * lv[l * DD + c];
          qv[L::U + c] += N[l] * lu[l * DD + c];
          fz.a[c] += N[l] * lvb[l * DD + c];
          fz.vold[c] += N[l] * 0.9 * lvb[l * DD + c];
          fz.uold[c] += N[l] * 0.9 * lub[l * DD + c];
          for (int k = 0; k < DD; ++k) {
            qv[L::GV + c * DD + k] += dN[l][k] * lv[l * DD + c];
            qv[L::GU + c * DD + k] += dN[l][k] * lu[l * DD + c];
            gub[c][k] += dN[l][k] * lub[l * DD + c];
          }
        }
      if (!solid)
        for (int l = 0; l < NQ1; ++l) qv[L::P] += M[l] * lp[l];
      {
        Mat<double, DD> Fb;
        for (int c = 0; c < DD; ++c)
          for (int k = 0; k < DD; ++k) Fb.a[c][k] = gub[c][k] + (c == k ? 1.0 : 0.0);
        fz.Jbar = detD(Fb);
        jmin = std::min(jmin, fz.Jbar);
        jmax = std::max(jmax, fz.Jbar);
      }
      Dual<NQ> q[NQ], out[NQ];
      for (int i = 0; i < NQ; ++i) {
        q[i] = dconst<NQ>(qv[i]);
        q[i].d[i] = 1.0;
        out[i] = dconst<NQ>(0.0);
      }
      if (face) outflow_integrand<DD>(q, ph, out);
      else if (solid) solid_integrand<DD>(q, fz, ph, out);
      else fluid_integrand<DD>(q, fz, ph, out);

      // residual
      auto test_val = [&](int t, const double* o) -> double {
        if (t < 2 * NV) {
          const int base = t < NV ? 0 : 1;  // 0: v, 1: u
          const int l = (t % NV) / DD, c = (t % NV) % DD;
          const int fo = base == 0 ? L::V : L::U, go = base == 0 ? L::GV : L::GU;
          double s = o[fo + c] * N[l];
          for (int k = 0; k < DD; ++k) s += o[go + c * DD + k] * dN[l][k];
          return s;
        }
        return o[L::P] * M[t - 2 * NV];
      };
      {
        double ov[NQ];
        for (int i = 0; i < NQ; ++i) ov[i] = out[i].v;
        for (int t = 0; t < nloc; ++t)
          if (test_on[t]) Re[t] += w * test_val(t, ov);
      }
      if (!want_matrix) continue;
      // DB[s][o] = sum_{inputs i of trial s} dout_o/dq_i * B_i(s)
      for (int s = 0; s < nloc; ++s) {
        double* db = &DB[size_t(s) * NQ];
        if (s < 2 * NV) {
          const int base = s < NV ? 0 : 1;
          const int l = (s % NV) / DD, e = (s % NV) % DD;
          const int fi = base == 0 ? L::V : L::U, gi = base == 0 ? L::GV : L::GU;
          for (int o = 0; o < NQ; ++o) {
            double v = out[o].d[fi + e] * N[l];
            for (int k = 0; k < DD; ++k) v += out[o].d[gi + e * DD + k] * dN[l][k];
            db[o] = v;
          }
        } else {
          const double m = M[s - 2 * NV];
          for (int o = 0; o < NQ; ++o) db[o] = out[o].d[L::P] * m;
        }
      }
      for (int t = 0; t < nloc; ++t) {
        if (!test_on[t]) continue;
        double* krow = &Ke[size_t(t) * nloc];
        if (t < 2 * NV) {
          const int base = t < NV ? 0 : 1;
          const int l = (t % NV) / DD, c = (t % NV) % DD;
          const int fo = base == 0 ? L::V : L::U, go = base == 0 ? L::GV : L::GU;
          double tw[4];
          tw[0] = w * N[l];
          for (int k = 0; k < DD; ++k) tw[1 + k] = w * dN[l][k];
          for (int s = 0; s < nloc; ++s) {
            const double* db = &DB[size_t(s) * NQ];
            double v = tw[0] * db[fo + c];
            for (int k = 0; k < DD; ++k) v += tw[1 + k] * db[go + c * DD + k];
            krow[s] += v;
          }
        } else {
          const double tw = w * M[t - 2 * NV];
          for (int s = 0; s < nloc; ++s) krow[s] += tw * DB[size_t(s) * NQ + L::P];
        }
      }
    }
  }

  template <int DD>
  void assemble(const std::vector<double>* dU, double eps, bool want_matrix) {
    int ncolor = 1 << D;
    double jmin = 1e300, jmax = -1e300;
    for (int color = 0; color < ncolor; ++color) {
#pragma omp parallel reduction(min : jmin) reduction(max : jmax)
      {
        std::vector<double> Ke, Re;
        std::vector<int64_t> gd;
        std::vector<uint8_t> ton;
#pragma omp for schedule(dynamic, 16)
        for (int64_t cell = 0; cell < ncells; ++cell) {
          int C[3] = {0, 0, 0};
          cell_ijk(cell, C);
          int cc = 0;
          for (int a = 0; a < D; ++a) cc |= (C[a] & 1) << a;
          if (cc != color) continue;
          element<DD>(cell, dU, eps, Ke, Re, gd, ton, jmin, jmax, want_matrix);
          const int nloc = int(gd.size());
          for (int t = 0; t < nloc; ++t) {
            if (!ton[t] || gd[t] < 0) continue;
            res[gd[t]] += Re[t];
            if (!want_matrix) continue;
            for (int s = 0; s < nloc; ++s) {
              if (gd[s] < 0) continue;
              add_entry(gd[t], int32_t(gd[s]), Ke[size_t(t) * nloc + s]);
            }
          }
        }
      }
    }
    min_J = jmin;
    max_J = jmax;
  }

  bool run(const double* dU_ptr, double eps, bool want_matrix) {
    if (!setup()) return false;
    make_fields();
    if (want_matrix) build_pattern();
    else res.assign(N, 0.0);
    std::vector<double> dU;
    if (dU_ptr) dU.assign(dU_ptr, dU_ptr + N);
    if (D == 2) assemble<2>(dU_ptr ? &dU : nullptr, eps, want_matrix);
    else assemble<3>(dU_ptr ? &dU : nullptr, eps, want_matrix);
    if (bad_pattern) { err = "element entry outside the sparsity pattern"; return false; }
    if (!(min_J > 0.0)) { err = "linearisation state has J <= 0"; return false; }
    return true;
  }
};

// ---------------------------------------------------------------- block split
struct Block {
  int64_t nrows = 0, ncols = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<double> val;
};

}  // namespace

struct fsigen_handle {
  Gen g;
  Block blk[8];
};

extern "C" {

// Block order of A_h: 0 M, 1 C_ms, 2 C_sm, 3 S, 4 C_sf, 5 C_fm, 6 C_fs, 7 F.
int fsigen_build(const fsigen_cfg* cfg, fsigen_handle** out, char* errbuf, int errlen) {
  auto* h = new fsigen_handle();
  h->g.cfg = *cfg;
  if (!h->g.run(nullptr, 0.0, true)) {
    std::snprintf(errbuf, errlen, "%s", h->g.err.c_str());
    delete h;
    return -1;
  }
  Gen& g = h->g;
  const int64_t off[4] = {0, g.n_m, g.n_m + 2 * g.n_vs, g.N};
  const int map[3][3] = {{0, 1, -1}, {2, 3, 4}, {5, 6, 7}};
  for (int bi = 0; bi < 3; ++bi)
    for (int bj = 0; bj < 3; ++bj) {
      const int id = map[bi][bj];
      int64_t cnt = 0;
      for (int64_t r = off[bi]; r < off[bi + 1]; ++r)
        for (int64_t k = g.rowptr[r]; k < g.rowptr[r + 1]; ++k)
          if (g.col[k] >= off[bj] && g.col[k] < off[bj + 1] && g.val[k] != 0.0) ++cnt;
      if (id < 0) {
        if (cnt != 0) {
          std::snprintf(errbuf, errlen, "mesh-fluid block is not empty (%lld entries)", (long long)cnt);
          delete h;
          return -2;
        }
        continue;
      }
      Block& b = h->blk[id];
      b.nrows = off[bi + 1] - off[bi];
      b.ncols = off[bj + 1] - off[bj];
      b.rowptr.assign(b.nrows + 1, 0);
      b.col.reserve(cnt);
      b.val.reserve(cnt);
      for (int64_t r = off[bi]; r < off[bi + 1]; ++r) {
        for (int64_t k = g.rowptr[r]; k < g.rowptr[r + 1]; ++k)
          if (g.col[k] >= off[bj] && g.col[k] < off[bj + 1] && g.val[k] != 0.0) {
            b.col.push_back(int32_t(g.col[k] - off[bj]));
            b.val.push_back(g.val[k]);
          }
        b.rowptr[r - off[bi] + 1] = int64_t(b.col.size());
      }
    }
  // the monolithic pattern is no longer needed
  std::vector<int64_t>().swap(g.rowptr);
  std::vector<int32_t>().swap(g.col);
  std::vector<double>().swap(g.val);
  *out = h;
  return 0;
}

// Sizes: [dim, nnodes, N, n_m, n_s, n_f, n_vs, n_vf, n_p]
void fsigen_sizes(const fsigen_handle* h, int64_t* s) {
  const Gen& g = h->g;
  s[0] = g.D; s[1] = g.nnodes; s[2] = g.N; s[3] = g.n_m; s[4] = 2 * g.n_vs;
  s[5] = g.n_vf + g.n_p; s[6] = g.n_vs; s[7] = g.n_vf; s[8] = g.n_p;
}
void fsigen_block_sizes(const fsigen_handle* h, int id, int64_t* s) {
  s[0] = h->blk[id].nrows; s[1] = h->blk[id].ncols; s[2] = int64_t(h->blk[id].col.size());
}
void fsigen_block_copy(const fsigen_handle* h, int id, int64_t* rowptr, int32_t* col, double* val) {
  const Block& b = h->blk[id];
  std::memcpy(rowptr, b.rowptr.data(), sizeof(int64_t) * (b.nrows + 1));
  std::memcpy(col, b.col.data(), sizeof(int32_t) * b.col.size());
  std::memcpy(val, b.val.data(), sizeof(double) * b.val.size());
}
// Newton right-hand side b = -R(U_bar) on the free dofs.
void fsigen_rhs(const fsigen_handle* h, double* b) {
  const Gen& g = h->g;
  for (int64_t i = 0; i < g.N; ++i) b[i] = -g.res[i];
}
// Node data: coords (nnodes*dim), lattice index (nnodes*dim), flags (nnodes),
// dof -> node (N), dof -> component (N).
void fsigen_nodes(const fsigen_handle* h, double* coords, int32_t* ijk, uint8_t* flags,
                  int32_t* dof_node, int8_t* dof_comp) {
  const Gen& g = h->g;
  for (int64_t n = 0; n < g.nnodes; ++n) {
    int I[3] = {0, 0, 0};
    g.node_ijk(n, I);
    for (int a = 0; a < g.D; ++a) {
      coords[n * g.D + a] = 0.5 * g.h[a] * I[a];
      ijk[n * g.D + a] = I[a];
    }
    flags[n] = g.node_flags[n];
    for (int c = 0; c < g.D; ++c) {
      if (g.vdof[n] >= 0) { dof_node[g.vdof[n] + c] = int32_t(n); dof_comp[g.vdof[n] + c] = int8_t(c); }
      if (g.udof[n] >= 0) { dof_node[g.udof[n] + c] = int32_t(n); dof_comp[g.udof[n] + c] = int8_t(c); }
    }
    if (g.pdof[n] >= 0) { dof_node[g.pdof[n]] = int32_t(n); dof_comp[g.pdof[n]] = int8_t(0); }
  }
}
void fsigen_jrange(const fsigen_handle* h, double* jr) { jr[0] = h->g.min_J; jr[1] = h->g.max_J; }
// Finite-element description of the workload, for assembling it elsewhere:
// first dof of each node's velocity / displacement and its pressure dof (-1:
// none, i.e. Dirichlet or absent), and the nodal fields at Q2 nodes
// (component-interleaved): the linearisation state v, u, p (also the Dirichlet
// data), the previous time level v_old, u_old, the advecting velocity w of the
// convective term and the displacement u_fz whose Jacobian scales the mesh
// stiffness.
void fsigen_fe_data(const fsigen_handle* h, int64_t* vdof, int64_t* udof, int64_t* pdof, double* v, double* u,
                    double* p, double* v_old, double* u_old, double* w, double* u_fz) {
  const Gen& g = h->g;
  const int64_t nd = g.nnodes * g.D;
  std::memcpy(vdof, g.vdof.data(), sizeof(int64_t) * g.nnodes);
  std::memcpy(udof, g.udof.data(), sizeof(int64_t) * g.nnodes);
  std::memcpy(pdof, g.pdof.data(), sizeof(int64_t) * g.nnodes);
  for (int64_t i = 0; i < nd; ++i) {
    v[i] = g.vbar[i];
    u[i] = g.ubar[i];
    v_old[i] = 0.9 * g.vbar[i];
    u_old[i] = 0.9 * g.ubar[i];
    w[i] = g.vbar[i];
    u_fz[i] = g.ubar[i];
  }
  std::memcpy(p, g.pbar.data(), sizeof(double) * g.nnodes);
}
void fsigen_free(fsigen_handle* h) { delete h; }

// Residual R(U_bar + eps * dU) on the free dofs, frozen fields held at U_bar
// (used by the finite-difference tests of the assembled Jacobian).
int fsigen_residual(const fsigen_cfg* cfg, const double* dU, double eps, double* R, int64_t n,
                    char* errbuf, int errlen) {
  Gen g;
  g.cfg = *cfg;
  if (!g.run(dU, eps, false)) {
    std::snprintf(errbuf, errlen, "%s", g.err.c_str());
    return -1;
  }
  if (n != g.N) {
    std::snprintf(errbuf, errlen, "length mismatch");
    return -2;
  }
  for (int64_t i = 0; i < g.N; ++i) R[i] = g.res[i];
  return 0;
}

}  // extern "C"
