// Finite-element assembly of the ALE-FSI residual and Jacobian on the GPU.
//
// The residual is the semi-linear form A(U)(Phi) minus the linear form F(Phi)
// of Section 3 (the sum of the variational equations, equation fsi:all, with
// theta = 1) on a structured channel of Q2 (velocity, displacement) / Q1
// (pressure) quads or hexes; the Jacobian is its derivative A'(U), the matrix
// of the Newton step (Algorithm newton).  Per quadrature point the integrand
// maps the local field values q = (v, grad v, u, grad u, p) to outputs
// (f_v, g_v, f_u, g_u, f_p), and a test function phi of field X, component c
// receives f_X[c] phi + sum_k g_X[c][k] d_k phi.  The derivative d out / d q
// (the derivatives of F, J, F^{-1} of Section 3.3's derivative theorem enter
// through it) is evaluated by forward-mode dual numbers with one direction
// per thread: the thread of direction i seeds q_i.
//
// Launch: one workgroup of 256 threads per (cell, chunk of 32 local test
// rows), or per cell for the residual alone; the cells of one launch share
// one parity class per axis (2^d
// launches), so no two cells of a launch share a node and every row is
// written by one workgroup: plain read-add-write, deterministic.  A thread
// owns one test row t and the trial columns s = lane + 8 j of the cell matrix
// in registers across the quadrature loop.  The quadrature points go in
// batches of three: their rows of the basis table (the same for every cell,
// formed once by fe_basis_kernel) and the interpolated inputs into LDS, the
// integrand derivatives (75 (point, direction) pairs in 3D), then, point by
// point, DB[s][o] = sum over the inputs of trial s of d out_o / d q_i times
// its basis value, and the cell-matrix update.  About 60 KB of LDS in 3D, two
// workgroups per CU.  The cell matrix entries
// are added into the stored A_h (its row segments and row groups) at the
// position of (global row, global column), found by binary search in the
// row's sorted column list.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fsi {

struct FeParams {
  int D;
  int nc[3];       // cells per axis
  int NN[3];       // Q2 lattice nodes per axis (2 nc + 1)
  double h[3];     // cell size per axis
  int solid_lo[3], solid_hi[3];  // solid cells: solid_lo <= C < solid_hi on every axis
  double rho_f, nu_f, rho_s, mu_s, lambda_s, dtth;
  double theta, dt;  // one-step-theta scheme: dtth = dt theta; dt (1 - theta) at the previous level
  int newton_mesh;  // 1: the mesh stiffness 1/J uses the current J (else the given u_fz's)
};

struct FeNodes {   // per Q2 lattice node (row-major, axis 0 slowest)
  const int64_t* vdof;  // first velocity dof or -1
  const int64_t* udof;  // first displacement dof or -1
  const int64_t* pdof;  // pressure dof or -1
  const double* v;      // state fields (D per node; p: 1)
  const double* u;
  const double* p;
  const double* v_old;  // previous time level
  const double* u_old;
  const double* w;      // advecting velocity of the convective term
  const double* u_fz;   // displacement whose J scales the mesh stiffness
};

// Positions in the stored A_h: rows in up to four segments, each plain CSR
// (row pointers into ci/val, rows of grouped segments empty) or in groups of
// grp rows sharing one sorted column list (values grp per entry).
struct AhSlots {
  int nseg;
  int64_t row0[5];
  int grp[4];
  const int64_t* rp;
  const int32_t* ci;
  double* val;
  const int64_t* grp_rp[4];
  const int32_t* grp_ci[4];
  double* grp_val[4];
};

__device__ __forceinline__ double* ah_slot(const AhSlots& a, int64_t row, int32_t col) {
  int q = 0;
  while (q + 1 < a.nseg && row >= a.row0[q + 1]) ++q;
  const int32_t* ci;
  int64_t lo, end;
  double* base;
  int stride = 1, off = 0;
  if (a.grp[q] <= 1) {
    lo = a.rp[row];
    end = a.rp[row + 1];
    ci = a.ci;
    base = a.val;
  } else {
    const int g = a.grp[q];
    const int64_t lr = row - a.row0[q];
    const int64_t gi = lr / g;
    lo = a.grp_rp[q][gi];
    end = a.grp_rp[q][gi + 1];
    ci = a.grp_ci[q];
    base = a.grp_val[q];
    stride = g;
    off = int(lr - gi * g);
  }
  int64_t hi = end;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (ci[mid] < col) lo = mid + 1;
    else hi = mid;
  }
  if (lo < end && ci[lo] == col) return base + lo * stride + off;
  return nullptr;
}

// A value with one directional derivative.
struct Dn {
  double v, d;
};
__device__ __forceinline__ Dn dn(double c) { return Dn{c, 0.0}; }
__device__ __forceinline__ Dn operator+(Dn a, Dn b) { return Dn{a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dn operator-(Dn a, Dn b) { return Dn{a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dn operator*(Dn a, Dn b) { return Dn{a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dn operator*(double s, Dn a) { return Dn{s * a.v, s * a.d}; }
__device__ __forceinline__ Dn operator/(Dn a, Dn b) {
  const double r = 1.0 / b.v;
  return Dn{a.v * r, (a.d - a.v * r * b.d) * r};
}
__device__ __forceinline__ Dn operator+(Dn a, double s) { return Dn{a.v + s, a.d}; }
__device__ __forceinline__ Dn operator-(Dn a, double s) { return Dn{a.v - s, a.d}; }

template <int D> struct FeDims {
  static constexpr int NQ2 = D == 2 ? 9 : 27;   // Q2 nodes of a cell
  static constexpr int NQ1 = D == 2 ? 4 : 8;    // Q1 vertices
  static constexpr int NV = NQ2 * D;            // velocity (or displacement) dofs of a cell
  static constexpr int NLOC = 2 * NV + NQ1;     // local dofs: v | u | p
  static constexpr int QV = 0, QGV = D, QU = D + D * D, QGU = 2 * D + D * D, QP = 2 * D + 2 * D * D;
  static constexpr int NQ = QP + 1;             // integrand inputs (= outputs)
  static constexpr int NVOL = NQ2, NFACE = D == 2 ? 3 : 9;
  static constexpr int RT = 32, SL = 8;         // test rows per workgroup, trial lanes per row
  static constexpr int NCHUNK = (NLOC + RT - 1) / RT;
  static constexpr int NJ = (NLOC + SL - 1) / SL;
  // interpolated given fields: w, v_old, u_old, grad u_fz, grad v_old, grad u_old
  static constexpr int NFR = 3 * D + 3 * D * D;
  static constexpr int NPT = NVOL + NFACE;      // quadrature points (volume, then the outflow face)
  static constexpr int SH = NQ2 + NQ2 * D + NQ1 + 1;  // basis table row: N | grad N | M | weight
};

template <int D>
__device__ __forceinline__ Dn det_d(const Dn (&F)[D][D]) {
  if constexpr (D == 2) {
    return F[0][0] * F[1][1] - F[0][1] * F[1][0];
  } else {
    return F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) - F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
           F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
  }
}

// G = F^{-1} by cofactors.
template <int D>
__device__ __forceinline__ void inv_d(const Dn (&F)[D][D], Dn J, Dn (&G)[D][D]) {
  if constexpr (D == 2) {
    G[0][0] = F[1][1] / J;
    G[0][1] = dn(0.0) - F[0][1] / J;
    G[1][0] = dn(0.0) - F[1][0] / J;
    G[1][1] = F[0][0] / J;
  } else {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        // cofactor of F[j][i]: rows != j, columns != i
        const int r0 = j == 0 ? 1 : 0, r1 = j == 2 ? 1 : 2;
        const int c0 = i == 0 ? 1 : 0, c1 = i == 2 ? 1 : 2;
        const Dn m = F[r0][c0] * F[r1][c1] - F[r0][c1] * F[r1][c0];
        G[i][j] = ((i + j) % 2 == 0 ? m : dn(0.0) - m) / J;
      }
  }
}

// The integrand at one quadrature point.  kind: 0 fluid cell, 1 solid cell,
// 2 outflow face (normal e_0).  fr: w[D] | v_old[D] | u_old[D] | grad u_fz[D][D]
// | grad v_old[D][D] | grad u_old[D][D].  With theta < 1 the previous level's
// explicit share (Section 3.2) enters as constants: dt (1 - theta) times the
// convection (the previous velocity advecting itself), viscous stress, outflow
// correction and solid stress of v_old, u_old; the fluid mass term takes
// theta J + (1 - theta) J_old and the kinematics dt (theta v + (1 - theta) v_old).
template <int D>
__device__ __forceinline__ double det_plain(const double (&F)[D][D]) {
  if constexpr (D == 2) {
    return F[0][0] * F[1][1] - F[0][1] * F[1][0];
  } else {
    return F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) - F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
           F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
  }
}

// The previous level's F_old = I + grad u_old, J_old and F_old^{-1} (plain values).
template <int D>
__device__ __forceinline__ double previous_level(const double* fr, double (&Fo)[D][D], double (&Fio)[D][D]) {
  const double* gu = fr + 3 * D + 2 * D * D;
  for (int c = 0; c < D; ++c)
    for (int k = 0; k < D; ++k) Fo[c][k] = gu[c * D + k] + (c == k ? 1.0 : 0.0);
  const double Jo = det_plain<D>(Fo);
  if constexpr (D == 2) {
    Fio[0][0] = Fo[1][1] / Jo;
    Fio[0][1] = -Fo[0][1] / Jo;
    Fio[1][0] = -Fo[1][0] / Jo;
    Fio[1][1] = Fo[0][0] / Jo;
  } else {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const int r0 = j == 0 ? 1 : 0, r1 = j == 2 ? 1 : 2;
        const int c0 = i == 0 ? 1 : 0, c1 = i == 2 ? 1 : 2;
        const double m = Fo[r0][c0] * Fo[r1][c1] - Fo[r0][c1] * Fo[r1][c0];
        Fio[i][j] = ((i + j) % 2 == 0 ? m : -m) / Jo;
      }
  }
  return Jo;
}

template <int D>
__device__ void fe_integrand(int kind, const Dn* q, const double* fr, const FeParams& P, Dn* out) {
  using Q = FeDims<D>;
  for (int o = 0; o < Q::NQ; ++o) out[o] = dn(0.0);
  const bool explicit_share = P.theta < 1.0;
  const double dto = (1.0 - P.theta) * P.dt;
  const double* gvo = fr + 3 * D + D * D;  // grad v_old
  Dn F[D][D], Fi[D][D];
  for (int c = 0; c < D; ++c)
    for (int k = 0; k < D; ++k) F[c][k] = q[Q::QGU + c * D + k] + (c == k ? 1.0 : 0.0);
  const Dn J = det_d<D>(F);
  if (kind == 1) {
    // St. Venant-Kirchhoff: F S with S = 2 mu E + lambda tr(E) I
    Dn E[D][D];
    for (int c = 0; c < D; ++c)
      for (int k = 0; k < D; ++k) {
        Dn s = F[0][c] * F[0][k];
        for (int m = 1; m < D; ++m) s = s + F[m][c] * F[m][k];
        E[c][k] = 0.5 * (s - (c == k ? 1.0 : 0.0));
      }
    Dn tr = E[0][0];
    for (int c = 1; c < D; ++c) tr = tr + E[c][c];
    Dn S[D][D];
    for (int c = 0; c < D; ++c)
      for (int k = 0; k < D; ++k) {
        S[c][k] = (2.0 * P.mu_s) * E[c][k];
        if (c == k) S[c][k] = S[c][k] + P.lambda_s * tr;
      }
    for (int c = 0; c < D; ++c) {
      for (int k = 0; k < D; ++k) {
        Dn s = F[c][0] * S[0][k];
        for (int m = 1; m < D; ++m) s = s + F[c][m] * S[m][k];
        out[Q::QGV + c * D + k] = P.dtth * s;
      }
      out[Q::QV + c] = P.rho_s * (q[Q::QV + c] - fr[D + c]);
      out[Q::QU + c] = (q[Q::QU + c] - fr[2 * D + c]) - P.dtth * q[Q::QV + c];
    }
    if (explicit_share) {
      double Fo[D][D], Fio[D][D], Eo[D][D];
      (void)previous_level<D>(fr, Fo, Fio);
      double tro = 0.0;
      for (int c = 0; c < D; ++c)
        for (int k = 0; k < D; ++k) {
          double s = 0.0;
          for (int m = 0; m < D; ++m) s += Fo[m][c] * Fo[m][k];
          Eo[c][k] = 0.5 * (s - (c == k ? 1.0 : 0.0));
        }
      for (int c = 0; c < D; ++c) tro += Eo[c][c];
      for (int c = 0; c < D; ++c) {
        for (int k = 0; k < D; ++k) {
          double s = 0.0;
          for (int m = 0; m < D; ++m) s += Fo[c][m] * ((2.0 * P.mu_s) * Eo[m][k] + (m == k ? P.lambda_s * tro : 0.0));
          out[Q::QGV + c * D + k] = out[Q::QGV + c * D + k] + dto * s;
        }
        out[Q::QU + c] = out[Q::QU + c] - dto * fr[D + c];
      }
    }
    return;
  }
  inv_d<D>(F, J, Fi);
  if (kind == 2) {
    // -dt theta rho nu J F^{-T} grad v^T F^{-T} e_0
    Dn a[D], b[D];
    for (int m = 0; m < D; ++m) a[m] = Fi[0][m];
    for (int k = 0; k < D; ++k) {
      Dn s = q[Q::QGV + 0 * D + k] * a[0];
      for (int m = 1; m < D; ++m) s = s + q[Q::QGV + m * D + k] * a[m];
      b[k] = s;
    }
    const double coef = -P.dtth * P.rho_f * P.nu_f;
    for (int c = 0; c < D; ++c) {
      Dn s = Fi[0][c] * b[0];
      for (int k = 1; k < D; ++k) s = s + Fi[k][c] * b[k];
      out[Q::QV + c] = coef * (J * s);
    }
    if (explicit_share) {
      double Fo[D][D], Fio[D][D], bo[D];
      const double Jo = previous_level<D>(fr, Fo, Fio);
      for (int k = 0; k < D; ++k) {
        double s = 0.0;
        for (int m = 0; m < D; ++m) s += gvo[m * D + k] * Fio[0][m];
        bo[k] = s;
      }
      for (int c = 0; c < D; ++c) {
        double s = 0.0;
        for (int k = 0; k < D; ++k) s += Fio[k][c] * bo[k];
        out[Q::QV + c] = out[Q::QV + c] - (dto * P.rho_f * P.nu_f) * (Jo * s);
      }
    }
    return;
  }
  // fluid: ALE momentum, incompressibility, mesh motion
  Dn GF[D][D];  // grad v F^{-1}
  for (int c = 0; c < D; ++c)
    for (int k = 0; k < D; ++k) {
      Dn s = q[Q::QGV + c * D + 0] * Fi[0][k];
      for (int m = 1; m < D; ++m) s = s + q[Q::QGV + c * D + m] * Fi[m][k];
      GF[c][k] = s;
    }
  const double rho = P.rho_f, mu = P.rho_f * P.nu_f;
  // previous level (theta < 1): F_old, J_old, grad v_old F_old^{-1}
  double Jo = 1.0, Fo[D][D], Fio[D][D], GFo[D][D];
  Dn Jmass = J;  // the mass term's J: theta J + (1 - theta) J_old
  if (explicit_share) {
    Jo = previous_level<D>(fr, Fo, Fio);
    for (int c = 0; c < D; ++c)
      for (int k = 0; k < D; ++k) {
        double s = 0.0;
        for (int m = 0; m < D; ++m) s += gvo[c * D + m] * Fio[m][k];
        GFo[c][k] = s;
      }
    Jmass = P.theta * J + dn((1.0 - P.theta) * Jo);
  }
  for (int c = 0; c < D; ++c) {
    Dn adv = GF[c][0] * dn(fr[0]);
    Dn mv = GF[c][0] * (q[Q::QU + 0] - fr[2 * D + 0]);
    for (int k = 1; k < D; ++k) {
      adv = adv + GF[c][k] * dn(fr[k]);
      mv = mv + GF[c][k] * (q[Q::QU + k] - fr[2 * D + k]);
    }
    out[Q::QV + c] = rho * (Jmass * (q[Q::QV + c] - fr[D + c])) + (P.dtth * rho) * (J * adv) - rho * (J * mv);
    for (int k = 0; k < D; ++k) {
      Dn s = (GF[c][0] + GF[0][c]) * Fi[k][0];
      for (int m = 1; m < D; ++m) s = s + (GF[c][m] + GF[m][c]) * Fi[k][m];
      out[Q::QGV + c * D + k] = (P.dtth * mu) * (J * s) - J * (q[Q::QP] * Fi[k][c]);
    }
    if (explicit_share) {
      // dt (1 - theta) times the previous level's convection (v_old advecting
      // itself) and viscous stress
      double cv = 0.0;
      for (int k = 0; k < D; ++k) cv += GFo[c][k] * fr[D + k];
      out[Q::QV + c] = out[Q::QV + c] + dto * rho * (Jo * cv);
      for (int k = 0; k < D; ++k) {
        double s = 0.0;
        for (int m = 0; m < D; ++m) s += (GFo[c][m] + GFo[m][c]) * Fio[k][m];
        out[Q::QGV + c * D + k] = out[Q::QGV + c * D + k] + (dto * mu) * (Jo * s);
      }
    }
  }
  Dn tr = GF[0][0];
  for (int c = 1; c < D; ++c) tr = tr + GF[c][c];
  out[Q::QP] = J * tr;
  Dn Jm;
  if (P.newton_mesh) {
    Jm = J;
  } else {
    Dn Fz[D][D];
    for (int c = 0; c < D; ++c)
      for (int k = 0; k < D; ++k) Fz[c][k] = dn(fr[3 * D + c * D + k] + (c == k ? 1.0 : 0.0));
    Jm = det_d<D>(Fz);
  }
  for (int c = 0; c < D; ++c)
    for (int k = 0; k < D; ++k) out[Q::QGU + c * D + k] = q[Q::QGU + c * D + k] / Jm;
}

__device__ __forceinline__ void q2_basis(double x, double* n, double* dn1) {
  n[0] = (2.0 * x - 1.0) * (x - 1.0);
  n[1] = 4.0 * x * (1.0 - x);
  n[2] = x * (2.0 * x - 1.0);
  dn1[0] = 4.0 * x - 3.0;
  dn1[1] = 4.0 - 8.0 * x;
  dn1[2] = 4.0 * x - 1.0;
}

// The basis table, the same for every cell of the uniform grid: per
// quadrature point (3^d volume points, then the 3^{d-1} points of the face
// x_0 = 1) the Q2 values and physical gradients, the Q1 values and the
// weight (cell volume or face area included).  One thread per (point, basis
// function); formed once per fsi_fe_setup.
template <int D>
__global__ __launch_bounds__(256) void fe_basis_kernel(FeParams P, double* __restrict__ tab) {
  using Q = FeDims<D>;
  constexpr int NQ2 = Q::NQ2, NQ1 = Q::NQ1, SH = Q::SH;
  const int job = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (job >= Q::NPT * (NQ2 + NQ1)) return;
  const double gx[3] = {0.5 - 0.38729833462074168852, 0.5, 0.5 + 0.38729833462074168852};
  const double gw[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
  const int ip = job / (NQ2 + NQ1), l = job % (NQ2 + NQ1);
  double xi[3] = {0.0, 0.0, 0.0}, w = 1.0;
  if (ip < Q::NVOL) {
    int r = ip;
    for (int a = 0; a < D; ++a) { xi[a] = gx[r % 3]; w *= gw[r % 3] * P.h[a]; r /= 3; }
  } else {
    int r = ip - Q::NVOL;
    xi[0] = 1.0;
    for (int a = 1; a < D; ++a) { xi[a] = gx[r % 3]; w *= gw[r % 3] * P.h[a]; r /= 3; }
  }
  double* row = tab + ip * SH;
  if (l < NQ2) {
    double n1[3][3], d1[3][3];
    for (int a = 0; a < D; ++a) q2_basis(xi[a], n1[a], d1[a]);
    int ia[3], r = l;
    for (int a = 0; a < D; ++a) { ia[a] = r % 3; r /= 3; }
    double prod = 1.0;
    for (int a = 0; a < D; ++a) prod *= n1[a][ia[a]];
    row[l] = prod;
    for (int k = 0; k < D; ++k) {
      double g = d1[k][ia[k]] / P.h[k];
      for (int a = 0; a < D; ++a)
        if (a != k) g *= n1[a][ia[a]];
      row[NQ2 + l * D + k] = g;
    }
    if (l == 0) row[SH - 1] = w;
  } else {
    int r = l - NQ2;
    double prod = 1.0;
    for (int a = 0; a < D; ++a) { prod *= (r % 2) ? xi[a] : 1.0 - xi[a]; r /= 2; }
    row[NQ2 + NQ2 * D + (l - NQ2)] = prod;
  }
}

// Launch modes of fe_assemble_kernel: the residual R(U) of the cells' tested
// rows; the integrand values and derivatives d out / d q at every quadrature
// point of every cell into a buffer (FE_POINTS); the cell matrices from that
// buffer, added into A_h (FE_CONTRACT).  Each mode is its own instance, so the
// contraction carries none of the integrand's registers.
enum { FE_RESIDUAL = 0, FE_POINTS = 1, FE_CONTRACT = 2 };

// flag bits: 1 J <= 0 (current or mesh-stiffness), 2 a cell entry outside
// the stored pattern, 4 a non-finite residual or matrix value.
// pts: FE_POINTS writes, FE_CONTRACT reads, per cell of the launch (blockIdx.x)
// and point, d out / d q (NQ x NQ, o-major) then the values (NQ).
template <int D, int MODE>
__global__ __launch_bounds__(256) void fe_assemble_kernel(FeParams P, FeNodes nd, const double* __restrict__ basis,
                                                          const double* __restrict__ dU, int color,
                                                          double* __restrict__ R, double* __restrict__ pts,
                                                          AhSlots ah, int* flag) {
  using Q = FeDims<D>;
  constexpr int NQ2 = Q::NQ2, NQ1 = Q::NQ1, NV = Q::NV, NLOC = Q::NLOC, NQ = Q::NQ;
  constexpr int NIN = NQ + Q::NFR, SH = Q::SH, GS = NQ * NQ + NQ;
  constexpr int QB = MODE == FE_CONTRACT ? 1 : 9;  // points per batch
  constexpr bool kFields = MODE != FE_CONTRACT, kRows = MODE != FE_POINTS;
  __shared__ double s_f[kFields ? 7 * NV + NQ1 : 1];  // v | u | w | v_old | u_old | u_fz (node-major, comp) | p
  __shared__ int64_t s_gd[kRows ? NLOC : 1];
  __shared__ unsigned char s_ton[kRows ? NLOC : 1];
  __shared__ double s_sh[QB * SH];                      // basis table rows of the batch's points
  __shared__ double s_q[kFields ? QB * NIN : 1];        // inputs q and given fields at the batch's points
  __shared__ double s_ov[MODE == FE_RESIDUAL ? QB * NQ : 1];
  __shared__ double s_Dm[MODE == FE_CONTRACT ? NQ * NQ : 1];  // s_Dm[o * NQ + i] = d out_o / d q_i
  __shared__ double s_DB[MODE == FE_CONTRACT ? NLOC * NQ : 1];
  __shared__ int s_olist[NQ];  // FE_CONTRACT: the outputs this chunk's test rows use
  __shared__ int s_nout;
  __shared__ int s_cellflag;
  const int tid = threadIdx.x;
  // the cell of this workgroup within its parity class
  int C[3] = {0, 0, 0};
  {
    int64_t r = blockIdx.x;
    for (int a = D - 1; a >= 0; --a) {
      const int bit = (color >> a) & 1;
      const int m = (P.nc[a] - bit + 1) / 2;
      C[a] = 2 * int(r % m) + bit;
      r /= m;
    }
  }
  bool solid = true;
  for (int a = 0; a < D; ++a) solid = solid && C[a] >= P.solid_lo[a] && C[a] < P.solid_hi[a];
  const bool outflow = !solid && C[0] == P.nc[0] - 1;
  auto node_of = [&](const int* off) {
    int64_t id = 0;
    for (int a = 0; a < D; ++a) id = id * P.NN[a] + (2 * C[a] + off[a]);
    return id;
  };
  // gather the cell's fields, dof numbers and test flags
  if (tid == 0) s_cellflag = 0;
  for (int l = tid; l < NQ2; l += blockDim.x) {
    int off[3], r = l;
    for (int a = 0; a < D; ++a) { off[a] = r % 3; r /= 3; }
    const int64_t n = node_of(off);
    const int64_t vd = nd.vdof[n], ud = nd.udof[n];
    // is the node in a solid cell: on every axis a neighbouring cell lies in the box
    bool in_solid = true;
    for (int a = 0; a < D; ++a) {
      const int I = 2 * C[a] + off[a];
      int lo = I % 2 ? (I - 1) / 2 : I / 2 - 1, hi = I % 2 ? (I - 1) / 2 : I / 2;
      lo = lo < 0 ? 0 : lo;
      hi = hi > P.nc[a] - 1 ? P.nc[a] - 1 : hi;
      in_solid = in_solid && hi >= P.solid_lo[a] && lo < P.solid_hi[a];
    }
    for (int c = 0; c < D; ++c) {
      const int k = l * D + c;
      if constexpr (kFields) {
        s_f[k] = nd.v[n * D + c] + (vd >= 0 && dU ? dU[vd + c] : 0.0);
        s_f[NV + k] = nd.u[n * D + c] + (ud >= 0 && dU ? dU[ud + c] : 0.0);
        s_f[2 * NV + k] = nd.w[n * D + c];
        s_f[3 * NV + k] = nd.v_old[n * D + c];
        s_f[4 * NV + k] = nd.u_old[n * D + c];
        s_f[5 * NV + k] = nd.u_fz[n * D + c];
      }
      if constexpr (kRows) {
        s_gd[k] = vd >= 0 ? vd + c : -1;
        s_gd[NV + k] = ud >= 0 ? ud + c : -1;
        s_ton[k] = vd >= 0;
        s_ton[NV + k] = ud >= 0 && (solid || !in_solid);
      }
    }
  }
  for (int l = tid; l < NQ1; l += blockDim.x) {
    int off[3], r = l;
    for (int a = 0; a < D; ++a) { off[a] = 2 * (r % 2); r /= 2; }
    const int64_t n = node_of(off);
    const int64_t pd = solid ? -1 : nd.pdof[n];
    if constexpr (kFields) s_f[6 * NV + l] = nd.p[n] + (pd >= 0 && dU ? dU[pd] : 0.0);
    if constexpr (kRows) {
      s_gd[2 * NV + l] = pd;
      s_ton[2 * NV + l] = pd >= 0;
    }
  }
  __syncthreads();
  // residual: one thread per local row; contraction: 32 test rows per
  // workgroup (blockIdx.y), 8 threads per row
  const int tr = tid / Q::SL, sl = MODE == FE_CONTRACT ? tid % Q::SL : 0;
  const int t = MODE == FE_CONTRACT ? int(blockIdx.y) * Q::RT + tr : tid;
  bool row_on = false;
  if constexpr (kRows) row_on = t < NLOC && s_ton[t] && s_gd[t] >= 0;
  if constexpr (MODE == FE_CONTRACT) {
    // a test row of field X, component c reads f_X[c] and g_X[c][k] only
    if (tid == 0) {
      bool need[NQ];
      for (int o = 0; o < NQ; ++o) need[o] = false;
      const int r0 = int(blockIdx.y) * Q::RT;
      for (int r = r0; r < r0 + Q::RT && r < NLOC; ++r) {
        if (r < 2 * NV) {
          const int c = (r % NV) % D;
          const int fo = r < NV ? Q::QV : Q::QU, go = r < NV ? Q::QGV : Q::QGU;
          need[fo + c] = true;
          for (int k = 0; k < D; ++k) need[go + c * D + k] = true;
        } else {
          need[Q::QP] = true;
        }
      }
      int n = 0;
      for (int o = 0; o < NQ; ++o)
        if (need[o]) s_olist[n++] = o;
      s_nout = n;
    }
    __syncthreads();
  }
  double acc[MODE == FE_CONTRACT ? Q::NJ : 1];
#pragma unroll
  for (int j = 0; j < (MODE == FE_CONTRACT ? Q::NJ : 1); ++j) acc[j] = 0.0;
  double res = 0.0;
  const int npts = Q::NVOL + (outflow ? Q::NFACE : 0);
  double* cell_pts = pts ? pts + int64_t(blockIdx.x) * Q::NPT * GS : nullptr;
  for (int b0 = 0; b0 < npts; b0 += QB) {
    const int nb = npts - b0 < QB ? npts - b0 : QB;
    for (int i = tid; i < nb * SH; i += blockDim.x) s_sh[i] = basis[b0 * SH + i];
    if constexpr (MODE == FE_CONTRACT)
      for (int i = tid; i < NQ * NQ; i += blockDim.x) s_Dm[i] = cell_pts[b0 * GS + i];
    __syncthreads();
    if constexpr (kFields) {
      // interpolated inputs q and given fields at the batch's points
      for (int job = tid; job < nb * NIN; job += blockDim.x) {
        const int jb = job / NIN, i = job % NIN;
        const double* N = s_sh + jb * SH;
        const double* dN = N + NQ2;
        const double* M = dN + NQ2 * D;
        double s = 0.0;
        if (i < NQ) {
          if (i == Q::QP) {
            for (int l = 0; l < NQ1; ++l) s += M[l] * s_f[6 * NV + l];
          } else {
            const bool vel = i < Q::QU;
            const int j = vel ? i : i - Q::QU;  // 0..D-1 value, D.. gradient
            const double* f = s_f + (vel ? 0 : NV);
            if (j < D) {
              for (int l = 0; l < NQ2; ++l) s += N[l] * f[l * D + j];
            } else {
              const int c = (j - D) / D, k = (j - D) % D;
              for (int l = 0; l < NQ2; ++l) s += dN[l * D + k] * f[l * D + c];
            }
          }
        } else {
          const int j = i - NQ;
          if (j < 3 * D) {  // w, v_old, u_old
            const double* f = s_f + (2 + j / D) * NV;
            const int c = j % D;
            for (int l = 0; l < NQ2; ++l) s += N[l] * f[l * D + c];
          } else {          // grad u_fz, grad v_old, grad u_old
            const int g = (j - 3 * D) / (D * D), r = (j - 3 * D) % (D * D);
            const int c = r / D, k = r % D;
            const double* f = s_f + (g == 0 ? 5 : g == 1 ? 3 : 4) * NV;
            for (int l = 0; l < NQ2; ++l) s += dN[l * D + k] * f[l * D + c];
          }
        }
        s_q[jb * NIN + i] = s;
      }
      __syncthreads();
      // the integrand at the batch's points: d out / d q_i, one (point,
      // direction) per thread, or the values alone for the residual
      constexpr int ndir = MODE == FE_POINTS ? NQ : 1;
      for (int job = tid; job < nb * ndir; job += blockDim.x) {
        const int jb = job / ndir, dir = job % ndir, ip = b0 + jb;
        const double* qv = s_q + jb * NIN;
        Dn qd[NQ], out[NQ];
        for (int i = 0; i < NQ; ++i) qd[i] = Dn{qv[i], (MODE == FE_POINTS && i == dir) ? 1.0 : 0.0};
        const bool face = ip >= Q::NVOL;
        fe_integrand<D>(face ? 2 : (solid ? 1 : 0), qd, qv + NQ, P, out);
        if constexpr (MODE == FE_POINTS)
          for (int o = 0; o < NQ; ++o) cell_pts[ip * GS + o * NQ + dir] = out[o].d;
        if (dir == 0) {
          if constexpr (MODE == FE_POINTS) {
            for (int o = 0; o < NQ; ++o) {
              cell_pts[ip * GS + NQ * NQ + o] = out[o].v;
              if (!isfinite(out[o].v)) atomicOr(&s_cellflag, 4);
            }
          } else {
            for (int o = 0; o < NQ; ++o) s_ov[jb * NQ + o] = out[o].v;
          }
          // J of the current state and of the mesh-stiffness field must stay positive
          if (!solid && !face) {
            double Fv[D][D], Fz[D][D];
            for (int c = 0; c < D; ++c)
              for (int k = 0; k < D; ++k) {
                Fv[c][k] = qv[Q::QGU + c * D + k] + (c == k ? 1.0 : 0.0);
                Fz[c][k] = qv[NQ + 3 * D + c * D + k] + (c == k ? 1.0 : 0.0);
              }
            if (!(det_plain<D>(Fv) > 0.0) || !(det_plain<D>(Fz) > 0.0)) atomicOr(&s_cellflag, 1);
          }
        }
      }
      __syncthreads();
    }
    if constexpr (MODE == FE_RESIDUAL) {
      for (int jb = 0; jb < nb; ++jb) {
        const double* N = s_sh + jb * SH;
        const double* dN = N + NQ2;
        const double* M = dN + NQ2 * D;
        const double w = M[NQ1];
        const double* ov = s_ov + jb * NQ;
        if (row_on) {
          if (t < 2 * NV) {
            const int fo = t < NV ? Q::QV : Q::QU, go = t < NV ? Q::QGV : Q::QGU;
            const int l = (t % NV) / D, c = (t % NV) % D;
            double s = ov[fo + c] * N[l];
            for (int k = 0; k < D; ++k) s += ov[go + c * D + k] * dN[l * D + k];
            res += w * s;
          } else {
            res += w * ov[Q::QP] * M[t - 2 * NV];
          }
        }
      }
      __syncthreads();  // the next batch overwrites the tables
    }
    if constexpr (MODE == FE_CONTRACT) {
      const double* N = s_sh;
      const double* dN = N + NQ2;
      const double* M = dN + NQ2 * D;
      const double w = M[NQ1];
      const double* Dm = s_Dm;
      const int nout = s_nout;
      for (int idx = tid; idx < NLOC * nout; idx += blockDim.x) {
        const int s = idx / nout, o = s_olist[idx % nout];
        double val = 0.0;
        if (s_gd[s] >= 0) {
          if (s < 2 * NV) {
            const int fi = s < NV ? Q::QV : Q::QU, gi = s < NV ? Q::QGV : Q::QGU;
            const int l = (s % NV) / D, e = (s % NV) % D;
            val = Dm[o * NQ + fi + e] * N[l];
            for (int k = 0; k < D; ++k) val += Dm[o * NQ + gi + e * D + k] * dN[l * D + k];
          } else {
            val = Dm[o * NQ + Q::QP] * M[s - 2 * NV];
          }
        }
        s_DB[s * NQ + o] = val;
      }
      __syncthreads();
      if (row_on) {
        if (t < 2 * NV) {
          const int fo = t < NV ? Q::QV : Q::QU, go = t < NV ? Q::QGV : Q::QGU;
          const int l = (t % NV) / D, c = (t % NV) % D;
          double tw[4];
          tw[0] = w * N[l];
          for (int k = 0; k < D; ++k) tw[1 + k] = w * dN[l * D + k];
#pragma unroll
          for (int j = 0; j < Q::NJ; ++j) {  // unrolled: acc stays in registers
            const int s = sl + Q::SL * j;
            if (s < NLOC) {
              const double* db = s_DB + s * NQ;
              double v = tw[0] * db[fo + c];
              for (int k = 0; k < D; ++k) v += tw[1 + k] * db[go + c * D + k];
              acc[j] += v;
            }
          }
        } else {
          const double tw = w * M[t - 2 * NV];
#pragma unroll
          for (int j = 0; j < Q::NJ; ++j) {
            const int s = sl + Q::SL * j;
            if (s < NLOC) acc[j] += tw * s_DB[s * NQ + Q::QP];
          }
        }
      }
      __syncthreads();  // the next point overwrites the tables
    }
    if constexpr (MODE == FE_POINTS) __syncthreads();
  }
  int bad = 0;
  if (row_on) {
    const int64_t grow = s_gd[t];
    if constexpr (MODE == FE_RESIDUAL) {
      if (!isfinite(res)) bad |= 4;
      R[grow] += res;
    }
    if constexpr (MODE == FE_CONTRACT) {
#pragma unroll
      for (int j = 0; j < Q::NJ; ++j) {
        const int s = sl + Q::SL * j;
        const int64_t gcol = s < NLOC ? s_gd[s] : -1;
        if (gcol >= 0) {
          const double v = acc[j];
          if (!isfinite(v)) bad |= 4;
          double* slot = ah_slot(ah, grow, int32_t(gcol));
          if (slot) *slot += v;
          else if (v != 0.0) bad |= 2;
        }
      }
    }
  }
  if (tid == 0) bad |= s_cellflag;
  if (bad) atomicOr(flag, bad);
}

// Values of one block's entries read back from the stored A_h (block rows and
// columns offset by row_off / col_off); one thread per row.
__global__ __launch_bounds__(256) void ah_block_gather_kernel(int64_t nrows, const int64_t* __restrict__ rp,
                                                              const int32_t* __restrict__ ci, int64_t row_off,
                                                              int64_t col_off, AhSlots ah, double* __restrict__ out,
                                                              int* flag) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
    const double* slot = ah_slot(ah, row_off + i, int32_t(col_off + ci[k]));
    if (!slot) {
      atomicOr(flag, 2);
      out[k] = 0.0;
    } else {
      out[k] = *slot;
    }
  }
}

// Block-wise max |x_i| (NaN counts as +inf).
__global__ __launch_bounds__(256) void absmax_kernel(int64_t n, const double* __restrict__ x, double* __restrict__ part) {
  __shared__ double red[256];
  double m = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    const double a = fabs(x[i]);
    m = (a != a) ? INFINITY : (a > m ? a : m);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// End of a time step: the state U = fields + dU becomes the fields of the next
// step and its previous level (v_old, u_old), the advecting velocity w and
// the mesh-stiffness displacement u_fz; constrained dofs keep their values.
__global__ __launch_bounds__(256) void fe_advance_kernel(int64_t nn, int D, const int64_t* __restrict__ vdof,
                                                         const int64_t* __restrict__ udof,
                                                         const int64_t* __restrict__ pdof, double* v, double* u,
                                                         double* p, double* v_old, double* u_old, double* w,
                                                         double* u_fz, const double* __restrict__ dU) {
  const int64_t n = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (n >= nn) return;
  for (int c = 0; c < D; ++c) {
    const int64_t k = n * D + c;
    const double vn = v[k] + (vdof[n] >= 0 ? dU[vdof[n] + c] : 0.0);
    const double un = u[k] + (udof[n] >= 0 ? dU[udof[n] + c] : 0.0);
    v[k] = vn;
    v_old[k] = vn;
    w[k] = vn;
    u[k] = un;
    u_old[k] = un;
    u_fz[k] = un;
  }
  if (pdof[n] >= 0) p[n] = p[n] + dU[pdof[n]];
}

// y -= x (the Newton update U_{k+1} = U_k + delta with delta = -x).
__global__ __launch_bounds__(256) void sub_inplace_kernel(int64_t n, const double* __restrict__ x, double* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] -= x[i];
}

}  // namespace fsi
