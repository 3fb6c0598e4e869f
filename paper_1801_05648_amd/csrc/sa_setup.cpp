// Smoothed-aggregation AMG hierarchy construction.
//
// The paper approximates the inverses of its block preconditioner by
// algebraic multigrid (Sections 4.2-4.4) without fixing the method's
// parameters.  This file implements one deterministic smoothed-aggregation
// setup (strength of connection on node blocks, three-phase greedy
// aggregation in node order, aggregate-wise QR of the near-nullspace, one
// damped-Jacobi prolongator smoothing step on the filtered matrix, Galerkin
// coarse operators), whose every rule is spelled out at the point where it
// is applied below.
#include "sa_setup.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <thread>

namespace fsi {

namespace {

constexpr int kPowerIters = 30;
constexpr double kRankTol = 1e-10;
constexpr double kTieRel = 1e-8;
constexpr int64_t kMaxDenseCoarse = 6000;

double norm2(const std::vector<double>& x) {
  double s = 0.0;
  for (double v : x) s += v * v;
  return std::sqrt(s);
}

// rho(D^{-1} A): 30 normalised power steps from x_i = 1 + (i mod 7)/7, then
// the norm of one more application; `product` (if set) forms y = D^{-1} A x.
double spectral_radius(const HCsr& A, const std::vector<double>& dinv, const ScaledProduct& product) {
  const int64_t n = A.nrows;
  std::vector<double> x(n), y(n);
  auto apply = [&]() {
    if (product) {
      product(x.data(), y.data());
      return;
    }
    matvec(A, x.data(), y.data());
    for (int64_t i = 0; i < n; ++i) y[i] = dinv[i] * y[i];
  };
  for (int64_t i = 0; i < n; ++i) x[i] = 1.0 + double(i % 7) / 7.0;
  double nx = norm2(x);
  for (int64_t i = 0; i < n; ++i) x[i] /= nx;
  for (int it = 0; it < kPowerIters; ++it) {
    apply();
    double ny = norm2(y);
    for (int64_t i = 0; i < n; ++i) x[i] = y[i] / ny;
  }
  apply();
  return norm2(y);
}

struct Strength {
  // per node: strong neighbours (ascending) with their squared block norms
  std::vector<int64_t> ptr;
  std::vector<int32_t> nbr;
  std::vector<double> sval;
  std::vector<double> sdiag;
};

// Node-block squared Frobenius norms s_IJ accumulated over the rows of node I
// (ascending) and, within a row, in column storage order.  I != J is strong
// iff s_IJ > 0 and s_IJ^2 >= eps^4 (s_II s_JJ).
Strength strength(const HCsr& A, int b, double eps) {
  const int64_t nn = A.nrows / b;
  Strength S;
  S.sdiag.assign(nn, 0.0);
  // s_II first (every node's test needs the diagonals of its neighbours)
  parallel_for(nn, [&](int64_t I0, int64_t I1) {
    for (int64_t I = I0; I < I1; ++I) {
      double sII = 0.0;
      for (int c = 0; c < b; ++c) {
        const int64_t i = I * b + c;
        for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
          if (A.ci[k] / b == I) sII += A.v[k] * A.v[k];
      }
      S.sdiag[I] = sII;
    }
  });
  // then each node's s_IJ in a dense per-thread accumulator (first-touch
  // list, sorted by J), the strong ones kept; chunks of nodes on the host
  // threads, concatenated in node order
  const double e2 = eps * eps, e4 = e2 * e2;
  const int64_t nchunk = std::max<int64_t>(1, std::min<int64_t>(256, nn / 256));
  std::vector<std::vector<int32_t>> cn(nchunk);
  std::vector<std::vector<double>> cs(nchunk);
  std::vector<int64_t> len(nn, 0);
  parallel_for(nchunk, [&](int64_t cb, int64_t ce) {
    std::vector<double> acc(nn, 0.0);
    std::vector<int64_t> mark(nn, -1);
    std::vector<int32_t> js;
    for (int64_t ch = cb; ch < ce; ++ch) {
      const int64_t I0 = nn * ch / nchunk, I1 = nn * (ch + 1) / nchunk;
      for (int64_t I = I0; I < I1; ++I) {
        js.clear();
        for (int c = 0; c < b; ++c) {
          const int64_t i = I * b + c;
          for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            const int32_t J = A.ci[k] / b;
            if (mark[J] != I) {
              mark[J] = I;
              acc[J] = 0.0;
              js.push_back(J);
            }
            acc[J] += A.v[k] * A.v[k];
          }
        }
        std::sort(js.begin(), js.end());
        const size_t before = cn[ch].size();
        for (int32_t J : js) {
          const double sIJ = acc[J];
          if (J == I || !(sIJ > 0.0)) continue;
          if (sIJ * sIJ >= e4 * (S.sdiag[I] * S.sdiag[J])) {
            cn[ch].push_back(J);
            cs[ch].push_back(sIJ);
          }
        }
        len[I] = int64_t(cn[ch].size() - before);
      }
    }
  }, 2);
  S.ptr.assign(nn + 1, 0);
  for (int64_t I = 0; I < nn; ++I) S.ptr[I + 1] = S.ptr[I] + len[I];
  S.nbr.reserve(S.ptr[nn]);
  S.sval.reserve(S.ptr[nn]);
  for (int64_t ch = 0; ch < nchunk; ++ch) {
    S.nbr.insert(S.nbr.end(), cn[ch].begin(), cn[ch].end());
    S.sval.insert(S.sval.end(), cs[ch].begin(), cs[ch].end());
  }
  return S;
}

// Three-phase greedy aggregation in increasing node id.
int64_t aggregate(const Strength& S, int64_t nn, std::vector<int32_t>& agg) {
  agg.assign(nn, -1);
  int64_t nagg = 0;
  // phase 1: a node whose (non-empty) strong neighbourhood is entirely
  // unaggregated seeds an aggregate with that neighbourhood
  for (int64_t I = 0; I < nn; ++I) {
    if (agg[I] >= 0) continue;
    const int64_t lo = S.ptr[I], hi = S.ptr[I + 1];
    if (hi == lo) continue;
    bool free = true;
    for (int64_t k = lo; k < hi && free; ++k) free = agg[S.nbr[k]] < 0;
    if (!free) continue;
    agg[I] = int32_t(nagg);
    for (int64_t k = lo; k < hi; ++k) agg[S.nbr[k]] = int32_t(nagg);
    ++nagg;
  }
  // phase 2: remaining nodes join the aggregate of their strongest phase-1
  // neighbour (within a relative 1e-8 of the largest: smallest aggregate id)
  std::vector<int32_t> next(agg);
  for (int64_t I = 0; I < nn; ++I) {
    if (agg[I] >= 0) continue;
    double smax = -1.0;
    for (int64_t k = S.ptr[I]; k < S.ptr[I + 1]; ++k)
      if (agg[S.nbr[k]] >= 0) smax = std::max(smax, S.sval[k]);
    if (smax < 0.0) continue;
    const double thr = smax * (1.0 - kTieRel);
    int32_t best = INT32_MAX;
    for (int64_t k = S.ptr[I]; k < S.ptr[I + 1]; ++k)
      if (agg[S.nbr[k]] >= 0 && S.sval[k] >= thr) best = std::min(best, agg[S.nbr[k]]);
    next[I] = best;
  }
  agg.swap(next);
  // phase 3: leftovers seed aggregates with their unaggregated strong
  // neighbours; isolated nodes become singletons
  for (int64_t I = 0; I < nn; ++I) {
    if (agg[I] >= 0) continue;
    agg[I] = int32_t(nagg);
    for (int64_t k = S.ptr[I]; k < S.ptr[I + 1]; ++k)
      if (agg[S.nbr[k]] < 0) agg[S.nbr[k]] = int32_t(nagg);
    ++nagg;
  }
  return nagg;
}

// Aggregate-wise thin QR (modified Gram-Schmidt, columns in the order of B).
void tentative(const std::vector<int32_t>& agg, int64_t nagg, int b, const std::vector<double>& B, int k,
               int64_t n, HCsr& Pt, std::vector<double>& Bc) {
  std::vector<std::vector<int32_t>> members(nagg);
  for (int64_t I = 0; I < int64_t(agg.size()); ++I) members[agg[I]].push_back(int32_t(I));
  Bc.assign(size_t(nagg) * k * k, 0.0);
  // triplets by row: (row, col, val)
  std::vector<std::vector<std::pair<int32_t, double>>> rows(n);
  std::vector<double> Ba, Q, w;
  for (int64_t a = 0; a < nagg; ++a) {
    const auto& nodes = members[a];
    const int64_t m = int64_t(nodes.size()) * b;
    Ba.assign(size_t(m) * k, 0.0);
    std::vector<int64_t> dofs(m);
    for (size_t t = 0; t < nodes.size(); ++t)
      for (int c = 0; c < b; ++c) dofs[t * b + c] = int64_t(nodes[t]) * b + c;
    double fro2 = 0.0;
    for (int64_t r = 0; r < m; ++r)
      for (int j = 0; j < k; ++j) {
        double v = B[size_t(dofs[r]) * k + j];
        Ba[size_t(r) * k + j] = v;
      }
    for (int64_t r = 0; r < m; ++r)
      for (int j = 0; j < k; ++j) fro2 += Ba[size_t(r) * k + j] * Ba[size_t(r) * k + j];
    const double fro = std::sqrt(fro2);
    Q.assign(size_t(m) * k, 0.0);
    double* R = &Bc[size_t(a) * k * k];
    for (int j = 0; j < k; ++j) {
      w.resize(m);
      for (int64_t r = 0; r < m; ++r) w[r] = Ba[size_t(r) * k + j];
      for (int i = 0; i < j; ++i) {
        double dot = 0.0;
        for (int64_t r = 0; r < m; ++r) dot += Q[size_t(r) * k + i] * w[r];
        R[i * k + j] = dot;
        for (int64_t r = 0; r < m; ++r) w[r] = w[r] - dot * Q[size_t(r) * k + i];
      }
      double ww = 0.0;
      for (int64_t r = 0; r < m; ++r) ww += w[r] * w[r];
      const double rjj = std::sqrt(ww);
      if (rjj <= kRankTol * fro) continue;  // rank deficient: zero column
      R[j * k + j] = rjj;
      for (int64_t r = 0; r < m; ++r) {
        Q[size_t(r) * k + j] = w[r] / rjj;
        rows[dofs[r]].emplace_back(int32_t(a * k + j), Q[size_t(r) * k + j]);
      }
    }
  }
  Pt = HCsr();
  Pt.nrows = n;
  Pt.ncols = nagg * k;
  Pt.rp.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    std::sort(rows[i].begin(), rows[i].end());
    for (auto& e : rows[i]) {
      Pt.ci.push_back(e.first);
      Pt.v.push_back(e.second);
    }
    Pt.rp[i + 1] = int64_t(Pt.ci.size());
  }
}

// A^F: entries between weakly connected nodes are dropped and their sum (in
// storage order) is added to the diagonal entry of the row.
HCsr filtered(const HCsr& A, int b, const Strength& S) {
  HCsr F;
  F.nrows = A.nrows;
  F.ncols = A.ncols;
  F.rp.assign(A.nrows + 1, 0);
  auto keep = [&](int64_t i, int64_t k) {
    const int64_t I = i / b;
    const int32_t J = A.ci[k] / b;
    return J == I || std::binary_search(S.nbr.begin() + S.ptr[I], S.nbr.begin() + S.ptr[I + 1], J);
  };
  // rows are independent: count the kept entries, then fill, on the host
  // threads (each row formed as in a serial pass)
  parallel_for(A.nrows, [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i) {
      int64_t c = 0;
      for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) c += keep(i, k) ? 1 : 0;
      F.rp[i + 1] = c;
    }
  });
  for (int64_t i = 0; i < A.nrows; ++i) F.rp[i + 1] += F.rp[i];
  F.ci.resize(size_t(F.rp[A.nrows]));
  F.v.resize(size_t(F.rp[A.nrows]));
  parallel_for(A.nrows, [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i) {
      double lump = 0.0;
      int64_t dpos = -1, p = F.rp[i];
      for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
        if (!keep(i, k)) {
          lump += A.v[k];
          continue;
        }
        if (A.ci[k] == i) dpos = p;
        F.ci[size_t(p)] = A.ci[k];
        F.v[size_t(p)] = A.v[k];
        ++p;
      }
      if (dpos >= 0) F.v[size_t(dpos)] = F.v[size_t(dpos)] + lump;
    }
  });
  drop_zeros(F);
  return F;
}

}  // namespace

namespace {

// Barrier of a fixed team of host threads (spinning with yields: the team
// lives only for one dense inversion).
struct SpinBarrier {
  explicit SpinBarrier(int n) : n_(n) {}
  void wait() {
    const int g = gen_.load();
    if (count_.fetch_add(1) + 1 == n_) {
      count_.store(0);
      gen_.fetch_add(1);
    } else {
      while (gen_.load() == g) std::this_thread::yield();
    }
  }
  int n_;
  std::atomic<int> count_{0}, gen_{0};
};

}  // namespace

// LU with partial pivoting (largest magnitude, smallest row on ties), then
// the columns of the identity through the triangular factors.  The row
// updates of each elimination step and the column solves are shared among
// host threads; every entry goes through the same operations in the same
// order as in a single-threaded run, so the result does not depend on the
// thread count.
bool dense_inverse(std::vector<double> a, int64_t n, std::vector<double>& inv) {
  std::vector<int64_t> piv(n);
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const int nt = n < 256 ? 1 : int(std::min<unsigned>(16u, hw));
  SpinBarrier bar(nt);
  std::atomic<bool> singular{false};
  inv.assign(size_t(n) * n, 0.0);
  auto work = [&](int tid) {
    for (int64_t k = 0; k < n; ++k) {
      if (tid == 0) {
        int64_t p = k;
        double best = std::fabs(a[k * n + k]);
        for (int64_t r = k + 1; r < n; ++r)
          if (std::fabs(a[r * n + k]) > best) { best = std::fabs(a[r * n + k]); p = r; }
        if (a[p * n + k] == 0.0) singular.store(true);
        piv[k] = p;
        if (p != k)
          for (int64_t c = 0; c < n; ++c) std::swap(a[k * n + c], a[p * n + c]);
      }
      bar.wait();
      if (singular.load()) return;
      const double akk = a[k * n + k];
      for (int64_t r = k + 1 + tid; r < n; r += nt) {
        const double l = a[r * n + k] / akk;
        a[r * n + k] = l;
        if (l != 0.0)
          for (int64_t c = k + 1; c < n; ++c) a[r * n + c] -= l * a[k * n + c];
      }
      bar.wait();
    }
    // the columns of the inverse, in a contiguous range per thread, solved
    // together row by row: entry (i, col) takes its updates in the order of
    // c, as a column-by-column substitution would, but the updates of a row
    // run along the range (vectorisable)
    const int64_t c0 = n * tid / nt, c1 = n * (tid + 1) / nt, w = c1 - c0;
    if (w > 0) {
      std::vector<double> X(size_t(n) * w, 0.0);  // rows of the range, row-major
      for (int64_t col = c0; col < c1; ++col) {
        int64_t r = col;  // where the row swaps take the 1 of e_col
        for (int64_t k = 0; k < n; ++k) {
          if (piv[k] == k) continue;
          if (r == k) r = piv[k];
          else if (r == piv[k]) r = k;
        }
        X[size_t(r) * w + (col - c0)] = 1.0;
      }
      for (int64_t i = 0; i < n; ++i) {
        double* xi = X.data() + size_t(i) * w;
        for (int64_t c = 0; c < i; ++c) {
          const double l = a[i * n + c];
          const double* xc = X.data() + size_t(c) * w;
          for (int64_t j = 0; j < w; ++j) xi[j] -= l * xc[j];
        }
      }
      for (int64_t i = n - 1; i >= 0; --i) {
        double* xi = X.data() + size_t(i) * w;
        for (int64_t c = i + 1; c < n; ++c) {
          const double u = a[i * n + c];
          const double* xc = X.data() + size_t(c) * w;
          for (int64_t j = 0; j < w; ++j) xi[j] -= u * xc[j];
        }
        const double d = a[i * n + i];
        for (int64_t j = 0; j < w; ++j) xi[j] = xi[j] / d;
      }
      for (int64_t i = 0; i < n; ++i)
        std::copy(X.begin() + size_t(i) * w, X.begin() + size_t(i + 1) * w, inv.begin() + i * n + c0);
    }
  };
  std::vector<std::thread> team;
  for (int t = 1; t < nt; ++t) team.emplace_back(work, t);
  work(0);
  for (auto& t : team) t.join();
  return !singular.load();
}

std::string sa_finalize(SaHierarchy& H) {
  for (auto& L : H.levels) {
    std::vector<double> d = diagonal(L.A);
    L.dinv.resize(d.size());
    for (size_t i = 0; i < d.size(); ++i) {
      if (d[i] == 0.0) return "zero diagonal in an AMG level matrix";
      L.dinv[i] = 1.0 / d[i];
    }
  }
  const HCsr& C = H.levels.back().A;
  const int64_t n = C.nrows;
  if (n > kMaxDenseCoarse) return "AMG coarsening stalled: coarsest level too large for a dense solve";
  std::vector<double> dense(size_t(n) * n, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = C.rp[i]; k < C.rp[i + 1]; ++k) dense[size_t(i) * n + C.ci[k]] = C.v[k];
  if (!dense_inverse(dense, n, H.coarse_inv)) return "singular coarsest AMG matrix";
  return "";
}

std::string sa_setup(HCsr A, int block, const std::vector<double>& B0, int k0, const SaParams& prm,
                     SaHierarchy& H, const SpgemmFn& mul, const ScaledProductFactory& power) {
  auto product = [&](const HCsr& X, const HCsr& Y) { return mul ? mul(X, Y) : spgemm(X, Y); };
  H.levels.clear();
  std::vector<double> B = B0;
  int b = block, k = k0;
  double eps = prm.eps0;
  if (A.nrows % b != 0) return "matrix size is not a multiple of the node block size";
  while (true) {
    SaLevel L;
    L.A = std::move(A);  // the level keeps its matrix; Al refers to it below
    L.block = b;
    std::vector<double> d = diagonal(L.A);
    L.dinv.resize(d.size());
    for (size_t i = 0; i < d.size(); ++i) {
      if (d[i] == 0.0) return "zero diagonal in an AMG level matrix";
      L.dinv[i] = 1.0 / d[i];
    }
    H.levels.push_back(std::move(L));
    SaLevel& lev = H.levels.back();
    const HCsr& Al = lev.A;
    const int64_t n = Al.nrows;
    if (n <= prm.max_coarse || int(H.levels.size()) == prm.max_levels) break;
    const double rho = spectral_radius(Al, lev.dinv, power ? power(Al, lev.dinv) : ScaledProduct{});
    if (!(rho > 0.0) || !std::isfinite(rho)) return "non-finite spectral radius estimate";
    lev.omega = (4.0 / 3.0) / rho;
    Strength S = strength(Al, b, eps);
    std::vector<int32_t> agg;
    const int64_t nagg = aggregate(S, n / b, agg);
    HCsr Pt;
    std::vector<double> Bc;
    tentative(agg, nagg, b, B, k, n, Pt, Bc);
    HCsr AF = filtered(Al, b, S);
    std::vector<double> dF = diagonal(AF);
    std::vector<double> scale(n);
    for (int64_t i = 0; i < n; ++i) {
      // lumping weak entries can cancel a diagonal: the damped smoothing step
      // is then undefined
      if (dF[i] == 0.0) return "zero diagonal in the filtered AMG matrix";
      scale[i] = lev.omega / dF[i];
    }
    HCsr T = product(AF, Pt);
    scale_rows(T, scale);
    HCsr P = add(Pt, T, -1.0);
    drop_zeros(P);
    const int64_t nc = P.ncols;
    if (double(nc) > 0.8 * double(n) || nc == 0) {
      lev.omega = 0.0;
      break;
    }
    HCsr R = transpose(P);
    HCsr AP = product(Al, P);
    HCsr Ac = product(R, AP);
    drop_zeros(Ac);
    // a coarse dof with an empty row (rank-deficient aggregate column) gets 1
    bool any_empty = false;
    for (int64_t i = 0; i < Ac.nrows && !any_empty; ++i) any_empty = Ac.rp[i + 1] == Ac.rp[i];
    if (any_empty) {
      HCsr E;
      E.nrows = E.ncols = Ac.nrows;
      E.rp.assign(Ac.nrows + 1, 0);
      for (int64_t i = 0; i < Ac.nrows; ++i) {
        if (Ac.rp[i + 1] == Ac.rp[i]) {
          E.ci.push_back(int32_t(i));
          E.v.push_back(1.0);
        }
        E.rp[i + 1] = int64_t(E.ci.size());
      }
      Ac = add(Ac, E, 1.0);
    }
    lev.P = std::move(P);
    lev.R = std::move(R);
    lev.AP = std::move(AP);
    lev.agg = std::move(agg);
    A = std::move(Ac);
    B = std::move(Bc);
    b = k;
    eps = eps / 2.0;
  }
  const HCsr& C = H.levels.back().A;
  const int64_t n = C.nrows;
  if (n > kMaxDenseCoarse) return "AMG coarsening stalled: coarsest level too large for a dense solve";
  std::vector<double> dense(size_t(n) * n, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t kk = C.rp[i]; kk < C.rp[i + 1]; ++kk) dense[size_t(i) * n + C.ci[kk]] = C.v[kk];
  if (!dense_inverse(dense, n, H.coarse_inv)) return "singular coarsest AMG matrix";
  return "";
}

}  // namespace fsi
