// Smoothed-aggregation AMG setup (preconditioner build only): the steps on
// the host, the sparse products wherever the caller runs them.
#pragma once

#include <functional>
#include <string>
#include <vector>

#include "host_csr.hpp"

namespace fsi {

struct SaParams {
  double eps0 = 0.08;      // strength threshold on the finest level, halved per level
  int max_coarse = 500;    // coarsest level size bound
  int max_levels = 10;     // level bound (the coarsest included)
};

struct SaLevel {
  HCsr A, P, R;
  HCsr AP;  // A P of the Galerkin product, kept for the level sweeps (empty: not formed yet)
  int64_t ra_nnz = -1;  // nonzeros of R A once counted (-1: not yet)
  std::vector<double> dinv;
  double omega = 0.0;
  int block = 1;
  std::vector<int32_t> agg;  // aggregate of every node (levels that are not the coarsest)
};

struct SaHierarchy {
  std::vector<SaLevel> levels;
  std::vector<double> coarse_inv;  // dense inverse of the coarsest matrix, row-major
};

// Build the hierarchy of A with node block size `block` and near-nullspace B
// (row-major n x k).  Returns an empty string on success, else a message.
// The sparse products C = A B of the setup; a replacement of the host
// product must return spgemm's result bit for bit (empty: spgemm).
using SpgemmFn = std::function<HCsr(const HCsr&, const HCsr&)>;
// y = D^{-1} A x of the power iteration behind the Jacobi weight; a
// replacement must return the host product bit for bit (each row summed in
// storage order, then scaled).  The factory prepares it for one level
// matrix; an empty factory keeps the host product.
using ScaledProduct = std::function<void(const double* x, double* y)>;
using ScaledProductFactory = std::function<ScaledProduct(const HCsr& A, const std::vector<double>& dinv)>;
std::string sa_setup(HCsr A, int block, const std::vector<double>& B, int k, const SaParams& prm,
                     SaHierarchy& H, const SpgemmFn& mul = {}, const ScaledProductFactory& power = {});

// Dense inverse (LU with partial pivoting, smallest row index on ties) of the
// n x n row-major matrix a; returns false on a zero pivot.
bool dense_inverse(std::vector<double> a, int64_t n, std::vector<double>& inv);

// Finalise a caller-provided hierarchy (diagonal inverses, coarse inverse).
std::string sa_finalize(SaHierarchy& H);

}  // namespace fsi
