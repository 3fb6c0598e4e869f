// Device kernels of the preconditioner setup: the sparse products C = A B of
// the AMG setup (prolongator smoothing, the Galerkin product, the products of
// the level sweeps), one wavefront per row of C, and the grouping of rows
// that share their columns (at the end of the file).
//
// Every row is formed as the host product forms it: the products a_ik b_kj
// are rounded and added in the order of k along row i of A, and entries that
// sum to exactly zero are dropped.  The device and host products are
// therefore bitwise equal, and the AMG hierarchy does not depend on where it
// was built.
//
// A row's distinct columns are collected in an LDS hash set (at most
// CAP of them), sorted, and then accumulated in LDS: within one k the
// columns of row k of B are distinct, so the lanes never add to the same
// entry at once, and successive k follow program order.  Rows with more
// distinct columns are reported (count -1) and left to the host.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fsi {

// Distinct columns of a row kept in LDS: 1024 (12 KiB per workgroup) for the
// first pass over all rows, 4096 (48 KiB) for the rows that overflow it.
constexpr int kSpgSmall = 1024;
constexpr int kSpgLarge = 4096;

__device__ inline uint64_t spg_lanes_below(int lane) {
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// kFill false: cnt[r] = nonzeros of row r of C (-1: more than CAP distinct
// columns).  kFill true: rows with cnt[r] >= 0 written at crp[r] (columns
// ascending).  One 64-lane workgroup per row: row rows[blockIdx.x], or
// blockIdx.x itself when rows is null.
template <int CAP, bool kFill>
__global__ __launch_bounds__(64) void spgemm_rows_kernel(const int32_t* __restrict__ rows,
                                                         const int64_t* __restrict__ arp,
                                                         const int32_t* __restrict__ aci,
                                                         const double* __restrict__ av,
                                                         const int64_t* __restrict__ brp,
                                                         const int32_t* __restrict__ bci,
                                                         const double* __restrict__ bv, int64_t* __restrict__ cnt,
                                                         const int64_t* __restrict__ crp, int32_t* __restrict__ cci,
                                                         double* __restrict__ cv) {
#pragma clang fp contract(off)
  constexpr int kHash = 2 * CAP;  // load factor at most 1/2 (+ one step's inserts)
  constexpr int kLogHash = CAP == 1024 ? 11 : CAP == 4096 ? 13 : -1;
  static_assert(kLogHash > 0, "CAP must be 1024 or 4096");
  __shared__ double s_val[CAP];   // hash slots (as int32) while collecting, then the row's values
  __shared__ int32_t s_key[CAP];  // the distinct columns, ascending
  __shared__ int s_n;
  __shared__ int s_over;
  int32_t* tab = reinterpret_cast<int32_t*>(s_val);
  const int lane = threadIdx.x;
  const int64_t r = rows ? int64_t(rows[blockIdx.x]) : int64_t(blockIdx.x);
  if (kFill && cnt[r] < 0) return;  // the whole workgroup leaves
  for (int s = lane; s < kHash; s += 64) tab[s] = -1;
  if (lane == 0) {
    s_n = 0;
    s_over = 0;
  }
  __syncthreads();
  const int64_t a0 = arp[r], a1 = arp[r + 1];
  // 1. the distinct columns of the row
  for (int64_t ka = a0; ka < a1; ++ka) {
    const int32_t k = aci[ka];
    const int64_t b0 = brp[k], b1 = brp[k + 1];
    for (int64_t kb = b0 + lane; kb < b1; kb += 64) {
      const int32_t j = bci[kb];
      uint32_t h = (uint32_t(j) * 2654435761u) >> (32 - kLogHash);
      int t = 0;
      for (; t < kHash; ++t) {
        const int32_t prev = atomicCAS(&tab[h], -1, j);
        if (prev == -1) {
          atomicAdd(&s_n, 1);
          break;
        }
        if (prev == j) break;
        h = (h + 1) & (kHash - 1);
      }
      if (t == kHash) atomicOr(&s_over, 1);  // table full: the row goes to the host
    }
    __syncthreads();
    if (s_over || s_n > CAP) break;  // uniform: shared values after the barrier
  }
  __syncthreads();
  if (s_over || s_n > CAP) {
    if (!kFill && lane == 0) cnt[r] = -1;
    return;
  }
  const int u = s_n;
  // 2. compact the set and sort it (bitonic, padded to a power of two)
  int base = 0;
  for (int s0 = 0; s0 < kHash; s0 += 64) {
    const int32_t v = tab[s0 + lane];
    const uint64_t m = __ballot(v >= 0);
    if (v >= 0) s_key[base + __popcll(m & spg_lanes_below(lane))] = v;
    base += __popcll(m);
  }
  int P = 1;
  while (P < u) P <<= 1;
  for (int i = u + lane; i < P; i += 64) s_key[i] = 0x7fffffff;
  __syncthreads();
  for (int kk = 2; kk <= P; kk <<= 1) {
    for (int jj = kk >> 1; jj > 0; jj >>= 1) {
      for (int i = lane; i < P; i += 64) {
        const int l = i ^ jj;
        if (l > i) {
          const int32_t x = s_key[i], y = s_key[l];
          if ((x > y) == ((i & kk) == 0)) {
            s_key[i] = y;
            s_key[l] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  // 3. the values, in the order of k
  for (int i = lane; i < u; i += 64) s_val[i] = 0.0;
  __syncthreads();
  for (int64_t ka = a0; ka < a1; ++ka) {
    const int32_t k = aci[ka];
    const double a = av[ka];
    const int64_t b0 = brp[k], b1 = brp[k + 1];
    for (int64_t kb = b0 + lane; kb < b1; kb += 64) {
      const int32_t j = bci[kb];
      int lo = 0, hi = u;  // first key >= j (present)
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (s_key[mid] < j) lo = mid + 1;
        else hi = mid;
      }
      const double p = a * bv[kb];
      s_val[lo] = s_val[lo] + p;
    }
    __syncthreads();
  }
  // 4. nonzeros: count, or write them in column order
  int64_t out = kFill ? crp[r] : 0;
  int nz = 0;
  for (int i0 = 0; i0 < u; i0 += 64) {
    const int i = i0 + lane;
    const double v = i < u ? s_val[i] : 0.0;
    const uint64_t m = __ballot(v != 0.0);
    if (kFill && v != 0.0) {
      const int64_t o = out + nz + __popcll(m & spg_lanes_below(lane));
      cci[o] = s_key[i];
      cv[o] = v;
    }
    nz += __popcll(m);
  }
  if (!kFill && lane == 0) cnt[r] = nz;
}

}  // namespace fsi

namespace fsi {

// Rows of a matrix in groups of G consecutive rows sharing one column list
// (the sorted union of the G rows' columns, G values per listed column, 0
// where a row has no entry), one thread per group: the G sorted lists are
// merged in column order.  kFill false: cnt[q] = entries of group q.  kFill
// true: group q written at grp[q] (columns gci, values gval, value times
// colscale[column] when colscale is not null, rounded to T).  Rows are rows
// r0 + q G + r of the device CSR rp, ci, v (rp[0] need not be 0).
template <int G, bool kFill, typename T>
__global__ __launch_bounds__(256) void group_merge_kernel(int64_t ngroups, const int64_t* __restrict__ rp,
                                                          const int32_t* __restrict__ ci,
                                                          const double* __restrict__ v,
                                                          const double* __restrict__ colscale,
                                                          int64_t* __restrict__ cnt, const int64_t* __restrict__ grp,
                                                          int32_t* __restrict__ gci, T* __restrict__ gval) {
#pragma clang fp contract(off)
  const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= ngroups) return;
  int64_t k[G], e[G];
  for (int r = 0; r < G; ++r) {
    k[r] = rp[q * G + r];
    e[r] = rp[q * G + r + 1];
  }
  int64_t n = 0;
  const int64_t out = kFill ? grp[q] : 0;
  while (true) {
    int32_t c = 0x7fffffff;
    for (int r = 0; r < G; ++r)
      if (k[r] < e[r]) c = min(c, ci[k[r]]);
    if (c == 0x7fffffff) break;
    if (kFill) gci[out + n] = c;
    for (int r = 0; r < G; ++r) {
      const bool has = k[r] < e[r] && ci[k[r]] == c;
      if (kFill) {
        double x = 0.0;
        if (has) x = colscale ? v[k[r]] * colscale[c] : v[k[r]];
        gval[(out + n) * G + r] = T(x);
      }
      if (has) ++k[r];
    }
    ++n;
  }
  if (!kFill) cnt[q] = n;
}

}  // namespace fsi

namespace fsi {

// y_i = dinv_i * sum_k a_ik x_k with the row summed in storage order by one
// thread (FMA contraction off): the host power iteration's product bit for
// bit, for the spectral estimate of the AMG setup.
__global__ __launch_bounds__(256) void rowseq_scaled_matvec_kernel(int64_t n, const int64_t* __restrict__ rp,
                                                                   const int32_t* __restrict__ ci,
                                                                   const double* __restrict__ v,
                                                                   const double* __restrict__ dinv,
                                                                   const double* __restrict__ x,
                                                                   double* __restrict__ y) {
#pragma clang fp contract(off)
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t k = rp[i]; k < rp[i + 1]; ++k) s += v[k] * x[ci[k]];
  y[i] = dinv[i] * s;
}

}  // namespace fsi
