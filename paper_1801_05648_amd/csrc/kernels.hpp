// CDNA4 (gfx950) device kernels of the FSI Jacobian solve.
//
// Everything on the solve path is a stream over HBM: CSR products with
// 0.17 flop/byte, vector updates and Gram-Schmidt dots.  The kernels are
// therefore built around coalesced streaming of the matrix arrays:
//   * CSR products: a group of G lanes (G = 4..64, a power of two chosen from
//     the average row length) walks one row, each lane striding by G through
//     the column/value arrays so that one 64-wide wavefront issues 64
//     consecutive entries per step; the group is reduced with cross-lane
//     shuffles.  The row's result is combined in an epilogue (plain store,
//     r - A x, y += A x, or a damped-Jacobi update), which fuses the
//     smoothers and residuals of the V-cycle into the product that feeds them.
//   * NV interleaved right-hand sides (NV = d for the mesh Laplacian L, which
//     acts on the d displacement components: M = L (x) I_d) share one pass
//     over the matrix.
//   * Gram-Schmidt: one pass over the basis per fused step (dots; update +
//     next dots; update + norm), deterministic two-stage reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace fsi {

constexpr int kBlock = 256;

// ------------------------------------------------------------ CSR products
template <typename T, int NV>
struct GatherPlain {
  const T* x;
  __device__ __forceinline__ T operator()(int32_t c, int n) const { return x[int64_t(c) * NV + n]; }
};


// Epilogues of a row product.  load(i, pre) reads what the row's result
// needs besides A x before the product starts, so those loads overlap the
// row's own memory chain instead of following the reduction.
template <typename T, int NV>
struct EpiStore {  // y = A x
  T* y;
  __device__ __forceinline__ void load(int64_t, T*) const {}
  __device__ __forceinline__ void operator()(int64_t i, const T* acc, const T*) const {
#pragma unroll
    for (int n = 0; n < NV; ++n) y[i * NV + n] = acc[n];
  }
};

// The fluid block's product in the inner GMRES of the fluid step: EpiStore
// under a name of its own, so that a kernel trace tells it from A_h's.
template <typename T, int NV>
struct EpiStoreFluid : EpiStore<T, NV> {};

template <typename T, int NV>
struct EpiSub {  // y = r - A x   (y may alias r)
  const T* r;
  T* y;
  __device__ __forceinline__ void load(int64_t i, T* pre) const {
#pragma unroll
    for (int n = 0; n < NV; ++n) pre[n] = r[i * NV + n];
  }
  __device__ __forceinline__ void operator()(int64_t i, const T* acc, const T* pre) const {
#pragma unroll
    for (int n = 0; n < NV; ++n) y[i * NV + n] = pre[n] - acc[n];
  }
};

template <typename T, int NV>
struct EpiAcc {  // y += A x
  T* y;
  __device__ __forceinline__ void load(int64_t i, T* pre) const {
#pragma unroll
    for (int n = 0; n < NV; ++n) pre[n] = y[i * NV + n];
  }
  __device__ __forceinline__ void operator()(int64_t i, const T* acc, const T* pre) const {
#pragma unroll
    for (int n = 0; n < NV; ++n) y[i * NV + n] = pre[n] + acc[n];
  }
};

// Inverse diagonal of a level as the smoothers read it: T values, or, for
// FP32 levels with BF16-stored diagonals, BF16 values widened on load.
template <typename T>
struct Diag {
  const T* v = nullptr;
  const uint16_t* h = nullptr;  // BF16 bit patterns (FP32 levels only) when not null
  __device__ __forceinline__ T operator[](int64_t i) const {
    if constexpr (std::is_same<T, float>::value) {
      if (h) return __uint_as_float(uint32_t(h[i]) << 16);
    }
    return v[i];
  }
};

// Accumulate row `row` of a CSR matrix into acc[NV] with the G lanes of a
// group (lane strides by G).  DEEP: four entries in flight per lane, then
// two, then one (long rows of large streamed matrices); otherwise two, then
// one (short latency-bound rows).
template <typename T, int G, int NV, class Gather, bool DEEP = false>
__device__ __forceinline__ void row_accumulate(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                               const T* __restrict__ val, int64_t row, int lane,
                                               const Gather& gx, T* acc) {
  const int64_t b = rp[row], e = rp[row + 1];
  int64_t k = b + lane;
  if (DEEP) {
    for (; k + 3 * G < e; k += 4 * G) {
      const int32_t c0 = ci[k], c1 = ci[k + G], c2 = ci[k + 2 * G], c3 = ci[k + 3 * G];
      const T a0 = val[k], a1 = val[k + G], a2 = val[k + 2 * G], a3 = val[k + 3 * G];
#pragma unroll
      for (int n = 0; n < NV; ++n) acc[n] += (a0 * gx(c0, n) + a1 * gx(c1, n)) + (a2 * gx(c2, n) + a3 * gx(c3, n));
    }
    if (k + G < e) {
      const int32_t c0 = ci[k], c1 = ci[k + G];
      const T a0 = val[k], a1 = val[k + G];
#pragma unroll
      for (int n = 0; n < NV; ++n) acc[n] += a0 * gx(c0, n) + a1 * gx(c1, n);
      k += 2 * G;
    }
  } else {
    for (; k + G < e; k += 2 * G) {
      const int32_t c0 = ci[k], c1 = ci[k + G];
      const T a0 = val[k], a1 = val[k + G];
#pragma unroll
      for (int n = 0; n < NV; ++n) acc[n] += a0 * gx(c0, n) + a1 * gx(c1, n);
    }
  }
  if (k < e) {
    const int32_t c0 = ci[k];
    const T a0 = val[k];
#pragma unroll
    for (int n = 0; n < NV; ++n) acc[n] += a0 * gx(c0, n);
  }
}

template <typename T, int G, int NV>
__device__ __forceinline__ void group_reduce(T* acc) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1)
#pragma unroll
    for (int n = 0; n < NV; ++n) acc[n] += __shfl_xor(acc[n], off, G);
}

template <typename T, int G, int NV, class Gather, class Epi, bool DEEP = false>
__global__ __launch_bounds__(kBlock) void csr_rows_kernel(int64_t nrows, const int64_t* __restrict__ rp,
                                                           const int32_t* __restrict__ ci,
                                                           const T* __restrict__ val, Gather gx, Epi epi) {
  constexpr int RPB = kBlock / G;  // rows per block
  const int64_t row = int64_t(blockIdx.x) * RPB + threadIdx.x / G;
  const int lane = threadIdx.x % G;
  if (row >= nrows) return;  // whole groups leave together (G divides 64)
  T acc[NV], pre[NV];
#pragma unroll
  for (int n = 0; n < NV; ++n) acc[n] = pre[n] = T(0);
  if (lane == 0) epi.load(row, pre);
  row_accumulate<T, G, NV, Gather, DEEP>(rp, ci, val, row, lane, gx, acc);
  group_reduce<T, G, NV>(acc);
  if (lane == 0) epi(row, acc, pre);
}

// Row product over up to four consecutive row segments, each with its own
// lanes per row (blocks [blk0[s], blk0[s+1]) serve segment s); for a matrix
// whose row blocks have very different lengths, e.g. the mesh, solid,
// fluid-velocity and pressure rows of A_h.  A segment may store its rows in
// groups of grp consecutive rows sharing one column list (values of the
// group's rows side by side): one column index and one gathered x serve grp
// rows.  Four loads in flight per lane.
// Accumulate the GR rows of row group `grp` of a grouped matrix (one column
// list per group, the GR rows' values of an entry side by side) into acc[GR]
// with the G lanes of a group: one column index and one gathered x value
// serve GR products.  Four entries in flight per lane.
template <typename T, int G, int GR, class Gather>
__device__ __forceinline__ void group_accumulate(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                 const T* __restrict__ val, int64_t grp, int lane, const Gather& gx,
                                                 T* acc) {
  const int64_t b = rp[grp], e = rp[grp + 1];
  int64_t k = b + lane;
  for (; k + 3 * G < e; k += 4 * G) {
    int32_t c[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) c[u] = ci[k + u * G];
    T a[4][GR];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int r = 0; r < GR; ++r) a[u][r] = val[(k + u * G) * GR + r];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const T xv = gx(c[u], 0);
#pragma unroll
      for (int r = 0; r < GR; ++r) acc[r] += a[u][r] * xv;
    }
  }
  for (; k < e; k += G) {
    const T xv = gx(ci[k], 0);
#pragma unroll
    for (int r = 0; r < GR; ++r) acc[r] += val[k * GR + r] * xv;
  }
}

struct RowSegments {
  int64_t row0[5];            // segment s: rows [row0[s], row0[s+1])
  unsigned blk0[5];           // segment s: blocks [blk0[s], blk0[s+1])
  int g[4];                   // lanes per row or group (4, 8, 16 or 32)
  int grp[4];                 // rows per group: 1 (the matrix's own CSR rows), 2 or 3
  const int64_t* grp_rp[4];   // grouped segments: group pointers (segment-local)
  const int32_t* grp_ci[4];   //   column list per group entry
  const void* grp_val[4];     //   grp values per entry (T)
  int nseg;
};

// Workgroups are handed to the 8 XCDs round-robin by index.  Within a range
// [b0, b0 + n) of workgroups, renumber them so that the ones an XCD receives
// take one contiguous run of the range (sizes differ by at most one): rows
// that share columns then share that XCD's L2, and every XCD still gets an
// equal share of each range.  A bijection of [0, n).
__device__ __forceinline__ unsigned xcd_contiguous(unsigned b, unsigned b0, unsigned n) {
  constexpr unsigned kXcd = 8;
  const unsigned x = b % kXcd;
  unsigned before = 0, first = 0;
  for (unsigned y = 0; y < kXcd; ++y) {
    const unsigned off = (y + kXcd - b0 % kXcd) % kXcd;  // first workgroup of the range on XCD y
    const unsigned cnt = n > off ? (n - off + kXcd - 1) / kXcd : 0;
    if (y < x) before += cnt;
    if (y == x) first = b0 + off;
  }
  return before + (b - first) / kXcd;
}

template <typename T, int G, class Gather, class Epi>
__device__ __forceinline__ void segment_rows(int64_t r0, int64_t r1, unsigned blk, const int64_t* __restrict__ rp,
                                             const int32_t* __restrict__ ci, const T* __restrict__ val,
                                             const Gather& gx, const Epi& epi) {
  const int64_t row = r0 + int64_t(blk) * (kBlock / G) + threadIdx.x / G;
  const int lane = threadIdx.x % G;
  if (row >= r1) return;
  T acc[1] = {T(0)}, pre[1] = {T(0)};
  if (lane == 0) epi.load(row, pre);
  row_accumulate<T, G, 1, Gather, true>(rp, ci, val, row, lane, gx, acc);
  group_reduce<T, G, 1>(acc);
  if (lane == 0) epi(row, acc, pre);
}

template <typename T, int G, int GR, class Gather, class Epi>
__device__ __forceinline__ void segment_groups(int64_t r0, int64_t r1, unsigned blk, const int64_t* __restrict__ rp,
                                               const int32_t* __restrict__ ci, const T* __restrict__ val,
                                               const Gather& gx, const Epi& epi) {
  const int64_t grp = int64_t(blk) * (kBlock / G) + threadIdx.x / G;
  const int lane = threadIdx.x % G;
  const int64_t row = r0 + grp * GR;
  if (row >= r1) return;
  T acc[GR], pre[GR];
#pragma unroll
  for (int r = 0; r < GR; ++r) acc[r] = pre[r] = T(0);
  if (lane == 0)
#pragma unroll
    for (int r = 0; r < GR; ++r) epi.load(row + r, pre + r);
  group_accumulate<T, G, GR>(rp, ci, val, grp, lane, gx, acc);
  group_reduce<T, G, GR>(acc);
  if (lane == 0)
#pragma unroll
    for (int r = 0; r < GR; ++r) epi(row + r, acc + r, pre + r);
}

template <typename T, int G, class Gather, class Epi>
__device__ __forceinline__ void segment_any(const RowSegments& sg, int s, unsigned blk, const int64_t* rp,
                                            const int32_t* ci, const T* val, const Gather& gx, const Epi& epi) {
  const int64_t r0 = sg.row0[s], r1 = sg.row0[s + 1];
  switch (sg.grp[s]) {
    case 2:
      segment_groups<T, G, 2>(r0, r1, blk, sg.grp_rp[s], sg.grp_ci[s], static_cast<const T*>(sg.grp_val[s]), gx, epi);
      break;
    case 3:
      segment_groups<T, G, 3>(r0, r1, blk, sg.grp_rp[s], sg.grp_ci[s], static_cast<const T*>(sg.grp_val[s]), gx, epi);
      break;
    default: segment_rows<T, G>(r0, r1, blk, rp, ci, val, gx, epi); break;
  }
}

template <typename T, class Gather, class Epi>
__global__ __launch_bounds__(kBlock) void csr_segments_kernel(RowSegments sg, const int64_t* __restrict__ rp,
                                                               const int32_t* __restrict__ ci,
                                                               const T* __restrict__ val, Gather gx, Epi epi) {
  int s = 0;
  while (s + 1 < sg.nseg && blockIdx.x >= sg.blk0[s + 1]) ++s;
  const unsigned blk = xcd_contiguous(blockIdx.x, sg.blk0[s], sg.blk0[s + 1] - sg.blk0[s]);
  switch (sg.g[s]) {
    case 4: segment_any<T, 4>(sg, s, blk, rp, ci, val, gx, epi); break;
    case 8: segment_any<T, 8>(sg, s, blk, rp, ci, val, gx, epi); break;
    case 16: segment_any<T, 16>(sg, s, blk, rp, ci, val, gx, epi); break;
    default: segment_any<T, 32>(sg, s, blk, rp, ci, val, gx, epi); break;
  }
}

// ------------------------------------------------ fused V-cycle level sweeps
// Down-sweep of a V(1,1) level with a zero initial guess: the pre-smoothed
// x = omega D^{-1} b gives the residual r = b - omega (A D^{-1}) b on the fine
// rows (A D^{-1}: A with its columns scaled at setup), and the restricted
// residual b_c = R r = Q b on the coarse rows, Q = R (I - omega A D^{-1})
// formed at setup.  Both read only b, so one launch covers both row sets
// (blocks [0, nblk_a) the fine rows, the rest the coarse rows).
template <typename T, int GA, int GQ, int NV, bool DEEP = false>
__global__ __launch_bounds__(kBlock) void vdown_kernel(
    int64_t na, const int64_t* __restrict__ rpa, const int32_t* __restrict__ cia, const T* __restrict__ va,
    int64_t nq, const int64_t* __restrict__ rpq, const int32_t* __restrict__ ciq, const T* __restrict__ vq,
    const T* __restrict__ b, T omega, T* __restrict__ r, T* __restrict__ bc, unsigned nblk_a) {
  T acc[NV];
#pragma unroll
  for (int n = 0; n < NV; ++n) acc[n] = T(0);
  // each of the two row sets is spread over the XCDs in contiguous runs
  const unsigned blk = blockIdx.x < nblk_a ? xcd_contiguous(blockIdx.x, 0, nblk_a)
                                           : nblk_a + xcd_contiguous(blockIdx.x, nblk_a, gridDim.x - nblk_a);
  if (blk < nblk_a) {
    const int64_t row = int64_t(blk) * (kBlock / GA) + threadIdx.x / GA;
    const int lane = threadIdx.x % GA;
    if (row >= na) return;
    T bi[NV];
#pragma unroll
    for (int n = 0; n < NV; ++n) bi[n] = lane == 0 ? b[row * NV + n] : T(0);
    row_accumulate<T, GA, NV, GatherPlain<T, NV>, DEEP>(rpa, cia, va, row, lane, GatherPlain<T, NV>{b}, acc);
    group_reduce<T, GA, NV>(acc);
    if (lane == 0)
#pragma unroll
      for (int n = 0; n < NV; ++n) r[row * NV + n] = bi[n] - omega * acc[n];
  } else {
    const int64_t row = int64_t(blk - nblk_a) * (kBlock / GQ) + threadIdx.x / GQ;
    const int lane = threadIdx.x % GQ;
    if (row >= nq) return;
    row_accumulate<T, GQ, NV, GatherPlain<T, NV>, DEEP>(rpq, ciq, vq, row, lane, GatherPlain<T, NV>{b}, acc);
    group_reduce<T, GQ, NV>(acc);
    if (lane == 0)
#pragma unroll
      for (int n = 0; n < NV; ++n) bc[row * NV + n] = acc[n];
  }
}

// Up-sweep: with x = omega D^{-1} b + P e (prolongated coarse correction) the
// post-smoothing step x + omega D^{-1} (b - A x) equals
//   y = omega D^{-1} b + P e + omega D^{-1} (r - (A P) e),
// r from the down-sweep and A P formed at setup: one pass over the rows of P
// and A P.  y may alias b.
template <typename T, int G, int NV, bool DEEP = false>
__global__ __launch_bounds__(kBlock) void vup_kernel(
    int64_t n, const int64_t* __restrict__ rpp, const int32_t* __restrict__ cip, const T* __restrict__ vp,
    const int64_t* __restrict__ rpap, const int32_t* __restrict__ ciap, const T* __restrict__ vap,
    const T* __restrict__ e, const T* b, Diag<T> dinv, T omega, const T* __restrict__ r, T* y) {
  constexpr int RPB = kBlock / G;
  const int64_t row = int64_t(xcd_contiguous(blockIdx.x, 0, gridDim.x)) * RPB + threadIdx.x / G;
  const int lane = threadIdx.x % G;
  if (row >= n) return;
  T ap[NV], pe[NV], bi[NV], ri[NV];
  T wd = T(0);
#pragma unroll
  for (int q = 0; q < NV; ++q) ap[q] = pe[q] = bi[q] = ri[q] = T(0);
  if (lane == 0) {  // the row's own values, loaded ahead of the products
    wd = omega * dinv[row];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      bi[q] = b[row * NV + q];
      ri[q] = r[row * NV + q];
    }
  }
  const GatherPlain<T, NV> ge{e};
  row_accumulate<T, G, NV, GatherPlain<T, NV>, DEEP>(rpp, cip, vp, row, lane, ge, pe);
  row_accumulate<T, G, NV, GatherPlain<T, NV>, DEEP>(rpap, ciap, vap, row, lane, ge, ap);
  group_reduce<T, G, NV>(pe);
  group_reduce<T, G, NV>(ap);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) y[row * NV + q] = wd * bi[q] + pe[q] + wd * (ri[q] - ap[q]);
}

// The two level sweeps above for matrices stored in groups of GR rows (the
// GR components of a node; fine and coarse levels with the same block size):
// A D^{-1}, Q, P and A P each read one column index per GR values.
template <typename T, int GA, int GQ, int GR>
__global__ __launch_bounds__(kBlock) void vdown_grp_kernel(
    int64_t na, const int64_t* __restrict__ rpa, const int32_t* __restrict__ cia, const T* __restrict__ va,
    int64_t nq, const int64_t* __restrict__ rpq, const int32_t* __restrict__ ciq, const T* __restrict__ vq,
    const T* __restrict__ b, T omega, T* __restrict__ r, T* __restrict__ bc, unsigned nblk_a) {
  T acc[GR];
#pragma unroll
  for (int q = 0; q < GR; ++q) acc[q] = T(0);
  const unsigned blk = blockIdx.x < nblk_a ? xcd_contiguous(blockIdx.x, 0, nblk_a)
                                           : nblk_a + xcd_contiguous(blockIdx.x, nblk_a, gridDim.x - nblk_a);
  const GatherPlain<T, 1> gb{b};
  if (blk < nblk_a) {
    const int64_t grp = int64_t(blk) * (kBlock / GA) + threadIdx.x / GA;
    const int lane = threadIdx.x % GA;
    const int64_t row = grp * GR;
    if (row >= na) return;
    T bi[GR];
#pragma unroll
    for (int q = 0; q < GR; ++q) bi[q] = lane == 0 ? b[row + q] : T(0);
    group_accumulate<T, GA, GR>(rpa, cia, va, grp, lane, gb, acc);
    group_reduce<T, GA, GR>(acc);
    if (lane == 0)
#pragma unroll
      for (int q = 0; q < GR; ++q) r[row + q] = bi[q] - omega * acc[q];
  } else {
    const int64_t grp = int64_t(blk - nblk_a) * (kBlock / GQ) + threadIdx.x / GQ;
    const int lane = threadIdx.x % GQ;
    const int64_t row = grp * GR;
    if (row >= nq) return;
    group_accumulate<T, GQ, GR>(rpq, ciq, vq, grp, lane, gb, acc);
    group_reduce<T, GQ, GR>(acc);
    if (lane == 0)
#pragma unroll
      for (int q = 0; q < GR; ++q) bc[row + q] = acc[q];
  }
}

template <typename T, int G, int GR>
__global__ __launch_bounds__(kBlock) void vup_grp_kernel(
    int64_t n, const int64_t* __restrict__ rpp, const int32_t* __restrict__ cip, const T* __restrict__ vp,
    const int64_t* __restrict__ rpap, const int32_t* __restrict__ ciap, const T* __restrict__ vap,
    const T* __restrict__ e, const T* b, Diag<T> dinv, T omega, const T* __restrict__ r, T* y) {
  const int64_t grp = int64_t(xcd_contiguous(blockIdx.x, 0, gridDim.x)) * (kBlock / G) + threadIdx.x / G;
  const int lane = threadIdx.x % G;
  const int64_t row = grp * GR;
  if (row >= n) return;
  T ap[GR], pe[GR], bi[GR], ri[GR], wd[GR];
#pragma unroll
  for (int q = 0; q < GR; ++q) ap[q] = pe[q] = bi[q] = ri[q] = wd[q] = T(0);
  if (lane == 0)  // the rows' own values, loaded ahead of the products
#pragma unroll
    for (int q = 0; q < GR; ++q) {
      wd[q] = omega * dinv[row + q];
      bi[q] = b[row + q];
      ri[q] = r[row + q];
    }
  const GatherPlain<T, 1> ge{e};
  group_accumulate<T, G, GR>(rpp, cip, vp, grp, lane, ge, pe);
  group_accumulate<T, G, GR>(rpap, ciap, vap, grp, lane, ge, ap);
  group_reduce<T, G, GR>(pe);
  group_reduce<T, G, GR>(ap);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < GR; ++q) y[row + q] = wd[q] * bi[q] + pe[q] + wd[q] * (ri[q] - ap[q]);
}

// Residual of the learned pre-smoother's correction and the partials of its
// acceptance test: r = b - A x on every row (fixed grid of kDecideBlocks
// blocks striding over the rows), part[2 k] = sum of r^2 and part[2 k + 1] =
// sum of b^2 over the rows of block k, summed in a fixed order.
constexpr int kDecideBlocks = 1024;
// After this many consecutive rejections in a solve the learned pre-smoother
// is not tried again until the next solve (or new weights): its inference
// and residual kernels return at once and the down-sweep takes the Jacobi
// branch.  The count lives in device memory, advanced by the up-sweep.
constexpr int kLearnedStreak = 8;

template <typename T, int G, int NV>
__global__ __launch_bounds__(kBlock) void learned_resid_kernel(int64_t n, const int64_t* __restrict__ rp,
                                                                const int32_t* __restrict__ ci,
                                                                const T* __restrict__ val, const T* __restrict__ x,
                                                                const T* __restrict__ b, T* __restrict__ r,
                                                                double* __restrict__ part,
                                                                const int* __restrict__ streak) {
  if (streak[0] >= kLearnedStreak) return;  // not tried any more in this solve
  constexpr int RPB = kBlock / G;
  __shared__ double sh[2][kBlock / 64];
  const int lane = threadIdx.x % G;
  double rr = 0.0, bb = 0.0;
  for (int64_t row0 = int64_t(blockIdx.x) * RPB; row0 < n; row0 += int64_t(gridDim.x) * RPB) {
    const int64_t row = row0 + threadIdx.x / G;
    T acc[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = T(0);
    if (row < n) row_accumulate<T, G, NV>(rp, ci, val, row, lane, GatherPlain<T, NV>{x}, acc);
    group_reduce<T, G, NV>(acc);
    if (lane == 0 && row < n)
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const T bi = b[row * NV + q];
        const T ri = bi - acc[q];
        r[row * NV + q] = ri;
        rr += double(ri) * double(ri);
        bb += double(bi) * double(bi);
      }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    rr += __shfl_xor(rr, off, 64);
    bb += __shfl_xor(bb, off, 64);
  }
  if (threadIdx.x % 64 == 0) {
    sh[0][threadIdx.x / 64] = rr;
    sh[1][threadIdx.x / 64] = bb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
      a += sh[0][w];
      c += sh[1][w];
    }
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = c;
  }
}

// Acceptance of the learned correction: ||r|| <= ||b|| (NaN: rejected), from
// the partials above.  Every block evaluates it in the same order, so all
// agree; the owner block stores it in flag[0] and counts a rejection.
__device__ __forceinline__ bool learned_accept(const double* __restrict__ part, int* flag, int* fallbacks,
                                               const int* __restrict__ streak, bool owner) {
  __shared__ int s_ok;
  if (streak[0] >= kLearnedStreak) {  // not tried (the partials are stale): Jacobi
    if (threadIdx.x == 0 && owner) {
      flag[0] = 0;
      fallbacks[0] = fallbacks[0] + 1;
    }
    return false;
  }
  if (threadIdx.x < 64) {
    double rr = 0.0, bb = 0.0;
#pragma unroll
    for (int i = 0; i < kDecideBlocks / 64; ++i) {
      rr += part[2 * (threadIdx.x + 64 * i)];
      bb += part[2 * (threadIdx.x + 64 * i) + 1];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      rr += __shfl_xor(rr, off, 64);
      bb += __shfl_xor(bb, off, 64);
    }
    if (threadIdx.x == 0) {
      const int ok = (rr <= bb) ? 1 : 0;
      s_ok = ok;
      if (owner) {
        flag[0] = ok;
        if (!ok) fallbacks[0] = fallbacks[0] + 1;
      }
    }
  }
  __syncthreads();
  return s_ok != 0;
}

// Finest-level sweeps with the learned pre-smoothing (accepted) or its
// Jacobi fallback (rejected); the down-sweep decides (learned_accept) and
// leaves the decision in flag[0] for the up-sweep.  With the network's correction x_m the
// residual r_m = b - A x_m is formed beforehand; the down-sweep then only
// restricts it (b_c = R r_m) and the up-sweep starts from x_m:
//   y = x_m + P e + omega D^{-1} (r_m - (A P) e).
// With the fallback both sweeps are exactly vdown/vup above.
template <typename T, int GA, int GQ, int NV>
__global__ __launch_bounds__(kBlock) void vdown_sel_kernel(
    int64_t na, const int64_t* __restrict__ rpa, const int32_t* __restrict__ cia, const T* __restrict__ va,
    int64_t nq, const int64_t* __restrict__ rpq, const int32_t* __restrict__ ciq, const T* __restrict__ vq,
    const int64_t* __restrict__ rpr, const int32_t* __restrict__ cir, const T* __restrict__ vr,
    const T* __restrict__ b, T omega, T* __restrict__ r, T* __restrict__ bc, const T* __restrict__ r_m,
    const double* __restrict__ part, int* flag, int* fallbacks, const int* __restrict__ streak, unsigned nblk_a) {
  const bool learned = learned_accept(part, flag, fallbacks, streak, blockIdx.x == 0);
  T acc[NV];
#pragma unroll
  for (int n = 0; n < NV; ++n) acc[n] = T(0);
  if (blockIdx.x < nblk_a) {
    if (learned) return;  // r_m is already formed
    const int64_t row = int64_t(blockIdx.x) * (kBlock / GA) + threadIdx.x / GA;
    const int lane = threadIdx.x % GA;
    if (row >= na) return;
    T bi[NV];
#pragma unroll
    for (int n = 0; n < NV; ++n) bi[n] = lane == 0 ? b[row * NV + n] : T(0);
    row_accumulate<T, GA, NV>(rpa, cia, va, row, lane, GatherPlain<T, NV>{b}, acc);
    group_reduce<T, GA, NV>(acc);
    if (lane == 0)
#pragma unroll
      for (int n = 0; n < NV; ++n) r[row * NV + n] = bi[n] - omega * acc[n];
  } else {
    const int64_t row = int64_t(blockIdx.x - nblk_a) * (kBlock / GQ) + threadIdx.x / GQ;
    const int lane = threadIdx.x % GQ;
    if (row >= nq) return;
    if (learned) row_accumulate<T, GQ, NV>(rpr, cir, vr, row, lane, GatherPlain<T, NV>{r_m}, acc);
    else row_accumulate<T, GQ, NV>(rpq, ciq, vq, row, lane, GatherPlain<T, NV>{b}, acc);
    group_reduce<T, GQ, NV>(acc);
    if (lane == 0)
#pragma unroll
      for (int n = 0; n < NV; ++n) bc[row * NV + n] = acc[n];
  }
}

template <typename T, int G, int NV>
__global__ __launch_bounds__(kBlock) void vup_sel_kernel(
    int64_t n, const int64_t* __restrict__ rpp, const int32_t* __restrict__ cip, const T* __restrict__ vp,
    const int64_t* __restrict__ rpap, const int32_t* __restrict__ ciap, const T* __restrict__ vap,
    const T* __restrict__ e, const T* b, Diag<T> dinv, T omega, const T* __restrict__ r,
    const T* __restrict__ x_m, const T* __restrict__ r_m, const int* __restrict__ flag, int* streak, T* y) {
  constexpr int RPB = kBlock / G;
  const int64_t row = int64_t(blockIdx.x) * RPB + threadIdx.x / G;
  const int lane = threadIdx.x % G;
  if (blockIdx.x == 0 && threadIdx.x == 0)  // consecutive rejections (read by the next cycle)
    streak[0] = flag[0] ? 0 : (streak[0] < kLearnedStreak ? streak[0] + 1 : kLearnedStreak);
  if (row >= n) return;
  T ap[NV], pe[NV], x0[NV], rr[NV];
  T wd = T(0);
#pragma unroll
  for (int q = 0; q < NV; ++q) ap[q] = pe[q] = x0[q] = rr[q] = T(0);
  if (lane == 0) {  // the row's own values, loaded ahead of the products
    const bool learned = flag[0] != 0;
    wd = omega * dinv[row];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int64_t k = row * NV + q;
      x0[q] = learned ? x_m[k] : wd * b[k];
      rr[q] = learned ? r_m[k] : r[k];
    }
  }
  const GatherPlain<T, NV> ge{e};
  row_accumulate<T, G, NV>(rpp, cip, vp, row, lane, ge, pe);
  row_accumulate<T, G, NV>(rpap, ciap, vap, row, lane, ge, ap);
  group_reduce<T, G, NV>(pe);
  group_reduce<T, G, NV>(ap);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) y[row * NV + q] = x0[q] + pe[q] + wd * (rr[q] - ap[q]);
}

// ------------------------------------------------ Chebyshev level sweeps
// Chebyshev smoothing of a level (D^{-1} A on [lam/ratio, lam]) with the
// three-term recurrence
//   d_j = a_j d_{j-1} + c_j D^{-1} r_{j-1},  x_j = x_{j-1} + d_j,  r_j = r_{j-1} - A d_j
// (a_1 = 0, c_1 = 1/theta).  One launch per step: the step's direction is
// formed at every gathered column from the previous step's d and r, so a
// launch reads only vectors of the step before it.
template <typename T, int NV>
struct ChebGather {
  const T* d;     // d_{j-1} (unused when a == 0)
  const T* r;     // r_{j-1}
  Diag<T> dinv;  // per row (shared by the NV interleaved columns)
  T a, c;
  __device__ __forceinline__ T operator()(int32_t col, int n) const {
    const T v = c * dinv[col] * r[int64_t(col) * NV + n];
    return a != T(0) ? a * d[int64_t(col) * NV + n] + v : v;
  }
};

// Step j on every row: d_j, r_j stored (dout, rout), x += d_j (x = d_j when
// xinit).  With `fuse` the next step's direction d_{j+1} = a2 d_j + c2 D^{-1}
// r_j (which needs row i only) is added to x as well and d_j, r_j are not
// stored: the last step of a post-smoothing sweep.
template <typename T, int G, int NV>
__global__ __launch_bounds__(kBlock) void cheb_step_kernel(int64_t n, const int64_t* __restrict__ rp,
                                                            const int32_t* __restrict__ ci,
                                                            const T* __restrict__ val, ChebGather<T, NV> g,
                                                            T* __restrict__ dout, T* __restrict__ rout, T* x,
                                                            int xinit, int fuse, T a2, T c2) {
  constexpr int RPB = kBlock / G;
  const int64_t row = int64_t(xcd_contiguous(blockIdx.x, 0, gridDim.x)) * RPB + threadIdx.x / G;
  const int lane = threadIdx.x % G;
  if (row >= n) return;
  T acc[NV], dj[NV], rp0[NV], xi[NV];
  T di = T(0);
#pragma unroll
  for (int q = 0; q < NV; ++q) acc[q] = dj[q] = rp0[q] = xi[q] = T(0);
  if (lane == 0) {  // the row's own values, loaded ahead of the product
    di = g.dinv[row];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int64_t k = row * NV + q;
      dj[q] = g(int32_t(row), q);
      rp0[q] = g.r[k];
      xi[q] = xinit ? T(0) : x[k];
    }
  }
  row_accumulate<T, G, NV>(rp, ci, val, row, lane, g, acc);
  group_reduce<T, G, NV>(acc);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int64_t k = row * NV + q;
      const T rj = rp0[q] - acc[q];
      if (fuse) {
        x[k] = xi[q] + dj[q] + (a2 * dj[q] + c2 * di * rj);
      } else {
        dout[k] = dj[q];
        rout[k] = rj;
        x[k] = xinit ? dj[q] : xi[q] + dj[q];
      }
    }
  }
}

// The last pre-smoothing step of a Chebyshev level with the restriction in
// the same launch: blocks [0, nblk_f) run the step on the fine rows (d_k, r_k
// stored, x updated), the others compute the coarse right-hand side
//   b_c = R r_k = R r_{k-1} - (R A) d_k
// with d_k formed at every gathered column like the fine rows do.  R and R A
// share one column list (the union pattern), their two values side by side.
template <typename T, int G, int GC, int NV>
__global__ __launch_bounds__(kBlock) void cheb_step_restrict_kernel(
    int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci, const T* __restrict__ val,
    ChebGather<T, NV> g, T* __restrict__ dout, T* __restrict__ rout, T* x, int xinit, int64_t nc,
    const int64_t* __restrict__ rpc, const int32_t* __restrict__ cic, const T* __restrict__ vrc, T* __restrict__ bc,
    unsigned nblk_f) {
  if (blockIdx.x < nblk_f) {
    constexpr int RPB = kBlock / G;
    const int64_t row = int64_t(blockIdx.x) * RPB + threadIdx.x / G;
    const int lane = threadIdx.x % G;
    if (row >= n) return;
    T acc[NV], dj[NV], rp0[NV], xi[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] = dj[q] = rp0[q] = xi[q] = T(0);
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const int64_t k = row * NV + q;
        dj[q] = g(int32_t(row), q);
        rp0[q] = g.r[k];
        xi[q] = xinit ? T(0) : x[k];
      }
    }
    row_accumulate<T, G, NV>(rp, ci, val, row, lane, g, acc);
    group_reduce<T, G, NV>(acc);
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const int64_t k = row * NV + q;
        dout[k] = dj[q];
        rout[k] = rp0[q] - acc[q];
        x[k] = xinit ? dj[q] : xi[q] + dj[q];
      }
    }
    return;
  }
  constexpr int RPB = kBlock / GC;
  const int64_t row = int64_t(blockIdx.x - nblk_f) * RPB + threadIdx.x / GC;
  const int lane = threadIdx.x % GC;
  if (row >= nc) return;
  T acc[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) acc[q] = T(0);
  const int64_t b = rpc[row], e = rpc[row + 1];
  for (int64_t k = b + lane; k < e; k += GC) {
    const int32_t c = cic[k];
    const T rv = vrc[2 * k], rav = vrc[2 * k + 1];
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[q] += rv * g.r[int64_t(c) * NV + q] - rav * g(c, q);
  }
  group_reduce<T, GC, NV>(acc);
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) bc[row * NV + q] = acc[q];
}

// Coarse correction of a Chebyshev level: x += P e, r -= (A P) e (r in place;
// both only at the row itself).  With `fuse` (degree 1) the post-smoothing
// step x += c1 D^{-1} r follows in the same pass.
template <typename T, int G, int NV>
__global__ __launch_bounds__(kBlock) void cheb_prolong_kernel(
    int64_t n, const int64_t* __restrict__ rpp, const int32_t* __restrict__ cip, const T* __restrict__ vp,
    const int64_t* __restrict__ rpap, const int32_t* __restrict__ ciap, const T* __restrict__ vap,
    const T* __restrict__ e, Diag<T> dinv, T* x, T* r, int fuse, T c1) {
  constexpr int RPB = kBlock / G;
  const int64_t row = int64_t(blockIdx.x) * RPB + threadIdx.x / G;
  const int lane = threadIdx.x % G;
  if (row >= n) return;
  T ap[NV], pe[NV], x0[NV], r0[NV];
  T di = T(0);
#pragma unroll
  for (int q = 0; q < NV; ++q) ap[q] = pe[q] = x0[q] = r0[q] = T(0);
  if (lane == 0) {  // the row's own values, loaded ahead of the products
    di = dinv[row];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      x0[q] = x[row * NV + q];
      r0[q] = r[row * NV + q];
    }
  }
  const GatherPlain<T, NV> ge{e};
  row_accumulate<T, G, NV>(rpp, cip, vp, row, lane, ge, pe);
  row_accumulate<T, G, NV>(rpap, ciap, vap, row, lane, ge, ap);
  group_reduce<T, G, NV>(pe);
  group_reduce<T, G, NV>(ap);
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int64_t k = row * NV + q;
      const T rk = r0[q] - ap[q];
      T xk = x0[q] + pe[q];
      if (fuse) xk = xk + c1 * di * rk;
      x[k] = xk;
      r[k] = rk;
    }
  }
}

// -------------------------------------------------------------- coarse solve
// X = Ainv B with a dense row-major n x n inverse (FP64); WPR wavefronts per
// row (one for short rows; four, the whole workgroup, for long ones, so each
// lane's chain of dependent loads stays short); B, X hold NV interleaved
// columns.  X must not alias B.
template <typename TI, typename TO, int NV, int WPR = 1>
__global__ __launch_bounds__(kBlock) void dense_gemv_kernel(int64_t n, const double* __restrict__ Ainv,
                                                             const TI* __restrict__ B, TO* __restrict__ X) {
  constexpr int LPR = 64 * WPR;  // lanes per row
  const int64_t row = int64_t(blockIdx.x) * (kBlock / LPR) + threadIdx.x / LPR;
  const int lane = threadIdx.x % LPR;
  const bool valid = row < n;  // uniform per row (WPR > 1: one row per workgroup)
  if (WPR == 1 && !valid) return;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  if (valid) {
    const double* a = Ainv + row * n;
    int64_t j = lane;
    for (; j + 3 * LPR < n; j += 4 * LPR) {  // four independent loads in flight per lane
      const double a0 = a[j], a1 = a[j + LPR], a2 = a[j + 2 * LPR], a3 = a[j + 3 * LPR];
#pragma unroll
      for (int v = 0; v < NV; ++v)
        acc[v] += (a0 * double(B[j * NV + v]) + a1 * double(B[(j + LPR) * NV + v])) +
                  (a2 * double(B[(j + 2 * LPR) * NV + v]) + a3 * double(B[(j + 3 * LPR) * NV + v]));
    }
    for (; j < n; j += LPR) {
      const double aj = a[j];
#pragma unroll
      for (int v = 0; v < NV; ++v) acc[v] += aj * double(B[j * NV + v]);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += __shfl_xor(acc[v], off, 64);
  if constexpr (WPR > 1) {
    __shared__ double red[WPR][NV];
    if (threadIdx.x % 64 == 0)
#pragma unroll
      for (int v = 0; v < NV; ++v) red[threadIdx.x / 64][v] = acc[v];
    __syncthreads();
    if (threadIdx.x == 0 && valid)
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < WPR; ++w) t += red[w][v];
        X[row * NV + v] = TO(t);
      }
  } else {
    if (lane == 0)
#pragma unroll
      for (int v = 0; v < NV; ++v) X[row * NV + v] = TO(acc[v]);
  }
}

// -------------------------------------------------------------- vector ops
template <typename T>
__global__ __launch_bounds__(kBlock) void vsub_kernel(int64_t n, T* __restrict__ y, const T* __restrict__ x) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    y[i] = y[i] - x[i];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void vadd_kernel(int64_t n, T* __restrict__ y, const T* __restrict__ x) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    y[i] = y[i] + x[i];
}

template <typename TI, typename TO>
__global__ __launch_bounds__(kBlock) void cast_kernel(int64_t n, const TI* __restrict__ x, TO* __restrict__ y) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    y[i] = TO(x[i]);
}

// y = f x, converted to TO (f applied in FP64)
template <typename TI, typename TO>
__global__ __launch_bounds__(kBlock) void cast_scale_kernel(int64_t n, const TI* __restrict__ x, double f,
                                                            TO* __restrict__ y) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    y[i] = TO(f * double(x[i]));
}

// y *= f (in place)
__global__ __launch_bounds__(kBlock) void scale_kernel(int64_t n, double* y, double f) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    y[i] = y[i] * f;
}

// ---------------------------------------------------------- Gram-Schmidt
// One fused pass over the Krylov basis V (vectors V_i = V + i * ld) and the
// new vector w on a fixed grid; every block writes one partial per output
// into part[i * gridDim.x + block], and gs_reduce_kernel adds them in block
// order (bit-reproducible; no cross-block synchronisation inside a kernel,
// which would need a device-scope release, i.e. an L2 write-back, per block).
//   mode 0: out[i] = V_i . w (i < nv),            out[nv] = w . w
//   mode 1: w -= sum_i h_i V_i, then out[i] = V_i . w, out[nv] = w . w
//   mode 2: w -= sum_i h_i V_i, then                  out[nv] = w . w
constexpr int kGsBlocks = 1024;
constexpr int kMaxBasis = 208;
constexpr int kWaves = kBlock / 64;
constexpr int kGsTile = 8;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ __launch_bounds__(kBlock) void gs_pass_kernel(int64_t n, int nv, const double* __restrict__ V,
                                                          int64_t ld, double* __restrict__ w,
                                                          const double* __restrict__ h, int mode,
                                                          double* __restrict__ part) {
  __shared__ double hs[kMaxBasis];
  __shared__ double ws[kWaves][kMaxBasis + 1];
  const int tid = threadIdx.x, wid = tid / 64, lane = tid % 64;
  if (mode != 0)
    for (int i = tid; i < nv; i += kBlock) hs[i] = h[i];
  __syncthreads();
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = int64_t(blockIdx.x) * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  if (mode != 0) {
    // w -= V h with kGsTile independent loads per element
    for (int64_t k = lo + tid; k < hi; k += kBlock) {
      double acc[kGsTile];
#pragma unroll
      for (int t = 0; t < kGsTile; ++t) acc[t] = 0.0;
      int i0 = 0;
      for (; i0 + kGsTile <= nv; i0 += kGsTile)
#pragma unroll
        for (int t = 0; t < kGsTile; ++t) acc[t] += hs[i0 + t] * V[(i0 + t) * ld + k];
      for (int i = i0; i < nv; ++i) acc[i - i0] += hs[i] * V[i * ld + k];
      double s = 0.0;
#pragma unroll
      for (int t = 0; t < kGsTile; ++t) s += acc[t];
      w[k] = w[k] - s;
    }
  }
  // dots in tiles of kGsTile vectors (kGsTile independent loads per element,
  // no branches inside the element loop)
  const int first = mode == 2 ? nv : 0;
  int i0 = first;
  for (; i0 + kGsTile <= nv; i0 += kGsTile) {
    double acc[kGsTile];
#pragma unroll
    for (int t = 0; t < kGsTile; ++t) acc[t] = 0.0;
    const double* vt = V + i0 * ld;
    for (int64_t k = lo + tid; k < hi; k += kBlock) {
      const double wk = w[k];
#pragma unroll
      for (int t = 0; t < kGsTile; ++t) acc[t] += vt[t * ld + k] * wk;
    }
#pragma unroll
    for (int t = 0; t < kGsTile; ++t) {
      const double sv = wave_sum(acc[t]);
      if (lane == 0) ws[wid][i0 + t] = sv;
    }
  }
  {
    // tail: the remaining cnt < kGsTile vectors and w . w (index nv); loads
    // of the unused slots are clamped to a valid vector and masked out
    const int cnt = nv - i0;
    double acc[kGsTile];
    double aw = 0.0;
#pragma unroll
    for (int t = 0; t < kGsTile; ++t) acc[t] = 0.0;
    if (cnt > 0) {
      for (int64_t k = lo + tid; k < hi; k += kBlock) {
        const double wk = w[k];
        aw += wk * wk;
#pragma unroll
        for (int t = 0; t < kGsTile; ++t) {
          const int i = t < cnt ? i0 + t : nv - 1;
          const double m = t < cnt ? 1.0 : 0.0;
          acc[t] += m * (V[i * ld + k] * wk);
        }
      }
    } else {
      for (int64_t k = lo + tid; k < hi; k += kBlock) {
        const double wk = w[k];
        aw += wk * wk;
      }
    }
#pragma unroll
    for (int t = 0; t < kGsTile; ++t) {
      if (t < cnt) {
        const double sv = wave_sum(acc[t]);
        if (lane == 0) ws[wid][i0 + t] = sv;
      }
    }
    const double sw = wave_sum(aw);
    if (lane == 0) ws[wid][nv] = sw;
  }
  __syncthreads();
  for (int i = first + tid; i <= nv; i += kBlock) {
    double p = 0.0;
    for (int q = 0; q < kWaves; ++q) p += ws[q][i];
    part[int64_t(i) * gridDim.x + blockIdx.x] = p;
  }
}

// out[first + b] = sum over the nb block partials of output first + b, in
// block order (one block per output).
__global__ __launch_bounds__(kBlock) void gs_reduce_kernel(int nb, int first, const double* __restrict__ part,
                                                            double* __restrict__ out) {
  __shared__ double sh[kWaves];
  const int i = first + blockIdx.x;
  const double* p = part + int64_t(i) * nb;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBlock) s += p[b];
  s = wave_sum(s);
  if (threadIdx.x % 64 == 0) sh[threadIdx.x / 64] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < kWaves; ++q) t += sh[q];
    out[i] = t;
  }
}

// V_{j+1} = w / ||w|| with the norm read on the device (out of the last
// Gram-Schmidt pass); left untouched on a breakdown (||w|| <= 1e-14 of its
// norm before orthogonalisation), which the host detects with the same test.
__global__ __launch_bounds__(kBlock) void gs_normalise_kernel(int64_t n, double* w, const double* __restrict__ nrm2,
                                                               const double* __restrict__ nrm2_before) {
  const double hn = sqrt(nrm2[0] > 0.0 ? nrm2[0] : 0.0);
  const double wb = sqrt(nrm2_before[0]);
  if (!(hn > 1e-14 * wb)) return;
  const double f = 1.0 / hn;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    w[i] = w[i] * f;
}

// x += sum_i y_i Z_i
__global__ __launch_bounds__(kBlock) void multi_axpy_kernel(int64_t n, int nv, const double* __restrict__ Z,
                                                             int64_t ld, const double* __restrict__ y,
                                                             double* __restrict__ x) {
  __shared__ double ys[kMaxBasis];
  for (int i = threadIdx.x; i < nv; i += kBlock) ys[i] = y[i];
  __syncthreads();
  for (int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x; k < n; k += int64_t(gridDim.x) * kBlock) {
    double s = x[k];
    for (int i = 0; i < nv; ++i) s += ys[i] * Z[i * ld + k];
    x[k] = s;
  }
}

// ------------------------------------------------ inner GMRES of the fluid step
// k <= kInnerMax steps of flexible GMRES on the fluid block (vectors in the
// preconditioner's precision T, sums and the Hessenberg matrix in FP64, all
// scalars kept on the device: no host round trip inside P^{-1}).
constexpr int kInnerMax = 16;
constexpr int kInnerBlocks = 512;

// One Gram-Schmidt pass of the inner GMRES (the pattern of gs_pass_kernel):
// first w -= sum_{i < nu} h_i V_i (nu = 0: none), then block partial sums
// part[i * gridDim.x + block] = V_i . w for i < nd and part[nd * gridDim.x +
// block] = w . w; V_i is read once when both are asked for.  gs_reduce_kernel
// adds the partial sums in block order.
template <typename T>
__global__ __launch_bounds__(kBlock) void inner_pass_kernel(int64_t n, int nu, int nd, const T* __restrict__ V,
                                                            int64_t ld, const double* __restrict__ h,
                                                            T* __restrict__ w, double* __restrict__ part) {
  __shared__ double hs[kInnerMax];
  __shared__ double sh[kWaves][kInnerMax + 1];
  if (threadIdx.x < nu) hs[threadIdx.x] = h[threadIdx.x];
  __syncthreads();
  const int nl = nu > nd ? nu : nd;
  double acc[kInnerMax + 1];
#pragma unroll
  for (int i = 0; i <= kInnerMax; ++i) acc[i] = 0.0;
  for (int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x; k < n; k += int64_t(gridDim.x) * kBlock) {
    double v[kInnerMax];
#pragma unroll
    for (int i = 0; i < kInnerMax; ++i) v[i] = i < nl ? double(V[i * ld + k]) : 0.0;
    double wk = double(w[k]);
    if (nu > 0) {
#pragma unroll
      for (int i = 0; i < kInnerMax; ++i)
        if (i < nu) wk -= hs[i] * v[i];
      const T st = T(wk);
      w[k] = st;
      wk = double(st);
    }
#pragma unroll
    for (int i = 0; i < kInnerMax; ++i)
      if (i < nd) acc[i] += v[i] * wk;
    acc[kInnerMax] += wk * wk;
  }
  const int wid = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
  for (int i = 0; i <= kInnerMax; ++i) {
    if (i < nd || i == kInnerMax) {
      const double t = wave_sum(acc[i]);
      if (lane == 0) sh[wid][i] = t;
    }
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t <= nd) {
    const int slot = t < nd ? t : kInnerMax;
    double v = 0.0;
    for (int q = 0; q < kWaves; ++q) v += sh[q][slot];
    part[int64_t(t) * gridDim.x + blockIdx.x] = v;
  }
}

// Start of the inner GMRES: beta = sqrt(rr[0]); V_0 = r / beta (0 when r = 0).
// Block 0 records st[0] = beta and brk[kInnerMax] = (beta == 0).
template <typename T>
__global__ __launch_bounds__(kBlock) void inner_start_kernel(int64_t n, const double* __restrict__ rr,
                                                             double* __restrict__ st, int* __restrict__ brk,
                                                             const T* __restrict__ r, T* __restrict__ v0) {
  const double b = sqrt(rr[0] > 0.0 ? rr[0] : 0.0);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st[0] = b;
    brk[kInnerMax] = b > 0.0 ? 0 : 1;
  }
  const double f = b > 0.0 ? 1.0 / b : 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    v0[i] = T(double(r[i]) * f);
}

// End of Arnoldi step j: column j of the Hessenberg matrix (column-major,
// leading dimension k + 1) from the two passes a1, a2 (a1[j + 1] = ||w||^2
// before them) and the final squared norm nn[0], written by block 0 with the
// step's breakdown flag brk[j] (an exact solve in the current space); every
// block normalises w = V_{j+1}, or zeroes it once a breakdown has happened
// (brk of earlier steps come from earlier launches).
template <typename T>
__global__ __launch_bounds__(kBlock) void inner_column_kernel(int64_t n, int j, int k, const double* __restrict__ a1,
                                                              const double* __restrict__ a2,
                                                              const double* __restrict__ nn,
                                                              double* __restrict__ H, int* __restrict__ brk,
                                                              T* __restrict__ w) {
  const double hn = sqrt(nn[0] > 0.0 ? nn[0] : 0.0);
  const double wb = sqrt(a1[j + 1] > 0.0 ? a1[j + 1] : 0.0);
  const bool here = !(hn > 1e-14 * wb);
  bool before = brk[kInnerMax] != 0;
  for (int i = 0; i < j; ++i) before = before || brk[i] != 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double* col = H + int64_t(j) * (k + 1);
    for (int i = 0; i <= j; ++i) col[i] = a1[i] + a2[i];
    col[j + 1] = hn;
    brk[j] = here ? 1 : 0;
  }
  const double f = (before || here) ? 0.0 : 1.0 / hn;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    w[i] = T(double(w[i]) * f);
}

// Least squares min ||beta e_1 - Hbar y|| over the first m columns (m: k, or
// the step of the first breakdown + 1, or 0 when beta = 0) by Givens
// rotations and back substitution, y_j = 0 for j >= m; one thread, its work
// arrays in LDS.
struct InnerLsqWork {
  double R[kInnerMax + 1][kInnerMax];
  double g[kInnerMax + 1], cs[kInnerMax], sn[kInnerMax];
};

__device__ void inner_lsq(int k, const double* __restrict__ H, double beta, const int* __restrict__ brk,
                          InnerLsqWork& wk, double* __restrict__ y) {
  auto& R = wk.R;
  double* g = wk.g;
  double* cs = wk.cs;
  double* sn = wk.sn;
  int m = brk[kInnerMax] ? 0 : k;
  for (int j = 0; j < m; ++j)
    if (brk[j]) { m = j + 1; break; }
  for (int j = 0; j <= k; ++j) g[j] = 0.0;
  g[0] = beta;
  for (int j = 0; j < m; ++j) {
    for (int i = 0; i <= j + 1; ++i) R[i][j] = H[int64_t(j) * (k + 1) + i];
    for (int i = 0; i < j; ++i) {
      const double a = R[i][j], b = R[i + 1][j];
      R[i][j] = cs[i] * a + sn[i] * b;
      R[i + 1][j] = -sn[i] * a + cs[i] * b;
    }
    const double a = R[j][j], b = R[j + 1][j];
    const double r = sqrt(a * a + b * b);
    cs[j] = r > 0.0 ? a / r : 1.0;
    sn[j] = r > 0.0 ? b / r : 0.0;
    R[j][j] = r;
    R[j + 1][j] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
  }
  for (int j = k - 1; j >= 0; --j) {
    if (j >= m) { y[j] = 0.0; continue; }
    double t = g[j];
    for (int i = j + 1; i < m; ++i) t -= R[j][i] * y[i];
    y[j] = R[j][j] != 0.0 ? t / R[j][j] : 0.0;
  }
}

// z = sum_{i < k} y_i Z_i with y from the least squares above (each block
// solves the (k + 1) x k problem itself in LDS: no extra launch).
template <typename T>
__global__ __launch_bounds__(kBlock) void inner_combine_kernel(int64_t n, int k, const T* __restrict__ Z, int64_t ld,
                                                               const double* __restrict__ H,
                                                               const double* __restrict__ st,
                                                               const int* __restrict__ brk, T* __restrict__ z) {
  __shared__ double ys[kInnerMax];
  __shared__ InnerLsqWork wk;
  if (threadIdx.x == 0) inner_lsq(k, H, st[0], brk, wk, ys);
  __syncthreads();
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock) {
    double s = 0.0;
    for (int q = 0; q < k; ++q) s += ys[q] * double(Z[q * ld + i]);
    z[i] = T(s);
  }
}

// Non-finite check: flag[0] = 1 if any x_i is NaN or Inf.
__global__ __launch_bounds__(kBlock) void nonfinite_kernel(int64_t n, const double* __restrict__ x,
                                                            int* __restrict__ flag) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    if (!isfinite(x[i])) atomicOr(flag, 1);
}

// Sums of squares of three consecutive segments of x (bounds[0..3]): blocks
// [s * nb, (s + 1) * nb) stride over segment s; each block writes its partial
// (tree in LDS, fixed order) to part[block].  The host adds the nb partials of
// a segment in block order, so the result does not depend on timing.
__global__ __launch_bounds__(kBlock) void sumsq3_kernel(const double* __restrict__ x, int64_t b0, int64_t b1,
                                                        int64_t b2, int64_t b3, int nb, double* __restrict__ part) {
  __shared__ double red[kBlock];
  const int seg = blockIdx.x / nb;
  const int64_t lo = seg == 0 ? b0 : (seg == 1 ? b1 : b2);
  const int64_t hi = seg == 0 ? b1 : (seg == 1 ? b2 : b3);
  double acc = 0.0;
  for (int64_t i = lo + int64_t(blockIdx.x % nb) * kBlock + threadIdx.x; i < hi; i += int64_t(nb) * kBlock)
    acc += x[i] * x[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (int(threadIdx.x) < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

}  // namespace fsi
