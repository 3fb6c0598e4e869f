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

namespace fsi {

constexpr int kBlock = 256;

// ------------------------------------------------------------ CSR products
template <typename T, int NV>
struct GatherPlain {
  const T* x;
  __device__ __forceinline__ T operator()(int32_t c, int n) const { return x[int64_t(c) * NV + n]; }
};

// x_j = omega * dinv_j * b_j formed on the fly (first pre-smoothing sweep
// from a zero initial guess).
template <typename T, int NV>
struct GatherJacobi0 {
  const T* b;
  const T* dinv;
  T omega;
  __device__ __forceinline__ T operator()(int32_t c, int n) const {
    return omega * dinv[c] * b[int64_t(c) * NV + n];
  }
};

template <typename T, int NV>
struct EpiStore {  // y = A x
  T* y;
  __device__ __forceinline__ void operator()(int64_t i, const T* acc) const {
#pragma unroll
    for (int n = 0; n < NV; ++n) y[i * NV + n] = acc[n];
  }
};

template <typename T, int NV>
struct EpiSub {  // y = r - A x   (y may alias r)
  const T* r;
  T* y;
  __device__ __forceinline__ void operator()(int64_t i, const T* acc) const {
#pragma unroll
    for (int n = 0; n < NV; ++n) y[i * NV + n] = r[i * NV + n] - acc[n];
  }
};

template <typename T, int NV>
struct EpiAcc {  // y += A x
  T* y;
  __device__ __forceinline__ void operator()(int64_t i, const T* acc) const {
#pragma unroll
    for (int n = 0; n < NV; ++n) y[i * NV + n] = y[i * NV + n] + acc[n];
  }
};

// Pre-smoothing from zero: x = omega D^{-1} b and r = b - A x in one pass.
template <typename T, int NV>
struct EpiJacobi0 {
  const T* b;
  const T* dinv;
  T omega;
  T* x;
  T* r;
  __device__ __forceinline__ void operator()(int64_t i, const T* acc) const {
    const T wd = omega * dinv[i];
#pragma unroll
    for (int n = 0; n < NV; ++n) {
      const T bi = b[i * NV + n];
      x[i * NV + n] = wd * bi;
      r[i * NV + n] = bi - acc[n];
    }
  }
};

// Post-smoothing: y = x + omega D^{-1} (b - A x).  y must not alias x.
template <typename T, int NV>
struct EpiJacobiPost {
  const T* b;
  const T* x;
  const T* dinv;
  T omega;
  T* y;
  __device__ __forceinline__ void operator()(int64_t i, const T* acc) const {
    const T wd = omega * dinv[i];
#pragma unroll
    for (int n = 0; n < NV; ++n) y[i * NV + n] = x[i * NV + n] + wd * (b[i * NV + n] - acc[n]);
  }
};

template <typename T, int G, int NV, class Gather, class Epi>
__global__ __launch_bounds__(kBlock) void csr_rows_kernel(int64_t nrows, const int64_t* __restrict__ rp,
                                                           const int32_t* __restrict__ ci,
                                                           const T* __restrict__ val, Gather gx, Epi epi) {
  constexpr int RPB = kBlock / G;  // rows per block
  const int64_t row = int64_t(blockIdx.x) * RPB + threadIdx.x / G;
  const int lane = threadIdx.x % G;
  if (row >= nrows) return;  // whole groups leave together (G divides 64)
  T acc[NV];
#pragma unroll
  for (int n = 0; n < NV; ++n) acc[n] = T(0);
  const int64_t b = rp[row], e = rp[row + 1];
  int64_t k = b + lane;
  // two entries in flight per lane
  for (; k + G < e; k += 2 * G) {
    const int32_t c0 = ci[k], c1 = ci[k + G];
    const T a0 = val[k], a1 = val[k + G];
#pragma unroll
    for (int n = 0; n < NV; ++n) acc[n] += a0 * gx(c0, n) + a1 * gx(c1, n);
  }
  if (k < e) {
    const int32_t c0 = ci[k];
    const T a0 = val[k];
#pragma unroll
    for (int n = 0; n < NV; ++n) acc[n] += a0 * gx(c0, n);
  }
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1)
#pragma unroll
    for (int n = 0; n < NV; ++n) acc[n] += __shfl_xor(acc[n], off, G);
  if (lane == 0) epi(row, acc);
}

// -------------------------------------------------------------- coarse solve
// X = Ainv B with a dense row-major n x n inverse (FP64); one wavefront per
// row; B, X hold NV interleaved columns.  X must not alias B.
template <typename TI, typename TO, int NV>
__global__ __launch_bounds__(kBlock) void dense_gemv_kernel(int64_t n, const double* __restrict__ Ainv,
                                                             const TI* __restrict__ B, TO* __restrict__ X) {
  const int64_t row = int64_t(blockIdx.x) * (kBlock / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (row >= n) return;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  const double* a = Ainv + row * n;
  for (int64_t j = lane; j < n; j += 64) {
    const double aj = a[j];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += aj * double(B[j * NV + v]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += __shfl_xor(acc[v], off, 64);
  if (lane == 0)
#pragma unroll
    for (int v = 0; v < NV; ++v) X[row * NV + v] = TO(acc[v]);
}

// -------------------------------------------------------------- vector ops
template <typename T>
__global__ __launch_bounds__(kBlock) void vsub_kernel(int64_t n, T* __restrict__ y, const T* __restrict__ x) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    y[i] = y[i] - x[i];
}

template <typename TI, typename TO>
__global__ __launch_bounds__(kBlock) void cast_kernel(int64_t n, const TI* __restrict__ x, TO* __restrict__ y) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    y[i] = TO(x[i]);
}

// y *= f (in place)
__global__ __launch_bounds__(kBlock) void scale_kernel(int64_t n, double* y, double f) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    y[i] = y[i] * f;
}

// ---------------------------------------------------------- Gram-Schmidt
// Partial dots of w with nv basis vectors V_i (V_i = V + i * ld) plus w.w,
// over a fixed grid (deterministic), written to part[block * (nv + 1) + i].
constexpr int kGsBlocks = 512;
constexpr int kMaxBasis = 208;

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int wid = threadIdx.x / 64, lane = threadIdx.x % 64;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kBlock / 64; ++i) s += sh[i];
  return s;  // valid in thread 0
}

// mode 0: dots V_i . w and w . w
// mode 1: w -= sum_i h_i V_i, then dots V_i . w and w . w of the updated w
// mode 2: w -= sum_i h_i V_i, then only w . w (written at index nv)
__global__ __launch_bounds__(kBlock) void gs_pass_kernel(int64_t n, int nv, const double* __restrict__ V,
                                                          int64_t ld, double* __restrict__ w,
                                                          const double* __restrict__ h, int mode,
                                                          double* __restrict__ part) {
  __shared__ double sh[kBlock / 64];
  __shared__ double hs[kMaxBasis];
  if (mode != 0)
    for (int i = threadIdx.x; i < nv; i += kBlock) hs[i] = h[i];
  __syncthreads();
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = int64_t(blockIdx.x) * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  if (mode != 0) {
    for (int64_t k = lo + threadIdx.x; k < hi; k += kBlock) {
      double s = w[k];
      for (int i = 0; i < nv; ++i) s -= hs[i] * V[i * ld + k];
      w[k] = s;
    }
    __syncthreads();
  }
  for (int i = mode == 2 ? nv : 0; i <= nv; ++i) {
    const double* vi = i < nv ? V + i * ld : w;
    double s = 0.0;
    for (int64_t k = lo + threadIdx.x; k < hi; k += kBlock) s += vi[k] * w[k];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[int64_t(blockIdx.x) * (nv + 1) + i] = s;
  }
}

// out[i] = sum over blocks of part[b * (nv + 1) + i], fixed order.
__global__ __launch_bounds__(kBlock) void gs_reduce_kernel(int nblocks, int nv, const double* __restrict__ part,
                                                            double* __restrict__ out) {
  __shared__ double sh[kBlock / 64];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kBlock) s += part[int64_t(b) * (nv + 1) + i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[i] = s;
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

// Non-finite check: flag[0] = 1 if any x_i is NaN or Inf.
__global__ __launch_bounds__(kBlock) void nonfinite_kernel(int64_t n, const double* __restrict__ x,
                                                            int* __restrict__ flag) {
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += int64_t(gridDim.x) * kBlock)
    if (!isfinite(x[i])) atomicOr(flag, 1);
}

}  // namespace fsi
