// Per-node MLP smoother on CDNA4 matrix cores (BF16 MFMA, FP32 accumulate).
//
// The learned part replaces the first (pre-)smoothing sweep on the finest
// level of the mesh-motion and solid-Schur hierarchies.  For node i the input
// z_i holds the Jacobi-scaled residual D^{-1} b at the 3^d lattice nodes
// around i (d components each, zero where a neighbour is not an unknown of the
// operator); the output is the correction at node i:
//     delta = W3^T relu(W2^T relu(W1^T z))      (bias-free: delta(a z) = a delta(z))
//
// All products are evaluated transposed, H^T = W^T Z^T, with
// v_mfma_f32_16x16x16_bf16 on 16-node tiles (one tile per wavefront).  With
// lane l = 16 q + n (n = l % 16, q = l / 16) the operands are
//     A[m][k]: lane holds A[n][4q + j], j = 0..3
//     B[k][c]: lane holds B[4q + j][n]
//     D[m][c]: lane holds D[4q + i][n], i = 0..3
// so the output of one layer (rows = hidden units, columns = nodes) is, lane
// by lane, already the B operand of the next layer: no data exchange between
// layers.  The weight gradients contract over the nodes of a tile and go
// through LDS.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fsi {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);  // NaN stays NaN
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float(uint32_t(h) << 16); }

__device__ __forceinline__ f32x4_t mfma16(bf16x4_t a, bf16x4_t b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

template <int D>
struct MlpDims {
  static constexpr int S = D == 2 ? 9 : 27;  // stencil nodes
  static constexpr int KIN = S * D;          // inputs per node
  static constexpr int KP = D == 2 ? 32 : 96;  // padded to whole 16-blocks
  static constexpr int KB = KP / 16;
  static constexpr int H = 64;                 // hidden width
  static constexpr int HB = H / 16;
  static constexpr int NP = 16;                // padded outputs
  static constexpr int NPARAM = KP * H + H * H + H * NP;
};

// Device weights, BF16, in the layouts the fragments read contiguously:
//   w1t [H][KP]  (W1 transposed)      w2t [H][H] (W2 transposed: [out][in])
//   w2  [H][H]   (W2: [in][out])      w3t [NP][H] (W3 transposed, rows >= d zero)
//   w3  [H][NP]  (W3: [hid][c], columns >= d zero)
struct MlpW {
  const unsigned short *w1t, *w2t, *w2, *w3t, *w3;
};

// Order the LDS writes of a wavefront before its other lanes read them (the
// waves of a block run different numbers of tiles, so no block barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ bf16x4_t load4(const unsigned short* p) {
  return *reinterpret_cast<const bf16x4_t*>(p);
}

// Weight fragments of one lane, loaded once and kept in registers (inference).
template <int D>
struct MlpFrag {
  using M = MlpDims<D>;
  bf16x4_t w1[M::HB][M::KB], w2[M::HB][M::HB], w3[M::HB];
  __device__ __forceinline__ void load(const MlpW& w, int n, int q) {
#pragma unroll
    for (int mb = 0; mb < M::HB; ++mb) {
#pragma unroll
      for (int kb = 0; kb < M::KB; ++kb) w1[mb][kb] = load4(w.w1t + (16 * mb + n) * M::KP + 16 * kb + 4 * q);
#pragma unroll
      for (int kb = 0; kb < M::HB; ++kb) w2[mb][kb] = load4(w.w2t + (16 * mb + n) * M::H + 16 * kb + 4 * q);
      w3[mb] = load4(w.w3t + n * M::H + 16 * mb + 4 * q);
    }
  }
};

// Forward of one 16-node tile given the input fragments zf[kb] (B layout:
// lane holds z[node n][k = 16 kb + 4 q + j]).  Keeps the pre-activations
// (for the ReLU masks) and the BF16 activation fragments.  The weight
// fragments come from f1(mb, kb), f2(mb, kb), f3(kb) (A layout).
template <int D>
struct MlpTile {
  using M = MlpDims<D>;
  f32x4_t a1[M::HB], a2[M::HB], y;
  bf16x4_t h1[M::HB], h2[M::HB];

  template <class F1, class F2, class F3>
  __device__ __forceinline__ void run(const F1& f1, const F2& f2, const F3& f3, const bf16x4_t* zf) {
#pragma unroll
    for (int mb = 0; mb < M::HB; ++mb) {
      f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < M::KB; ++kb) acc = mfma16(f1(mb, kb), zf[kb], acc);
      a1[mb] = acc;
#pragma unroll
      for (int i = 0; i < 4; ++i) h1[mb][i] = short(f2bf(acc[i] > 0.f ? acc[i] : 0.f));
    }
#pragma unroll
    for (int mb = 0; mb < M::HB; ++mb) {
      f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < M::HB; ++kb) acc = mfma16(f2(mb, kb), h1[kb], acc);
      a2[mb] = acc;
#pragma unroll
      for (int i = 0; i < 4; ++i) h2[mb][i] = short(f2bf(acc[i] > 0.f ? acc[i] : 0.f));
    }
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < M::HB; ++kb) acc = mfma16(f3(kb), h2[kb], acc);
    y = acc;  // lane holds y[node n][c = 4 q + i]; only q == 0, i < D are outputs
  }

  // weights read from memory as they are needed (training: registers are short)
  __device__ __forceinline__ void forward(const MlpW& w, const bf16x4_t* zf, int n, int q) {
    run([&](int mb, int kb) { return load4(w.w1t + (16 * mb + n) * M::KP + 16 * kb + 4 * q); },
        [&](int mb, int kb) { return load4(w.w2t + (16 * mb + n) * M::H + 16 * kb + 4 * q); },
        [&](int kb) { return load4(w.w3t + n * M::H + 16 * kb + 4 * q); }, zf);
  }
  __device__ __forceinline__ void forward(const MlpFrag<D>& f, const bf16x4_t* zf) {
    run([&](int mb, int kb) { return f.w1[mb][kb]; }, [&](int mb, int kb) { return f.w2[mb][kb]; },
        [&](int kb) { return f.w3[kb]; }, zf);
  }
};

// Input k (= s D + c) of node `node`: component c of D^{-1} b at stencil node s.
template <int D, bool PER_DOF, typename T>
__device__ __forceinline__ float node_input(int64_t node, int k, const int32_t* __restrict__ nbr,
                                            const T* __restrict__ b, const T* __restrict__ dinv) {
  using M = MlpDims<D>;
  if (k >= M::KIN) return 0.f;
  const int s = k / D, c = k % D;
  const int32_t nb = nbr[node * M::S + s];
  if (nb < 0) return 0.f;
  return float((PER_DOF ? dinv[int64_t(nb) * D + c] : dinv[nb]) * b[int64_t(nb) * D + c]);
}

// Inference over the nodes of an operator: x[node * D + c] = delta_c(z_node),
// z from b through the stencil table nbr [n][S] (-1: no neighbour) and the
// inverse diagonal (per node when PER_DOF is false: the scalar Laplacian
// acting on D interleaved components; per dof otherwise).  Each wavefront
// loads the weights once and walks 16-node tiles with a grid stride.
template <int D, bool PER_DOF, typename T>
__global__ __launch_bounds__(256) void mlp_infer_kernel(int64_t n_nodes, const int32_t* __restrict__ nbr,
                                                         const T* __restrict__ b, const T* __restrict__ dinv,
                                                         MlpW w, T* __restrict__ x,
                                                         const int* __restrict__ streak = nullptr, int limit = 0) {
  if (streak && streak[0] >= limit) return;  // the solver stopped trying the network
  using M = MlpDims<D>;
  const int lane = threadIdx.x % 64, n = lane % 16, q = lane / 16;
  const int64_t ntiles = (n_nodes + 15) / 16, nwaves = int64_t(gridDim.x) * 4;
  int64_t tile = int64_t(blockIdx.x) * 4 + threadIdx.x / 64;
  if (tile >= ntiles) return;  // whole wave leaves together
  MlpFrag<D> f;
  f.load(w, n, q);
  for (; tile < ntiles; tile += nwaves) {
    const int64_t node = tile * 16 + n;
    bf16x4_t zf[M::KB];
#pragma unroll
    for (int kb = 0; kb < M::KB; ++kb)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        zf[kb][j] = short(f2bf(node < n_nodes ? node_input<D, PER_DOF, T>(node, 16 * kb + 4 * q + j, nbr, b, dinv) : 0.f));
    MlpTile<D> t;
    t.forward(f, zf);
    if (q == 0 && node < n_nodes)
#pragma unroll
      for (int i = 0; i < D; ++i) x[node * D + i] = T(t.y[i]);
  }
}

// Blocks of mlp_infer_kernel for n nodes: one tile per wave (the gathers of
// all tiles in flight at once) up to 4096 blocks.
inline unsigned mlp_infer_grid(int64_t n_nodes) {
  const int64_t blocks = ((n_nodes + 15) / 16 + 3) / 4;
  return unsigned(blocks < 1 ? 1 : (blocks > 4096 ? 4096 : blocks));
}

// Forward over m stored input rows (Z [m][KP] BF16): y[row * D + c].
template <int D, typename T>
__global__ __launch_bounds__(256) void mlp_forward_rows_kernel(int64_t m, const unsigned short* __restrict__ Z, MlpW w,
                                                                T* __restrict__ y) {
  using M = MlpDims<D>;
  const int lane = threadIdx.x % 64, n = lane % 16, q = lane / 16;
  const int64_t tile = int64_t(blockIdx.x) * 4 + threadIdx.x / 64;
  const int64_t row = tile * 16 + n;
  if (tile * 16 >= m) return;
  bf16x4_t zf[M::KB];
#pragma unroll
  for (int kb = 0; kb < M::KB; ++kb) {
    if (row < m) zf[kb] = load4(Z + row * M::KP + 16 * kb + 4 * q);
    else zf[kb] = bf16x4_t{0, 0, 0, 0};
  }
  MlpTile<D> t;
  t.forward(w, zf, n, q);
  if (q == 0 && row < m)
#pragma unroll
    for (int i = 0; i < D; ++i) y[row * D + i] = T(t.y[i]);
}

// Training: loss and weight gradients of (coef) * sum_s w_s ||delta(z_s) - e_s||^2
// over the samples of this launch.  Z: [m][KP] BF16 rows (zero padded),
// E: [m][D], wgt: [m].  Each wavefront takes `tiles_per_wave` consecutive
// 16-sample tiles starting at sample `first`, accumulates its gradient in
// registers and writes it to part[wave][NPARAM] (layouts [k][hid], [in][out],
// [hid][NP]) plus its loss to part_loss[wave].
// With GIVEN, E holds dL/dy itself (scaled by coef) and wgt is unused.
template <int D, bool GIVEN>
__global__ __launch_bounds__(256) void mlp_train_kernel(int64_t first, int64_t m, int tiles_per_wave,
                                                         const unsigned short* __restrict__ Z,
                                                         const float* __restrict__ E, const float* __restrict__ wgt,
                                                         float coef, MlpW w, float* __restrict__ part,
                                                         float* __restrict__ part_loss) {
  using M = MlpDims<D>;
  constexpr int ROWS = M::KP + 4 * M::H + 16;  // zT | h1T | h2T | da1T | da2T | dyT, 16 nodes each
  __shared__ unsigned short lds[4][ROWS * 16];
  const int wv = threadIdx.x / 64, lane = threadIdx.x % 64, n = lane % 16, q = lane / 16;
  unsigned short* zT = lds[wv];
  unsigned short* h1T = zT + M::KP * 16;
  unsigned short* h2T = h1T + M::H * 16;
  unsigned short* da1T = h2T + M::H * 16;
  unsigned short* da2T = da1T + M::H * 16;
  unsigned short* dyT = da2T + M::H * 16;
  const int64_t wave = int64_t(blockIdx.x) * 4 + wv;
  f32x4_t g1[M::KB][M::HB], g2[M::HB][M::HB], g3[M::HB];
#pragma unroll
  for (int a = 0; a < M::KB; ++a)
#pragma unroll
    for (int c = 0; c < M::HB; ++c) g1[a][c] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int a = 0; a < M::HB; ++a) {
    g3[a] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < M::HB; ++c) g2[a][c] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  }
  float lsum = 0.f;
  for (int t = 0; t < tiles_per_wave; ++t) {
    const int64_t s0 = first + (wave * tiles_per_wave + t) * 16;
    if (s0 >= first + m) break;
    const int64_t smp = s0 + n;
    const bool valid = smp < first + m;
    bf16x4_t zf[M::KB];
#pragma unroll
    for (int kb = 0; kb < M::KB; ++kb) {
      if (valid) zf[kb] = load4(Z + smp * M::KP + 16 * kb + 4 * q);
      else zf[kb] = bf16x4_t{0, 0, 0, 0};
#pragma unroll
      for (int j = 0; j < 4; ++j) zT[(16 * kb + 4 * q + j) * 16 + n] = (unsigned short)zf[kb][j];
    }
    MlpTile<D> tl;
    tl.forward(w, zf, n, q);
    // dY^T: lane holds dy[node n][c = 4 q + i]
    f32x4_t dy = {0.f, 0.f, 0.f, 0.f};
    if (q == 0 && valid) {
      if (GIVEN) {
#pragma unroll
        for (int i = 0; i < D; ++i) dy[i] = coef * E[smp * D + i];
      } else {
        const float ws = wgt[smp];
#pragma unroll
        for (int i = 0; i < D; ++i) {
          const float r = tl.y[i] - E[smp * D + i];
          lsum += ws * r * r;
          dy[i] = coef * ws * r;
        }
      }
    }
    bf16x4_t dyf;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      dyf[i] = short(f2bf(dy[i]));
      dyT[(4 * q + i) * 16 + n] = (unsigned short)dyf[i];
    }
    // dA2^T = (W3 dY^T) .* [a2 > 0]
    bf16x4_t da2[M::HB];
#pragma unroll
    for (int mb = 0; mb < M::HB; ++mb) {
      f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
      acc = mfma16(load4(w.w3 + (16 * mb + n) * M::NP + 4 * q), dyf, acc);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        da2[mb][i] = short(f2bf(tl.a2[mb][i] > 0.f ? acc[i] : 0.f));
        const int r = 16 * mb + 4 * q + i;
        da2T[r * 16 + n] = (unsigned short)da2[mb][i];
        h2T[r * 16 + n] = (unsigned short)tl.h2[mb][i];
        h1T[r * 16 + n] = (unsigned short)tl.h1[mb][i];
      }
    }
    // dA1^T = (W2 dA2^T) .* [a1 > 0]
#pragma unroll
    for (int mb = 0; mb < M::HB; ++mb) {
      f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < M::HB; ++kb) acc = mfma16(load4(w.w2 + (16 * mb + n) * M::H + 16 * kb + 4 * q), da2[kb], acc);
#pragma unroll
      for (int i = 0; i < 4; ++i) da1T[(16 * mb + 4 * q + i) * 16 + n] = f2bf(tl.a1[mb][i] > 0.f ? acc[i] : 0.f);
    }
    wave_sync();
    // weight gradients, contracting over the 16 nodes of the tile:
    //   dW1 += Z^T dA1, dW2 += H1^T dA2, dW3 += H2^T dY
#pragma unroll
    for (int nb = 0; nb < M::HB; ++nb) {
      const bf16x4_t bda1 = load4(da1T + (16 * nb + n) * 16 + 4 * q);
      const bf16x4_t bda2 = load4(da2T + (16 * nb + n) * 16 + 4 * q);
#pragma unroll
      for (int mb = 0; mb < M::KB; ++mb) g1[mb][nb] = mfma16(load4(zT + (16 * mb + n) * 16 + 4 * q), bda1, g1[mb][nb]);
#pragma unroll
      for (int mb = 0; mb < M::HB; ++mb) g2[mb][nb] = mfma16(load4(h1T + (16 * mb + n) * 16 + 4 * q), bda2, g2[mb][nb]);
    }
    const bf16x4_t bdy = load4(dyT + n * 16 + 4 * q);
#pragma unroll
    for (int mb = 0; mb < M::HB; ++mb) g3[mb] = mfma16(load4(h2T + (16 * mb + n) * 16 + 4 * q), bdy, g3[mb]);
    wave_sync();  // the next tile overwrites this wave's LDS rows
  }
  float* out = part + wave * M::NPARAM;
#pragma unroll
  for (int mb = 0; mb < M::KB; ++mb)
#pragma unroll
    for (int nb = 0; nb < M::HB; ++nb)
#pragma unroll
      for (int i = 0; i < 4; ++i) out[(16 * mb + 4 * q + i) * M::H + 16 * nb + n] = g1[mb][nb][i];
  float* o2 = out + M::KP * M::H;
#pragma unroll
  for (int mb = 0; mb < M::HB; ++mb)
#pragma unroll
    for (int nb = 0; nb < M::HB; ++nb)
#pragma unroll
      for (int i = 0; i < 4; ++i) o2[(16 * mb + 4 * q + i) * M::H + 16 * nb + n] = g2[mb][nb][i];
  float* o3 = o2 + M::H * M::H;
#pragma unroll
  for (int mb = 0; mb < M::HB; ++mb)
#pragma unroll
    for (int i = 0; i < 4; ++i) o3[(16 * mb + 4 * q + i) * M::NP + n] = g3[mb][i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
  if (lane == 0) part_loss[wave] = lsum;
}

// Two-stage sum of the per-wave gradients in a fixed order: stage 1 adds the
// waves of chunk blockIdx.y (kGradChunks chunks of consecutive waves) into
// part2[chunk][p]; stage 2 adds the chunks in order into g[p].  Loss likewise.
constexpr int kGradChunks = 32;

__global__ __launch_bounds__(256) void mlp_grad_chunk_kernel(int nwaves, int nparam, const float* __restrict__ part,
                                                              const float* __restrict__ part_loss,
                                                              float* __restrict__ part2, float* __restrict__ loss2) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  const int per = (nwaves + kGradChunks - 1) / kGradChunks;
  const int w0 = blockIdx.y * per, w1 = min(nwaves, w0 + per);
  if (p < nparam) {
    float s = 0.f;
    for (int wv = w0; wv < w1; ++wv) s += part[int64_t(wv) * nparam + p];
    part2[int64_t(blockIdx.y) * nparam + p] = s;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    float s = 0.f;
    for (int wv = w0; wv < w1; ++wv) s += part_loss[wv];
    loss2[blockIdx.y] = s;
  }
}

__global__ __launch_bounds__(256) void mlp_grad_reduce_kernel(int nparam, const float* __restrict__ part2,
                                                               const float* __restrict__ loss2,
                                                               float* __restrict__ g, float* __restrict__ loss) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < nparam) {
    float s = 0.f;
    for (int c = 0; c < kGradChunks; ++c) s += part2[int64_t(c) * nparam + p];
    g[p] = s;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    float s = 0.f;
    for (int c = 0; c < kGradChunks; ++c) s += loss2[c];
    loss[0] = s;
  }
}

// Adam on the FP32 master weights (layouts [k][hid], [in][out], [hid][NP];
// padded entries are kept at zero), then the BF16 fragment copies.
template <int D>
__global__ __launch_bounds__(256) void mlp_adam_kernel(float* __restrict__ wm, float* __restrict__ mom1,
                                                        float* __restrict__ mom2, const float* __restrict__ g,
                                                        float lr, float b1, float b2, float eps, float bc1, float bc2,
                                                        unsigned short* w1t, unsigned short* w2t, unsigned short* w2,
                                                        unsigned short* w3t, unsigned short* w3) {
  using M = MlpDims<D>;
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= M::NPARAM) return;
  bool live;
  if (p < M::KP * M::H) live = p / M::H < M::KIN;
  else if (p < M::KP * M::H + M::H * M::H) live = true;
  else live = (p - M::KP * M::H - M::H * M::H) % M::NP < D;
  float wv = 0.f;
  if (live) {
    const float gg = g[p];
    const float m1 = b1 * mom1[p] + (1.f - b1) * gg;
    const float m2 = b2 * mom2[p] + (1.f - b2) * gg * gg;
    mom1[p] = m1;
    mom2[p] = m2;
    wv = wm[p] - lr * (m1 / bc1) / (sqrtf(m2 / bc2) + eps);
    wm[p] = wv;
  }
  const unsigned short h = f2bf(wv);
  if (p < M::KP * M::H) {
    const int k = p / M::H, hid = p % M::H;
    w1t[hid * M::KP + k] = h;
  } else if (p < M::KP * M::H + M::H * M::H) {
    const int q = p - M::KP * M::H, in = q / M::H, out = q % M::H;
    w2[in * M::H + out] = h;
    w2t[out * M::H + in] = h;
  } else {
    const int q = p - M::KP * M::H - M::H * M::H, hid = q / M::NP, c = q % M::NP;
    w3[hid * M::NP + c] = h;
    w3t[c * M::H + hid] = h;
  }
}

// Training samples of one recorded residual b with its exact correction e:
// Z row = scale * z(b) in BF16 (zero padded to KP), E row = scale * e, and the
// weight of the node (its mean diagonal entry relative to the operator's
// mean, precomputed on the host in wnode).
template <int D, bool PER_DOF, typename T>
__global__ __launch_bounds__(256) void mlp_samples_kernel(int64_t n_nodes, const int32_t* __restrict__ nbr,
                                                           const T* __restrict__ b, const T* __restrict__ dinv,
                                                           const double* __restrict__ e, const float* __restrict__ wnode,
                                                           float scale, unsigned short* __restrict__ Z,
                                                           float* __restrict__ E, float* __restrict__ W) {
  using M = MlpDims<D>;
  const int64_t node = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (node >= n_nodes) return;
  for (int k = 0; k < M::KP; ++k) Z[node * M::KP + k] = f2bf(scale * node_input<D, PER_DOF, T>(node, k, nbr, b, dinv));
  for (int c = 0; c < D; ++c) E[node * D + c] = scale * float(e[node * D + c]);
  W[node] = wnode[node];
}

// Network inputs of every node for one residual b: Z [n][KP] BF16.
template <int D, bool PER_DOF, typename T>
__global__ __launch_bounds__(256) void mlp_inputs_kernel(int64_t n_nodes, const int32_t* __restrict__ nbr,
                                                          const T* __restrict__ b, const T* __restrict__ dinv,
                                                          unsigned short* __restrict__ Z) {
  using M = MlpDims<D>;
  const int64_t node = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (node >= n_nodes) return;
  for (int k = 0; k < M::KP; ++k) Z[node * M::KP + k] = f2bf(node_input<D, PER_DOF, T>(node, k, nbr, b, dinv));
}

// Rows `perm` of a sample set into a shuffled copy.
template <int KP, int D>
__global__ __launch_bounds__(256) void mlp_gather_samples_kernel(int64_t m, const int64_t* __restrict__ perm,
                                                                  const unsigned short* __restrict__ Zi,
                                                                  const float* __restrict__ Ei, const float* __restrict__ Wi,
                                                                  unsigned short* __restrict__ Zo, float* __restrict__ Eo,
                                                                  float* __restrict__ Wo) {
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (i >= m) return;
  const int64_t s = perm[i];
  for (int k = 0; k < KP; ++k) Zo[i * KP + k] = Zi[s * KP + k];
  for (int c = 0; c < D; ++c) Eo[i * D + c] = Ei[s * D + c];
  Wo[i] = Wi[s];
}

// Per-block partial sums of r.r and b.b (exact corrections' convergence test).
constexpr int kNormBlocks = 256;

template <typename T>
__global__ __launch_bounds__(256) void norm_pair_partial_kernel(int64_t n, const T* __restrict__ r,
                                                                 const T* __restrict__ b, double* __restrict__ part) {
  __shared__ double sh[2][4];
  double rr = 0.0, bb = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const double ri = double(r[i]), bi = double(b[i]);
    rr += ri * ri;
    bb += bi * bi;
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
    part[2 * blockIdx.x] = sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3];
    part[2 * blockIdx.x + 1] = sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3];
  }
}

}  // namespace fsi
