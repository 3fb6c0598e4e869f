// C ABI of the MI355X FSI Jacobian solver: context, validation, device
// upload, the block-LDU preconditioner application and the FGMRES driver.
//
// Solve path (all on one HIP stream):
//   FGMRES(m), right preconditioned (flexible: z_j = P^{-1} v_j stored),
//   per iteration:
//     z_j = P^{-1} v_j      block LDU algorithm of Section 4.1 with the AMG
//                           sub-inverses of Sections 4.2-4.4
//     w   = A_h z_j         one CSR pass over the monolithic A_h
//     classical Gram-Schmidt with one reorthogonalisation (three fused passes)
//     j+2 FP64 scalars to the host for the Givens least squares
//   restart / acceptance on the recomputed FP64 true residual.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <memory>
#include <mutex>
#include <type_traits>
#include <new>
#include <random>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "../../include/fsi.h"
#include "host_csr.hpp"
#include "kernels.hpp"
#include "mlp.hpp"
#include "sa_setup.hpp"
#include "spgemm.hpp"
#include "fe_assembly.hpp"

// Staging of fsi_mlp_forward_noalloc: the FP32 copies of the residual and of
// the network's correction (kNoAllocStage entries each) in one array per GPU,
// so that the call allocates nothing.  The array lives as long as the process
// (32 MiB on each GPU the library runs on).  Host code must use its device
// address from hipGetSymbolAddress, never the symbol itself.
constexpr int64_t kNoAllocStage = int64_t(1) << 22;
static __device__ __align__(256) float scratch[2 * kNoAllocStage];

namespace fsi {

// ------------------------------------------------------------------ errors
struct Error : std::runtime_error {
  fsi_status code;
  Error(fsi_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIP_TRY(expr)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      throw ::fsi::Error(e_ == hipErrorOutOfMemory ? FSI_ERR_OOM : FSI_ERR_HIP,               \
                         std::string(#expr) + ": " + hipGetErrorString(e_));                  \
  } while (0)

// ------------------------------------------------------------------ logging
// FSI_LOG set (to anything but "0") in the environment: one stderr line per
// setup phase and per solve, with wall times (the phases are host work or end
// with a stream synchronisation, so the times are the phases' own).
inline bool log_on() {
  static const bool on = [] {
    const char* v = std::getenv("FSI_LOG");
    return v && std::strcmp(v, "0") != 0;
  }();
  return on;
}

__attribute__((format(printf, 1, 2))) inline void log_line(const char* fmt, ...) {
  if (!log_on()) return;
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  std::fprintf(stderr, "[fsi] %s\n", buf);
}

// Wall clock of a phase, logged when it ends.
struct PhaseTimer {
  const char* what;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  explicit PhaseTimer(const char* w) : what(w) {}
  double ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  void done(const char* extra = "") const { log_line("%s: %.1f ms%s", what, ms(), extra); }
};

// ---------------------------------------------------------- device memory
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  void alloc(size_t b) {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = b;
    if (b) HIP_TRY(hipMalloc(&p, b));
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

// ---------------------------------------------------------- host -> device
// Setup uploads: the source image is written, on the host threads, into one
// of two pinned staging buffers while the other one is in flight to the
// device; every upload has finished when the call returns, so the host source
// may be released right after.  fill(buf, off, n) writes bytes [off, off + n)
// of the destination image into buf (a copy, or a conversion to the device
// type); off and n are multiples of 8 except at the end of the image.
struct Staging {
  static constexpr size_t kChunk = size_t(32) << 20;
  std::mutex mu;
  char* buf[2] = {nullptr, nullptr};
  // bytes and wall time of the copies through the buffers (for the log)
  std::atomic<int64_t> up_bytes{0}, up_ns{0}, down_bytes{0}, down_ns{0};
};

inline Staging& staging() {
  // pinned once per process and kept until it ends
  static Staging* st = new Staging;
  return *st;
}

template <class Fill>
void staged_upload(void* dst, size_t bytes, hipStream_t s, Fill&& fill) {
  if (bytes == 0) return;
  constexpr size_t kPiece = size_t(1) << 20;  // bytes per host thread item
  if (bytes <= kPiece) {
    std::vector<char> tmp(bytes);
    fill(tmp.data(), 0, bytes);
    HIP_TRY(hipMemcpyAsync(dst, tmp.data(), bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return;
  }
  Staging& st = staging();
  std::lock_guard<std::mutex> lock(st.mu);
  const auto t0 = std::chrono::steady_clock::now();
  for (auto& b : st.buf)
    if (!b) HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&b), Staging::kChunk, hipHostMallocPortable));
  struct Events {  // both buffers idle again on any exit
    hipEvent_t e[2] = {nullptr, nullptr};
    hipStream_t s;
    ~Events() {
      (void)hipStreamSynchronize(s);
      for (auto& x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } ev{{nullptr, nullptr}, s};
  for (auto& e : ev.e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  bool busy[2] = {false, false};
  for (size_t off = 0, c = 0; off < bytes; off += Staging::kChunk, ++c) {
    const int b = int(c & 1);
    const size_t n = std::min(Staging::kChunk, bytes - off);
    if (busy[b]) HIP_TRY(hipEventSynchronize(ev.e[b]));
    char* buf = st.buf[b];
    parallel_for(int64_t((n + kPiece - 1) / kPiece), [&](int64_t p0, int64_t p1) {
      const size_t a = size_t(p0) * kPiece, z = std::min(n, size_t(p1) * kPiece);
      fill(buf + a, off + a, z - a);
    }, 2);
    HIP_TRY(hipMemcpyAsync(static_cast<char*>(dst) + off, buf, n, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(ev.e[b], s));
    busy[b] = true;
  }
  HIP_TRY(hipStreamSynchronize(s));
  st.up_bytes += int64_t(bytes);
  st.up_ns += std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0).count();
}

// count elements of src to dst (same type)
template <typename U>
void h2d(void* dst, const U* src, size_t count, hipStream_t s) {
  staged_upload(dst, sizeof(U) * count, s, [src](char* buf, size_t off, size_t n) {
    std::memcpy(buf, reinterpret_cast<const char*>(src) + off, n);
  });
}

// count FP64 values of src to dst as T (rounded to nearest when T is float)
template <typename T>
void h2d_as(void* dst, const double* src, size_t count, hipStream_t s) {
  if constexpr (std::is_same_v<T, double>) {
    h2d(dst, src, count, s);
  } else {
    staged_upload(dst, sizeof(T) * count, s, [src](char* buf, size_t off, size_t n) {
      T* o = reinterpret_cast<T*>(buf);
      const double* x = src + off / sizeof(T);
      for (size_t i = 0; i < n / sizeof(T); ++i) o[i] = T(x[i]);
    });
  }
}

// count elements of device array src to host array dst, through the same
// staging buffers (filled by the DMA engine, emptied on the host threads)
template <typename U>
void d2h(U* dst, const void* src, size_t count, hipStream_t s) {
  const size_t bytes = sizeof(U) * count;
  if (bytes == 0) return;
  constexpr size_t kPiece = size_t(1) << 20;
  if (bytes <= kPiece) {
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return;
  }
  Staging& st = staging();
  std::lock_guard<std::mutex> lock(st.mu);
  const auto t0 = std::chrono::steady_clock::now();
  for (auto& b : st.buf)
    if (!b) HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&b), Staging::kChunk, hipHostMallocPortable));
  auto drain = [&](int b, size_t off, size_t n) {
    char* out = reinterpret_cast<char*>(dst) + off;
    const char* buf = st.buf[b];
    parallel_for(int64_t((n + kPiece - 1) / kPiece), [&](int64_t p0, int64_t p1) {
      const size_t a = size_t(p0) * kPiece, z = std::min(n, size_t(p1) * kPiece);
      std::memcpy(out + a, buf + a, z - a);
    }, 2);
  };
  struct Events {
    hipEvent_t e[2] = {nullptr, nullptr};
    hipStream_t s;
    ~Events() {
      (void)hipStreamSynchronize(s);
      for (auto& x : e)
        if (x) (void)hipEventDestroy(x);
    }
  } ev{{nullptr, nullptr}, s};
  for (auto& e : ev.e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  size_t prev_off = 0, prev_n = 0;
  int prev_b = -1;
  for (size_t off = 0, c = 0; off < bytes; off += Staging::kChunk, ++c) {
    const int b = int(c & 1);
    const size_t n = std::min(Staging::kChunk, bytes - off);
    HIP_TRY(hipMemcpyAsync(st.buf[b], static_cast<const char*>(src) + off, n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipEventRecord(ev.e[b], s));
    if (prev_b >= 0) {
      HIP_TRY(hipEventSynchronize(ev.e[prev_b]));
      drain(prev_b, prev_off, prev_n);
    }
    prev_b = b;
    prev_off = off;
    prev_n = n;
  }
  HIP_TRY(hipEventSynchronize(ev.e[prev_b]));
  drain(prev_b, prev_off, prev_n);
  st.down_bytes += int64_t(bytes);
  st.down_ns += std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0).count();
}

// Log line of the staged copies so far.
void log_staging(const char* when) {
  if (!log_on()) return;
  const Staging& st = staging();
  log_line("%s: staged copies %.2f GB up in %.1f ms, %.2f GB down in %.1f ms", when, st.up_bytes.load() / 1e9,
           st.up_ns.load() / 1e6, st.down_bytes.load() / 1e9, st.down_ns.load() / 1e6);
}

template <typename T>
struct DCsr {
  int64_t nrows = 0, ncols = 0, nnz = 0;
  int group = 8;
  bool deep = false;  // four entries in flight per lane (large streamed matrices)
  RowSegments seg{};  // nseg > 0: row segments with their own lanes per row
  std::shared_ptr<DevBuf> rp, ci, val;
  std::shared_ptr<DevBuf> grp_rp[4], grp_ci[4], grp_val[4];  // grouped segments
  double seg_bytes = 0.0;  // segmented matrices: bytes of the matrix as stored
  int rgroup = 1;          // > 1: rows stored in groups of rgroup (nnz counts column-list entries)
  const int64_t* drp() const { return rp ? rp->as<int64_t>() : nullptr; }
  const int32_t* dci() const { return ci ? ci->as<int32_t>() : nullptr; }
  const T* dval() const { return val ? val->as<T>() : nullptr; }
  double bytes() const {
    if (seg.nseg > 0) return seg_bytes;
    if (rgroup > 1) return double(nnz) * (4.0 + sizeof(T) * rgroup) + double(nrows / rgroup + 1) * 8;
    return double(nnz) * (sizeof(T) + 4) + double(nrows + 1) * 8;
  }
};

// Lanes per row of a CSR product: the smallest power of two in [4, 64] with
// `per_lane` x lanes >= the mean row length.  Small matrices take 3 entries
// per lane (short latency chains); the monolithic A_h product, a pure HBM
// stream, takes 8 (measured best on the 2D and 3D workloads).
int pick_group(int64_t nnz, int64_t nrows, int per_lane = 3) {
  const double avg = nrows ? double(nnz) / double(nrows) : 1.0;
  int g = 4;
  while (g < 64 && g * per_lane < avg) g *= 2;
  return g;
}

template <typename T>
DCsr<T> upload(const HCsr& A, hipStream_t s) {
  DCsr<T> D;
  D.nrows = A.nrows;
  D.ncols = A.ncols;
  D.nnz = A.nnz();
  D.deep = D.nnz >= (int64_t(1) << 21);  // large: a bandwidth stream
  D.group = pick_group(D.nnz, D.nrows, D.deep ? 8 : 3);
  D.rp = std::make_shared<DevBuf>();
  D.rp->alloc(sizeof(int64_t) * (A.nrows + 1));
  h2d(D.rp->p, A.rp.data(), size_t(A.nrows + 1), s);
  if (D.nnz) {
    D.ci = std::make_shared<DevBuf>();
    D.ci->alloc(sizeof(int32_t) * D.nnz);
    h2d(D.ci->p, A.ci.data(), size_t(D.nnz), s);
    D.val = std::make_shared<DevBuf>();
    D.val->alloc(sizeof(T) * D.nnz);
    h2d_as<T>(D.val->p, A.v.data(), size_t(D.nnz), s);
  }
  return D;
}

// Device copy of a host array (setup only; finished on return).
template <typename U>
std::shared_ptr<DevBuf> upload_raw(const std::vector<U>& v, hipStream_t s = nullptr) {
  auto b = std::make_shared<DevBuf>();
  b->alloc(sizeof(U) * std::max<size_t>(v.size(), 1));
  h2d(b->p, v.data(), v.size(), s);
  return b;
}

// Device copy of FP64 host values as T (setup only; finished on return).
template <typename T>
std::shared_ptr<DevBuf> upload_as(const std::vector<double>& v, hipStream_t s = nullptr) {
  auto b = std::make_shared<DevBuf>();
  b->alloc(sizeof(T) * std::max<size_t>(v.size(), 1));
  h2d_as<T>(b->p, v.data(), v.size(), s);
  return b;
}

// C = A B on the device, bitwise equal to the host product spgemm(A, B) (the
// kernels form every row as the host does).  Rows with more than 4096
// distinct columns are formed on the host.  Small products stay on the host.
// With count_only the result holds only the row pointers (C.rp.back() is the
// number of nonzeros) and nothing is written or copied back.
HCsr device_spgemm(const HCsr& A, const HCsr& B, hipStream_t s, bool count_only = false) {
  if (A.ncols != B.nrows) throw Error(FSI_ERR_ARG, "sparse product of mismatched shapes");
  const int64_t m = A.nrows;
  if (m > INT32_MAX || A.nnz() + B.nnz() < (int64_t(1) << 16) || A.nnz() == 0 || B.nnz() == 0)
    return spgemm(A, B);
  auto up = [&](const auto& v) { return upload_raw(v, s); };
  auto arp = up(A.rp), aci = up(A.ci), av = up(A.v), brp = up(B.rp), bci = up(B.ci), bv = up(B.v);
  DevBuf cnt;
  cnt.alloc(sizeof(int64_t) * m);
  const int64_t* drp = arp->as<int64_t>();
  const int32_t* dci = aci->as<int32_t>();
  const double* dv = av->as<double>();
  const int64_t* ebp = brp->as<int64_t>();
  const int32_t* eci = bci->as<int32_t>();
  const double* ev = bv->as<double>();
  int64_t* dcnt = cnt.as<int64_t>();
  // counts: every row with the small table, the overflowing rows with the large one
  spgemm_rows_kernel<kSpgSmall, false><<<unsigned(m), 64, 0, s>>>(nullptr, drp, dci, dv, ebp, eci, ev, dcnt,
                                                                  nullptr, nullptr, nullptr);
  HIP_TRY(hipGetLastError());
  std::vector<int64_t> hc(m);
  d2h(hc.data(), dcnt, size_t(m), s);
  std::vector<int32_t> small_rows, large_rows, host_rows;
  for (int64_t i = 0; i < m; ++i)
    if (hc[i] < 0) large_rows.push_back(int32_t(i));
  std::shared_ptr<DevBuf> dlarge;
  if (!large_rows.empty()) {
    dlarge = up(large_rows);
    spgemm_rows_kernel<kSpgLarge, false><<<unsigned(large_rows.size()), 64, 0, s>>>(
        dlarge->as<int32_t>(), drp, dci, dv, ebp, eci, ev, dcnt, nullptr, nullptr, nullptr);
    HIP_TRY(hipGetLastError());
    d2h(hc.data(), dcnt, size_t(m), s);
  }
  std::vector<char> cls(m, 0);  // 0: small table, 1: large table, 2: host
  for (int32_t i : large_rows) cls[i] = hc[i] < 0 ? 2 : 1;
  for (int64_t i = 0; i < m; ++i) {
    if (cls[i] == 0) small_rows.push_back(int32_t(i));
    else if (cls[i] == 2) host_rows.push_back(int32_t(i));
  }
  // rows formed on the host
  std::vector<std::vector<int32_t>> hcols(host_rows.size());
  std::vector<std::vector<double>> hvals(host_rows.size());
  parallel_for(int64_t(host_rows.size()), [&](int64_t b, int64_t e) {
    SpgemmWork w;
    for (int64_t q = b; q < e; ++q) spgemm_row(A, B, host_rows[q], w, hcols[q], hvals[q]);
  }, 2);
  for (size_t q = 0; q < host_rows.size(); ++q) hc[host_rows[q]] = int64_t(hcols[q].size());
  HCsr C;
  C.nrows = m;
  C.ncols = B.ncols;
  C.rp.assign(m + 1, 0);
  for (int64_t i = 0; i < m; ++i) C.rp[i + 1] = C.rp[i] + hc[i];
  const int64_t nnz = C.rp[m];
  if (count_only) return C;
  auto crp = up(C.rp);
  DevBuf cci, cv;
  cci.alloc(sizeof(int32_t) * std::max<int64_t>(nnz, 1));
  cv.alloc(sizeof(double) * std::max<int64_t>(nnz, 1));
  if (!small_rows.empty()) {
    auto dsmall = up(small_rows);
    spgemm_rows_kernel<kSpgSmall, true><<<unsigned(small_rows.size()), 64, 0, s>>>(
        dsmall->as<int32_t>(), drp, dci, dv, ebp, eci, ev, dcnt, crp->as<int64_t>(), cci.as<int32_t>(),
        cv.as<double>());
    HIP_TRY(hipGetLastError());
  }
  std::vector<int32_t> dev_large;
  for (int32_t i : large_rows)
    if (cls[i] == 1) dev_large.push_back(i);
  if (!dev_large.empty()) {
    auto dl = up(dev_large);
    spgemm_rows_kernel<kSpgLarge, true><<<unsigned(dev_large.size()), 64, 0, s>>>(
        dl->as<int32_t>(), drp, dci, dv, ebp, eci, ev, dcnt, crp->as<int64_t>(), cci.as<int32_t>(),
        cv.as<double>());
    HIP_TRY(hipGetLastError());
  }
  C.ci.resize(nnz);
  C.v.resize(nnz);
  d2h(C.ci.data(), cci.p, size_t(nnz), s);
  d2h(C.v.data(), cv.p, size_t(nnz), s);
  for (size_t q = 0; q < host_rows.size(); ++q) {
    std::copy(hcols[q].begin(), hcols[q].end(), C.ci.begin() + C.rp[host_rows[q]]);
    std::copy(hvals[q].begin(), hvals[q].end(), C.v.begin() + C.rp[host_rows[q]]);
  }
  return C;
}


// Rows per group of a grouped level (the components of a node).
template <class F>
void with_rgroup(int g, F&& f) {
  if (g == 2) f(std::integral_constant<int, 2>{});
  else f(std::integral_constant<int, 3>{});
}

// Rows [r0, r1) of A grouped g at a time (g = 2 or 3) on the device: the
// rows' entries are uploaded once, a count pass gives each group's entries (the
// union of its rows' columns), a fill pass writes the group row pointers,
// column lists and g values per entry as T (times colscale[column] when given),
// exactly as the host's group_rows followed by a conversion to T.
struct DevGroups {
  int64_t ngroups = 0, entries = 0;
  std::shared_ptr<DevBuf> rp, ci, val;
};

struct DevRows {  // rows [r0, r1) of a host CSR on the device, row pointers from 0
  int64_t nrows = 0, nnz = 0;
  std::shared_ptr<DevBuf> rp, ci, v;
};

DevRows upload_rows(const HCsr& A, int64_t r0, int64_t r1, hipStream_t s) {
  DevRows R;
  R.nrows = r1 - r0;
  const int64_t e0 = A.rp[r0];
  R.nnz = A.rp[r1] - e0;
  std::vector<int64_t> rp(size_t(R.nrows + 1));
  parallel_for(R.nrows + 1, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) rp[i] = A.rp[r0 + i] - e0;
  });
  R.rp = upload_raw(rp, s);
  R.ci = std::make_shared<DevBuf>();
  R.ci->alloc(sizeof(int32_t) * std::max<int64_t>(R.nnz, 1));
  h2d(R.ci->p, A.ci.data() + e0, size_t(R.nnz), s);
  R.v = std::make_shared<DevBuf>();
  R.v->alloc(sizeof(double) * std::max<int64_t>(R.nnz, 1));
  h2d(R.v->p, A.v.data() + e0, size_t(R.nnz), s);
  return R;
}

// Entries of each group (count pass); g must be 2 or 3.
std::vector<int64_t> device_group_counts(const DevRows& R, int g, hipStream_t s) {
  const int64_t ng = R.nrows / g;
  std::vector<int64_t> cnt(size_t(ng), 0);
  if (ng == 0) return cnt;
  DevBuf dc;
  dc.alloc(sizeof(int64_t) * ng);
  with_rgroup(g, [&](auto gc) {
    constexpr int G = decltype(gc)::value;
    group_merge_kernel<G, false, double><<<unsigned((ng + 255) / 256), 256, 0, s>>>(
        ng, R.rp->as<int64_t>(), R.ci->as<int32_t>(), R.v->as<double>(), nullptr, dc.as<int64_t>(), nullptr,
        nullptr, nullptr);
  });
  HIP_TRY(hipGetLastError());
  d2h(cnt.data(), dc.p, size_t(ng), s);
  return cnt;
}

// The grouped arrays from the counts (fill pass).
template <typename T>
DevGroups device_group_fill(const DevRows& R, int g, const std::vector<int64_t>& cnt, const double* dcolscale,
                            hipStream_t s) {
  DevGroups out;
  out.ngroups = int64_t(cnt.size());
  std::vector<int64_t> grp(cnt.size() + 1, 0);
  for (size_t q = 0; q < cnt.size(); ++q) grp[q + 1] = grp[q] + cnt[q];
  out.entries = grp.back();
  out.rp = upload_raw(grp, s);
  out.ci = std::make_shared<DevBuf>();
  out.ci->alloc(sizeof(int32_t) * std::max<int64_t>(out.entries, 1));
  out.val = std::make_shared<DevBuf>();
  out.val->alloc(sizeof(T) * std::max<int64_t>(out.entries * g, 1));
  if (out.ngroups) {
    with_rgroup(g, [&](auto gc) {
      constexpr int G = decltype(gc)::value;
      group_merge_kernel<G, true, T><<<unsigned((out.ngroups + 255) / 256), 256, 0, s>>>(
          out.ngroups, R.rp->as<int64_t>(), R.ci->as<int32_t>(), R.v->as<double>(), dcolscale, nullptr,
          out.rp->as<int64_t>(), out.ci->as<int32_t>(), out.val->as<T>());
    });
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
  }
  return out;
}

// y = D^{-1} A x of the setup's power iteration on the device, the host's
// product bit for bit (one thread per row, storage order); A and D^{-1} are
// uploaded once per level, x and y travel per step.  Small levels keep the
// host product (empty function).
ScaledProduct device_scaled_product(const HCsr& A, const std::vector<double>& dinv, hipStream_t s) {
  if (A.nnz() < (int64_t(1) << 20)) return {};
  struct State {
    DevRows R;
    std::shared_ptr<DevBuf> dinv, x, y;
    int64_t n = 0;
    hipStream_t s = nullptr;
  };
  auto st = std::make_shared<State>();
  st->n = A.nrows;
  st->s = s;
  st->R = upload_rows(A, 0, A.nrows, s);
  st->dinv = upload_raw(dinv, s);
  st->x = std::make_shared<DevBuf>();
  st->x->alloc(sizeof(double) * st->n);
  st->y = std::make_shared<DevBuf>();
  st->y->alloc(sizeof(double) * st->n);
  return [st](const double* x, double* y) {
    h2d(st->x->p, x, size_t(st->n), st->s);
    rowseq_scaled_matvec_kernel<<<unsigned((st->n + 255) / 256), 256, 0, st->s>>>(
        st->n, st->R.rp->as<int64_t>(), st->R.ci->as<int32_t>(), st->R.v->as<double>(), st->dinv->as<double>(),
        st->x->as<double>(), st->y->as<double>());
    HIP_TRY(hipGetLastError());
    d2h(y, st->y->p, size_t(st->n), st->s);
  };
}

// Rows [r0, r1) of A grouped g at a time on the device; colscale: optional
// host column scale (A D^{-1}).
template <typename T>
DevGroups device_group_rows(const HCsr& A, int64_t r0, int64_t r1, int g, const std::vector<double>* colscale,
                            hipStream_t s) {
  if (g != 2 && g != 3) throw Error(FSI_ERR_ARG, "row groups of 2 or 3 rows only");
  const DevRows R = upload_rows(A, r0, r1, s);
  const std::vector<int64_t> cnt = device_group_counts(R, g, s);
  std::shared_ptr<DevBuf> dscale;
  if (colscale) dscale = upload_raw(*colscale, s);
  return device_group_fill<T>(R, g, cnt, dscale ? dscale->as<double>() : nullptr, s);
}

// A in groups of g consecutive rows sharing one column list (g values per
// entry), for the grouped level sweeps, grouped on the device (A's columns
// scaled by colscale when given); with `as_segment` also described as a
// one-segment RowSegments, so that launch_rows runs it.
template <typename T>
DCsr<T> upload_grouped(const HCsr& A, int g, bool as_segment = false, const std::vector<double>* colscale = nullptr,
                       hipStream_t s = nullptr) {
  DevGroups G = device_group_rows<T>(A, 0, A.nrows, g, colscale, s);
  DCsr<T> D;
  D.nrows = A.nrows;
  D.ncols = A.ncols;
  D.nnz = G.entries;
  D.rgroup = g;
  D.deep = true;
  D.rp = G.rp;
  D.ci = G.ci;
  D.val = G.val;
  if (as_segment) {
    const int64_t units = G.ngroups;
    const double avg = units ? double(D.nnz) / double(units) : 1.0;
    int lanes = 4;
    while (lanes < 32 && lanes * 12 < avg) lanes *= 2;
    RowSegments& sg = D.seg;
    sg.nseg = 1;
    sg.row0[0] = 0;
    sg.row0[1] = A.nrows;
    sg.blk0[0] = 0;
    sg.blk0[1] = unsigned((units + kBlock / lanes - 1) / (kBlock / lanes));
    sg.g[0] = lanes;
    sg.grp[0] = g;
    sg.grp_rp[0] = D.drp();
    sg.grp_ci[0] = D.dci();
    sg.grp_val[0] = D.dval();
    D.seg_bytes = double(D.nnz) * (4.0 + sizeof(T) * g) + double(units + 1) * 8;
  }
  return D;
}

// A as up to four consecutive row segments [bounds[q], bounds[q+1]) that
// start at row 0, each with its own lanes per row or row group (about twelve
// entries per lane, 4 to 32 lanes; measured best for long rows); segment q is
// stored in groups of group[q] rows where that costs at most 5% zero fill.
// bytes(): the matrix as stored (values, column lists, row or group pointers).
// The plain arrays hold the rows of the ungrouped segments only (the rows of a
// grouped segment are empty there); nnz stays the matrix's own count.
// The row grouping of each segment (group[q], or 1 where the segment does
// not split into whole groups or grouping costs more than 5% zero fill) and
// the row pointers of the plain arrays: the rows of the ungrouped segments,
// grouped rows empty (segment q's entries follow those of the ungrouped
// segments before it).
std::vector<int64_t> segment_plan(const HCsr& A, const int64_t* bounds, const int* group, int nseg, int* grs) {
  if (nseg < 1 || nseg > 4 || bounds[0] != 0 || bounds[nseg] != A.nrows)
    throw Error(FSI_ERR_ARG, "row segments must cover the matrix in at most four parts");
  std::vector<int64_t> rp(size_t(A.nrows + 1), 0);
  int64_t skipped = 0;  // entries of the grouped segments before the current one
  for (int q = 0; q < nseg; ++q) {
    const int64_t r0 = bounds[q], r1 = bounds[q + 1];
    const int64_t units = r1 - r0, nz = r1 > r0 ? A.rp[r1] - A.rp[r0] : 0;
    int gr = group[q];
    if (gr > 1 && (units <= 0 || units % gr != 0 ||
                   double(group_entries(A, r0, r1, gr)) * gr > 1.05 * double(nz)))
      gr = 1;
    grs[q] = gr;
    const int64_t sk = skipped;
    if (gr == 1) {
      parallel_for(units + 1, [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i) rp[r0 + i] = A.rp[r0 + i] - sk;
      });
    } else {
      std::fill(rp.begin() + r0, rp.begin() + r1 + 1, A.rp[r0] - sk);
      skipped += nz;
    }
  }
  return rp;
}

// The plain arrays' entries (segments with grs[q] == 1), ci and/or values as T,
// copied straight from A's arrays into the device arrays.
template <typename T>
void upload_plain_entries(const HCsr& A, const int64_t* bounds, int nseg, const int* grs, DevBuf* ci, DevBuf* val,
                          hipStream_t s) {
  int64_t dst = 0;
  for (int q = 0; q < nseg; ++q) {
    if (grs[q] != 1 || bounds[q + 1] <= bounds[q]) continue;
    const int64_t e0 = A.rp[bounds[q]], n = A.rp[bounds[q + 1]] - e0;
    if (ci) h2d(ci->as<int32_t>() + dst, A.ci.data() + e0, size_t(n), s);
    if (val) h2d_as<T>(val->as<T>() + dst, A.v.data() + e0, size_t(n), s);
    dst += n;
  }
}

// New values for a matrix uploaded by upload_segments from a matrix of the
// same sparsity pattern: written in place into the same device arrays (the
// layout, and any captured graph that reads them, stay valid).
template <typename T>
void refresh_segments(const DCsr<T>& D, const HCsr& A, const int64_t* bounds, const int* group, int nseg,
                      hipStream_t s) {
  int grs[4];
  const std::vector<int64_t> rp = segment_plan(A, bounds, group, nseg, grs);
  const int64_t plain_nnz = rp.back();
  auto fits = [](const std::shared_ptr<DevBuf>& b, size_t n) { return n == 0 || (b && b->bytes == sizeof(T) * n); };
  if (!fits(D.val, size_t(plain_nnz))) throw Error(FSI_ERR_ARG, "new values do not fit the stored layout");
  if (plain_nnz) upload_plain_entries<T>(A, bounds, nseg, grs, nullptr, D.val.get(), s);
  for (int q = 0, k = 0; q < nseg; ++q) {
    if (bounds[q + 1] <= bounds[q]) continue;
    const int kk = k++;
    if ((D.seg.grp[kk] > 1) != (grs[q] > 1) || (grs[q] > 1 && D.seg.grp[kk] != grs[q]))
      throw Error(FSI_ERR_ARG, "new values do not fit the stored layout");
    if (grs[q] == 1) continue;
    DevGroups Gm = device_group_rows<T>(A, bounds[q], bounds[q + 1], grs[q], nullptr, s);
    if (!fits(D.grp_val[kk], size_t(Gm.entries * grs[q])))
      throw Error(FSI_ERR_ARG, "new values do not fit the stored layout");
    HIP_TRY(hipMemcpyAsync(D.grp_val[kk]->p, Gm.val->p, sizeof(T) * size_t(Gm.entries * grs[q]),
                           hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
}

template <typename T>
DCsr<T> upload_segments(const HCsr& A, const int64_t* bounds, const int* group, int nseg, hipStream_t s) {
  int grs[4];
  const std::vector<int64_t> prp = segment_plan(A, bounds, group, nseg, grs);
  DCsr<T> D;
  D.nrows = A.nrows;
  D.ncols = A.ncols;
  D.nnz = A.nnz();
  D.deep = true;
  D.rp = upload_raw(prp, s);
  const int64_t plain_nnz = prp.back();
  D.group = pick_group(plain_nnz, A.nrows, plain_nnz >= (int64_t(1) << 21) ? 8 : 3);
  if (plain_nnz) {
    D.ci = std::make_shared<DevBuf>();
    D.ci->alloc(sizeof(int32_t) * plain_nnz);
    D.val = std::make_shared<DevBuf>();
    D.val->alloc(sizeof(T) * plain_nnz);
    upload_plain_entries<T>(A, bounds, nseg, grs, D.ci.get(), D.val.get(), s);
  }
  RowSegments sg{};
  sg.nseg = 0;
  sg.blk0[0] = 0;
  sg.row0[0] = bounds[0];
  double bytes = 0.0;
  for (int q = 0; q < nseg; ++q) {
    const int64_t r0 = bounds[q], r1 = bounds[q + 1];
    if (r1 <= r0) continue;
    const int k = sg.nseg++;
    int64_t units = r1 - r0, nz = A.rp[r1] - A.rp[r0];
    const int gr = grs[q];
    if (gr > 1) {
      DevGroups Gm = device_group_rows<T>(A, r0, r1, gr, nullptr, s);
      units = Gm.ngroups;
      nz = Gm.entries;
      D.grp_rp[k] = Gm.rp;
      D.grp_ci[k] = Gm.ci;
      D.grp_val[k] = Gm.val;
      sg.grp_rp[k] = D.grp_rp[k]->template as<int64_t>();
      sg.grp_ci[k] = D.grp_ci[k]->template as<int32_t>();
      sg.grp_val[k] = D.grp_val[k]->template as<T>();
      bytes += double(nz) * (4.0 + sizeof(T) * gr) + 8.0 * double(units + 1);
    } else {
      bytes += double(nz) * (4.0 + sizeof(T)) + 8.0 * double(units + 1);
    }
    sg.grp[k] = gr;
    const double avg = double(nz) / double(units);
    int g = 4;
    while (g < 32 && g * 12 < avg) g *= 2;
    sg.g[k] = g;
    sg.row0[k + 1] = r1;
    sg.blk0[k + 1] = sg.blk0[k] + unsigned((units + kBlock / g - 1) / (kBlock / g));
  }
  D.seg = sg;
  D.seg_bytes = bytes;
  return D;
}

// R and R A of a Chebyshev level on the union of their column patterns, the
// two values of an entry side by side (0 where a matrix has no entry).
template <typename T>
DCsr<T> upload_pair(const HCsr& R, const HCsr& RA) {
  DCsr<T> D;
  D.nrows = R.nrows;
  D.ncols = R.ncols;
  std::vector<int64_t> rp(R.nrows + 1, 0);
  std::vector<int32_t> ci;
  std::vector<T> v;
  for (int64_t i = 0; i < R.nrows; ++i) {
    int64_t a = R.rp[i], b = RA.rp[i];
    while (a < R.rp[i + 1] || b < RA.rp[i + 1]) {
      const int32_t ca = a < R.rp[i + 1] ? R.ci[a] : INT32_MAX;
      const int32_t cb = b < RA.rp[i + 1] ? RA.ci[b] : INT32_MAX;
      const int32_t c = std::min(ca, cb);
      ci.push_back(c);
      v.push_back(T(ca == c ? R.v[a++] : 0.0));
      v.push_back(T(cb == c ? RA.v[b++] : 0.0));
    }
    rp[i + 1] = int64_t(ci.size());
  }
  D.nnz = int64_t(ci.size());
  D.rp = upload_raw(rp);
  D.ci = upload_raw(ci);
  D.val = upload_raw(v);
  D.group = pick_group(D.nnz, std::max<int64_t>(D.nrows, 1));
  return D;
}

template <typename T>
std::shared_ptr<DevBuf> upload_vec(const std::vector<double>& v, hipStream_t s) {
  auto b = std::make_shared<DevBuf>();
  b->alloc(sizeof(T) * v.size());
  h2d_as<T>(b->p, v.data(), v.size(), s);
  return b;
}


inline unsigned grid_for(int64_t n, int per_block) {
  int64_t g = (n + per_block - 1) / per_block;
  return unsigned(std::max<int64_t>(1, std::min<int64_t>(g, int64_t(1) << 30)));
}

// X = Ainv B with the dense coarsest inverse: a workgroup per row from 768
// rows on (at least three entries per lane), else a wavefront per row.
template <typename TI, typename TO, int NV>
void dense_gemv(int64_t n, const double* Ainv, const TI* B, TO* X, hipStream_t s) {
  if (n >= 768)
    dense_gemv_kernel<TI, TO, NV, kBlock / 64><<<grid_for(n, 1), kBlock, 0, s>>>(n, Ainv, B, X);
  else
    dense_gemv_kernel<TI, TO, NV, 1><<<grid_for(n, kBlock / 64), kBlock, 0, s>>>(n, Ainv, B, X);
}

template <class F>
void with_group(int G, F&& f) {
  switch (G) {
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    case 32: f(std::integral_constant<int, 32>{}); break;
    default: f(std::integral_constant<int, 64>{}); break;
  }
}

// Launch a row-grouped CSR product with epilogue.
template <typename T, int NV, class Gather, class Epi>
void launch_rows(const DCsr<T>& A, Gather g, Epi e, hipStream_t s) {
  if (A.nrows == 0) return;
  if constexpr (NV == 1) {
    if (A.seg.nseg > 0) {
      csr_segments_kernel<T, Gather, Epi><<<A.seg.blk0[A.seg.nseg], kBlock, 0, s>>>(A.seg, A.drp(), A.dci(),
                                                                                    A.dval(), g, e);
      return;
    }
  }
  with_group(A.group, [&](auto gc) {
    constexpr int G = decltype(gc)::value;
    const unsigned grid = grid_for(A.nrows, kBlock / G);
    if (A.deep)
      csr_rows_kernel<T, G, NV, Gather, Epi, true><<<grid, kBlock, 0, s>>>(A.nrows, A.drp(), A.dci(), A.dval(), g, e);
    else
      csr_rows_kernel<T, G, NV, Gather, Epi, false><<<grid, kBlock, 0, s>>>(A.nrows, A.drp(), A.dci(), A.dval(), g, e);
  });
}

template <typename T, int NV = 1>
void spmv(const DCsr<T>& A, const T* x, T* y, hipStream_t s) {
  launch_rows<T, NV>(A, GatherPlain<T, NV>{x}, EpiStore<T, NV>{y}, s);
}
template <typename T, int NV = 1>
void spmv_sub(const DCsr<T>& A, const T* x, const T* r, T* y, hipStream_t s) {
  launch_rows<T, NV>(A, GatherPlain<T, NV>{x}, EpiSub<T, NV>{r, y}, s);
}

template <typename T>
void vsub(int64_t n, T* y, const T* x, hipStream_t s) {
  if (n) vsub_kernel<T><<<grid_for(n, kBlock * 4), kBlock, 0, s>>>(n, y, x);
}

// ---------------------------------------------------------------- AMG on device
// Device view of the learned pre-smoother of a hierarchy's finest level.
struct MlpUse {
  bool enabled = false;
  int d = 2;
  bool per_dof = false;  // inverse diagonal per dof (block operator) or per node (L (x) I_d)
  int64_t n_nodes = 0;
  const int32_t* nbr = nullptr;
  MlpW w{};
  double* npart = nullptr;
  int* flag = nullptr;
  int* fallbacks = nullptr;
  int* streak = nullptr;  // consecutive rejections in the current solve
};

// Recording of finest-level V-cycle inputs (training data of the smoother).
struct MlpRecord {
  bool active = false;
  int max_vectors = 0, every = 1;
  long calls = 0;
  std::vector<std::shared_ptr<DevBuf>> vecs;  // FP64 copies
};

template <typename T>
struct DLevel {
  DCsr<T> AD, Q, P, AP;  // A D^{-1}, Q = R (I - omega A D^{-1}), prolongator, A P
  DCsr<T> A0, R0;        // A and R themselves: learned smoother (A: levels 0, 1; R: level 0) or Chebyshev levels
  std::shared_ptr<DevBuf> dinv, y, r, b;
  std::shared_ptr<DevBuf> dinv_h;  // BF16-stored inverse diagonal (in place of dinv)
  T omega = T(0);
  int64_t n = 0;
  int gdown = 8, gdownq = 64, gup = 8;
  int rgroup = 1;                      // > 1: AD, Q (or R), P, AP stored in groups of rgroup rows
  bool deep = false;                   // large level: four loads in flight per lane
  bool split = false;                  // restriction by R in its own launch (no Q)
  bool split_plain = false;            // the learned smoother's level: Q kept for its own
                                       //   sweep, the plain cycle restricts by R apart
  int cheb = 0;                        // Chebyshev degree of this level's sweeps (0: Jacobi)
  DCsr<T> RRA;                         // Chebyshev levels: R and R A on one column list (fused restriction)
  int gres = 16;                       //   its lanes per coarse row
  std::vector<T> ca, cc;               // recurrence coefficients a_j, c_j, j = 1..cheb
  std::shared_ptr<DevBuf> d0, d1, r1;  // Chebyshev directions and second residual buffer
  Diag<T> diag() const {
    return Diag<T>{dinv ? dinv->template as<T>() : nullptr, dinv_h ? dinv_h->template as<uint16_t>() : nullptr};
  }
};

template <typename T>
struct DHier {
  int nv = 1;  // interleaved right-hand sides (d for the mesh Laplacian)
  std::vector<DLevel<T>> lev;
  std::shared_ptr<DevBuf> cinv;
  int64_t nc = 0;
  double bytes_per_cycle = 0.0;  // algorithmic bytes of one cycle as executed
  bool poly = false;             // inverse = level 0's Chebyshev steps alone (no coarse grid)
  MlpUse* mlp = nullptr;         // learned pre-smoother of level 0 (if any)
  MlpRecord* rec = nullptr;      // recording of level-0 inputs (if any)
  std::shared_ptr<DevBuf> xm, rm;  // its correction and residual
};

// BF16 bit pattern of f, rounded to nearest even (f finite), and its value.
inline uint16_t bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
inline double bf16_round(float f) {
  const uint32_t u = uint32_t(bf16_bits(f)) << 16;
  float r;
  std::memcpy(&r, &u, 4);
  return double(r);
}

// Chebyshev recurrence of degree k for D^{-1} A on [lam/30, lam], lam = 1.1 rho
// (rho = (4/3)/omega, the setup's power estimate): a_1 = 0, c_1 = 1/theta,
// rho_0 = delta/theta, rho_j = 1/(2 theta/delta - rho_{j-1}), a_j = rho_j rho_{j-1},
// c_j = 2 rho_j / delta.
constexpr double kChebRatio = 30.0, kChebBoost = 1.1;

template <typename T>
void cheb_coefficients(double omega, int k, std::vector<T>& a, std::vector<T>& c, double ratio = kChebRatio) {
  const double lmax = kChebBoost * (4.0 / 3.0) / omega, lmin = lmax / ratio;
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
  a.assign(k + 1, T(0));
  c.assign(k + 1, T(0));
  c[1] = T(1.0 / theta);
  double rho = 1.0 / sigma;
  for (int j = 2; j <= k; ++j) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    a[j] = T(rn * rho);
    c[j] = T(2.0 * rn / delta);
    rho = rn;
  }
}

constexpr int64_t kDeepNnz = int64_t(1) << 21;
constexpr int64_t kSplitNnz = int64_t(1) << 21;
constexpr int64_t kFuseRestrictNnz = int64_t(1) << 18;

template <typename T>
DHier<T> upload_hier(SaHierarchy& H, int nv, hipStream_t s, bool keep_a0 = false, int cheb = 0,
                     int poly = 0, double poly_ratio = 8.0, int group = 1, bool bf16diag = false) {
  DHier<T> D;
  D.nv = nv;
  // BF16-stored inverse diagonals: every use of D^{-1} (the sweeps and the
  // setup products A D^{-1}, Q) takes the values rounded to BF16 (through
  // FP32, nearest even), so the smoother is the same Jacobi/Chebyshev
  // smoother with a perturbed diagonal
  const double db = bf16diag ? 2.0 : double(sizeof(T));  // bytes per diagonal entry
  auto level_dinv = [&](const std::vector<double>& dv) {
    if (!bf16diag) return dv;
    std::vector<double> r(dv.size());
    for (size_t i = 0; i < dv.size(); ++i) r[i] = bf16_round(float(dv[i]));
    return r;
  };
  auto put_dinv = [&](DLevel<T>& d, const std::vector<double>& dv) {
    if (!bf16diag) {
      d.dinv = upload_vec<T>(dv, s);
      return;
    }
    std::vector<uint16_t> bits(dv.size());
    for (size_t i = 0; i < dv.size(); ++i) bits[i] = bf16_bits(float(dv[i]));
    d.dinv_h = upload_raw(bits);
  };
  const int L = int(H.levels.size()) - 1;
  if (poly > 0 && L > 0) {
    // Chebyshev steps alone on the finest matrix: the other levels are not used
    const SaLevel& h = H.levels[0];
    if (!(h.omega > 0.0)) throw Error(FSI_ERR_NUMERIC, "Chebyshev steps need a positive spectral estimate");
    DLevel<T> d;
    d.n = h.A.nrows;
    d.omega = T(h.omega);
    d.cheb = poly;
    cheb_coefficients<T>(h.omega, poly, d.ca, d.cc, poly_ratio);
    d.A0 = upload<T>(h.A, s);
    put_dinv(d, level_dinv(h.dinv));
    auto mkv = [&]() {
      auto b = std::make_shared<DevBuf>();
      b->alloc(sizeof(T) * std::max<int64_t>(d.n * nv, 1));
      return b;
    };
    d.d0 = mkv();
    d.d1 = mkv();
    d.r1 = mkv();
    d.r = mkv();
    d.y = mkv();
    d.b = mkv();
    D.bytes_per_cycle = (d.A0.bytes() + double(d.n) * (6.0 * sizeof(T) * nv + db)) * (poly - 1);
    D.lev.push_back(std::move(d));
    D.poly = true;
    D.nc = 0;
    return D;
  }
  for (int l = 0; l <= L; ++l) {
    SaLevel& h = H.levels[l];
    DLevel<T> d;
    d.n = h.A.nrows;
    d.omega = T(h.omega);
    if (l < L && cheb > 0) {
      if (!(h.omega > 0.0)) throw Error(FSI_ERR_NUMERIC, "Chebyshev smoothing needs a positive spectral estimate");
      if (!h.AP.nrows) h.AP = device_spgemm(h.A, h.P, s);  // A P unless the setup kept it
      const HCsr& AP = h.AP;
      d.cheb = cheb;
      cheb_coefficients<T>(h.omega, cheb, d.ca, d.cc);
      d.A0 = upload<T>(h.A, s);
      // small finest levels (latency-bound launches): the restriction joins
      // the last pre-smoothing step's launch, reading R and R A instead of R.
      // Above 2^18 entries of R A, or on coarser levels (where R A's rows are
      // long next to the level's own), the fused coarse rows outlast the
      // launch saved (measured on the 2D and 3D workloads).
      if (l == 0 && h.ra_nnz < 0) h.ra_nnz = device_spgemm(h.R, h.A, s, true).rp.back();
      if (l == 0 && h.ra_nnz < kFuseRestrictNnz) {
        d.RRA = upload_pair<T>(h.R, device_spgemm(h.R, h.A, s));
        d.gres = d.RRA.group >= 32 ? 64 : 16;
      } else {
        d.R0 = upload<T>(h.R, s);
      }
      d.P = upload<T>(h.P, s);
      d.AP = upload<T>(AP, s);
      put_dinv(d, level_dinv(h.dinv));
      d.gup = pick_group(d.AP.nnz + d.P.nnz, std::max<int64_t>(d.AP.nrows, 1));
      auto mkv = [&]() {
        auto b = std::make_shared<DevBuf>();
        b->alloc(sizeof(T) * std::max<int64_t>(d.n * nv, 1));
        return b;
      };
      d.d0 = mkv();
      d.d1 = mkv();
      d.r1 = mkv();
      const double vb = double(sizeof(T)) * nv;
      // pre: cheb steps over A + R; post: P, AP, cheb - 1 steps over A; per step
      // d, r, dinv gathered and d, r, x written at the row
      const double rbytes = d.RRA.rp ? double(d.RRA.nnz) * (4.0 + 2.0 * sizeof(T)) + 8.0 * double(d.RRA.nrows + 1)
                                     : d.R0.bytes();
      D.bytes_per_cycle += d.A0.bytes() * (2 * cheb - 1) + rbytes + d.P.bytes() + d.AP.bytes() +
                           double(d.n) * (6.0 * cheb * vb + 2 * db) + double(h.P.ncols) * 2 * vb;
    } else if (l < L) {
      // setup-time products for the two-launch level sweeps (A P unless the
      // setup kept it)
      if (!h.AP.nrows) h.AP = device_spgemm(h.A, h.P, s);  // kept for later builds
      const HCsr& AP = h.AP;
      const std::vector<double> dv = level_dinv(h.dinv);
      // Restricting through Q = R (I - omega A D^{-1}) fuses the restriction
      // into the down-sweep but reads Q's entries (about R A's pattern)
      // instead of R's; where R A has kSplitNnz more nonzeros than R (counted
      // on the device), restrict the residual with R in a launch of its own
      // and leave Q unformed (unless the learned smoother's sweep needs it).
      if (h.ra_nnz < 0) h.ra_nnz = device_spgemm(h.R, h.A, s, true).rp.back();  // kept for later builds
      const bool split_worthy = h.ra_nnz - h.R.nnz() >= kSplitNnz;
      d.split = !(l == 0 && keep_a0) && split_worthy;
      d.split_plain = l == 0 && keep_a0 && split_worthy;  // R is uploaded for that level below
      HCsr Q;
      if (!d.split) {
        HCsr RA = device_spgemm(h.R, h.A, s);
        std::vector<double> wd(dv.size());
        for (size_t i = 0; i < wd.size(); ++i) wd[i] = h.omega * dv[i];
        scale_cols(RA, wd);
        Q = add(h.R, RA, -1.0);
      }
      // Large levels of a vector problem (group = components per node): where
      // the rows of a node share their columns in all four matrices (at most
      // 5% zero fill), store them in groups of `group` rows.  Decided on the
      // structure alone, so imported hierarchies take the same path.
      const HCsr& Rq = d.split ? h.R : Q;
      auto fits = [&](const HCsr& M) {
        return M.nrows % group == 0 && double(group_entries(M, 0, M.nrows, group)) * group <= 1.05 * double(M.nnz());
      };
      // (A D^{-1} has A's pattern: it is formed from A where it is stored)
      if (group > 1 && nv == 1 && !(l == 0 && keep_a0) && h.A.nnz() >= kDeepNnz && fits(h.A) && fits(Rq) &&
          fits(h.P) && fits(AP))
        d.rgroup = group;
      if (d.rgroup > 1) {
        d.AD = upload_grouped<T>(h.A, group, false, &dv, s);  // grouped and scaled on the device
        if (d.split) d.R0 = upload_grouped<T>(h.R, group, true, nullptr, s);
        else d.Q = upload_grouped<T>(Q, group, false, nullptr, s);
        d.P = upload_grouped<T>(h.P, group, false, nullptr, s);
        d.AP = upload_grouped<T>(AP, group, false, nullptr, s);
      } else {
        HCsr AD = h.A;
        scale_cols(AD, dv);
        d.AD = upload<T>(AD, s);
        if (d.split) d.R0 = upload<T>(h.R, s);
        else d.Q = upload<T>(Q, s);
        d.P = upload<T>(h.P, s);
        d.AP = upload<T>(AP, s);
      }
      put_dinv(d, dv);
      if (l == 1 && keep_a0) d.A0 = upload<T>(h.A, s);  // exact coarse solves of the training loss
      if (l == 0 && keep_a0) {
        d.A0 = upload<T>(h.A, s);
        d.R0 = upload<T>(h.R, s);
        D.xm = std::make_shared<DevBuf>();
        D.xm->alloc(sizeof(T) * d.n * nv);
        D.rm = std::make_shared<DevBuf>();
        D.rm->alloc(sizeof(T) * d.n * nv);
      }
      // large levels are bandwidth streams (about ten entries per lane, four
      // loads in flight); small ones latency chains (about three per lane)
      d.deep = h.A.nnz() >= kDeepNnz;
      const int per_lane = d.deep ? 10 : 3;
      const int64_t units = d.n / d.rgroup;  // rows or row groups
      d.gdown = pick_group(d.AD.nnz, units, per_lane);
      // coarse rows of Q: 64 lanes where they are long (the few coarse rows of
      // a large level otherwise outlast its many fine rows), else 16
      const int64_t qunits = std::max<int64_t>(d.Q.nrows / d.rgroup, 1);
      d.gdownq = d.split ? 16 : (pick_group(d.Q.nnz, qunits, d.deep ? 12 : 3) >= 32 ? 64 : 16);
      d.gup = pick_group(d.AP.nnz + d.P.nnz, std::max<int64_t>(units, 1), per_lane);
      const double vb = double(sizeof(T)) * nv;
      // down: A, Q, dinv, b (x1 + gathers), r and b_c writes; up: P, AP, e, b, r, dinv, y
      // (the plain cycle's bytes: with split_plain the restriction by R apart)
      const bool apart = d.split || d.split_plain;
      D.bytes_per_cycle += d.AD.bytes() + (apart ? d.R0.bytes() + double(d.n) * vb : d.Q.bytes()) + d.P.bytes() +
                           d.AP.bytes() + double(d.n) * (2 * db + 5 * vb) + double(h.P.ncols) * 2 * vb;
    }
    auto mk = [&](int64_t cnt) {
      auto b = std::make_shared<DevBuf>();
      b->alloc(sizeof(T) * std::max<int64_t>(cnt, 1));
      return b;
    };
    d.y = mk(d.n * nv);
    d.r = mk(d.n * nv);
    d.b = mk(d.n * nv);
    D.lev.push_back(std::move(d));
  }
  D.nc = H.levels.back().A.nrows;
  D.cinv = upload_vec<double>(H.coarse_inv, s);
  D.bytes_per_cycle += double(D.nc) * D.nc * 8;
  return D;
}

// Learned pre-smoothing of level 0: x_m = MLP(stencil(D^{-1} b)),
// r_m = b - A x_m, and the device-side choice between x_m and the Jacobi
// sweep (flag), counted when falling back.
template <typename T, int NV>
void mlp_presmooth(DHier<T>& H, const T* b, hipStream_t s) {
  MlpUse& u = *H.mlp;
  DLevel<T>& d0 = H.lev[0];
  T* xm = H.xm->template as<T>();
  T* rm = H.rm->template as<T>();
  const T* dinv = d0.dinv->template as<T>();
  const unsigned grid = mlp_infer_grid(u.n_nodes);
  if (u.d == 2) {
    if (u.per_dof) mlp_infer_kernel<2, true, T><<<grid, 256, 0, s>>>(u.n_nodes, u.nbr, b, dinv, u.w, xm, u.streak,
                                                                       kLearnedStreak);
    else mlp_infer_kernel<2, false, T><<<grid, 256, 0, s>>>(u.n_nodes, u.nbr, b, dinv, u.w, xm, u.streak,
                                                                       kLearnedStreak);
  } else {
    if (u.per_dof) mlp_infer_kernel<3, true, T><<<grid, 256, 0, s>>>(u.n_nodes, u.nbr, b, dinv, u.w, xm, u.streak,
                                                                       kLearnedStreak);
    else mlp_infer_kernel<3, false, T><<<grid, 256, 0, s>>>(u.n_nodes, u.nbr, b, dinv, u.w, xm, u.streak,
                                                                       kLearnedStreak);
  }
  const DCsr<T>& A = d0.A0;
  with_group(A.group, [&](auto gc) {
    constexpr int G = decltype(gc)::value;
    learned_resid_kernel<T, G, NV><<<kDecideBlocks, kBlock, 0, s>>>(A.nrows, A.drp(), A.dci(), A.dval(), xm, b,
                                                                     rm, u.npart, u.streak);
  });
}

template <typename T, int NV>
void vcycle_rec(DHier<T>& H, int l, const T* b, T* out, hipStream_t s, bool plain);

// A level with Chebyshev sweeps of degree k: k step launches (the first from
// x = 0), the restriction b_c = R r_k, the coarse cycle, the coarse
// correction (x += P e, r -= A P e), then k - 1 step launches of which the last
// also applies step k.  out must not alias b.
template <typename T, int NV>
void cheb_level(DHier<T>& H, int l, const T* b, T* out, hipStream_t s, bool plain) {
  DLevel<T>& d = H.lev[l];
  DLevel<T>& c = H.lev[l + 1];
  if (out == b) throw Error(FSI_ERR_ARG, "a Chebyshev V-cycle cannot run in place");
  const int k = d.cheb;
  const Diag<T> dinv = d.diag();
  T* rb[2] = {d.r->template as<T>(), d.r1->template as<T>()};
  T* db[2] = {d.d0->template as<T>(), d.d1->template as<T>()};
  const DCsr<T>& A = d.A0;
  auto step = [&](const T* dp, const T* rp, T a, T cj, T* dout, T* rout, int xinit, int fuse, T a2, T c2) {
    with_group(A.group, [&](auto gc) {
      constexpr int G = decltype(gc)::value;
      cheb_step_kernel<T, G, NV><<<grid_for(A.nrows, kBlock / G), kBlock, 0, s>>>(
          A.nrows, A.drp(), A.dci(), A.dval(), ChebGather<T, NV>{dp, rp, dinv, a, cj}, dout, rout, out, xinit, fuse,
          a2, c2);
    });
  };
  const T* rp = b;
  const T* dp = nullptr;
  int cur = 0;
  T* bc = c.b->template as<T>();
  const bool fused = bool(d.RRA.rp);
  for (int j = 1; j <= k; ++j) {  // pre-smoothing from x = 0
    if (j == k && fused) {  // with b_c = R r_{k-1} - (R A) d_k in the same launch
      with_group(A.group, [&](auto gc) {
        constexpr int G = decltype(gc)::value;
        const unsigned nf = grid_for(A.nrows, kBlock / G);
        auto go = [&](auto gq) {
          constexpr int GC = decltype(gq)::value;
          const unsigned ncb = grid_for(d.RRA.nrows, kBlock / GC);
          cheb_step_restrict_kernel<T, G, GC, NV><<<nf + ncb, kBlock, 0, s>>>(
              A.nrows, A.drp(), A.dci(), A.dval(), ChebGather<T, NV>{dp, rp, dinv, d.ca[j], d.cc[j]}, db[cur],
              rb[cur], out, j == 1, d.RRA.nrows, d.RRA.drp(), d.RRA.dci(), d.RRA.dval(), bc, nf);
        };
        if (d.gres == 64) go(std::integral_constant<int, 64>{});
        else go(std::integral_constant<int, 16>{});
      });
    } else {
      step(dp, rp, d.ca[j], d.cc[j], db[cur], rb[cur], j == 1, 0, T(0), T(0));
    }
    dp = db[cur];
    rp = rb[cur];
    cur ^= 1;
  }
  T* rk = rb[cur ^ 1];
  if (!fused) launch_rows<T, NV>(d.R0, GatherPlain<T, NV>{rk}, EpiStore<T, NV>{bc}, s);
  T* e = c.y->template as<T>();
  vcycle_rec<T, NV>(H, l + 1, bc, e, s, plain);
  with_group(d.gup, [&](auto gc) {
    constexpr int G = decltype(gc)::value;
    cheb_prolong_kernel<T, G, NV><<<grid_for(d.n, kBlock / G), kBlock, 0, s>>>(
        d.n, d.P.drp(), d.P.dci(), d.P.dval(), d.AP.drp(), d.AP.dci(), d.AP.dval(), e, dinv, out, rk, k == 1,
        d.cc[1]);
  });
  dp = nullptr;
  rp = rk;
  for (int j = 1; j < k; ++j) {  // post-smoothing; the last launch also applies step k
    const bool last = j == k - 1;
    step(dp, rp, d.ca[j], d.cc[j], db[cur], rb[cur], 0, last, last ? d.ca[k] : T(0), last ? d.cc[k] : T(0));
    dp = db[cur];
    rp = rb[cur];
    cur ^= 1;
  }
}

// Inverse by k Chebyshev steps alone on the finest matrix (x = 0 start): k - 1
// launches, the last one also applying step k (it needs the row's own
// residual only).  out must not alias b.
template <typename T, int NV>
void cheb_only(DHier<T>& H, const T* b, T* out, hipStream_t s) {
  DLevel<T>& d = H.lev[0];
  if (out == b) throw Error(FSI_ERR_ARG, "a Chebyshev inverse cannot run in place");
  const int k = d.cheb;
  const Diag<T> dinv = d.diag();
  T* rb[2] = {d.r->template as<T>(), d.r1->template as<T>()};
  T* db[2] = {d.d0->template as<T>(), d.d1->template as<T>()};
  const DCsr<T>& A = d.A0;
  const T* rp = b;
  const T* dp = nullptr;
  int cur = 0;
  for (int j = 1; j < k; ++j) {
    const bool last = j == k - 1;
    with_group(A.group, [&](auto gc) {
      constexpr int G = decltype(gc)::value;
      cheb_step_kernel<T, G, NV><<<grid_for(A.nrows, kBlock / G), kBlock, 0, s>>>(
          A.nrows, A.drp(), A.dci(), A.dval(), ChebGather<T, NV>{dp, rp, dinv, d.ca[j], d.cc[j]}, db[cur], rb[cur],
          out, j == 1, last, last ? d.ca[k] : T(0), last ? d.cc[k] : T(0));
    });
    dp = db[cur];
    rp = rb[cur];
    cur ^= 1;
  }
}

// One V(1,1) cycle from level l: two launches per level (down, up) and a
// dense product with the coarsest inverse.  `plain` disables the learned
// pre-smoother (used for the exact corrections it is trained on).
template <typename T, int NV>
void vcycle_rec(DHier<T>& H, int l, const T* b, T* out, hipStream_t s, bool plain) {
  if (H.poly) {
    cheb_only<T, NV>(H, b, out, s);
    return;
  }
  const int L = int(H.lev.size()) - 1;
  if (l == L) {
    const int64_t n = H.nc;
    dense_gemv<T, T, NV>(n, H.cinv->template as<double>(), b, out, s);
    return;
  }
  DLevel<T>& d = H.lev[l];
  DLevel<T>& c = H.lev[l + 1];
  if (d.cheb > 0) {
    cheb_level<T, NV>(H, l, b, out, s, plain);
    return;
  }
  const bool learned = l == 0 && !plain && H.mlp && H.mlp->enabled && H.xm;
  if (learned) mlp_presmooth<T, NV>(H, b, s);
  const Diag<T> dinv = d.diag();
  T* r = d.r->template as<T>();
  T* bc = c.b->template as<T>();
  if constexpr (NV == 1) {
    if (d.rgroup > 1) {  // grouped level (never a learned one)
      with_group(d.gdown, [&](auto gc) {
        constexpr int GA = decltype(gc)::value;
        const unsigned na = grid_for(d.n / d.rgroup, kBlock / GA);
        auto go = [&](auto gq) {
          constexpr int GQ = decltype(gq)::value;
          const unsigned nq = d.split ? 0u : grid_for(d.Q.nrows / d.rgroup, kBlock / GQ);
          with_rgroup(d.rgroup, [&](auto gr) {
            constexpr int GR = decltype(gr)::value;
            vdown_grp_kernel<T, GA, GQ, GR><<<na + nq, kBlock, 0, s>>>(
                d.AD.nrows, d.AD.drp(), d.AD.dci(), d.AD.dval(), d.Q.nrows, d.Q.drp(), d.Q.dci(), d.Q.dval(), b,
                d.omega, r, bc, na);
          });
        };
        if (d.gdownq == 64) go(std::integral_constant<int, 64>{});
        else go(std::integral_constant<int, 16>{});
      });
      if (d.split) launch_rows<T, 1>(d.R0, GatherPlain<T, 1>{r}, EpiStore<T, 1>{bc}, s);  // b_c = R r
      T* e = c.y->template as<T>();
      vcycle_rec<T, NV>(H, l + 1, bc, e, s, plain);
      with_group(d.gup, [&](auto gc) {
        constexpr int G = decltype(gc)::value;
        with_rgroup(d.rgroup, [&](auto gr) {
          constexpr int GR = decltype(gr)::value;
          vup_grp_kernel<T, G, GR><<<grid_for(d.n / d.rgroup, kBlock / G), kBlock, 0, s>>>(
              d.n, d.P.drp(), d.P.dci(), d.P.dval(), d.AP.drp(), d.AP.dci(), d.AP.dval(), e, b, dinv, d.omega, r,
              out);
        });
      });
      return;
    }
  }
  const bool apart = d.split || (d.split_plain && !learned);  // restriction by R in a launch of its own
  with_group(d.gdown, [&](auto gc) {
    constexpr int GA = decltype(gc)::value;
    const unsigned na = grid_for(d.AD.nrows, kBlock / GA);
    auto go = [&](auto gq) {
      constexpr int GQ = decltype(gq)::value;
      const unsigned nq = apart ? 0u : grid_for(d.Q.nrows, kBlock / GQ);
      if (learned)
        vdown_sel_kernel<T, GA, GQ, NV><<<na + nq, kBlock, 0, s>>>(
            d.AD.nrows, d.AD.drp(), d.AD.dci(), d.AD.dval(), d.Q.nrows, d.Q.drp(), d.Q.dci(), d.Q.dval(),
            d.R0.drp(), d.R0.dci(), d.R0.dval(), b, d.omega, r, bc, H.rm->template as<T>(), H.mlp->npart,
            H.mlp->flag, H.mlp->fallbacks, H.mlp->streak, na);
      else if (d.deep)
        vdown_kernel<T, GA, GQ, NV, true><<<na + nq, kBlock, 0, s>>>(d.AD.nrows, d.AD.drp(), d.AD.dci(), d.AD.dval(),
                                                                      d.Q.nrows, d.Q.drp(), d.Q.dci(), d.Q.dval(),
                                                                      b, d.omega, r, bc, na);
      else
        vdown_kernel<T, GA, GQ, NV><<<na + nq, kBlock, 0, s>>>(d.AD.nrows, d.AD.drp(), d.AD.dci(), d.AD.dval(),
                                                                d.Q.nrows, d.Q.drp(), d.Q.dci(), d.Q.dval(), b,
                                                                d.omega, r, bc, na);
    };
    if (d.gdownq == 64) go(std::integral_constant<int, 64>{});
    else go(std::integral_constant<int, 16>{});
  });
  if (apart) launch_rows<T, NV>(d.R0, GatherPlain<T, NV>{r}, EpiStore<T, NV>{bc}, s);  // b_c = R r
  T* e = c.y->template as<T>();
  vcycle_rec<T, NV>(H, l + 1, bc, e, s, plain);
  with_group(d.gup, [&](auto gc) {
    constexpr int G = decltype(gc)::value;
    if (learned)
      vup_sel_kernel<T, G, NV><<<grid_for(d.n, kBlock / G), kBlock, 0, s>>>(
          d.n, d.P.drp(), d.P.dci(), d.P.dval(), d.AP.drp(), d.AP.dci(), d.AP.dval(), e, b, dinv, d.omega, r,
          H.xm->template as<T>(), H.rm->template as<T>(), H.mlp->flag, H.mlp->streak, out);
    else if (d.deep)
      vup_kernel<T, G, NV, true><<<grid_for(d.n, kBlock / G), kBlock, 0, s>>>(
          d.n, d.P.drp(), d.P.dci(), d.P.dval(), d.AP.drp(), d.AP.dci(), d.AP.dval(), e, b, dinv, d.omega, r, out);
    else
      vup_kernel<T, G, NV><<<grid_for(d.n, kBlock / G), kBlock, 0, s>>>(d.n, d.P.drp(), d.P.dci(), d.P.dval(),
                                                                        d.AP.drp(), d.AP.dci(), d.AP.dval(), e, b,
                                                                        dinv, d.omega, r, out);
  });
}

// Record the input of this cycle (every `every`-th call) for training.
template <typename T>
void record_input(DHier<T>& H, const T* b, hipStream_t s) {
  MlpRecord& R = *H.rec;
  if (++R.calls % R.every != 0 || int(R.vecs.size()) >= R.max_vectors) return;
  const int64_t n = H.lev[0].n * H.nv;
  auto v = std::make_shared<DevBuf>();
  v->alloc(sizeof(double) * n);
  cast_kernel<T, double><<<grid_for(n, kBlock * 4), kBlock, 0, s>>>(n, b, v->as<double>());
  R.vecs.push_back(v);
}

template <typename T>
void vcycle(DHier<T>& H, const T* b, T* out, hipStream_t s, bool plain = false) {
  if (H.rec && H.rec->active && !plain) record_input(H, b, s);
  switch (H.nv) {
    case 1: vcycle_rec<T, 1>(H, 0, b, out, s, plain); break;
    case 2: vcycle_rec<T, 2>(H, 0, b, out, s, plain); break;
    default: vcycle_rec<T, 3>(H, 0, b, out, s, plain); break;
  }
}

// ------------------------------------------------------ block preconditioner
template <typename T>
struct Precond {
  int d = 2;
  int64_t n_m = 0, n_s = 0, n_f = 0, n_vs = 0, n_vf = 0, n_p = 0, N = 0;
  DHier<T> H[FSI_NHIER];
  DCsr<T> S_vu, S_uv, Cfms, Csf, Cms, Dm, Gm;
  std::shared_ptr<DevBuf> tu, tu2, tv, tf, ta, ta2, tp, ts, ts2, tm, tm2, rT, zT;
  // inner GMRES of the fluid step (inner_k > 0): F, Arnoldi vectors V
  // ((k + 1) x n_f), preconditioned vectors Z (k x n_f), FP64 scalars,
  // breakdown flags (ibrk: one per step, and one for a zero residual)
  int inner_k = 0;
  int inner_pc = FSI_INNER_UZAWA;
  DCsr<T> Fm;
  // Section 4.4 as written (uz_k > 0): every inverse of the Uzawa-like step
  // taken as uz_k GMRES steps on A_f (velocity rows grouped d at a time) or
  // on S_p, preconditioned by its V-cycle; they share the inner buffers
  int uz_k = 0;
  DCsr<T> Am, Spm;
  int order = FSI_ORDER_MSF;  // block order of the factorisation
  std::shared_ptr<DevBuf> tf2;  // other orders: the second fluid inverse's output
  DCsr<T> Cfm, Cfs;             // orders with the fluid in the middle: C_fm and C_fs apart
  std::shared_ptr<DevBuf> iV, iZ, ipart, iscal, ibrk;
  int inner_nb = 1;

  void alloc_tmp() {
    auto mk = [](int64_t n) {
      auto b = std::make_shared<DevBuf>();
      b->alloc(sizeof(T) * std::max<int64_t>(n, 1));
      return b;
    };
    tu = mk(n_vs); tu2 = mk(n_vs); tv = mk(n_vs);
    tf = mk(n_f); ta = mk(n_vf); ta2 = mk(n_vf); tp = mk(n_p);
    ts = mk(n_s); ts2 = mk(n_s); tm = mk(n_m); tm2 = mk(n_m);
    if (order != FSI_ORDER_MSF) tf2 = mk(n_f);
    if (sizeof(T) != sizeof(double)) { rT = mk(N); zT = mk(N); }
    const int kmax = std::max(inner_k, uz_k);
    if (kmax > 0) {
      iV = mk((kmax + 1) * n_f);
      iZ = mk(kmax * n_f);
      inner_nb = int(std::min<int64_t>(kInnerBlocks, std::max<int64_t>(1, (n_f + kBlock - 1) / kBlock)));
      ipart = std::make_shared<DevBuf>();
      ipart->alloc(sizeof(double) * (kInnerMax + 1) * inner_nb);
      iscal = std::make_shared<DevBuf>();
      iscal->alloc(sizeof(double) * kInnerScal);
      ibrk = std::make_shared<DevBuf>();
      ibrk->alloc(sizeof(int) * (kInnerMax + 1));
    }
  }

  // FP64 scalars of the inner GMRES: two Gram-Schmidt passes and a norm
  // (kInnerMax + 2 each), beta, the Hessenberg matrix
  static constexpr int kInnerScal = 3 * (kInnerMax + 2) + 1 + (kInnerMax + 1) * kInnerMax;

  // Solid algorithm of Section 4.3 (u_s eliminated through Sigma_s):
  //   y = M_s^{-1} r_u;  x_v = Sigma_s^{-1} (r_v - S_vu y);  x_u = M_s^{-1} (r_u - S_uv x_v)
  void solid(const T* r_s, T* z_s, hipStream_t s) {
    const T* r_v = r_s;
    const T* r_u = r_s + n_vs;
    T* z_v = z_s;
    T* z_u = z_s + n_vs;
    vcycle(H[FSI_H_MS], r_u, tu->as<T>(), s);
    spmv_sub<T>(S_vu, tu->as<T>(), r_v, tv->as<T>(), s);
    vcycle(H[FSI_H_SIG], tv->as<T>(), z_v, s);
    spmv_sub<T>(S_uv, z_v, r_u, tu2->as<T>(), s);
    vcycle(H[FSI_H_MS], tu2->as<T>(), z_u, s);
  }

  // Uzawa-like elimination of the fluid saddle point (Section 4.4):
  //   y = A_f^{-1} r_v;  x_p = S_p^{-1} (r_p - D y);  x_v = A_f^{-1} (r_v - G x_p)
  void fluid(const T* r_f, T* z_f, hipStream_t s) {
    const T* r_v = r_f;
    const T* r_p = r_f + n_vf;
    vcycle(H[FSI_H_A], r_v, ta->as<T>(), s);
    spmv_sub<T>(Dm, ta->as<T>(), r_p, tp->as<T>(), s);
    vcycle(H[FSI_H_P], tp->as<T>(), z_f + n_vf, s);
    spmv_sub<T>(Gm, z_f + n_vf, r_v, ta2->as<T>(), s);
    vcycle(H[FSI_H_A], ta2->as<T>(), z_f, s);
  }

  // Block upper-triangular step, the inverse of [[A_f, G], [0, S_p]]:
  //   x_p = S_p^{-1} r_p;  x_v = A_f^{-1} (r_v - G x_p)
  void fluid_tri(const T* r_f, T* z_f, hipStream_t s) {
    const T* r_v = r_f;
    const T* r_p = r_f + n_vf;
    vcycle(H[FSI_H_P], r_p, z_f + n_vf, s);
    spmv_sub<T>(Gm, z_f + n_vf, r_v, ta2->as<T>(), s);
    vcycle(H[FSI_H_A], ta2->as<T>(), z_f, s);
  }

  // The fluid sub-problem solved by k steps of flexible GMRES on F from zero,
  // right-preconditioned by the Uzawa-like step (Section 4.4): z_f minimises
  // ||r_f - F z|| over the span of the preconditioned Arnoldi vectors.
  // Classical Gram-Schmidt with one reorthogonalisation; every scalar stays
  // on the device.
  // one Gram-Schmidt pass (update by nu vectors, nd dot products and the
  // norm) and its block-order reduction into out[0..nd]
  void inner_pass(int64_t n, int nu, int nd, const double* h, T* w, double* out, hipStream_t s) {
    inner_pass_kernel<T><<<inner_nb, kBlock, 0, s>>>(n, nu, nd, iV->as<T>(), n, h, w, ipart->as<double>());
    gs_reduce_kernel<<<nd + 1, kBlock, 0, s>>>(inner_nb, 0, ipart->as<double>(), out);
  }

  // k steps of flexible GMRES on an n x n operator from zero, right
  // preconditioned: pc(v, z) forms z_j = M^{-1} v_j, op(z, w) forms
  // w = A z_j.  z minimises ||r - A z|| over the span of the z_j.  Classical
  // Gram-Schmidt with one reorthogonalisation, stopping early only at an
  // exact solve; every scalar stays on the device (one captured graph).
  template <class PC, class OP>
  void gmres_steps(int k, int64_t n, PC&& pc, OP&& op, const T* r, T* z, hipStream_t s) {
    const unsigned g = grid_for(n, kBlock * 4);
    T* V = iV->as<T>();
    T* Z = iZ->as<T>();
    double* a1 = iscal->as<double>();
    double* a2 = a1 + (kInnerMax + 2);
    double* nn = a2 + (kInnerMax + 2);
    double* beta = nn + (kInnerMax + 2);
    double* Hm = beta + 1;
    int* brk = ibrk->as<int>();
    // ||r||^2 (r read as "w" with no update: the pass only reads it)
    inner_pass(n, 0, 0, nullptr, const_cast<T*>(r), nn, s);
    inner_start_kernel<T><<<g, kBlock, 0, s>>>(n, nn, beta, brk, r, V);
    for (int j = 0; j < k; ++j) {
      T* zj = Z + int64_t(j) * n;
      T* w = V + int64_t(j + 1) * n;
      pc(static_cast<const T*>(V + int64_t(j) * n), zj);
      op(static_cast<const T*>(zj), w);
      inner_pass(n, 0, j + 1, nullptr, w, a1, s);   // h1 = V^T w, ||w||^2
      inner_pass(n, j + 1, j + 1, a1, w, a2, s);    // w -= V h1; h2 = V^T w
      inner_pass(n, j + 1, 0, a2, w, nn, s);        // w -= V h2; ||w||^2
      inner_column_kernel<T><<<g, kBlock, 0, s>>>(n, j, k, a1, a2, nn, Hm, brk, w);
    }
    inner_combine_kernel<T><<<g, kBlock, 0, s>>>(n, k, Z, n, Hm, beta, brk, z);
  }

  // The fluid sub-problem solved by k steps of flexible GMRES on F from zero,
  // right-preconditioned by the Uzawa-like step or the block upper-triangular
  // step: z_f minimises ||r_f - F z|| over the span of the preconditioned
  // Arnoldi vectors.
  void fluid_gmres(const T* r_f, T* z_f, hipStream_t s) {
    gmres_steps(
        inner_k, n_f,
        [&](const T* v, T* zj) {
          if (inner_pc == FSI_INNER_TRIANGULAR) fluid_tri(v, zj, s);
          else fluid(v, zj, s);
        },
        [&](const T* zj, T* w) { launch_rows<T, 1>(Fm, GatherPlain<T, 1>{zj}, EpiStoreFluid<T, 1>{{w}}, s); },
        r_f, z_f, s);
  }

  // Section 4.4 as written: the Uzawa-like elimination with every occurring
  // inverse approximated by AMG-preconditioned GMRES (uz_k steps each):
  //   y = A_f^{-1} r_v;  x_p = S_p^{-1} (r_p - D y);  x_v = A_f^{-1} (r_v - G x_p)
  void fluid_uzawa_gmres(const T* r_f, T* z_f, hipStream_t s) {
    const T* r_v = r_f;
    const T* r_p = r_f + n_vf;
    auto pc_a = [&](const T* v, T* zj) { vcycle(H[FSI_H_A], v, zj, s); };
    auto op_a = [&](const T* zj, T* w) {
      launch_rows<T, 1>(Am, GatherPlain<T, 1>{zj}, EpiStoreFluid<T, 1>{{w}}, s);
    };
    auto pc_p = [&](const T* v, T* zj) { vcycle(H[FSI_H_P], v, zj, s); };
    auto op_p = [&](const T* zj, T* w) {
      launch_rows<T, 1>(Spm, GatherPlain<T, 1>{zj}, EpiStoreFluid<T, 1>{{w}}, s);
    };
    gmres_steps(uz_k, n_vf, pc_a, op_a, r_v, ta->as<T>(), s);
    spmv_sub<T>(Dm, ta->as<T>(), r_p, tp->as<T>(), s);
    gmres_steps(uz_k, n_p, pc_p, op_p, static_cast<const T*>(tp->as<T>()), z_f + n_vf, s);
    spmv_sub<T>(Gm, z_f + n_vf, r_v, ta2->as<T>(), s);
    gmres_steps(uz_k, n_vf, pc_a, op_a, static_cast<const T*>(ta2->as<T>()), z_f, s);
  }

  void fluid_inverse(const T* r_f, T* z_f, hipStream_t s) {
    if (inner_k > 0 && n_f > 0) fluid_gmres(r_f, z_f, s);
    else if (uz_k > 0 && n_vf > 0 && n_p > 0) fluid_uzawa_gmres(r_f, z_f, s);
    else fluid(r_f, z_f, s);
  }

  // Fields of a block order (0 mesh, 1 solid, 2 fluid), in FSI_ORDER_* order.
  static constexpr int kOrderFields[6][3] = {{0, 1, 2}, {2, 1, 0}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}};

  int64_t field_off(int i) const { return i == 0 ? 0 : (i == 1 ? n_m : n_m + n_s); }

  // Which couplings A_ij x_j (j among o[j0..j1)) row field i has: the
  // fluid rows couple to mesh and solid, the solid rows to the fluid, the
  // mesh rows to the solid (C_sm is dropped; there is no mesh-fluid block).
  static void coupled_to(int i, const int* o, int j0, int j1, bool& m, bool& sd, bool& f) {
    m = sd = f = false;
    for (int k = j0; k < j1; ++k) {
      if (i == 2 && o[k] == 0) m = true;
      if (i == 2 && o[k] == 1) sd = true;
      if (i == 1 && o[k] == 2) f = true;
      if (i == 0 && o[k] == 1) sd = true;
    }
  }

  // Bytes of sum_j A_ij x_j over j among o[j0..j1) (0 when there is none);
  // touches 2 for r - A x.
  double coupling_bytes(int i, const int* o, int j0, int j1, int touches) const {
    const double w = double(sizeof(T));
    bool m, sd, f;
    coupled_to(i, o, j0, j1, m, sd, f);
    auto prod = [&](const DCsr<T>& A, int64_t nin, int64_t nout) {
      return A.bytes() + w * (double(nin) + touches * double(nout));
    };
    if (i == 2 && m && sd) return prod(Cfms, n_m + n_s, n_f);
    if (i == 2 && m) return prod(Cfm, n_m, n_f);
    if (i == 2 && sd) return prod(Cfs, n_s, n_f);
    if (i == 1 && f) return prod(Csf, n_f, n_s);
    if (i == 0 && sd) return prod(Cms, n_s, n_m);
    return 0.0;
  }

  // out = sum_j A_ij z_j (sub: out = r_i - sum_j A_ij z_j) over j among
  // o[j0..j1); false (nothing written) when row field i has none of them.
  bool couple(int i, const int* o, int j0, int j1, const T* r_i, const T* z, T* out, bool sub, hipStream_t s) {
    bool m, sd, f;
    coupled_to(i, o, j0, j1, m, sd, f);
    const DCsr<T>* A = nullptr;
    const T* x = nullptr;
    if (i == 2 && m && sd) { A = &Cfms; x = z; }  // [x_m | x_s] are contiguous
    else if (i == 2 && m) { A = &Cfm; x = z; }
    else if (i == 2 && sd) { A = &Cfs; x = z + n_m; }
    else if (i == 1 && f) { A = &Csf; x = z + n_m + n_s; }
    else if (i == 0 && sd) { A = &Cms; x = z + n_m; }
    if (!A) return false;
    if (sub) spmv_sub<T>(*A, x, r_i, out, s);
    else spmv<T>(*A, x, out, s);
    return true;
  }

  void field_inverse(int i, const T* in, T* out, hipStream_t s) {
    if (i == 0) vcycle(H[FSI_H_M], in, out, s);
    else if (i == 1) solid(in, out, s);
    else fluid_inverse(in, out, s);
  }

  // The factorisation with the fields in another order (a, b, c), its
  // perturbations dropped as the paper drops its own: a block symmetric
  // Gauss-Seidel sweep in that order,
  //   forward   x_i = A_ii^{-1} (r_i - sum_{j before i} A_ij x_j),
  //   backward  x_i -= A_ii^{-1} sum_{j after i} A_ij x_j   (i = b, then a).
  void apply_ordered(const T* r, T* z, hipStream_t s) {
    const int* o = kOrderFields[order];
    T* t_in[3] = {tm->as<T>(), ts->as<T>(), tf->as<T>()};
    T* t_out[3] = {tm2->as<T>(), ts2->as<T>(), tf2->as<T>()};
    const int64_t nb[3] = {n_m, n_s, n_f};
    for (int k = 0; k < 3; ++k) {
      const int i = o[k];
      const T* r_i = r + field_off(i);
      const bool c = couple(i, o, 0, k, r_i, z, t_in[i], true, s);
      field_inverse(i, c ? static_cast<const T*>(t_in[i]) : r_i, z + field_off(i), s);
    }
    for (int k = 1; k >= 0; --k) {
      const int i = o[k];
      if (!couple(i, o, k + 1, 3, nullptr, z, t_in[i], false, s)) continue;
      field_inverse(i, t_in[i], t_out[i], s);
      vsub<T>(nb[i], z + field_off(i), t_out[i], s);
    }
  }

  // Bytes one application of P^{-1} moves as stored: every V-cycle (or
  // Chebyshev-only inverse) as executed, every product's matrix once with its
  // input read and its output written (and read, for r - A x) once, the
  // inner GMRES vectors and the vector updates.
  double bytes_per_apply() const {
    const double w = double(sizeof(T));
    auto prod = [&](const DCsr<T>& A, int64_t nin, int64_t nout, int touches) {
      return A.bytes() + w * (double(nin) + touches * double(nout));
    };
    const double mesh = H[FSI_H_M].bytes_per_cycle;
    const double solid = 2 * H[FSI_H_MS].bytes_per_cycle + H[FSI_H_SIG].bytes_per_cycle +
                         prod(S_vu, n_vs, n_vs, 2) + prod(S_uv, n_vs, n_vs, 2);
    const double uzawa = 2 * H[FSI_H_A].bytes_per_cycle + H[FSI_H_P].bytes_per_cycle + prod(Dm, n_vf, n_p, 2) +
                         prod(Gm, n_p, n_vf, 2);
    const double tri = H[FSI_H_A].bytes_per_cycle + H[FSI_H_P].bytes_per_cycle + prod(Gm, n_p, n_vf, 2);
    // k GMRES steps on n unknowns: ||r|| and v_0 = r / beta; per step the
    // preconditioner, the product, three passes over j+1 vectors and the
    // column; z = Z y
    auto gmres = [&](int k, int64_t n, double pcb, double opb) {
      double b = w * double(n) * 3.0;
      for (int j = 0; j < k; ++j) b += pcb + opb + w * double(n) * (3.0 * j + 10.0);
      return b + w * double(n) * (k + 1);
    };
    double fluid = uzawa;
    if (inner_k > 0 && n_f > 0) {
      const double pc = inner_pc == FSI_INNER_TRIANGULAR ? tri : uzawa;
      fluid = gmres(inner_k, n_f, pc, prod(Fm, n_f, n_f, 1));
    } else if (uz_k > 0 && n_vf > 0 && n_p > 0) {
      const double ga = gmres(uz_k, n_vf, H[FSI_H_A].bytes_per_cycle, prod(Am, n_vf, n_vf, 1));
      fluid = 2 * ga + gmres(uz_k, n_p, H[FSI_H_P].bytes_per_cycle, prod(Spm, n_p, n_p, 1)) +
              prod(Dm, n_vf, n_p, 2) + prod(Gm, n_p, n_vf, 2);
    }
    if (order != FSI_ORDER_MSF) {
      // the steps of apply_ordered: an inverse per field, a second one for
      // every backward update, the coupling products (r - A x reads r too)
      const double inv_b[3] = {mesh, solid, fluid};
      const int64_t nb[3] = {n_m, n_s, n_f};
      const int* o = kOrderFields[order];
      double b = 0.0;
      for (int k = 0; k < 3; ++k) {
        b += inv_b[o[k]];
        b += coupling_bytes(o[k], o, 0, k, 2);
      }
      for (int k = 1; k >= 0; --k) {
        const double cb = coupling_bytes(o[k], o, k + 1, 3, 1);
        if (cb > 0.0) b += inv_b[o[k]] + cb + 3.0 * w * double(nb[o[k]]);
      }
      return b;
    }
    return 2 * mesh + 2 * solid + prod(Cfms, n_m + n_s, n_f, 2) + fluid + prod(Csf, n_f, n_s, 1) +
           prod(Cms, n_s, n_m, 1) + 3.0 * w * double(n_s + n_m);
  }

  // Block LDU algorithm of Section 4.1 ("Evaluation of P^{-1} r").
  void apply(const T* r, T* z, hipStream_t s) {
    const T* r_m = r;
    const T* r_s = r + n_m;
    const T* r_f = r + n_m + n_s;
    T* z_m = z;
    T* z_s = z + n_m;
    T* z_f = z + n_m + n_s;
    if (order != FSI_ORDER_MSF) {
      apply_ordered(r, z, s);
      return;
    }
    vcycle(H[FSI_H_M], r_m, z_m, s);                         // 1. x_m = M^{-1} r_m
    solid(r_s, z_s, s);                                      // 2. x_s = S^{-1} r_s
    spmv_sub<T>(Cfms, z, r_f, tf->as<T>(), s);               // 3. r_f - C_fm x_m - C_fs x_s
    fluid_inverse(tf->as<T>(), z_f, s);                      //    x_f = F^{-1} (...)
    spmv<T>(Csf, z_f, ts->as<T>(), s);                       // 4. x_s -= S^{-1} C_sf x_f
    solid(ts->as<T>(), ts2->as<T>(), s);
    vsub<T>(n_s, z_s, ts2->as<T>(), s);
    spmv<T>(Cms, z_s, tm->as<T>(), s);                       // 5. x_m -= M^{-1} C_ms x_s
    vcycle(H[FSI_H_M], tm->as<T>(), tm2->as<T>(), s);
    vsub<T>(n_m, z_m, tm2->as<T>(), s);
  }
};

}  // namespace fsi

using namespace fsi;

// Learned smoother of one hierarchy (index 0: H_M, 1: H_SIG): weights,
// optimiser state, stencil table, training samples and recording.  It
// survives fsi_setup_blocks / fsi_build_precond (a trained network is reused
// on the next Newton systems of the same lattice).
struct MlpState {
  bool have_weights = false;
  int d = 0;
  int64_t n_nodes = 0;
  MlpUse use;
  MlpRecord rec;
  std::vector<float> wnode;  // node weights of the loss (mean diagonal / operator mean)
  DevBuf nbr, npart, flag, fallbacks, streak;
  DevBuf wm, m1, m2, g, loss, w1t, w2t, w2, w3t, w3, part, part_loss, part2, loss2;
  int adam_t = 0;
  int nparam() const { return d == 2 ? MlpDims<2>::NPARAM : MlpDims<3>::NPARAM; }
  int kp() const { return d == 2 ? MlpDims<2>::KP : MlpDims<3>::KP; }
  int kin() const { return d == 2 ? MlpDims<2>::KIN : MlpDims<3>::KIN; }
};

// Finite-element description uploaded by fsi_fe_setup: the grid, the
// material data and the node arrays; the block patterns are uploaded on the
// first read-back of block values.
struct FeState {
  FeParams prm{};
  int64_t n_nodes = 0;
  DevBuf vdof, udof, pdof, v, u, p, v_old, u_old, w, u_fz, flag, part;
  DevBuf basis;  // basis values and weights at the quadrature points (the same for every cell)
  DevBuf pts;    // integrand values and derivatives at every point of the cells of one launch
  std::shared_ptr<DevBuf> brp[FSI_NBLK], bci[FSI_NBLK];
  std::vector<double> spare[FSI_NBLK];  // host value arrays of the blocks' previous values, reused
  FeNodes nodes() const {
    return FeNodes{vdof.as<int64_t>(), udof.as<int64_t>(), pdof.as<int64_t>(), v.as<double>(),
                   u.as<double>(),     p.as<double>(),     v_old.as<double>(), u_old.as<double>(),
                   w.as<double>(),     u_fz.as<double>()};
  }
};

// ------------------------------------------------------------------ context
struct fsi_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  float* scratch = nullptr;  // this device's address of the allocation-free staging array
  std::string err;
  // system
  bool have_system = false, have_precond = false;
  int d = 2;
  int64_t n_m = 0, n_s = 0, n_f = 0, n_vs = 0, n_vf = 0, n_p = 0, N = 0;
  double dt_theta = 0.0;
  std::vector<double> coords;
  std::vector<int32_t> dof_node;
  std::vector<int32_t> node_ijk;  // empty: no lattice, no learned smoother
  HCsr blk[FSI_NBLK];
  MlpState mlp[2];
  DCsr<double> Ah;
  std::unique_ptr<FeState> fe;  // fsi_fe_setup
  // preconditioner
  fsi_precond_opts popts{};     // options of the last fsi_build_precond
  bool have_popts = false;
  int precision = FSI_P_F64;
  int gs_blocks = kGsBlocks;
  int cheb[FSI_NHIER] = {0, 0, 0, 0, 0};  // Chebyshev degree per hierarchy (0: Jacobi)
  int poly[FSI_NHIER] = {0, 0, 0, 0, 0};  // Chebyshev steps alone, no coarse grid (0: off)
  int fluid_inner = 0;                     // inner GMRES steps of the fluid inverse (0: off)
  int fluid_inner_pc = FSI_INNER_UZAWA;    // their preconditioner
  int uzawa_inner = 0;                     // GMRES steps per inverse of the Uzawa-like step (0: off)
  int order = FSI_ORDER_MSF;               // block order of the factorisation
  double poly_ratio = 8.0;
  SaHierarchy host_h[FSI_NHIER];
  bool have_host_h = false;  // host_h built for the current system
  SaParams host_prm;         // the SA parameters and pressure Schur option host_h was built with
  int host_schur = FSI_SCHUR_SIMPLE;
  int host_x_approx = FSI_X_F;
  HCsr fluid_op;             // FSI_X_BLOCKDIAG: the preconditioner's fluid operator (else F is used)
  std::unique_ptr<Precond<double>> p64;
  std::unique_ptr<Precond<float>> p32;
  // Krylov workspace
  int m_alloc = -1;
  DevBuf V, Z, part, dh, dy, flag;
  double* hpin = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  // one captured HIP graph per Arnoldi step j (its kernels depend on j);
  // captured on a private stream, launched on the context stream
  bool use_graphs = true;
  hipStream_t cap_stream = nullptr;
  std::vector<hipGraphExec_t> step_graph;  // whole step j
  std::vector<hipGraphExec_t> pre_graph;   // timed mode: P^{-1} v_j
  std::vector<hipGraphExec_t> gs_graph;    // timed mode: Gram-Schmidt + copy of step j
  hipEvent_t tev[2][4] = {};  // phase events of the two in-flight Arnoldi steps
  hipEvent_t tsolve[2] = {nullptr, nullptr};  // start / end of a whole solve
  void drop_graphs() {
    for (auto* v : {&step_graph, &pre_graph, &gs_graph}) {
      for (auto& g : *v)
        if (g) (void)hipGraphExecDestroy(g);
      v->clear();
    }
  }
  ~fsi_ctx() {
    drop_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (hpin) (void)hipHostFree(hpin);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    for (auto& r : tev)
      for (auto& e : r)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : tsolve)
      if (e) (void)hipEventDestroy(e);
  }
};

namespace {

thread_local std::string g_create_err;

fsi_status set_err(fsi_ctx* c, fsi_status code, const std::string& m) {
  if (c) c->err = m;
  return code;
}

template <class F>
fsi_status guarded(fsi_ctx* c, F&& f) {
  if (!c) return FSI_ERR_ARG;
  try {
    HIP_TRY(hipSetDevice(c->device));
    fsi_status st = f();
    if (st >= 0) c->err.clear();
    return st;
  } catch (const Error& e) {
    return set_err(c, e.code, e.what());
  } catch (const std::bad_alloc&) {
    return set_err(c, FSI_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return set_err(c, FSI_ERR_HIP, e.what());
  }
}

void check_device_ptr(const void* p, const char* what) {
  if (!p) throw Error(FSI_ERR_ARG, std::string(what) + " is NULL");
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess || at.type != hipMemoryTypeDevice) {
    (void)hipGetLastError();
    throw Error(FSI_ERR_ARG, std::string(what) + " is not a device pointer");
  }
}

// Rigid-body modes of the solid velocity nodes, centred at their centroid:
// d translations, then rotations (2D: (-y, x); 3D: about x, y, z).
std::vector<double> rigid_modes(const fsi_ctx& c, int& k) {
  const int d = c.d;
  const int64_t nn = c.n_vs / d;
  std::vector<double> xyz(nn * d), cen(d, 0.0);
  for (int64_t i = 0; i < nn; ++i) {
    const int32_t node = c.dof_node[c.n_m + i * d];
    for (int a = 0; a < d; ++a) xyz[i * d + a] = c.coords[int64_t(node) * d + a];
  }
  for (int64_t i = 0; i < nn; ++i)
    for (int a = 0; a < d; ++a) cen[a] += xyz[i * d + a];
  for (int a = 0; a < d; ++a) cen[a] /= double(nn);
  k = d == 2 ? 3 : 6;
  std::vector<double> B(size_t(c.n_vs) * k, 0.0);
  for (int64_t i = 0; i < nn; ++i) {
    const double x = xyz[i * d] - cen[0], y = xyz[i * d + 1] - cen[1];
    const double z = d == 3 ? xyz[i * d + 2] - cen[2] : 0.0;
    auto at = [&](int comp, int col) -> double& { return B[size_t(i * d + comp) * k + col]; };
    for (int t = 0; t < d; ++t) at(t, t) = 1.0;
    if (d == 2) {
      at(0, 2) = -y;
      at(1, 2) = x;
    } else {
      at(1, 3) = -z; at(2, 3) = y;
      at(0, 4) = z;  at(2, 4) = -x;
      at(0, 5) = -y; at(1, 5) = x;
    }
  }
  return B;
}

// Components per node of the operator of hierarchy h: d for the vector
// blocks (solid Schur matrix, solid mass block, fluid velocity block), 1 for
// the scalar mesh Laplacian and the pressure Schur approximation.
int node_components(const fsi_ctx& c, int h) {
  return h == FSI_H_SIG || h == FSI_H_MS || h == FSI_H_A ? c.d : 1;
}

// The learned pre-smoother exists for H_M and H_SIG with Jacobi sweeps and
// lattice indices of the nodes.
bool learned_capable(const fsi_ctx& c, int h) {
  return !c.node_ijk.empty() && (h == FSI_H_M || h == FSI_H_SIG) && c.cheb[h] == 0 && c.poly[h] == 0 &&
         c.precision != FSI_P_F32_BF16DIAG;
}

// Point the finest levels of H_M and H_SIG at their learned smoothers (or at
// none when the hierarchy has a single level).
template <typename T>
void link_mlp(fsi_ctx& c, Precond<T>& P) {
  for (int i = 0; i < 2; ++i) {
    DHier<T>& H = P.H[i == 0 ? FSI_H_M : FSI_H_SIG];
    const bool ok = H.xm && c.mlp[i].n_nodes > 0;
    H.mlp = ok ? &c.mlp[i].use : nullptr;
    H.rec = ok ? &c.mlp[i].rec : nullptr;
  }
}

template <typename T>
std::unique_ptr<Precond<T>> make_precond(fsi_ctx& c) {
  auto P = std::make_unique<Precond<T>>();
  hipStream_t s = c.stream;
  P->d = c.d;
  P->n_m = c.n_m; P->n_s = c.n_s; P->n_f = c.n_f; P->n_vs = c.n_vs; P->n_vf = c.n_vf;
  P->n_p = c.n_p; P->N = c.N;
  static const char* hname[FSI_NHIER] = {"H_M", "H_SIG", "H_MS", "H_A", "H_P"};
  for (int h = 0; h < FSI_NHIER; ++h) {
    PhaseTimer t("upload (products, grouping, copies)");
    P->H[h] = upload_hier<T>(c.host_h[h], h == FSI_H_M ? c.d : 1, s, learned_capable(c, h), c.cheb[h], c.poly[h],
                             c.poly_ratio, node_components(c, h), c.precision == FSI_P_F32_BF16DIAG);
    if (log_on()) {
      HIP_TRY(hipStreamSynchronize(s));
      log_line("upload %s: %.1f ms (%zu levels, %.3f GB per cycle)", hname[h], t.ms(), P->H[h].lev.size(),
           P->H[h].bytes_per_cycle / 1e9);
    }
  }
  link_mlp(c, *P);
  PhaseTimer t_cb("coupling blocks (and F for the inner steps)");
  const HCsr& S = c.blk[FSI_S];
  const HCsr& F = c.host_x_approx == FSI_X_BLOCKDIAG ? c.fluid_op : c.blk[FSI_F];  // F, or its refinement
  P->S_vu = upload<T>(sub_block(S, 0, c.n_vs, c.n_vs, c.n_s), s);
  P->S_uv = upload<T>(sub_block(S, c.n_vs, c.n_s, 0, c.n_vs), s);
  P->Dm = upload<T>(sub_block(F, c.n_vf, c.n_f, 0, c.n_vf), s);
  P->Gm = upload<T>(sub_block(F, 0, c.n_vf, c.n_vf, c.n_f), s);
  P->Csf = upload<T>(c.blk[FSI_CSF], s);
  P->Cms = upload<T>(c.blk[FSI_CMS], s);
  // C_fm and C_fs merged into one product over the contiguous [x_m | x_s]
  {
    const HCsr& A = c.blk[FSI_CFM];
    const HCsr& B = c.blk[FSI_CFS];
    const int32_t nm = int32_t(c.n_m);
    HCsr M = build_rows(
        c.n_f, c.n_m + c.n_s, [&](int64_t i) { return A.rp[i + 1] - A.rp[i] + B.rp[i + 1] - B.rp[i]; },
        [&](int64_t i, int32_t* oc, double* ov) {
          for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) { *oc++ = A.ci[k]; *ov++ = A.v[k]; }
          for (int64_t k = B.rp[i]; k < B.rp[i + 1]; ++k) { *oc++ = B.ci[k] + nm; *ov++ = B.v[k]; }
        });
    // velocity rows in groups of d (a node's rows share their columns), then
    // the pressure rows
    const int64_t bounds[3] = {0, c.n_vf, c.n_f};
    const int groups[2] = {c.d, 1};
    P->Cfms = upload_segments<T>(M, bounds, groups, 2, s);
    P->inner_k = c.fluid_inner;
    P->inner_pc = c.fluid_inner_pc;
    if (c.fluid_inner > 0) P->Fm = upload_segments<T>(F, bounds, groups, 2, s);
    P->order = c.order;
    if (c.order == FSI_ORDER_MFS || c.order == FSI_ORDER_SFM) {  // the fluid in the middle
      P->Cfm = upload<T>(c.blk[FSI_CFM], s);
      P->Cfs = upload<T>(c.blk[FSI_CFS], s);
    }
    P->uz_k = c.uzawa_inner;
    if (c.uzawa_inner > 0) {
      const int64_t vb[2] = {0, c.n_vf};
      const int vg[1] = {c.d};
      P->Am = upload_segments<T>(sub_block(F, 0, c.n_vf, 0, c.n_vf), vb, vg, 1, s);
      P->Spm = upload<T>(c.host_h[FSI_H_P].levels[0].A, s);
    }
  }
  P->alloc_tmp();
  HIP_TRY(hipStreamSynchronize(s));
  t_cb.done();
  return P;
}

void apply_precond(fsi_ctx& c, const double* r, double* z, hipStream_t s) {
  if (c.precision == FSI_P_F64) {
    c.p64->apply(r, z, s);
  } else {
    Precond<float>& P = *c.p32;
    cast_kernel<double, float><<<grid_for(c.N, kBlock * 4), kBlock, 0, s>>>(c.N, r, P.rT->as<float>());
    P.apply(P.rT->as<float>(), P.zT->as<float>(), s);
    cast_kernel<float, double><<<grid_for(c.N, kBlock * 4), kBlock, 0, s>>>(c.N, P.zT->as<float>(), z);
  }
}

// Bytes of one P^{-1} r (FP32 precisions: with the casts of r and z).
double precond_bytes(const fsi_ctx& c) {
  if (c.precision == FSI_P_F64) return c.p64->bytes_per_apply();
  return c.p32->bytes_per_apply() + 24.0 * double(c.N);
}

template <typename T>
DHier<T>& hier_of(fsi_ctx& c, int which) {
  if constexpr (sizeof(T) == sizeof(double)) return c.p64->H[which];
  else return c.p32->H[which];
}

void ensure_krylov(fsi_ctx& c, int m) {
  if (c.m_alloc == m) return;
  c.drop_graphs();
  c.V.alloc(sizeof(double) * size_t(m + 1) * c.N);
  c.Z.alloc(sizeof(double) * size_t(m) * c.N);
  // Gram-Schmidt blocks: about four elements per thread (one reduction per
  // tile of vectors is shared by more elements), two below 2^19 rows (more
  // blocks in flight on the smaller systems; measured on the 2D and 3D
  // workloads), at most kGsBlocks
  const int64_t per = c.N < (int64_t(1) << 19) ? 2 : 4;
  c.gs_blocks = int(std::min<int64_t>(kGsBlocks, std::max<int64_t>(64, (c.N + per * kBlock - 1) / (per * kBlock))));
  c.part.alloc(sizeof(double) * size_t(kGsBlocks) * (m + 2));
  c.dh.alloc(sizeof(double) * 2 * size_t(3 * (m + 2)));
  c.dy.alloc(sizeof(double) * size_t(m + 1));
  c.flag.alloc(sizeof(int));
  if (!c.hpin) HIP_TRY(hipHostMalloc((void**)&c.hpin, sizeof(double) * 2 * 3 * (kMaxBasis + 2)));
  for (auto& e : c.ev)
    if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  for (auto& r : c.tev)
    for (auto& e : r)
      if (!e) HIP_TRY(hipEventCreate(&e));
  for (auto& e : c.tsolve)
    if (!e) HIP_TRY(hipEventCreate(&e));
  c.step_graph.assign(m, nullptr);
  c.pre_graph.assign(m, nullptr);
  c.gs_graph.assign(m, nullptr);
  c.m_alloc = m;
}

// One fused Gram-Schmidt pass and its reduction: out[first..nv] on the device.
void gs_pass(fsi_ctx& c, int mode, int nv, double* w, const double* h, double* out, hipStream_t s) {
  gs_pass_kernel<<<c.gs_blocks, kBlock, 0, s>>>(c.N, nv, c.V.as<double>(), c.N, w, h, mode, c.part.as<double>());
  const int first = mode == 2 ? nv : 0;
  gs_reduce_kernel<<<nv + 1 - first, kBlock, 0, s>>>(c.gs_blocks, first, c.part.as<double>(), out);
}

void givens(double a, double b, double& cs, double& sn) {
  if (b == 0.0) { cs = 1.0; sn = 0.0; return; }
  if (std::fabs(b) > std::fabs(a)) {
    const double t = a / b;
    sn = 1.0 / std::sqrt(1.0 + t * t);
    cs = sn * t;
  } else {
    const double t = b / a;
    cs = 1.0 / std::sqrt(1.0 + t * t);
    sn = cs * t;
  }
}

// FGMRES(m), right preconditioned, CGS2 Arnoldi.  The host-side Givens
// update of column j runs while the device already executes iteration j+1
// (its scalars travel in one asynchronous copy per iteration); when column j
// meets the stopping test the speculative iteration j+1 is simply discarded.
fsi_status solve_impl(fsi_ctx& c, const double* b, double* x, const fsi_solve_opts& o, fsi_solve_info& info) {
  hipStream_t s = c.stream;
  for (auto& M : c.mlp)
    for (DevBuf* b : {&M.fallbacks, &M.streak})
      if (b->p) HIP_TRY(hipMemsetAsync(b->p, 0, sizeof(int), s));
  const bool recording = c.mlp[0].rec.active || c.mlp[1].rec.active;
  const bool graphs = c.use_graphs && !recording;  // recording copies vectors from the host side
  const int64_t N = c.N;
  const int m = o.restart;
  ensure_krylov(c, m);
  double* V = c.V.as<double>();
  double* Z = c.Z.as<double>();
  double* dh = c.dh.as<double>();
  double* hp = c.hpin;
  const int slot = 3 * (m + 2);  // per iteration: h1 | h2 | h3
  hipEvent_t e0 = c.tsolve[0], e1 = c.tsolve[1];  // owned by the context: nothing leaks on a throw
  HIP_TRY(hipEventRecord(e0, s));
  auto fetch1 = [&](const double* src) {
    HIP_TRY(hipMemcpyAsync(hp, src, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return hp[0];
  };
  // ||b|| and finiteness of b and x0
  HIP_TRY(hipMemsetAsync(c.flag.p, 0, sizeof(int), s));
  nonfinite_kernel<<<grid_for(N, kBlock * 4), kBlock, 0, s>>>(N, b, c.flag.as<int>());
  nonfinite_kernel<<<grid_for(N, kBlock * 4), kBlock, 0, s>>>(N, x, c.flag.as<int>());
  gs_pass(c, 0, 0, const_cast<double*>(b), nullptr, dh, s);
  int flag = 0;
  HIP_TRY(hipMemcpyAsync(&flag, c.flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
  const double bnorm = std::sqrt(fetch1(dh));
  if (flag) throw Error(FSI_ERR_NUMERIC, "b or the initial guess holds NaN or Inf");
  info = fsi_solve_info{};
  if (bnorm == 0.0) {
    HIP_TRY(hipMemsetAsync(x, 0, sizeof(double) * N, s));
    HIP_TRY(hipStreamSynchronize(s));
    info.converged = 1;
    info.true_rel_resid = 0.0;
    return FSI_OK;
  }
  const double ah_bytes = c.Ah.bytes() + 16.0 * double(N);  // A_h, x read once, y written
  const double pc_bytes = precond_bytes(c);
  double bytes_spmv = 0.0, bytes_precond = 0.0, bytes_gs = 8.0 * double(N);  // ||b||
  std::vector<double> H(size_t(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), rhist(m + 2);
  auto Hat = [&](int i, int j) -> double& { return H[size_t(i) * m + j]; };
  int iters = 0, restarts = 0;
  bool converged = false;
  double rel = 0.0;
  // device work of Arnoldi step j (scalars of column j into slot j % 2)
  const bool timing = o.timing != 0;
  double t_pre = 0.0, t_spmv = 0.0, t_gs = 0.0;
  int n_timed = 0;
  auto record_pre = [&](int j, hipStream_t st) {
    apply_precond(c, V + size_t(j) * N, Z + size_t(j) * N, st);
  };
  auto record_spmv = [&](int j, hipStream_t st) {
    spmv<double>(c.Ah, Z + size_t(j) * N, V + size_t(j + 1) * N, st);
  };
  auto record_gs = [&](int j, hipStream_t st) {
    double* w = V + size_t(j + 1) * N;
    double* h1 = dh + (j % 2) * slot;
    double* h2 = h1 + (m + 2);
    double* h3 = h2 + (m + 2);
    gs_pass(c, 0, j + 1, w, nullptr, h1, st);  // h1 = V^T w, |w|^2 before
    gs_pass(c, 1, j + 1, w, h1, h2, st);       // w -= V h1; h2 = V^T w
    gs_pass(c, 2, j + 1, w, h2, h3, st);       // w -= V h2; |w|^2 after
    gs_normalise_kernel<<<grid_for(N, kBlock * 4), kBlock, 0, st>>>(N, w, h3 + (j + 1), h1 + (j + 1));
    HIP_TRY(hipMemcpyAsync(hp + (j % 2) * slot, h1, sizeof(double) * slot, hipMemcpyDeviceToHost, st));
  };
  // capture `rec` into an executable graph (private capture stream)
  auto capture = [&](hipGraphExec_t& ex, auto&& rec) {
    if (ex) return;
    if (!c.cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c.cap_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(c.cap_stream, hipStreamCaptureModeThreadLocal));
    try {
      rec(c.cap_stream);
    } catch (...) {
      (void)hipStreamEndCapture(c.cap_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    HIP_TRY(hipStreamEndCapture(c.cap_stream, &g));
    hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIP_TRY(e);
  };
  // timed mode: the phases are separated by events recorded between launches
  // (events inside a captured graph carry no timestamps), the A_h product is
  // launched on its own between the two graphs of the step
  auto launch_step = [&](int j) {
    hipEvent_t* te = c.tev[j % 2];
    bytes_precond += pc_bytes;
    bytes_spmv += ah_bytes;
    bytes_gs += 8.0 * double(N) * (3.0 * j + 10.0);  // three passes over j+1 vectors, normalisation
    if (graphs && !timing) {
      capture(c.step_graph[j], [&](hipStream_t st) {
        record_pre(j, st);
        record_spmv(j, st);
        record_gs(j, st);
      });
      HIP_TRY(hipGraphLaunch(c.step_graph[j], s));
    } else if (graphs) {
      capture(c.pre_graph[j], [&](hipStream_t st) { record_pre(j, st); });
      capture(c.gs_graph[j], [&](hipStream_t st) { record_gs(j, st); });
      HIP_TRY(hipEventRecord(te[0], s));
      HIP_TRY(hipGraphLaunch(c.pre_graph[j], s));
      HIP_TRY(hipEventRecord(te[1], s));
      record_spmv(j, s);
      HIP_TRY(hipEventRecord(te[2], s));
      HIP_TRY(hipGraphLaunch(c.gs_graph[j], s));
      HIP_TRY(hipEventRecord(te[3], s));
    } else {
      if (timing) HIP_TRY(hipEventRecord(te[0], s));
      record_pre(j, s);
      if (timing) HIP_TRY(hipEventRecord(te[1], s));
      record_spmv(j, s);
      if (timing) HIP_TRY(hipEventRecord(te[2], s));
      record_gs(j, s);
      if (timing) HIP_TRY(hipEventRecord(te[3], s));
    }
    HIP_TRY(hipEventRecord(c.ev[j % 2], s));
  };
  // host part of step j: Hessenberg column, Givens rotations; true = stop
  auto finish_step = [&](int j) -> bool {
    HIP_TRY(hipEventSynchronize(c.ev[j % 2]));
    if (timing) {
      float a = 0.f, b2 = 0.f, c3 = 0.f;
      hipEvent_t* te = c.tev[j % 2];
      HIP_TRY(hipEventElapsedTime(&a, te[0], te[1]));
      HIP_TRY(hipEventElapsedTime(&b2, te[1], te[2]));
      HIP_TRY(hipEventElapsedTime(&c3, te[2], te[3]));
      t_pre += a;
      t_spmv += b2;
      t_gs += c3;
      ++n_timed;
    }
    const double* q1 = hp + (j % 2) * slot;
    const double* q2 = q1 + (m + 2);
    const double* q3 = q2 + (m + 2);
    const double wbefore = std::sqrt(q1[j + 1]);
    for (int i = 0; i <= j; ++i) Hat(i, j) = q1[i] + q2[i];
    const double hn = std::sqrt(q3[j + 1] > 0.0 ? q3[j + 1] : 0.0);
    Hat(j + 1, j) = hn;
    const bool breakdown = !(hn > 1e-14 * wbefore);
    for (int i = 0; i < j; ++i) {
      const double a = Hat(i, j), bb = Hat(i + 1, j);
      Hat(i, j) = cs[i] * a + sn[i] * bb;
      Hat(i + 1, j) = -sn[i] * a + cs[i] * bb;
    }
    givens(Hat(j, j), Hat(j + 1, j), cs[j], sn[j]);
    Hat(j, j) = cs[j] * Hat(j, j) + sn[j] * Hat(j + 1, j);
    Hat(j + 1, j) = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    rhist[j + 1] = std::fabs(g[j + 1]);  // residual estimate after step j
    ++iters;
    if (!std::isfinite(g[j + 1])) throw Error(FSI_ERR_NUMERIC, "non-finite Arnoldi coefficients");
    return std::fabs(g[j + 1]) / bnorm <= o.tol || breakdown || iters >= o.maxit;
  };
  while (true) {
    // true residual r = b - A x into V_0
    spmv_sub<double>(c.Ah, x, b, V, s);
    gs_pass(c, 0, 0, V, nullptr, dh, s);
    bytes_spmv += ah_bytes + 8.0 * double(N);  // b read as well
    bytes_gs += 8.0 * double(N);
    const double beta = std::sqrt(fetch1(dh));
    rel = beta / bnorm;
    if (!std::isfinite(rel)) throw Error(FSI_ERR_NUMERIC, "non-finite residual");
    if (rel <= o.tol) { converged = true; break; }
    if (iters >= o.maxit) break;
    scale_kernel<<<grid_for(N, kBlock * 4), kBlock, 0, s>>>(N, V, 1.0 / beta);  // V_0 = r / beta
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    rhist.assign(m + 2, 0.0);
    rhist[0] = beta;
    int k = 0;
    launch_step(0);
    int launched = 0;
    for (int j = 0; j < m; ++j) {
      if (launched < j) {  // not launched ahead: the previous step was expected to converge
        launch_step(j);
        launched = j;
      }
      const bool more = j + 1 < m && iters + 1 < o.maxit;
      // Step j+1 is launched ahead (it overlaps the host work of step j)
      // unless the residual estimate, extrapolated by its last reduction
      // factor, already meets the tolerance after step j: then the
      // speculative step would most likely be thrown away.
      bool ahead = more;
      if (ahead && j >= 2) {
        const double r1 = rhist[j], r0 = rhist[j - 1];  // estimates after steps j-1, j-2
        ahead = !(r0 > 0.0 && r1 * (r1 / r0) <= o.tol * bnorm);
      }
      if (ahead) {
        launch_step(j + 1);
        launched = j + 1;
      }
      const bool stop = finish_step(j);
      k = j + 1;
      if (stop || !more) break;
    }
    for (int i = k - 1; i >= 0; --i) {
      double sum = g[i];
      for (int l = i + 1; l < k; ++l) sum -= Hat(i, l) * y[l];
      if (Hat(i, i) == 0.0) throw Error(FSI_ERR_NUMERIC, "singular Hessenberg matrix");
      y[i] = sum / Hat(i, i);
    }
    HIP_TRY(hipMemcpyAsync(c.dy.p, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
    multi_axpy_kernel<<<grid_for(N, kBlock * 4), kBlock, 0, s>>>(N, k, Z, N, c.dy.as<double>(), x);
    bytes_gs += 8.0 * double(N) * (k + 2);
    HIP_TRY(hipStreamSynchronize(s));  // y lives in host memory
    ++restarts;
  }
  // per-block norms of the final true residual (V_0 holds b - A_h x)
  {
    constexpr int nb = 64;
    double* part = c.part.as<double>();  // at least kGsBlocks * (m + 2) >= 3 * nb doubles
    sumsq3_kernel<<<3 * nb, kBlock, 0, s>>>(V, 0, c.n_m, c.n_m + c.n_s, N, nb, part);
    std::vector<double> hpart(3 * nb);
    HIP_TRY(hipMemcpyAsync(hpart.data(), part, sizeof(double) * 3 * nb, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int q = 0; q < 3; ++q) {
      double ss = 0.0;
      for (int i = 0; i < nb; ++i) ss += hpart[q * nb + i];
      info.resid_block[q] = std::sqrt(ss) / bnorm;
    }
    bytes_gs += 8.0 * double(N);
  }
  HIP_TRY(hipEventRecord(e1, s));
  HIP_TRY(hipEventSynchronize(e1));
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  info.iters = iters;
  info.mlp_fallbacks = 0;
  for (auto& M : c.mlp)
    if (M.fallbacks.p) {
      int fb = 0;
      HIP_TRY(hipMemcpy(&fb, M.fallbacks.p, sizeof(int), hipMemcpyDeviceToHost));
      info.mlp_fallbacks += fb;
    }
  info.t_precond_ms = t_pre;
  info.t_spmv_ms = t_spmv;
  info.t_gs_ms = t_gs;
  info.n_timed = n_timed;
  info.restarts = restarts;
  info.converged = converged ? 1 : 0;
  info.true_rel_resid = rel;
  info.t_total_ms = ms;
  info.bytes_spmv = bytes_spmv;
  info.bytes_precond = bytes_precond;
  info.bytes_gs = bytes_gs;
  log_line("solve: %d iterations, %d restarts, true rel. residual %.3e (mesh %.2e, solid %.2e, fluid %.2e), %.3f ms, "
       "%.2f GB moved (A_h %.2f, P^-1 %.2f, Krylov %.2f)",
       iters, restarts, rel, info.resid_block[0], info.resid_block[1], info.resid_block[2], ms,
       (bytes_spmv + bytes_precond + bytes_gs) / 1e9, bytes_spmv / 1e9, bytes_precond / 1e9, bytes_gs / 1e9);
  return converged ? FSI_OK : FSI_NOT_CONVERGED;
}

// ------------------------------------------------------- learned smoother
uint16_t host_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return uint16_t((u >> 16) | 0x40u);
  return uint16_t((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// Stencil tables of the finest levels of H_M (nodes = rows of L) and H_SIG
// (nodes = solid velocity nodes): for every node the operator index of its 3^d
// lattice neighbours (lexicographic offsets in {-1,0,1}^d), -1 where absent.
void prepare_mlp(fsi_ctx& c) {
  for (int i = 0; i < 2; ++i) {
    MlpState& M = c.mlp[i];
    const int h = i == 0 ? FSI_H_M : FSI_H_SIG;
    const SaHierarchy& HH = c.host_h[h];
    const int d = c.d;
    if (!learned_capable(c, h) || HH.levels.size() < 2) {
      M.n_nodes = 0;
      M.use.n_nodes = 0;
      M.use.enabled = false;
      continue;
    }
    const int64_t n_nodes = i == 0 ? c.n_m / d : c.n_vs / d;
    if (M.d != d) {
      M.have_weights = false;
      M.adam_t = 0;
      M.use.enabled = false;
    }
    if (M.n_nodes != n_nodes || M.d != d) M.rec.vecs.clear();
    M.d = d;
    M.n_nodes = n_nodes;
    const int S = d == 2 ? 9 : 27;
    const int64_t total = int64_t(c.node_ijk.size()) / d;
    std::vector<int32_t> gnode(n_nodes), opnode(total, -1);
    for (int64_t k = 0; k < n_nodes; ++k) {
      gnode[k] = c.dof_node[(i == 0 ? 0 : c.n_m) + k * d];
      opnode[gnode[k]] = int32_t(k);
    }
    int64_t ext[3] = {1, 1, 1};
    for (int64_t g = 0; g < total; ++g)
      for (int a = 0; a < d; ++a) ext[a] = std::max<int64_t>(ext[a], c.node_ijk[g * d + a] + 1);
    std::vector<int32_t> lat(size_t(ext[0] * ext[1] * ext[2]), -1);
    auto lidx = [&](const int* I) { return (int64_t(I[0]) * ext[1] + I[1]) * ext[2] + (d == 3 ? I[2] : 0); };
    for (int64_t g = 0; g < total; ++g) {
      int I[3] = {0, 0, 0};
      for (int a = 0; a < d; ++a) I[a] = c.node_ijk[g * d + a];
      lat[lidx(I)] = int32_t(g);
    }
    std::vector<int32_t> nbr(size_t(n_nodes) * S, -1);
    for (int64_t k = 0; k < n_nodes; ++k) {
      for (int sidx = 0; sidx < S; ++sidx) {
        int off[3] = {0, 0, 0}, r = sidx;
        for (int a = d - 1; a >= 0; --a) { off[a] = r % 3 - 1; r /= 3; }
        int I[3] = {0, 0, 0};
        bool inside = true;
        for (int a = 0; a < d; ++a) {
          I[a] = c.node_ijk[int64_t(gnode[k]) * d + a] + off[a];
          inside = inside && I[a] >= 0 && I[a] < ext[a];
        }
        if (!inside) continue;
        const int32_t g2 = lat[lidx(I)];
        if (g2 >= 0) nbr[k * S + sidx] = opnode[g2];
      }
    }
    // loss weights: the node's mean diagonal entry relative to the mean
    const std::vector<double>& dv = HH.levels[0].dinv;
    M.wnode.assign(n_nodes, 0.f);
    double mean = 0.0;
    std::vector<double> dn(n_nodes);
    for (int64_t k = 0; k < n_nodes; ++k) {
      double a = 0.0;
      if (i == 0) a = 1.0 / dv[k];
      else {
        for (int q = 0; q < d; ++q) a += 1.0 / dv[k * d + q];
        a /= d;
      }
      dn[k] = a;
      mean += a;
    }
    mean /= double(n_nodes);
    for (int64_t k = 0; k < n_nodes; ++k) M.wnode[k] = float(dn[k] / mean);
    M.nbr.alloc(sizeof(int32_t) * nbr.size());
    HIP_TRY(hipMemcpyAsync(M.nbr.p, nbr.data(), sizeof(int32_t) * nbr.size(), hipMemcpyHostToDevice, c.stream));
    if (!M.npart.p) M.npart.alloc(sizeof(double) * 2 * kDecideBlocks);
    if (!M.flag.p) M.flag.alloc(sizeof(int));
    if (!M.fallbacks.p) {
      M.fallbacks.alloc(sizeof(int));
      HIP_TRY(hipMemsetAsync(M.fallbacks.p, 0, sizeof(int), c.stream));
    }
    if (!M.streak.p) {
      M.streak.alloc(sizeof(int));
      HIP_TRY(hipMemsetAsync(M.streak.p, 0, sizeof(int), c.stream));
    }
    const size_t np = size_t(M.nparam());
    if (M.wm.bytes != sizeof(float) * np) {
      for (DevBuf* b : {&M.wm, &M.m1, &M.m2, &M.g}) {
        b->alloc(sizeof(float) * np);
        HIP_TRY(hipMemsetAsync(b->p, 0, sizeof(float) * np, c.stream));
      }
      M.loss.alloc(sizeof(float));
      const int kp = M.kp();
      M.w1t.alloc(2 * 64 * kp);
      M.w2t.alloc(2 * 64 * 64);
      M.w2.alloc(2 * 64 * 64);
      M.w3t.alloc(2 * 16 * 64);
      M.w3.alloc(2 * 64 * 16);
      for (DevBuf* b : {&M.w1t, &M.w2t, &M.w2, &M.w3t, &M.w3}) HIP_TRY(hipMemsetAsync(b->p, 0, b->bytes, c.stream));
      M.have_weights = false;
      M.use.enabled = false;
    }
    M.use.d = d;
    M.use.per_dof = i == 1;
    M.use.n_nodes = n_nodes;
    M.use.nbr = M.nbr.as<int32_t>();
    M.use.w = MlpW{M.w1t.as<unsigned short>(), M.w2t.as<unsigned short>(), M.w2.as<unsigned short>(),
                   M.w3t.as<unsigned short>(), M.w3.as<unsigned short>()};
    M.use.npart = M.npart.as<double>();
    M.use.flag = M.flag.as<int>();
    M.use.fallbacks = M.fallbacks.as<int>();
    M.use.streak = M.streak.as<int>();
  }
  HIP_TRY(hipStreamSynchronize(c.stream));
}

MlpState& mlp_state(fsi_ctx& c, int which) {
  if (which != FSI_H_M && which != FSI_H_SIG) throw Error(FSI_ERR_ARG, "which must be FSI_H_M or FSI_H_SIG");
  if (!c.have_precond) throw Error(FSI_ERR_STATE, "fsi_build_precond must come first");
  MlpState& M = c.mlp[which == FSI_H_M ? 0 : 1];
  if (M.n_nodes == 0)
    throw Error(FSI_ERR_STATE,
                "no learned smoother here: needs layout.node_ijk, Jacobi sweeps, at least two AMG levels and FP64 or "
                "FP32 diagonals");
  return M;
}

// Master FP32 weights (padded layouts [k][hid], [in][out], [hid][16]) from
// natural FP32 W1 (K x 64), W2 (64 x 64), W3 (64 x d), and their BF16 copies.
void mlp_upload_weights(fsi_ctx& c, MlpState& M, const float* W1, const float* W2, const float* W3) {
  const int kp = M.kp(), kin = M.kin(), d = M.d, H = 64, NP = 16;
  std::vector<float> wm(size_t(M.nparam()), 0.f);
  std::vector<uint16_t> w1t(size_t(H) * kp, 0), w2t(H * H, 0), w2(H * H, 0), w3t(NP * H, 0), w3(H * NP, 0);
  for (int k = 0; k < kin; ++k)
    for (int h = 0; h < H; ++h) {
      wm[size_t(k) * H + h] = W1[k * H + h];
      w1t[size_t(h) * kp + k] = host_bf16(W1[k * H + h]);
    }
  float* m2 = wm.data() + size_t(kp) * H;
  for (int a = 0; a < H; ++a)
    for (int b = 0; b < H; ++b) {
      m2[a * H + b] = W2[a * H + b];
      w2[a * H + b] = host_bf16(W2[a * H + b]);
      w2t[b * H + a] = host_bf16(W2[a * H + b]);
    }
  float* m3 = m2 + H * H;
  for (int h = 0; h < H; ++h)
    for (int q = 0; q < d; ++q) {
      m3[h * NP + q] = W3[h * d + q];
      w3[h * NP + q] = host_bf16(W3[h * d + q]);
      w3t[q * H + h] = host_bf16(W3[h * d + q]);
    }
  hipStream_t s = c.stream;
  HIP_TRY(hipMemcpyAsync(M.wm.p, wm.data(), sizeof(float) * wm.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemsetAsync(M.m1.p, 0, M.m1.bytes, s));
  HIP_TRY(hipMemsetAsync(M.m2.p, 0, M.m2.bytes, s));
  HIP_TRY(hipMemcpyAsync(M.w1t.p, w1t.data(), 2 * w1t.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(M.w2t.p, w2t.data(), 2 * w2t.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(M.w2.p, w2.data(), 2 * w2.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(M.w3t.p, w3t.data(), 2 * w3t.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(M.w3.p, w3.data(), 2 * w3.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  M.adam_t = 0;
  M.have_weights = true;
}

// One gradient pass over m samples already on the device (Z [m][KP] BF16,
// E [m][d], W [m]) starting at `first`: gradient into M.g, loss sum into M.loss.
void mlp_grad_pass(fsi_ctx& c, MlpState& M, const unsigned short* Z, const float* E, const float* W, int64_t first,
                   int64_t m, float coef, bool given = false) {
  hipStream_t s = c.stream;
  const int64_t tiles = (m + 15) / 16;
  const int tpw = int(std::max<int64_t>(4, (tiles + 1023) / 1024));  // at most ~1024 partial gradients
  const int64_t waves = (tiles + tpw - 1) / tpw;
  const int64_t blocks = (waves + 3) / 4;
  const int64_t nwv = blocks * 4;
  const size_t need = sizeof(float) * size_t(nwv) * M.nparam();
  if (M.part.bytes < need) M.part.alloc(need);
  if (M.part_loss.bytes < sizeof(float) * nwv) M.part_loss.alloc(sizeof(float) * nwv);
  const MlpW& w = M.use.w;
  float* part = M.part.as<float>();
  float* pl = M.part_loss.as<float>();
  const unsigned nb = unsigned(blocks);
  if (M.d == 2) {
    if (given) mlp_train_kernel<2, true><<<nb, 256, 0, s>>>(first, m, tpw, Z, E, W, coef, w, part, pl);
    else mlp_train_kernel<2, false><<<nb, 256, 0, s>>>(first, m, tpw, Z, E, W, coef, w, part, pl);
  } else {
    if (given) mlp_train_kernel<3, true><<<nb, 256, 0, s>>>(first, m, tpw, Z, E, W, coef, w, part, pl);
    else mlp_train_kernel<3, false><<<nb, 256, 0, s>>>(first, m, tpw, Z, E, W, coef, w, part, pl);
  }
  if (M.part2.bytes < sizeof(float) * size_t(kGradChunks) * M.nparam()) {
    M.part2.alloc(sizeof(float) * size_t(kGradChunks) * M.nparam());
    M.loss2.alloc(sizeof(float) * kGradChunks);
  }
  const unsigned pb = unsigned((M.nparam() + 255) / 256);
  mlp_grad_chunk_kernel<<<dim3(pb, kGradChunks), 256, 0, s>>>(int(nwv), M.nparam(), part, pl, M.part2.as<float>(),
                                                               M.loss2.as<float>());
  mlp_grad_reduce_kernel<<<pb, 256, 0, s>>>(M.nparam(), M.part2.as<float>(), M.loss2.as<float>(), M.g.as<float>(),
                                            M.loss.as<float>());
}

void mlp_adam(fsi_ctx& c, MlpState& M, float lr) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  ++M.adam_t;
  const float bc1 = 1.f - std::pow(b1, float(M.adam_t)), bc2 = 1.f - std::pow(b2, float(M.adam_t));
  const unsigned grid = unsigned((M.nparam() + 255) / 256);
  auto u16 = [](DevBuf& b) { return b.as<unsigned short>(); };
  if (M.d == 2)
    mlp_adam_kernel<2><<<grid, 256, 0, c.stream>>>(M.wm.as<float>(), M.m1.as<float>(), M.m2.as<float>(),
                                                   M.g.as<float>(), lr, b1, b2, eps, bc1, bc2, u16(M.w1t),
                                                   u16(M.w2t), u16(M.w2), u16(M.w3t), u16(M.w3));
  else
    mlp_adam_kernel<3><<<grid, 256, 0, c.stream>>>(M.wm.as<float>(), M.m1.as<float>(), M.m2.as<float>(),
                                                   M.g.as<float>(), lr, b1, b2, eps, bc1, bc2, u16(M.w1t),
                                                   u16(M.w2t), u16(M.w2), u16(M.w3t), u16(M.w3));
}

// Exact correction e = A0^{-1} b of a recorded residual by iterating plain
// V-cycles (e += V(b - A0 e)) to a relative residual tol; false if it does
// not get there within maxit cycles.
template <typename T, int NV>
bool exact_correction(fsi_ctx& c, DHier<T>& H, const double* b, double* e, double tol, int maxit) {
  hipStream_t s = c.stream;
  DLevel<T>& d0 = H.lev[0];
  const int64_t n = d0.n * NV;
  DevBuf bt, et, rt, ct, np;
  bt.alloc(sizeof(T) * n);
  et.alloc(sizeof(T) * n);
  rt.alloc(sizeof(T) * n);
  ct.alloc(sizeof(T) * n);
  np.alloc(sizeof(double) * 2 * kNormBlocks);
  const unsigned g = grid_for(n, kBlock * 4);
  cast_kernel<double, T><<<g, kBlock, 0, s>>>(n, b, bt.as<T>());
  HIP_TRY(hipMemsetAsync(et.p, 0, sizeof(T) * n, s));
  HIP_TRY(hipMemcpyAsync(rt.p, bt.p, sizeof(T) * n, hipMemcpyDeviceToDevice, s));
  std::vector<double> hpart(2 * kNormBlocks);
  bool ok = false;
  for (int it = 1; it <= maxit; ++it) {
    vcycle_rec<T, NV>(H, 0, rt.as<T>(), ct.as<T>(), s, true);
    vadd_kernel<T><<<g, kBlock, 0, s>>>(n, et.as<T>(), ct.as<T>());  // e += V(r)
    launch_rows<T, NV>(d0.A0, GatherPlain<T, NV>{et.as<T>()}, EpiSub<T, NV>{bt.as<T>(), rt.as<T>()}, s);
    if (it % 5 == 0 || it == maxit) {
      norm_pair_partial_kernel<T><<<kNormBlocks, 256, 0, s>>>(n, rt.as<T>(), bt.as<T>(), np.as<double>());
      HIP_TRY(hipMemcpyAsync(hpart.data(), np.p, sizeof(double) * hpart.size(), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      double rr = 0.0, bb = 0.0;
      for (int k = 0; k < kNormBlocks; ++k) {
        rr += hpart[2 * k];
        bb += hpart[2 * k + 1];
      }
      if (!(rr <= 1e6 * bb)) break;  // diverging or NaN
      if (std::sqrt(rr) <= tol * std::sqrt(bb)) {
        ok = true;
        break;
      }
    }
  }
  cast_kernel<T, double><<<g, kBlock, 0, s>>>(n, et.as<T>(), e);
  HIP_TRY(hipStreamSynchronize(s));
  return ok;
}

template <typename T>
void mlp_samples(const MlpState& M, const T* b, const T* dinv, const double* e, const float* wn, float scale,
                 unsigned short* Z, float* E, float* W, hipStream_t s) {
  const unsigned g = grid_for(M.n_nodes, 256);
  const int32_t* nbr = M.nbr.as<int32_t>();
  if (M.d == 2) {
    if (M.use.per_dof) mlp_samples_kernel<2, true, T><<<g, 256, 0, s>>>(M.n_nodes, nbr, b, dinv, e, wn, scale, Z, E, W);
    else mlp_samples_kernel<2, false, T><<<g, 256, 0, s>>>(M.n_nodes, nbr, b, dinv, e, wn, scale, Z, E, W);
  } else {
    if (M.use.per_dof) mlp_samples_kernel<3, true, T><<<g, 256, 0, s>>>(M.n_nodes, nbr, b, dinv, e, wn, scale, Z, E, W);
    else mlp_samples_kernel<3, false, T><<<g, 256, 0, s>>>(M.n_nodes, nbr, b, dinv, e, wn, scale, Z, E, W);
  }
}

// Train the learned smoothers on the recorded finest-level residuals with
// the squared-error loss against exact corrections (FSI_MLP_LOSS_L2).
template <typename T>
void mlp_train_l2(fsi_ctx& c, Precond<T>& P, const fsi_mlp_train_opts& o, fsi_mlp_train_info& info) {
  hipStream_t s = c.stream;
  for (int i = 0; i < 2; ++i) {
    MlpState& M = c.mlp[i];
    info.vectors[i] = 0;
    info.samples[i] = 0;
    info.loss_first[i] = info.loss_last[i] = 0.0;
    if (M.n_nodes == 0 || !M.have_weights || M.rec.vecs.empty()) continue;
    const int h = i == 0 ? FSI_H_M : FSI_H_SIG;
    DHier<T>& H = P.H[h];
    if (!H.xm) continue;
    const int d = M.d, kp = M.kp();
    const int64_t n_dof = M.n_nodes * d;
    const int64_t maxm = int64_t(M.rec.vecs.size()) * M.n_nodes;
    DevBuf Z, E, W, Z2, E2, W2, e, wn, bt, perm;
    Z.alloc(2 * size_t(maxm) * kp);
    E.alloc(4 * size_t(maxm) * d);
    W.alloc(4 * size_t(maxm));
    e.alloc(8 * size_t(n_dof));
    bt.alloc(sizeof(T) * size_t(n_dof));
    wn.alloc(4 * size_t(M.n_nodes));
    HIP_TRY(hipMemcpyAsync(wn.p, M.wnode.data(), 4 * M.wnode.size(), hipMemcpyHostToDevice, s));
    const std::vector<double>& dv = c.host_h[h].levels[0].dinv;
    const T* dinv = H.lev[0].dinv->template as<T>();
    std::vector<double> hb(n_dof);
    int64_t m = 0;
    for (auto& v : M.rec.vecs) {
      HIP_TRY(hipMemcpyAsync(hb.data(), v->p, 8 * size_t(n_dof), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      double ss = 0.0;
      for (int64_t k = 0; k < n_dof; ++k) {
        const double z = (i == 0 ? dv[k / d] : dv[k]) * hb[k];
        ss += z * z;
      }
      const double rms = std::sqrt(ss / double(n_dof));
      if (!(rms > 0.0) || !std::isfinite(rms)) continue;
      bool ok;
      if (H.nv == 1) ok = exact_correction<T, 1>(c, H, v->as<double>(), e.as<double>(), o.exact_tol, o.exact_maxit);
      else if (H.nv == 2) ok = exact_correction<T, 2>(c, H, v->as<double>(), e.as<double>(), o.exact_tol, o.exact_maxit);
      else ok = exact_correction<T, 3>(c, H, v->as<double>(), e.as<double>(), o.exact_tol, o.exact_maxit);
      if (!ok) continue;
      cast_kernel<double, T><<<grid_for(n_dof, kBlock * 4), kBlock, 0, s>>>(n_dof, v->as<double>(), bt.as<T>());
      mlp_samples<T>(M, bt.as<T>(), dinv, e.as<double>(), wn.as<float>(), float(1.0 / rms),
                     Z.as<unsigned short>() + size_t(m) * kp, E.as<float>() + size_t(m) * d, W.as<float>() + m, s);
      m += M.n_nodes;
      ++info.vectors[i];
    }
    info.samples[i] = m;
    if (m == 0) continue;
    // seeded shuffle of the node samples
    std::vector<int64_t> pm(m);
    for (int64_t k = 0; k < m; ++k) pm[k] = k;
    std::mt19937_64 rng(uint64_t(o.seed) * 2 + uint64_t(i));
    for (int64_t k = m - 1; k > 0; --k) std::swap(pm[k], pm[int64_t(rng() % uint64_t(k + 1))]);
    perm.alloc(8 * size_t(m));
    Z2.alloc(2 * size_t(m) * kp);
    E2.alloc(4 * size_t(m) * d);
    W2.alloc(4 * size_t(m));
    HIP_TRY(hipMemcpyAsync(perm.p, pm.data(), 8 * size_t(m), hipMemcpyHostToDevice, s));
    if (d == 2)
      mlp_gather_samples_kernel<MlpDims<2>::KP, 2><<<grid_for(m, 256), 256, 0, s>>>(
          m, perm.as<int64_t>(), Z.as<unsigned short>(), E.as<float>(), W.as<float>(), Z2.as<unsigned short>(),
          E2.as<float>(), W2.as<float>());
    else
      mlp_gather_samples_kernel<MlpDims<3>::KP, 3><<<grid_for(m, 256), 256, 0, s>>>(
          m, perm.as<int64_t>(), Z.as<unsigned short>(), E.as<float>(), W.as<float>(), Z2.as<unsigned short>(),
          E2.as<float>(), W2.as<float>());
    const int64_t batch = std::min<int64_t>(o.batch, m);
    float lossv = 0.f;
    for (int step = 0; step < o.steps; ++step) {
      const int64_t first = (int64_t(step) * batch) % m;
      const int64_t mb = std::min<int64_t>(batch, m - first);
      mlp_grad_pass(c, M, Z2.as<unsigned short>(), E2.as<float>(), W2.as<float>(), first, mb, float(2.0 / double(mb)));
      if (step == 0) {
        HIP_TRY(hipMemcpyAsync(&lossv, M.loss.p, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        info.loss_first[i] = double(lossv) / double(mb);
      }
      mlp_adam(c, M, float(o.lr));
    }
    const int64_t mb = std::min<int64_t>(batch, m);
    mlp_grad_pass(c, M, Z2.as<unsigned short>(), E2.as<float>(), W2.as<float>(), 0, mb, float(2.0 / double(mb)));
    HIP_TRY(hipMemcpyAsync(&lossv, M.loss.p, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    info.loss_last[i] = double(lossv) / double(mb);
    M.use.enabled = true;
  }
  c.drop_graphs();
  c.m_alloc = -1;
}

// ------------------------------------------------ two-grid energy training
// For a residual b of level 0 (exact correction e = A^{-1} b) and the
// network's correction delta, the loss is the A-norm error that is left once
// an exact coarse-grid correction follows delta, minus a constant:
//     L = ||(I - P A_1^{-1} R A)(e - delta)||_A^2 - e.b .
// With r = b - A delta, rc = R r and c = A_1^{-1} rc this is
//     L = -delta.b - delta.r - rc.c,   dL/d delta = -2 (r - A P c)
// (A symmetric, R = P^T; no exact solve on level 0 is needed).  Minimising it
// asks the network for the error the coarse grid cannot represent, which is
// what a pre-smoother has to remove.
struct EnergyWork {
  DevBuf r, g, rc, cc, t, t2;
  template <typename T>
  void alloc(int64_t n, int64_t nc) {
    for (DevBuf* b : {&r, &g}) b->alloc(sizeof(T) * size_t(n));
    for (DevBuf* b : {&rc, &cc, &t, &t2}) b->alloc(sizeof(T) * size_t(nc));
  }
};

// cc = A_1^{-1} rc: the dense inverse when level 1 is the coarsest, otherwise
// `cycles` Richardson steps with plain V-cycles from level 1.
template <typename T, int NV>
void coarse_solve(DHier<T>& H, const T* rc, T* cc, T* t, T* t2, int cycles, hipStream_t s) {
  if (H.lev.size() == 2) {
    dense_gemv<T, T, NV>(H.nc, H.cinv->template as<double>(), rc, cc, s);
    return;
  }
  DLevel<T>& d1 = H.lev[1];
  const int64_t n = d1.n * NV;
  vcycle_rec<T, NV>(H, 1, rc, cc, s, true);
  for (int k = 1; k < cycles; ++k) {
    launch_rows<T, NV>(d1.A0, GatherPlain<T, NV>{cc}, EpiSub<T, NV>{rc, t}, s);
    vcycle_rec<T, NV>(H, 1, t, t2, s, true);
    vadd_kernel<T><<<grid_for(n, kBlock * 4), kBlock, 0, s>>>(n, cc, t2);
  }
}

// x.y of two device vectors, summed on the host in FP64 (loss reporting only).
template <typename T>
double host_dot(int64_t n, const T* pa, const T* pb, hipStream_t s) {
  std::vector<T> x(n), y(n);
  HIP_TRY(hipMemcpyAsync(x.data(), pa, sizeof(T) * n, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(y.data(), pb, sizeof(T) * n, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  double acc = 0.0;
  for (int64_t i = 0; i < n; ++i) acc += double(x[i]) * double(y[i]);
  return acc;
}

// dy = coef dL/d delta (FP32) for one residual b; *loss = L if requested.
template <typename T, int NV>
void energy_grad(DHier<T>& H, EnergyWork& w, const T* delta, const T* b, double coef, float* dy, int cycles,
                 hipStream_t s, double* loss) {
  DLevel<T>& d0 = H.lev[0];
  const int64_t n = d0.n * NV, nc = H.lev[1].n * NV;
  T* r = w.r.as<T>();
  T* g = w.g.as<T>();
  T* rc = w.rc.as<T>();
  T* cc = w.cc.as<T>();
  launch_rows<T, NV>(d0.A0, GatherPlain<T, NV>{delta}, EpiSub<T, NV>{b, r}, s);  // r = b - A delta
  launch_rows<T, NV>(d0.R0, GatherPlain<T, NV>{r}, EpiStore<T, NV>{rc}, s);      // rc = R r
  coarse_solve<T, NV>(H, rc, cc, w.t.as<T>(), w.t2.as<T>(), cycles, s);         // cc = A_1^{-1} rc
  launch_rows<T, NV>(d0.AP, GatherPlain<T, NV>{cc}, EpiSub<T, NV>{r, g}, s);     // g = r - A P cc
  cast_scale_kernel<T, float><<<grid_for(n, kBlock * 4), kBlock, 0, s>>>(n, g, -2.0 * coef, dy);
  if (loss) {
    const double db = host_dot<T>(n, delta, b, s);
    const double dr = host_dot<T>(n, delta, r, s);
    const double rcc = host_dot<T>(nc, rc, cc, s);
    *loss = -db - dr - rcc;
  }
}

// Network inputs (BF16 rows) of one level-0 vector b of learned smoother M.
template <typename T>
void mlp_inputs(const MlpState& M, const T* b, const T* dinv, unsigned short* Z, hipStream_t s) {
  const unsigned g = grid_for(M.n_nodes, 256);
  const int32_t* nbr = M.nbr.as<int32_t>();
  if (M.d == 2) {
    if (M.use.per_dof) mlp_inputs_kernel<2, true, T><<<g, 256, 0, s>>>(M.n_nodes, nbr, b, dinv, Z);
    else mlp_inputs_kernel<2, false, T><<<g, 256, 0, s>>>(M.n_nodes, nbr, b, dinv, Z);
  } else {
    if (M.use.per_dof) mlp_inputs_kernel<3, true, T><<<g, 256, 0, s>>>(M.n_nodes, nbr, b, dinv, Z);
    else mlp_inputs_kernel<3, false, T><<<g, 256, 0, s>>>(M.n_nodes, nbr, b, dinv, Z);
  }
}

template <typename T>
void mlp_forward_rows(const MlpState& M, int64_t m, const unsigned short* Z, T* y, hipStream_t s) {
  const unsigned g = grid_for(m, 64);
  if (M.d == 2) mlp_forward_rows_kernel<2, T><<<g, 256, 0, s>>>(m, Z, M.use.w, y);
  else mlp_forward_rows_kernel<3, T><<<g, 256, 0, s>>>(m, Z, M.use.w, y);
}

template <typename T, int NV>
void energy_fit(fsi_ctx& c, MlpState& M, DHier<T>& H, const std::vector<double>& dv, bool per_node,
                const fsi_mlp_train_opts& o, int which, fsi_mlp_train_info& info) {
  hipStream_t s = c.stream;
  const int kp = M.kp();
  const int64_t nn = M.n_nodes, n = H.lev[0].n * NV, nc = H.lev[1].n * NV;
  const T* dinv = H.lev[0].dinv->template as<T>();
  // recorded residuals in a seeded random order, scaled to ||b||_{D^{-1}} = 1
  std::vector<size_t> order(M.rec.vecs.size());
  for (size_t k = 0; k < order.size(); ++k) order[k] = k;
  std::mt19937_64 rng(uint64_t(o.seed) * 2 + uint64_t(which));
  for (size_t k = order.size(); k > 1; --k) std::swap(order[k - 1], order[size_t(rng() % k)]);
  std::vector<double> hb(n), scale;
  std::vector<size_t> keep;
  for (size_t k : order) {
    HIP_TRY(hipMemcpyAsync(hb.data(), M.rec.vecs[k]->p, 8 * size_t(n), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double ss = 0.0;
    for (int64_t q = 0; q < n; ++q) ss += hb[q] * hb[q] * (per_node ? dv[q / NV] : dv[q]);
    if (!(ss > 0.0) || !std::isfinite(ss)) continue;
    keep.push_back(k);
    scale.push_back(1.0 / std::sqrt(ss));
  }
  const int64_t nvec = int64_t(keep.size());
  info.vectors[which] = int32_t(nvec);
  info.samples[which] = nvec * nn;
  if (nvec == 0) return;
  DevBuf Bs, Z, Y, DY;
  Bs.alloc(sizeof(T) * size_t(n) * nvec);
  Z.alloc(2 * size_t(nn) * kp * nvec);
  for (int64_t j = 0; j < nvec; ++j) {
    T* bj = Bs.as<T>() + j * n;
    cast_scale_kernel<double, T><<<grid_for(n, kBlock * 4), kBlock, 0, s>>>(n, M.rec.vecs[keep[j]]->as<double>(),
                                                                          scale[j], bj);
    mlp_inputs<T>(M, bj, dinv, Z.as<unsigned short>() + size_t(j) * nn * kp, s);
  }
  const int64_t k = std::min<int64_t>(nvec, std::max<int64_t>(1, (int64_t(o.batch) + nn - 1) / nn));
  Y.alloc(sizeof(T) * size_t(n) * k);
  DY.alloc(4 * size_t(n) * k);
  EnergyWork w;
  w.alloc<T>(n, nc);
  const int cyc = std::max(1, o.coarse_cycles);
  auto eval = [&]() {
    double acc = 0.0;
    for (int64_t j0 = 0; j0 < nvec; j0 += k) {
      const int64_t kk = std::min<int64_t>(k, nvec - j0);
      mlp_forward_rows<T>(M, kk * nn, Z.as<unsigned short>() + size_t(j0) * nn * kp, Y.as<T>(), s);
      for (int64_t j = 0; j < kk; ++j) {
        double l = 0.0;
        energy_grad<T, NV>(H, w, Y.as<T>() + j * n, Bs.as<T>() + (j0 + j) * n, 1.0, DY.as<float>(), cyc, s, &l);
        acc += l;
      }
    }
    return acc / double(nvec);
  };
  info.loss_first[which] = eval();
  for (int step = 0; step < o.steps; ++step) {
    const int64_t j0 = (int64_t(step) * k) % nvec;
    const int64_t kk = std::min<int64_t>(k, nvec - j0);
    const unsigned short* Zb = Z.as<unsigned short>() + size_t(j0) * nn * kp;
    mlp_forward_rows<T>(M, kk * nn, Zb, Y.as<T>(), s);
    for (int64_t j = 0; j < kk; ++j)
      energy_grad<T, NV>(H, w, Y.as<T>() + j * n, Bs.as<T>() + (j0 + j) * n, 1.0 / double(kk),
                         DY.as<float>() + j * n, cyc, s, nullptr);
    mlp_grad_pass(c, M, Zb, DY.as<float>(), nullptr, 0, kk * nn, 1.f, true);
    mlp_adam(c, M, float(o.lr));
  }
  info.loss_last[which] = eval();
  M.use.enabled = true;
}

template <typename T>
void mlp_train_energy(fsi_ctx& c, Precond<T>& P, const fsi_mlp_train_opts& o, fsi_mlp_train_info& info) {
  for (int i = 0; i < 2; ++i) {
    MlpState& M = c.mlp[i];
    info.vectors[i] = 0;
    info.samples[i] = 0;
    info.loss_first[i] = info.loss_last[i] = 0.0;
    if (M.n_nodes == 0 || !M.have_weights || M.rec.vecs.empty()) continue;
    const int h = i == 0 ? FSI_H_M : FSI_H_SIG;
    DHier<T>& H = P.H[h];
    if (!H.xm || H.lev.size() < 2) continue;
    const std::vector<double>& dv = c.host_h[h].levels[0].dinv;
    const bool per_node = i == 0;
    if (H.nv == 1) energy_fit<T, 1>(c, M, H, dv, per_node, o, i, info);
    else if (H.nv == 2) energy_fit<T, 2>(c, M, H, dv, per_node, o, i, info);
    else energy_fit<T, 3>(c, M, H, dv, per_node, o, i, info);
  }
  c.drop_graphs();
  c.m_alloc = -1;
}

// Gradient of the energy loss for one level-0 residual b (device FP64),
// copied out in the natural weight layouts.
template <typename T, int NV>
double energy_grad_once(fsi_ctx& c, MlpState& M, DHier<T>& H, const double* b, int cycles) {
  hipStream_t s = c.stream;
  const int64_t nn = M.n_nodes, n = H.lev[0].n * NV, nc = H.lev[1].n * NV;
  DevBuf bt, Z, Y, DY;
  bt.alloc(sizeof(T) * size_t(n));
  Z.alloc(2 * size_t(nn) * M.kp());
  Y.alloc(sizeof(T) * size_t(n));
  DY.alloc(4 * size_t(n));
  cast_kernel<double, T><<<grid_for(n, kBlock * 4), kBlock, 0, s>>>(n, b, bt.as<T>());
  mlp_inputs<T>(M, bt.as<T>(), H.lev[0].dinv->template as<T>(), Z.as<unsigned short>(), s);
  mlp_forward_rows<T>(M, nn, Z.as<unsigned short>(), Y.as<T>(), s);
  EnergyWork w;
  w.alloc<T>(n, nc);
  double loss = 0.0;
  energy_grad<T, NV>(H, w, Y.as<T>(), bt.as<T>(), 1.0, DY.as<float>(), cycles, s, &loss);
  mlp_grad_pass(c, M, Z.as<unsigned short>(), DY.as<float>(), nullptr, 0, nn, 1.f, true);
  HIP_TRY(hipStreamSynchronize(s));
  return loss;
}

// Copy M.g (padded layouts) to natural W1 (K x 64), W2 (64 x 64), W3 (64 x d).
void unpack_grad(fsi_ctx& c, MlpState& M, float* G1, float* G2, float* G3) {
  const int kp = M.kp(), kin = M.kin(), d = M.d;
  std::vector<float> g(size_t(M.nparam()));
  HIP_TRY(hipMemcpyAsync(g.data(), M.g.p, 4 * g.size(), hipMemcpyDeviceToHost, c.stream));
  HIP_TRY(hipStreamSynchronize(c.stream));
  for (int k = 0; k < kin; ++k)
    for (int h = 0; h < 64; ++h) G1[k * 64 + h] = g[size_t(k) * 64 + h];
  const float* g2 = g.data() + size_t(kp) * 64;
  for (int a = 0; a < 64 * 64; ++a) G2[a] = g2[a];
  const float* g3 = g2 + 64 * 64;
  for (int h = 0; h < 64; ++h)
    for (int q = 0; q < d; ++q) G3[h * d + q] = g3[h * 16 + q];
}


// The five operators of Section 4 (the scalar mesh Laplacian, Sigma_s, the
// solid mass block, A_f and the pressure Schur approximation) and their SA
// hierarchies, on the host.  Replaces c.host_h only when all five succeed.
// Inverse of the node-block diagonal of A (the entries (i, j) with
// i / b == j / b), block by block: Gauss-Jordan with partial pivoting on each
// b x b block, stored as a CSR matrix of dense blocks.
HCsr node_block_inverse(const HCsr& A, int b) {
  const int64_t n = A.nrows;
  if (n % b != 0) throw Error(FSI_ERR_STRUCT, "block size does not divide the matrix");
  HCsr R;
  R.nrows = R.ncols = n;
  R.rp.assign(n + 1, 0);
  R.ci.resize(size_t(n) * b);
  R.v.resize(size_t(n) * b);
  std::vector<double> a(size_t(b) * b), inv(size_t(b) * b);
  for (int64_t k = 0; k < n / b; ++k) {
    std::fill(a.begin(), a.end(), 0.0);
    std::fill(inv.begin(), inv.end(), 0.0);
    for (int r = 0; r < b; ++r) {
      const int64_t i = k * b + r;
      for (int64_t q = A.rp[i]; q < A.rp[i + 1]; ++q)
        if (A.ci[q] / b == k) a[size_t(r) * b + (A.ci[q] - k * b)] = A.v[q];
      inv[size_t(r) * b + r] = 1.0;
    }
    for (int c = 0; c < b; ++c) {
      int p = c;
      for (int r = c + 1; r < b; ++r)
        if (std::fabs(a[size_t(r) * b + c]) > std::fabs(a[size_t(p) * b + c])) p = r;
      if (a[size_t(p) * b + c] == 0.0) throw Error(FSI_ERR_NUMERIC, "singular node block in the diagonal");
      for (int q = 0; q < b; ++q) {
        std::swap(a[size_t(c) * b + q], a[size_t(p) * b + q]);
        std::swap(inv[size_t(c) * b + q], inv[size_t(p) * b + q]);
      }
      const double piv = a[size_t(c) * b + c];
      for (int q = 0; q < b; ++q) {
        a[size_t(c) * b + q] /= piv;
        inv[size_t(c) * b + q] /= piv;
      }
      for (int r = 0; r < b; ++r) {
        if (r == c) continue;
        const double f = a[size_t(r) * b + c];
        if (f == 0.0) continue;
        for (int q = 0; q < b; ++q) {
          a[size_t(r) * b + q] -= f * a[size_t(c) * b + q];
          inv[size_t(r) * b + q] -= f * inv[size_t(c) * b + q];
        }
      }
    }
    for (int r = 0; r < b; ++r) {
      const int64_t i = k * b + r;
      R.rp[i + 1] = (i + 1) * b;
      for (int q = 0; q < b; ++q) {
        R.ci[size_t(i) * b + q] = int32_t(k * b + q);
        R.v[size_t(i) * b + q] = inv[size_t(r) * b + q];
      }
    }
  }
  drop_zeros(R);
  return R;
}

// The fluid operator the preconditioner inverts in place of the Schur
// complement X = F - C~_fs S^{-1} C_sf (C~_fs = C_fs - C_fm M^{-1} C_ms) of
// the factorisation in Section 4.1: F itself (FSI_X_F, the perturbation
// dropped), or with S and M replaced by their node-block diagonals D_S, D_M
// (d x d blocks per field and node; FSI_X_BLOCKDIAG, the block-diagonal
// approximation Section 4.1 cites from Langer and Yang, 2016):
// X ~ F - (C_fs - C_fm (D_M^{-1} C_ms)) (D_S^{-1} C_sf).
HCsr fluid_operator_refined(const fsi_ctx& c) {
  const HCsr& F = c.blk[FSI_F];
  const HCsr DSi = node_block_inverse(c.blk[FSI_S], c.d);
  const HCsr DMi = node_block_inverse(c.blk[FSI_M], c.d);
  const HCsr Ct = add(c.blk[FSI_CFS], spgemm(c.blk[FSI_CFM], spgemm(DMi, c.blk[FSI_CMS])), -1.0);
  HCsr X = add(F, spgemm(Ct, spgemm(DSi, c.blk[FSI_CSF])), -1.0);
  drop_zeros(X);
  return X;
}

void build_host_hierarchies(fsi_ctx& c, const fsi_precond_opts& o, const SaParams& prm) {
    const int d = c.d;
    const HCsr& S = c.blk[FSI_S];
    HCsr Xop;  // stays empty with X ~ F (the fluid block itself is used)
    if (o.x_approx == FSI_X_BLOCKDIAG) Xop = fluid_operator_refined(c);
    const HCsr& F = o.x_approx == FSI_X_BLOCKDIAG ? Xop : c.blk[FSI_F];
    // operators of the five hierarchies
    // scalar L of M = L (x) I_d: the first row of every node, columns / d
    const HCsr& M = c.blk[FSI_M];
    HCsr Lm = build_rows(
        M.nrows / d, M.nrows / d, [&](int64_t I) { return M.rp[I * d + 1] - M.rp[I * d]; },
        [&](int64_t I, int32_t* oc, double* ov) {
          for (int64_t k = M.rp[I * d]; k < M.rp[I * d + 1]; ++k) {
            *oc++ = M.ci[k] / d;
            *ov++ = M.v[k];
          }
        });
    HCsr Svv = sub_block(S, 0, c.n_vs, 0, c.n_vs);
    HCsr Svu = sub_block(S, 0, c.n_vs, c.n_vs, c.n_s);
    HCsr Sig = add(Svv, Svu, c.dt_theta);            // Sigma_s = S_vv + dt theta S_vu
    HCsr Suu = sub_block(S, c.n_vs, c.n_s, c.n_vs, c.n_s);
    HCsr Af = sub_block(F, 0, c.n_vf, 0, c.n_vf);
    HCsr Dm = sub_block(F, c.n_vf, c.n_f, 0, c.n_vf);
    HCsr Gm = sub_block(F, 0, c.n_vf, c.n_vf, c.n_f);
    HCsr Zpp = sub_block(F, c.n_vf, c.n_f, c.n_vf, c.n_f);  // empty unless X ~ F was refined
    HCsr Sp;  // Z - D W^{-1} G: W = diag(A_f) (SIMPLE) or its absolute row sums (SIMPLEC)
    {
      std::vector<double> dA = diagonal(Af);
      std::vector<double> dinv(dA.size());
      std::atomic<bool> zero{false};
      parallel_for(int64_t(dA.size()), [&](int64_t b, int64_t e) {
        for (int64_t i = b; i < e; ++i) {
          if (dA[i] == 0.0) zero.store(true);
          double w = dA[i];
          if (o.schur == FSI_SCHUR_SIMPLEC) {
            w = 0.0;
            for (int64_t k = Af.rp[i]; k < Af.rp[i + 1]; ++k) w += std::fabs(Af.v[k]);
          }
          dinv[i] = 1.0 / w;
        }
      });
      if (zero.load()) throw Error(FSI_ERR_NUMERIC, "zero diagonal in the fluid velocity block");
      HCsr Ds = Dm;
      scale_cols(Ds, dinv);
      Sp = device_spgemm(Ds, Gm, c.stream);
      parallel_for(Sp.nnz(), [&](int64_t b, int64_t e) {
        for (int64_t k = b; k < e; ++k) Sp.v[k] = -Sp.v[k];
      });
      if (Zpp.nnz() > 0) Sp = add(Sp, Zpp, 1.0);
      drop_zeros(Sp);
    }
    int krig = 0;
    std::vector<double> Brig = rigid_modes(c, krig);
    std::vector<double> Bt(size_t(c.n_vf) * d, 0.0);
    for (int64_t i = 0; i < c.n_vf; ++i) Bt[size_t(i) * d + (i % d)] = 1.0;
    HCsr* ops[FSI_NHIER] = {&Lm, &Sig, &Suu, &Af, &Sp};
    const int blocks[FSI_NHIER] = {1, d, 1, d, 1};
    const std::vector<double> ones_m(Lm.nrows, 1.0), ones_s(c.n_vs, 1.0), ones_p(c.n_p, 1.0);
    const std::vector<double>* Bs[FSI_NHIER] = {&ones_m, &Brig, &ones_s, &Bt, &ones_p};
    const int ks[FSI_NHIER] = {1, krig, 1, d, 1};
    static const char* hn[FSI_NHIER] = {"H_M", "H_SIG", "H_MS", "H_A", "H_P"};
    SaHierarchy hh[FSI_NHIER];
    // the sparse products and the power iteration's products on the device
    // (bitwise equal to the host's)
    const SpgemmFn mul = [&](const HCsr& X, const HCsr& Y) { return device_spgemm(X, Y, c.stream); };
    const ScaledProductFactory power = [&](const HCsr& X, const std::vector<double>& dv) {
      return device_scaled_product(X, dv, c.stream);
    };
    // H_A (by far the largest) on a host thread of its own while this thread
    // sets up the other four; each setup is deterministic, so the hierarchies
    // do not depend on the overlap
    std::string msg[FSI_NHIER];
    double ms[FSI_NHIER] = {};
    long long rows[FSI_NHIER];
    for (int h = 0; h < FSI_NHIER; ++h) rows[h] = (long long)ops[h]->nrows;
    auto run = [&](int h) {
      PhaseTimer t("sa_setup");
      msg[h] = sa_setup(std::move(*ops[h]), blocks[h], *Bs[h], ks[h], prm, hh[h], mul, power);
      ms[h] = t.ms();
    };
    std::exception_ptr err_a, err_o;
    std::thread ta([&] {
      try {
        HIP_TRY(hipSetDevice(c.device));  // the current device is per thread
        run(FSI_H_A);
      } catch (...) {
        err_a = std::current_exception();
      }
    });
    try {
      for (int h = 0; h < FSI_NHIER; ++h)
        if (h != FSI_H_A) run(h);
    } catch (...) {
      err_o = std::current_exception();
    }
    ta.join();
    if (err_o) std::rethrow_exception(err_o);
    if (err_a) std::rethrow_exception(err_a);
    for (int h = 0; h < FSI_NHIER; ++h) {
      if (!msg[h].empty()) throw Error(FSI_ERR_NUMERIC, std::string(hn[h]) + ": " + msg[h]);
      log_line("SA setup %s: %.1f ms (%lld rows, %zu levels)", hn[h], ms[h], rows[h], hh[h].levels.size());
    }
    for (int h = 0; h < FSI_NHIER; ++h) c.host_h[h] = std::move(hh[h]);
    c.fluid_op = std::move(Xop);
    c.have_host_h = true;
    c.host_prm = prm;
    c.host_schur = o.schur;
    c.host_x_approx = o.x_approx;
}

constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current), taken once
// per device; nullptr if the runtime cannot give it.
float* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[device] = static_cast<float*>(p);
  }
  return g_scratch_ptr[device];
}

// The learned correction x = MLP(b) of hierarchy `which` (shared by
// fsi_mlp_forward and its allocation-free variant): in FP32 precision b and x
// pass through the FP32 staging vectors bf, xf.
void mlp_forward_impl(fsi_ctx& c, int which, const double* b, double* x, float* bf, float* xf) {
  MlpState& M = mlp_state(c, which);
  hipStream_t s = c.stream;
  const unsigned grid = mlp_infer_grid(M.n_nodes);
  const int32_t* nbr = M.nbr.as<int32_t>();
  auto run = [&](auto tag, const auto* bb, const auto* dinv, auto* xx) {
    using T = decltype(tag);
    if (M.d == 2) {
      if (M.use.per_dof) mlp_infer_kernel<2, true, T><<<grid, 256, 0, s>>>(M.n_nodes, nbr, bb, dinv, M.use.w, xx);
      else mlp_infer_kernel<2, false, T><<<grid, 256, 0, s>>>(M.n_nodes, nbr, bb, dinv, M.use.w, xx);
    } else {
      if (M.use.per_dof) mlp_infer_kernel<3, true, T><<<grid, 256, 0, s>>>(M.n_nodes, nbr, bb, dinv, M.use.w, xx);
      else mlp_infer_kernel<3, false, T><<<grid, 256, 0, s>>>(M.n_nodes, nbr, bb, dinv, M.use.w, xx);
    }
  };
  if (c.precision == FSI_P_F64) {
    DHier<double>& H = c.p64->H[which];
    run(double(0), b, H.lev[0].dinv->as<double>(), x);
  } else {
    DHier<float>& H = c.p32->H[which];
    const int64_t n = M.n_nodes * M.d;
    cast_kernel<double, float><<<grid_for(n, kBlock * 4), kBlock, 0, s>>>(n, b, bf);
    run(float(0), static_cast<const float*>(bf), H.lev[0].dinv->as<float>(), xf);
    cast_kernel<float, double><<<grid_for(n, kBlock * 4), kBlock, 0, s>>>(n, xf, x);
  }
}


}  // namespace

// =================================================================== C ABI
extern "C" {

void fsi_default_precond_opts(fsi_precond_opts* o) {
  if (!o) return;
  *o = fsi_precond_opts{};
  o->precision = FSI_P_F64;
  o->max_coarse = 500;
  o->max_levels = 10;
  o->strength0 = 0.08;
  o->cheb_degree = 0;
  o->cheb_mask = (1 << FSI_H_MS) | (1 << FSI_H_SIG) | (1 << FSI_H_P);
  o->poly_mask = 0;
  o->poly_degree = 3;
  o->schur = FSI_SCHUR_SIMPLE;
  o->poly_ratio = 8.0;
  o->fluid_inner = 0;
  o->fluid_inner_pc = FSI_INNER_UZAWA;
  o->reuse = 0;
  o->x_approx = FSI_X_F;
  o->uzawa_inner = 0;
  o->order = FSI_ORDER_MSF;
}

void fsi_default_solve_opts(fsi_solve_opts* o) {
  if (!o) return;
  o->tol = 1e-8;
  o->restart = 50;
  o->maxit = 2000;
  o->timing = 0;
  o->pad = 0;
}

fsi_status fsi_create(fsi_ctx** ctx, int device, void* hip_stream) {
  if (!ctx) return FSI_ERR_ARG;
  *ctx = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n == 0) {
    g_create_err = "no HIP device available";
    return FSI_ERR_HIP;
  }
  if (device < 0 || device >= n) {
    g_create_err = "device index out of range";
    return FSI_ERR_ARG;
  }
  auto* c = new (std::nothrow) fsi_ctx();
  if (!c) return FSI_ERR_OOM;
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (const char* g = std::getenv("FSI_GRAPHS")) c->use_graphs = std::strcmp(g, "0") != 0;
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    g_create_err = "hipSetDevice failed";
    return FSI_ERR_HIP;
  }
  c->scratch = scratch_address(device);
  if (!c->scratch) {
    delete c;
    g_create_err = "hipGetSymbolAddress of the staging array failed";
    return FSI_ERR_HIP;
  }
  *ctx = c;
  return FSI_OK;
}

fsi_status fsi_destroy(fsi_ctx* ctx) {
  if (!ctx) return FSI_OK;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  delete ctx;
  return FSI_OK;
}

const char* fsi_last_error(const fsi_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

// The structural identities the preconditioner relies on (Sections 4.3,
// 4.4 and the mesh model): S_uv = -dt_theta S_uu within 1e-12 relative, an
// empty pressure block of F, and M = L (x) I_d.  Throws FSI_ERR_STRUCT.
void check_structure(const HCsr* H, int d, int64_t nvs, int64_t nvf, int64_t nf, double dt_theta) {
  HCsr Suv = sub_block(H[FSI_S], nvs, 2 * nvs, 0, nvs);
  HCsr Suu = sub_block(H[FSI_S], nvs, 2 * nvs, nvs, 2 * nvs);
  double mx = 0.0;
  for (double v : Suu.v) mx = std::max(mx, std::fabs(v));
  HCsr diff = add(Suv, Suu, dt_theta);
  double dmax = 0.0;
  for (double v : diff.v) dmax = std::max(dmax, std::fabs(v));
  if (!(dmax <= 1e-12 * dt_theta * mx))
    throw Error(FSI_ERR_STRUCT, "S_uv != -dt_theta S_uu (equal-order solid mass identity)");
  HCsr Fpp = sub_block(H[FSI_F], nvf, nf, nvf, nf);
  if (Fpp.nnz() != 0) throw Error(FSI_ERR_STRUCT, "pressure-pressure block of F must be empty");
  const HCsr& M = H[FSI_M];
  std::atomic<bool> kron_ok{true};
  parallel_for(M.nrows, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e && kron_ok.load(std::memory_order_relaxed); ++i) {
      const int64_t I = i / d, ci = i % d;
      const int64_t r0 = I * d;
      bool ok = M.rp[i + 1] - M.rp[i] == M.rp[r0 + 1] - M.rp[r0];
      for (int64_t k = M.rp[i], k0 = M.rp[r0]; ok && k < M.rp[i + 1]; ++k, ++k0)
        ok = M.ci[k] % d == ci && M.ci[k] / d == M.ci[k0] / d && M.v[k] == M.v[k0];
      if (!ok) kron_ok.store(false);
    }
  });
  if (!kron_ok.load()) throw Error(FSI_ERR_STRUCT, "mesh block is not L (x) I_d");
}

// Block rows and columns of the eight stored blocks (mesh 0, solid 1, fluid 2).
constexpr int kBlkRow[FSI_NBLK] = {0, 0, 1, 1, 1, 2, 2, 2};
constexpr int kBlkCol[FSI_NBLK] = {0, 1, 0, 1, 2, 0, 1, 2};

// Monolithic A_h with global columns (row i of block row r: the blocks of
// that row in column order, their columns shifted; built on the host threads).
HCsr assemble_ah(const HCsr* H, int64_t n_m, int64_t n_s, int64_t N) {
  const int64_t off[3] = {0, n_m, n_m + n_s};
  auto block_row = [&](int64_t gi, int& r, int64_t& i) {
    r = gi < off[1] ? 0 : gi < off[2] ? 1 : 2;
    i = gi - off[r];
  };
  return build_rows(
      N, N,
      [&](int64_t gi) {
        int r;
        int64_t i, n = 0;
        block_row(gi, r, i);
        for (int b = 0; b < FSI_NBLK; ++b)
          if (kBlkRow[b] == r) n += H[b].rp[i + 1] - H[b].rp[i];
        return n;
      },
      [&](int64_t gi, int32_t* oc, double* ov) {
        int r;
        int64_t i;
        block_row(gi, r, i);
        for (int b = 0; b < FSI_NBLK; ++b) {
          if (kBlkRow[b] != r) continue;
          const HCsr& A = H[b];
          for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
            *oc++ = int32_t(A.ci[k] + off[kBlkCol[b]]);
            *ov++ = A.v[k];
          }
        }
      });
}

// The row segments of the stored A_h: mesh, solid, fluid-velocity and
// pressure rows; the d velocity rows of a fluid node share their columns (the
// stress couples the components) and are stored as groups of d rows, one
// column index per d values.  Solid rows differ in about half their columns:
// plain rows.
void ah_segments(int64_t n_m, int64_t n_s, int64_t n_vf, int64_t N, int d, int64_t* bounds, int* groups) {
  const int64_t b[5] = {0, n_m, n_m + n_s, n_m + n_s + n_vf, N};
  const int g[4] = {1, 1, d, 1};
  std::copy(b, b + 5, bounds);
  std::copy(g, g + 4, groups);
}

fsi_status fsi_setup_blocks(fsi_ctx* ctx, const fsi_layout* L, const fsi_csr blk[FSI_NBLK], int mem) {
  return guarded(ctx, [&]() -> fsi_status {
    if (!L || !blk) throw Error(FSI_ERR_ARG, "layout or blocks is NULL");
    if (mem != 0) throw Error(FSI_ERR_ARG, "only host CSR input (mem = 0) is supported");
    const int d = L->dim;
    if (d != 2 && d != 3) throw Error(FSI_ERR_ARG, "dim must be 2 or 3");
    if (L->n_m < 0 || L->n_s <= 0 || L->n_f <= 0 || L->n_vs <= 0 || L->n_vf <= 0)
      throw Error(FSI_ERR_ARG, "block sizes must be positive");
    if (L->n_s != 2 * L->n_vs) throw Error(FSI_ERR_ARG, "n_s must equal 2 n_vs");
    if (L->n_vf >= L->n_f) throw Error(FSI_ERR_ARG, "n_vf must be smaller than n_f");
    if (L->n_m % d || L->n_vs % d || L->n_vf % d) throw Error(FSI_ERR_ARG, "vector blocks must be multiples of dim");
    if (!(L->dt_theta > 0.0)) throw Error(FSI_ERR_ARG, "dt_theta must be positive");
    const int64_t N = L->n_m + L->n_s + L->n_f;
    if (N >= (int64_t(1) << 31)) throw Error(FSI_ERR_ARG, "N must be below 2^31");
    if (!L->coords || !L->dof_node || L->n_nodes <= 0) throw Error(FSI_ERR_ARG, "coords and dof_node are required");
    const int64_t sz[3] = {L->n_m, L->n_s, L->n_f};
    const int bi[FSI_NBLK] = {0, 0, 1, 1, 1, 2, 2, 2};
    const int bj[FSI_NBLK] = {0, 1, 0, 1, 2, 0, 1, 2};
    static const char* names[FSI_NBLK] = {"M", "C_ms", "C_sm", "S", "C_sf", "C_fm", "C_fs", "F"};
    for (int b = 0; b < FSI_NBLK; ++b) {
      const fsi_csr& A = blk[b];
      if (A.nrows != sz[bi[b]] || A.ncols != sz[bj[b]])
        throw Error(FSI_ERR_ARG, std::string("block ") + names[b] + " has the wrong shape");
      std::string m = csr_check(A.nrows, A.ncols, A.nnz, A.rowptr, A.col, A.val);
      if (!m.empty()) throw Error(FSI_ERR_CSR, std::string("block ") + names[b] + ": " + m);
    }
    for (int64_t i = 0; i < N; ++i)
      if (L->dof_node[i] < 0 || L->dof_node[i] >= L->n_nodes) throw Error(FSI_ERR_ARG, "dof_node out of range");
    if (L->node_ijk)
      for (int64_t i = 0; i < L->n_nodes * d; ++i)
        if (L->node_ijk[i] < 0 || L->node_ijk[i] > (1 << 20)) throw Error(FSI_ERR_ARG, "node_ijk out of range");
    // host copies (the context is only modified once everything validated)
    HCsr H[FSI_NBLK];
    for (int b = 0; b < FSI_NBLK; ++b) H[b] = csr_copy(blk[b].nrows, blk[b].ncols, blk[b].rowptr, blk[b].col, blk[b].val);
    const int64_t nvs = L->n_vs, nvf = L->n_vf;
    check_structure(H, d, nvs, nvf, L->n_f, L->dt_theta);
    HCsr Ah = assemble_ah(H, L->n_m, L->n_s, N);
    int64_t bounds[5];
    int groups[4];
    ah_segments(L->n_m, L->n_s, nvf, N, d, bounds, groups);
    PhaseTimer t_up("setup_blocks: A_h segments upload");
    DCsr<double> dAh = upload_segments<double>(Ah, bounds, groups, 4, ctx->stream);
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    t_up.done();
    log_staging("setup_blocks");
    // commit
    fsi_ctx& c = *ctx;
    c.d = d;
    c.n_m = L->n_m; c.n_s = L->n_s; c.n_f = L->n_f; c.n_vs = nvs; c.n_vf = nvf;
    c.n_p = L->n_f - nvf; c.N = N;
    c.dt_theta = L->dt_theta;
    c.coords.assign(L->coords, L->coords + L->n_nodes * d);
    if (L->node_ijk) c.node_ijk.assign(L->node_ijk, L->node_ijk + L->n_nodes * d);
    else c.node_ijk.clear();
    c.dof_node.assign(L->dof_node, L->dof_node + N);
    for (int b = 0; b < FSI_NBLK; ++b) c.blk[b] = std::move(H[b]);
    c.Ah = dAh;
    c.fe.reset();
    c.have_system = true;
    c.have_precond = false;
    c.have_host_h = false;
    c.drop_graphs();
    c.m_alloc = -1;
    c.p64.reset();
    c.p32.reset();
    c.m_alloc = -1;
    return FSI_OK;
  });
}

fsi_status fsi_update_values(fsi_ctx* ctx, const fsi_csr blk[FSI_NBLK]) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    if (!c.have_system) throw Error(FSI_ERR_STATE, "fsi_setup_blocks must come first");
    if (!blk) throw Error(FSI_ERR_ARG, "blocks is NULL");
    static const char* names[FSI_NBLK] = {"M", "C_ms", "C_sm", "S", "C_sf", "C_fm", "C_fs", "F"};
    for (int b = 0; b < FSI_NBLK; ++b) {
      const fsi_csr& A = blk[b];
      const HCsr& O = c.blk[b];
      if (A.nrows != O.nrows || A.ncols != O.ncols || A.nnz != O.nnz() || !A.rowptr || (A.nnz && (!A.col || !A.val)))
        throw Error(FSI_ERR_ARG, std::string("block ") + names[b] + ": not the stored sparsity pattern");
      std::atomic<bool> same{true};
      parallel_for(A.nrows, [&](int64_t i0, int64_t i1) {
        bool ok = std::memcmp(A.rowptr + i0, O.rp.data() + i0, sizeof(int64_t) * size_t(i1 - i0 + 1)) == 0;
        if (ok && O.rp[i1] > O.rp[i0])
          ok = std::memcmp(A.col + O.rp[i0], O.ci.data() + O.rp[i0], sizeof(int32_t) * size_t(O.rp[i1] - O.rp[i0])) == 0;
        if (ok)
          for (int64_t k = O.rp[i0]; k < O.rp[i1] && ok; ++k) ok = std::isfinite(A.val[k]);
        if (!ok) same.store(false);
      });
      if (!same.load())
        throw Error(FSI_ERR_ARG, std::string("block ") + names[b] + ": not the stored sparsity pattern, or non-finite values");
    }
    HCsr H[FSI_NBLK];
    for (int b = 0; b < FSI_NBLK; ++b) H[b] = csr_copy(blk[b].nrows, blk[b].ncols, blk[b].rowptr, blk[b].col, blk[b].val);
    check_structure(H, c.d, c.n_vs, c.n_vf, c.n_f, c.dt_theta);
    const HCsr Ah = assemble_ah(H, c.n_m, c.n_s, c.N);
    int64_t bounds[5];
    int groups[4];
    ah_segments(c.n_m, c.n_s, c.n_vf, c.N, c.d, bounds, groups);
    PhaseTimer t_up("update_values: A_h values refresh");
    refresh_segments<double>(c.Ah, Ah, bounds, groups, 4, c.stream);
    HIP_TRY(hipStreamSynchronize(c.stream));
    t_up.done();
    for (int b = 0; b < FSI_NBLK; ++b) c.blk[b] = std::move(H[b]);
    return FSI_OK;
  });
}

static fsi_status build_precond_impl(fsi_ctx& c, const fsi_precond_opts* opts);

fsi_status fsi_build_precond(fsi_ctx* ctx, const fsi_precond_opts* opts) {
  return guarded(ctx, [&]() -> fsi_status { return build_precond_impl(*ctx, opts); });
}

static fsi_status build_precond_impl(fsi_ctx& c, const fsi_precond_opts* opts) {
  {
    if (!c.have_system) throw Error(FSI_ERR_STATE, "fsi_setup_blocks must come first");
    fsi_precond_opts o;
    fsi_default_precond_opts(&o);
    if (opts) o = *opts;
    if (o.precision != FSI_P_F64 && o.precision != FSI_P_F32 && o.precision != FSI_P_F32_BF16DIAG)
      throw Error(FSI_ERR_ARG, "unknown precision");
    if (o.schur != FSI_SCHUR_SIMPLE && o.schur != FSI_SCHUR_SIMPLEC)
      throw Error(FSI_ERR_ARG, "unknown pressure Schur approximation");
    if (o.fluid_inner < 0 || o.fluid_inner > kInnerMax)
      throw Error(FSI_ERR_ARG, "inner GMRES steps of the fluid inverse must be in 0..16");
    if (o.fluid_inner_pc != FSI_INNER_UZAWA && o.fluid_inner_pc != FSI_INNER_TRIANGULAR)
      throw Error(FSI_ERR_ARG, "unknown preconditioner of the inner fluid GMRES");
    if (o.max_coarse < 1 || o.max_levels < 1 || o.max_levels > 16 || !(o.strength0 >= 0.0))
      throw Error(FSI_ERR_ARG, "bad AMG options");
    if (o.cheb_degree < 0 || o.cheb_degree > 8 || (o.cheb_mask & ~0x1f) != 0)
      throw Error(FSI_ERR_ARG, "bad Chebyshev options");
    if (o.cheb_degree > 0 && (o.cheb_mask & (1 << FSI_H_A)))
      throw Error(FSI_ERR_ARG, "Chebyshev sweeps need a real spectrum: not for the nonsymmetric H_A");
    if ((o.poly_mask & ~0x1f) != 0 || (o.poly_mask && (o.poly_degree < 2 || o.poly_degree > 16)) ||
        (o.poly_mask && !(o.poly_ratio > 1.0)) || (o.poly_mask & (1 << FSI_H_A)))
      throw Error(FSI_ERR_ARG, "bad Chebyshev-only options (degree 2..16, ratio > 1, not H_A)");
    if (o.reuse != 0 && o.reuse != 1) throw Error(FSI_ERR_ARG, "reuse must be 0 or 1");
    if (o.uzawa_inner < 0 || o.uzawa_inner > kInnerMax)
      throw Error(FSI_ERR_ARG, "GMRES steps per inverse of the Uzawa-like step must be in 0..16");
    if (o.uzawa_inner > 0 && o.fluid_inner > 0)
      throw Error(FSI_ERR_ARG, "GMRES on F and GMRES on the Uzawa-like step's inverses do not combine");
    if (o.x_approx != FSI_X_F && o.x_approx != FSI_X_BLOCKDIAG)
      throw Error(FSI_ERR_ARG, "unknown approximation of the fluid Schur complement X");
    if (o.order < FSI_ORDER_MSF || o.order > FSI_ORDER_FMS) throw Error(FSI_ERR_ARG, "unknown block order");
    SaParams prm;
    prm.eps0 = o.strength0;
    prm.max_coarse = o.max_coarse;
    prm.max_levels = o.max_levels;
    PhaseTimer t_build("build_precond");
    if (o.reuse) {
      if (!c.have_host_h) throw Error(FSI_ERR_STATE, "reuse needs a previous fsi_build_precond of this system");
      if (c.host_prm.eps0 != prm.eps0 || c.host_prm.max_coarse != prm.max_coarse ||
          c.host_prm.max_levels != prm.max_levels || c.host_schur != o.schur || c.host_x_approx != o.x_approx)
        throw Error(FSI_ERR_STATE,
                    "reuse needs the AMG parameters and the Schur and X options of the previous build");
    } else {
      PhaseTimer t("host hierarchies (operators and SA setups)");
      build_host_hierarchies(c, o, prm);
      t.done();
    }
    for (int h = 0; h < FSI_NHIER; ++h) {
      c.poly[h] = ((o.poly_mask >> h) & 1) ? o.poly_degree : 0;
      c.cheb[h] = (c.poly[h] == 0 && o.cheb_degree > 0 && (o.cheb_mask >> h) & 1) ? o.cheb_degree : 0;
    }
    c.poly_ratio = o.poly_ratio;
    c.fluid_inner = o.fluid_inner;
    c.fluid_inner_pc = o.fluid_inner_pc;
    c.uzawa_inner = o.uzawa_inner;
    c.order = o.order;
    c.precision = o.precision;  // before prepare_mlp: it decides which hierarchies can learn
    prepare_mlp(c);
    c.drop_graphs();
    c.m_alloc = -1;
    c.p64.reset();
    c.p32.reset();
    {
      PhaseTimer t("device preconditioner (uploads, coupling blocks, workspace)");
      if (o.precision == FSI_P_F64) c.p64 = make_precond<double>(c);
      else c.p32 = make_precond<float>(c);
      t.done();
    }
    c.have_precond = true;
    c.popts = o;
    c.have_popts = true;
    t_build.done(o.reuse ? " (hierarchies reused)" : "");
    log_staging("build_precond");
    return FSI_OK;
  }
}


fsi_status fsi_solve(fsi_ctx* ctx, const double* b, double* x, const fsi_solve_opts* opts, fsi_solve_info* info) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    if (!c.have_precond) throw Error(FSI_ERR_STATE, "fsi_build_precond must come first");
    fsi_solve_opts o;
    fsi_default_solve_opts(&o);
    if (opts) o = *opts;
    if (!(o.tol > 0.0) || o.restart < 1 || o.restart > kMaxBasis - 8 || o.maxit < 0)
      throw Error(FSI_ERR_ARG, "bad solve options");
    check_device_ptr(b, "b");
    check_device_ptr(x, "x");
    if (b == x) throw Error(FSI_ERR_ARG, "b and x must not alias");
    fsi_solve_info local;
    fsi_status st = solve_impl(c, b, x, o, local);
    if (info) *info = local;
    return st;
  });
}

fsi_status fsi_spmv(fsi_ctx* ctx, const double* x, double* y) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    if (!c.have_system) throw Error(FSI_ERR_STATE, "fsi_setup_blocks must come first");
    check_device_ptr(x, "x");
    check_device_ptr(y, "y");
    if (x == y) throw Error(FSI_ERR_ARG, "x and y must not alias");
    spmv<double>(c.Ah, x, y, c.stream);
    HIP_TRY(hipGetLastError());
    return FSI_OK;
  });
}

fsi_status fsi_apply_precond(fsi_ctx* ctx, const double* r, double* z) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    if (!c.have_precond) throw Error(FSI_ERR_STATE, "fsi_build_precond must come first");
    check_device_ptr(r, "r");
    check_device_ptr(z, "z");
    if (r == z) throw Error(FSI_ERR_ARG, "r and z must not alias");
    apply_precond(c, r, z, c.stream);
    HIP_TRY(hipGetLastError());
    return FSI_OK;
  });
}

fsi_status fsi_vcycle(fsi_ctx* ctx, int which, const double* b, double* x) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    if (!c.have_precond) throw Error(FSI_ERR_STATE, "fsi_build_precond must come first");
    if (which < 0 || which >= FSI_NHIER) throw Error(FSI_ERR_ARG, "unknown hierarchy");
    check_device_ptr(b, "b");
    check_device_ptr(x, "x");
    if (b == x) throw Error(FSI_ERR_ARG, "b and x must not alias");
    hipStream_t s = c.stream;
    if (c.precision == FSI_P_F64) {
      vcycle(c.p64->H[which], b, x, s);
    } else {
      DHier<float>& H = c.p32->H[which];
      const int64_t n = H.lev[0].n * H.nv;
      Precond<float>& P = *c.p32;
      cast_kernel<double, float><<<grid_for(n, kBlock * 4), kBlock, 0, s>>>(n, b, P.rT->as<float>());
      vcycle(H, P.rT->as<float>(), P.zT->as<float>(), s);
      cast_kernel<float, double><<<grid_for(n, kBlock * 4), kBlock, 0, s>>>(n, P.zT->as<float>(), x);
    }
    HIP_TRY(hipGetLastError());
    return FSI_OK;
  });
}

fsi_status fsi_set_hierarchy(fsi_ctx* ctx, int which, int nlev, const fsi_csr* A, const fsi_csr* P,
                             const fsi_csr* R, const double* omega) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    if (!c.have_precond) throw Error(FSI_ERR_STATE, "fsi_build_precond must come first");
    if (which < 0 || which >= FSI_NHIER || nlev < 1 || nlev > 16 || !A) throw Error(FSI_ERR_ARG, "bad arguments");
    if (nlev > 1 && (!P || !R || !omega)) throw Error(FSI_ERR_ARG, "P, R and omega are required");
    SaHierarchy H;
    const int64_t n0 = c.host_h[which].levels[0].A.nrows;
    for (int l = 0; l < nlev; ++l) {
      std::string m = csr_check(A[l].nrows, A[l].ncols, A[l].nnz, A[l].rowptr, A[l].col, A[l].val);
      if (!m.empty()) throw Error(FSI_ERR_CSR, "level matrix: " + m);
      if (A[l].nrows != A[l].ncols) throw Error(FSI_ERR_ARG, "level matrices must be square");
      if (l == 0 && A[l].nrows != n0) throw Error(FSI_ERR_ARG, "finest level size mismatch");
      SaLevel L;
      L.A = csr_copy(A[l].nrows, A[l].ncols, A[l].rowptr, A[l].col, A[l].val);
      if (l < nlev - 1) {
        m = csr_check(P[l].nrows, P[l].ncols, P[l].nnz, P[l].rowptr, P[l].col, P[l].val);
        if (!m.empty()) throw Error(FSI_ERR_CSR, "prolongator: " + m);
        m = csr_check(R[l].nrows, R[l].ncols, R[l].nnz, R[l].rowptr, R[l].col, R[l].val);
        if (!m.empty()) throw Error(FSI_ERR_CSR, "restriction: " + m);
        if (P[l].nrows != A[l].nrows || P[l].ncols != A[l + 1].nrows || R[l].nrows != A[l + 1].nrows ||
            R[l].ncols != A[l].nrows)
          throw Error(FSI_ERR_ARG, "prolongator/restriction shapes do not chain");
        if (!std::isfinite(omega[l])) throw Error(FSI_ERR_ARG, "non-finite omega");
        L.P = csr_copy(P[l].nrows, P[l].ncols, P[l].rowptr, P[l].col, P[l].val);
        L.R = csr_copy(R[l].nrows, R[l].ncols, R[l].rowptr, R[l].col, R[l].val);
        L.omega = omega[l];
      }
      H.levels.push_back(std::move(L));
    }
    std::string m = sa_finalize(H);
    if (!m.empty()) throw Error(FSI_ERR_NUMERIC, m);
    const int nv = which == FSI_H_M ? c.d : 1;
    const bool lc = learned_capable(c, which);
    c.drop_graphs();
    c.m_alloc = -1;
    if (c.precision == FSI_P_F64)
      c.p64->H[which] = upload_hier<double>(H, nv, c.stream, lc, c.cheb[which], c.poly[which], c.poly_ratio,
                                            node_components(c, which));
    else
      c.p32->H[which] = upload_hier<float>(H, nv, c.stream, lc, c.cheb[which], c.poly[which], c.poly_ratio,
                                           node_components(c, which), c.precision == FSI_P_F32_BF16DIAG);
    HIP_TRY(hipStreamSynchronize(c.stream));
    c.host_h[which] = std::move(H);
    if (lc) {
      prepare_mlp(c);
      if (c.precision == FSI_P_F64) link_mlp(c, *c.p64);
      else link_mlp(c, *c.p32);
    }
    return FSI_OK;
  });
}

fsi_status fsi_hierarchy_info(fsi_ctx* ctx, int which, int32_t* nlev, int64_t* n, int64_t* nnz, double* omega) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    if (!c.have_precond) throw Error(FSI_ERR_STATE, "fsi_build_precond must come first");
    if (which < 0 || which >= FSI_NHIER || !nlev) throw Error(FSI_ERR_ARG, "bad arguments");
    const SaHierarchy& H = c.host_h[which];
    *nlev = int32_t(H.levels.size());
    for (size_t l = 0; l < H.levels.size() && l < 16; ++l) {
      if (n) n[l] = H.levels[l].A.nrows;
      if (nnz) nnz[l] = H.levels[l].A.nnz();
      if (omega) omega[l] = H.levels[l].omega;
    }
    return FSI_OK;
  });
}

fsi_status fsi_spmv_bytes(fsi_ctx* ctx, double* bytes) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    if (!c.have_system) throw Error(FSI_ERR_STATE, "fsi_setup_blocks must come first");
    if (!bytes) throw Error(FSI_ERR_ARG, "bad arguments");
    *bytes = c.Ah.bytes() + 16.0 * double(c.N);  // the matrix, x read once, y written
    return FSI_OK;
  });
}

fsi_status fsi_precond_bytes(fsi_ctx* ctx, double* bytes) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    if (!c.have_precond) throw Error(FSI_ERR_STATE, "fsi_build_precond must come first");
    if (!bytes) throw Error(FSI_ERR_ARG, "bad arguments");
    *bytes = precond_bytes(c);
    return FSI_OK;
  });
}

fsi_status fsi_vcycle_bytes(fsi_ctx* ctx, int which, double* bytes) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    if (!c.have_precond) throw Error(FSI_ERR_STATE, "fsi_build_precond must come first");
    if (which < 0 || which >= FSI_NHIER || !bytes) throw Error(FSI_ERR_ARG, "bad arguments");
    *bytes = c.precision == FSI_P_F64 ? c.p64->H[which].bytes_per_cycle : c.p32->H[which].bytes_per_cycle;
    return FSI_OK;
  });
}

fsi_status fsi_get_level(fsi_ctx* ctx, int which, int level, int what, int64_t* nrows, int64_t* ncols, int64_t* nnz,
                         int64_t* rowptr, int32_t* col, double* val) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    if (!c.have_precond) throw Error(FSI_ERR_STATE, "fsi_build_precond must come first");
    if (which < 0 || which >= FSI_NHIER) throw Error(FSI_ERR_ARG, "unknown hierarchy");
    const SaHierarchy& H = c.host_h[which];
    if (level < 0 || level >= int(H.levels.size())) throw Error(FSI_ERR_ARG, "level out of range");
    if (what == 1 && level == int(H.levels.size()) - 1) throw Error(FSI_ERR_ARG, "the coarsest level has no prolongator");
    if (what != 0 && what != 1) throw Error(FSI_ERR_ARG, "what must be 0 (A) or 1 (P)");
    const HCsr& A = what == 0 ? H.levels[level].A : H.levels[level].P;
    if (nrows) *nrows = A.nrows;
    if (ncols) *ncols = A.ncols;
    if (nnz) *nnz = A.nnz();
    if (rowptr) std::memcpy(rowptr, A.rp.data(), sizeof(int64_t) * (A.nrows + 1));
    if (col) std::memcpy(col, A.ci.data(), sizeof(int32_t) * A.nnz());
    if (val) std::memcpy(val, A.v.data(), sizeof(double) * A.nnz());
    return FSI_OK;
  });
}

fsi_status fsi_get_aggregates(fsi_ctx* ctx, int which, int level, int32_t* agg, int64_t* count) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    if (!c.have_precond) throw Error(FSI_ERR_STATE, "fsi_build_precond must come first");
    if (which < 0 || which >= FSI_NHIER) throw Error(FSI_ERR_ARG, "unknown hierarchy");
    const SaHierarchy& H = c.host_h[which];
    if (level < 0 || level >= int(H.levels.size()) - 1) throw Error(FSI_ERR_ARG, "level out of range");
    const auto& a = H.levels[level].agg;
    if (a.empty()) throw Error(FSI_ERR_STATE, "aggregates unknown for an imported hierarchy");
    if (count) *count = int64_t(a.size());
    if (agg) std::memcpy(agg, a.data(), sizeof(int32_t) * a.size());
    return FSI_OK;
  });
}

void fsi_default_mlp_train_opts(fsi_mlp_train_opts* o) {
  if (!o) return;
  o->steps = 400;
  o->batch = 16384;
  o->lr = 1e-3;
  o->exact_tol = 1e-10;
  o->exact_maxit = 300;
  o->seed = 0;
  o->loss = FSI_MLP_LOSS_ENERGY;
  o->coarse_cycles = 4;
}

fsi_status fsi_mlp_set_weights(fsi_ctx* ctx, int which, const float* W1, const float* W2, const float* W3) {
  return guarded(ctx, [&]() -> fsi_status {
    MlpState& M = mlp_state(*ctx, which);
    if (!W1 || !W2 || !W3) throw Error(FSI_ERR_ARG, "weights are NULL");
    mlp_upload_weights(*ctx, M, W1, W2, W3);
    HIP_TRY(hipMemsetAsync(M.streak.p, 0, sizeof(int), ctx->stream));  // new weights are tried again
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return FSI_OK;
  });
}

fsi_status fsi_mlp_get_weights(fsi_ctx* ctx, int which, float* W1, float* W2, float* W3) {
  return guarded(ctx, [&]() -> fsi_status {
    MlpState& M = mlp_state(*ctx, which);
    if (!W1 || !W2 || !W3) throw Error(FSI_ERR_ARG, "weights are NULL");
    if (!M.have_weights) throw Error(FSI_ERR_STATE, "no weights set");
    std::vector<float> wm(size_t(M.nparam()));
    HIP_TRY(hipMemcpyAsync(wm.data(), M.wm.p, 4 * wm.size(), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    const int kp = M.kp(), kin = M.kin(), d = M.d;
    for (int k = 0; k < kin; ++k)
      for (int h = 0; h < 64; ++h) W1[k * 64 + h] = wm[size_t(k) * 64 + h];
    const float* m2 = wm.data() + size_t(kp) * 64;
    for (int a = 0; a < 64 * 64; ++a) W2[a] = m2[a];
    const float* m3 = m2 + 64 * 64;
    for (int h = 0; h < 64; ++h)
      for (int q = 0; q < d; ++q) W3[h * d + q] = m3[h * 16 + q];
    return FSI_OK;
  });
}

fsi_status fsi_mlp_enable(fsi_ctx* ctx, int which, int enable) {
  return guarded(ctx, [&]() -> fsi_status {
    MlpState& M = mlp_state(*ctx, which);
    if (enable && !M.have_weights) throw Error(FSI_ERR_STATE, "no weights set");
    HIP_TRY(hipMemsetAsync(M.streak.p, 0, sizeof(int), ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (M.use.enabled != (enable != 0)) {
      M.use.enabled = enable != 0;
      ctx->drop_graphs();  // the captured kernel sequence changes
      ctx->m_alloc = -1;
    }
    return FSI_OK;
  });
}

fsi_status fsi_mlp_forward(fsi_ctx* ctx, int which, const double* b, double* x) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    MlpState& M = mlp_state(c, which);
    if (!M.have_weights) throw Error(FSI_ERR_STATE, "no weights set");
    check_device_ptr(b, "b");
    check_device_ptr(x, "x");
    if (c.precision == FSI_P_F64) {
      mlp_forward_impl(c, which, b, x, nullptr, nullptr);
    } else {
      const int64_t n = M.n_nodes * M.d;
      DevBuf bf, xf;
      bf.alloc(4 * n);
      xf.alloc(4 * n);
      mlp_forward_impl(c, which, b, x, bf.as<float>(), xf.as<float>());
      HIP_TRY(hipStreamSynchronize(c.stream));
    }
    HIP_TRY(hipGetLastError());
    return FSI_OK;
  });
}

fsi_status fsi_mlp_forward_noalloc(fsi_ctx* ctx, int which, const double* b, double* x) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    MlpState& M = mlp_state(c, which);
    if (!M.have_weights) throw Error(FSI_ERR_STATE, "no weights set");
    check_device_ptr(b, "b");
    check_device_ptr(x, "x");
    const int64_t n = M.n_nodes * M.d;
    if (c.precision != FSI_P_F64 && n > kNoAllocStage)
      throw Error(FSI_ERR_ARG, "the allocation-free call stages at most " + std::to_string(kNoAllocStage) +
                                   " entries; this level has " + std::to_string(n));
    float* st = c.scratch;  // device address of the staging array, taken in fsi_create
    if (!st) throw Error(FSI_ERR_STATE, "no staging array on this device");
    mlp_forward_impl(c, which, b, x, st, st + kNoAllocStage);
    HIP_TRY(hipGetLastError());
    return FSI_OK;
  });
}

fsi_status fsi_mlp_loss_grad(fsi_ctx* ctx, int which, int64_t m, const float* Z, const float* E, const float* w,
                             float* G1, float* G2, float* G3, double* loss) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    MlpState& M = mlp_state(c, which);
    if (!M.have_weights) throw Error(FSI_ERR_STATE, "no weights set");
    if (m <= 0 || !Z || !E || !w || !G1 || !G2 || !G3 || !loss) throw Error(FSI_ERR_ARG, "bad arguments");
    hipStream_t s = c.stream;
    const int kp = M.kp(), kin = M.kin(), d = M.d;
    std::vector<uint16_t> zb(size_t(m) * kp, 0);
    for (int64_t i = 0; i < m; ++i)
      for (int k = 0; k < kin; ++k) zb[size_t(i) * kp + k] = host_bf16(Z[i * kin + k]);
    DevBuf dZ, dE, dW;
    dZ.alloc(2 * zb.size());
    dE.alloc(4 * size_t(m) * d);
    dW.alloc(4 * size_t(m));
    HIP_TRY(hipMemcpyAsync(dZ.p, zb.data(), 2 * zb.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(dE.p, E, 4 * size_t(m) * d, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(dW.p, w, 4 * size_t(m), hipMemcpyHostToDevice, s));
    mlp_grad_pass(c, M, dZ.as<unsigned short>(), dE.as<float>(), dW.as<float>(), 0, m, float(2.0 / double(m)));
    float lsum = 0.f;
    HIP_TRY(hipMemcpyAsync(&lsum, M.loss.p, 4, hipMemcpyDeviceToHost, s));
    unpack_grad(c, M, G1, G2, G3);
    *loss = double(lsum) / double(m);
    return FSI_OK;
  });
}

fsi_status fsi_mlp_energy_grad(fsi_ctx* ctx, int which, const double* b, int coarse_cycles, float* G1, float* G2,
                               float* G3, double* loss) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    MlpState& M = mlp_state(c, which);
    if (!M.have_weights) throw Error(FSI_ERR_STATE, "no weights set");
    if (!G1 || !G2 || !G3 || !loss || coarse_cycles < 1) throw Error(FSI_ERR_ARG, "bad arguments");
    check_device_ptr(b, "b");
    double l = 0.0;
    if (c.precision == FSI_P_F64) {
      DHier<double>& H = c.p64->H[which];
      if (H.nv == 1) l = energy_grad_once<double, 1>(c, M, H, b, coarse_cycles);
      else if (H.nv == 2) l = energy_grad_once<double, 2>(c, M, H, b, coarse_cycles);
      else l = energy_grad_once<double, 3>(c, M, H, b, coarse_cycles);
    } else {
      DHier<float>& H = c.p32->H[which];
      if (H.nv == 1) l = energy_grad_once<float, 1>(c, M, H, b, coarse_cycles);
      else if (H.nv == 2) l = energy_grad_once<float, 2>(c, M, H, b, coarse_cycles);
      else l = energy_grad_once<float, 3>(c, M, H, b, coarse_cycles);
    }
    unpack_grad(c, M, G1, G2, G3);
    *loss = l;
    return FSI_OK;
  });
}

fsi_status fsi_mlp_collect(fsi_ctx* ctx, int max_vectors, int every) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    if (max_vectors < 0 || every < 1) throw Error(FSI_ERR_ARG, "bad arguments");
    for (auto& M : c.mlp) {
      M.rec.active = max_vectors > 0;
      M.rec.max_vectors = max_vectors;
      M.rec.every = every;
      M.rec.calls = 0;
      if (max_vectors == 0) M.rec.vecs.clear();
    }
    return FSI_OK;
  });
}

fsi_status fsi_mlp_train(fsi_ctx* ctx, const fsi_mlp_train_opts* opts, fsi_mlp_train_info* info) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    if (!c.have_precond) throw Error(FSI_ERR_STATE, "fsi_build_precond must come first");
    fsi_mlp_train_opts o;
    fsi_default_mlp_train_opts(&o);
    if (opts) o = *opts;
    if (o.steps < 0 || o.batch < 16 || !(o.lr > 0.0) || !(o.exact_tol > 0.0) || o.exact_maxit < 1 ||
        (o.loss != FSI_MLP_LOSS_L2 && o.loss != FSI_MLP_LOSS_ENERGY) || o.coarse_cycles < 1)
      throw Error(FSI_ERR_ARG, "bad training options");
    bool any = false;
    for (auto& M : c.mlp) any = any || (M.n_nodes > 0 && M.have_weights && !M.rec.vecs.empty());
    if (!any) throw Error(FSI_ERR_STATE, "nothing to train: set weights and record residuals first");
    for (auto& M : c.mlp) M.rec.active = false;
    fsi_mlp_train_info local{};
    if (o.loss == FSI_MLP_LOSS_L2) {
      if (c.precision == FSI_P_F64) mlp_train_l2<double>(c, *c.p64, o, local);
      else mlp_train_l2<float>(c, *c.p32, o, local);
    } else {
      if (c.precision == FSI_P_F64) mlp_train_energy<double>(c, *c.p64, o, local);
      else mlp_train_energy<float>(c, *c.p32, o, local);
    }
    for (auto& M : c.mlp)  // the trained networks are tried again
      if (M.streak.p) HIP_TRY(hipMemsetAsync(M.streak.p, 0, sizeof(int), c.stream));
    HIP_TRY(hipStreamSynchronize(c.stream));
    if (info) *info = local;
    return FSI_OK;
  });
}

// ------------------------------------------------- finite-element assembly
// The stored A_h as kernel-visible slot tables.
static AhSlots ah_slots(fsi_ctx& c) {
  AhSlots a{};
  const RowSegments& sg = c.Ah.seg;
  a.nseg = sg.nseg;
  for (int q = 0; q <= sg.nseg; ++q) a.row0[q] = sg.row0[q];
  for (int q = 0; q < sg.nseg; ++q) {
    a.grp[q] = sg.grp[q];
    a.grp_rp[q] = sg.grp_rp[q];
    a.grp_ci[q] = sg.grp_ci[q];
    a.grp_val[q] = static_cast<double*>(const_cast<void*>(sg.grp_val[q]));
  }
  a.rp = c.Ah.drp();
  a.ci = c.Ah.dci();
  a.val = c.Ah.val ? c.Ah.val->as<double>() : nullptr;
  return a;
}

// Residual R(U) into R (when R is given) and, with want_mat, the Jacobian's
// values into the stored A_h (cleared first); U = the given fields + dU.
static void fe_assemble(fsi_ctx& c, const double* dU, double* R, bool want_mat) {
  FeState& F = *c.fe;
  hipStream_t s = c.stream;
  AhSlots ah = ah_slots(c);
  if (R) HIP_TRY(hipMemsetAsync(R, 0, sizeof(double) * size_t(c.N), s));
  if (want_mat) {
    if (ah.val) HIP_TRY(hipMemsetAsync(ah.val, 0, c.Ah.val->bytes, s));
    for (int q = 0; q < ah.nseg; ++q)
      if (ah.grp[q] > 1) HIP_TRY(hipMemsetAsync(ah.grp_val[q], 0, c.Ah.grp_val[q]->bytes, s));
  }
  HIP_TRY(hipMemsetAsync(F.flag.p, 0, sizeof(int), s));
  const int D = F.prm.D;
  auto launch = [&](auto dc) {
    constexpr int DD = decltype(dc)::value;
    using Q = FeDims<DD>;
    constexpr int64_t GS = Q::NQ * Q::NQ + Q::NQ;
    int64_t max_cells = 0;
    for (int color = 0; color < (1 << DD); ++color) {
      int64_t n = 1;
      for (int a = 0; a < DD; ++a) n *= (F.prm.nc[a] - ((color >> a) & 1) + 1) / 2;
      max_cells = std::max(max_cells, n);
    }
    if (want_mat && F.pts.bytes < sizeof(double) * size_t(max_cells * Q::NPT * GS))
      F.pts.alloc(sizeof(double) * size_t(max_cells * Q::NPT * GS));
    for (int color = 0; color < (1 << DD); ++color) {
      int64_t ncell = 1;
      for (int a = 0; a < DD; ++a) ncell *= (F.prm.nc[a] - ((color >> a) & 1) + 1) / 2;
      if (ncell == 0) continue;
      const FeNodes nd = F.nodes();
      const double* bt = F.basis.as<double>();
      int* fl = F.flag.as<int>();
      if (R)
        fe_assemble_kernel<DD, FE_RESIDUAL><<<dim3(unsigned(ncell), 1), 256, 0, s>>>(F.prm, nd, bt, dU, color, R,
                                                                                     nullptr, ah, fl);
      if (want_mat) {
        double* pts = F.pts.as<double>();
        fe_assemble_kernel<DD, FE_POINTS><<<dim3(unsigned(ncell), 1), 256, 0, s>>>(F.prm, nd, bt, dU, color,
                                                                                   nullptr, pts, ah, fl);
        fe_assemble_kernel<DD, FE_CONTRACT><<<dim3(unsigned(ncell), Q::NCHUNK), 256, 0, s>>>(
            F.prm, nd, bt, dU, color, nullptr, pts, ah, fl);
      }
      HIP_TRY(hipGetLastError());
    }
  };
  if (D == 2) launch(std::integral_constant<int, 2>{});
  else launch(std::integral_constant<int, 3>{});
  int flag = 0;
  HIP_TRY(hipMemcpyAsync(&flag, F.flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (flag & 1) throw Error(FSI_ERR_NUMERIC, "the state has J <= 0 at a quadrature point of a fluid cell");
  if (flag & 4) throw Error(FSI_ERR_NUMERIC, "non-finite residual or Jacobian value");
  if (flag & 2) throw Error(FSI_ERR_STRUCT, "a cell matrix entry lies outside the stored sparsity pattern");
}

// The host copies of the eight blocks take the values of the stored A_h (for
// a preconditioner built from the assembled Jacobian).
static void fe_refresh_host_blocks(fsi_ctx& c) {
  FeState& F = *c.fe;
  hipStream_t s = c.stream;
  const int64_t off[4] = {0, c.n_m, c.n_m + c.n_s, c.N};
  const int bi[FSI_NBLK] = {0, 0, 1, 1, 1, 2, 2, 2};
  const int bj[FSI_NBLK] = {0, 1, 0, 1, 2, 0, 1, 2};
  AhSlots ah = ah_slots(c);
  PhaseTimer t("fe_jacobian: host block values read back");
  std::vector<double> vals[FSI_NBLK];  // new values; the patterns stay where they are
  HIP_TRY(hipMemsetAsync(F.flag.p, 0, sizeof(int), s));
  for (int b = 0; b < FSI_NBLK; ++b) {
    const HCsr& O = c.blk[b];
    if (!F.brp[b]) {
      F.brp[b] = upload_raw(O.rp, s);
      F.bci[b] = upload_raw(O.ci, s);
    }
    vals[b] = std::move(F.spare[b]);  // the previous read-back's array: no fresh zero-filled pages
    vals[b].resize(size_t(O.nnz()));
    if (O.nnz() == 0) continue;
    DevBuf dv;
    dv.alloc(sizeof(double) * size_t(O.nnz()));
    ah_block_gather_kernel<<<grid_for(O.nrows, kBlock), kBlock, 0, s>>>(
        O.nrows, F.brp[b]->as<int64_t>(), F.bci[b]->as<int32_t>(), off[bi[b]], off[bj[b]], ah, dv.as<double>(),
        F.flag.as<int>());
    HIP_TRY(hipGetLastError());
    d2h(vals[b].data(), dv.p, size_t(O.nnz()), s);
  }
  int flag = 0;
  HIP_TRY(hipMemcpyAsync(&flag, F.flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (flag) throw Error(FSI_ERR_STRUCT, "a block entry is missing from the stored A_h");
  // swap the values in, check the structural identities, swap back on failure
  for (int b = 0; b < FSI_NBLK; ++b) c.blk[b].v.swap(vals[b]);
  try {
    check_structure(c.blk, c.d, c.n_vs, c.n_vf, c.n_f, c.dt_theta);
  } catch (...) {
    for (int b = 0; b < FSI_NBLK; ++b) {
      c.blk[b].v.swap(vals[b]);
      F.spare[b] = std::move(vals[b]);
    }
    throw;
  }
  for (int b = 0; b < FSI_NBLK; ++b) F.spare[b] = std::move(vals[b]);  // the old values' arrays
  t.done();
}

// A'(U) into A_h (and, with host_blocks, into the host blocks); on any
// failure the stored values are restored from a device copy taken first, so
// the context is left as it was.
static void fe_jacobian_into_ah(fsi_ctx& c, const double* dU, bool host_blocks) {
  hipStream_t s = c.stream;
  AhSlots ah = ah_slots(c);
  std::vector<std::pair<double*, size_t>> arrays;
  if (ah.val) arrays.emplace_back(ah.val, c.Ah.val->bytes);
  for (int q = 0; q < ah.nseg; ++q)
    if (ah.grp[q] > 1) arrays.emplace_back(ah.grp_val[q], c.Ah.grp_val[q]->bytes);
  size_t total = 0;
  for (auto& a : arrays) total += a.second;
  DevBuf backup;
  backup.alloc(total);
  size_t off = 0;
  for (auto& a : arrays) {
    HIP_TRY(hipMemcpyAsync(backup.as<char>() + off, a.first, a.second, hipMemcpyDeviceToDevice, s));
    off += a.second;
  }
  try {
    fe_assemble(c, dU, nullptr, true);
    if (host_blocks) fe_refresh_host_blocks(c);
  } catch (...) {
    off = 0;
    for (auto& a : arrays) {
      (void)hipMemcpyAsync(a.first, backup.as<char>() + off, a.second, hipMemcpyDeviceToDevice, s);
      off += a.second;
    }
    (void)hipStreamSynchronize(s);
    throw;
  }
}

// max |x_i| over a device vector (NaN reads as +inf).
static double device_absmax(fsi_ctx& c, const double* x, int64_t n) {
  FeState& F = *c.fe;
  const unsigned nb = std::min<unsigned>(grid_for(n, kBlock * 4), 1024u);
  absmax_kernel<<<nb, kBlock, 0, c.stream>>>(n, x, F.part.as<double>());
  HIP_TRY(hipGetLastError());
  std::vector<double> h(nb);
  HIP_TRY(hipMemcpyAsync(h.data(), F.part.p, sizeof(double) * nb, hipMemcpyDeviceToHost, c.stream));
  HIP_TRY(hipStreamSynchronize(c.stream));
  double m = 0.0;
  for (double v : h) m = std::max(m, v);
  return m;
}


void fsi_default_newton_opts(fsi_newton_opts* o) {
  if (!o) return;
  *o = fsi_newton_opts{};
  o->rtol = 1e-6;
  o->reassemble_ratio = 0.1;
  o->max_steps = 25;
  o->precond = FSI_NEWTON_PC_REBUILD;
  o->lin_tol = 1e-3;
  o->restart = 50;
  o->maxit = 2000;
}

fsi_status fsi_fe_setup(fsi_ctx* ctx, const fsi_fe_mesh* m) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    if (!c.have_system) throw Error(FSI_ERR_STATE, "fsi_setup_blocks must come first");
    if (!m) throw Error(FSI_ERR_ARG, "mesh is NULL");
    if (m->dim != c.d) throw Error(FSI_ERR_ARG, "mesh dimension differs from the system's");
    if (!(m->theta > 0.0 && m->theta <= 1.0)) throw Error(FSI_ERR_ARG, "theta must lie in (0, 1]");
    if (!(m->dt > 0.0) || !(m->rho_f > 0.0) || !(m->nu_f > 0.0) || !(m->rho_s > 0.0) || !(m->mu_s > 0.0) ||
        !(m->lambda_s >= 0.0))
      throw Error(FSI_ERR_ARG, "material data and dt must be positive");
    if (std::fabs(m->dt * m->theta - c.dt_theta) > 1e-14 * c.dt_theta)
      throw Error(FSI_ERR_ARG, "dt * theta differs from the system's");
    const int D = m->dim;
    FeParams P{};
    P.D = D;
    int64_t nn = 1;
    for (int a = 0; a < 3; ++a) {
      P.nc[a] = a < D ? m->cells[a] : 1;
      P.NN[a] = 2 * P.nc[a] + 1;
      P.h[a] = a < D ? m->extent[a] / double(m->cells[a]) : 1.0;
      P.solid_lo[a] = a < D ? m->solid_lo[a] : 0;
      P.solid_hi[a] = a < D ? m->solid_hi[a] : 1;
      if (a < D) {
        if (m->cells[a] < 1 || m->cells[a] > 65535 || !(m->extent[a] > 0.0))
          throw Error(FSI_ERR_ARG, "cells must be in 1..65535 and extents positive");
        nn *= P.NN[a];
      }
    }
    if (nn != m->n_nodes) throw Error(FSI_ERR_ARG, "n_nodes must be the product of 2 cells + 1");
    // one launch per parity class holds its cells in blockIdx.x
    if (int64_t(P.nc[0]) * P.nc[1] * P.nc[2] > int64_t(INT32_MAX))
      throw Error(FSI_ERR_ARG, "more than 2^31 - 1 cells");
    P.rho_f = m->rho_f; P.nu_f = m->nu_f; P.rho_s = m->rho_s; P.mu_s = m->mu_s; P.lambda_s = m->lambda_s;
    P.dtth = m->dt * m->theta;
    P.theta = m->theta;
    P.dt = m->dt;
    P.newton_mesh = m->newton_mesh ? 1 : 0;
    const int64_t* dofs[3] = {m->vdof, m->udof, m->pdof};
    const double* fields[7] = {m->v, m->u, m->p, m->v_old, m->u_old, m->w, m->u_fz};
    for (auto* q : dofs)
      if (!q) throw Error(FSI_ERR_ARG, "dof arrays are required");
    for (auto* q : fields)
      if (!q) throw Error(FSI_ERR_ARG, "node fields are required");
    // dof numbers within range; every free dof named exactly once
    std::vector<unsigned char> seen(size_t(c.N), 0);
    for (int64_t n = 0; n < nn; ++n) {
      for (int f = 0; f < 2; ++f) {
        const int64_t b = dofs[f][n];
        if (b < -1 || b + D > c.N) throw Error(FSI_ERR_ARG, "dof number out of range");
        if (b >= 0)
          for (int k = 0; k < D; ++k) {
            if (seen[size_t(b + k)]) throw Error(FSI_ERR_ARG, "a dof is named twice");
            seen[size_t(b + k)] = 1;
          }
      }
      const int64_t pd = m->pdof[n];
      if (pd < -1 || pd >= c.N) throw Error(FSI_ERR_ARG, "dof number out of range");
      if (pd >= 0) {
        if (seen[size_t(pd)]) throw Error(FSI_ERR_ARG, "a dof is named twice");
        seen[size_t(pd)] = 1;
      }
    }
    for (unsigned char x : seen)
      if (!x) throw Error(FSI_ERR_ARG, "a free dof belongs to no node");
    for (int f = 0; f < 7; ++f) {
      const int64_t len = f == 2 ? nn : nn * D;
      for (int64_t i = 0; i < len; ++i)
        if (!std::isfinite(fields[f][i])) throw Error(FSI_ERR_NUMERIC, "node fields hold NaN or Inf");
    }
    auto fe = std::make_unique<FeState>();
    fe->prm = P;
    fe->n_nodes = nn;
    hipStream_t s = c.stream;
    DevBuf* db[3] = {&fe->vdof, &fe->udof, &fe->pdof};
    for (int f = 0; f < 3; ++f) {
      db[f]->alloc(sizeof(int64_t) * size_t(nn));
      h2d(db[f]->p, dofs[f], size_t(nn), s);
    }
    DevBuf* fb[7] = {&fe->v, &fe->u, &fe->p, &fe->v_old, &fe->u_old, &fe->w, &fe->u_fz};
    for (int f = 0; f < 7; ++f) {
      const int64_t len = f == 2 ? nn : nn * D;
      fb[f]->alloc(sizeof(double) * size_t(len));
      h2d(fb[f]->p, fields[f], size_t(len), s);
    }
    fe->flag.alloc(sizeof(int));
    fe->part.alloc(sizeof(double) * 1024);
    if (D == 2) {
      fe->basis.alloc(sizeof(double) * FeDims<2>::NPT * FeDims<2>::SH);
      const int jobs = FeDims<2>::NPT * (FeDims<2>::NQ2 + FeDims<2>::NQ1);
      fe_basis_kernel<2><<<(jobs + 255) / 256, 256, 0, s>>>(P, fe->basis.as<double>());
    } else {
      fe->basis.alloc(sizeof(double) * FeDims<3>::NPT * FeDims<3>::SH);
      const int jobs = FeDims<3>::NPT * (FeDims<3>::NQ2 + FeDims<3>::NQ1);
      fe_basis_kernel<3><<<(jobs + 255) / 256, 256, 0, s>>>(P, fe->basis.as<double>());
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    c.fe = std::move(fe);
    return FSI_OK;
  });
}

fsi_status fsi_fe_residual(fsi_ctx* ctx, const double* dU, double* R) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    if (!c.fe) throw Error(FSI_ERR_STATE, "fsi_fe_setup must come first");
    if (dU) check_device_ptr(dU, "dU");
    check_device_ptr(R, "R");
    if (dU == R) throw Error(FSI_ERR_ARG, "dU and R must not alias");
    fe_assemble(c, dU, R, false);
    return FSI_OK;
  });
}

fsi_status fsi_fe_jacobian(fsi_ctx* ctx, const double* dU, int host_blocks) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    if (!c.fe) throw Error(FSI_ERR_STATE, "fsi_fe_setup must come first");
    if (dU) check_device_ptr(dU, "dU");
    PhaseTimer t("fe_jacobian: A_h assembled on the device");
    fe_jacobian_into_ah(c, dU, host_blocks != 0);
    t.done();
    return FSI_OK;
  });
}

static void check_newton_opts(const fsi_ctx& c, const fsi_newton_opts& o) {
  if (!(o.rtol > 0.0) || !(o.reassemble_ratio >= 0.0) || o.max_steps < 0 || o.max_steps > FSI_NEWTON_MAX ||
      !(o.lin_tol > 0.0) || o.restart < 1 || o.restart > kMaxBasis - 8 || o.maxit < 1 ||
      (o.precond != FSI_NEWTON_PC_REBUILD && o.precond != FSI_NEWTON_PC_REUSE && o.precond != FSI_NEWTON_PC_KEEP))
    throw Error(FSI_ERR_ARG, "bad Newton options");
  if (o.precond == FSI_NEWTON_PC_KEEP && !c.have_precond)
    throw Error(FSI_ERR_STATE, "keeping the preconditioner needs a fsi_build_precond first");
}

// Algorithm newton with Section 6's quasi-Newton rule from U = fields + dU.
static fsi_status newton_impl(fsi_ctx& c, const fsi_newton_opts& o, double* dU, fsi_newton_info& out) {
  const auto t_start = std::chrono::steady_clock::now();
  auto ms_since = [](std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  };
  out = fsi_newton_info{};
  const int64_t N = c.N;
  DevBuf R, delta;
  R.alloc(sizeof(double) * size_t(N));
  delta.alloc(sizeof(double) * size_t(N));
  auto tic = std::chrono::steady_clock::now();
  fe_assemble(c, dU, R.as<double>(), false);
  out.t_assemble_ms += ms_since(tic);
  out.resid[0] = device_absmax(c, R.as<double>(), N);
  if (!std::isfinite(out.resid[0])) throw Error(FSI_ERR_NUMERIC, "the initial residual is not finite");
  fsi_precond_opts po;
  fsi_default_precond_opts(&po);
  if (c.have_popts) po = c.popts;
  fsi_solve_opts so;
  fsi_default_solve_opts(&so);
  so.tol = o.lin_tol;
  so.restart = o.restart;
  so.maxit = o.maxit;
  for (int k = 0;; ++k) {
    const double rk = out.resid[k];
    if (rk == 0.0 || rk < o.rtol * out.resid[0]) {
      out.converged = 1;
      break;
    }
    if (k == o.max_steps) break;
    // Section 6: assemble at the first step, then only when the last step
    // reduced the max-norm residual by less than 1 / ratio
    const bool assemble = k == 0 || rk > o.reassemble_ratio * out.resid[k - 1];
    out.reassembled[k] = assemble ? 1 : 0;
    if (assemble) {
      tic = std::chrono::steady_clock::now();
      fe_jacobian_into_ah(c, dU, o.precond != FSI_NEWTON_PC_KEEP);
      out.t_assemble_ms += ms_since(tic);
      ++out.reassemblies;
      if (o.precond != FSI_NEWTON_PC_KEEP) {
        tic = std::chrono::steady_clock::now();
        fsi_precond_opts pk = po;
        pk.reuse = (o.precond == FSI_NEWTON_PC_REUSE && c.have_host_h) ? 1 : 0;
        build_precond_impl(c, &pk);
        out.t_precond_ms += ms_since(tic);
      }
    }
    // J delta = R, then U_{k+1} = U_k - delta
    tic = std::chrono::steady_clock::now();
    HIP_TRY(hipMemsetAsync(delta.p, 0, sizeof(double) * size_t(N), c.stream));
    fsi_solve_info si{};
    solve_impl(c, R.as<double>(), delta.as<double>(), so, si);
    out.lin_iters[k] = si.iters;
    out.lin_iters_total += si.iters;
    sub_inplace_kernel<<<grid_for(N, kBlock), kBlock, 0, c.stream>>>(N, delta.as<double>(), dU);
    HIP_TRY(hipGetLastError());
    out.t_solve_ms += ms_since(tic);
    tic = std::chrono::steady_clock::now();
    fe_assemble(c, dU, R.as<double>(), false);
    out.t_assemble_ms += ms_since(tic);
    out.resid[k + 1] = device_absmax(c, R.as<double>(), N);
    out.steps = k + 1;
    if (!std::isfinite(out.resid[k + 1])) throw Error(FSI_ERR_NUMERIC, "the Newton residual is not finite");
  }
  out.t_total_ms = ms_since(t_start);
  log_line("newton: %d steps, %d assemblies, %d GMRES iterations, ||r||_inf %.3e -> %.3e, %.1f ms "
           "(assembly %.1f, preconditioner %.1f, solves %.1f)",
           out.steps, out.reassemblies, out.lin_iters_total, out.resid[0], out.resid[out.steps], out.t_total_ms,
           out.t_assemble_ms, out.t_precond_ms, out.t_solve_ms);
  return out.converged ? FSI_OK : FSI_NOT_CONVERGED;
}

fsi_status fsi_newton(fsi_ctx* ctx, const fsi_newton_opts* opts, double* dU, fsi_newton_info* info) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    if (!c.fe) throw Error(FSI_ERR_STATE, "fsi_fe_setup must come first");
    fsi_newton_opts o;
    fsi_default_newton_opts(&o);
    if (opts) o = *opts;
    check_newton_opts(c, o);
    check_device_ptr(dU, "dU");
    fsi_newton_info out{};
    const fsi_status st = newton_impl(c, o, dU, out);
    if (info) *info = out;
    return st;
  });
}

static void fe_advance(fsi_ctx& c, const double* dU) {
  FeState& F = *c.fe;
  fe_advance_kernel<<<grid_for(F.n_nodes, kBlock), kBlock, 0, c.stream>>>(
      F.n_nodes, F.prm.D, F.vdof.as<int64_t>(), F.udof.as<int64_t>(), F.pdof.as<int64_t>(), F.v.as<double>(),
      F.u.as<double>(), F.p.as<double>(), F.v_old.as<double>(), F.u_old.as<double>(), F.w.as<double>(),
      F.u_fz.as<double>(), dU);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(c.stream));
}

fsi_status fsi_fe_advance(fsi_ctx* ctx, const double* dU) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    if (!c.fe) throw Error(FSI_ERR_STATE, "fsi_fe_setup must come first");
    check_device_ptr(dU, "dU");
    fe_advance(c, dU);
    return FSI_OK;
  });
}

fsi_status fsi_fe_get_fields(fsi_ctx* ctx, double* v, double* u, double* p) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    if (!c.fe) throw Error(FSI_ERR_STATE, "fsi_fe_setup must come first");
    if (!v || !u || !p) throw Error(FSI_ERR_ARG, "field arrays are required");
    FeState& F = *c.fe;
    d2h(v, F.v.p, size_t(F.n_nodes * F.prm.D), c.stream);
    d2h(u, F.u.p, size_t(F.n_nodes * F.prm.D), c.stream);
    d2h(p, F.p.p, size_t(F.n_nodes), c.stream);
    return FSI_OK;
  });
}

fsi_status fsi_time_step(fsi_ctx* ctx, const fsi_newton_opts* opts, fsi_newton_info* info) {
  return guarded(ctx, [&]() -> fsi_status {
    fsi_ctx& c = *ctx;
    if (!c.fe) throw Error(FSI_ERR_STATE, "fsi_fe_setup must come first");
    fsi_newton_opts o;
    fsi_default_newton_opts(&o);
    if (opts) o = *opts;
    check_newton_opts(c, o);
    DevBuf dU;
    dU.alloc(sizeof(double) * size_t(c.N));
    HIP_TRY(hipMemsetAsync(dU.p, 0, sizeof(double) * size_t(c.N), c.stream));
    fsi_newton_info out{};
    const fsi_status st = newton_impl(c, o, dU.as<double>(), out);
    if (info) *info = out;
    if (st == FSI_OK) fe_advance(c, dU.as<double>());
    return st;
  });
}

}  // extern "C"
