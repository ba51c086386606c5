// Shared definitions of the Tucker sGMRES HIP library (gfx950 / CDNA4).
//
// Data layout on the device (all buffers capacity-padded, zero beyond rank):
//   * a core of capacity rc per mode is row-major over (i_1..i_d), mode d
//     fastest, with strides rc^(d-1-k); entries with i_k >= r_k are zero;
//   * a factor U_k is n_k x rc column-major (ld = n_k); columns >= r_k are zero;
//   * ranks, sketch widths, coefficients and status flags live in device
//     memory, so an iteration never needs the host to know a rank.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

namespace tk {

constexpr int kMaxD = 4;
constexpr int kWave = 64;

// ---------------------------------------------------------------- errors
enum Status : int {
  kOk = 0,
  kNotConverged = 1,
  kBreakdown = 2,
  kRankFloor = 3,
  kErrInvalidArg = -1,
  kErrShape = -2,
  kErrCapacity = -3,
  kErrWorkspace = -4,
  kErrHip = -5,
  kErrNonFinite = -6,
  kErrUnsupported = -7,
};

void set_error(const std::string& msg);
const char* last_error();

struct Error {
  int code;
  std::string msg;
};

#define TK_HIP(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess)                                                         \
      throw ::tk::Error{::tk::kErrHip, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define TK_CHECK(cond, code, msg)                                                 \
  do {                                                                            \
    if (!(cond)) throw ::tk::Error{(code), (msg)};                                \
  } while (0)

// Every kernel launch of the library is followed by this check, which also
// counts the launch (for the benchmark's launch-latency floor).
void count_launch();
#define TK_LAUNCH_CHECK()   \
  do {                      \
    ::tk::count_launch();   \
    TK_HIP(hipGetLastError()); \
  } while (0)

// ---------------------------------------------------------------- workspace
// Bump allocator over the caller's workspace.  With a null base it only
// measures, so every entry point can report its exact workspace need by
// running its planning phase without data.
class Arena {
 public:
  Arena(void* base, size_t bytes) : base_(static_cast<char*>(base)), cap_(bytes) {}
  template <typename T>
  T* alloc(size_t count) {
    size_t off = (used_ + 255) & ~size_t(255);
    used_ = off + count * sizeof(T);
    peak_ = used_ > peak_ ? used_ : peak_;
    if (base_ == nullptr) return reinterpret_cast<T*>(uintptr_t(0x1000) + off);  // measuring only
    if (used_ > cap_) throw Error{kErrWorkspace, "workspace too small: need at least " + std::to_string(used_) + " bytes"};
    return reinterpret_cast<T*>(base_ + off);
  }
  // Bytes the workspace must hold (the high-water mark).
  size_t used() const { return peak_; }
  bool measuring() const { return base_ == nullptr; }
  // Scratch scopes: buffers allocated after mark() are handed out again after
  // rewind(); valid only for plans whose steps never run concurrently.  An
  // allocation that must outlive every scope (read by steps of several
  // scopes) is made after seal(), which moves past the high-water mark.
  size_t mark() const { return used_; }
  void rewind(size_t m) { used_ = m; }
  void seal() { used_ = peak_; }

 private:
  char* base_;
  size_t cap_;
  size_t used_ = 0;
  size_t peak_ = 0;
};

// ---------------------------------------------------------------- device helpers
// Wave-uniform read of one lane's value (v_readlane; `lane` must be uniform).
__device__ __forceinline__ float rdlane(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ double rdlane(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = unsigned(__builtin_amdgcn_readlane(int(b), lane));
  const unsigned hi = unsigned(__builtin_amdgcn_readlane(int(b >> 32), lane));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Cross-lane move inside a row of 16 lanes through the DPP network (a few
// cycles, no LDS crossbar).  CTRL: 0xB1 quad_perm[1,0,3,2], 0x4E
// quad_perm[2,3,0,1], 0x141 row_half_mirror, 0x140 row_mirror.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = unsigned(__builtin_amdgcn_update_dpp(0, int(b), CTRL, 0xF, 0xF, false));
  const unsigned hi = unsigned(__builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, 0xF, 0xF, false));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the 64 lanes of a wave (all lanes active); every lane gets the
// total.  Row sums of 16 lanes through DPP, then the four rows through
// readlane; fixed order, so deterministic.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  v += dpp_mov<0xB1>(v);
  v += dpp_mov<0x4E>(v);
  v += dpp_mov<0x141>(v);
  v += dpp_mov<0x140>(v);
  return (rdlane(v, 0) + rdlane(v, 16)) + (rdlane(v, 32) + rdlane(v, 48));
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
  T o = dpp_mov<0xB1>(v);
  v = o > v ? o : v;
  o = dpp_mov<0x4E>(v);
  v = o > v ? o : v;
  o = dpp_mov<0x141>(v);
  v = o > v ? o : v;
  o = dpp_mov<0x140>(v);
  v = o > v ? o : v;
  const T a = rdlane(v, 0), b = rdlane(v, 16), c = rdlane(v, 32), d = rdlane(v, 48);
  const T ab = a > b ? a : b, cd = c > d ? c : d;
  return ab > cd ? ab : cd;
}

// Block-wide sum for blockDim.x a multiple of 64; `red` holds >= nwaves values.
// Every thread gets the same result (fixed reduction order: deterministic).
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* red) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  T s = 0;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

// Optional HIP-event timing of one kernel class (for live roofline numbers):
// when enabled, launches of that class record an event pair on their stream.
enum KernelClass : int {
  kKcGemm = 0, kKcJacobi = 1, kKcQr = 2, kKcKrp = 3, kKcLs = 4, kKcEigVals = 5, kKcTikhonov = 6, kKcCount = 7
};
bool timer_on(int kind);
void timer_begin(int kind, hipStream_t st, double flops = 0.0, double bytes = 0.0);
void timer_end(int kind, hipStream_t st);
void timer_enable(int kind, bool on);
void timer_read(int kind, int64_t* launches, double* total_ms, double* total_flops, double* total_bytes);
// Kernel launches issued by the library since it was loaded.
int64_t launch_count();
// Microseconds per launch of an empty kernel, n launches back to back on st.
double empty_launch_us(int n, hipStream_t st);

inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
inline int64_t ipow(int64_t b, int e) {
  int64_t r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

}  // namespace tk
