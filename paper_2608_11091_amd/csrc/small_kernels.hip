// Small bookkeeping kernels: coefficient gathering, zero-sum fix-up,
// accumulation, vector sums and the per-iteration status record.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <map>
#include <mutex>

#include "kernels.hpp"

namespace tk {

namespace {

__global__ void gather_coef_kernel(const double* const* cptr, const double* cscale, int nb, double* coef) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nb) coef[b] = cscale[b] * (cptr[b] ? *cptr[b] : 1.0);
}

__global__ void zero_threshold_kernel(const double* w, int nb, double tol, double* zthr) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += w[b];
  s *= tol;
  *zthr = s * s;
}

__global__ __launch_bounds__(256) void coef_weights_threshold_kernel(const double* const* cptr, const double* cscale,
                                                                     const double* sumsq, int nb, double tol,
                                                                     double* coef, double* w, double* zthr) {
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    const double c = cscale[b] * (cptr[b] ? *cptr[b] : 1.0);
    coef[b] = c;
    w[b] = fabs(c) * sqrt(sumsq[b]);
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += w[b];
  s *= tol;
  *zthr = s * s;
}

template <typename T>
__global__ void zero_sum_fixup_kernel(const double* total, const double* zthr, int d, int n0, int n1, int n2, int n3, int rc, T* U0, T* U1,
                                      T* U2, T* U3, T* core, size_t core_len, int* rank) {
  if (*total > *zthr) return;
  const int ns[4] = {n0, n1, n2, n3};
  T* Us[4] = {U0, U1, U2, U3};
  const size_t tid = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const size_t nth = (size_t)gridDim.x * blockDim.x;
  for (int k = 0; k < d; ++k) {
    const size_t len = size_t(ns[k]) * rc;
    for (size_t e = tid; e < len; e += nth) Us[k][e] = (e == 0) ? T(1) : T(0);
  }
  for (size_t e = tid; e < core_len; e += nth) core[e] = T(0);
  if (tid < size_t(d)) rank[tid] = 1;
}

template <typename T>
__global__ void mat_axpy_kernel(const T* X, int ldx, T* Y, int ldy, int rows, int cols) {
  const size_t total = size_t(rows) * cols;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = int(e % rows), j = int(e / rows);
    Y[i + size_t(j) * ldy] += X[i + size_t(j) * ldx];
  }
}

template <typename T>
__global__ void sum_vectors_kernel(const T* base, size_t stride, int nb, int len, double* out) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= len) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += double(base[b * stride + l]);
  out[l] = s;
}

template <typename T>
__global__ void zero_cols_from_kernel(T* A, int ld, int rows, int cols, const int* from_dev) {
  const int from = max(*from_dev, 0);
  const size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const size_t len = size_t(rows) * cols;
  if (e >= len) return;
  const int c = int(e / rows), r = int(e % rows);
  if (c >= from) A[r + size_t(c) * ld] = T(0);
}

// The sketch width s = min(max_k (rt_k + p), cap + p), or force when force >= 0
// (rt_k < 0: the mode's rule was skipped, counted as cap).
__device__ inline int width_from_ranks(const int* rt, int d, int p, int cap, int force) {
  if (force >= 0) return force;
  int est = 0;
  for (int k = 0; k < d; ++k) {
    const int v = rt[k] < 0 ? cap + p : rt[k] + p;
    est = v > est ? v : est;
  }
  return est < cap + p ? est : cap + p;
}

// Zeroes basis columns (part < d) and core indices (part == d) at or beyond
// the width s; s comes from *s_dev, or from the ranks rt when rt is given (and
// is then written to *s_out by one thread).
template <typename T>
__global__ void zero_beyond_width_kernel(WidthZero<T> a, int d, int sc, const int* s_dev, const int* rt, int p,
                                         int cap, int force, int* s_out) {
  int s;
  if (rt) {
    s = width_from_ranks(rt, d, p, cap, force);
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *s_out = s;
  } else {
    s = *s_dev;
  }
  s = max(s, 0);
  const int part = blockIdx.y;
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  const size_t e0 = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (part < d) {
    T* U = nullptr;
    int n = 1;
#pragma unroll
    for (int k = 0; k < kMaxD; ++k)
      if (k == part) {
        U = a.U[k];
        n = a.n[k];
      }
    const size_t len = size_t(n) * sc;
    for (size_t e = e0; e < len; e += stride)
      if (int(e / n) >= s) U[e] = T(0);
  } else {
    size_t len = 1;
    for (int k = 0; k < d; ++k) len *= size_t(sc);
    for (size_t e = e0; e < len; e += stride) {
      size_t rem = e;
      bool out = false;
      for (int k = 0; k < d; ++k) {
        out = out || int(rem % sc) >= s;
        rem /= sc;
      }
      if (out) a.core[e] = T(0);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void lincomb_kernel(T* const* y, const T* const* x, const double* const* c,
                                                      const double* s, const size_t* len, int ldx, int nx,
                                                      int accumulate) {
  __shared__ double cf[kLincombMax];
  __shared__ const T* xp[kLincombMax];
  const int t = blockIdx.y;
  for (int j = threadIdx.x; j < nx; j += blockDim.x) {
    cf[j] = s[j] * (c[j] ? *c[j] : 1.0);
    xp[j] = x[size_t(t) * ldx + j];
  }
  __syncthreads();
  T* yt = y[t];
  const size_t n = len[t];
  const size_t step = (size_t)gridDim.x * blockDim.x;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += step) {
    double acc = accumulate ? double(yt[e]) : 0.0;
    for (int j = 0; j < nx; ++j) acc += cf[j] * double(xp[j][e]);
    yt[e] = T(acc);
  }
}

template <typename T>
__global__ void exp_scale_rows_kernel(const ExpScaleTask<T>* tasks, int n, int cols) {
  const ExpScaleTask<T> tk_ = tasks[blockIdx.y];
  const size_t len = size_t(n) * cols;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < len; e += (size_t)gridDim.x * blockDim.x) {
    const int i = int(e % n);
    tk_.out[e] = T(exp(-tk_.t * (double(tk_.lam[i]) - *tk_.shift))) * tk_.in[e];
  }
}

template <typename T>
__global__ void expsum_shift_kernel(const T* l0, const T* l1, const T* l2, const T* l3, int n0, int n1, int n2,
                                    int n3, int d, int q, double eta, double* lmin, double* coef) {
  __shared__ double m[kMaxD];
  const T* ls[kMaxD] = {l0, l1, l2, l3};
  const int ns[kMaxD] = {n0, n1, n2, n3};
  if (threadIdx.x < d) {
    const int k = threadIdx.x;
    double v = double(ls[k][0]);
    for (int i = 1; i < ns[k]; ++i) v = fmin(v, double(ls[k][i]));
    m[k] = v;
    lmin[k] = v;
  }
  __syncthreads();
  double sum = 0.0;
  for (int k = 0; k < d; ++k) sum += m[k];
  for (int h = threadIdx.x; h < 2 * q + 1; h += blockDim.x) {
    const double t = exp((h - q) * eta);
    coef[h] = eta * t * exp(-t * sum);
  }
}

template <typename T>
__global__ void strided_gather_kernel(const T* src, size_t stride, int n, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = double(src[size_t(i) * stride]);
}

__global__ void ints_at_least_kernel(const int* src, int* dst, int n, int lo) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = max(src[i], lo);
}

__global__ void copy_ints_kernel(const int* src, int* dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__global__ void vec_sqrt_kernel(const double* src, double* dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = sqrt(src[i]);
}

// Column k of the Arnoldi Hessenberg matrix (Alg. 1): h_0..h_k, then
// h_{k+1,k} = sqrt(norm2), then zeros up to len.
__global__ void hess_column_kernel(const double* h, int nh, const double* norm2, double* col, int len) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) col[i] = i < nh ? h[i] : (i == nh ? sqrt(fmax(*norm2, 0.0)) : 0.0);
}

// v = (*beta) e_1 of length len.
__global__ void scaled_unit_kernel(const double* beta, double* v, int len) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) v[i] = i == 0 ? *beta : 0.0;
}

__global__ void iter_status_kernel(const double* sumsq2, const int* ls_flags, const double* res_k, const int* rank,
                                   int d, double bd_tol, double* omega, IterStatus* out) {
  if (threadIdx.x != 0) return;
  const double wn = sqrt(sumsq2[0]);
  const double om = sqrt(sumsq2[1]);
  *omega = om;
  IterStatus s;
  s.breakdown_ls = ls_flags[0];
  s.converged = ls_flags[1];
  s.breakdown_w = (om <= bd_tol * wn) ? 1 : 0;
  s.pad = 0;
  for (int k = 0; k < kMaxD; ++k) s.rank[k] = k < d ? rank[k] : 0;
  s.res = *res_k;
  s.omega = om;
  *out = s;
}

inline unsigned gsz(size_t n) {
  size_t g = (n + 255) / 256;
  return (unsigned)(g == 0 ? 1 : (g > 1024 ? 1024 : g));
}

}  // namespace

void gather_coef(const double* const* cptr, const double* cscale, int nb, double* coef, hipStream_t st) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(gather_coef_kernel, dim3(ceil_div(nb, 64)), dim3(64), 0, st, cptr, cscale, nb, coef);
  TK_LAUNCH_CHECK();
}

void zero_threshold(const double* w, int nb, double tol, double* zthr, hipStream_t st) {
  hipLaunchKernelGGL(zero_threshold_kernel, dim3(1), dim3(64), 0, st, w, nb, tol, zthr);
  TK_LAUNCH_CHECK();
}

template <typename T>
void zero_sum_fixup(const double* total, const double* zthr, int d, const int* n, int rc, T* const* U, T* core,
                    size_t core_len, int* rank, hipStream_t st) {
  int nn[4] = {0, 0, 0, 0};
  T* uu[4] = {nullptr, nullptr, nullptr, nullptr};
  for (int k = 0; k < d; ++k) {
    nn[k] = n[k];
    uu[k] = U[k];
  }
  hipLaunchKernelGGL((zero_sum_fixup_kernel<T>), dim3(gsz(core_len)), dim3(256), 0, st, total, zthr, d, nn[0], nn[1], nn[2],
                     nn[3], rc, uu[0], uu[1], uu[2], uu[3], core, core_len, rank);
  TK_LAUNCH_CHECK();
}

template <typename T>
void mat_axpy(const T* X, int ldx, T* Y, int ldy, int rows, int cols, hipStream_t st) {
  hipLaunchKernelGGL((mat_axpy_kernel<T>), dim3(gsz(size_t(rows) * cols)), dim3(256), 0, st, X, ldx, Y, ldy, rows, cols);
  TK_LAUNCH_CHECK();
}

template <typename T>
void sum_vectors(const T* base, size_t stride, int nb, int len, double* out, hipStream_t st) {
  hipLaunchKernelGGL((sum_vectors_kernel<T>), dim3(ceil_div(len, 256)), dim3(256), 0, st, base, stride, nb, len, out);
  TK_LAUNCH_CHECK();
}

template <typename T>
void zero_cols_from(T* A, int ld, int rows, int cols, const int* from_dev, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL((zero_cols_from_kernel<T>), dim3(gsz(size_t(rows) * cols)), dim3(256), 0, st, A, ld, rows, cols,
                     from_dev);
  TK_LAUNCH_CHECK();
}

template <typename T>
void zero_beyond_width(const WidthZero<T>& a, int d, int sc, const int* s_dev, hipStream_t st) {
  size_t mx = 1;
  for (int k = 0; k < d; ++k) mx *= size_t(sc);
  for (int k = 0; k < d; ++k) mx = std::max(mx, size_t(a.n[k]) * sc);
  const unsigned gx = unsigned(std::min<size_t>((mx + 255) / 256, 1024));
  const unsigned parts = a.core ? d + 1 : d;
  hipLaunchKernelGGL((zero_beyond_width_kernel<T>), dim3(gx, parts), dim3(256), 0, st, a, d, sc, s_dev, nullptr, 0,
                     0, 0, nullptr);
  TK_LAUNCH_CHECK();
}

template <typename T>
void width_and_zero(const WidthZero<T>& a, int d, int sc, const int* rt, int p, int cap, int force, int* s_out,
                    hipStream_t st) {
  size_t mx = 1;
  for (int k = 0; k < d; ++k) mx *= size_t(sc);
  for (int k = 0; k < d; ++k) mx = std::max(mx, size_t(a.n[k]) * sc);
  const unsigned gx = unsigned(std::min<size_t>((mx + 255) / 256, 1024));
  const unsigned parts = a.core ? d + 1 : d;
  hipLaunchKernelGGL((zero_beyond_width_kernel<T>), dim3(gx, parts), dim3(256), 0, st, a, d, sc, nullptr, rt, p, cap,
                     force, s_out);
  TK_LAUNCH_CHECK();
}

void coef_weights_threshold(const double* const* cptr, const double* cscale, const double* sumsq, int nb, double tol,
                            double* coef, double* w, double* zthr, hipStream_t st) {
  hipLaunchKernelGGL(coef_weights_threshold_kernel, dim3(1), dim3(256), 0, st, cptr, cscale, sumsq, nb, tol, coef, w,
                     zthr);
  TK_LAUNCH_CHECK();
}


hipStream_t side_stream(int which) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, hipStream_t> streams;
  int dev = 0;
  TK_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  const auto key = std::make_pair(dev, which);
  auto it = streams.find(key);
  if (it != streams.end()) return it->second;
  hipStream_t s = nullptr;
  TK_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  streams[key] = s;
  return s;
}

template <typename T>
void lincomb(T* const* y, const T* const* x, const double* const* c, const double* s, const size_t* len,
             int ntasks, int nx, size_t maxlen, int accumulate, int limit, hipStream_t st) {
  TK_CHECK(nx <= kLincombMax, kErrUnsupported, "linear combination of more than 128 arrays");
  const int na = std::max(0, std::min(nx, limit));
  if (ntasks <= 0 || maxlen == 0) return;
  const size_t want = (maxlen + 1023) / 1024;  // about 4 elements per thread
  const int blocks = int(want < 1024 ? want : 1024);
  hipLaunchKernelGGL((lincomb_kernel<T>), dim3(blocks, ntasks), dim3(256), 0, st, y, x, c, s, len, nx, na,
                     accumulate);
  TK_LAUNCH_CHECK();
}

template <typename T>
void exp_scale_rows(const ExpScaleTask<T>* tasks_d, int ntasks, int n, int cols, hipStream_t st) {
  if (ntasks <= 0 || n <= 0 || cols <= 0) return;
  const size_t len = size_t(n) * cols;
  const size_t want = (len + 255) / 256;
  const int blocks = int(want < 256 ? want : 256);
  hipLaunchKernelGGL((exp_scale_rows_kernel<T>), dim3(blocks, ntasks), dim3(256), 0, st, tasks_d, n, cols);
  TK_LAUNCH_CHECK();
}

template <typename T>
void expsum_shift(const T* const* lam, const int* n, int d, int q, double eta, double* lmin, double* coef,
                  hipStream_t st) {
  TK_CHECK(d >= 1 && d <= kMaxD, kErrInvalidArg, "expsum_shift: order");
  const T* l[kMaxD] = {lam[0], d > 1 ? lam[1] : lam[0], d > 2 ? lam[2] : lam[0], d > 3 ? lam[3] : lam[0]};
  int nn[kMaxD] = {n[0], d > 1 ? n[1] : 1, d > 2 ? n[2] : 1, d > 3 ? n[3] : 1};
  hipLaunchKernelGGL((expsum_shift_kernel<T>), dim3(1), dim3(256), 0, st, l[0], l[1], l[2], l[3], nn[0], nn[1],
                     nn[2], nn[3], d, q, eta, lmin, coef);
  TK_LAUNCH_CHECK();
}

template <typename T>
void strided_gather(const T* src, size_t stride, int n, double* out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((strided_gather_kernel<T>), dim3(ceil_div(n, 256)), dim3(256), 0, st, src, stride, n, out);
  TK_LAUNCH_CHECK();
}

void ints_at_least(const int* src, int* dst, int n, int lo, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(ints_at_least_kernel, dim3(1), dim3(64), 0, st, src, dst, n, lo);
  TK_LAUNCH_CHECK();
}

void copy_ints(const int* src, int* dst, int n, hipStream_t st) {
  hipLaunchKernelGGL(copy_ints_kernel, dim3(1), dim3(64), 0, st, src, dst, n);
  TK_LAUNCH_CHECK();
}

void vec_sqrt(const double* src, double* dst, int n, hipStream_t st) {
  hipLaunchKernelGGL(vec_sqrt_kernel, dim3(1), dim3(64), 0, st, src, dst, n);
  TK_LAUNCH_CHECK();
}

void hess_column(const double* h, int nh, const double* norm2, double* col, int len, hipStream_t st) {
  hipLaunchKernelGGL(hess_column_kernel, dim3(ceil_div(len, 64)), dim3(64), 0, st, h, nh, norm2, col, len);
  TK_LAUNCH_CHECK();
}

void scaled_unit(const double* beta, double* v, int len, hipStream_t st) {
  hipLaunchKernelGGL(scaled_unit_kernel, dim3(ceil_div(len, 64)), dim3(64), 0, st, beta, v, len);
  TK_LAUNCH_CHECK();
}

void iter_status(const double* sumsq2, const int* ls_flags, const double* res_k, const int* rank, int d, double bd_tol,
                 double* omega, IterStatus* out, hipStream_t st) {
  hipLaunchKernelGGL(iter_status_kernel, dim3(1), dim3(64), 0, st, sumsq2, ls_flags, res_k, rank, d, bd_tol, omega, out);
  TK_LAUNCH_CHECK();
}

// ---- launch counter and empty-kernel latency
namespace {
std::atomic<int64_t> g_launches{0};
__global__ void empty_kernel() {}
}  // namespace

void count_launch() { g_launches.fetch_add(1, std::memory_order_relaxed); }
int64_t launch_count() { return g_launches.load(std::memory_order_relaxed); }

double empty_launch_us(int n, hipStream_t st) {
  TK_HIP(hipStreamSynchronize(st));
  const auto t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < n; ++i) hipLaunchKernelGGL(empty_kernel, dim3(1), dim3(64), 0, st);
  TK_HIP(hipGetLastError());
  TK_HIP(hipStreamSynchronize(st));
  const double us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
  return n > 0 ? us / n : 0.0;
}

// ---- kernel-class timers
namespace {
struct TimerState {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  double flops = 0.0;
  double bytes = 0.0;
};
TimerState g_timers[kKcCount];
}  // namespace

bool timer_on(int kind) { return kind >= 0 && kind < kKcCount && g_timers[kind].on; }

void timer_begin(int kind, hipStream_t st, double flops, double bytes) {
  if (!timer_on(kind)) return;
  g_timers[kind].flops += flops;
  g_timers[kind].bytes += bytes;
  hipEvent_t a, b;
  TK_HIP(hipEventCreate(&a));
  TK_HIP(hipEventCreate(&b));
  TK_HIP(hipEventRecord(a, st));
  g_timers[kind].ev.emplace_back(a, b);
}

void timer_end(int kind, hipStream_t st) {
  if (!timer_on(kind) || g_timers[kind].ev.empty()) return;
  TK_HIP(hipEventRecord(g_timers[kind].ev.back().second, st));
}

void timer_enable(int kind, bool on) {
  TimerState& t = g_timers[kind];
  for (auto& e : t.ev) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  t.ev.clear();
  t.flops = 0.0;
  t.bytes = 0.0;
  t.on = on;
}

void timer_read(int kind, int64_t* launches, double* total_ms, double* total_flops, double* total_bytes) {
  TimerState& t = g_timers[kind];
  double tot = 0.0;
  for (auto& e : t.ev) {
    TK_HIP(hipEventSynchronize(e.second));
    float ms = 0.f;
    TK_HIP(hipEventElapsedTime(&ms, e.first, e.second));
    tot += ms;
  }
  *launches = int64_t(t.ev.size());
  *total_ms = tot;
  *total_flops = t.flops;
  *total_bytes = t.bytes;
}

template void zero_sum_fixup<double>(const double*, const double*, int, const int*, int, double* const*, double*,
                                     size_t, int*, hipStream_t);
template void zero_sum_fixup<float>(const double*, const double*, int, const int*, int, float* const*, float*, size_t,
                                    int*, hipStream_t);
template void zero_cols_from<double>(double*, int, int, int, const int*, hipStream_t);
template void zero_beyond_width<double>(const WidthZero<double>&, int, int, const int*, hipStream_t);
template void zero_beyond_width<float>(const WidthZero<float>&, int, int, const int*, hipStream_t);
template void width_and_zero<double>(const WidthZero<double>&, int, int, const int*, int, int, int, int*, hipStream_t);
template void width_and_zero<float>(const WidthZero<float>&, int, int, const int*, int, int, int, int*, hipStream_t);
template void zero_cols_from<float>(float*, int, int, int, const int*, hipStream_t);
template void mat_axpy<double>(const double*, int, double*, int, int, int, hipStream_t);
template void mat_axpy<float>(const float*, int, float*, int, int, int, hipStream_t);
template void sum_vectors<double>(const double*, size_t, int, int, double*, hipStream_t);
template void sum_vectors<float>(const float*, size_t, int, int, double*, hipStream_t);
template void lincomb<double>(double* const*, const double* const*, const double* const*, const double*,
                              const size_t*, int, int, size_t, int, int, hipStream_t);
template void strided_gather<double>(const double*, size_t, int, double*, hipStream_t);
template void exp_scale_rows<double>(const ExpScaleTask<double>*, int, int, int, hipStream_t);
template void exp_scale_rows<float>(const ExpScaleTask<float>*, int, int, int, hipStream_t);
template void expsum_shift<double>(const double* const*, const int*, int, int, double, double*, double*, hipStream_t);
template void expsum_shift<float>(const float* const*, const int*, int, int, double, double*, double*, hipStream_t);

}  // namespace tk
