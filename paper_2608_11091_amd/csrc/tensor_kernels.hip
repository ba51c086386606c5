// Khatri-Rao reductions, flat reductions and layout kernels.
#include "kernels.hpp"

namespace tk {

namespace {

struct Dims4 {
  int v[kMaxD];
};

constexpr int KRP_NT = 256;
constexpr int KRP_ZMAX = 128;

// One workgroup per (column l, task).  M_j[:, l] is staged in LDS; threads
// split the contraction over the non-free multi-index and combine partial
// sums in a fixed order (bitwise reproducible).
template <typename T>
__global__ __launch_bounds__(KRP_NT) void krp_kernel(const KrpTask<T>* __restrict__ tasks, int m, Dims4 z,
                                                     int P, int S) {
  __shared__ T mv[kMaxD][KRP_ZMAX];
  __shared__ T part[KRP_NT];
  const int l = blockIdx.x;
  const KrpTask<T> tk_ = tasks[blockIdx.y];
  const int f = tk_.f, ldo = tk_.ldo;
  const int tid = threadIdx.x;
#pragma unroll
  for (int j = 0; j < kMaxD; ++j) {
    if (j >= m || j == f) continue;
    for (int i = tid; i < z.v[j]; i += KRP_NT) mv[j][i] = tk_.Mj[j][i + (size_t)l * tk_.ldm[j]];
  }
  __syncthreads();
  const T* Zl = tk_.Z + (size_t)l * P;
  double coef = tk_.scale * (tk_.coef ? *tk_.coef : 1.0);
  if (f >= 0) {
    const int zf = z.v[f];
    const int nparts = KRP_NT / zf;
    const int a = tid % zf, pp = tid / zf;
    const int O = P / zf;
    T acc = T(0);
    if (pp < nparts) {
      // strides of the row-major multi-index (loops over the fixed kMaxD
      // modes, unrolled, so that the index arrays stay in registers)
      int stride[kMaxD];
#pragma unroll
      for (int j = kMaxD - 1; j >= 0; --j) stride[j] = (j >= m - 1) ? 1 : stride[j + 1 < kMaxD ? j + 1 : j] * z.v[j + 1 < kMaxD ? j + 1 : j];
      int sf = 1;
#pragma unroll
      for (int j = 0; j < kMaxD; ++j)
        if (j == f) sf = stride[j];
      for (int o = pp; o < O; o += nparts) {
        int rem = o, row = a * sf;
        T prod = T(1);
#pragma unroll
        for (int j = kMaxD - 1; j >= 0; --j) {
          if (j >= m || j == f) continue;
          const int ij = rem % z.v[j];
          rem /= z.v[j];
          row += ij * stride[j];
          prod *= mv[j][ij];
        }
        acc += Zl[row] * prod;
      }
    }
    part[tid] = acc;
    __syncthreads();
    if (tid < zf) {
      T s = T(0);
      for (int q = 0; q < nparts; ++q) s += part[q * zf + tid];
      T* o = tk_.out + tid + (size_t)l * ldo;
      const T v = T(coef) * s;
      *o = tk_.accumulate ? *o + v : v;
    }
  } else {
    T acc = T(0);
    for (int e = tid; e < P; e += KRP_NT) {
      int rem = e;
      T prod = T(1);
#pragma unroll
      for (int j = kMaxD - 1; j >= 0; --j) {
        if (j >= m) continue;
        const int ij = rem % z.v[j];
        rem /= z.v[j];
        prod *= mv[j][ij];
      }
      acc += Zl[e] * prod;
    }
    __shared__ T red[KRP_NT / kWave];
    const T s = block_sum(acc, red);
    if (tid == 0) {
      T* o = tk_.out + (size_t)l * ldo;
      const T v = T(coef) * s;
      *o = tk_.accumulate ? *o + v : v;
    }
  }
}

template <typename T>
__global__ void sumsq_kernel(const T* __restrict__ base, size_t stride, size_t len, double* __restrict__ out) {
  __shared__ double red[4];
  const T* x = base + blockIdx.x * stride;
  double acc = 0.0;
  for (size_t e = threadIdx.x; e < len; e += blockDim.x) {
    const double v = double(x[e]);
    acc += v * v;
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

__global__ void weights_kernel(const double* coef, const double* sumsq, int n, double* w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] = fabs(coef ? coef[i] : 1.0) * sqrt(sumsq[i]);
}

// One workgroup per dot product; 16-byte loads, four independent
// accumulators per thread so that a wave keeps several loads in flight.
template <typename T> struct Vec16;
template <> struct Vec16<float> { using V = float4; static constexpr int W = 4; };
template <> struct Vec16<double> { using V = double2; static constexpr int W = 2; };

template <typename T>
__device__ __forceinline__ double vdot(const typename Vec16<T>::V& a, const typename Vec16<T>::V& b);
template <>
__device__ __forceinline__ double vdot<float>(const float4& a, const float4& b) {
  return double(a.x) * double(b.x) + double(a.y) * double(b.y) + double(a.z) * double(b.z) + double(a.w) * double(b.w);
}
template <>
__device__ __forceinline__ double vdot<double>(const double2& a, const double2& b) {
  return a.x * b.x + a.y * b.y;
}

constexpr int DOT_NT = 1024;

template <typename T>
__global__ __launch_bounds__(DOT_NT) void dot_kernel(const T* const* xs, const T* const* ys, size_t len, double scale,
                                                     double* out) {
  __shared__ double red[DOT_NT / kWave];
  using V = typename Vec16<T>::V;
  constexpr int W = Vec16<T>::W;
  const T* x = xs[blockIdx.x];
  const T* y = ys[blockIdx.x];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  size_t head = 0;
  if (((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) & 15) == 0) {
    const V* xv = reinterpret_cast<const V*>(x);
    const V* yv = reinterpret_cast<const V*>(y);
    const size_t nv = len / W;
    size_t e = threadIdx.x;
    for (; e + 3 * DOT_NT < nv; e += 4 * DOT_NT) {
      const V x0 = xv[e], x1 = xv[e + DOT_NT], x2 = xv[e + 2 * DOT_NT], x3 = xv[e + 3 * DOT_NT];
      const V y0 = yv[e], y1 = yv[e + DOT_NT], y2 = yv[e + 2 * DOT_NT], y3 = yv[e + 3 * DOT_NT];
      a0 += vdot<T>(x0, y0);
      a1 += vdot<T>(x1, y1);
      a2 += vdot<T>(x2, y2);
      a3 += vdot<T>(x3, y3);
    }
    for (; e < nv; e += DOT_NT) a0 += vdot<T>(xv[e], yv[e]);
    head = nv * W;
  }
  for (size_t e = head + threadIdx.x; e < len; e += DOT_NT) a1 += double(x[e]) * double(y[e]);
  const double sum = block_sum((a0 + a1) + (a2 + a3), red);
  if (threadIdx.x == 0) out[blockIdx.x] = scale * sum;
}

template <typename T>
__global__ void scale_kernel(const T* __restrict__ x, T* __restrict__ y, size_t len, double scale, const double* num,
                             const double* den) {
  double a = scale;
  if (num) a *= *num;
  if (den) {
    // a norm as denominator: zero (a breakdown) or non-finite gives a zero
    // result instead of inf / NaN
    const double dv = *den;
    a = (dv > 0.0 && dv < INFINITY) ? a / dv : 0.0;
  }
  const T at = T(a);
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < len; e += (size_t)gridDim.x * blockDim.x)
    y[e] = at * x[e];
}

template <typename T>
__global__ void fill_kernel(T* y, size_t len, T v) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < len; e += (size_t)gridDim.x * blockDim.x)
    y[e] = v;
}

// Counts the non-finite entries of every task's array into *count (zeroed by
// the caller); one atomic per non-finite entry found.
__global__ void nonfinite_kernel(const double* const* xs, const size_t* lens, int ntasks, int* count) {
  const int t = blockIdx.y;
  if (t >= ntasks) return;
  const double* x = xs[t];
  const size_t len = lens[t];
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < len; e += (size_t)gridDim.x * blockDim.x)
    if (!isfinite(x[e])) atomicAdd(count, 1);
}

template <typename A, typename B>
__global__ void cast_kernel(const A* __restrict__ x, B* __restrict__ y, size_t len) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < len; e += (size_t)gridDim.x * blockDim.x)
    y[e] = B(x[e]);
}

template <typename A, typename B>
__global__ void cast_multi_kernel(CastSet<A, B> set) {
  const A* x = nullptr;
  B* y = nullptr;
  size_t len = 0;
#pragma unroll
  for (int k = 0; k < kMaxD; ++k)
    if (k == int(blockIdx.y)) {
      x = set.x[k];
      y = set.y[k];
      len = set.len[k];
    }
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < len; e += (size_t)gridDim.x * blockDim.x)
    y[e] = B(x[e]);
}

template <typename T>
__global__ void core_recap_kernel(const T* __restrict__ src, Dims4 sd, Dims4 sv, T* __restrict__ dst, Dims4 dd,
                                  int d, size_t total) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    size_t rem = e, so = 0, sstr = 1;
    bool inside = true;
    for (int k = d - 1; k >= 0; --k) {
      const int ik = int(rem % dd.v[k]);
      rem /= dd.v[k];
      if (ik >= sv.v[k] || ik >= sd.v[k]) inside = false;
      so += size_t(ik) * sstr;
      sstr *= sd.v[k];
    }
    dst[e] = inside ? src[so] : T(0);
  }
}

// core_recap_kernel without a view limit, and the zero-sum fix-up of the
// same step: when *tot <= *zthr (or NaN) the core is zero, every factor is
// e_1 in its first column and every rank is 1.
template <typename T>
__global__ void core_recap_fixup_kernel(const T* __restrict__ src, Dims4 sd, T* __restrict__ dst, Dims4 dd, int d,
                                        size_t total, const double* tot, const double* zthr, Dims4 nn, int rc,
                                        T* U0, T* U1, T* U2, T* U3, int* rank) {
  const bool zs = !(*tot > *zthr);
  const size_t tid = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const size_t nth = (size_t)gridDim.x * blockDim.x;
  for (size_t e = tid; e < total; e += nth) {
    size_t rem = e, so = 0, sstr = 1;
    bool inside = true;
    for (int k = d - 1; k >= 0; --k) {
      const int ik = int(rem % dd.v[k]);
      rem /= dd.v[k];
      if (ik >= sd.v[k]) inside = false;
      so += size_t(ik) * sstr;
      sstr *= sd.v[k];
    }
    dst[e] = (inside && !zs) ? src[so] : T(0);
  }
  if (!zs) return;
  T* Us[4] = {U0, U1, U2, U3};
  for (int k = 0; k < d; ++k) {
    const size_t len = size_t(nn.v[k]) * rc;
    for (size_t e = tid; e < len; e += nth) Us[k][e] = (e == 0) ? T(1) : T(0);
  }
  if (tid < size_t(d)) rank[tid] = 1;
}

template <typename T>
__global__ void mat_recap_kernel(const T* __restrict__ src, int lds, int rs, int cs, T* __restrict__ dst, int ldd,
                                 int rd, int cd) {
  const size_t total = size_t(rd) * cd;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = int(e % rd), j = int(e / rd);
    dst[i + size_t(j) * ldd] = (i < rs && j < cs) ? src[i + size_t(j) * lds] : T(0);
  }
}

__global__ void sketch_width_kernel(const int* rt, int d, int p, int cap, int force, int* s_out) {
  if (threadIdx.x != 0) return;
  if (force >= 0) {
    *s_out = force;
    return;
  }
  int est = 0;
  for (int k = 0; k < d; ++k) {
    const int v = rt[k] < 0 ? cap + p : rt[k] + p;
    est = v > est ? v : est;
  }
  *s_out = est < cap + p ? est : cap + p;
}

__global__ void gram_prep_kernel(const int* const* ranks, int nb, int d, int rmax, double* enable, int* nact,
                                 int* skip_small, int* skip_big) {
  const int k = threadIdx.x;
  if (k >= d) return;
  int R = 0;
  for (int b = 0; b < nb; ++b) R += ranks[b][k];
  enable[k] = R <= rmax ? 1.0 : 0.0;
  nact[k] = R <= rmax ? R : -1;
  if (skip_small) skip_small[k] = R > rmax;
  if (skip_big) skip_big[k] = R <= rmax;
}

// Compacts the lower triangle of a padded block Gram: compact index i maps to
// (block b, local a) through the prefix sums of the block ranks.
template <typename T>
__global__ void gram_compact_kernel(const T* __restrict__ padded, int ldp, const int* const* ranks, int nb, int rc,
                                    const int* nact, T* __restrict__ compact, int ldc, size_t msp, size_t msc) {
  const int k = blockIdx.y;
  const int R = nact[k];
  if (R <= 0) return;
  const T* P = padded + k * msp;
  T* C = compact + k * msc;
  const size_t total = size_t(R) * R;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = int(e % R), j = int(e / R);
    if (i < j) continue;
    int bi = 0, oi = i;
    while (oi >= ranks[bi][k]) { oi -= ranks[bi][k]; ++bi; }
    int bj = 0, oj = j;
    while (oj >= ranks[bj][k]) { oj -= ranks[bj][k]; ++bj; }
    C[i + size_t(j) * ldc] = P[(bi * rc + oi) + size_t(bj * rc + oj) * ldp];
  }
}

inline unsigned grid_for(size_t n, unsigned nt = 256) {
  size_t g = (n + nt - 1) / nt;
  return (unsigned)(g < 2048 ? (g == 0 ? 1 : g) : 2048);
}

}  // namespace

template <typename T>
void krp_reduce(const KrpTask<T>* tasks_d, int ntasks, int m, const int* z, int P, int S, hipStream_t st) {
  if (ntasks <= 0 || S <= 0) return;
  Dims4 zz{};
  for (int j = 0; j < m; ++j) {
    zz.v[j] = z[j];
    TK_CHECK(z[j] <= KRP_ZMAX, kErrUnsupported, "Khatri-Rao reduction: mode size above 128");
  }
  timer_begin(kKcKrp, st);
  hipLaunchKernelGGL((krp_kernel<T>), dim3(S, ntasks), dim3(KRP_NT), 0, st, tasks_d, m, zz, P, S);
  TK_LAUNCH_CHECK();
  timer_end(kKcKrp, st);
}

template <typename T>
void sumsq_batched(const T* base, size_t stride, size_t len, int n, double* out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((sumsq_kernel<T>), dim3(n), dim3(256), 0, st, base, stride, len, out);
  TK_LAUNCH_CHECK();
}

void block_weights(const double* coef, const double* sumsq, int n, double* w, hipStream_t st) {
  hipLaunchKernelGGL(weights_kernel, dim3(ceil_div(n, 64)), dim3(64), 0, st, coef, sumsq, n, w);
  TK_LAUNCH_CHECK();
}

template <typename T>
void dot_batched(const T* const* xs, const T* const* ys, size_t len, int n, double scale, double* out,
                 hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL((dot_kernel<T>), dim3(n), dim3(DOT_NT), 0, st, xs, ys, len, scale, out);
  TK_LAUNCH_CHECK();
}

template <typename T>
void scale_copy(const T* x, T* y, size_t len, double scale, const double* num, const double* den, hipStream_t st) {
  hipLaunchKernelGGL((scale_kernel<T>), dim3(grid_for(len)), dim3(256), 0, st, x, y, len, scale, num, den);
  TK_LAUNCH_CHECK();
}

void count_nonfinite(const double* const* xs, const size_t* lens, int ntasks, size_t maxlen, int* count,
                     hipStream_t st) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(fill_kernel<int>, dim3(1), dim3(64), 0, st, count, size_t(1), 0);
  TK_LAUNCH_CHECK();
  hipLaunchKernelGGL(nonfinite_kernel, dim3(std::min<unsigned>(grid_for(maxlen), 256u), ntasks), dim3(256), 0, st, xs,
                     lens, ntasks, count);
  TK_LAUNCH_CHECK();
}

template <typename T>
void fill(T* y, size_t len, T v, hipStream_t st) {
  if (len == 0) return;
  hipLaunchKernelGGL((fill_kernel<T>), dim3(grid_for(len)), dim3(256), 0, st, y, len, v);
  TK_LAUNCH_CHECK();
}

template <typename A, typename B>
void cast_multi(const CastSet<A, B>& set, hipStream_t st) {
  TK_CHECK(set.count >= 0 && set.count <= kMaxD, kErrInvalidArg, "cast_multi: too many buffers");
  size_t mx = 0;
  for (int k = 0; k < set.count; ++k) mx = std::max(mx, set.len[k]);
  if (mx == 0) return;
  hipLaunchKernelGGL((cast_multi_kernel<A, B>), dim3(grid_for(mx), set.count), dim3(256), 0, st, set);
  TK_LAUNCH_CHECK();
}

template <typename A, typename B>
void cast_copy(const A* x, B* y, size_t len, hipStream_t st) {
  if (len == 0) return;
  hipLaunchKernelGGL((cast_kernel<A, B>), dim3(grid_for(len)), dim3(256), 0, st, x, y, len);
  TK_LAUNCH_CHECK();
}

template <typename T>
void core_recap(const T* src, const int* sd, const int* sv, T* dst, const int* dd, int d, hipStream_t st) {
  Dims4 a{}, v{}, b{};
  size_t total = 1;
  for (int k = 0; k < d; ++k) {
    a.v[k] = sd[k];
    v.v[k] = sv ? sv[k] : sd[k];
    b.v[k] = dd[k];
    total *= size_t(dd[k]);
  }
  hipLaunchKernelGGL((core_recap_kernel<T>), dim3(grid_for(total)), dim3(256), 0, st, src, a, v, dst, b, d, total);
  TK_LAUNCH_CHECK();
}

template <typename T>
void core_recap_fixup(const T* src, const int* sd, T* dst, const int* dd, int d, const double* total,
                      const double* zthr, const int* n, int rc, T* const* U, int* rank, hipStream_t st) {
  Dims4 a{}, b{}, nn{};
  T* uu[4] = {nullptr, nullptr, nullptr, nullptr};
  size_t len = 1, mx = 1;
  for (int k = 0; k < d; ++k) {
    a.v[k] = sd[k];
    b.v[k] = dd[k];
    nn.v[k] = n[k];
    uu[k] = U[k];
    len *= size_t(dd[k]);
    mx = std::max(mx, size_t(n[k]) * rc);
  }
  hipLaunchKernelGGL((core_recap_fixup_kernel<T>), dim3(grid_for(std::max(len, mx))), dim3(256), 0, st, src, a, dst,
                     b, d, len, total, zthr, nn, rc, uu[0], uu[1], uu[2], uu[3], rank);
  TK_LAUNCH_CHECK();
}

template <typename T>
void mat_recap(const T* src, int ld_src, int rows_src, int cols_src, T* dst, int ld_dst, int rows_dst, int cols_dst,
               hipStream_t st) {
  const size_t total = size_t(rows_dst) * cols_dst;
  if (total == 0) return;
  hipLaunchKernelGGL((mat_recap_kernel<T>), dim3(grid_for(total)), dim3(256), 0, st, src, ld_src, rows_src, cols_src,
                     dst, ld_dst, rows_dst, cols_dst);
  TK_LAUNCH_CHECK();
}

void gram_prep(const int* const* ranks, int nb, int d, int rmax, double* enable, int* nact, hipStream_t st,
               int* skip_small, int* skip_big) {
  hipLaunchKernelGGL(gram_prep_kernel, dim3(1), dim3(64), 0, st, ranks, nb, d, rmax, enable, nact, skip_small,
                     skip_big);
  TK_LAUNCH_CHECK();
}

template <typename T>
void gram_compact(const T* padded, int ldp, const int* const* ranks, int nb, int d, int rc, const int* nact,
                  T* compact, int ldc, size_t mode_stride_p, size_t mode_stride_c, hipStream_t st) {
  hipLaunchKernelGGL((gram_compact_kernel<T>), dim3(64, d), dim3(256), 0, st, padded, ldp, ranks, nb, rc, nact,
                     compact, ldc, mode_stride_p, mode_stride_c);
  TK_LAUNCH_CHECK();
}

void sketch_width(const int* rt, int d, int p, int cap, int force, int* s_out, hipStream_t st) {
  hipLaunchKernelGGL(sketch_width_kernel, dim3(1), dim3(64), 0, st, rt, d, p, cap, force, s_out);
  TK_LAUNCH_CHECK();
}

#define TK_INST(T)                                                                                         \
  template void krp_reduce<T>(const KrpTask<T>*, int, int, const int*, int, int, hipStream_t);             \
  template void sumsq_batched<T>(const T*, size_t, size_t, int, double*, hipStream_t);                     \
  template void dot_batched<T>(const T* const*, const T* const*, size_t, int, double, double*, hipStream_t); \
  template void scale_copy<T>(const T*, T*, size_t, double, const double*, const double*, hipStream_t);    \
  template void fill<T>(T*, size_t, T, hipStream_t);                                                       \
  template void core_recap<T>(const T*, const int*, const int*, T*, const int*, int, hipStream_t);         \
  template void mat_recap<T>(const T*, int, int, int, T*, int, int, int, hipStream_t);                     \
  template void core_recap_fixup<T>(const T*, const int*, T*, const int*, int, const double*, const double*,    \
                                    const int*, int, T* const*, int*, hipStream_t);                     \
  template void gram_compact<T>(const T*, int, const int* const*, int, int, int, const int*, T*, int, size_t, \
                                size_t, hipStream_t);
TK_INST(double)
TK_INST(float)
#undef TK_INST
template void cast_copy<double, float>(const double*, float*, size_t, hipStream_t);
template void cast_multi<double, float>(const CastSet<double, float>&, hipStream_t);
template void cast_multi<float, double>(const CastSet<float, double>&, hipStream_t);
template void cast_copy<float, double>(const float*, double*, size_t, hipStream_t);
template void fill<int>(int*, size_t, int, hipStream_t);

}  // namespace tk
