// Grouped GEMM kernel on MFMA (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32).
//
// Tile: 64 x 64 outputs per workgroup of 256 threads (4 waves in a 2 x 2
// arrangement), each wave owning a 32 x 32 sub-tile = 2 x 2 MFMA 16x16
// accumulators so four independent MFMA chains hide the pipeline latency.
// K is staged through LDS in slabs of 32 (16 in the bf16 form) with global
// loads coalesced along the contiguous dimension of each operand; the alpha
// of a term is folded into the A slab while it is staged.
#include "gemm.hpp"
#include "kernels.hpp"

namespace tk {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Acc;
template <> struct Acc<double> { typedef d4 type; static constexpr bool f64 = true; };
template <> struct Acc<float> { typedef f4 type; static constexpr bool f64 = false; };

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// BF16 operand form (FP32 storage and accumulation): operands are rounded to
// bfloat16 (round to nearest even; NaN kept quiet) as they are staged, and
// multiplied on v_mfma_f32_16x16x16_bf16.  Lane l supplies rows / columns
// l % 16 and the four consecutive k values 4 (l / 16) .. 4 (l / 16) + 3.
typedef short s4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ unsigned short bf16_rne(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ f4 mfma_bf16(s4 a, s4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

constexpr int BM = 64, BN = 64, NT = 256;


// Split-K: the (term, K-slab) iteration space of a group is divided evenly
// over `splits` workgroups per output tile; each writes its partial tile and a
// second pass sums the partials in split order.  (Summing them in the last
// workgroup to arrive at a tile needs device-scope fences, whose L2
// write-back across the XCDs cost more than the second launch.)
template <typename T, bool TA, bool TB, bool BF = false>
__global__ __launch_bounds__(NT) void gemm_kernel(int M, int N, int K, int lda, int ldb, int ldc,
                                                  const GemmTerm<T>* __restrict__ terms,
                                                  const GemmGroup<T>* __restrict__ groups, double beta,
                                                  int splits, T* __restrict__ partial, int max_terms) {
  static_assert(!BF || sizeof(T) == 4, "bf16 operands with FP32 storage only");
  // K depth of a slab: 32 (8 loads per operand and thread in flight at once,
  // half the slab iterations of a 16-deep slab on the path's short-K
  // workgroups); 16 for the bf16 form, one 16-deep MFMA per output tile
  constexpr int KB = BF ? 16 : 32;
  constexpr int SA = (BM * KB) / NT, SB = (BN * KB) / NT;  // staged elements per thread
  constexpr int BKP = 16 + 4;  // bf16 row: 16 k values + 4 pad (40 bytes: conflict-free 8-byte reads)
  __shared__ T As[BF ? 1 : KB][BM + 1];
  __shared__ T Bs[BF ? 1 : KB][BN + 1];
  __shared__ __align__(8) unsigned short Asb[BF ? BM : 1][BKP];  // [m][k]
  __shared__ __align__(8) unsigned short Bsb[BF ? BN : 1][BKP];  // [n][k]
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  const int wm = wid & 1, wn = wid >> 1;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int g = blockIdx.z / splits;
  const int sp = blockIdx.z % splits;
  const GemmGroup<T> grp = groups[g];

  typedef typename Acc<T>::type AT;
  AT acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][j][v] = T(0);

  const int t1 = min(grp.t1, grp.t0 + max_terms);
  const int nterm = max(0, t1 - grp.t0);
  const int nks = (K + KB - 1) / KB;
  const int total = nterm * nks;
  const int per = (total + splits - 1) / splits;
  const int sb = sp * per, se = min(total, sb + per);

  // staging coordinates of this thread (fixed over slabs)
  int am[SA], ak[SA], bn[SB], bk[SB];
#pragma unroll
  for (int i = 0; i < SA; ++i) {
    if (!TA) { am[i] = tid & 63; ak[i] = (tid >> 6) + 4 * i; }
    else { ak[i] = tid % KB; am[i] = tid / KB + (NT / KB) * i; }
  }
#pragma unroll
  for (int i = 0; i < SB; ++i) {
    if (!TB) { bk[i] = tid % KB; bn[i] = tid / KB + (NT / KB) * i; }
    else { bn[i] = tid & 63; bk[i] = (tid >> 6) + 4 * i; }
  }
  // Slab s is fetched into registers one slab ahead of its use, so its global
  // loads are in flight while the matrix cores work on slab s - 1.  The loads
  // are unconditional (an out-of-range element reads element 0 of its live
  // operand) and go through the global address space; the range test and the
  // term's alpha are applied when the slab is staged into LDS: a select or a
  // multiply right after a load, or a flat load (counted with the LDS
  // operations that every barrier waits for), would make the thread wait for
  // that load before issuing the next.  A term with alpha == 0 stages zeros
  // and reads neither operand.
  int cur = -1;
  T alpha = T(0);
  T alpha_next = T(0);     // alpha of the fetched slab's term (uniform)
  bool live_next = false;  // whether that alpha is nonzero (uniform)
  const T* Ap = nullptr;
  const T* Bp = nullptr;
  T ra[SA], rb[SB];
  auto fetch = [&](int slab) {
    const int t = grp.t0 + slab / nks;
    const int k0 = (slab % nks) * KB;
    if (t != cur) {
      const GemmTerm<T> tm = terms[t];
      double al = tm.scale;
      if (tm.c1) al *= *tm.c1;
      if (tm.c2) al *= *tm.c2;
      if (tm.c3) al *= *tm.c3;
      alpha = T(al);
      Ap = tm.A;
      Bp = tm.B;
      cur = t;
    }
    alpha_next = alpha;
    live_next = alpha != T(0);
    if (!live_next) return;
    const GPtr<T> ga = (GPtr<T>)Ap;
    const GPtr<T> gb = (GPtr<T>)Bp;
#pragma unroll
    for (int i = 0; i < SA; ++i) {
      const int gm = m0 + am[i], gk = k0 + ak[i];
      const size_t at = (gm < M && gk < K) ? (TA ? gk + (size_t)gm * lda : gm + (size_t)gk * lda) : 0;
      ra[i] = ga[at];
    }
#pragma unroll
    for (int i = 0; i < SB; ++i) {
      const int gn = n0 + bn[i], gk = k0 + bk[i];
      const size_t at = (gn < N && gk < K) ? (TB ? gn + (size_t)gk * ldb : gk + (size_t)gn * ldb) : 0;
      rb[i] = gb[at];
    }
  };
  if (sb < se) fetch(sb);
  for (int slab = sb; slab < se; ++slab) {
    // a slab of a zero-coefficient term (e.g. a disabled Gram block) adds
    // nothing: it is neither staged nor multiplied (the branch is uniform)
    const bool lv = live_next;
    const T al = alpha_next;
    if (!lv) {
      if (slab + 1 < se) fetch(slab + 1);
      continue;
    }
    const int k0 = (slab % nks) * KB;
    T va[SA], vb[SB];
#pragma unroll
    for (int i = 0; i < SA; ++i) va[i] = (m0 + am[i] < M && k0 + ak[i] < K) ? ra[i] * al : T(0);
#pragma unroll
    for (int i = 0; i < SB; ++i) vb[i] = (n0 + bn[i] < N && k0 + bk[i] < K) ? rb[i] : T(0);
    if constexpr (BF) {
#pragma unroll
      for (int i = 0; i < SA; ++i) Asb[am[i]][ak[i]] = bf16_rne(float(va[i]));
#pragma unroll
      for (int i = 0; i < SB; ++i) Bsb[bn[i]][bk[i]] = bf16_rne(float(vb[i]));
    } else {
#pragma unroll
      for (int i = 0; i < SA; ++i) As[ak[i]][am[i]] = va[i];
#pragma unroll
      for (int i = 0; i < SB; ++i) Bs[bk[i]][bn[i]] = vb[i];
    }
    __syncthreads();
    if (slab + 1 < se) fetch(slab + 1);
    if constexpr (BF) {
      // the whole 16-deep slab in one MFMA per 16 x 16 output tile
      const int kq = 4 * (lane >> 4);
      s4 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const s4*>(&Asb[wm * 32 + i * 16 + (lane & 15)][kq]);
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const s4*>(&Bsb[wn * 32 + j * 16 + (lane & 15)][kq]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma_bf16(a[i], b[j], acc[i][j]);
    } else {
#pragma unroll
      for (int kk = 0; kk < KB; kk += 4) {
        const int kr = kk + (lane >> 4);
        T a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = As[kr][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = Bs[kr][wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc[i][j] = mfma(a[i], b[j], acc[i][j]);
      }
    }
    __syncthreads();
  }

  // Accumulator layout of a 16x16 tile (measured on gfx950): for FP32, D[r][c]
  // sits in lane c + 16*(r/4), element r%4; for FP64 in lane c + 16*(r%4),
  // element r/4.
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r16 = Acc<T>::f64 ? 4 * v + (lane >> 4) : 4 * (lane >> 4) + v;
        const int row = m0 + wm * 32 + i * 16 + r16;
        const int col = n0 + wn * 32 + j * 16 + (lane & 15);
        if (row < M && col < N) {
          if (splits == 1) {
            T* c = grp.C + row + (size_t)col * ldc;
            *c = (beta == 0.0) ? acc[i][j][v] : T(beta) * (*c) + acc[i][j][v];
          } else {
            partial[((size_t)blockIdx.z * N + col) * M + row] = acc[i][j][v];
          }
        }
      }
}

template <typename T>
__global__ void splitk_reduce(int M, int N, int ldc, const GemmGroup<T>* __restrict__ groups, double beta,
                              int splits, const T* __restrict__ partial) {
  const int g = blockIdx.y;
  const size_t MN = (size_t)M * N;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < MN; e += (size_t)gridDim.x * blockDim.x) {
    T s = T(0);
    for (int sp = 0; sp < splits; ++sp) s += partial[((size_t)g * splits + sp) * MN + e];
    const int row = int(e % M), col = int(e / M);
    T* c = groups[g].C + row + (size_t)col * ldc;
    *c = (beta == 0.0) ? s : T(beta) * (*c) + s;
  }
}

}  // namespace

template <typename T>
void gemm_run(const GemmLaunch<T>& g, hipStream_t st) {
  if (g.ngroups <= 0 || g.M <= 0 || g.N <= 0) return;
  dim3 grid(ceil_div(g.M, BM), ceil_div(g.N, BN), g.ngroups * g.splits);
  T* part = g.splits > 1 ? g.partial : nullptr;
  timer_begin(kKcGemm, st, g.flops);
  TK_CHECK(!g.bf16 || sizeof(T) == 4, kErrUnsupported, "bf16 operands need FP32 storage");
#define TK_GEMM_CASE(TA, TB, BF)                                                                          \
  if (g.ta == TA && g.tb == TB && g.bf16 == BF)                                                            \
    hipLaunchKernelGGL((gemm_kernel<T, TA, TB, BF && sizeof(T) == 4>), grid, dim3(NT), 0, st, g.M, g.N, g.K, \
                       g.lda, g.ldb, g.ldc, g.terms, g.groups, g.beta, g.splits, part, g.max_terms);
  TK_GEMM_CASE(false, false, false)
  TK_GEMM_CASE(false, true, false)
  TK_GEMM_CASE(true, false, false)
  TK_GEMM_CASE(true, true, false)
  if constexpr (sizeof(T) == 4) {
    TK_GEMM_CASE(false, false, true)
    TK_GEMM_CASE(false, true, true)
    TK_GEMM_CASE(true, false, true)
    TK_GEMM_CASE(true, true, true)
  }
#undef TK_GEMM_CASE
  TK_LAUNCH_CHECK();
  if (g.splits > 1 && !g.defer_reduce) {
    const size_t MN = (size_t)g.M * g.N;
    dim3 rg((unsigned)std::min<size_t>((MN + 255) / 256, 64), g.ngroups);
    hipLaunchKernelGGL((splitk_reduce<T>), rg, dim3(256), 0, st, g.M, g.N, g.ldc, g.groups, g.beta, g.splits, part);
    TK_LAUNCH_CHECK();
  }
  timer_end(kKcGemm, st);
}

template void gemm_run<double>(const GemmLaunch<double>&, hipStream_t);
template void gemm_run<float>(const GemmLaunch<float>&, hipStream_t);

}  // namespace tk
