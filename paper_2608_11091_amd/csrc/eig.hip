// Small symmetric eigensolvers, one workgroup per matrix.
//
//  * Eigenvalues only (N <= 160): Householder reduction to tridiagonal form
//    with the full matrix in LDS, one lane per row and the trailing columns
//    dealt out to 16 waves (a packed-storage variant serves FP64 orders whose
//    full matrix does not fit in LDS), then every eigenvalue by multisection
//    on Sturm counts.  Used by the RoundSum effective-rank rule, which needs
//    the spectrum but no vectors.
//  * Eigenvalues and vectors (N <= 64): cyclic Jacobi with the round-robin
//    parallel ordering, full matrix and eigenvector block in LDS, one lane
//    per row and one wave per rotation pair.  A rotation is taken only when
//    |a_pq| > eps * sqrt(|a_pp a_qq|), the relative criterion under which
//    Jacobi resolves the small eigenvalues of graded positive semidefinite
//    matrices to high relative accuracy; a sweep without rotations ends it.
// Results are sorted in descending order; an optional rank rule (RoundSum
// effective rank / ST-HOSVD truncation) runs on the sorted spectrum.
#include <cfloat>

#include "kernels.hpp"

namespace tk {

namespace {

constexpr int VAL_NT = 512;
constexpr int VAL_NMAX = 160;
constexpr int TG = 4;  // threads per row in the tridiagonal reduction
constexpr int VEC_NMAX = 64;

template <typename T> struct Lim;
template <> struct Lim<double> {
  static __device__ constexpr double eps() { return DBL_EPSILON; }
  static __device__ constexpr double tiny() { return 1e-300; }
};
template <> struct Lim<float> {
  static __device__ constexpr float eps() { return FLT_EPSILON; }
  static __device__ constexpr float tiny() { return 1e-37f; }
};

__device__ __forceinline__ int pk(int i, int j) { return i >= j ? (i * (i + 1)) / 2 + j : (j * (j + 1)) / 2 + i; }

// Rank rules on a descending spectrum; returns the rank (run by one thread).
template <typename T>
__device__ int apply_rule(const EigRule& ru, const T* lam_desc, int N) {
  int r = 0;
  if (ru.kind == 1) {
    const double l0 = N > 0 ? double(lam_desc[0]) : 0.0;
    if (N > 0 && l0 > 0.0) {
      double total = 0.0;
      for (int i = 0; i < N; ++i) {
        const double li = double(lam_desc[i]);
        total += li > ru.delta * l0 ? li : 0.0;
      }
      const double tau = *ru.tau;
      const double thr = tau * tau * total;
      double tail = 0.0;
      r = N;
      for (int i = N - 1; i >= 0; --i) {
        const double li = double(lam_desc[i]);
        tail += li > ru.delta * l0 ? li : 0.0;
        if (tail <= thr) r = i;
        else break;
      }
    }
  } else if (ru.kind == 2) {
    const double total = *ru.total;
    if (ru.force && *ru.force >= 0) {
      r = *ru.force < N ? *ru.force : N;
    } else if (total <= *ru.zthr) {
      r = 1;
    } else {
      const double eps = *ru.eps;
      const double thr = eps * eps * total / ru.d;
      double tail = 0.0;
      r = N;
      for (int i = N - 1; i >= 0; --i) {
        const double li = double(lam_desc[i]);
        tail += li > 0.0 ? li : 0.0;
        if (tail <= thr) r = i;
        else break;
      }
      if (r < 1) r = 1;
      if (r > ru.cap) r = ru.cap;
    }
  }
  return r;
}

// ------------------------------------------------------------ eigenvalues only

// Number of eigenvalues of the tridiagonal (d, e) below x, from the signs of
// the LDL^T pivots of T - x I (e2 = squared off-diagonal).  FP32 takes the
// hardware reciprocal: a Sturm count tolerates ulp-level relative errors in
// each pivot (the computed count is exact for a nearby matrix).
__device__ __forceinline__ float sturm_div(float a, float q) { return a * __builtin_amdgcn_rcpf(q); }
__device__ __forceinline__ double sturm_div(double a, double q) { return a / q; }
template <typename T>
__device__ int sturm_count(const T* d, const T* e2, int n, T x, T pivmin) {
  int c = 0;
  T q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  c += q < T(0);
  for (int k = 1; k < n; ++k) {
    q = d[k] - x - sturm_div(e2[k - 1], q);
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < T(0);
  }
  return c;
}

// Eigenvalues of the symmetric tridiagonal (dd, ee) (ee[k] couples k, k+1),
// both in LDS, by multisection on Sturm counts: G lanes per eigenvalue test G
// interior points of the current interval at once.  Writes them descending to
// `lam` (LDS) and the task's outputs, then applies the task's rank rule.
// Called by all `nthreads` threads of the block; ee is squared in place.
template <typename T>
__device__ void tridiag_spectrum(const EigTask<T>& tk_, T* dd, T* ee, T* lam, T* sc, int N, int tid, int nthreads) {
  if (tid == 0) {
    T gl = dd[0], gu = dd[0], emax2 = T(0);
    for (int k = 0; k < N; ++k) {
      const T r = (k > 0 ? fabs(ee[k - 1]) : T(0)) + (k + 1 < N ? fabs(ee[k]) : T(0));
      gl = fmin(gl, dd[k] - r);
      gu = fmax(gu, dd[k] + r);
    }
    for (int k = 0; k + 1 < N; ++k) emax2 = fmax(emax2, ee[k] * ee[k]);
    sc[1] = gl;
    sc[2] = gu;
    sc[3] = emax2;
  }
  __syncthreads();
  const T gl = sc[1], gu = sc[2], emax2 = sc[3];
  for (int k = tid; k + 1 < N; k += nthreads) ee[k] = ee[k] * ee[k];
  __syncthreads();
  const T bnorm = fmax(fabs(gl), fabs(gu));
  const T pivmin = fmax(Lim<T>::tiny(), emax2 * Lim<T>::tiny() * T(1e10));
  const T tolx = T(2) * Lim<T>::eps() * bnorm;
  // G = lanes per eigenvalue: the largest power of two <= min(16, nthreads / N)
  int G = 1;
  while (G < 16 && 2 * G * N <= nthreads) G *= 2;
  const int g = tid % G;
  const int gshift = (tid & (kWave - 1)) - g;  // first lane of the group within the wave
  const unsigned long long gmask = (G == 64 ? ~0ull : ((1ull << G) - 1ull));
  for (int i = tid / G; i < N; i += nthreads / G) {
    T lo = gl - tolx, hi = gu + tolx;
    for (int it = 0; it < 200 && hi - lo > tolx; ++it) {
      // interior points lo + (hi - lo) (q + 1) / (G + 1), q < G; counts are
      // monotone in q, so the new interval is (point f-1, point f] with f
      // the first point above eigenvalue i (every lane recomputes them)
      const T span = hi - lo;
      const T mid = lo + span * T(g + 1) / T(G + 1);
      const int above = (mid > lo && mid < hi) ? (sturm_count(dd, ee, N, mid, pivmin) > i) : (mid >= hi);
      const unsigned long long bits = (__ballot(above) >> gshift) & gmask;
      const int f = bits ? __builtin_ctzll(bits) : G;
      const T nhi = f < G ? lo + span * T(f + 1) / T(G + 1) : hi;
      const T nlo = f > 0 ? lo + span * T(f) / T(G + 1) : lo;
      if (!(nhi < hi || nlo > lo)) break;
      lo = fmax(lo, nlo);
      hi = fmin(hi, nhi);
    }
    lam[N - 1 - i] = T(0.5) * (lo + hi);
  }
  __syncthreads();
  if (tk_.lam)
    for (int i = tid; i < N; i += nthreads) tk_.lam[i] = lam[i];
  if (tid == 0 && tk_.rule.kind != 0) *tk_.rule.rank_out = apply_rule<T>(tk_.rule, lam, N);
}

constexpr int TF_NT = 1024;
constexpr int TF_NW = TF_NT / kWave;
constexpr int TF_CH = (VAL_NMAX + kWave - 1) / kWave;  // row chunks of 64

template <typename T>
size_t tfull_smem(int NL) {
  return sizeof(T) * (size_t(NL) * (NL + 1) + size_t(TF_NW) * NL + 5 * size_t(NL)) + 64;
}
template <typename T>
bool tfull_fits(int NL) {
  return tfull_smem<T>(NL) <= size_t(160 * 1024 - 1024);
}

// Householder tridiagonalisation with the full matrix in LDS, column-major
// (A[col * LDA + row]), one lane per row and the trailing columns dealt out
// to the 16 waves: step j forms v from column j (every wave, in registers),
// the partial products A_sub v per wave, p = tau * A_sub v and
// w = p - (tau/2)(v.p) v, and the rank-2 update A_sub -= v w^T + w v^T of
// each wave's columns.  Then the spectrum as above.
template <typename T>
__global__ __launch_bounds__(TF_NT) void tridiag_full_kernel(const EigTask<T>* __restrict__ tasks, int NL) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const EigTask<T> tk_ = tasks[blockIdx.x];
  int N = NL;
  if (tk_.ndyn != nullptr) {
    const int nd = *tk_.ndyn;
    if (nd < 0 || nd > NL) {
      if (threadIdx.x == 0 && tk_.rule.rank_out) *tk_.rule.rank_out = -1;
      return;
    }
    N = nd;
  }
  if (N == 0) {
    if (threadIdx.x == 0 && tk_.rule.rank_out) *tk_.rule.rank_out = 0;
    return;
  }
  const int LDA = NL + 1;
  T* A = reinterpret_cast<T*>(smem_raw);
  T* pp = A + size_t(NL) * LDA;  // [TF_NW][NL] partial products
  T* vb = pp + TF_NW * NL;       // Householder vector by absolute row
  T* wb = vb + NL;               // w by absolute row
  T* dd = wb + NL;
  T* ee = dd + NL;
  T* lam = ee + NL;
  __shared__ T red[TF_NW];
  __shared__ T sc[4];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  for (int e = tid; e < N * N; e += TF_NT) {
    const int i = e % N, j = e / N;
    A[j * LDA + i] = (i >= j) ? tk_.A[i + (size_t)j * tk_.lda] : tk_.A[j + (size_t)i * tk_.lda];
  }
  __syncthreads();
  for (int j = 0; j + 2 < N; ++j) {
    const int r0 = j + 1;
    T xs[TF_CH], vs[TF_CH];
    T s2 = T(0);
#pragma unroll
    for (int c = 0; c < TF_CH; ++c) {
      const int row = r0 + lane + kWave * c;
      xs[c] = row < N ? A[j * LDA + row] : T(0);
      if (row > r0 && row < N) s2 += xs[c] * xs[c];
    }
    s2 = wave_sum(s2);
    const T alpha = rdlane(xs[0], 0);
    T beta, tau, scal;
    if (s2 == T(0)) {
      beta = alpha;
      tau = T(0);
      scal = T(0);
    } else {
      beta = -copysign(sqrt(alpha * alpha + s2), alpha);
      tau = (beta - alpha) / beta;
      scal = T(1) / (alpha - beta);
    }
#pragma unroll
    for (int c = 0; c < TF_CH; ++c) {
      const int row = r0 + lane + kWave * c;
      vs[c] = row == r0 ? T(1) : xs[c] * scal;
      if (wave == 0 && row < N) vb[row] = vs[c];
    }
    if (tid == 0) {
      dd[j] = A[j * LDA + j];
      ee[j] = beta;
    }
    __syncthreads();
    if (tau != T(0)) {
      T acc[TF_CH];
#pragma unroll
      for (int c = 0; c < TF_CH; ++c) acc[c] = T(0);
      for (int k = r0 + wave; k < N; k += TF_NW) {
        const T vk = vb[k];
#pragma unroll
        for (int c = 0; c < TF_CH; ++c) {
          const int row = r0 + lane + kWave * c;
          if (row < N) acc[c] += A[k * LDA + row] * vk;
        }
      }
#pragma unroll
      for (int c = 0; c < TF_CH; ++c) {
        const int row = r0 + lane + kWave * c;
        if (row < N) pp[wave * NL + row] = acc[c];
      }
      __syncthreads();
      const int row = r0 + tid;
      T prow = T(0), pv = T(0);
      if (row < N) {
        T sacc = T(0);
        for (int w = 0; w < TF_NW; ++w) sacc += pp[w * NL + row];
        prow = tau * sacc;
        pv = vb[row] * prow;
      }
      const T K = block_sum(pv, red) * T(0.5) * tau;
      if (row < N) wb[row] = prow - K * vb[row];
      __syncthreads();
      T wr[TF_CH];
#pragma unroll
      for (int c = 0; c < TF_CH; ++c) {
        const int rr = r0 + lane + kWave * c;
        wr[c] = rr < N ? wb[rr] : T(0);
      }
      for (int k = r0 + wave; k < N; k += TF_NW) {
        const T vk = vb[k], wk = wb[k];
#pragma unroll
        for (int c = 0; c < TF_CH; ++c) {
          const int rr = r0 + lane + kWave * c;
          if (rr < N) A[k * LDA + rr] -= vs[c] * wk + wr[c] * vk;
        }
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    if (N >= 2) {
      dd[N - 2] = A[(N - 2) * LDA + (N - 2)];
      ee[N - 2] = A[(N - 2) * LDA + (N - 1)];
    }
    dd[N - 1] = A[(N - 1) * LDA + (N - 1)];
  }
  __syncthreads();
  tridiag_spectrum<T>(tk_, dd, ee, lam, sc, N, tid, TF_NT);
}

template <typename T>
__global__ __launch_bounds__(VAL_NT) void tridiag_bisect_kernel(const EigTask<T>* __restrict__ tasks, int NL) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const EigTask<T> tk_ = tasks[blockIdx.x];
  int N = NL;
  if (tk_.ndyn != nullptr) {
    const int nd = *tk_.ndyn;
    if (nd < 0 || nd > NL) {
      if (threadIdx.x == 0 && tk_.rule.rank_out) *tk_.rule.rank_out = -1;
      return;
    }
    N = nd;
  }
  if (N == 0) {
    if (threadIdx.x == 0 && tk_.rule.rank_out) *tk_.rule.rank_out = 0;
    return;
  }
  T* A = reinterpret_cast<T*>(smem_raw);  // packed lower, NL(NL+1)/2
  const int NPK = NL * (NL + 1) / 2;
  T* v = A + NPK;        // NL
  T* p = v + NL;         // NL
  T* dd = p + NL;        // NL diagonal
  T* ee = dd + NL;       // NL off-diagonal (squared later)
  T* lam = ee + NL;      // NL eigenvalues (descending)
  __shared__ T red[VAL_NT / kWave];
  __shared__ T sc[4];
  const int tid = threadIdx.x;
  const int sub = tid % TG, rloc = tid / TG;
  for (int i = tid; i < N; i += VAL_NT)
    for (int j = 0; j <= i; ++j) A[pk(i, j)] = tk_.A[i + (size_t)j * tk_.lda];
  __syncthreads();
  // ---- Householder tridiagonalisation (lower): columns j = 0 .. N-3
  for (int j = 0; j + 2 < N; ++j) {
    const int m = N - j - 1;  // trailing size; rows j+1 .. N-1
    T xi = T(0);
    if (tid < m) xi = A[pk(j + 1 + tid, j)];
    const T s2 = block_sum(tid > 0 && tid < m ? xi * xi : T(0), red);
    if (tid == 0) sc[0] = xi;  // alpha
    __syncthreads();
    const T alpha = sc[0];
    T beta, tau, scal;
    if (s2 == T(0)) {
      beta = alpha;
      tau = T(0);
      scal = T(0);
    } else {
      beta = -copysign(sqrt(alpha * alpha + s2), alpha);
      tau = (beta - alpha) / beta;
      scal = T(1) / (alpha - beta);
    }
    if (tid < m) v[tid] = (tid == 0) ? T(1) : xi * scal;
    if (tid == 0) {
      dd[j] = A[pk(j, j)];
      ee[j] = beta;
    }
    __syncthreads();
    if (tau != T(0)) {
      // p = tau * A_sub v: TG threads per row of the trailing block
      for (int r0 = 0; r0 < m; r0 += VAL_NT / TG) {
        const int r = r0 + rloc;
        T acc = T(0);
        if (r < m) {
          const int gi = j + 1 + r;
          const int base = (gi * (gi + 1)) / 2 + (j + 1);
          auto ix = [&](int k) {
            const int col = j + 1 + k;
            return k <= r ? base + k : (col * (col + 1)) / 2 + gi;
          };
          int k = sub;
          for (; k + 3 * TG < m; k += 4 * TG) {
            const T a0 = A[ix(k)], a1 = A[ix(k + TG)], a2 = A[ix(k + 2 * TG)], a3 = A[ix(k + 3 * TG)];
            const T v0 = v[k], v1 = v[k + TG], v2 = v[k + 2 * TG], v3 = v[k + 3 * TG];
            acc += (a0 * v0 + a1 * v1) + (a2 * v2 + a3 * v3);
          }
          for (; k < m; k += TG) acc += A[ix(k)] * v[k];
        }
        acc += __shfl_xor(acc, 1, kWave);
        acc += __shfl_xor(acc, 2, kWave);
        if (r < m && sub == 0) p[r] = tau * acc;
      }
      __syncthreads();
      const T kk = block_sum(tid < m ? v[tid] * p[tid] : T(0), red) * T(0.5) * tau;
      if (tid < m) p[tid] = p[tid] - kk * v[tid];  // w = p - K v
      __syncthreads();
      // A_sub -= v w^T + w v^T (lower part), TG threads per row
      for (int r0 = 0; r0 < m; r0 += VAL_NT / TG) {
        const int r = r0 + rloc;
        if (r < m) {
          const int gi = j + 1 + r;
          const int base = (gi * (gi + 1)) / 2 + (j + 1);
          const T vi = v[r], wi = p[r];
          int k = sub;
          for (; k + 3 * TG <= r; k += 4 * TG) {
            const T a0 = A[base + k], a1 = A[base + k + TG], a2 = A[base + k + 2 * TG], a3 = A[base + k + 3 * TG];
            const T p0 = p[k], p1 = p[k + TG], p2 = p[k + 2 * TG], p3 = p[k + 3 * TG];
            const T v0 = v[k], v1 = v[k + TG], v2 = v[k + 2 * TG], v3 = v[k + 3 * TG];
            A[base + k] = a0 - (vi * p0 + wi * v0);
            A[base + k + TG] = a1 - (vi * p1 + wi * v1);
            A[base + k + 2 * TG] = a2 - (vi * p2 + wi * v2);
            A[base + k + 3 * TG] = a3 - (vi * p3 + wi * v3);
          }
          for (; k <= r; k += TG) A[base + k] -= vi * p[k] + wi * v[k];
        }
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    if (N >= 2) {
      dd[N - 2] = A[pk(N - 2, N - 2)];
      ee[N - 2] = A[pk(N - 1, N - 2)];
    }
    dd[N - 1] = A[pk(N - 1, N - 1)];
  }
  __syncthreads();
  tridiag_spectrum<T>(tk_, dd, ee, lam, sc, N, tid, VAL_NT);
}

// ------------------------------------------------------------ eigenvalues + vectors
__device__ __forceinline__ int player(int s, int t, int NP) { return s == 0 ? 0 : ((s - 1 + t) % (NP - 1)) + 1; }


// Jacobi rotation annihilating a_pq: t = tan(phi), c = cos(phi).  FP32 uses
// the hardware reciprocal / square-root approximations (about 1 ulp, below
// the rounding of applying the rotation); FP64 uses IEEE operations.
__device__ __forceinline__ float jac_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double jac_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ void jac_rot(float app, float aqq, float apq, float& tt, float& c) {
  const float theta = (aqq - app) * __builtin_amdgcn_rcpf(2.0f * apq);
  const float at = fabsf(theta);
  const float tmag = at > 1e15f ? 0.5f * __builtin_amdgcn_rcpf(at)
                                : __builtin_amdgcn_rcpf(at + __builtin_amdgcn_sqrtf(fmaf(theta, theta, 1.0f)));
  tt = theta >= 0.0f ? tmag : -tmag;
  c = __builtin_amdgcn_rsqf(fmaf(tt, tt, 1.0f));
}
__device__ __forceinline__ void jac_rot(double app, double aqq, double apq, double& tt, double& c) {
  const double theta = (aqq - app) / (2.0 * apq);
  if (fabs(theta) > 1e15) tt = 0.5 / theta;
  else tt = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
  c = 1.0 / sqrt(tt * tt + 1.0);
}


// One lane per matrix row, one wave per rotation pair.  A round applies the
// N/2 disjoint rotations of the round-robin ordering as A <- J^T (A J): first
// the column pairs (p, q) from A into the second buffer B = A J (and V <- V J
// in place), then the row pairs from B back into A (rows of different pairs
// are disjoint), with the 2x2 pivot blocks set to their exact diagonal form.
// Every wave computes all angles of the round in its lanes from A, which no
// wave writes between the row phase of one round and the row phase of the
// next, so every wave sees the same values and takes identical decisions
// (which pairs rotate, whether the round and the sweep rotate anything); a
// round in which no pair rotates is skipped by all waves together, barriers
// included.  A wave issues the loads of all its pairs before any store, and an
// executed round has two barriers.
template <typename T, int JV_NT>
__global__ __launch_bounds__(JV_NT) void jacobi_vec_kernel(const EigTask<T>* __restrict__ tasks, int N) {
  constexpr int JV_NW = JV_NT / kWave;
  constexpr int JV_PPW = (VEC_NMAX / 2) / JV_NW;  // pair slots per wave
  constexpr int LD = VEC_NMAX + 1;
  __shared__ T AV[3][VEC_NMAX][LD];  // A = AV[0], V = AV[1], B = AV[2], all [col][row]
  auto& A = AV[0];
  auto& V = AV[1];
  auto& B = AV[2];
  __shared__ int rank_s;
  __shared__ int posv[VEC_NMAX];
  __shared__ T lam_s[VEC_NMAX];
  const EigTask<T> tk_ = tasks[blockIdx.x];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int NP = N + (N & 1);
  const int H = NP / 2;
  // a pair slot beyond H rotates a zero padding column with itself (c = 1)
  const int dummy = N < VEC_NMAX ? N : VEC_NMAX - 1;
  static_assert(JV_PPW * JV_NW == VEC_NMAX / 2, "pair slots must cover every pair");
  for (int e = tid; e < VEC_NMAX * VEC_NMAX; e += JV_NT) {
    const int i = e % VEC_NMAX, j = e / VEC_NMAX;  // row i, col j
    T a = T(0);
    if (i < N && j < N) a = (i >= j) ? tk_.A[i + (size_t)j * tk_.lda] : tk_.A[j + (size_t)i * tk_.lda];
    A[j][i] = a;
    B[j][i] = T(0);
    V[j][i] = (i == j) ? T(1) : T(0);
  }
  __syncthreads();
  // round-robin players of pair `lane` at round t: 0 and NP-1-lane fixed
  // positions, the others rotate; kept incrementally (no modulo per round)
  int s1 = lane == 0 ? 0 : lane - 1;           // (lane - 1 + t) mod (NP - 1) for lane > 0
  int s2 = NP - 2 - lane;                      // (NP - 2 - lane + t) mod (NP - 1)
  for (int sweep = 0; sweep < 40; ++sweep) {
    unsigned long long anyrot = 0;
    for (int t = 0; t < NP - 1; ++t) {
      int p = lane == 0 ? 0 : s1 + 1, q = s2 + 1;
      if (p > q) {
        const int x = p;
        p = q;
        q = x;
      }
      const bool live = lane < H;
      const bool valid = live && q < N;
      const int pc = valid ? p : 0, qc = valid ? q : 0;
      const T app = A[pc][pc], aqq = A[qc][qc], apq = A[qc][pc];
      const T aa = fabs(apq);
      const int flag = valid && aa > Lim<T>::tiny() && aa > Lim<T>::eps() * jac_sqrt(fabs(app * aqq));
      T tt, cr;
      jac_rot(app, aqq, apq, tt, cr);
      const T c = flag ? cr : T(1);
      const T sn = flag ? tt * cr : T(0);
      const T dp = app - tt * apq, dq = aqq + tt * apq;
      // slots without a real pair (padding, the odd-size dummy player) carry p == q
      const int pl = live ? p : dummy;
      const int ql = live ? (q < N ? q : p) : dummy;
      if (++s1 == NP - 1) s1 = 0;
      if (++s2 == NP - 1) s2 = 0;
      const unsigned long long fm = __ballot(flag);
      anyrot |= fm;
      if (fm == 0) continue;  // wave-uniform and equal in every wave (see above)
      int P_[JV_PPW], Q_[JV_PPW];
      T C_[JV_PPW], S_[JV_PPW];
#pragma unroll
      for (int i = 0; i < JV_PPW; ++i) {
        const int P = wave + i * JV_NW;  // < 32 lanes
        P_[i] = __builtin_amdgcn_readlane(pl, P);
        Q_[i] = __builtin_amdgcn_readlane(ql, P);
        C_[i] = rdlane(c, P);
        S_[i] = rdlane(sn, P);
      }
      // ---- columns: A <- A J, V <- V J
      {
        T ap[JV_PPW], aq[JV_PPW], vp[JV_PPW], vq[JV_PPW];
#pragma unroll
        for (int i = 0; i < JV_PPW; ++i) {
          ap[i] = A[P_[i]][lane];
          aq[i] = A[Q_[i]][lane];
          vp[i] = V[P_[i]][lane];
          vq[i] = V[Q_[i]][lane];
        }
        // slots without a real pair (P == Q) copy unchanged values (c = 1, s = 0)
#pragma unroll
        for (int i = 0; i < JV_PPW; ++i) {
          const T cc = C_[i], ss = S_[i];
          B[P_[i]][lane] = cc * ap[i] - ss * aq[i];
          B[Q_[i]][lane] = ss * ap[i] + cc * aq[i];
          V[P_[i]][lane] = cc * vp[i] - ss * vq[i];
          V[Q_[i]][lane] = ss * vp[i] + cc * vq[i];
        }
      }
      __syncthreads();
      // ---- rows: A <- J^T A, pivot blocks exact
      {
        T bp[JV_PPW], bq[JV_PPW];
#pragma unroll
        for (int i = 0; i < JV_PPW; ++i) {
          bp[i] = B[lane][P_[i]];
          bq[i] = B[lane][Q_[i]];
        }
#pragma unroll
        for (int i = 0; i < JV_PPW; ++i) {
          const int P = wave + i * JV_NW;
          const T cc = C_[i], ss = S_[i];
          const T dpp = rdlane(dp, P), dqq = rdlane(dq, P);
          T np_ = cc * bp[i] - ss * bq[i], nq = ss * bp[i] + cc * bq[i];
          const bool rot = (fm >> P) & 1ull;
          if (rot && lane == P_[i]) {
            np_ = dpp;
            nq = T(0);
          } else if (rot && lane == Q_[i]) {
            np_ = T(0);
            nq = dqq;
          }
          A[lane][P_[i]] = np_;
          A[lane][Q_[i]] = nq;
        }
      }
      __syncthreads();
    }
    if (anyrot == 0) break;
  }
  // sort descending (stable by index), rank rule, write out
  for (int i = tid; i < N; i += JV_NT) {
    const T li = A[i][i];
    int pos = 0;
    for (int j = 0; j < N; ++j) {
      const T lj = A[j][j];
      pos += (lj > li) || (lj == li && j < i);
    }
    posv[i] = pos;
    lam_s[pos] = li;
  }
  __syncthreads();
  const EigRule& ru = tk_.rule;
  if (tid == 0) {
    rank_s = (ru.kind != 0) ? apply_rule<T>(ru, lam_s, N) : N;
    if (ru.kind != 0) *ru.rank_out = rank_s;
  }
  __syncthreads();
  const int rkeep = (ru.kind == 2) ? rank_s : N;
  if (tk_.lam)
    for (int i = tid; i < N; i += JV_NT) tk_.lam[i] = lam_s[i];
  if (tk_.V)
    for (int e = tid; e < N * N; e += JV_NT) {
      const int i = e / N, r = e % N;  // source column i, row r
      const int pos = posv[i];
      tk_.V[r + (size_t)pos * N] = pos < rkeep ? V[i][r] : T(0);
    }
}

template <typename T>
size_t vals_smem(int N) {
  return sizeof(T) * (size_t(N) * (N + 1) / 2 + 5 * size_t(N)) + 64;
}

}  // namespace

template <typename T>
void jacobi_eig(const EigTask<T>* tasks_d, int ntasks, int N, bool want_v, hipStream_t st) {
  if (ntasks <= 0 || N <= 0) return;
  // algorithmic work of a symmetric eigendecomposition of order N: 9 N^3 with
  // eigenvectors (symmetric QR algorithm count), (4/3) N^3 for the tridiagonal
  // reduction behind the eigenvalues-only path
  const int kc = want_v ? kKcJacobi : kKcEigVals;
  const double nn = double(N);
  timer_begin(kc, st, double(ntasks) * (want_v ? 9.0 : 4.0 / 3.0) * nn * nn * nn,
              double(ntasks) * sizeof(T) * ((want_v ? 2.0 : 1.0) * nn * nn + nn));
  if (want_v) {
    TK_CHECK(N <= VEC_NMAX, kErrUnsupported, "symmetric eigensolver: eigenvectors above size 64");
    // measured on gfx950 (N = 53): 16 waves for FP32, 8 for FP64 (register pressure)
    constexpr int nt = sizeof(T) == 4 ? 1024 : 512;
    hipLaunchKernelGGL((jacobi_vec_kernel<T, nt>), dim3(ntasks), dim3(nt), 0, st, tasks_d, N);
  } else {
    TK_CHECK(N <= VAL_NMAX, kErrUnsupported, "symmetric eigensolver: matrix larger than 160");
    static bool attr_set[4] = {false, false, false, false};
    const bool full = tfull_fits<T>(N);
    bool& done = attr_set[(sizeof(T) == 8 ? 2 : 0) + (full ? 1 : 0)];
    if (full) {
      if (!done) {
        TK_HIP(hipFuncSetAttribute((const void*)tridiag_full_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   int(160 * 1024 - 1024)));
        done = true;
      }
      hipLaunchKernelGGL((tridiag_full_kernel<T>), dim3(ntasks), dim3(TF_NT), tfull_smem<T>(N), st, tasks_d, N);
    } else {
      // the full matrix does not fit in LDS (FP64 above order 128): packed storage
      if (!done) {
        TK_HIP(hipFuncSetAttribute((const void*)tridiag_bisect_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   int(vals_smem<T>(VAL_NMAX))));
        done = true;
      }
      hipLaunchKernelGGL((tridiag_bisect_kernel<T>), dim3(ntasks), dim3(VAL_NT), vals_smem<T>(N), st, tasks_d, N);
    }
  }
  TK_LAUNCH_CHECK();
  timer_end(kc, st);
}

template void jacobi_eig<double>(const EigTask<double>*, int, int, bool, hipStream_t);
template void jacobi_eig<float>(const EigTask<float>*, int, int, bool, hipStream_t);

}  // namespace tk
