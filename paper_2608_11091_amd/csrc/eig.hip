// Small symmetric eigensolvers, one workgroup per matrix.
//
//  * Eigenvalues only (N <= 160): Householder reduction to tridiagonal form
//    with the matrix distributed over the registers of 16 waves, then every
//    eigenvalue by multisection on Sturm counts.  Used by the RoundSum
//    effective-rank rule, which needs the spectrum but no vectors.
//  * Eigenvalues only (160 < N <= 512): the same reduction with the matrix in
//    global memory (it stays in the L2 of the workgroup's XCD), reduced in
//    place; each step streams the trailing block once, applying the previous
//    step's rank-2 update and forming the next product A v in the same pass.
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

constexpr int VAL_NMAX = kEigRegMax;
constexpr int VEC_NMAX = 64;
constexpr int GM_NMAX = 512;

template <typename T> struct Lim;
template <> struct Lim<double> {
  static __device__ constexpr double eps() { return DBL_EPSILON; }
  static __device__ constexpr double tiny() { return 1e-300; }
};
template <> struct Lim<float> {
  static __device__ constexpr float eps() { return FLT_EPSILON; }
  static __device__ constexpr float tiny() { return 1e-37f; }
};

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

// Householder tridiagonalisation with the matrix in registers: lane l of
// wave w of W holds the entries (l + 64 a, w + W b), a < 3, so the rank-2
// update of a step touches only registers and LDS carries vectors and partial
// sums, never the matrix.  Step j: the wave holding column j forms v (the
// Householder vector of the part below the diagonal) and tau; every thread
// forms its partial products of A_sub v and of v^T A_sub v, which are summed
// across the waves through LDS into p = tau A_sub v and
// w = p - (tau^2 / 2)(v^T A_sub v) v; every thread applies
// A_sub -= v w^T + w v^T to its entries.  Vectors alternate between two LDS
// buffers with the step parity.  Then the spectrum as above.
constexpr int TRG_RR = (VAL_NMAX + kWave - 1) / kWave;  // rows per thread

// 16 waves (FP64 spills some registers; 8 waves with twice the entries per
// thread spill more)
template <typename T>
constexpr int trg_nt() { return 1024; }

template <typename T, int TRG_NT>
__global__ __launch_bounds__(TRG_NT) void tridiag_reg_kernel(const EigTask<T>* __restrict__ tasks, int NL) {
  constexpr int TRG_NW = TRG_NT / kWave;                   // waves
  constexpr int TRG_RC = (VAL_NMAX + TRG_NW - 1) / TRG_NW;  // columns per thread
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
  __shared__ T vb[2][VAL_NMAX], wb[2][VAL_NMAX];
  __shared__ T pp[TRG_NW][VAL_NMAX];
  __shared__ T qs[TRG_NW];
  __shared__ T tau_s[2];
  __shared__ T dd[VAL_NMAX], ee[VAL_NMAX], lam[VAL_NMAX];
  __shared__ T sc[4];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  for (int e = tid; e < 2 * VAL_NMAX; e += TRG_NT) {
    vb[e / VAL_NMAX][e % VAL_NMAX] = T(0);
    wb[e / VAL_NMAX][e % VAL_NMAX] = T(0);
  }
  T a[TRG_RR][TRG_RC];
#pragma unroll
  for (int i = 0; i < TRG_RR; ++i)
#pragma unroll
    for (int k = 0; k < TRG_RC; ++k) {
      const int r = lane + kWave * i, c = wave + TRG_NW * k;
      T v = T(0);
      if (r < N && c < N) v = (r >= c) ? tk_.A[r + (size_t)c * tk_.lda] : tk_.A[c + (size_t)r * tk_.lda];
      a[i][k] = v;
    }
  // Householder vector of column jj from this wave's registers (called by the
  // wave holding column jj only; jj + 2 < N)
  auto householder = [&](int jj) {
    const int buf = jj & 1;
    const int r0 = jj + 1;
    const int kb = jj / TRG_NW;  // uniform
    T x[TRG_RR];
    T s2 = T(0);
#pragma unroll
    for (int i = 0; i < TRG_RR; ++i) {
      T v = T(0);
#pragma unroll
      for (int k = 0; k < TRG_RC; ++k)
        if (k == kb) v = a[i][k];
      x[i] = v;
      const int r = lane + kWave * i;
      if (r > r0 && r < N) s2 += v * v;
    }
    s2 = wave_sum(s2);
    T xa = T(0);
#pragma unroll
    for (int i = 0; i < TRG_RR; ++i)
      if (i == r0 / kWave) xa = x[i];
    const T alpha = rdlane(xa, r0 & (kWave - 1));
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
    for (int i = 0; i < TRG_RR; ++i) {
      const int r = lane + kWave * i;
      if (r >= r0 && r < N) vb[buf][r] = r == r0 ? T(1) : x[i] * scal;
      if (r == jj) dd[jj] = x[i];
    }
    if (lane == 0) {
      tau_s[buf] = tau;
      ee[jj] = beta;
    }
  };
  for (int j = 0; j + 2 < N; ++j) {
    const int buf = j & 1;
    const int r0 = j + 1;
    if (wave == (j & (TRG_NW - 1))) householder(j);
    __syncthreads();
    const T tau = tau_s[buf];
    if (tau == T(0)) continue;  // the same value in every thread: nothing to apply
    // unconditional loads (in-bounds indices; the buffers hold finite values)
    // times a 0/1 mask, so that all loads issue before a single wait
    T vr[TRG_RR], vc[TRG_RC];
#pragma unroll
    for (int i = 0; i < TRG_RR; ++i) {
      const int r = lane + kWave * i;
      vr[i] = vb[buf][min(r, VAL_NMAX - 1)] * T(r >= r0 && r < N);
    }
#pragma unroll
    for (int k = 0; k < TRG_RC; ++k) {
      const int c = wave + TRG_NW * k;
      vc[k] = vb[buf][c] * T(c >= r0 && c < N);
    }
    // ---- partial products over this wave's columns
    T q = T(0);
#pragma unroll
    for (int i = 0; i < TRG_RR; ++i) {
      T acc = T(0);
#pragma unroll
      for (int k = 0; k < TRG_RC; ++k) acc += a[i][k] * vc[k];
      q += vr[i] * acc;
      const int r = lane + kWave * i;
      if (r < N) pp[wave][r] = acc;
    }
    q = wave_sum(q);
    if (lane == 0) qs[wave] = q;
    __syncthreads();
    if (tid >= r0 && tid < N) {
      T sacc = T(0), vav = T(0);
#pragma unroll
      for (int w = 0; w < TRG_NW; ++w) {
        sacc += pp[w][tid];
        vav += qs[w];
      }
      const T K = T(0.5) * tau * tau * vav;
      wb[buf][tid] = tau * sacc - K * vb[buf][tid];
    }
    __syncthreads();
    // ---- rank-2 update of this thread's entries
    T wr[TRG_RR], wc[TRG_RC];
#pragma unroll
    for (int i = 0; i < TRG_RR; ++i) {
      const int r = lane + kWave * i;
      wr[i] = wb[buf][min(r, VAL_NMAX - 1)] * T(r >= r0 && r < N);
    }
#pragma unroll
    for (int k = 0; k < TRG_RC; ++k) {
      const int c = wave + TRG_NW * k;
      wc[k] = wb[buf][c] * T(c >= r0 && c < N);
    }
#pragma unroll
    for (int i = 0; i < TRG_RR; ++i)
#pragma unroll
      for (int k = 0; k < TRG_RC; ++k) a[i][k] -= vr[i] * wc[k] + wr[i] * vc[k];
    __syncthreads();
  }
  // last 2 x 2 block: diagonal entries and the coupling, from their holders
#pragma unroll
  for (int i = 0; i < TRG_RR; ++i)
#pragma unroll
    for (int k = 0; k < TRG_RC; ++k) {
      const int r = lane + kWave * i, c = wave + TRG_NW * k;
      if (N >= 2 && r == N - 2 && c == N - 2) dd[N - 2] = a[i][k];
      if (N >= 2 && r == N - 1 && c == N - 2) ee[N - 2] = a[i][k];
      if (r == N - 1 && c == N - 1) dd[N - 1] = a[i][k];
    }
  __syncthreads();
  tridiag_spectrum<T>(tk_, dd, ee, lam, sc, N, tid, TRG_NT);
}

// Householder tridiagonalisation of an N x N symmetric matrix (160 < N <= 512)
// held in global memory, column-major with leading dimension lda; only the
// lower triangle of the input is read and the matrix is overwritten.  One
// workgroup of 16 waves.  The lower triangle is first mirrored into the upper
// one through LDS tiles, so that the reduction can keep full storage and form
// A v as row sums (each lane owns rows, no cross-lane sums per column).
// Step j (sub-block S = rows/columns j+1..N-1, Householder vector v with
// v_{j+1} = 1, tau, and the pending update (vp, wp) of step j-1):
//   1. column j of the updated matrix, x_i = a_ij - vp_i wp_j - wp_i vp_j;
//      the diagonal entry and ||x_{j+2..}||^2 give v, tau and beta;
//   2. one pass over S: a <- a - vp wp^T - wp vp^T (stored back), and every
//      lane accumulates its rows of S v; the same pass accumulates v^T S v;
//   3. w = tau S v - (tau^2 / 2)(v^T S v) v becomes the pending update.
// The final 2 x 2 block takes the last pending update; then the spectrum by
// multisection as above.
template <typename T>
__global__ __launch_bounds__(1024) void tridiag_gm_kernel(const EigTask<T>* __restrict__ tasks, int NL) {
  constexpr int NT = 1024;
  constexpr int NW = NT / kWave;          // 16 waves
  constexpr int RCH = GM_NMAX / kWave;    // row chunks of 64
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
  T* A = const_cast<T*>(tk_.A);
  const size_t lda = size_t(tk_.lda);
  __shared__ T xb[GM_NMAX], vp[GM_NMAX], wp[GM_NMAX];
  __shared__ T rowp[NW][GM_NMAX];  // per-wave row sums; also the mirror tiles
  __shared__ T part[NW], qpart[NW];
  __shared__ T dd[GM_NMAX], ee[GM_NMAX], lam[GM_NMAX];
  __shared__ T sc[4];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  for (int i = tid; i < GM_NMAX; i += NT) {
    vp[i] = T(0);
    wp[i] = T(0);
  }
  // ---- mirror the lower triangle into the upper one, 64 x 64 tiles through LDS
  {
    T* tile = &rowp[0][0];  // 64 x 65 staging (fits in rowp)
    const int nt = (N + kWave - 1) / kWave;
    for (int I = 0; I < nt; ++I)
      for (int J = 0; J <= I; ++J) {
        // load tile (I, J): column c of the tile by the threads with c % 16 == wave
        for (int c = wave; c < kWave; c += NW) {
          const int r = I * kWave + lane, col = J * kWave + c;
          tile[c * (kWave + 1) + lane] = (r < N && col < N) ? A[r + size_t(col) * lda] : T(0);
        }
        __syncthreads();
        // store its transpose into tile (J, I), upper-triangle entries only
        for (int c = wave; c < kWave; c += NW) {
          const int r = J * kWave + lane, col = I * kWave + c;  // destination (r, col), r < col
          if (r < N && col < N && r < col) A[r + size_t(col) * lda] = tile[lane * (kWave + 1) + c];
        }
        __syncthreads();
      }
  }
  for (int j = 0; j + 2 < N; ++j) {
    // ---- 1. column j after the pending update, ||x_{j+2..N-1}||^2
    T s2p = T(0);
    if (tid >= j && tid < N) {
      const T x = A[tid + size_t(j) * lda] - (vp[tid] * wp[j] + wp[tid] * vp[j]);
      xb[tid] = x;
      if (tid == j) dd[j] = x;
      if (tid >= j + 2) s2p = x * x;
    }
    s2p = wave_sum(s2p);
    if (lane == 0) part[wave] = s2p;
    __syncthreads();
    T s2 = T(0);
#pragma unroll
    for (int w = 0; w < NW; ++w) s2 += part[w];
    const T alpha = xb[j + 1];
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
    if (tid == 0) ee[j] = beta;
    const T vmask = tau != T(0) ? T(1) : T(0);
    auto vval = [&](int i) -> T {  // Householder vector entry (0 outside j+1..N-1)
      return i == j + 1 ? vmask : (i > j + 1 && i < N ? xb[i] * scal : T(0));
    };
    // ---- 2. pass over the trailing block
    const int r0 = j + 1;
    const int t0 = r0 / kWave;  // first row chunk touched (uniform)
    T vpr[RCH], wpr[RCH], vr[RCH], acc[RCH];
#pragma unroll
    for (int t = 0; t < RCH; ++t) {
      const int i = t * kWave + lane;
      const bool ok = i >= r0 && i < N;
      vpr[t] = ok ? vp[i] : T(0);
      wpr[t] = ok ? wp[i] : T(0);
      vr[t] = ok ? vval(i) : T(0);
      acc[t] = T(0);
    }
    for (int c = r0 + wave; c < N; c += NW) {
      const T vpc = vp[c], wpc = wp[c], vc = vval(c);
      T* col = A + size_t(c) * lda;
      T a[RCH];
#pragma unroll
      for (int t = 0; t < RCH; ++t) {
        const int i = t * kWave + lane;
        a[t] = (t >= t0 && i >= r0 && i < N) ? col[i] : T(0);
      }
#pragma unroll
      for (int t = 0; t < RCH; ++t) {
        const int i = t * kWave + lane;
        if (t >= t0 && i >= r0 && i < N) {
          const T v = a[t] - (vpr[t] * wpc + wpr[t] * vpc);
          col[i] = v;
          acc[t] += v * vc;
        }
      }
    }
    T q = T(0);
#pragma unroll
    for (int t = 0; t < RCH; ++t) {
      q += vr[t] * acc[t];
      const int i = t * kWave + lane;
      if (i >= r0 && i < N) rowp[wave][i] = acc[t];
    }
    q = wave_sum(q);
    if (lane == 0) qpart[wave] = q;
    __syncthreads();
    // ---- 3. the new pending update
    if (tid >= r0 && tid < N) {
      T sv = T(0), vav = T(0);
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        sv += rowp[w][tid];
        vav += qpart[w];
      }
      const T vi = vval(tid);
      const T K = T(0.5) * tau * tau * vav;
      vp[tid] = vi;
      wp[tid] = tau * sv - K * vi;
    }
    __syncthreads();
  }
  // last 2 x 2 block (or the single entry) after the last pending update
  if (tid == 0) {
    if (N >= 2) {
      const int a = N - 2, b = N - 1;
      dd[a] = A[a + size_t(a) * lda] - T(2) * vp[a] * wp[a];
      ee[a] = A[b + size_t(a) * lda] - (vp[b] * wp[a] + wp[b] * vp[a]);
      dd[b] = A[b + size_t(b) * lda] - T(2) * vp[b] * wp[b];
    } else {
      dd[0] = A[0];
    }
  }
  __syncthreads();
  tridiag_spectrum<T>(tk_, dd, ee, lam, sc, N, tid, NT);
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
      // ---- columns: B <- A J, V <- V J
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
      // ---- rows: A <- J^T B, pivot blocks exact
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
    TK_CHECK(N <= GM_NMAX, kErrUnsupported, "symmetric eigensolver: matrix larger than 512");
    if (N <= VAL_NMAX)
      hipLaunchKernelGGL((tridiag_reg_kernel<T, trg_nt<T>()>), dim3(ntasks), dim3(trg_nt<T>()), 0, st, tasks_d, N);
    else
      hipLaunchKernelGGL((tridiag_gm_kernel<T>), dim3(ntasks), dim3(1024), 0, st, tasks_d, N);
  }
  TK_LAUNCH_CHECK();
  timer_end(kc, st);
}

template void jacobi_eig<double>(const EigTask<double>*, int, int, bool, hipStream_t);
template void jacobi_eig<float>(const EigTask<float>*, int, int, bool, hipStream_t);

}  // namespace tk
