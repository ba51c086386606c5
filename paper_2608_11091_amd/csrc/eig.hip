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
//    parallel ordering on 2 x 2 blocks, full matrix and eigenvector block in
//    LDS.  A rotation is taken only when |a_pq| > eps * sqrt(|a_pp a_qq|),
//    the relative criterion under which Jacobi resolves the small eigenvalues
//    of graded positive semidefinite matrices to high relative accuracy; a
//    sweep without rotations ends it.
// Results are sorted in descending order; an optional rank rule (RoundSum
// effective rank / ST-HOSVD truncation) runs on the sorted spectrum.
#include <cfloat>

#include "kernels.hpp"

namespace tk {

namespace {

constexpr int VAL_NMAX = kEigRegMax;
constexpr int VEC_NMAX = 64;
constexpr int GM_NMAX = 512;

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float __attribute__((ext_vector_type(4))); };
template <> struct Vec4<double> { using type = double __attribute__((ext_vector_type(4))); };

template <typename T> struct Lim;
template <> struct Lim<double> {
  static __device__ constexpr double eps() { return DBL_EPSILON; }
  static __device__ constexpr double sqrt_eps() { return 1.4901161193847656e-08; }  // 2^-26
  static __device__ constexpr double tiny() { return 1e-300; }
};
template <> struct Lim<float> {
  static __device__ constexpr float eps() { return FLT_EPSILON; }
  static __device__ constexpr float sqrt_eps() { return 3.4526698e-04f; }  // 2^-11.5
  static __device__ constexpr float tiny() { return 1e-37f; }
};

// A task does nothing when its pair flag or any rank certificate is set.
template <typename T>
__device__ __forceinline__ bool task_skipped(const EigTask<T>& t) {
  if (t.skip != nullptr && *t.skip != 0) return true;
  bool c = false;
  for (int i = 0; i < t.ncert; ++i) c |= t.cert[i] != 0;
  return c;
}

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
  // Rank rule with a cap (kind 1, cap1 > 0): only min(r~, cap1) is needed,
  // and one Sturm count settles the common case.  If at least cap1
  // eigenvalues lie at or above x = max(tau^2 tot, delta (gu + tolx)) + 2 tolx,
  // with tot = trace + N (max(0, -gl) + tolx) bounding the rule's total (the
  // positive eigenvalues, as the multisection would compute them), then the
  // cap1-th largest counts as nonzero and alone exceeds tau^2 total, so the
  // tail from it on does too and r~ >= cap1.
  if (tk_.rule.kind == 1 && tk_.rule.cap1 > 0 && tk_.rule.cap1 <= N) {
    if (tid == 0) {
      double tr = 0.0;
      for (int k = 0; k < N; ++k) tr += double(dd[k]);
      const double tau = *tk_.rule.tau;
      const double tx = double(tolx);
      const double tot = tr + double(N) * (fmax(0.0, -double(gl)) + tx);
      const double x = fmax(tau * tau * tot, tk_.rule.delta * (double(gu) + tx)) + 2.0 * tx;
      const int below = sturm_count<T>(dd, ee, N, T(x), pivmin);
      sc[0] = (N - below >= tk_.rule.cap1) ? T(1) : T(0);
    }
    __syncthreads();
    if (sc[0] != T(0)) {
      if (tid == 0) *tk_.rule.rank_out = tk_.rule.cap1;
      return;  // uniform: every thread read the same flag after the barrier
    }
  }
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
  if (task_skipped(tk_)) return;
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
    // no barrier here: the next step's Householder vector comes from its
    // wave's own registers and goes to the other buffer, and every shared
    // array this step reads is written again only after the next step's
    // first barrier (pp, qs) or two steps on (vb, wb, tau_s by parity)
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
  if (task_skipped(tk_)) return;
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
  using T4 = typename Vec4<T>::type;
  T* const W = A;          // the trailing-block pass reads columns as 16-byte vectors
  const size_t ldw = lda;  // (lda is a multiple of 4 and A 16-byte aligned: checked by the launcher)
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
    // ---- 2. pass over the trailing block: lane l owns rows 4l + 256u .. +3
    //         (u < 2), 16-byte accesses; several columns per wave in flight
    const int r0 = j + 1;
    T4 vpr[2], wpr[2], acc[2];
    bool live[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int rb = 4 * lane + 256 * u;
      live[u] = rb < N && rb + 3 >= r0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = rb + e;
        const bool ok = i >= r0 && i < N;
        vpr[u][e] = ok ? vp[i] : T(0);
        wpr[u][e] = ok ? wp[i] : T(0);
        acc[u][e] = T(0);
      }
    }
    constexpr int CU = sizeof(T) == 4 ? 4 : 2;  // columns in flight per wave (FP64: register budget)
    for (int c0 = r0 + wave; c0 < N; c0 += CU * NW) {
      T4 a[CU][2];
      T vpc[CU], wpc[CU], vc[CU];
#pragma unroll
      for (int m = 0; m < CU; ++m) {
        const int c = c0 + m * NW;
        const bool cok = c < N;  // uniform across the wave
        vpc[m] = cok ? vp[c] : T(0);
        wpc[m] = cok ? wp[c] : T(0);
        vc[m] = cok ? vval(c) : T(0);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const T4* src = reinterpret_cast<const T4*>(W + size_t(cok ? c : r0) * ldw + 4 * lane + 256 * u);
          a[m][u] = (cok && live[u]) ? *src : T4{};
        }
      }
#pragma unroll
      for (int m = 0; m < CU; ++m) {
        const int c = c0 + m * NW;
        if (c >= N) continue;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          if (!live[u]) continue;
          const int rb = 4 * lane + 256 * u;
          T4 v = a[m][u] - (vpr[u] * wpc[m] + wpr[u] * vpc[m]);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const bool ok = rb + e >= r0 && rb + e < N;
            v[e] = ok ? v[e] : a[m][u][e];
            acc[u][e] += ok ? v[e] * vc[m] : T(0);
          }
          *reinterpret_cast<T4*>(W + size_t(c) * ldw + rb) = v;
        }
      }
    }
    T q = T(0);
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = 4 * lane + 256 * u + e;
        const bool ok = i >= r0 && i < N;
        q += ok ? vval(i) * acc[u][e] : T(0);
        if (ok) rowp[wave][i] = acc[u][e];
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


// Two-sided cyclic Jacobi on 2 x 2 blocks.  With the round-robin ordering a
// round applies N/2 disjoint rotations J, A <- J^T A J; every entry of A
// belongs to exactly one block (rows of pair I) x (columns of pair J), and the
// block's new value depends on that block and the two rotations only.  One
// thread per block with I <= J updates it in place and writes the mirrored
// block (J, I) too, so A stays exactly symmetric (full storage, column-major,
// leading dimension 65 = 1 mod 32: both a column and a row of the lanes'
// entries fall in distinct banks).  The kernel is bound by instruction issue
// (16 waves share 4 SIMDs), so every index that does not change between
// rounds is computed once, and V is rotated four rows per lane with 16-byte
// LDS accesses.  Per round:
//   phase 1: wave 0 computes the round's rotations from A (one lane per pair)
//            and decides whether any pair rotates -- if none does, the round
//            is skipped; meanwhile other waves apply the previous executed
//            round's rotations to the eigenvector block (V <- V J, one round
//            behind);
//   phase 2: every block thread rotates its block (the 2 x 2 pivot blocks are
//            set to their exact diagonal form).
// A rotation is taken only when |a_pq| > eps sqrt(|a_pp a_qq|) (relative
// criterion: small eigenvalues of graded matrices keep their digits); a sweep
// without rotations ends the iteration.  Every decision is taken once, by
// wave 0, and read by all threads after a barrier; decisions are
// double-buffered by round parity because wave 0 may enter the next round's
// first phase while slower waves still read the current one.
template <typename T>
__global__ __launch_bounds__(1024) void jacobi_blk_kernel(const EigTask<T>* __restrict__ tasks, int N) {
  constexpr int NT = 1024;
  constexpr int NPM = VEC_NMAX;
  constexpr int HM = NPM / 2;
  constexpr int LD = NPM + 1;            // A leading dimension (65 = 1 mod 32)
  constexpr int LDV = NPM + 4;           // V leading dimension: 16-byte aligned columns
  constexpr int RQ = NPM / 4;            // row quads of V
  using T4 = typename Vec4<T>::type;
  __shared__ T A[NPM * LD];              // A[c * LD + r]
  __shared__ __align__(16) T V[NPM * LDV];
  __shared__ T csb[2][HM][2];            // rotations (c, s) of a round, by buffer
  __shared__ T tnb[2][HM];               // tan of the round's rotations, by buffer
  __shared__ unsigned short sch[NPM][HM];  // round-robin schedule: pair k of round t = p | q << 8, p < q
  __shared__ unsigned int rmask[2];      // pairs that rotate (bit k), by round parity
  __shared__ int skip_s[2];
  __shared__ int rotflag[3];
  __shared__ int bigflag[3];             // a rotation of the sweep had a scaled off-diagonal above sqrt(eps)
  __shared__ int rank_s;
  __shared__ int posv[NPM];
  __shared__ T lam_s[NPM];
  const EigTask<T> tk_ = tasks[blockIdx.x];
  if (task_skipped(tk_)) return;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  const int NP = N + (N & 1);
  const int H = NP / 2;
  const int M = NP - 1;  // rounds per sweep
  for (int e = tid; e < M * H; e += NT) {
    const int t = e / H, k = e % H;
    const int a = k == 0 ? 0 : ((k - 1 + t) % M) + 1;
    const int b = ((NP - 2 - k + t) % M) + 1;
    const int p = a < b ? a : b, q = a < b ? b : a;
    sch[t][k] = (unsigned short)(p | (q << 8));
  }
  // the lower triangle, column by column (contiguous reads of whole cache
  // lines), mirrored into the upper one in LDS; the padding row and column
  // of an odd order are zero
  for (int e = tid; e < NP * NP; e += NT) {
    const int c = e / NP, r = e % NP;
    if (r < c) continue;
    T a = T(0);
    if (r < N) {
      const size_t at = r + (size_t)c * tk_.lda;
      if (tk_.part) {  // the matrix's split-K partials, summed in split order
        // (eight loads in flight at a time; the additions keep their order)
        const T* pp = tk_.part + at;
        int sp = 0;
        for (; sp + 8 <= tk_.splits; sp += 8) {
          T v[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) v[u] = pp[(sp + u) * tk_.pstride];
#pragma unroll
          for (int u = 0; u < 8; ++u) a += v[u];
        }
        for (; sp < tk_.splits; ++sp) a += pp[sp * tk_.pstride];
      } else {
        a = tk_.A[at];
      }
    }
    A[c * LD + r] = a;
    A[r * LD + c] = a;
  }
  for (int e = tid; e < NP * LDV; e += NT) {
    const int c = e / LDV, r = e % LDV;
    V[e] = (r == c) ? T(1) : T(0);
  }
  if (tid < 3) {
    rotflag[tid] = 0;
    bigflag[tid] = 0;
  }
  // block task of this thread (pair I <= pair J), fixed for the whole kernel
  const int nblk = H * (H + 1) / 2;
  int bI = 0, bJ = 0;
  const bool blk = tid < nblk;
  if (blk) {
    int J = 0, rem = tid;
    while (rem >= J + 1) {
      rem -= J + 1;
      ++J;
    }
    bI = rem;
    bJ = J;
  }
  // V task: rows 4 vi .. 4 vi + 3 of the columns of pair vJ (threads of waves 1..)
  const int vt = tid - kWave;
  const int nq = (NP + 3) / 4;
  const bool vtask = vt >= 0 && vt < nq * H;
  const int vi = vtask ? vt % nq : 0, vJ = vtask ? vt / nq : 0;
  const bool vtask2 = vt >= 0 && vt + (NT - kWave) < nq * H;  // a second task for large N
  const int vi2 = vtask2 ? (vt + NT - kWave) % nq : 0, vJ2 = vtask2 ? (vt + NT - kWave) / nq : 0;
  static_assert(RQ * HM <= 2 * (NT - kWave), "two V tasks per thread cover every row quad and pair");
  __syncthreads();
  int g = 0;            // rounds executed or skipped so far (buffer parity)
  int prev_t = -1;      // round whose rotations V still has to take (-1: none)
  int prev_buf = 0;
  auto v_rot = [&](int t, int buf, int i4, int J) {
    const unsigned pq = sch[t][J];
    const int p = int(pq & 0xffu), q = int(pq >> 8);
    const T c = csb[buf][J][0], sn = csb[buf][J][1];
    T4* vp = reinterpret_cast<T4*>(&V[p * LDV + 4 * i4]);
    T4* vq = reinterpret_cast<T4*>(&V[q * LDV + 4 * i4]);
    const T4 a = *vp, b = *vq;
    *vp = c * a - sn * b;
    *vq = sn * a + c * b;
  };
  for (int sweep = 0; sweep < 40; ++sweep) {
    for (int t = 0; t < M; ++t) {
      const int cur = g & 1;
      // ---- phase 1
      if (wave == 0) {
        T c = T(1), sn = T(0), tt = T(0);
        int flag = 0, big = 0;
        if (lane < H) {
          const unsigned pq = sch[t][lane];
          const int p = int(pq & 0xffu), q = int(pq >> 8);
          const T app = A[p * LD + p], aqq = A[q * LD + q], apq = A[q * LD + p];
          const T aa = fabs(apq);
          const T sc = jac_sqrt(fabs(app * aqq));
          flag = (q < N) && aa > Lim<T>::tiny() && aa > Lim<T>::eps() * sc;
          big = flag && aa > Lim<T>::sqrt_eps() * sc;
          T tr, cr;
          jac_rot(app, aqq, flag ? apq : T(1), tr, cr);
          if (flag) {
            c = cr;
            sn = tr * cr;
            tt = tr;
          }
          csb[cur][lane][0] = c;
          csb[cur][lane][1] = sn;
          tnb[cur][lane] = tt;
        }
        const unsigned long long fm = __ballot(flag);
        const unsigned long long bm = __ballot(big);
        if (lane == 0) {
          skip_s[cur] = fm == 0;
          rmask[cur] = (unsigned int)fm;
          if (fm != 0) rotflag[sweep % 3] = 1;
          if (bm != 0) bigflag[sweep % 3] = 1;
          if (t == 0) {
            rotflag[(sweep + 1) % 3] = 0;
            bigflag[(sweep + 1) % 3] = 0;
          }
        }
      } else if (prev_t >= 0) {
        if (vtask) v_rot(prev_t, prev_buf, vi, vJ);
        if (vtask2) v_rot(prev_t, prev_buf, vi2, vJ2);
      }
      __syncthreads();
      ++g;
      if (skip_s[cur]) {
        prev_t = -1;
        continue;  // uniform: every thread read the same flag after the barrier
      }
      // ---- phase 2
      if (blk) {
        const unsigned pqI = sch[t][bI], pqJ = sch[t][bJ];
        const int pI = int(pqI & 0xffu), qI = int(pqI >> 8);
        const int pJ = int(pqJ & 0xffu), qJ = int(pqJ >> 8);
        const T cI = csb[cur][bI][0], sI = csb[cur][bI][1];
        const T cJ = csb[cur][bJ][0], sJ = csb[cur][bJ][1];
        const T x00 = A[pJ * LD + pI], x01 = A[qJ * LD + pI];
        const T x10 = A[pJ * LD + qI], x11 = A[qJ * LD + qI];
        // columns (X J_J), then rows (J_I^T Y)
        const T y00 = cJ * x00 - sJ * x01, y01 = sJ * x00 + cJ * x01;
        const T y10 = cJ * x10 - sJ * x11, y11 = sJ * x10 + cJ * x11;
        T z00 = cI * y00 - sI * y10, z10 = sI * y00 + cI * y10;
        T z01 = cI * y01 - sI * y11, z11 = sI * y01 + cI * y11;
        if (bI == bJ) {
          if ((rmask[cur] >> bI) & 1u) {
            const T tI = tnb[cur][bI];
            z00 = x00 - tI * x01;
            z11 = x11 + tI * x01;
            z01 = T(0);
          } else {
            z01 = T(0.5) * (z01 + z10);
          }
          z10 = z01;
        }
        A[pJ * LD + pI] = z00;
        A[qJ * LD + pI] = z01;
        A[pJ * LD + qI] = z10;
        A[qJ * LD + qI] = z11;
        if (bI != bJ) {  // the mirrored block
          A[pI * LD + pJ] = z00;
          A[pI * LD + qJ] = z01;
          A[qI * LD + pJ] = z10;
          A[qI * LD + qJ] = z11;
        }
      }
      prev_t = t;
      prev_buf = cur;
      __syncthreads();
    }
    // Read after the sweep's last barrier: the same values in every thread.
    // Stop after a sweep without rotations, or after one whose rotations all
    // had scaled off-diagonals |a_pq| / sqrt(a_pp a_qq) <= sqrt(eps): cyclic
    // Jacobi converges quadratically, so the off-diagonal it leaves is
    // O(eps) relative to the diagonal, and another sweep would only confirm.
    if (rotflag[sweep % 3] == 0 || bigflag[sweep % 3] == 0) break;
  }
  if (prev_t >= 0) {
    if (vtask) v_rot(prev_t, prev_buf, vi, vJ);
    if (vtask2) v_rot(prev_t, prev_buf, vi2, vJ2);
  }
  __syncthreads();
  // sort descending (stable by index), rank rule, write out
  for (int i = tid; i < N; i += NT) {
    const T li = A[i * LD + i];
    int pos = 0;
    for (int j = 0; j < N; ++j) {
      const T lj = A[j * LD + j];
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
    for (int i = tid; i < N; i += NT) tk_.lam[i] = lam_s[i];
  if (tk_.V)
    for (int e = tid; e < N * N; e += NT) {
      const int i = e / N, r = e % N;  // source column i, row r
      const int pos = posv[i];
      tk_.V[r + (size_t)pos * N] = pos < rkeep ? V[i * LDV + r] : T(0);
    }
}

// Rank certificate of the effective-rank rule, one workgroup per mode (the
// statement is next to its declaration).  The Cholesky factorisation of
// H - theta I follows the right-looking form of the Cholesky-QR kernel: every
// thread reads the pivot after the step's barrier, so all threads stop at the
// same failed pivot; lane j owns column j of the trailing update and the
// waves stride over its rows.
constexpr int CERT_NT = 256;
constexpr int CERT_MAX = 64;

// certificates tried and passed since the library was loaded (per device)
__device__ unsigned long long g_cert_count[2];

template <typename T>
__global__ __launch_bounds__(CERT_NT) void rank_cert_kernel(const T* __restrict__ H, const double* __restrict__ w,
                                                            const double* __restrict__ fro, int nb_act,
                                                            const double* __restrict__ tau_dev, CertParams cp,
                                                            int* __restrict__ cert, int* __restrict__ rt) {
  constexpr int NW = CERT_NT / kWave;
  __shared__ double G[CERT_MAX][CERT_MAX + 1];
  __shared__ double red[NW];
  const int k = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  const int m = cp.cap;
  const int nb = min(cp.nb, nb_act);
  double part = 0.0;
  for (int b = tid; b < nb; b += CERT_NT) part += w[b] * w[b] * fro[(size_t)k * cp.nb + b];
  const double tr = block_sum(part, red);
  const double tau = *tau_dev;
  const double theta = (4.0 * fmax(cp.delta, tau * tau) + cp.rnd[k]) * tr;
  const T* Hk = H + (size_t)k * m * m;
  for (int e = tid; e < m * m; e += CERT_NT) {
    const int i = e % m, j = e / m;
    G[i][j] = double(Hk[i + (size_t)j * m]) - (i == j ? theta : 0.0);
  }
  __syncthreads();
  bool ok = tr > 0.0 && tr < INFINITY;  // the same in every thread
  const int j = lane;
  for (int kk = 0; kk < m && ok; ++kk) {
    const double pv = G[kk][kk];
    if (!(pv > 0.0 && pv < INFINITY)) {
      ok = false;
      break;
    }
    if (j > kk && j < m) {
      const double f = G[kk][j] / pv;
      for (int i = kk + 1 + wave; i <= j; i += NW) G[i][j] -= G[kk][i] * f;
    }
    __syncthreads();
  }
  if (tid == 0) {
    cert[k] = ok ? 1 : 0;
    if (ok)
      for (int i = 0; i < cp.d; ++i) rt[i] = cp.cap;
    atomicAdd(&g_cert_count[0], 1ull);
    if (ok) atomicAdd(&g_cert_count[1], 1ull);
  }
}

}  // namespace

template <typename T>
void jacobi_eig(const EigTask<T>* tasks_d, int ntasks, int N, bool want_v, hipStream_t st, int in_splits) {
  if (ntasks <= 0 || N <= 0) return;
  // algorithmic work of a symmetric eigendecomposition of order N: 9 N^3 with
  // eigenvectors (symmetric QR algorithm count), (4/3) N^3 for the tridiagonal
  // reduction behind the eigenvalues-only path.  Bytes: the lower triangle of
  // every input slab (the matrix, or each split-K partial that the load sums),
  // plus the eigenvalues and, with vectors, the N x N eigenvectors.
  const int kc = want_v ? kKcJacobi : kKcEigVals;
  const double nn = double(N);
  const double in_b = (want_v ? double(in_splits) * nn * (nn + 1.0) / 2.0 : nn * nn);
  timer_begin(kc, st, double(ntasks) * (want_v ? 9.0 : 4.0 / 3.0) * nn * nn * nn,
              double(ntasks) * sizeof(T) * (in_b + (want_v ? nn * nn : 0.0) + nn));
  if (want_v) {
    TK_CHECK(N <= VEC_NMAX, kErrUnsupported, "symmetric eigensolver: eigenvectors above size 64");
    hipLaunchKernelGGL((jacobi_blk_kernel<T>), dim3(ntasks), dim3(1024), 0, st, tasks_d, N);
  } else {
    TK_CHECK(N <= GM_NMAX, kErrUnsupported, "symmetric eigensolver: matrix larger than 512");
    if (N <= VAL_NMAX)
      hipLaunchKernelGGL((tridiag_reg_kernel<T, trg_nt<T>()>), dim3(ntasks), dim3(trg_nt<T>()), 0, st, tasks_d, N);
    else
      hipLaunchKernelGGL((tridiag_gm_kernel<T>), dim3(ntasks), dim3(1024), 0, st, tasks_d, N);
    // (the planner gives the order-512 path matrices with a leading dimension
    // that is a multiple of 4, in 256-byte aligned workspace blocks)
  }
  TK_LAUNCH_CHECK();
  timer_end(kc, st);
}

template <typename T>
void rank_certificate(const T* H, const double* w, const double* fro, int nb_active, const double* tau,
                      const CertParams& cp, int* cert, int* rt, hipStream_t st) {
  TK_CHECK(cp.cap >= 1 && cp.cap <= CERT_MAX && cp.d >= 1 && cp.d <= kMaxD && cp.nb >= 1 && nb_active >= 0,
           kErrUnsupported, "rank certificate: sizes out of range");
  timer_begin(kKcEigVals, st);
  hipLaunchKernelGGL((rank_cert_kernel<T>), dim3(cp.d), dim3(CERT_NT), 0, st, H, w, fro, nb_active, tau, cp, cert,
                     rt);
  TK_LAUNCH_CHECK();
  timer_end(kKcEigVals, st);
}

void rank_cert_counts(int64_t* tried, int64_t* passed) {
  unsigned long long h[2] = {0, 0};
  TK_HIP(hipMemcpyFromSymbol(h, HIP_SYMBOL(g_cert_count), sizeof(h), 0, hipMemcpyDeviceToHost));
  *tried = int64_t(h[0]);
  *passed = int64_t(h[1]);
}

template void rank_certificate<double>(const double*, const double*, const double*, int, const double*,
                                       const CertParams&, int*, int*, hipStream_t);
template void rank_certificate<float>(const float*, const double*, const double*, int, const double*,
                                      const CertParams&, int*, int*, hipStream_t);

template void jacobi_eig<double>(const EigTask<double>*, int, int, bool, hipStream_t, int);
template void jacobi_eig<float>(const EigTask<float>*, int, int, bool, hipStream_t, int);

}  // namespace tk
