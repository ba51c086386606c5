// Small symmetric eigensolvers, one workgroup per matrix.
//
//  * Eigenvalues only (N <= 160): Householder reduction to tridiagonal form in
//    LDS (packed lower triangle, one thread per row for the symmetric
//    matrix-vector product and the rank-2 update), then every eigenvalue by
//    bisection on Sturm counts, one thread per eigenvalue.  Used by the
//    RoundSum effective-rank rule, which needs the spectrum but no vectors.
//  * Eigenvalues and vectors (N <= 64): cyclic Jacobi with the round-robin
//    parallel ordering, full matrix and eigenvector block in LDS.  Each step
//    applies N/2 disjoint rotations to all 2x2 blocks at once (2-D thread
//    layout, no index decoding).  A rotation is taken only when
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
constexpr int VEC_NMAX = 64;
constexpr int VEC_TX = 32, VEC_TY = 16;  // 512 threads

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
template <typename T>
__device__ int sturm_count(const T* d, const T* e2, int n, T x, T pivmin) {
  // number of eigenvalues of the tridiagonal (d, e) smaller than x
  int c = 0;
  T q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  c += q < T(0);
  for (int k = 1; k < n; ++k) {
    q = d[k] - x - e2[k - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    c += q < T(0);
  }
  return c;
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
      // p = tau * A_sub v, one thread per row of the trailing block
      if (tid < m) {
        const int gi = j + 1 + tid;
        T acc = T(0);
        for (int k = 0; k < m; ++k) acc += A[pk(gi, j + 1 + k)] * v[k];
        p[tid] = tau * acc;
      }
      __syncthreads();
      const T kk = block_sum(tid < m ? v[tid] * p[tid] : T(0), red) * T(0.5) * tau;
      if (tid < m) p[tid] = p[tid] - kk * v[tid];  // w = p - K v
      __syncthreads();
      if (tid < m) {  // A_sub -= v w^T + w v^T (lower part, row tid)
        const int gi = j + 1 + tid;
        const T vi = v[tid], wi = p[tid];
        for (int k = 0; k <= tid; ++k) A[pk(gi, j + 1 + k)] -= vi * p[k] + wi * v[k];
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
  for (int k = tid; k + 1 < N; k += VAL_NT) ee[k] = ee[k] * ee[k];
  __syncthreads();
  // ---- bisection, one thread per eigenvalue (ascending index i)
  const T bnorm = fmax(fabs(gl), fabs(gu));
  const T pivmin = fmax(Lim<T>::tiny(), emax2 * Lim<T>::tiny() * T(1e10));
  const T tolx = T(2) * Lim<T>::eps() * bnorm;
  for (int i = tid; i < N; i += VAL_NT) {
    T lo = gl - tolx, hi = gu + tolx;
    for (int it = 0; it < 200 && hi - lo > tolx; ++it) {
      const T mid = T(0.5) * (lo + hi);
      if (mid <= lo || mid >= hi) break;
      if (sturm_count(dd, ee, N, mid, pivmin) > i) hi = mid;
      else lo = mid;
    }
    lam[N - 1 - i] = T(0.5) * (lo + hi);
  }
  __syncthreads();
  if (tk_.lam)
    for (int i = tid; i < N; i += VAL_NT) tk_.lam[i] = lam[i];
  if (tid == 0 && tk_.rule.kind != 0) *tk_.rule.rank_out = apply_rule<T>(tk_.rule, lam, N);
}

// ------------------------------------------------------------ eigenvalues + vectors
__device__ __forceinline__ int player(int s, int t, int NP) { return s == 0 ? 0 : ((s - 1 + t) % (NP - 1)) + 1; }

template <typename T>
__global__ __launch_bounds__(VEC_TX* VEC_TY) void jacobi_vec_kernel(const EigTask<T>* __restrict__ tasks, int N) {
  constexpr int LD = VEC_NMAX + 1;
  constexpr int HM = VEC_NMAX / 2 + 1;
  __shared__ T A[VEC_NMAX][LD];
  __shared__ T V[VEC_NMAX][LD];  // V[col][row]
  __shared__ T rc[HM], rs[HM], rt[HM];
  __shared__ int rp[HM], rq[HM], rflag[HM];
  __shared__ int anyrot, rank_s;
  __shared__ int posv[VEC_NMAX];
  __shared__ T lam_s[VEC_NMAX];
  const EigTask<T> tk_ = tasks[blockIdx.x];
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int tid = ty * VEC_TX + tx;
  const int NT = VEC_TX * VEC_TY;
  const int NP = N + (N & 1);
  const int H = NP / 2;
  for (int e = tid; e < N * N; e += NT) {
    const int i = e % N, j = e / N;
    A[i][j] = (i >= j) ? tk_.A[i + (size_t)j * tk_.lda] : tk_.A[j + (size_t)i * tk_.lda];
    V[j][i] = (i == j) ? T(1) : T(0);
  }
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) anyrot = 0;
    __syncthreads();
    for (int t = 0; t < NP - 1; ++t) {
      if (tid < H) {
        const int P = tid;
        int p = player(P, t, NP), q = player(NP - 1 - P, t, NP);
        if (p > q) {
          const int x = p;
          p = q;
          q = x;
        }
        T c = T(1), s = T(0), tt = T(0);
        int flag = 0;
        if (q < N) {
          const T app = A[p][p], aqq = A[q][q], apq = A[p][q];
          const T aa = fabs(apq);
          if (aa > Lim<T>::tiny() && aa > Lim<T>::eps() * sqrt(fabs(app * aqq))) {
            const T theta = (aqq - app) / (T(2) * apq);
            if (fabs(theta) > T(1e15)) tt = T(0.5) / theta;
            else tt = (theta >= T(0) ? T(1) : T(-1)) / (fabs(theta) + sqrt(theta * theta + T(1)));
            c = T(1) / sqrt(tt * tt + T(1));
            s = tt * c;
            flag = 1;
            anyrot = 1;
          }
        }
        rc[P] = c;
        rs[P] = s;
        rt[P] = tt;
        rp[P] = p;
        rq[P] = q;
        rflag[P] = flag;
      }
      __syncthreads();
      // A <- J^T A J on every 2x2 block (both triangles), V <- V J
      for (int P = ty; P < H; P += VEC_TY) {
        const int f1 = rflag[P];
        const int p1 = rp[P], q1 = rq[P];
        const T c1 = rc[P], s1 = rs[P];
        for (int Q = tx; Q < H; Q += VEC_TX) {
          const int f2 = rflag[Q];
          if (!f1 && !f2) continue;
          if (P == Q) {
            const T apq = A[p1][q1];
            const T tt = rt[P];
            A[p1][p1] -= tt * apq;
            A[q1][q1] += tt * apq;
            A[p1][q1] = T(0);
            A[q1][p1] = T(0);
            continue;
          }
          const int p2 = rp[Q], q2 = rq[Q];
          const T c2 = rc[Q], s2 = rs[Q];
          const bool v1 = q1 < N, v2 = q2 < N;
          const T x00 = A[p1][p2];
          const T x01 = v2 ? A[p1][q2] : T(0);
          const T x10 = v1 ? A[q1][p2] : T(0);
          const T x11 = (v1 && v2) ? A[q1][q2] : T(0);
          const T y00 = c2 * x00 - s2 * x01, y01 = s2 * x00 + c2 * x01;
          const T y10 = c2 * x10 - s2 * x11, y11 = s2 * x10 + c2 * x11;
          A[p1][p2] = c1 * y00 - s1 * y10;
          if (v2) A[p1][q2] = c1 * y01 - s1 * y11;
          if (v1) A[q1][p2] = s1 * y00 + c1 * y10;
          if (v1 && v2) A[q1][q2] = s1 * y01 + c1 * y11;
        }
      }
      for (int P = ty; P < H; P += VEC_TY) {
        if (!rflag[P]) continue;
        const int p = rp[P], q = rq[P];
        const T c = rc[P], s = rs[P];
        for (int r = tx; r < N; r += VEC_TX) {
          const T vp = V[p][r], vq = V[q][r];
          V[p][r] = c * vp - s * vq;
          V[q][r] = s * vp + c * vq;
        }
      }
      __syncthreads();
    }
    if (anyrot == 0) break;
    __syncthreads();
  }
  // sort descending (stable by index), rank rule, write out
  for (int i = tid; i < N; i += NT) {
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
    for (int i = tid; i < N; i += NT) tk_.lam[i] = lam_s[i];
  if (tk_.V)
    for (int e = tid; e < N * N; e += NT) {
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
  timer_begin(kKcJacobi, st);
  if (want_v) {
    TK_CHECK(N <= VEC_NMAX, kErrUnsupported, "symmetric eigensolver: eigenvectors above size 64");
    hipLaunchKernelGGL((jacobi_vec_kernel<T>), dim3(ntasks), dim3(VEC_TX, VEC_TY), 0, st, tasks_d, N);
  } else {
    TK_CHECK(N <= VAL_NMAX, kErrUnsupported, "symmetric eigensolver: matrix larger than 160");
    static bool attr_set[2] = {false, false};
    bool& done = attr_set[sizeof(T) == 8];
    if (!done) {
      TK_HIP(hipFuncSetAttribute((const void*)tridiag_bisect_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 int(vals_smem<T>(VAL_NMAX))));
      done = true;
    }
    hipLaunchKernelGGL((tridiag_bisect_kernel<T>), dim3(ntasks), dim3(VAL_NT), vals_smem<T>(N), st, tasks_d, N);
  }
  TK_LAUNCH_CHECK();
  timer_end(kKcJacobi, st);
}

template void jacobi_eig<double>(const EigTask<double>*, int, int, bool, hipStream_t);
template void jacobi_eig<float>(const EigTask<float>*, int, int, bool, hipStream_t);

}  // namespace tk
