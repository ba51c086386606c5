// Cyclic Jacobi eigensolver for small symmetric matrices, one workgroup per
// matrix, matrix (packed lower triangle) and optional eigenvectors in LDS.
//
// Each step applies N/2 disjoint plane rotations chosen by the round-robin
// tournament ordering: phase 1 computes the rotations from the diagonal 2x2
// blocks, phase 2 applies them to every 2x2 block of the matrix (one thread
// per block pair, no two threads touch the same element) and to the
// eigenvector columns.  A rotation is taken only when
// |a_pq| > eps * sqrt(|a_pp a_qq|), the relative criterion under which
// Jacobi resolves small eigenvalues of graded positive semidefinite
// matrices to high relative accuracy; a sweep without rotations ends the
// iteration.  Results are sorted in descending order and an optional rank
// rule (RoundSum effective rank / ST-HOSVD truncation) runs on the sorted
// spectrum.
#include <cfloat>

#include "kernels.hpp"

namespace tk {

namespace {

constexpr int EIG_NT = 1024;
constexpr int EIG_NMAX = 160;
constexpr int EIG_NMAX_V = 64;

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

// Player at slot `s` in round `t` of the round-robin tournament over NP players.
__device__ __forceinline__ int player(int s, int t, int NP) { return s == 0 ? 0 : ((s - 1 + t) % (NP - 1)) + 1; }

template <typename T, bool WANT_V>
__global__ __launch_bounds__(EIG_NT) void jacobi_kernel(const EigTask<T>* __restrict__ tasks, int NL) {
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
  T* A = reinterpret_cast<T*>(smem_raw);
  const int NPK = N * (N + 1) / 2;
  T* V = A + NPK;                            // N x N, V[c * N + r]
  const int NP = N + (N & 1);
  const int H = NP / 2;
  T* rc = V + (WANT_V ? N * N : 0);          // cos per pair
  T* rs = rc + H;                            // sin per pair
  T* rt = rs + H;                            // tan per pair
  int* rp = reinterpret_cast<int*>(rt + H);  // p per pair
  int* rq = rp + H;                          // q per pair
  int* rflag = rq + H;                       // rotated? per pair
  __shared__ int anyrot;
  __shared__ int rank_s;

  const int tid = threadIdx.x;
  for (int e = tid; e < NPK; e += EIG_NT) {
    // packed index e -> (i, j), i >= j
    int i = int((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
    while ((i * (i + 1)) / 2 > e) --i;
    while (((i + 1) * (i + 2)) / 2 <= e) ++i;
    const int j = e - (i * (i + 1)) / 2;
    A[e] = tk_.A[i + (size_t)j * tk_.lda];
  }
  if (WANT_V)
    for (int e = tid; e < N * N; e += EIG_NT) V[e] = (e / N == e % N) ? T(1) : T(0);
  __syncthreads();

  const int NB = H * (H + 1) / 2;
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (tid == 0) anyrot = 0;
    __syncthreads();
    for (int t = 0; t < NP - 1; ++t) {
      // ---- phase 1: rotations of the diagonal blocks
      for (int P = tid; P < H; P += EIG_NT) {
        int p = player(P, t, NP), q = player(NP - 1 - P, t, NP);
        if (p > q) {
          const int x = p;
          p = q;
          q = x;
        }
        T c = T(1), s = T(0), tt = T(0);
        int flag = 0;
        if (q < N) {
          const T app = A[pk(p, p)], aqq = A[pk(q, q)], apq = A[pk(p, q)];
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
      // ---- phase 2: A <- J^T A J on every 2x2 block, V <- V J
      for (int b = tid; b < NB; b += EIG_NT) {
        int Q = int((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
        while ((Q * (Q + 1)) / 2 > b) --Q;
        while (((Q + 1) * (Q + 2)) / 2 <= b) ++Q;
        const int P = b - (Q * (Q + 1)) / 2;  // P <= Q
        const int f1 = rflag[P], f2 = rflag[Q];
        if (!f1 && !f2) continue;
        const int p1 = rp[P], q1 = rq[P];
        if (P == Q) {
          const T apq = A[pk(p1, q1)];
          const T tt = rt[P];
          A[pk(p1, p1)] -= tt * apq;
          A[pk(q1, q1)] += tt * apq;
          A[pk(p1, q1)] = T(0);
          continue;
        }
        const int p2 = rp[Q], q2 = rq[Q];
        const T c1 = rc[P], s1 = rs[P], c2 = rc[Q], s2 = rs[Q];
        const bool v1 = q1 < N, v2 = q2 < N;
        T x00 = A[pk(p1, p2)];
        T x01 = v2 ? A[pk(p1, q2)] : T(0);
        T x10 = v1 ? A[pk(q1, p2)] : T(0);
        T x11 = (v1 && v2) ? A[pk(q1, q2)] : T(0);
        // columns (right rotation)
        T y00 = c2 * x00 - s2 * x01, y01 = s2 * x00 + c2 * x01;
        T y10 = c2 * x10 - s2 * x11, y11 = s2 * x10 + c2 * x11;
        // rows (left rotation)
        A[pk(p1, p2)] = c1 * y00 - s1 * y10;
        if (v2) A[pk(p1, q2)] = c1 * y01 - s1 * y11;
        if (v1) A[pk(q1, p2)] = s1 * y00 + c1 * y10;
        if (v1 && v2) A[pk(q1, q2)] = s1 * y01 + c1 * y11;
      }
      if (WANT_V) {
        for (int e = tid; e < N * H; e += EIG_NT) {
          const int r = e % N, P = e / N;
          if (!rflag[P]) continue;
          const int p = rp[P], q = rq[P];
          const T c = rc[P], s = rs[P];
          const T vp = V[p * N + r], vq = V[q * N + r];
          V[p * N + r] = c * vp - s * vq;
          V[q * N + r] = s * vp + c * vq;
        }
      }
      __syncthreads();
    }
    if (anyrot == 0) break;
    __syncthreads();
  }

  // ---- sort descending (stable by index) and write out
  T* lam_s = rc;  // reuse: needs N entries -> rc/rs/rt hold 3H >= N
  for (int i = tid; i < N; i += EIG_NT) {
    const T li = A[pk(i, i)];
    int pos = 0;
    for (int j = 0; j < N; ++j) {
      const T lj = A[pk(j, j)];
      pos += (lj > li) || (lj == li && j < i);
    }
    if (tk_.lam) tk_.lam[pos] = li;
    if (WANT_V && tk_.V) {
      for (int r = 0; r < N; ++r) tk_.V[r + (size_t)pos * NL] = V[i * N + r];
    }
  }
  __syncthreads();
  for (int i = tid; i < N; i += EIG_NT) {
    const T li = A[pk(i, i)];
    int pos = 0;
    for (int j = 0; j < N; ++j) {
      const T lj = A[pk(j, j)];
      pos += (lj > li) || (lj == li && j < i);
    }
    lam_s[pos] = li;
  }
  __syncthreads();

  // ---- rank rule on the sorted spectrum
  const EigRule& ru = tk_.rule;
  if (ru.kind != 0 && tid == 0) {
    int r = 0;
    if (ru.kind == 1) {
      const double l0 = double(lam_s[0]);
      if (N > 0 && l0 > 0.0) {
        double total = 0.0;
        for (int i = 0; i < N; ++i) {
          const double li = double(lam_s[i]);
          total += li > ru.delta * l0 ? li : 0.0;
        }
        const double tau = *ru.tau;
        const double thr = tau * tau * total;
        double tail = 0.0;
        r = N;
        for (int i = N - 1; i >= 0; --i) {
          const double li = double(lam_s[i]);
          tail += li > ru.delta * l0 ? li : 0.0;
          if (tail <= thr) r = i;
          else break;
        }
      }
    } else {
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
          const double li = double(lam_s[i]);
          tail += li > 0.0 ? li : 0.0;
          if (tail <= thr) r = i;
          else break;
        }
        if (r < 1) r = 1;
        if (r > ru.cap) r = ru.cap;
      }
    }
    *ru.rank_out = r;
    rank_s = r;
  }
  if (WANT_V && ru.kind == 2 && tk_.V) {
    __syncthreads();
    const int r = rank_s;
    for (int e = tid; e < N * N; e += EIG_NT) {
      const int c = e / N, row = e % N;
      if (c >= r) tk_.V[row + (size_t)c * NL] = T(0);
    }
  }
}

template <typename T, bool WANT_V>
size_t eig_smem(int N) {
  const int NP = N + (N & 1);
  const int H = NP / 2;
  return sizeof(T) * (size_t(N) * (N + 1) / 2 + (WANT_V ? size_t(N) * N : 0) + 3 * H) + sizeof(int) * 3 * H + 64;
}

}  // namespace

template <typename T>
void jacobi_eig(const EigTask<T>* tasks_d, int ntasks, int N, bool want_v, hipStream_t st) {
  if (ntasks <= 0 || N <= 0) return;
  TK_CHECK(N <= EIG_NMAX, kErrUnsupported, "Jacobi eigensolver: matrix larger than 160");
  TK_CHECK(!want_v || N <= EIG_NMAX_V, kErrUnsupported, "Jacobi eigensolver: eigenvectors above size 64");
  if (want_v) {
    const size_t sm = eig_smem<T, true>(N);
    TK_HIP(hipFuncSetAttribute((const void*)jacobi_kernel<T, true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm));
    hipLaunchKernelGGL((jacobi_kernel<T, true>), dim3(ntasks), dim3(EIG_NT), sm, st, tasks_d, N);
  } else {
    const size_t sm = eig_smem<T, false>(N);
    TK_HIP(hipFuncSetAttribute((const void*)jacobi_kernel<T, false>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm));
    hipLaunchKernelGGL((jacobi_kernel<T, false>), dim3(ntasks), dim3(EIG_NT), sm, st, tasks_d, N);
  }
  TK_LAUNCH_CHECK();
}

template void jacobi_eig<double>(const EigTask<double>*, int, int, bool, hipStream_t);
template void jacobi_eig<float>(const EigTask<float>*, int, int, bool, hipStream_t);

}  // namespace tk
