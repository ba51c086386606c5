// Householder QR of tall-skinny FP64 matrices, one workgroup per matrix.
//
// Thread t owns row t of the n x m matrix (n <= 512, m <= 64) in registers.
// Step j forms the reflector of column j (a block reduction of the column
// tail), then the row vector w = v^T A[:, j+1:] is reduced with a wave-level
// reduce-scatter (each lane ends with one column's wave partial, 63
// shuffles per wave) followed by an 8-way LDS sum in fixed order.  Q is then
// formed in place by backward accumulation of the reflectors.  Everything
// is deterministic: no atomics, fixed reduction trees.
#include "kernels.hpp"

namespace tk {

namespace {

constexpr int QR_NT = 512;
constexpr int QR_MC = 64;
constexpr int QR_NW = QR_NT / kWave;

// Sums p[c] over the workgroup for every c < 64 (p computed by `term(c)`),
// result in wv[c].  Uses red[QR_NW][64].
template <typename F>
__device__ __forceinline__ void column_sums(F term, double (*red)[QR_MC], double* wv) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  double p[32];
  {
    const bool up = lane & 32;
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      const double lo = term(i), hi = term(i + 32);
      const double send = up ? lo : hi, keep = up ? hi : lo;
      p[i] = keep + __shfl_xor(send, 32, 64);
    }
  }
#pragma unroll
  for (int h = 16; h >= 1; h >>= 1) {
    const bool up = lane & h;
#pragma unroll
    for (int i = 0; i < h; ++i) {
      const double lo = p[i], hi = p[i + h];
      const double send = up ? lo : hi, keep = up ? hi : lo;
      p[i] = keep + __shfl_xor(send, h, 64);
    }
  }
  red[w][lane] = p[0];  // wave partial of column `lane`
  __syncthreads();
  if (threadIdx.x < QR_MC) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < QR_NW; ++q) s += red[q][threadIdx.x];
    wv[threadIdx.x] = s;
  }
  __syncthreads();
}

__global__ __launch_bounds__(QR_NT) void qr_kernel(const QrTask* __restrict__ tasks, int n, int cap,
                                                   const int* __restrict__ m_dev) {
  __shared__ double red[QR_NW][QR_MC];
  __shared__ double wv[QR_MC];
  __shared__ double tau_s[QR_MC];
  __shared__ double r2[2][QR_NW];
  const QrTask tk_ = tasks[blockIdx.x];
  const int row = threadIdx.x;
  const int lane = row & 63, wid = row >> 6;
  int m = tk_.m ? *tk_.m : (m_dev ? *m_dev : cap);
  m = min(m, cap);
  m = min(m, n);

  double a[QR_MC];
#pragma unroll
  for (int c = 0; c < QR_MC; ++c) a[c] = (row < n && c < m) ? tk_.Y[row + (size_t)c * n] : 0.0;

  // ---------------- factorisation
  for (int j = 0; j < m; ++j) {
    double xj = 0.0;
#pragma unroll
    for (int c = 0; c < QR_MC; ++c) xj = (c == j) ? a[c] : xj;
    // alpha = A[j][j], xnorm^2 = sum_{i>j} A[i][j]^2, one two-value block reduction
    double va = (row == j) ? xj : 0.0;
    double vn = (row > j) ? xj * xj : 0.0;
    va = wave_sum(va);
    vn = wave_sum(vn);
    if (lane == 0) {
      r2[0][wid] = va;
      r2[1][wid] = vn;
    }
    __syncthreads();
    double alpha = 0.0, xnorm2 = 0.0;
#pragma unroll
    for (int q = 0; q < QR_NW; ++q) {
      alpha += r2[0][q];
      xnorm2 += r2[1][q];
    }
    double beta, tau, scal;
    if (xnorm2 == 0.0) {
      beta = alpha;
      tau = 0.0;
      scal = 0.0;
    } else {
      beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    const double vr = (row == j) ? 1.0 : (row > j ? xj * scal : 0.0);
    if (tau != 0.0) {
      column_sums([&](int c) { return c > j ? vr * a[c] : 0.0; }, red, wv);
      const double tv = tau * vr;
#pragma unroll
      for (int c = 0; c < QR_MC; ++c)
        if (c > j) a[c] -= tv * wv[c];
    } else {
      __syncthreads();  // keep r2 reads ahead of the next step's writes
    }
    const double nj = (row == j) ? beta : (row > j ? vr : xj);
#pragma unroll
    for (int c = 0; c < QR_MC; ++c) a[c] = (c == j) ? nj : a[c];
    if (row == 0) tau_s[j] = tau;
  }
  __syncthreads();

  // ---------------- R (upper triangle of the leading m x m block)
  if (tk_.R != nullptr && row < cap) {
#pragma unroll
    for (int c = 0; c < QR_MC; ++c)
      if (c < cap) tk_.R[row + (size_t)c * cap] = (row < m && c < m && c >= row) ? a[c] : 0.0;
  }

  // ---------------- Q, backward accumulation in place (LAPACK org2r order)
  for (int j = m - 1; j >= 0; --j) {
    const double tau = tau_s[j];
    double xj = 0.0;
#pragma unroll
    for (int c = 0; c < QR_MC; ++c) xj = (c == j) ? a[c] : xj;
    const double vr = (row == j) ? 1.0 : (row > j ? xj : 0.0);
    if (j < m - 1 && tau != 0.0) {
      column_sums([&](int c) { return (c > j && c < m) ? vr * a[c] : 0.0; }, red, wv);
      const double tv = tau * vr;
#pragma unroll
      for (int c = 0; c < QR_MC; ++c)
        if (c > j && c < m) a[c] -= tv * wv[c];
    }
    const double nj = (row == j) ? 1.0 - tau : (row > j ? -tau * xj : 0.0);
#pragma unroll
    for (int c = 0; c < QR_MC; ++c) a[c] = (c == j) ? nj : a[c];
  }
  if (row < n) {
#pragma unroll
    for (int c = 0; c < QR_MC; ++c)
      if (c < cap) tk_.Q[row + (size_t)c * n] = (c < m) ? a[c] : 0.0;
  }
}

// Column-pivoted Householder QR with a rank cut, for the per-factor blocks of
// the exact norm.  Each step picks the unchosen column with the largest
// remaining norm relative to its reference norm (the factor column before
// projection); once that ratio is <= drop_tol every remaining column is
// numerically inside the span already built, and the factorisation stops.
// Outputs Q (live columns in pivot order, zeros after) and R with
// R[j][c] = coefficient of input column c on basis column j, so that
// Y = Q R up to the dropped remainders.  Column bookkeeping uses 64-bit masks
// (uniform across the block), so all register indices stay static.
__global__ __launch_bounds__(QR_NT) void qr_piv_kernel(const QrPivTask* __restrict__ tasks, int n, int cap,
                                                       double drop_tol) {
  __shared__ double red[QR_NW][QR_MC];
  __shared__ double wv[QR_MC];
  __shared__ double fref2[QR_MC];
  __shared__ double tau_s[QR_MC];
  __shared__ double r2[2][QR_NW];
  __shared__ int piv_s[QR_MC];
  __shared__ int inv_s[QR_MC];
  __shared__ int ctl;
  const QrPivTask tk_ = tasks[blockIdx.x];
  const int row = threadIdx.x;
  const int lane = row & 63, wid = row >> 6;
  int m = tk_.m ? *tk_.m : cap;
  m = min(m, cap);
  const int kmax = min(m, n);

  double a[QR_MC];
#pragma unroll
  for (int c = 0; c < QR_MC; ++c) a[c] = (row < n && c < m) ? tk_.Y[row + (size_t)c * n] : 0.0;
  column_sums(
      [&](int c) {
        const double v = (row < n && c < m) ? (tk_.ref ? tk_.ref[row + (size_t)c * n] : a[c]) : 0.0;
        return v * v;
      },
      red, fref2);
  if (tk_.ref == nullptr) {
    // global cut: every column is measured against the largest input column
    if (row == 0) {
      double mx = 0.0;
      for (int c = 0; c < m; ++c) mx = fmax(mx, fref2[c]);
      for (int c = 0; c < m; ++c) fref2[c] = mx;
    }
    __syncthreads();
  }

  unsigned long long unch = m >= 64 ? ~0ull : ((1ull << m) - 1ull);
  int nlive = 0;
  for (int j = 0; j < kmax; ++j) {
    // squared norms (rows >= j) of the unchosen columns
    column_sums([&](int c) { return (((unch >> c) & 1ull) && row >= j) ? a[c] * a[c] : 0.0; }, red, wv);
    if (row == 0) {
      int best = -1;
      double br = 0.0;
      for (int c = 0; c < m; ++c) {
        if (!((unch >> c) & 1ull) || !(fref2[c] > 0.0)) continue;
        const double rel = wv[c] / fref2[c];
        if (rel > br) {
          br = rel;
          best = c;
        }
      }
      ctl = (best >= 0 && br > drop_tol * drop_tol) ? best : -1;
    }
    __syncthreads();
    const int p = ctl;
    if (p < 0) break;
    unch &= ~(1ull << p);
    double xj = 0.0;
#pragma unroll
    for (int c = 0; c < QR_MC; ++c) xj = (c == p) ? a[c] : xj;
    double va = (row == j) ? xj : 0.0;
    double vn = (row > j) ? xj * xj : 0.0;
    va = wave_sum(va);
    vn = wave_sum(vn);
    if (lane == 0) {
      r2[0][wid] = va;
      r2[1][wid] = vn;
    }
    __syncthreads();
    double alpha = 0.0, xnorm2 = 0.0;
#pragma unroll
    for (int q = 0; q < QR_NW; ++q) {
      alpha += r2[0][q];
      xnorm2 += r2[1][q];
    }
    double beta, tau, scal;
    if (xnorm2 == 0.0) {
      beta = alpha;
      tau = 0.0;
      scal = 0.0;
    } else {
      beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    const double vr = (row == j) ? 1.0 : (row > j ? xj * scal : 0.0);
    if (tau != 0.0) {
      column_sums([&](int c) { return ((unch >> c) & 1ull) ? vr * a[c] : 0.0; }, red, wv);
      const double tv = tau * vr;
#pragma unroll
      for (int c = 0; c < QR_MC; ++c)
        if ((unch >> c) & 1ull) a[c] -= tv * wv[c];
    } else {
      __syncthreads();  // keep r2 reads ahead of the next step's writes
    }
    const double nj = (row == j) ? beta : (row > j ? vr : xj);
#pragma unroll
    for (int c = 0; c < QR_MC; ++c) a[c] = (c == p) ? nj : a[c];
    if (row == 0) {
      tau_s[j] = tau;
      piv_s[j] = p;
    }
    nlive = j + 1;
  }
  __syncthreads();

  // ---------------- R: row j holds the coefficients on basis column j of every
  // input column chosen at step >= j or never chosen
  if (tk_.R != nullptr && row < cap) {
    unsigned long long ok = unch;
    for (int jj = row; jj < nlive; ++jj) ok |= 1ull << piv_s[jj];
#pragma unroll
    for (int c = 0; c < QR_MC; ++c)
      if (c < cap) tk_.R[row + (size_t)c * cap] = (row < nlive && c < m && ((ok >> c) & 1ull)) ? a[c] : 0.0;
  }
  if (tk_.Rt != nullptr && row < cap) {
    unsigned long long ok = unch;
    for (int jj = row; jj < nlive; ++jj) ok |= 1ull << piv_s[jj];
#pragma unroll
    for (int c = 0; c < QR_MC; ++c)
      if (c < cap) tk_.Rt[c + (size_t)row * cap] = (row < nlive && c < m && ((ok >> c) & 1ull)) ? a[c] : 0.0;
  }
  if (tk_.rank_out != nullptr && row == 0) *tk_.rank_out = nlive;

  // ---------------- Q, backward accumulation in place (reflector j stored in column piv[j])
  unsigned long long later = 0ull;
  for (int j = nlive - 1; j >= 0; --j) {
    const int p = piv_s[j];
    const double tau = tau_s[j];
    double xj = 0.0;
#pragma unroll
    for (int c = 0; c < QR_MC; ++c) xj = (c == p) ? a[c] : xj;
    const double vr = (row == j) ? 1.0 : (row > j ? xj : 0.0);
    if (later != 0ull && tau != 0.0) {
      column_sums([&](int c) { return ((later >> c) & 1ull) ? vr * a[c] : 0.0; }, red, wv);
      const double tv = tau * vr;
#pragma unroll
      for (int c = 0; c < QR_MC; ++c)
        if ((later >> c) & 1ull) a[c] -= tv * wv[c];
    }
    const double nj = (row == j) ? 1.0 - tau : (row > j ? -tau * xj : 0.0);
#pragma unroll
    for (int c = 0; c < QR_MC; ++c) a[c] = (c == p) ? nj : a[c];
    later |= 1ull << p;
  }
  // basis column j sits in register column piv[j]: write it through the
  // inverse permutation, then zero the columns beyond the rank
  if (row < QR_MC) inv_s[row] = -1;
  __syncthreads();
  if (row < nlive) inv_s[piv_s[row]] = row;
  __syncthreads();
  if (row < n) {
#pragma unroll
    for (int c = 0; c < QR_MC; ++c) {
      const int j = inv_s[c];
      if (j >= 0) tk_.Q[row + (size_t)j * n] = a[c];
    }
    for (int j = nlive; j < cap; ++j) tk_.Q[row + (size_t)j * n] = 0.0;
  }
}

constexpr int CH_NT = 256;
constexpr int CH_MAX = 64;

// Right-looking Cholesky of one small Gram in LDS (one workgroup per task),
// one barrier per step: every thread derives the pivot of step k from G[k][k]
// itself, and the trailing update G[i][j] -= G[k][i] G[k][j] / pivot (k < i
// <= j, lane = column j, waves stride over the rows i) reads row k unscaled,
// which no thread writes after step k.  Row k of R = row k / sqrt(pivot) is
// formed at the end.  A pivot that is not above max(dead_rel tr, dead_abs)
// marks a dead column: its row of R is zero and it updates nothing.
__global__ __launch_bounds__(CH_NT) void chol_kernel(const CholTask* __restrict__ tasks, int cap,
                                                     const int* __restrict__ m_dev, double shift, double dead_rel,
                                                     double dead_abs) {
  constexpr int NW = CH_NT / kWave;
  __shared__ double G[CH_MAX][CH_MAX + 1];
  __shared__ double red[NW];
  __shared__ double rk_s[CH_MAX];
  const CholTask tk_ = tasks[blockIdx.x];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  int m = m_dev ? *m_dev : cap;
  m = min(m, cap);
  for (int e = tid; e < cap * cap; e += CH_NT) {
    const int i = e % cap, j = e / cap;
    G[i][j] = (i < m && j < m) ? tk_.G[i + (size_t)j * cap] : 0.0;
  }
  __syncthreads();
  const double tr = block_sum(tid < m ? G[tid][tid] : 0.0, red);
  const double s = shift * tr;
  const double dtol = fmax(dead_rel * tr, dead_abs);
  if (tid < m) G[tid][tid] += s;
  __syncthreads();
  const int j = lane;  // this thread's column of the trailing update
  for (int k = 0; k < m; ++k) {
    const double pv = G[k][k];
    const bool dk = !(pv > dtol);
    if (tid == 0) rk_s[k] = dk ? 0.0 : sqrt(pv);
    if (!dk && j > k && j < m) {
      const double f = G[k][j] / pv;
      for (int i = k + 1 + wave; i <= j; i += NW) G[i][j] -= G[k][i] * f;
    }
    __syncthreads();
  }
  for (int e = tid; e < cap * cap; e += CH_NT) {
    const int i = e % cap, jj = e / cap;
    double r = 0.0;
    if (i < m && jj < m && i <= jj) {
      const double rkk = rk_s[i];
      r = rkk == 0.0 ? 0.0 : (i == jj ? rkk : G[i][jj] / rkk);
    }
    tk_.R[i + (size_t)jj * cap] = r;
  }
}

constexpr int TR_NT = 128;

// Q = Y R^{-1}: each thread owns one row of Y in registers (compile-time
// column indices) and runs the forward substitution q R = y.
__global__ __launch_bounds__(TR_NT) void trsm_rows_kernel(const TrsmTask* __restrict__ tasks, int n, int cap,
                                                          const int* __restrict__ m_dev) {
  __shared__ double R[CH_MAX][CH_MAX + 1];
  const TrsmTask tk_ = tasks[blockIdx.y];
  const int tid = threadIdx.x;
  int m = m_dev ? *m_dev : cap;
  m = min(m, cap);
  for (int e = tid; e < cap * cap; e += TR_NT) {
    const int i = e % cap, j = e / cap;
    R[i][j] = tk_.R[i + (size_t)j * cap];
  }
  __syncthreads();
  const int row = blockIdx.x * TR_NT + tid;
  if (row >= n) return;
  double q[CH_MAX];
#pragma unroll
  for (int j = 0; j < CH_MAX; ++j) q[j] = (j < m) ? tk_.Y[row + (size_t)j * n] : 0.0;
#pragma unroll
  for (int j = 0; j < CH_MAX; ++j) {
    if (j < m) {
      double acc = q[j];
#pragma unroll
      for (int k = 0; k < j; ++k) acc -= q[k] * R[k][j];
      const double rjj = R[j][j];
      q[j] = rjj != 0.0 ? acc / rjj : 0.0;
    }
  }
#pragma unroll
  for (int j = 0; j < CH_MAX; ++j)
    if (j < cap) tk_.Q[row + (size_t)j * n] = (j < m) ? q[j] : 0.0;
}

}  // namespace

void chol_batched(const CholTask* tasks_d, int ntasks, int cap, const int* m_dev, double shift, double dead_rel,
                  double dead_abs, hipStream_t st) {
  if (ntasks <= 0) return;
  TK_CHECK(cap <= CH_MAX, kErrUnsupported, "Cholesky-QR: more than 64 columns");
  timer_begin(kKcQr, st);
  hipLaunchKernelGGL(chol_kernel, dim3(ntasks), dim3(CH_NT), 0, st, tasks_d, cap, m_dev, shift, dead_rel, dead_abs);
  TK_LAUNCH_CHECK();
  timer_end(kKcQr, st);
}

void trsm_rows(const TrsmTask* tasks_d, int ntasks, int n, int cap, const int* m_dev, hipStream_t st) {
  if (ntasks <= 0) return;
  TK_CHECK(cap <= CH_MAX, kErrUnsupported, "Cholesky-QR: more than 64 columns");
  hipLaunchKernelGGL(trsm_rows_kernel, dim3(ceil_div(n, TR_NT), ntasks), dim3(TR_NT), 0, st, tasks_d, n, cap, m_dev);
  TK_LAUNCH_CHECK();
}

void qr_batched(const QrTask* tasks_d, int ntasks, int n, int cap, const int* m_dev, hipStream_t st) {
  if (ntasks <= 0) return;
  TK_CHECK(n <= QR_NT, kErrUnsupported, "Householder QR: more than 512 rows");
  TK_CHECK(cap <= QR_MC, kErrUnsupported, "Householder QR: more than 64 columns");
  timer_begin(kKcQr, st);
  hipLaunchKernelGGL(qr_kernel, dim3(ntasks), dim3(QR_NT), 0, st, tasks_d, n, cap, m_dev);
  TK_LAUNCH_CHECK();
  timer_end(kKcQr, st);
}

void qr_piv_batched(const QrPivTask* tasks_d, int ntasks, int n, int cap, double drop_tol, hipStream_t st) {
  if (ntasks <= 0) return;
  TK_CHECK(n <= QR_NT && cap <= QR_MC, kErrUnsupported, "pivoted QR: more than 512 rows or 64 columns");
  timer_begin(kKcQr, st);
  hipLaunchKernelGGL(qr_piv_kernel, dim3(ntasks), dim3(QR_NT), 0, st, tasks_d, n, cap, drop_tol);
  TK_LAUNCH_CHECK();
  timer_end(kKcQr, st);
}

}  // namespace tk
