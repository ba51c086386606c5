// Sketched least squares of sGMRES, updated one column at a time.
//
// M = [S^T vec(W_1), ..., S^T vec(W_k)] grows by one column per iteration.
// The kernel keeps a Householder QR of M: the new column is reflected by the
// k previous reflectors, a new reflector zeroes its tail, Q^T b_s is updated
// with it, and R y = (Q^T b_s)[:k] is solved by back substitution on one
// wave.  The residual ||M y - b_s|| is the norm of the tail of Q^T b_s,
// which does not suffer the cancellation of forming M y - b_s.  FP64
// throughout; one workgroup, thread i owns row i (s <= 256).
#include "kernels.hpp"

namespace tk {

namespace {

constexpr int LS_NT = 256;

__global__ __launch_bounds__(LS_NT) void ls_init_kernel(LsState S, int s) {
  const int i = threadIdx.x;
  if (i < s) S.qtb[i] = S.bs[i];
  if (i == 0) {
    *S.nrmM2 = 0.0;
    S.flags[0] = 0;
    S.flags[1] = 0;
  }
}

__global__ __launch_bounds__(LS_NT) void ls_add_kernel(LsState S, int s, int kmax, int k, double conv_tol,
                                                       double bd_tol) {
  __shared__ double red[LS_NT / kWave];
  __shared__ double red2[LS_NT / kWave];
  const int i = threadIdx.x;
  const int lane = i & 63, w = i >> 6;
  double x = i < s ? S.Mcol[i + (size_t)k * s] : 0.0;
  const double cn = block_sum(x * x, red);
  // previous reflectors
  for (int j = 0; j < k; ++j) {
    const double v = (i == j) ? 1.0 : (i > j && i < s ? S.Hv[i + (size_t)j * s] : 0.0);
    const double wsum = block_sum(v * x, red);
    x -= S.tau[j] * v * wsum;
  }
  // new reflector on x[k:]
  double va = (i == k) ? x : 0.0;
  double vn = (i > k) ? x * x : 0.0;
  va = wave_sum(va);
  vn = wave_sum(vn);
  __syncthreads();
  if (lane == 0) {
    red[w] = va;
    red2[w] = vn;
  }
  __syncthreads();
  double alpha = 0.0, xnorm2 = 0.0;
  for (int q = 0; q < LS_NT / kWave; ++q) {
    alpha += red[q];
    xnorm2 += red2[q];
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
  const double v = (i == k) ? 1.0 : (i > k ? x * scal : 0.0);
  if (i < s) S.Hv[i + (size_t)k * s] = (i > k) ? v : 0.0;
  if (i == 0) S.tau[k] = tau;
  if (i < kmax) S.R[i + (size_t)k * kmax] = (i < k) ? x : (i == k ? beta : 0.0);
  // Q^T b update
  double q = i < s ? S.qtb[i] : 0.0;
  const double wq = block_sum(v * q, red);
  q -= tau * v * wq;
  if (i < s) S.qtb[i] = q;
  const double tail2 = block_sum(i > k ? q * q : 0.0, red);
  __syncthreads();
  // back substitution on wave 0: lane r holds b_r
  if (w == 0) {
    double b = (lane <= k) ? S.qtb[lane] : 0.0;
    for (int r = k; r >= 0; --r) {
      const double rr = S.R[r + (size_t)r * kmax];
      const double yr = __shfl(b, r, 64) / rr;
      if (lane == r) b = yr;
      else if (lane < r) b -= S.R[lane + (size_t)r * kmax] * yr;
    }
    if (lane <= k) S.y[lane] = b;
  }
  if (i == 0) {
    const double nrm2 = *S.nrmM2 + cn;
    *S.nrmM2 = nrm2;
    const double res = sqrt(tail2) / *S.bs_norm;
    S.res[k] = res;
    if (fabs(beta) <= bd_tol * sqrt(nrm2)) S.flags[0] = 1;
    if (res < conv_tol) S.flags[1] = 1;
  }
}

}  // namespace

void ls_init(const LsState& st_, int s, hipStream_t st) {
  TK_CHECK(s <= LS_NT, kErrUnsupported, "sketched least squares: sketch size above 256");
  hipLaunchKernelGGL(ls_init_kernel, dim3(1), dim3(LS_NT), 0, st, st_, s);
  TK_LAUNCH_CHECK();
}

void ls_add_column(const LsState& st_, int s, int kmax, int k, double conv_tol, double breakdown_tol,
                   hipStream_t st) {
  TK_CHECK(kmax <= 64, kErrUnsupported, "sketched least squares: more than 64 iterations per cycle");
  timer_begin(kKcLs, st);
  hipLaunchKernelGGL(ls_add_kernel, dim3(1), dim3(LS_NT), 0, st, st_, s, kmax, k, conv_tol, breakdown_tol);
  TK_LAUNCH_CHECK();
  timer_end(kKcLs, st);
}

}  // namespace tk
