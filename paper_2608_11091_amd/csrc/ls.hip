// Sketched least squares of sGMRES, updated one column at a time.
//
// M = [S^T vec(W_1), ..., S^T vec(W_k)] grows by one column per iteration.
// The kernel keeps a Householder QR of M: the new column is reflected by the
// k previous reflectors, a new reflector zeroes its tail, Q^T b_s is updated
// with it, and R y = (Q^T b_s)[:k] is solved by back substitution on one
// wave.  The residual ||M y - b_s|| is the norm of the tail of Q^T b_s,
// which does not suffer the cancellation of forming M y - b_s.  FP64
// throughout; one workgroup, thread i owns row i (s <= 256).  With
// regularisation on, ls_tikhonov then replaces y and the residual by the
// projected Tikhonov solution (below).
#include "kernels.hpp"

namespace tk {

namespace {

constexpr int LS_NT = 256;
constexpr int LS_KMAX = 64;  // columns per cycle (iterations per restart cycle)

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
  // this row of the k previous reflectors, staged in LDS with sixteen loads
  // in flight at a time (a load inside the barrier-separated loop below
  // would cost a full load latency per reflector); a row outside the sketch
  // reads row s - 1 and never uses it
  __shared__ double hvs[LS_KMAX * LS_NT];  // reflector j, row i at [j * LS_NT + i]
  __shared__ double taus[LS_KMAX];
  if (i < k) taus[i] = S.tau[i];  // read by all after block_sum's barriers
  {
    const size_t ic = (size_t)min(i, s - 1);
    for (int jb = 0; jb < k; jb += 16) {
      double t[16];
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (jb + u < k) t[u] = S.Hv[ic + (size_t)(jb + u) * s];
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (jb + u < k) hvs[(jb + u) * LS_NT + i] = t[u];
    }
  }
  const double cn = block_sum(x * x, red);
  // previous reflectors (each thread reads back only its own row)
  for (int j = 0; j < k; ++j) {
    const double v = (i == j) ? 1.0 : (i > j && i < s ? hvs[j * LS_NT + i] : 0.0);
    const double wsum = block_sum(v * x, red);
    x -= taus[j] * v * wsum;
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
  // back substitution on wave 0: lane r holds b_r and row r of R (columns
  // below k loaded up front, column k is this thread's new entry)
  if (w == 0) {
    const double rk = (i < k) ? x : (i == k ? beta : 0.0);
    double rrow[LS_KMAX];
#pragma unroll
    for (int r = 0; r < LS_KMAX; ++r)
      if (r < k) rrow[r] = S.R[lane + (size_t)r * kmax];
    double b = (lane <= k) ? q : 0.0;
#pragma unroll
    for (int r = LS_KMAX - 1; r >= 0; --r) {
      if (r > k) continue;
      const double rl = (r == k) ? rk : rrow[r];
      const double rr = __shfl(rl, r, 64);
      const double yr = __shfl(b, r, 64) / rr;
      if (lane == r) b = yr;
      else if (lane < r) b -= rl * yr;
    }
    if (lane <= k) {
      S.y[lane] = b;
      if (S.ysave) S.ysave[(size_t)k * kmax + lane] = b;
    }
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

// ---------------------------------------------------------------- Tikhonov
// Projected Tikhonov with GCV (Sec. 4.3) on the current factorisation
// M = Q R (K = k + 1 columns): the regularised y minimises
// ||R y - c||^2 + rho^2 + lambda^2 ||y||^2 with c = (Q^T b_s)[:K] and
// rho^2 = ||(Q^T b_s)[K:]||^2.
//
// SVD by one-sided Jacobi on X = [R^T; c^T] ((K+1) x K in LDS): rotating
// column pairs of R^T until they are orthogonal gives R^T U = W diag(sigma),
// and the same rotations turn the appended row c^T into beta_hat^T = c^T U.
// Then, with sigma_i = ||X[:K, i]|| and B_i = X[:K, i] = sigma_i W_i,
//   y_lambda = sum_i B_i beta_hat_i / (sigma_i^2 + lambda^2),
//   ||M y_lambda - b_s||^2 = sum_i (g_i beta_hat_i)^2 + rho^2,
//   G(lambda) = that / (1 + sum_i g_i)^2,   g_i = lambda^2 / (sigma_i^2 + lambda^2)
// (g_i = 1 where sigma_i = lambda = 0).  lambda minimises G: a log grid of
// kGcvGrid points over [1e-12, 1] sigma_1, then golden-section steps on
// the bracket around the grid minimum.  Column pairs follow the round-robin
// (circle) ordering, K/2 disjoint pairs per round on groups of 8 lanes.
constexpr int kTkLd = 66;           // LDS column stride (K + 1 <= 65 rows)
constexpr int kGcvGrid = 241;       // 20 points per decade
constexpr double kGcvDecades = 12.0;
constexpr int kGcvGolden = 60;
constexpr int kJacobiSweeps = 60;

// Sum over each aligned group of 8 lanes (all lanes active): quad_perm
// [1,0,3,2] and [2,3,0,1] give every lane its quad's sum, row_half_mirror
// (lane j <-> 7 - j within 8) adds the other quad's; every lane of the group
// ends with the same total.
__device__ __forceinline__ double group8_sum(double v) {
  v += dpp_mov<0xB1>(v);
  v += dpp_mov<0x4E>(v);
  v += dpp_mov<0x141>(v);
  return v;
}

__device__ __forceinline__ double gcv_g(double s2, double l2) {
  const double den = s2 + l2;
  return den > 0.0 ? l2 / den : 1.0;
}

__global__ __launch_bounds__(LS_NT) void ls_tikhonov_kernel(LsState S, int s, int kmax, int k, double conv_tol,
                                                            double lam_fixed) {
  __shared__ double X[64 * kTkLd];
  __shared__ double sg2[64], bh[64];
  __shared__ double red[LS_NT / kWave];
  __shared__ double wv[LS_NT / kWave];
  __shared__ int wi[LS_NT / kWave];
  __shared__ int rot_any;
  const int K = k + 1;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  for (int e = tid; e < K * (K + 1); e += LS_NT) {
    const int i = e / (K + 1), r = e - i * (K + 1);
    X[r + i * kTkLd] = (r < K) ? S.R[i + (size_t)r * kmax] : (i < s ? S.qtb[i] : 0.0);
  }
  const double q = (tid > k && tid < s) ? S.qtb[tid] : 0.0;
  const double rho2 = block_sum(q * q, red);  // also orders the LDS fill above

  // ---- one-sided Jacobi
  const int np = K + (K & 1), m = np - 1;
  const int g = tid >> 3, sub = tid & 7;
  // rotate when |c| > sqrt(K) u sqrt(a b), tested squared (no square roots)
  const double jtol2 = double(K) * 2.220446049250313e-16 * 2.220446049250313e-16;
  for (int sweep = 0; sweep < kJacobiSweeps && K > 1; ++sweep) {
    if (tid == 0) rot_any = 0;
    __syncthreads();
    for (int rnd = 0; rnd < m; ++rnd) {
      int p = K, qq = K;
      if (g < np / 2) {
        if (g == 0) {
          p = rnd;
          qq = m;
        } else {
          p = (rnd + g) % m;
          qq = (rnd - g + m) % m;
        }
      }
      const bool act = p < K && qq < K;
      double a = 0.0, b = 0.0, c = 0.0;
      if (act)
        for (int r = sub; r < K; r += 8) {
          const double x = X[r + p * kTkLd], y = X[r + qq * kTkLd];
          a = fma(x, x, a);
          b = fma(y, y, b);
          c = fma(x, y, c);
        }
      a = group8_sum(a);
      b = group8_sum(b);
      c = group8_sum(c);
      if (act && c * c > jtol2 * (a * b)) {
        const double zeta = (b - a) / (2.0 * c);
        const double az = fabs(zeta);
        const double t = (az > 1e150 ? 0.5 / az : 1.0 / (az + sqrt(1.0 + az * az))) * (zeta >= 0.0 ? 1.0 : -1.0);
        const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
        for (int r = sub; r <= K; r += 8) {
          const double x = X[r + p * kTkLd], y = X[r + qq * kTkLd];
          X[r + p * kTkLd] = cs * x - sn * y;
          X[r + qq * kTkLd] = sn * x + cs * y;
        }
        if (sub == 0) rot_any = 1;
      }
      __syncthreads();
    }
    const int any = rot_any;
    __syncthreads();
    if (!any) break;
  }
  if (tid < K) {
    double a = 0.0;
    for (int r = 0; r < K; ++r) {
      const double x = X[r + tid * kTkLd];
      a = fma(x, x, a);
    }
    sg2[tid] = a;
    bh[tid] = X[K + tid * kTkLd];
  }
  __syncthreads();
  double smax = 0.0;
  for (int i = 0; i < K; ++i) smax = fmax(smax, sg2[i]);
  const double s1 = sqrt(smax);

  // ---- lambda
  double lam;
  if (lam_fixed >= 0.0) {
    lam = lam_fixed;
  } else if (s1 == 0.0) {
    lam = 0.0;
  } else {
    const double e0 = log10(s1);
    // grid: thread j evaluates G(lambda_j)
    double gv = INFINITY;
    if (tid < kGcvGrid) {
      const double l = exp10(e0 - kGcvDecades * (1.0 - double(tid) / double(kGcvGrid - 1)));
      const double l2 = l * l;
      double num = 0.0, den = 0.0;
      for (int i = 0; i < K; ++i) {
        const double gi = gcv_g(sg2[i], l2);
        const double t = gi * bh[i];
        num = fma(t, t, num);
        den += gi;
      }
      gv = (num + rho2) / ((1.0 + den) * (1.0 + den));
    }
    // argmin, first index on ties
    double bv = gv;
    int bi = tid;
    for (int o = 1; o < 64; o <<= 1) {
      const double ov = __shfl_xor(bv, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ov < bv || (ov == bv && oi < bi)) {
        bv = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      wv[w] = bv;
      wi[w] = bi;
    }
    __syncthreads();
    double gmin = wv[0];
    int j = wi[0];
    for (int u = 1; u < LS_NT / kWave; ++u)
      if (wv[u] < gmin || (wv[u] == gmin && wi[u] < j)) {
        gmin = wv[u];
        j = wi[u];
      }
    // golden section in log10(lambda) on [e_{j-1}, e_{j+1}]; every wave runs
    // the same steps (lane i holds term i), so all threads agree
    const double s2l = lane < K ? sg2[lane] : 0.0;
    const double bhl = lane < K ? bh[lane] : 0.0;
    auto G = [&](double ex) {
      const double l = exp10(ex);
      const double gi = lane < K ? gcv_g(s2l, l * l) : 0.0;
      const double t = gi * bhl;
      const double num = wave_sum(t * t);
      const double den = wave_sum(gi);
      return (num + rho2) / ((1.0 + den) * (1.0 + den));
    };
    const double phi = 0.6180339887498949;
    double a = e0 - kGcvDecades * (1.0 - double(max(j - 1, 0)) / double(kGcvGrid - 1));
    double b = e0 - kGcvDecades * (1.0 - double(min(j + 1, kGcvGrid - 1)) / double(kGcvGrid - 1));
    double x1 = b - phi * (b - a), x2 = a + phi * (b - a);
    double f1 = G(x1), f2 = G(x2);
    for (int it = 0; it < kGcvGolden; ++it) {
      if (f1 < f2) {
        b = x2;
        x2 = x1;
        f2 = f1;
        x1 = b - phi * (b - a);
        f1 = G(x1);
      } else {
        a = x1;
        x1 = x2;
        f1 = f2;
        x2 = a + phi * (b - a);
        f2 = G(x2);
      }
    }
    const double em = 0.5 * (a + b);
    lam = G(em) <= gmin ? exp10(em) : exp10(e0 - kGcvDecades * (1.0 - double(j) / double(kGcvGrid - 1)));
  }
  const double l2 = lam * lam;

  // ---- y_lambda and the residual
  if (tid < K) {
    double y = 0.0;
    for (int i = 0; i < K; ++i) {
      const double den = sg2[i] + l2;
      if (den > 0.0) y = fma(X[tid + i * kTkLd], bh[i] / den, y);
    }
    S.y[tid] = y;
    if (S.ysave) S.ysave[(size_t)k * kmax + tid] = y;
  }
  if (w == 0) {
    const double gi = lane < K ? gcv_g(sg2[lane], l2) : 0.0;
    const double t = gi * (lane < K ? bh[lane] : 0.0);
    const double num = wave_sum(t * t);
    if (lane == 0) {
      const double res = sqrt(num + rho2) / *S.bs_norm;
      S.res[k] = res;
      if (S.lam) S.lam[k] = lam;
      S.flags[1] = res < conv_tol ? 1 : 0;
    }
  }
}

}  // namespace

void ls_tikhonov(const LsState& st_, int s, int kmax, int k, double conv_tol, double lam_fixed, hipStream_t st) {
  TK_CHECK(s <= LS_NT && kmax <= 64 && k < kmax, kErrUnsupported, "projected Tikhonov: sizes out of range");
  timer_begin(kKcTikhonov, st);
  hipLaunchKernelGGL(ls_tikhonov_kernel, dim3(1), dim3(LS_NT), 0, st, st_, s, kmax, k, conv_tol, lam_fixed);
  TK_LAUNCH_CHECK();
  timer_end(kKcTikhonov, st);
}

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
