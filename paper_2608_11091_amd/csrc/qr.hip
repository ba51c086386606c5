// Small dense factorisations of the hot path, one workgroup per matrix:
// Householder QR (plain and column-pivoted with a rank cut) of tall-skinny
// FP64 matrices, the Cholesky factor of a small Gram, and the row-wise
// triangular solve that turns a Gram's Cholesky factor into a basis.
// Everything is deterministic: no atomics, fixed reduction orders.
#include <algorithm>

#include "kernels.hpp"

namespace tk {

namespace {

// ---------------------------------------------------------------- Householder QR
// Column-distributed layout: lane c of every wave owns column c (c < 64) and
// wave w holds rows [RS w, RS w + RS) of it in registers (RS = 32 up to 256
// rows, 64 above), so a block of at most 8 waves covers n <= 512 rows.  Sums over rows are in-thread
// over the 32 rows plus one pass over the waves' partials in LDS (fixed
// order).  Every wave derives the pivot of a step from the same LDS partials,
// and the pivot column's lane of each wave hands the reflector of that
// wave's rows to the other lanes through a per-wave LDS slot (in-order LDS
// within a wave, no block barrier), so a factorisation step needs two
// barriers and a Q step one.
constexpr int QC_RS = 32;              // rows per wave up to 256 rows
constexpr int QC_MAXW = 16;
constexpr int QC_MAXROWS = 512;
constexpr int QC_NT_SMALL = 4 * kWave;
constexpr int QC_NT = 8 * kWave;
constexpr int QC_NT_BIG = 16 * kWave;

struct QrJob {
  const double* Y;
  const double* ref;
  double* Q;
  double* R;
  double* Rt;
  int* rank_out;
  int m;
};
__device__ __forceinline__ QrJob job_of(const QrTask& t, int cap, const int* m_dev) {
  QrJob j{t.Y, nullptr, t.Q, t.R, nullptr, nullptr, 0};
  j.m = t.m ? *t.m : (m_dev ? *m_dev : cap);
  return j;
}
__device__ __forceinline__ QrJob job_of(const QrPivTask& t, int cap, const int*) {
  QrJob j{t.Y, t.ref, t.Q, t.R, t.Rt, t.rank_out, 0};
  j.m = t.m ? *t.m : cap;
  return j;
}

// Sum of part[q][c] over the nw waves in fixed order (every wave gets the
// same result).
__device__ __forceinline__ double wave_partials_sum(const double (*part)[kWave], int nw, int c) {
  double s = 0.0;
#pragma unroll 2
  for (int q = 0; q < nw; ++q) s += part[q][c];
  return s;
}

// Eight independent accumulation chains combined by a fixed tree.
__device__ __forceinline__ double tree8(const double* s) {
  return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// PIV = false: plain Householder QR of the leading m columns (m from the task,
// else m_dev, else cap).  PIV = true: column pivoting by the largest remaining
// norm relative to the column's reference norm (or to the largest input
// column when the task has no reference) and a stop once that ratio is at or
// below drop_tol; R[j][c] is then the coefficient of input column c on basis
// column j.
//
// NTB is the largest block the instantiation is launched with and RS the
// rows each wave holds: at most 8 waves leave each thread at least 256
// registers (16 waves cap it at 128), so n <= 128 runs on up to 4 waves of
// 32 rows, n <= 256 on up to 8, and n <= 512 on 8 waves of 64 rows, except
// the pivoted form, whose extra state spills there: it takes 16 waves of 32
// rows with one select per row (the form with the smallest register need).
template <bool PIV, typename Task, int NTB, int RS>
__global__ __launch_bounds__(NTB) void qr_cols_kernel(const Task* __restrict__ tasks, int n, int cap,
                                                      double drop_tol, const int* __restrict__ m_dev) {
  static_assert(NTB / kWave * RS <= QC_MAXROWS && NTB / kWave <= QC_MAXW, "row blocks within the LDS arrays");
  __shared__ double pn1[QC_MAXW][kWave];  // per-wave sums of squares over rows >= j
  __shared__ double rowj[kWave];          // row j of every column
  __shared__ double pw[2][QC_MAXW][kWave];  // per-wave partials of v^T A
  __shared__ double fref2[kWave];
  __shared__ double tau_s[kWave];
  __shared__ int piv_s[kWave];
  __shared__ int step_of[kWave];
  __shared__ double vsh_all[QC_MAXROWS];  // reflector on each wave's rows
  // rows per chunk; a 16-wave block (n > 256 in the pivoted form) keeps one
  // select per row, the form whose register need is the smallest
  constexpr bool CHUNKED = NTB <= QC_NT;
  constexpr int QC_CH = 8;
  const QrJob jb = job_of(tasks[blockIdx.x], cap, m_dev);
  const int tid = threadIdx.x;
  const int c = tid & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane(tid / kWave);  // wave-uniform: row tests stay scalar
  const int nw = blockDim.x / kWave;
  const int r0 = w * RS;
  double* const vsh = vsh_all + w * RS;  // this wave's rows
  const int m = max(0, min(jb.m, cap));
  const int kmax = min(m, n);

  // unconditional loads at clamped indices (always inside the n x cap input),
  // masked afterwards: no per-row branches whose conditions stay live
  const int cl = min(c, cap - 1);
  const bool colin = c < m;
  double a[RS];
  double sref = 0.0;  // this thread's share of the squared reference norm
#pragma unroll
  for (int i = 0; i < RS; ++i) {
    const int r = r0 + i;
    const size_t at = (size_t)min(r, n - 1) + (size_t)cl * n;
    const bool in = colin && r < n;
    const double y = jb.Y[at];
    a[i] = in ? y : 0.0;
  }
  if (PIV) {
    if (jb.ref == nullptr) {
      // global cut: the reference columns are the input itself
#pragma unroll
      for (int i = 0; i < RS; ++i) sref += a[i] * a[i];
    } else {
      // reference columns read a chunk at a time, so that their loads do not
      // all hold registers beside the input's
#pragma unroll
      for (int q = 0; q < RS; q += QC_CH) {
#pragma unroll
        for (int i = q; i < q + QC_CH; ++i) {
          const int r = r0 + i;
          const size_t at = (size_t)min(r, n - 1) + (size_t)cl * n;
          const double v = (colin && r < n) ? jb.ref[at] : 0.0;
          sref += v * v;
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  // the pivot column's lane stores v on this wave's rows; the other lanes of
  // the wave read it back after a wave-scope fence
  // Rows are handled in chunks of QC_CH: the step's diagonal row t0 (relative
  // to the wave) is uniform, so a chunk lies wholly below it, wholly above
  // it, or holds it, and only that one chunk of the wave takes per-row
  // selects (uniform branches choose the case).
  auto publish = [&](bool own, int t0, double scale, double diag) {
    if constexpr (!CHUNKED) {
      if (own) {
#pragma unroll
        for (int i = 0; i < RS; ++i) vsh[i] = (i < t0) ? 0.0 : (i == t0 ? diag : a[i] * scale);
      }
    } else if (own) {
#pragma unroll
      for (int q = 0; q < RS; q += QC_CH) {
        if (t0 < q) {
#pragma unroll
          for (int i = q; i < q + QC_CH; ++i) vsh[i] = a[i] * scale;
        } else if (t0 >= q + QC_CH) {
#pragma unroll
          for (int i = q; i < q + QC_CH; ++i) vsh[i] = 0.0;
        } else {
#pragma unroll
          for (int i = q; i < q + QC_CH; ++i) vsh[i] = (i < t0) ? 0.0 : (i == t0 ? diag : a[i] * scale);
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  // column sums of squares over rows >= j, and row j of every column (from
  // the wave that holds it)
  auto norm_partials = [&](int j) {
    const int t0 = j - r0;
    double s1[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if constexpr (!CHUNKED) {
#pragma unroll
      for (int i = 0; i < RS; ++i) s1[i & 7] += (i >= t0) ? a[i] * a[i] : 0.0;
      pn1[w][c] = tree8(s1);
      if (t0 >= 0 && t0 < RS) {
        double x = 0.0;
#pragma unroll
        for (int i = 0; i < RS; ++i) x = (i == t0) ? a[i] : x;
        rowj[c] = x;
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < RS; q += QC_CH) {
      if (t0 < q) {
#pragma unroll
        for (int i = q; i < q + QC_CH; ++i) s1[i & 7] += a[i] * a[i];
      } else if (t0 < q + QC_CH) {  // the chunk holding row j
        double x = 0.0;
#pragma unroll
        for (int i = q; i < q + QC_CH; ++i) {
          s1[i & 7] += (i >= t0) ? a[i] * a[i] : 0.0;
          x = (i == t0) ? a[i] : x;
        }
        rowj[c] = x;
      }
    }
    pn1[w][c] = tree8(s1);
  };
  if (PIV) pw[0][w][c] = sref;
  if (tid < kWave) step_of[tid] = -1;
  norm_partials(0);
  __syncthreads();
  if (PIV) {
    if (w == 0) {
      double t = wave_partials_sum(pw[0], nw, c);
      if (jb.ref == nullptr) {
        // global cut: every column is measured against the largest input column
        t = wave_max(t);
      }
      fref2[c] = t;
    }
    __syncthreads();
  }

  // ---------------- factorisation
  bool alive = colin;  // this lane's column is still unchosen
  int nlive = 0;
  for (int j = 0; j < kmax; ++j) {
    const double n1 = wave_partials_sum(pn1, nw, c);
    int p = j;
    if (PIV) {
      double rel = (alive && fref2[c] > 0.0) ? n1 / fref2[c] : -1.0;
      if (!(rel >= 0.0)) rel = -1.0;  // NaN as well: every lane takes the same decision
      // the largest ratio (DPP reduction), then the lowest lane holding it
      const double best = wave_max(rel);
      const unsigned long long hit = __ballot(rel == best);
      const int idx = __ffsll((long long)hit) - 1;
      p = __builtin_amdgcn_readfirstlane(best > drop_tol * drop_tol ? idx : -1);
    }
    if (p < 0) break;
    // reflector of column p on rows >= j: beta = -sign(alpha) ||x||; the
    // column's norm over rows >= j is all that is needed besides alpha
    const double alpha = rowj[p];
    const double xx = rdlane(n1, p);
    double beta, tau, scal;
    if (xx == alpha * alpha) {  // nothing below the diagonal (to rounding): no reflection
      beta = alpha;
      tau = 0.0;
      scal = 0.0;
    } else {
      beta = -copysign(sqrt(xx), alpha);
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    if (tid == 0) {
      tau_s[j] = tau;
      piv_s[j] = p;
    }
    alive = alive && c != p;
    const int t0 = j - r0;
    const bool upd = tau != 0.0 && alive;
    publish(c == p, t0, scal, 1.0);
    double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if constexpr (!CHUNKED) {
#pragma unroll
      for (int i = 0; i < RS; ++i) s[i & 7] += vsh[i] * a[i];
    } else
#pragma unroll
    for (int q = 0; q < RS; q += QC_CH)
      if (t0 < q + QC_CH) {  // rows above the diagonal row carry v = 0
#pragma unroll
        for (int i = q; i < q + QC_CH; ++i) s[i & 7] += vsh[i] * a[i];
      }
    pw[0][w][c] = upd ? tree8(s) : 0.0;
    __syncthreads();
    const double wc = wave_partials_sum(pw[0], nw, c);
    const double tw = upd ? tau * wc : 0.0;
    // column p keeps its rows above j, takes beta at row j and the reflector
    // below; the other columns take a - tw v (a no-op above row j)
    const double keep = (c == p) ? 0.0 : 1.0;
    const double twp = (c == p) ? -1.0 : tw;
    if constexpr (!CHUNKED) {
#pragma unroll
      for (int i = 0; i < RS; ++i) {
        const double v = vsh[i];
        const double own = (i < t0) ? a[i] : (i == t0 ? beta : v);
        a[i] = (c == p) ? own : a[i] - tw * v;
      }
    } else
#pragma unroll
    for (int q = 0; q < RS; q += QC_CH) {
      if (t0 < q) {
#pragma unroll
        for (int i = q; i < q + QC_CH; ++i) a[i] = fma(-twp, vsh[i], keep * a[i]);
      } else if (t0 < q + QC_CH) {
#pragma unroll
        for (int i = q; i < q + QC_CH; ++i) {
          const double v = vsh[i];
          const double own = (i < t0) ? a[i] : (i == t0 ? beta : v);
          a[i] = (c == p) ? own : a[i] - tw * v;
        }
      }
    }
    nlive = j + 1;
    norm_partials(j + 1);
    __syncthreads();
  }
  if (tid < nlive) step_of[piv_s[tid]] = tid;
  __syncthreads();

  // ---------------- R (and its transpose): row jj of every column
  if (jb.R != nullptr || jb.Rt != nullptr) {
#pragma unroll
    for (int i = 0; i < RS; ++i) {
      const int row = r0 + i;
      if (row < cap && c < cap) {
        const int sc = step_of[c];
        const bool ok = PIV ? (row < nlive && c < m && (sc < 0 || sc >= row)) : (row < nlive && c < m && c >= row);
        const double val = ok ? a[i] : 0.0;
        if (jb.R) jb.R[row + (size_t)c * cap] = val;
        if (jb.Rt) jb.Rt[c + (size_t)row * cap] = val;
      }
    }
  }
  if (jb.rank_out != nullptr && tid == 0) *jb.rank_out = nlive;

  // ---------------- Q by backward accumulation; basis column j sits in column piv[j]
  if (jb.Q == nullptr) return;  // R only (uniform over the block)
  bool later = false;  // this lane's column already holds a finished basis column
  for (int j = nlive - 1; j >= 0; --j) {
    const int p = piv_s[j];
    const double tau = tau_s[j];
    const int t0 = j - r0;
    const int b = j & 1;
    const bool upd = later && tau != 0.0;
    publish(c == p, t0, 1.0, 1.0);
    double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if constexpr (!CHUNKED) {
#pragma unroll
      for (int i = 0; i < RS; ++i) s[i & 7] += vsh[i] * a[i];
    } else
#pragma unroll
    for (int q = 0; q < RS; q += QC_CH)
      if (t0 < q + QC_CH) {
#pragma unroll
        for (int i = q; i < q + QC_CH; ++i) s[i & 7] += vsh[i] * a[i];
      }
    pw[b][w][c] = upd ? tree8(s) : 0.0;
    __syncthreads();
    const double wc = wave_partials_sum(pw[b], nw, c);
    const double tw = upd ? tau * wc : 0.0;
    // column p becomes basis column j: 0 above row j, 1 - tau at row j,
    // -tau v below; the other columns take a - tw v
    const double keep = (c == p) ? 0.0 : 1.0;
    const double twp = (c == p) ? tau : tw;
    if constexpr (!CHUNKED) {
#pragma unroll
      for (int i = 0; i < RS; ++i) {
        const double v = vsh[i];
        const double own = (i < t0) ? 0.0 : (i == t0 ? 1.0 - tau : -tau * v);
        a[i] = (c == p) ? own : a[i] - tw * v;
      }
    } else
#pragma unroll
    for (int q = 0; q < RS; q += QC_CH) {
      if (t0 < q) {
#pragma unroll
        for (int i = q; i < q + QC_CH; ++i) a[i] = fma(-twp, vsh[i], keep * a[i]);
      } else if (t0 >= q + QC_CH) {
#pragma unroll
        for (int i = q; i < q + QC_CH; ++i) a[i] = keep * a[i];
      } else {
#pragma unroll
        for (int i = q; i < q + QC_CH; ++i) {
          const double v = vsh[i];
          const double own = (i < t0) ? 0.0 : (i == t0 ? 1.0 - tau : -tau * v);
          a[i] = (c == p) ? own : a[i] - tw * v;
        }
      }
    }
    later = later || c == p;
  }
  const int jj = step_of[c];
#pragma unroll
  for (int i = 0; i < RS; ++i) {
    const int row = r0 + i;
    if (row < n) {
      if (jj >= 0) jb.Q[row + (size_t)jj * n] = a[i];
      if (c >= nlive && c < cap) jb.Q[row + (size_t)c * n] = 0.0;
    }
  }
}

constexpr int CH_NT = 1024;  // 16 waves: a trailing-update column of at most 64 rows takes <= 4 entries per thread
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
    double g = 0.0;
    if (i < m && j < m) {
      if (tk_.part) {  // the Gram's split-K partials, summed in split order
        // (eight loads in flight at a time; the additions keep their order)
        const double* pp = tk_.part + i + (size_t)j * cap;
        int sp = 0;
        for (; sp + 8 <= tk_.splits; sp += 8) {
          double v[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) v[u] = pp[(sp + u) * tk_.pstride];
#pragma unroll
          for (int u = 0; u < 8; ++u) g += v[u];
        }
        for (; sp < tk_.splits; ++sp) g += pp[sp * tk_.pstride];
      } else {
        g = tk_.G[i + (size_t)j * cap];
      }
    }
    G[i][j] = g;
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
// column indices) and runs the forward substitution q R = y.  (A right-looking
// order, whose updates of a step are independent, measured slower: 35.6
// against 26.6 us at 512 x 53, its per-entry guards cost more than the
// dependency chain it breaks.)
__global__ __launch_bounds__(TR_NT) void trsm_rows_kernel(const TrsmTask* __restrict__ tasks, int n, int cap,
                                                          const int* __restrict__ m_dev) {
  __shared__ double R[CH_MAX][CH_MAX + 1];
  const TrsmTask tk_ = tasks[blockIdx.y];
  const int tid = threadIdx.x;
  int m = m_dev ? *m_dev : cap;
  m = min(m, cap);
  {
    // every load of R in flight at once, then the LDS writes
    constexpr int RPT = CH_MAX * CH_MAX / TR_NT;
    const GPtr<double> gr = (GPtr<double>)tk_.R;
    const int cc = cap * cap;
    double rv[RPT];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int e = tid + u * TR_NT;
      rv[u] = gr[e < cc ? e : 0];
    }
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int e = tid + u * TR_NT;
      if (e < cc) R[e % cap][e / cap] = rv[u];
    }
  }
  __syncthreads();
  const int row = blockIdx.x * TR_NT + tid;
  if (row >= n) return;
  double q[CH_MAX];
  const GPtr<double> gy = (GPtr<double>)tk_.Y;
#pragma unroll
  for (int j = 0; j < CH_MAX; ++j) q[j] = (j < m) ? gy[row + (size_t)j * n] : 0.0;
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
    if (j < cap) {
      const double qv = (j < m) ? q[j] : 0.0;
      tk_.Q[row + (size_t)j * n] = qv;
      if (tk_.Qf) tk_.Qf[row + (size_t)j * n] = float(qv);
    }
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

// Algorithmic flops of a launch at full column count m = min(cap, n): the
// Householder factorisation 2 n m^2 - (2/3) m^3, and as much again for the
// explicit thin Q.
static double qr_flops(int ntasks, int n, int cap, bool with_q) {
  const double m = std::min(cap, n), nn = n;
  const double f = 2.0 * nn * m * m - 2.0 / 3.0 * m * m * m;
  return ntasks * f * (with_q ? 2.0 : 1.0);
}

void qr_batched(const QrTask* tasks_d, int ntasks, int n, int cap, const int* m_dev, hipStream_t st) {
  if (ntasks <= 0) return;
  TK_CHECK(n >= 1 && n <= QC_MAXROWS, kErrUnsupported, "Householder QR: more than 512 rows");
  TK_CHECK(cap <= kWave, kErrUnsupported, "Householder QR: more than 64 columns");
  timer_begin(kKcQr, st, qr_flops(ntasks, n, cap, true));
  if (n <= 4 * QC_RS)
    hipLaunchKernelGGL((qr_cols_kernel<false, QrTask, QC_NT_SMALL, QC_RS>), dim3(ntasks),
                       dim3(kWave * ceil_div(n, QC_RS)), 0, st, tasks_d, n, cap, 0.0, m_dev);
  else if (n <= 8 * QC_RS)
    hipLaunchKernelGGL((qr_cols_kernel<false, QrTask, QC_NT, QC_RS>), dim3(ntasks), dim3(kWave * ceil_div(n, QC_RS)),
                       0, st, tasks_d, n, cap, 0.0, m_dev);
  else
    hipLaunchKernelGGL((qr_cols_kernel<false, QrTask, QC_NT, 2 * QC_RS>), dim3(ntasks),
                       dim3(kWave * ceil_div(n, 2 * QC_RS)), 0, st, tasks_d, n, cap, 0.0, m_dev);
  TK_LAUNCH_CHECK();
  timer_end(kKcQr, st);
}

void qr_piv_batched(const QrPivTask* tasks_d, int ntasks, int n, int cap, double drop_tol, hipStream_t st) {
  if (ntasks <= 0) return;
  TK_CHECK(n >= 1 && n <= QC_MAXROWS && cap <= kWave, kErrUnsupported,
           "pivoted QR: more than 512 rows or 64 columns");
  timer_begin(kKcQr, st, qr_flops(ntasks, n, cap, true));
  if (n <= 4 * QC_RS)
    hipLaunchKernelGGL((qr_cols_kernel<true, QrPivTask, QC_NT_SMALL, QC_RS>), dim3(ntasks),
                       dim3(kWave * ceil_div(n, QC_RS)), 0, st, tasks_d, n, cap, drop_tol, nullptr);
  else if (n <= 8 * QC_RS)
    hipLaunchKernelGGL((qr_cols_kernel<true, QrPivTask, QC_NT, QC_RS>), dim3(ntasks), dim3(kWave * ceil_div(n, QC_RS)),
                       0, st, tasks_d, n, cap, drop_tol, nullptr);
  else  // the pivoted form would spill with 64 rows per wave: 16 waves of 32
    hipLaunchKernelGGL((qr_cols_kernel<true, QrPivTask, QC_NT_BIG, QC_RS>), dim3(ntasks),
                       dim3(kWave * ceil_div(n, QC_RS)), 0, st, tasks_d, n, cap, drop_tol, nullptr);
  TK_LAUNCH_CHECK();
  timer_end(kKcQr, st);
}

}  // namespace tk
