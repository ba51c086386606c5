// Launchers of the non-GEMM kernels of the Tucker sGMRES hot path.
#pragma once

#include "common.hpp"

namespace tk {

// Device pointers read from task tables are generic to the compiler; loads
// through this global address space alias are global loads rather than flat
// ones (a flat load also counts as an LDS operation, so every barrier's LDS
// wait would wait for it, and prefetches would not stay in flight).
template <typename T>
using GPtr = const __attribute__((address_space(1))) T*;

// ---- Khatri-Rao reductions (MTTKRP tail and Khatri-Rao sketch) -------------
// Z is a P x S column-major matrix whose rows are a row-major multi-index over
// m modes of sizes z[0..m-1].  For free position f (0 <= f < m) it computes
//   out[i_f + l * ldo] = sum_{i_j, j != f} Z[(i), l] * prod_{j != f} M_j[i_j, l]
// and for f < 0 the full contraction
//   out[l * ldo] = sum_{(i)} Z[(i), l] * prod_j M_j[i_j, l].
// Result = scale * (*coef) * value, added to out when accumulate != 0.
template <typename T>
struct KrpTask {
  const T* Z;
  const T* Mj[kMaxD];
  int ldm[kMaxD];
  T* out;
  const double* coef;
  double scale;
  int accumulate;
  int f;    // free position (or -1 for the full contraction)
  int ldo;  // leading dimension of out (stride between columns l)
};
// Mode sizes z[0..m-1] are uniform across the tasks of one launch.
template <typename T>
void krp_reduce(const KrpTask<T>* tasks_d, int ntasks, int m, const int* z, int P, int S, hipStream_t st);

// ---- reductions over flat vectors --------------------------------------------
// out[i] = sum_e x_i[e]^2 for i < n (x_i = base + i * stride), deterministic order.
template <typename T>
void sumsq_batched(const T* base, size_t stride, size_t len, int n, double* out, hipStream_t st);
// out[i] = |coef[i]| * sqrt(sumsq[i]) (RoundSum energy weights).
void block_weights(const double* coef, const double* sumsq, int n, double* w, hipStream_t st);
// out[i] = scale_i * sum_e x_i[e] * y_i[e]; x_i = xs[i], y_i = ys[i] (device pointer tables).
template <typename T>
void dot_batched(const T* const* xs, const T* const* ys, size_t len, int n, double scale, double* out,
                 hipStream_t st);

// ---- elementwise --------------------------------------------------------------
// y = alpha * x with alpha = scale * (*num) / (*den) (num/den optional device
// scalars; a denominator that is not positive and finite gives alpha = 0).
template <typename T>
void scale_copy(const T* x, T* y, size_t len, double scale, const double* num, const double* den,
                hipStream_t st);
template <typename T>
void fill(T* y, size_t len, T v, hipStream_t st);
// *count = number of non-finite entries over the arrays xs[t] (length lens[t],
// device tables of ntasks entries, maxlen >= every length).
void count_nonfinite(const double* const* xs, const size_t* lens, int ntasks, size_t maxlen, int* count,
                     hipStream_t st);
template <typename A, typename B>
void cast_copy(const A* x, B* y, size_t len, hipStream_t st);
// Up to kMaxD conversions y[i] = B(x[i]) of lengths len[i] in one launch.
template <typename A, typename B>
struct CastSet {
  const A* x[kMaxD];
  B* y[kMaxD];
  size_t len[kMaxD];
  int count = 0;
};
template <typename A, typename B>
void cast_multi(const CastSet<A, B>& set, hipStream_t st);
// Copy a d-way core between capacity layouts: src has layout dims sd[] of
// which the leading sv[] are valid, dst has layout dims dd[]; dst entries
// outside the valid region are zero.
template <typename T>
void core_recap(const T* src, const int* sd, const int* sv, T* dst, const int* dd, int d, hipStream_t st);
// Zero columns [*from_dev, cols) of a column-major rows x cols matrix.
template <typename T>
void zero_cols_from(T* A, int ld, int rows, int cols, const int* from_dev, hipStream_t st);
// One launch: columns >= s of the d factors U[k] (n[k] x sc, ld n[k]) and,
// unless core is null, every entry of the dense sc^d core (row-major) with an
// index >= s.
template <typename T>
struct WidthZero {
  T* U[kMaxD];
  int n[kMaxD];
  T* core;
};
template <typename T>
void zero_beyond_width(const WidthZero<T>& a, int d, int sc, const int* s_dev, hipStream_t st);
// The same zeroing with the width computed in the kernel from the kept ranks,
// as sketch_width does it, and written to *s_out.
template <typename T>
void width_and_zero(const WidthZero<T>& a, int d, int sc, const int* rt, int p, int cap, int force, int* s_out,
                    hipStream_t st);
// Side streams of the current device (created on first use: non-blocking,
// default priority) for work that a plan runs beside the caller's stream;
// `which` selects one of several independent ones.
hipStream_t side_stream(int which = 0);
// Copy the leading rows x cols of a column-major matrix (zero-filling dst beyond src).
template <typename T>
void mat_recap(const T* src, int ld_src, int rows_src, int cols_src, T* dst, int ld_dst, int rows_dst,
               int cols_dst, hipStream_t st);

// ---- Householder QR (one workgroup per matrix, rows in registers) ----------
// Y: n x cap col-major (ld n).  Active columns m = min(*m_dev (or cap), n).
// Writes Q (n x cap, zero columns >= m) and optionally R (cap x cap, col-major,
// upper triangle of the m x m factor, zero elsewhere).  n <= 512, cap <= 64.
struct QrTask {
  const double* Y;
  double* Q;          // or null: R only
  double* R;
  const int* m;  // optional per-task active column count (overrides m_dev)
};
void qr_batched(const QrTask* tasks_d, int ntasks, int n, int cap, const int* m_dev, hipStream_t st);

// Column-pivoted Householder QR with a rank cut (n <= 512, cap <= 64): columns
// whose remainder falls to <= drop_tol times their reference norm are left
// out of the basis.  Q: live basis columns in pivot order (zeros after);
// R[j][c]: coefficient of input column c on basis column j (cap x cap).
struct QrPivTask {
  const double* Y;    // n x cap, ld n
  const double* ref;  // n x cap, ld n: reference columns for the cut; null =
                      // the largest column of Y for every column (global cut)
  double* Q;          // n x cap, ld n, or null: R only
  double* R;          // cap x cap, or null
  const int* m;       // active columns (device), or null = cap
  double* Rt = nullptr;     // optional: R transposed (cap x cap, Rt[c][j] = R[j][c])
  int* rank_out = nullptr;  // optional: number of basis columns kept
};
void qr_piv_batched(const QrPivTask* tasks_d, int ntasks, int n, int cap, double drop_tol, hipStream_t st);

// ---- Cholesky-QR pieces (range-finder QR of RoundSum) ------------------------
// R = chol(G + s I) for the leading m x m block of a cap x cap Gram (m =
// min(*m_dev, cap)), with s = shift * trace(G).  A pivot that is not above
// max(dead_rel * trace(G), dead_abs) marks a numerically dependent column: its
// row of R is zeroed and the triangular solve below turns it into a zero
// basis column.
struct CholTask {
  const double* G;  // cap x cap, col-major
  double* R;        // cap x cap, col-major (upper triangle)
  // optional: G is not formed; its entries are the sums, in order, of
  // part[sp * pstride + i + j * cap] over sp < splits (split-K partials)
  const double* part = nullptr;
  int splits = 0;
  size_t pstride = 0;
};
void chol_batched(const CholTask* tasks_d, int ntasks, int cap, const int* m_dev, double shift, double dead_rel,
                  double dead_abs, hipStream_t st);
// Q = Y R^{-1} row by row (R upper triangular from chol_batched); columns
// >= m and dead columns of Q are zero.  Y, Q: n x cap col-major (ld n).
struct TrsmTask {
  const double* Y;
  const double* R;
  double* Q;
  float* Qf = nullptr;  // optional FP32 copy of Q (same layout), rounded to nearest
};
void trsm_rows(const TrsmTask* tasks_d, int ntasks, int n, int cap, const int* m_dev, hipStream_t st);

// ---- symmetric Jacobi eigensolver (one workgroup per matrix) ---------------
// A: N x N symmetric (lower triangle read, col-major, ld lda).  Eigenvalues
// sorted descending -> lam (N); eigenvectors -> V (N x N col-major, ld N) when
// V != nullptr (N <= 64).  Rank rule (optional, see EigRule).
struct EigRule {
  int kind;            // 0: none; 1: effective rank (RoundSum heuristic); 2: ST-HOSVD truncation
  const double* tau;   // kind 1: device energy threshold tau (tail <= tau^2 * total)
  double delta;        // kind 1: eigenvalues <= delta * lambda_max count as zero
  const double* eps;   // kind 2: device tolerance; threshold eps^2 * (*total) / d
  int d;               // kind 2
  int cap;             // kind 2: rank cap
  const double* total; // kind 2: ||C||_F^2 of the projected core
  const double* zthr;  // kind 2: total <= *zthr means a numerically zero sum (rank 1)
  const int* force;    // kind 2: forced rank (nullptr / negative = none)
  int* rank_out;       // resulting rank
  int cap1 = 0;        // kind 1: > 0 when only min(rank, cap1) is needed (and not the
                       // eigenvalues): rank_out may then be cap1 for any rank >= cap1
};
template <typename T>
struct EigTask {
  const T* A;
  int lda;
  T* lam;
  T* V;          // eigenvectors (ld = launch N); for rule kind 2 columns >= rank are zeroed
  const int* ndyn; // optional device size (< launch N); negative: skip, rank_out = -1
  const int* skip; // optional device flag: nonzero = do nothing (another task of the launch pair decides)
  const int* cert; // optional device flags cert[0..ncert): any nonzero = do nothing (the rank certificate decided)
  int ncert;
  EigRule rule;
  // optional (eigensolver with vectors): A is not formed; its entries are the
  // sums, in order sp = 0..splits-1, of part[sp * pstride + r + c * lda]
  // (the split-K partials of the product that would have written A)
  const T* part;
  int splits;
  size_t pstride;
};
// Eigenvalues only: N <= 512; above kEigRegMax the matrix is reduced in place
// (A must then be writable scratch).  With vectors: N <= 64.  in_splits is the
// number of split-K partials the tasks' loads sum (1 when they read A); it
// only enters the kernel timer's byte count.
constexpr int kEigRegMax = 160;
template <typename T>
void jacobi_eig(const EigTask<T>* tasks_d, int ntasks, int N, bool want_v, hipStream_t st, int in_splits = 1);

// Certificate for the effective-rank rule of RoundSum (Sec. 3.1), one task
// per mode k.  H_k = Q_k^T G_k Q_k (cap x cap, ld cap, T) is the compression of
// the rule's Gram G_k = sum_b w_b^2 U_bk U_bk^T onto the first cap columns of
// the range-finder basis Q_k; tr(G_k) = sum_{b < nb_active} w_b^2 fro[k nb + b]
// with fro the squared Frobenius norms of the factors (nb_active: the number
// of live blocks, a host value).  If H_k - theta_k I has
// a Cholesky factorisation, theta_k = (4 max(delta, tau^2) + rnd[k]) tr(G_k)
// (rnd[k]: bound on the rounding of H_k relative to tr(G_k)), then the cap-th
// eigenvalue of G_k exceeds both the zero clamp and the tail threshold, so
// r~_k >= cap and the sketch width is cap + p: cert[k] = 1 and rt[0..d) = cap.
// Otherwise cert[k] = 0 and rt is left alone.
struct CertParams {
  int d, cap, nb;
  double delta;
  double rnd[kMaxD];
};
// Certificates tried (one per mode) and passed on the current device since
// the library was loaded (synchronises the device).
void rank_cert_counts(int64_t* tried, int64_t* passed);
template <typename T>
void rank_certificate(const T* H, const double* w, const double* fro, int nb_active, const double* tau,
                      const CertParams& cp, int* cert, int* rt, hipStream_t st);

// Per mode k: R_k = sum_b rank_b[k]; enable[k] = (R_k <= rmax); nact[k] = R_k or -1.
// Then the padded Gram (blocks of rc rows/cols) is compacted to its R_k x R_k
// active part (ld = ldc) for every mode with enable[k] = 1.
// skip_small[k] = (R_k > rmax), skip_big[k] = (R_k <= rmax) when non-null.
void gram_prep(const int* const* ranks, int nb, int d, int rmax, double* enable, int* nact, hipStream_t st,
               int* skip_small = nullptr, int* skip_big = nullptr);
template <typename T>
void gram_compact(const T* padded, int ldp, const int* const* ranks, int nb, int d, int rc, const int* nact,
                  T* compact, int ldc, size_t mode_stride_p, size_t mode_stride_c, hipStream_t st);

// s_r = min(max_k (rt_k + p), cap + p), or *force when force >= 0; rt_k < 0 = skipped.
void sketch_width(const int* rt, int d, int p, int cap, int force, int* s_out, hipStream_t st);

// ---- small bookkeeping kernels ------------------------------------------------
// coef[b] = cscale[b] * (cptr[b] ? *cptr[b] : 1) for b < *nb (or nb_static).
void gather_coef(const double* const* cptr, const double* cscale, int nb, double* coef, hipStream_t st);
// If *total <= *zthr: ranks = 1, factor columns = e_1, core zero (capacity rc layout).
template <typename T>
void zero_sum_fixup(const double* total, const double* zthr, int d, const int* n, int rc, T* const* U, T* core,
                    size_t core_len, int* rank, hipStream_t st);
// zthr = (tol * sum_{b < nb} w[b])^2.
void zero_threshold(const double* w, int nb, double tol, double* zthr, hipStream_t st);
// gather_coef, block_weights and zero_threshold in one launch (one
// workgroup): coef[b], w[b] = |coef[b]| sqrt(sumsq[b]) and zthr.
void coef_weights_threshold(const double* const* cptr, const double* cscale, const double* sumsq, int nb, double tol,
                            double* coef, double* w, double* zthr, hipStream_t st);
// core_recap (no view limit) followed by zero_sum_fixup, in one launch.
template <typename T>
void core_recap_fixup(const T* src, const int* sd, T* dst, const int* dd, int d, const double* total,
                      const double* zthr, const int* n, int rc, T* const* U, int* rank, hipStream_t st);
// Y[:, :] += X[:, :] (rows x cols, col-major with their own leading dims).
template <typename T>
void mat_axpy(const T* X, int ldx, T* Y, int ldy, int rows, int cols, hipStream_t st);
// out[l] = sum_b base[b * stride + l] (fixed order), as double.
template <typename T>
void sum_vectors(const T* base, size_t stride, int nb, int len, double* out, hipStream_t st);
// Linear combinations of flat arrays, one task t < ntasks per output:
//   y[t][e] = (accumulate ? y[t][e] : 0) + sum_{j < min(nx, limit)} s[j] (*c[j]) x[t * nx + j][e]
// for e < len[t] (c[j] null = 1).  All tables are device arrays; nx <=
// kLincombMax; the outputs of one launch must not overlap any of its inputs.
constexpr int kLincombMax = 128;
template <typename T>
void lincomb(T* const* y, const T* const* x, const double* const* c, const double* s, const size_t* len,
             int ntasks, int nx, size_t maxlen, int accumulate, int limit, hipStream_t st);
// Row scaling by exponentials, one task per output: out[i + j*n] =
// exp(-t * (lam[i] - *shift)) * in[i + j*n] for i < n, j < cols (column-major, ld n).
template <typename T>
struct ExpScaleTask {
  const T* in;
  const T* lam;
  const double* shift;
  T* out;
  double t;
};
template <typename T>
void exp_scale_rows(const ExpScaleTask<T>* tasks_d, int ntasks, int n, int cols, hipStream_t st);
// Coefficients of the shifted exponential-sum terms: lmin[k] = min_i lam_k[i]
// (lam_k of length n[k], k < d) and coef[h] = eta t_h exp(-t_h sum_k lmin[k]),
// t_h = exp((h - q) eta), h < 2q + 1.
template <typename T>
void expsum_shift(const T* const* lam, const int* n, int d, int q, double eta, double* lmin, double* coef,
                  hipStream_t st);
// out[i] = src[i * stride] for i < n, as double.
template <typename T>
void strided_gather(const T* src, size_t stride, int n, double* out, hipStream_t st);
// dst[i] = max(src[i], lo) for i < n.
void ints_at_least(const int* src, int* dst, int n, int lo, hipStream_t st);
// Copy n ints.
void copy_ints(const int* src, int* dst, int n, hipStream_t st);
// dst[i] = sqrt(src[i]) for i < n.
void vec_sqrt(const double* src, double* dst, int n, hipStream_t st);
// col[0..nh) = h, col[nh] = sqrt(*norm2), zeros up to len (a Hessenberg column).
void hess_column(const double* h, int nh, const double* norm2, double* col, int len, hipStream_t st);
// v = (*beta) e_1, length len.
void scaled_unit(const double* beta, double* v, int len, hipStream_t st);
// Per-iteration status: omega = sqrt(sumsq[1]), ||W|| = sqrt(sumsq[0]); breakdown when
// omega <= bd_tol * ||W||; packs LS flags, residual and the ranks of the new basis tensor.
struct IterStatus {
  int breakdown_ls;
  int converged;
  int breakdown_w;
  int pad;
  int rank[kMaxD];
  double res;
  double omega;
};
void iter_status(const double* sumsq2, const int* ls_flags, const double* res_k, const int* rank, int d,
                 double bd_tol, double* omega, IterStatus* out, hipStream_t st);

// ---- sketched least squares, one column at a time --------------------------
struct LsState {
  const double* Mcol;  // s x kmax sketched columns (col-major, ld s)
  const double* bs;    // s
  double* Hv;          // s x kmax Householder vectors
  double* tau;         // kmax
  double* R;           // kmax x kmax
  double* qtb;         // s
  double* y;           // kmax
  double* res;         // relative sketched residual after each column (kmax)
  double* nrmM2;       // running ||M||_F^2
  int* flags;          // [0] breakdown, [1] converged
  double beta_s_inv;   // not used when bs_norm is given
  const double* bs_norm; // device ||b_s||
  double* lam = nullptr; // regularisation parameter per column (kmax), when regularised
  double* ysave = nullptr; // kmax x kmax: column k holds y after column k was added (optional)
};
void ls_add_column(const LsState& st_, int s, int kmax, int k, double conv_tol, double breakdown_tol,
                   hipStream_t st);
void ls_init(const LsState& st_, int s, hipStream_t st);
// Projected Tikhonov on the factorisation after column k (k + 1 columns):
// y, res[k], lam[k] and the converged flag are replaced by the regularised
// ones.  lam_fixed >= 0 uses that lambda, < 0 chooses it by GCV.
void ls_tikhonov(const LsState& st_, int s, int kmax, int k, double conv_tol, double lam_fixed, hipStream_t st);

}  // namespace tk
