/*
 * tsgmres.h -- C ABI of the MI355X (gfx950) Tucker-sketched GMRES library.
 *
 * The library implements the per-iteration Tucker arithmetic of RHOSVD-Tucker
 * sGMRES (Bucci, Iannacito, Pasha, Smith, "Randomized Tucker-Sketched GMRES",
 * Alg. 2) for Kronecker-sum tensor equations
 *     L(X) = sum_j alpha_j  X x_1 A_j^(1) x_2 ... x_d A_j^(d) = B      (Eq. (2))
 * with B and X in Tucker format (Sec. 2.3), plus restarts with FP64 iterative
 * refinement, an FP32 form, and the adjoint solve for gradients.
 *
 * Conventions shared by every entry point
 *   - Tensors are DEVICE memory owned by the caller.  A Tucker tensor
 *     X = G x_1 U_1 ... x_d U_d stores its core row-major over (i_1..i_d)
 *     (mode d fastest) with capacity strides: entry (i_1..i_d) sits at
 *     sum_k i_k * prod_{j>k} rcap_j.  Factor U_k is n_k x rcap_k column-major
 *     (leading dimension n_k).  Only the leading r_k columns / indices are
 *     read on input; on output everything beyond the ranks is zero.
 *   - Operator factors A_j^(k) are dense n_k x n_k ROW-major device matrices;
 *     a NULL pointer stands for the identity.
 *   - Random sketch matrices are always inputs (the library draws no random
 *     numbers): S_k is n_k x s and Omega_k is n_k x (rank_cap + oversample),
 *     both column-major device matrices.
 *   - `stream` is a hipStream_t (NULL = default stream).  Calls are ordered on
 *     it; entry points that return host results (ranks, norms, statuses)
 *     synchronise the stream before returning.
 *   - The library allocates no device memory of its own: every call takes a
 *     caller-provided device workspace `ws` of `ws_bytes` bytes.  The matching
 *     *_workspace function reports the size needed (same arguments, no data).
 *   - Return value: 0 = success; > 0 = informational solver status;
 *     < 0 = error (outputs unspecified, message via tk_last_error()).
 *     Nothing throws across the ABI.  The error message is thread-local.
 *   - Limits of this library: 2 <= d <= 4, n_k <= 512, rank_cap + oversample
 *     <= 64, sketch size s <= 256, maxiter <= 64; multilinear Nystrom calls:
 *     target rank r <= 64 and r + p <= 256.
 *   - Forms: tensors cross the ABI in FP64.  TK_FORM_FP32 runs a call in the
 *     arithmetic of the solver's FP32 form: operands are rounded to FP32 on
 *     entry, products, Gram matrices, eigensolves and contractions run in
 *     FP32 (matrix cores with FP32 accumulation), the range-sketch QR of a
 *     RoundSum stays FP64, and results are widened to FP64 on exit.
 *     TK_FORM_BF16 (tucker_apply_op, tucker_sketch, tucker_rhosvd only) is the
 *     FP32 form with bfloat16 factors: every product with a Tucker factor
 *     (operator factors times U, S_k^T U_k, U^T Omega, the range-sketch sum
 *     and the core projection) rounds both operands to bfloat16 (round to
 *     nearest even) and runs on the BF16 matrix cores with FP32 accumulation;
 *     cores, Grams, QRs and eigensolves keep the FP32 form's arithmetic.  The
 *     solver runs in FP64 or FP32 only.
 */
#ifndef TSGMRES_H_
#define TSGMRES_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TK_MAX_D 4

/* status codes */
#define TK_OK 0
#define TK_NOT_CONVERGED 1   /* tsgmres_solve: x is the iterate with the smallest true residual;
                                tsgmres_mln_solve: x is the last iterate */
#define TK_BREAKDOWN 2       /* exact solution in the Krylov space (lucky breakdown) */
#define TK_RANK_FLOOR 3      /* two cycles in a row reduced the true residual by < 10%
                                (x: the iterate with the smallest true residual) */
#define TK_ERR_INVALID_ARG -1
#define TK_ERR_SHAPE -2
#define TK_ERR_CAPACITY -3    /* an output rank exceeds the caller's capacity */
#define TK_ERR_WORKSPACE -4   /* ws_bytes smaller than the *_workspace size */
#define TK_ERR_HIP -5
#define TK_ERR_NONFINITE -6
#define TK_ERR_UNSUPPORTED -7 /* outside the limits listed above */

typedef enum { TK_FORM_FP64 = 0, TK_FORM_FP32 = 1, TK_FORM_BF16 = 2 } tk_form;

/* Tucker tensor (Sec. 2.3, Tucker format equation). */
typedef struct {
  int32_t d;
  int64_t n[TK_MAX_D];
  int64_t r[TK_MAX_D];    /* ranks: read on inputs, written on outputs */
  int64_t rcap[TK_MAX_D]; /* capacities (core strides and factor widths) */
  double* core;           /* device */
  double* U[TK_MAX_D];    /* device, n_k x rcap_k column-major */
} tk_tucker;

/* Linear combination sum_b coef[b] * blocks[b] of Tucker tensors. */
typedef struct {
  int32_t nblocks;
  const double* coef;       /* host [nblocks] */
  const tk_tucker* blocks;  /* host [nblocks] */
} tk_block_sum;

/* Kronecker-sum operator of Eq. (2): sum_j alpha_j A_j^(1) kron ... kron A_j^(d). */
typedef struct {
  int32_t d;
  int64_t n[TK_MAX_D];
  int32_t nterms;
  const double* alpha;          /* host [nterms] */
  const double* const* A;       /* host [nterms * d] of device row-major n_k x n_k, NULL = identity */
} tk_kron_op;

/* RoundSum parameters (Sec. 3.1): effective-rank sketch width, range
 * sketch, QR, core projection, ST-HOSVD truncation to tolerance eps. */
typedef struct {
  double eps;               /* relative ST-HOSVD tolerance */
  double tau;               /* effective-rank energy threshold; <= 0 uses eps */
  int32_t rank_cap;         /* output rank cap per mode */
  int32_t oversample;       /* p: sketch width = min(max_k r~_k + p, rank_cap + p) */
  int32_t force_s;          /* >= 0: use this sketch width (rank replay) */
  int32_t force_ranks[TK_MAX_D]; /* >= 0: use these output ranks (rank replay) */
  int32_t form;             /* tk_form of the arithmetic (see "Forms" above) */
} tk_round_params;

/* Restarted Tucker sGMRES parameters (Alg. 2 inputs plus restarts). */
typedef struct {
  int32_t form;             /* tk_form */
  double tol;               /* target relative residual ||B - L(X)|| / ||B|| */
  double eta;               /* sketched-residual correction factor (Alg. 2) */
  int32_t maxiter;          /* iterations per cycle (<= 64) */
  int32_t max_restarts;     /* cycles */
  int32_t k_trunc;          /* truncated-Arnoldi window */
  int32_t rank_cap;
  int32_t oversample;
  int64_t s;                /* columns of the sketch factors S_k */
  double eps_trunc;         /* inner RoundSum tolerance; <= 0: max(1e-2 * inner tol, eps_min) */
  double eps_min;           /* <= 0: 1e-13 (FP64) / 1e-6 (FP32) */
  double tol_inner_floor;   /* <= 0: 1e-13 (FP64) / 1e-5 (FP32) */
  const tk_tucker* x0;      /* optional initial guess (NULL = zero) */
  /* Optional separable spectral preconditioner (Sec. 3.4), which makes every
   * cycle flexible: Z_k = RoundSum(M(V_k)) at the full sketch width, L is
   * applied to Z_k and the cycle's solution is RoundSum(sum_i y_i Z_i), with
   *   M = sum_{h=-q..q} c_h (x)_k V_k exp(-t_h Lambda_k) V_k^T,
   *   t_h = exp(h eta), c_h = eta t_h, eta = pi / sqrt(q)
   * (for V_k, Lambda_k the eigenpairs of a 1D Laplacian, an exponential-sum
   * approximation of the inverse of the d-dimensional Laplacian). */
  int32_t precond_q;                   /* 0: none; >= 1: 2q + 1 terms */
  const double* const* precond_V;      /* host array of d device pointers: orthogonal V_k, n_k x n_k column-major */
  const double* const* precond_lambda; /* host array of d device pointers: eigenvalues lambda_k, length n_k */
  /* Projected Tikhonov (Sec. 4.3): 1 replaces every iteration's y_k by
   * argmin ||M_k y - b_s||^2 + lambda_k^2 ||y||^2 with lambda_k chosen by
   * GCV (see tsgmres_projected_tikhonov); the sketched residual and its
   * convergence test use that y_k.  0: plain sketched least squares. */
  int32_t tikhonov;
  /* Cycle method: 0 = RHOSVD-Tucker sGMRES (Alg. 2: truncated Arnoldi
   * window k_trunc, sketched least squares, stop at res_k < eta * tol);
   * 1 = RHOSVD-Tucker GMRES (Alg. 1: full Arnoldi, every basis tensor in the
   * orthogonalisation RoundSum, least squares on the Hessenberg matrix,
   * stop at res_k < tol; S and s are not used and S may be NULL; no
   * preconditioner).  Both run inside the same FP64 refinement loop. */
  int32_t method;
} tk_sgmres_params;

/* Solver report (host memory owned by the caller). */
typedef struct {
  int32_t status, iters_total, cycles;
  double true_relres, seconds;
  int32_t hist_cap, hist_len;  /* hist_cap: capacity of the arrays below */
  double* hist_sketched;       /* [hist_cap] sketched relative residual per iteration, or NULL */
  double* hist_true;           /* [hist_cap] true relative residual per cycle, or NULL */
  int32_t* hist_ranks;         /* [hist_cap * TK_MAX_D] ranks of each new basis tensor, or NULL */
  double* hist_cycle_seconds;  /* [hist_cap] elapsed seconds at the end of each cycle, or NULL */
  double* hist_lambda;         /* [hist_cap] Tikhonov lambda_k per iteration (when regularised), or NULL */
} tk_sgmres_info;

/* Operator factors applied to a Tucker tensor (Eq. (2)): for every term j and
 * mode k with A_j^(k) != NULL writes AU[j*d+k] = A_j^(k) U_k (transpose = 0)
 * or A_j^(k)^T U_k (transpose = 1) into caller buffers of n_k x x->rcap[k];
 * L(x) is then the block sum of terms alpha_j * (core; AU or U).  AU entries
 * of identity factors are ignored (may be NULL).  form: tk_form. */
int tucker_apply_op(const tk_kron_op* op, const tk_tucker* x, int32_t transpose, int32_t form, double* const* AU,
                    void* ws, size_t ws_bytes, void* stream);
int tucker_apply_op_workspace(const tk_kron_op* op, const tk_tucker* x, int32_t form, size_t* bytes);

/* Khatri-Rao sketch (Alg. 2, sketch of B and of each W): out[l] =
 * (S_1[:,l] kron ... kron S_d[:,l])^T vec(sum_b coef_b X_b), l < s; out is a
 * device vector of length s.  form: tk_form (the sketch vector is FP64 either way). */
int tucker_sketch(const tk_block_sum* x, const double* const* S, int64_t s, int32_t form, double* out, void* ws,
                  size_t ws_bytes, void* stream);
int tucker_sketch_workspace(const tk_block_sum* x, int64_t s, int32_t form, size_t* bytes);

/* Allocation-free variant of tucker_sketch, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, result and errors as tucker_sketch,
 * without the workspace: its temporaries live in a static device array of
 * 64 MiB that the library holds on every GPU it runs on until the process
 * ends.  A call whose workspace query (tucker_sketch_workspace) exceeds
 * 64 MiB launches nothing and returns TK_ERR_WORKSPACE.  The call allocates
 * no device memory (no hipMalloc / hipFree).  All calls on one GPU share that
 * array: calls that overlap in time on the same GPU (different streams or
 * host threads) race and must be serialised by the caller. */
int tucker_sketch_noalloc(const tk_block_sum* x, const double* const* S, int64_t s, int32_t form, double* out,
                          void* stream);

/* RoundSum (Sec. 3.1): randomized RHOSVD recompression of a block sum into
 * `out` (ranks written to out->r; out->rcap must hold them).  *s_out (host,
 * optional) receives the sketch width used. */
int tucker_rhosvd(const tk_block_sum* in, const tk_round_params* prm, const double* const* omega, tk_tucker* out,
                  int32_t* s_out, void* ws, size_t ws_bytes, void* stream);
int tucker_rhosvd_workspace(const tk_block_sum* in, const tk_round_params* prm, size_t* bytes);

/* Restarted RHOSVD-Tucker sGMRES (Alg. 2 cycles wrapped in FP64 iterative
 * refinement): solves L(X) = B to relative residual tol.  Returns the status
 * (TK_OK / TK_NOT_CONVERGED / TK_BREAKDOWN / TK_RANK_FLOOR) or an error.
 * Without convergence x is the iterate with the smallest true residual (an
 * initial guess included) and info->true_relres is that residual;
 * info->hist_true keeps every cycle's.  The refinement rounds x + d to
 * relative accuracy 1e-2 tol; when the true residual stalls for two cycles
 * while every rank of x is below rank_cap, that tolerance is divided by 100
 * (down to 1e-15) and the refinement goes on. */
int tsgmres_solve(const tk_kron_op* op, const tk_tucker* b, const tk_sgmres_params* prm, const double* const* S,
                  const double* const* omega, tk_tucker* x, tk_sgmres_info* info, void* ws, size_t ws_bytes,
                  void* stream);
int tsgmres_solve_workspace(const tk_kron_op* op, const tk_tucker* b, const tk_sgmres_params* prm, size_t* bytes);

/* Adjoint of the solve, for a loss l(x) with cotangent x_bar = dl/dx (a block
 * sum): solves L^T lambda = RoundSum(x_bar) with the same sGMRES on transposed
 * factors; lambda = dl/dB.  dalpha (host [nterms], optional) receives
 * dl/dalpha_j = -<lambda, x x_1 A_j^(1) ... x_d A_j^(d)>; dA[j*d+k] (device
 * row-major n_k x n_k, optional, NULL entries skipped) receives
 * dl/dA_j^(k) = -alpha_j lambda_(k) (kron_{l!=k} A_j^(l)) x_(k)^T. */
int tsgmres_backward(const tk_kron_op* op, const tk_tucker* x, const tk_block_sum* xbar,
                     const tk_sgmres_params* prm, const double* const* S, const double* const* omega,
                     tk_tucker* lambda, double* dalpha, double* const* dA, tk_sgmres_info* info, void* ws,
                     size_t ws_bytes, void* stream);
int tsgmres_backward_workspace(const tk_kron_op* op, const tk_tucker* x, const tk_block_sum* xbar,
                               const tk_sgmres_params* prm, size_t* bytes);

/* Exact Frobenius norm of a block sum without cancellation: per mode a
 * Householder QR of the concatenated distinct factors, then the norm of the
 * small coefficient core (the norm used for Alg. 2's beta and the restart
 * residual).  *out (host) receives ||sum_b coef_b X_b||_F.  Ranks <= 64. */
int tucker_norm(const tk_block_sum* x, double* out, void* ws, size_t ws_bytes, void* stream);
int tucker_norm_workspace(const tk_block_sum* x, size_t* bytes);

/* Multilinear Nystrom (MLN) sketching (Sec. 3.3).  Psi_k are n_k x (r + p)
 * column-major device matrices (inputs, like every sketch); Omega_k of mode k
 * is the Khatri-Rao product of the leading r columns of the other modes'
 * Psi_j: its column l is kron_{j != k} Psi_j[:, l] over j in increasing order
 * (the row-major unfolding order of the core convention above).  Sketched
 * form of a tensor X: the core G_Psi = X x_1 Psi_1^T ... x_d Psi_d^T
 * ((r + p)^d, row-major, dense) and the factor sketches F_k = X_(k) Omega_k
 * (n_k x r, column-major). */
typedef struct {
  int32_t r;             /* target rank of every recovered tensor, 1..64 */
  int32_t p;             /* oversampling: Psi_k has r + p <= 256 columns */
  double tol;            /* stop once the sketched relative residual < eta * tol */
  double eta;            /* sketched-residual correction factor, 0 < eta <= 1 */
  int32_t maxiter;       /* 1..64 */
  int32_t k_trunc;       /* window of the truncated orthogonalisation, >= 1 */
  double breakdown_tol;  /* <= 0: 1e-14 (relative basis-norm and least-squares pivot floor) */
  int32_t save_memory;   /* 1: memory-efficient variant, sketches outside the
                            window kept truncated to (r_sol + p_sol)^d cores and
                            r_sol factor columns; the solution is recovered from
                            the truncated sketches with Psi_k[:, :r_sol + p_sol] */
  int32_t r_sol, p_sol;  /* save_memory: 1 <= r_sol <= r, r_sol + p_sol <= r + p */
  int32_t tikhonov;      /* 1: projected Tikhonov with GCV, as in tk_sgmres_params */
  /* Optional exponential-sum preconditioner M (Sec. 3.4), given as in
   * tk_sgmres_params.  The method is then flexible: Z_i is the MLN recovery of
   * the MLN sketch of M(V_i) (its 2q + 1 terms sketched with the same Psi_k
   * and target rank r), L is applied to Z_i, and the solution is recovered
   * from sum_i y_i sketch(Z_i); with save_memory the sketches of the Z_i are
   * kept truncated to (r_sol + p_sol)^d cores and r_sol factor columns.  The
   * pointer arrays and the device data they name are read during the call
   * only.  precond_q = 0 (zero-initialised struct): no preconditioner. */
  int32_t precond_q;                   /* 0: none; 1..400: 2q + 1 terms */
  const double* const* precond_V;      /* host array of d device pointers: orthogonal V_k, n_k x n_k column-major */
  const double* const* precond_lambda; /* host array of d device pointers: eigenvalues lambda_k, length n_k */
} tk_mln_params;

/* MLN sketch of a block sum x = sum_b coef_b X_b (the sketch of every block
 * summed with its coefficient): writes core ((r + p)^d device doubles) and
 * F[k] (n_k x r device doubles); diag (device, r + p, optional) receives the
 * superdiagonal of the core, which equals the Khatri-Rao sketch of x with
 * S_k = Psi_k.  Block ranks <= 128. */
int tucker_mln_sketch(const tk_block_sum* x, const double* const* Psi, int32_t r, int32_t p, double* core,
                      double* const* F, double* diag, void* ws, size_t ws_bytes, void* stream);
int tucker_mln_sketch_workspace(const tk_block_sum* x, int32_t r, int32_t p, size_t* bytes);

/* MLN recovery of a sketched tensor (core, F) into the Tucker tensor
 * out = core x_1 P_1 ... x_d P_d with P_k = F_k (Psi_k^T F_k)^+, where the
 * pseudoinverse drops the directions of Psi_k^T F_k whose column-pivoted QR
 * remainder is at or below 1e-12 of its largest column.  out->d and out->n
 * give the shape; out->r receives the numerical ranks (1..r); out->rcap[k]
 * must be >= r. */
int tucker_mln_recover(const double* core, const double* const* F, const double* const* Psi, int32_t r, int32_t p,
                       tk_tucker* out, void* ws, size_t ws_bytes, void* stream);
int tucker_mln_recover_workspace(int32_t d, const int64_t* n, int32_t r, int32_t p, size_t* bytes);

/* MLN-Tucker sGMRES (Sec. 3.3): one run of at most maxiter iterations (no
 * restarts) with every basis tensor kept as an MLN sketch, the superdiagonal
 * of the sketched core as the least-squares sketch, and the solution
 * recovered from the coefficient-weighted sum of the stored sketches.
 * b: ranks <= r.  info (optional): status, iters_total, cycles = 1,
 * true_relres = ||b - L(x)|| / ||b|| (exact), seconds, per-iteration
 * hist_sketched and hist_ranks; hist_true[0] = true_relres.  Returns the
 * status (TK_OK / TK_NOT_CONVERGED / TK_BREAKDOWN) or an error. */
int tsgmres_mln_solve(const tk_kron_op* op, const tk_tucker* b, const tk_mln_params* prm, const double* const* Psi,
                      tk_tucker* x, tk_sgmres_info* info, void* ws, size_t ws_bytes, void* stream);
int tsgmres_mln_solve_workspace(const tk_kron_op* op, const tk_tucker* b, const tk_mln_params* prm, size_t* bytes);

/* Projected Tikhonov regularisation of a sketched least-squares problem
 * (Sec. 4.3): y = argmin ||M y - b||^2 + lambda^2 ||y||^2 for the device
 * matrix M (s x k, column-major, ld s) and device vector b (length s),
 * 1 <= k <= 64, k <= s <= 256.  M is factorised by Householder QR,
 * M = Q R, which reduces the problem to k + 1 data: c = (Q^T b)[:k] and
 * rho = ||b - Q c||.  With the SVD R = U diag(sigma) W^T (one-sided Jacobi)
 * and beta_hat = U^T c, y = W diag(sigma / (sigma^2 + lambda^2)) beta_hat.
 * lambda_fixed >= 0 uses that lambda; < 0 chooses it by generalised cross
 * validation on the projected problem,
 *   G(lambda) = ||M y - b||^2 / (1 + sum_i lambda^2 / (sigma_i^2 + lambda^2))^2,
 * minimised over 241 log-spaced points in [1e-12, 1] sigma_1 followed by 60
 * golden-section steps in log10(lambda) between the grid minimum's
 * neighbours (lambda = 0 for M = 0).  Writes y (device, k) and out (device,
 * 2): out[0] = lambda, out[1] = ||M y - b|| / ||b||.  Synchronous on
 * `stream`. */
int tsgmres_projected_tikhonov(const double* M, const double* b, int32_t s, int32_t k, double lambda_fixed,
                               double* y, double* out, void* ws, size_t ws_bytes, void* stream);
int tsgmres_projected_tikhonov_workspace(int32_t s, int32_t k, size_t* bytes);

/* Kernel-class timers for performance reporting (not thread-safe; for
 * benchmarks).  kind: 0 GEMM, 1 symmetric eigensolver with eigenvectors
 * (Jacobi), 2 QR (Cholesky-QR / Householder), 3 Khatri-Rao reduction,
 * 4 sketched least-squares update, 5 eigenvalues-only solver (tridiagonal
 * reduction + bisection), 6 projected Tikhonov (Jacobi SVD + GCV).  Enabling (or disabling) clears the record; while
 * enabled, every launch of the class records a HIP event pair on its stream.
 * tk_kernel_timer_read synchronises those events and returns the launch count,
 * the summed kernel time in milliseconds and (each optional, may be NULL) the
 * summed algorithmic flops and HBM bytes of those launches.  Flops: 2*M*N*K per
 * GEMM product, 9*N^3 per eigendecomposition with vectors, (4/3)*N^3 per
 * eigenvalues-only solve (N = launch order), 2*(2*n*m^2 - (2/3)*m^3) per
 * Householder QR of an n x m matrix (m = the launch's column capacity,
 * counted with its thin Q), 0 for the other classes.  Bytes
 * (eigensolvers only, 0 for the other classes): per matrix, the N*N input read
 * once plus the N eigenvalues written, plus the N*N eigenvectors written when
 * they are computed, in the launch's element size. */
int tk_kernel_timer(int32_t kind, int32_t enable);
int tk_kernel_timer_read(int32_t kind, int64_t* launches, double* total_ms, double* flops, double* bytes);

/* Kernel launches the library has issued since it was loaded (every launch
 * of every entry point counts; host only, no device work). */
int tk_launch_count(int64_t* count);
/* Empty-kernel launch latency: n launches of an empty kernel back to back on
 * `stream`, then a synchronisation; *us_per_launch = elapsed microseconds / n.
 * The floor a sequence of k dependent launches cannot go below is about
 * k * *us_per_launch. */
int tk_launch_latency(int32_t n, void* stream, double* us_per_launch);
/* Rank certificates of RoundSum's effective-rank rule (Sec. 3.1) on the
 * current device since the library was loaded: *tried counts the per-mode
 * checks, *passed those that settled r~_k >= rank cap without the Gram's
 * spectrum (the sketch width is then cap + p, as the rule gives).  Waits for
 * the device.  Diagnostics for tests and profiles. */
int tk_rank_cert_count(int64_t* tried, int64_t* passed);

/* Message of the last error on this thread ("" if none). */
const char* tk_last_error(void);
/* ABI version (major * 100 + minor).  2.0 (200): tk_sgmres_params gained
 * tikhonov and method, tk_mln_params gained tikhonov, tk_sgmres_info gained
 * hist_lambda (all appended), and tsgmres_projected_tikhonov was added.
 * 2.1 (201): tucker_sketch_noalloc was added.  2.2 (202): tk_launch_count and
 * tk_launch_latency were added.  2.3 (203): tk_rank_cert_count was added.
 * 2.4 (204): TK_FORM_BF16 for the per-call entry points.  2.5 (205):
 * tk_mln_params gained the preconditioner fields (appended). */
#define TK_ABI_VERSION 205
int tk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TSGMRES_H_ */
