// Host orchestration of the Tucker sGMRES hot path.
//
// Every operation is *planned* once: buffers are carved from the caller's
// workspace, GEMM / reduction task tables are collected on the host and
// uploaded in one copy, and the resulting sequence of launches is replayed
// as often as needed (every sGMRES iteration replays the plan built for its
// index).  All sizes in a plan are capacities; actual ranks, sketch widths
// and coefficients are device values read by the kernels.
#pragma once

#include <array>
#include <cstring>
#include <functional>
#include <memory>

#include "gemm.hpp"
#include "kernels.hpp"

namespace tk {

// ------------------------------------------------------------------ plumbing
struct Blob {
  std::vector<unsigned char> host;
  unsigned char* dev = nullptr;
  template <typename X>
  size_t add(const std::vector<X>& v) {
    size_t off = (host.size() + 15) & ~size_t(15);
    host.resize(off + v.size() * sizeof(X));
    if (!v.empty()) std::memcpy(host.data() + off, v.data(), v.size() * sizeof(X));
    return off;
  }
  template <typename X>
  X* at(size_t off) const {
    return reinterpret_cast<X*>(dev + off);
  }
};

struct Seq {
  std::vector<std::function<void(hipStream_t)>> steps;
  void run(hipStream_t st) const {
    for (auto& f : steps) f(st);
  }
};
// Moves steps [from, end) of q onto side stream `which` (after everything
// issued before them on the caller's stream); the returned step, pushed
// later, makes the caller's stream wait for them.
std::function<void(hipStream_t)> fork_steps(Seq& q, size_t from, int which);

struct Shape {
  int d = 3;
  int n[kMaxD] = {0, 0, 0, 0};
  int rc = 0;   // rank capacity of every internal Tucker tensor
  int cap = 0;  // rank cap of RoundSum outputs (<= rc)
  int p = 5;    // oversampling
  int sc() const { return cap + p; }  // range-sketch capacity
  size_t core_len() const { return size_t(ipow(rc, d)); }
};

// Device Tucker tensor of capacity rc (core rc^d, factors n_k x rc, ranks[d]).
template <typename T>
struct TT {
  T* core = nullptr;
  T* U[kMaxD] = {nullptr, nullptr, nullptr, nullptr};
  int* rank = nullptr;
};

template <typename T>
TT<T> alloc_tt(Arena& ar, const Shape& sh) {
  TT<T> t;
  t.core = ar.alloc<T>(sh.core_len());
  for (int k = 0; k < sh.d; ++k) t.U[k] = ar.alloc<T>(size_t(sh.n[k]) * sh.rc);
  t.rank = ar.alloc<int>(kMaxD);
  return t;
}

// Block sum: sum_b coef_b * Tucker_b with coef_b = cscale_b * (*cptr_b).
template <typename T>
struct Blocks {
  std::vector<const T*> core;
  std::vector<std::array<const T*, kMaxD>> U;
  std::vector<const int*> rank;
  std::vector<const double*> cptr;
  std::vector<double> cscale;
  int size() const { return int(core.size()); }
  void add(const T* c, const std::array<const T*, kMaxD>& u, const int* r, const double* cp, double cs) {
    core.push_back(c);
    U.push_back(u);
    rank.push_back(r);
    cptr.push_back(cp);
    cscale.push_back(cs);
  }
  void add(const TT<T>& t, const double* cp, double cs) {
    add(t.core, {t.U[0], t.U[1], t.U[2], t.U[3]}, t.rank, cp, cs);
  }
};

struct RoundCfg {
  double eps = 1e-10;
  double tau = -1.0;  // <= 0: eps
  const double* eps_dev = nullptr;  // optional device {eps, tau}; overrides eps/tau at run time
  double delta = 1e-12;
  int force_s = -1;
  int force_r[kMaxD] = {-1, -1, -1, -1};
  // range-finder basis by Householder QR (orthonormal to O(u)) instead of the
  // three-pass Cholesky-QR (O(10-100 u)); used where the sum must be rounded to
  // full FP64 accuracy (the refinement update and residual)
  bool householder = false;
};

// Planning context: arena + shared table blob.
struct Planner {
  Arena& ar;
  Blob& blob;
  // BF16-factor form (FP32 plans only): the products that multiply a Tucker
  // factor (operator factors times U, sketch factors, range-finder Omega and
  // basis products) round their operands to bfloat16 and run on the BF16
  // matrix cores with FP32 accumulation; cores, Grams, QRs and eigensolves
  // keep FP32 / FP64.
  bool bf16_factors = false;
  Planner(Arena& a, Blob& b) : ar(a), blob(b) {}
};

// RoundSum of a block sum (Sec. 3.1).  `nb_active` (optional) points to a host
// int limiting the blocks used at run time (blocks are consumed in order).
// Writes the output Tucker tensor and device ints s_dev (sketch width).
template <typename T>
struct RoundSumOut {
  int* s_dev = nullptr;
  double* total_dev = nullptr;
};
template <typename T>
RoundSumOut<T> plan_roundsum(Seq& q, Planner& pl, const Shape& sh, const Blocks<T>& in, const RoundCfg& cfg,
                             const std::array<const T*, kMaxD>& omega, const TT<T>& out, const int* nb_active);

// Operator factors: per term and mode a device matrix (row-major n x n) or null.
template <typename T>
struct OpDev {
  int nterms = 0;
  std::vector<double> alpha;
  std::vector<const T*> A;  // [j * d + k]
};

// apply(x): factor products into owned buffers; returns the block sum of L(x).
template <typename T>
Blocks<T> plan_apply(Seq& q, Planner& pl, const Shape& sh, const OpDev<T>& op, const TT<T>& x, bool transpose,
                     std::vector<T*>* products = nullptr);

// Khatri-Rao sketch of a block sum into a device vector (length s).
template <typename T>
void plan_sketch(Seq& q, Planner& pl, const Shape& sh, const Blocks<T>& in, const std::array<const T*, kMaxD>& S,
                 int s, double* out);

// Inner products <X_j, Y> (j over xs) into out[j] (device doubles), times scale.
template <typename T>
void plan_inner(Seq& q, Planner& pl, const Shape& sh, const std::vector<TT<T>>& xs, const Blocks<T>& ys_single,
                double* out, double scale, std::vector<T*>* grams_out = nullptr);

// Y = X x_k W for one tensor (W: newdim x dims[k], col-major, ld ldw), or with
// W given transposed (dims[k] x newdim) when w_transposed.
template <typename T>
void plan_ttm(Seq& q, Planner& pl, int d, const int* dims, int k, int newdim, const T* X, const T* W, int ldw,
              bool w_transposed, T* Y);
// G = X_(k) Y_(k)^T for two tensors of dims `dims` (mid x mid, ld ldg), times scale.
template <typename T>
void plan_unfold_gram(Seq& q, Planner& pl, int d, const int* dims, int k, const T* X, const T* Y, T* G, int ldg,
                      double scale);
// C = alpha * op(A) op(B) (+ beta C): a single plain GEMM (`factor_product`:
// one operand is a Tucker factor, BF16 operands in the BF16-factor form).
template <typename T>
void plan_gemm(Seq& q, Planner& pl, bool ta, bool tb, int M, int N, int K, const T* A, int lda, const T* B, int ldb,
               T* C, int ldc, double alpha, double beta, bool factor_product = false);

// C_i = alpha op(A_i) op(B_i) for equally shaped problems, one launch.
template <typename T>
void plan_gemm_batched(Seq& q, Planner& pl, bool ta, bool tb, int M, int N, int K, const std::vector<const T*>& A,
                       int lda, const std::vector<const T*>& B, int ldb, const std::vector<T*>& C, int ldc,
                       double alpha);

// Khatri-Rao range sketch of a block sum with per-block device coefficients
// coef[b]: Y_k = sum_b coef_b U_bk MTTKRP(G_b; {U_bj^T L_j[:, :w]}_{j != k}, k)
// (n_k x w; L_j column-major n_j x >= w).  The range sketch of RoundSum
// (Sec. 3.1) and the factor sketches of the multilinear Nystrom method.
template <typename T>
void plan_krp_range(Seq& q, Planner& pl, const Shape& sh, const Blocks<T>& in, const double* coef,
                    const std::array<const T*, kMaxD>& L, int w, const std::array<T*, kMaxD>& Y,
                    const int* nb_active);
// Core projection C = sum_b coef_b G_b x_1 (P_1^T U_b1) ... x_d (P_d^T U_bd)
// (w^d row-major; P_k column-major n_k x >= w).
template <typename T>
void plan_core_projection(Seq& q, Planner& pl, const Shape& sh, const Blocks<T>& in, const double* coef,
                          const std::array<const T*, kMaxD>& Pm, int w, T* C, const int* nb_active);

// Exact squared Frobenius norm of a block sum (QR of concatenated factors).
void plan_exact_norm2(Seq& q, Planner& pl, const Shape& sh, const Blocks<double>& in, double* out_norm2);

// ------------------------------------------------------------------ multilinear Nystrom
// Sketched form of a Tucker tensor X (Sec. 3.3): the projected core
// G_Psi = X x_1 Psi_1^T ... x_d Psi_d^T (rt^d, row-major) and the factor
// sketches F_k = X_(k) (Khatri-Rao product of the other modes' Psi_j[:, :r])
// (n_k x r, column-major).  Psi_k: n_k x rt column-major, rt = r + p.
struct MlnSk {
  double* core = nullptr;
  double* F[kMaxD] = {nullptr, nullptr, nullptr, nullptr};
};
MlnSk alloc_mln(Arena& ar, const Shape& sh, int r, int rt);
// Sketch of a block sum (every block sketched, then summed with its
// coefficient).  diag (optional, device rt): the superdiagonal of G_Psi, which
// is the Khatri-Rao sketch (Psi_1 (.) ... (.) Psi_d)^T vec(X).
void plan_mln_sketch(Seq& q, Planner& pl, const Shape& sh, const Blocks<double>& in,
                     const std::array<const double*, kMaxD>& Psi, int r, int rt, const MlnSk& out, double* diag);
// Recovery X~ = G_Psi x_k (F_k (Psi_k^T F_k)^+) into `out` (capacity sh.rc >= r;
// ranks = numerical ranks of Psi_k^T F_k, at least 1).
void plan_mln_recovery(Seq& q, Planner& pl, const Shape& sh, const MlnSk& sk,
                       const std::array<const double*, kMaxD>& Psi, int r, int rt, const TT<double>& out);

// Separable spectral preconditioner (Sec. 3.4): per mode an orthogonal V_k
// (n_k x n_k, column-major) and eigenvalues lambda_k of the 1D operator;
// M = sum_{h=-q..q} c_h (x)_k V_k exp(-t_h Lambda_k) V_k^T with t_h = exp(h eta),
// c_h = eta t_h, eta = pi / sqrt(q).  q = 0: no preconditioner.
template <typename T>
struct PrecondT {
  int q = 0;
  std::array<const T*, kMaxD> V{};
  std::array<const T*, kMaxD> lam{};
};
// The 2q + 1 terms of M(x) in the spectral basis: core of x, factors
// exp(-t_h (Lambda_k - lambda_min,k)) V_k^T U_k (n_k x rc, allocated from the
// planner's arena) and device coefficients c_h exp(-t_h sum_k lambda_min,k).
template <typename T>
Blocks<T> plan_precond_terms(Seq& q, Planner& pl, const Shape& sh, const PrecondT<T>& pc, const TT<T>& x);
// z = RoundSum of the 2q + 1 terms of M(x) in the spectral basis (full sketch
// width), factors mapped back by V_k.
template <typename T>
void plan_precond(Seq& q, Planner& pl, const Shape& sh, const PrecondT<T>& pc, const TT<T>& x, const TT<T>& z,
                  const RoundCfg& rcfg, const std::array<const T*, kMaxD>& omega);

struct MlnCfg {
  int r = 32, p = 32;
  double tol = 1e-8, eta = 0.4;
  int maxiter = 60, k_trunc = 2;
  double bd_tol = 1e-14;
  bool save_memory = false;
  int r_sol = 0, p_sol = 0;
  bool tikhonov = false;  // projected Tikhonov with GCV on the sketched least squares
};
struct MlnInfo {
  int status = 1, iters = 0;
  double true_relres = 1.0, seconds = 0.0;
  std::vector<double> hist;  // relative sketched residual per iteration
  std::vector<int> ranks;    // d per iteration: ranks of the new basis tensor
  std::vector<double> lambda;  // regularisation parameter per iteration (when regularised)
};
class MlnSolver;
struct MlnSolverDel {
  void operator()(MlnSolver* s) const;
};
using MlnSolverPtr = std::unique_ptr<MlnSolver, MlnSolverDel>;
// MLN-Tucker sGMRES on L(X) = b, planned once (b's ranks <= cfg.r).  With
// precond.q > 0 the method is flexible (Sec. 3.4): Z_k = MLN recovery of the
// MLN sketch of M(V_k), L acts on Z_k and the stored sketches of the Z_k give
// the solution.
MlnSolverPtr make_mln_solver(Arena& ar, const Shape& sh, const OpDev<double>& op, const TT<double>& b,
                             const MlnCfg& cfg, const std::array<const double*, kMaxD>& Psi, hipStream_t st,
                             const PrecondT<double>& precond = PrecondT<double>{});
void mln_solver_run(MlnSolver& s, TT<double>& x_out, MlnInfo& info, hipStream_t st);

// ------------------------------------------------------------------ solver
struct SolveCfg {
  int form = 0;  // 0 FP64, 1 FP32
  double tol = 1e-8, eta = 0.4;
  int maxiter = 60, max_restarts = 50, k_trunc = 2;
  int s = 120;
  double eps_trunc = -1, eps_min = -1, tol_inner_floor = -1;
  bool transpose = false;
  bool tikhonov = false;  // projected Tikhonov with GCV on the sketched least squares
  int method = 0;         // 0: sketched GMRES cycles (Alg. 2); 1: full Arnoldi (Alg. 1)
};

struct SolveInfo {
  int status = 1, iters = 0, cycles = 0;
  double true_relres = 1.0, seconds = 0.0;
  std::vector<double> hist_sketched, hist_true, hist_time;
  std::vector<int> hist_ranks;  // d per iteration
  std::vector<double> hist_lambda;  // regularisation parameter per iteration (when regularised)
};

// Solver bound to fixed device inputs; plans everything at construction.
class Solver;
struct SolverDel {
  void operator()(Solver* s) const;
};
using SolverPtr = std::unique_ptr<Solver, SolverDel>;
SolverPtr make_solver(Arena& ar, const Shape& sh, const OpDev<double>& op, const TT<double>& b,
                                    const SolveCfg& cfg, const std::array<const double*, kMaxD>& S,
                                    const std::array<const double*, kMaxD>& omega, const TT<double>* x0,
                                    hipStream_t st, const PrecondT<double>& precond = PrecondT<double>{});
void solver_run(Solver& s, TT<double>& x_out, SolveInfo& info, hipStream_t st);
TT<double> solver_solution(Solver& s);
TT<double> solver_slot(Solver& s, int i);  // 0, 1: the buffers the iterate alternates between; 2: best iterate
int solver_slot_index(Solver& s);           // slot holding the solution after solver_run

}  // namespace tk
