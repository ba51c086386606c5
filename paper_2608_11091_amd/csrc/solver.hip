// RHOSVD-Tucker sGMRES (Alg. 2) with restarts and FP64 iterative refinement.
//
// A cycle runs in the precision of its form (FP64, or FP32 operator applies,
// TTMs, sketches and Jacobi steps with FP64 range-finder QR and least
// squares).  Every iteration replays the plan built for its index and copies
// one small status record back to the host, which decides whether to stop.
// The outer loop is FP64: x <- RoundSum(x + d), the exact residual norm via
// QR of concatenated factors, and RoundSum(B - L(x)) as the next right-hand
// side.  A solve that stops without converging returns the iterate with the
// smallest true residual.  A rank floor reached with every rank of x below
// the cap tightens the truncation of the refinement RoundSums (x100, down to
// 1e-15) instead of stopping.
#include <chrono>
#include <cmath>
#include <limits>
#include <map>

#include "engine.hpp"

namespace tk {

namespace {

constexpr double kEpsOuterMin = 1e-15;  // floor of the refinement truncation tolerance

template <typename T>
void emit_copy_tt(Seq& q, const Shape& sh, const TT<T>& src, const TT<T>& dst, double scale = 1.0,
                  const double* den = nullptr) {
  const size_t cl = sh.core_len();
  const int d = sh.d;
  std::array<size_t, kMaxD> fl{};
  for (int k = 0; k < d; ++k) fl[k] = size_t(sh.n[k]) * sh.rc;
  q.steps.push_back([=](hipStream_t st) {
    scale_copy<T>(src.core, dst.core, cl, scale, nullptr, den, st);
    for (int k = 0; k < d; ++k) scale_copy<T>(src.U[k], dst.U[k], fl[k], 1.0, nullptr, nullptr, st);
    copy_ints(src.rank, dst.rank, d, st);
  });
}

template <typename A, typename B>
void emit_cast_tt(Seq& q, const Shape& sh, const TT<A>& src, const TT<B>& dst) {
  const size_t cl = sh.core_len();
  const int d = sh.d;
  std::array<size_t, kMaxD> fl{};
  for (int k = 0; k < d; ++k) fl[k] = size_t(sh.n[k]) * sh.rc;
  q.steps.push_back([=](hipStream_t st) {
    cast_copy<A, B>(src.core, dst.core, cl, st);
    for (int k = 0; k < d; ++k) cast_copy<A, B>(src.U[k], dst.U[k], fl[k], st);
    copy_ints(src.rank, dst.rank, d, st);
  });
}

}  // namespace

// ============================================================ one sGMRES cycle
template <typename T>
struct Cycle {
  Shape sh;
  int maxiter = 60, kt = 2, s = 120;
  bool tikhonov = false;
  // Full Arnoldi (Alg. 1): the window holds every basis tensor and the least
  // squares run on the Hessenberg columns (h, ||W||) against beta e_1 instead
  // of the sketches; the cycle stops at res_k < tol.
  bool full = false;
  int ls_rows = 0;  // rows of the least-squares problem: s, or maxiter + 1
  TT<T> rhs, W, dsol;
  std::vector<TT<T>> V;
  std::vector<TT<T>> Z;  // preconditioned basis (flexible cycle), when pc.q > 0
  PrecondT<T> pc;
  double* eps_pair = nullptr;  // device {eps, tau}
  double *beta2, *beta, *bs, *bsn2, *bsn, *Mcols, *h, *sumsq2, *omega;
  double *Hv, *tau, *R, *qtb, *y, *res, *nrmM2, *lam;
  int* flags;
  IterStatus* st_dev;
  IterStatus* st_host = nullptr;  // pinned, two slots (iteration parity)
  double* lam_host = nullptr;     // pinned, maxiter
  double* ysave = nullptr;        // maxiter x maxiter: y after each iteration
  hipEvent_t st_ev[2] = {nullptr, nullptr};
  Seq setup, fin;
  std::vector<Seq> iter;
  int nb_final = 0;
  double conv_tol = 0.0;
  double bd_tol = 1e-14;
  LsState ls{};

  ~Cycle() {
    if (st_host) (void)hipHostFree(st_host);
    if (lam_host) (void)hipHostFree(lam_host);
    for (auto& e : st_ev)
      if (e) (void)hipEventDestroy(e);
  }

  void plan(Planner& pl, const OpDev<T>& op, bool transpose, const std::array<const T*, kMaxD>& S,
            const std::array<const T*, kMaxD>& omega_, const PrecondT<T>& pc_) {
    pc = pc_;
    const bool flexible = pc.q > 0;
    Arena& ar = pl.ar;
    Blob* bl = &pl.blob;
    const int d = sh.d;
    rhs = alloc_tt<T>(ar, sh);
    W = alloc_tt<T>(ar, sh);
    dsol = alloc_tt<T>(ar, sh);
    for (int k = 0; k <= maxiter; ++k) V.push_back(alloc_tt<T>(ar, sh));
    if (flexible)
      for (int k = 0; k < maxiter; ++k) Z.push_back(alloc_tt<T>(ar, sh));
    if (full) kt = maxiter;
    ls_rows = full ? maxiter + 1 : s;
    const int lr = ls_rows;
    eps_pair = ar.alloc<double>(2);
    beta2 = ar.alloc<double>(1);
    beta = ar.alloc<double>(1);
    bs = ar.alloc<double>(lr);
    bsn2 = ar.alloc<double>(1);
    bsn = ar.alloc<double>(1);
    Mcols = ar.alloc<double>(size_t(lr) * maxiter);
    h = ar.alloc<double>(size_t(maxiter) * kt);
    sumsq2 = ar.alloc<double>(size_t(maxiter) * 2);
    omega = ar.alloc<double>(maxiter);
    Hv = ar.alloc<double>(size_t(lr) * maxiter);
    tau = ar.alloc<double>(maxiter);
    R = ar.alloc<double>(size_t(maxiter) * maxiter);
    qtb = ar.alloc<double>(lr);
    y = ar.alloc<double>(maxiter);
    res = ar.alloc<double>(maxiter);
    nrmM2 = ar.alloc<double>(1);
    lam = ar.alloc<double>(maxiter);
    ysave = ar.alloc<double>(size_t(maxiter) * maxiter);
    flags = ar.alloc<int>(4);
    st_dev = ar.alloc<IterStatus>(1);
    ls = LsState{Mcols, bs, Hv, tau, R, qtb, y, res, nrmM2, flags, 0.0, bsn, lam, ysave};
    if (!ar.measuring()) {
      TK_HIP(hipHostMalloc(reinterpret_cast<void**>(&st_host), 2 * sizeof(IterStatus), 0));
      TK_HIP(hipHostMalloc(reinterpret_cast<void**>(&lam_host), sizeof(double) * maxiter, 0));
      for (auto& e : st_ev) TK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }

    RoundCfg rcfg;
    rcfg.eps_dev = eps_pair;

    // ---- setup: beta = ||B|| (orthonormal factors), V_1 = B / beta, b_s = S^T vec(B)
    {
      std::vector<const T*> pc = {rhs.core};
      const size_t off = pl.blob.add(pc);
      const size_t cl = sh.core_len();
      setup.steps.push_back([=](hipStream_t st) {
        dot_batched<T>(bl->at<const T*>(off), bl->at<const T*>(off), cl, 1, 1.0, beta2, st);
        vec_sqrt(beta2, beta, 1, st);
      });
      emit_copy_tt<T>(setup, sh, rhs, V[0], 1.0, beta);
      if (full) {
        // Hessenberg right-hand side beta e_1
        double* bsv = bs;
        const double* be = beta;
        setup.steps.push_back([=](hipStream_t st) { scaled_unit(be, bsv, lr, st); });
      } else {
        Blocks<T> bb;
        bb.add(rhs, nullptr, 1.0);
        plan_sketch<T>(setup, pl, sh, bb, S, s, bs);
      }
      const int ss = lr;
      double* n2 = bsn2;
      double* n1 = bsn;
      LsState lsv = ls;
      setup.steps.push_back([=](hipStream_t st) { ls_init(lsv, ss, st); });
      // ||b_s||: dot of the device vector with itself
      {
        std::vector<const double*> pv = {bs};
        const size_t o2 = pl.blob.add(pv);
        setup.steps.push_back([=](hipStream_t st) {
          dot_batched<double>(bl->at<const double*>(o2), bl->at<const double*>(o2), size_t(ss), 1, 1.0, n2, st);
          vec_sqrt(n2, n1, 1, st);
        });
      }
    }

    // ---- iterations.  Each iteration plans its temporaries in a scratch
    // scope: iterations run in sequence (the host waits for each one's status,
    // and a RoundSum's side-stream work joins before the RoundSum ends), so
    // they share that memory.
    for (int k = 0; k < maxiter; ++k) {
      const size_t mk = ar.mark();
      Seq q;
      TT<T> Zk = V[k];
      if (flexible) {
        // flexible cycle (Sec. 3.4): Z_k = T(M(V_k)), and the operator acts on Z_k
        Zk = Z[k];
        plan_precond<T>(q, pl, sh, pc, V[k], Zk, rcfg, omega_);
      }
      Blocks<T> LV = plan_apply<T>(q, pl, sh, op, Zk, transpose);
      plan_roundsum<T>(q, pl, sh, LV, rcfg, omega_, W, nullptr);
      Blocks<T> wb;
      wb.add(W, nullptr, 1.0);
      const int ss = lr, mx = maxiter;
      LsState lsv = ls;
      const double* ctol = &conv_tol;
      const double bdt = bd_tol;
      const bool tik = tikhonov, fa = full;
      // The sketch of W and the least-squares column (a3, a7) need only W:
      // they run on a second side stream beside the inner products and the
      // orthogonalisation RoundSum, and join before the status record.
      std::function<void(hipStream_t)> ls_join;
      if (!full) {
        const size_t from = q.steps.size();
        plan_sketch<T>(q, pl, sh, wb, S, s, Mcols + size_t(k) * s);
        q.steps.push_back([=](hipStream_t st) {
          ls_add_column(lsv, ss, mx, k, *ctol, bdt, st);
          // regularised y_k and residual (Sec. 4.3); the breakdown test keeps
          // the unregularised R factor
          if (tik) ls_tikhonov(lsv, ss, mx, k, *ctol, -1.0, st);
        });
        ls_join = fork_steps(q, from, 1);
      }
      const int j0 = std::max(0, k - kt + 1);
      std::vector<TT<T>> win(V.begin() + j0, V.begin() + k + 1);
      double* hk = h + size_t(k) * kt;
      plan_inner<T>(q, pl, sh, win, wb, hk, 1.0);
      Blocks<T> ob;
      ob.add(W, nullptr, 1.0);
      for (size_t j = 0; j < win.size(); ++j) ob.add(win[j], hk + j, -1.0);
      plan_roundsum<T>(q, pl, sh, ob, rcfg, omega_, V[k + 1], nullptr);
      if (ls_join) q.steps.push_back(ls_join);
      std::vector<const T*> pc = {W.core, V[k + 1].core};
      const size_t off = pl.blob.add(pc);
      const size_t cl = sh.core_len();
      double* s2 = sumsq2 + 2 * k;
      double* om = omega + k;
      const double* resk = res + k;
      const int* rk = V[k + 1].rank;
      T* vc = V[k + 1].core;
      IterStatus* sd = st_dev;
      int* fl = flags;
      double* hcol = Mcols + size_t(k) * lr;
      q.steps.push_back([=](hipStream_t st) {
        dot_batched<T>(bl->at<const T*>(off), bl->at<const T*>(off), cl, 2, 1.0, s2, st);
        if (fa) {
          // Alg. 1: Hessenberg column (h_{1..k}, ||W||) in place of the sketch
          hess_column(hk, k + 1, s2 + 1, hcol, ss, st);
          ls_add_column(lsv, ss, mx, k, *ctol, bdt, st);
          if (tik) ls_tikhonov(lsv, ss, mx, k, *ctol, -1.0, st);
        }
        iter_status(s2, fl, resk, rk, d, bdt, om, sd, st);
        scale_copy<T>(vc, vc, cl, 1.0, nullptr, om, st);
      });
      iter.push_back(std::move(q));
      ar.rewind(mk);
    }

    // ---- final assembly X = RoundSum(sum_i y_i V_i) (sum_i y_i Z_i when flexible)
    Blocks<T> fb;
    for (int i = 0; i < maxiter; ++i) fb.add(flexible ? Z[i] : V[i], y + i, 1.0);
    plan_roundsum<T>(fin, pl, sh, fb, rcfg, omega_, dsol, &nb_final);
    // everything planned after the cycle lies past the iterations' scratch
    ar.seal();
  }

  // Runs one cycle; returns (status, iterations).
  std::pair<int, int> run(hipStream_t st, double eps, double tol_in, double eta, SolveInfo& info) {
    const double ep[2] = {eps, eps};
    TK_HIP(hipMemcpyAsync(eps_pair, ep, sizeof(ep), hipMemcpyHostToDevice, st));
    conv_tol = (full ? 1.0 : eta) * tol_in;
    setup.run(st);
    int status = kNotConverged, kend = maxiter;
    // Iteration k + 1 is enqueued before the host reads iteration k's status,
    // so the device does not drain while the host launches the next
    // iteration.  If k ends the cycle, the extra iteration's results are
    // never read: it writes V[k + 2] (Z[k + 1]), the next least-squares column
    // and status, and the final assembly takes y as it was after iteration k.
    // Near convergence (the last known residual within kSpecMargin of the
    // cycle's tolerance) iterations are enqueued one at a time, so a
    // converging cycle does not pay for an iteration it does not need.
    constexpr double kSpecMargin = 1e6;
    auto enqueue = [&](int k) {
      iter[k].run(st);
      TK_HIP(hipMemcpyAsync(st_host + (k & 1), st_dev, sizeof(IterStatus), hipMemcpyDeviceToHost, st));
      TK_HIP(hipEventRecord(st_ev[k & 1], st));
    };
    double last_res = 1.0;  // relative residual of B before the first iteration
    int queued = 0;         // iterations enqueued so far
    for (int k = 0; k < maxiter; ++k) {
      if (queued == k) enqueue(queued++);
      if (queued == k + 1 && k + 1 < maxiter && last_res > kSpecMargin * conv_tol) enqueue(queued++);
      TK_HIP(hipEventSynchronize(st_ev[k & 1]));
      const IterStatus s = st_host[k & 1];
      last_res = s.res;
      info.hist_sketched.push_back(s.res);
      for (int j = 0; j < sh.d; ++j) info.hist_ranks.push_back(s.rank[j]);
      if (!std::isfinite(s.res) || !std::isfinite(s.omega)) {
        TK_HIP(hipStreamSynchronize(st));  // no enqueued iteration outlives the error
        throw Error{kErrNonFinite, "non-finite sketched residual or basis norm"};
      }
      if (s.breakdown_ls || s.breakdown_w) {
        status = kBreakdown;
        kend = k + 1;
        break;
      }
      if (s.converged) {
        status = kOk;
        kend = k + 1;
        break;
      }
    }
    nb_final = kend;
    // the least-squares solution of the last iteration that counts
    TK_HIP(hipMemcpyAsync(y, ysave + size_t(kend - 1) * maxiter, sizeof(double) * kend, hipMemcpyDeviceToDevice, st));
    fin.run(st);
    if (tikhonov) {
      TK_HIP(hipMemcpyAsync(lam_host, lam, sizeof(double) * kend, hipMemcpyDeviceToHost, st));
      TK_HIP(hipStreamSynchronize(st));
      info.hist_lambda.insert(info.hist_lambda.end(), lam_host, lam_host + kend);
    }
    return {status, kend};
  }
};

// ============================================================ restarted solver
class Solver {
 public:
  Shape sh;
  SolveCfg cfg;
  Blob blob;
  OpDev<double> op64;
  OpDev<float> op32;
  // x[0], x[1]: the iterate alternates between them; x[2]: best iterate so far
  TT<double> b_in, bo, x[3], r, d64;
  bool have_x0 = false;
  std::unique_ptr<Cycle<double>> c64;
  std::unique_ptr<Cycle<float>> c32;
  Seq s_setup, s_x0, s_to_cycle, s_from_cycle, s_first_x, s_xupd[2], s_rnorm[2], s_rround[2], s_keep[2];
  double *bnorm2, *rnorm2;
  double* host2 = nullptr;  // pinned scratch
  // truncation tolerance of the refinement RoundSums, on the device so the
  // loop can tighten it (see solver_run); pinned staging for it and the ranks
  double* eps_out_dev = nullptr;
  double* host_eps = nullptr;
  int* host_rank = nullptr;
  int xc = 0;

  ~Solver() {
    if (host2) (void)hipHostFree(host2);
    if (host_eps) (void)hipHostFree(host_eps);
    if (host_rank) (void)hipHostFree(host_rank);
  }
};

void SolverDel::operator()(Solver* s) const { delete s; }

SolverPtr make_solver(Arena& ar, const Shape& sh, const OpDev<double>& op, const TT<double>& b,
                                    const SolveCfg& cfg, const std::array<const double*, kMaxD>& S,
                                    const std::array<const double*, kMaxD>& omega, const TT<double>* x0,
                                    hipStream_t st, const PrecondT<double>& precond) {
  SolverPtr sv(new Solver());
  Solver& s = *sv;
  s.sh = sh;
  s.cfg = cfg;
  s.op64 = op;
  s.b_in = b;
  Planner pl(ar, s.blob);
  const int d = sh.d;
  TK_CHECK(cfg.maxiter >= 1 && cfg.maxiter <= 64, kErrInvalidArg, "maxiter must be in [1, 64]");
  TK_CHECK(cfg.k_trunc >= 1, kErrInvalidArg, "k_trunc must be >= 1");
  TK_CHECK(cfg.method == 0 || cfg.method == 1, kErrInvalidArg, "method must be 0 (sGMRES) or 1 (GMRES)");
  TK_CHECK(cfg.method == 1 || (cfg.s >= cfg.maxiter && cfg.s <= 256), kErrInvalidArg,
           "sketch size must be in [maxiter, 256]");
  TK_CHECK(cfg.method == 0 || precond.q == 0, kErrUnsupported,
           "the preconditioner runs with the sketched cycles only (method 0)");
  s.bo = alloc_tt<double>(ar, sh);
  s.x[0] = alloc_tt<double>(ar, sh);
  s.x[1] = alloc_tt<double>(ar, sh);
  s.x[2] = alloc_tt<double>(ar, sh);
  s.bnorm2 = ar.alloc<double>(1);
  s.rnorm2 = ar.alloc<double>(1);
  s.eps_out_dev = ar.alloc<double>(2);
  if (!ar.measuring()) {
    TK_HIP(hipHostMalloc(reinterpret_cast<void**>(&s.host2), 2 * sizeof(double), 0));
    TK_HIP(hipHostMalloc(reinterpret_cast<void**>(&s.host_eps), 2 * sizeof(double), 0));
    TK_HIP(hipHostMalloc(reinterpret_cast<void**>(&s.host_rank), kMaxD * sizeof(int), 0));
  }
  Blob* bl = &s.blob;

  // ---- orthonormalise the right-hand side: U_k = Q_k R_k, core <- core x_k R_k
  {
    double* Rk = ar.alloc<double>(size_t(d) * sh.rc * sh.rc);
    double* Ct[2] = {ar.alloc<double>(sh.core_len()), ar.alloc<double>(sh.core_len())};
    for (int k = 0; k < d; ++k) {
      std::vector<QrTask> qt = {QrTask{b.U[k], s.bo.U[k], Rk + size_t(k) * sh.rc * sh.rc, b.rank + k}};
      const size_t off = s.blob.add(qt);
      const int n = sh.n[k], rc = sh.rc;
      s.s_setup.steps.push_back([=](hipStream_t st) { qr_batched(bl->at<QrTask>(off), 1, n, rc, nullptr, st); });
    }
    int dims[kMaxD];
    for (int j = 0; j < d; ++j) dims[j] = sh.rc;
    const double* cur = b.core;
    for (int k = d - 1; k >= 0; --k) {
      double* outp = (k == 0) ? s.bo.core : Ct[k & 1];
      plan_ttm<double>(s.s_setup, pl, d, dims, k, sh.rc, cur, Rk + size_t(k) * sh.rc * sh.rc, sh.rc, false, outp);
      cur = outp;
    }
    const int* br = b.rank;
    int* bor = s.bo.rank;
    std::vector<const double*> pc = {s.bo.core};
    const size_t off = s.blob.add(pc);
    const size_t cl = sh.core_len();
    double* bn = s.bnorm2;
    s.s_setup.steps.push_back([=](hipStream_t st) {
      copy_ints(br, bor, d, st);
      dot_batched<double>(bl->at<const double*>(off), bl->at<const double*>(off), cl, 1, 1.0, bn, st);
    });
  }

  // ---- cycle in the requested precision
  RoundCfg outer;
  outer.eps = 1e-2 * cfg.tol;
  outer.eps_dev = s.eps_out_dev;  // {eps, tau}, set by solver_run
  // full sketch width in the refinement RoundSums: a correction far below x
  // (a residual far below B and L(x)) is invisible to the effective-rank rule,
  // whose Gram of weighted factors puts it under its rounding level
  outer.force_s = sh.sc();
  // and Householder range-finder bases: the rounding of x + d must keep x to
  // O(u), or the residual floors at about kappa * 1e-14 (Cholesky-QR bases)
  outer.householder = true;
  if (cfg.form == 0) {
    s.c64 = std::make_unique<Cycle<double>>();
    auto& c = *s.c64;
    c.sh = sh;
    c.maxiter = cfg.maxiter;
    c.kt = cfg.k_trunc;
    c.s = cfg.s;
    c.tikhonov = cfg.tikhonov;
    c.full = cfg.method == 1;
    c.plan(pl, op, cfg.transpose, S, omega, precond);
    s.r = c.rhs;     // the cycle reads its right-hand side in place
    s.d64 = c.dsol;  // and leaves its solution in place
  } else {
    // FP32 copies of operator factors and sketches
    s.op32.nterms = op.nterms;
    s.op32.alpha = op.alpha;
    std::map<const double*, float*> conv;
    auto to32 = [&](const double* src, size_t len) -> float* {
      auto it = conv.find(src);
      if (it != conv.end()) return it->second;
      float* dst = ar.alloc<float>(len);
      s.s_setup.steps.push_back([=](hipStream_t st) { cast_copy<double, float>(src, dst, len, st); });
      conv[src] = dst;
      return dst;
    };
    for (int j = 0; j < op.nterms; ++j)
      for (int k = 0; k < d; ++k) {
        const double* A = op.A[j * d + k];
        s.op32.A.push_back(A ? to32(A, size_t(sh.n[k]) * sh.n[k]) : nullptr);
      }
    std::array<const float*, kMaxD> S32{}, O32{};
    const bool sketched = cfg.method == 0;  // full Arnoldi reads no sketch S
    for (int k = 0; k < d; ++k) {
      const double* src_s = S[k];
      const double* src_o = omega[k];
      const size_t ls = sketched ? size_t(sh.n[k]) * cfg.s : 0, lo = size_t(sh.n[k]) * sh.sc();
      float* ds = sketched ? ar.alloc<float>(ls) : nullptr;
      float* dom = ar.alloc<float>(lo);
      s.s_setup.steps.push_back([=](hipStream_t st) {
        if (ls) cast_copy<double, float>(src_s, ds, ls, st);
        cast_copy<double, float>(src_o, dom, lo, st);
      });
      S32[k] = ds;
      O32[k] = dom;
    }
    PrecondT<float> pc32;
    pc32.q = precond.q;
    if (precond.q > 0)
      for (int k = 0; k < d; ++k) {
        const size_t n = size_t(sh.n[k]);
        pc32.V[k] = to32(precond.V[k], n * n);
        pc32.lam[k] = to32(precond.lam[k], n);
      }
    s.c32 = std::make_unique<Cycle<float>>();
    auto& c = *s.c32;
    c.sh = sh;
    c.maxiter = cfg.maxiter;
    c.kt = cfg.k_trunc;
    c.s = cfg.s;
    c.tikhonov = cfg.tikhonov;
    c.full = cfg.method == 1;
    c.bd_tol = 1e-6;
    c.plan(pl, s.op32, cfg.transpose, S32, O32, pc32);
    s.r = alloc_tt<double>(ar, sh);
    s.d64 = alloc_tt<double>(ar, sh);
    emit_cast_tt<double, float>(s.s_to_cycle, sh, s.r, c.rhs);
    emit_cast_tt<float, double>(s.s_from_cycle, sh, c.dsol, s.d64);
  }
  // the first right-hand side is the orthonormalised B
  emit_copy_tt<double>(s.s_setup, sh, s.bo, s.r);
  if (cfg.form != 0) {
    // FP32 form: the first iterate is the FP64 rounding of the cycle's solution,
    // like every later update x <- RoundSum(x + d), so that x always carries
    // FP64-orthonormal factors
    Blocks<double> fb;
    fb.add(s.d64, nullptr, 1.0);
    plan_roundsum<double>(s.s_first_x, pl, sh, fb, outer, omega, s.x[0], nullptr);
  } else {
    emit_copy_tt<double>(s.s_first_x, sh, s.d64, s.x[0]);
  }
  if (x0) {
    s.have_x0 = true;
    emit_copy_tt<double>(s.s_x0, sh, *x0, s.x[0]);
  }
  for (int c = 0; c < 2; ++c) {
    // x[1-c] = RoundSum(x[c] + d)
    Blocks<double> xb;
    xb.add(s.x[c], nullptr, 1.0);
    xb.add(s.d64, nullptr, 1.0);
    plan_roundsum<double>(s.s_xupd[c], pl, sh, xb, outer, omega, s.x[1 - c], nullptr);
    // residual B - L(x[c]): exact norm, then rounding into the next right-hand side
    Blocks<double> lx = plan_apply<double>(s.s_rnorm[c], pl, sh, op, s.x[c], cfg.transpose);
    Blocks<double> rb;
    rb.add(s.bo, nullptr, 1.0);
    for (int j = 0; j < lx.size(); ++j) rb.add(lx.core[j], lx.U[j], lx.rank[j], nullptr, -lx.cscale[j]);
    plan_exact_norm2(s.s_rnorm[c], pl, sh, rb, s.rnorm2);
    plan_roundsum<double>(s.s_rround[c], pl, sh, rb, outer, omega, s.r, nullptr);
    emit_copy_tt<double>(s.s_keep[c], sh, s.x[c], s.x[2]);
  }
  // upload the tables
  s.blob.dev = ar.alloc<unsigned char>(std::max<size_t>(s.blob.host.size(), 16));
  if (!ar.measuring())
    TK_HIP(hipMemcpyAsync(s.blob.dev, s.blob.host.data(), s.blob.host.size(), hipMemcpyHostToDevice, st));
  return sv;
}

static double read_scalar(Solver& s, const double* dev, hipStream_t st) {
  TK_HIP(hipMemcpyAsync(s.host2, dev, sizeof(double), hipMemcpyDeviceToHost, st));
  TK_HIP(hipStreamSynchronize(st));
  return s.host2[0];
}

void solver_run(Solver& s, TT<double>& x_out, SolveInfo& info, hipStream_t st) {
  const auto t0 = std::chrono::steady_clock::now();
  const SolveCfg& cfg = s.cfg;
  const bool fp32 = cfg.form != 0;
  const double eps_min = cfg.eps_min > 0 ? cfg.eps_min : (fp32 ? 1e-6 : 1e-13);
  const double tin_floor = cfg.tol_inner_floor > 0 ? cfg.tol_inner_floor : (fp32 ? 1e-5 : 1e-13);
  info = SolveInfo{};
  // truncation tolerance of the refinement RoundSums: 1e-2 tol, tightened below
  double eps_out = 1e-2 * cfg.tol;
  auto set_eps_out = [&](double e) {
    s.host_eps[0] = e;
    s.host_eps[1] = e;
    TK_HIP(hipMemcpyAsync(s.eps_out_dev, s.host_eps, 2 * sizeof(double), hipMemcpyHostToDevice, st));
    TK_HIP(hipStreamSynchronize(st));
  };
  set_eps_out(eps_out);
  size_t floor_from = 0;  // the floor test looks at cycles from this index on
  s.s_setup.run(st);
  const double bnorm = std::sqrt(read_scalar(s, s.bnorm2, st));
  s.xc = 0;
  bool have_x = false;
  double rnorm = bnorm;
  // best iterate: refinement cycles on a rank floor can raise the residual
  // (x + d rounded back to the rank cap), so a solve that does not converge
  // returns the iterate with the smallest true residual
  double best = std::numeric_limits<double>::infinity();
  if (s.have_x0) {
    s.s_x0.run(st);
    have_x = true;
    s.s_rnorm[0].run(st);
    rnorm = std::sqrt(read_scalar(s, s.rnorm2, st));
    s.s_keep[0].run(st);
    best = rnorm;
    s.s_rround[0].run(st);
  }
  int status = kNotConverged;
  for (int c = 0; c < cfg.max_restarts; ++c) {
    if (rnorm <= cfg.tol * bnorm) {
      status = kOk;
      break;
    }
    info.cycles++;
    const double tol_in = std::min(0.5, std::max(cfg.tol * bnorm / rnorm, tin_floor));
    const double eps = cfg.eps_trunc > 0 ? cfg.eps_trunc : std::max(1e-2 * tol_in, eps_min);
    std::pair<int, int> r;
    if (fp32) {
      s.s_to_cycle.run(st);
      r = s.c32->run(st, eps, tol_in, cfg.eta, info);
      s.s_from_cycle.run(st);
    } else {
      r = s.c64->run(st, eps, tol_in, cfg.eta, info);
    }
    info.iters += r.second;
    if (!have_x) {
      s.s_first_x.run(st);
      s.xc = 0;
      have_x = true;
    } else {
      s.s_xupd[s.xc].run(st);
      s.xc = 1 - s.xc;
    }
    s.s_rnorm[s.xc].run(st);
    rnorm = std::sqrt(read_scalar(s, s.rnorm2, st));
    if (!std::isfinite(rnorm)) throw Error{kErrNonFinite, "non-finite residual norm"};
    if (rnorm < best) {
      best = rnorm;
      s.s_keep[s.xc].run(st);
    }
    info.hist_true.push_back(rnorm / bnorm);
    info.hist_time.push_back(std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
    if (rnorm <= cfg.tol * bnorm) {
      status = kOk;
      break;
    }
    const size_t nh = info.hist_true.size();
    if (nh >= floor_from + 3 && info.hist_true[nh - 1] > 0.9 * info.hist_true[nh - 2] &&
        info.hist_true[nh - 2] > 0.9 * info.hist_true[nh - 3]) {
      // A floor reached with every rank of x below the cap comes from the
      // update's truncation (rounding x + d to relative accuracy eps moves the
      // residual by up to about kappa eps): tighten it and go on.
      TK_HIP(hipMemcpyAsync(s.host_rank, s.x[s.xc].rank, s.sh.d * sizeof(int), hipMemcpyDeviceToHost, st));
      TK_HIP(hipStreamSynchronize(st));
      int rmax = 0;
      for (int k = 0; k < s.sh.d; ++k) rmax = std::max(rmax, s.host_rank[k]);
      if (rmax < s.sh.cap && eps_out > kEpsOuterMin) {
        eps_out = std::max(1e-2 * eps_out, kEpsOuterMin);
        set_eps_out(eps_out);
        floor_from = nh - 1;
      } else {
        status = kRankFloor;
        break;
      }
    }
    s.s_rround[s.xc].run(st);
  }
  if (!have_x) {
    // zero right-hand side: x = 0 (rank-1 zero tensor)
    const Shape& sh = s.sh;
    TT<double> x = s.x[0];
    std::vector<int> ones(kMaxD, 1);
    TK_HIP(hipMemsetAsync(x.core, 0, sh.core_len() * sizeof(double), st));
    for (int k = 0; k < sh.d; ++k) {
      TK_HIP(hipMemsetAsync(x.U[k], 0, size_t(sh.n[k]) * sh.rc * sizeof(double), st));
      const double one = 1.0;
      TK_HIP(hipMemcpyAsync(x.U[k], &one, sizeof(double), hipMemcpyHostToDevice, st));
    }
    TK_HIP(hipMemcpyAsync(x.rank, ones.data(), sizeof(int) * kMaxD, hipMemcpyHostToDevice, st));
    TK_HIP(hipStreamSynchronize(st));
    s.xc = 0;
  }
  if (status != kOk && have_x && best < rnorm) {
    s.xc = 2;
    rnorm = best;
  }
  x_out = s.x[s.xc];
  info.status = status;
  info.true_relres = rnorm / (bnorm > 0 ? bnorm : 1.0);
  TK_HIP(hipStreamSynchronize(st));
  info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

TT<double> solver_solution(Solver& s) { return s.x[s.xc]; }
TT<double> solver_slot(Solver& s, int i) { return s.x[i]; }  // i in [0, 3)
int solver_slot_index(Solver& s) { return s.xc; }

template struct Cycle<double>;
template struct Cycle<float>;

}  // namespace tk
