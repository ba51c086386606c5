// Multilinear Nystrom (MLN) sketching, summation and recovery of Tucker
// tensors and the MLN-Tucker sGMRES solver built on them (Sec. 3.3).
//
// Sketching is linear in the tensor, so the sketch of a block sum is formed
// directly as the coefficient-weighted sum of the block sketches (the sketch
// of every summand followed by their sum), with the Khatri-Rao range sketch
// and the core projection that RoundSum uses.  Recovery forms
//   X~ = G_Psi x_1 P_1 ... x_d P_d,   P_k = F_k (Psi_k^T F_k)^+,
// which does not depend on how the pseudoinverse is factored.  Here it comes
// from a column-pivoted QR of A_k = Psi_k^T F_k (rt x r) with a rank cut
// relative to its largest column, A_k ~ Q1 Rh with Rh (rho x r) of full row
// rank, and a Householder QR Rh^T = Q2 R2, so that A_k^+ = Q2 R2^{-T} Q1^T:
// the recovered factors are F_k Q2 (n_k x rho) and the core is
// G_Psi x_k (Q1 R2^{-1})^T.  No Gram matrix is formed, so the rank cut acts
// on the singular values of A_k themselves, as the pseudoinverse does.
#include <chrono>
#include <cmath>
#include <map>

#include "engine.hpp"

namespace tk {

namespace {

// Pseudoinverse cut: basis columns of Psi_k^T F_k whose remainder is at or
// below this fraction of the largest column are dropped.
constexpr double kMlnCut = 1e-12;

std::vector<std::vector<int>> group_modes(const Shape& sh) {
  std::map<int, std::vector<int>> m;
  for (int k = 0; k < sh.d; ++k) m[sh.n[k]].push_back(k);
  std::vector<std::vector<int>> out;
  for (auto& kv : m) out.push_back(kv.second);
  return out;
}

size_t ipow_sz(int b, int e) {
  size_t v = 1;
  for (int i = 0; i < e; ++i) v *= size_t(b);
  return v;
}

// One launch of y_t = (acc ? y_t : 0) + sum_j s_j c_j x_tj over every part
// (core and factor sketches) of MLN sketches.  xs[j] / cs[j] / ss[j] are the
// terms; `limit` (optional host int) caps the number of terms at run time.
void emit_mln_lincomb(Seq& q, Planner& pl, const Shape& sh, int rt, int r, const MlnSk& y,
                      const std::vector<MlnSk>& xs, const std::vector<const double*>& cs,
                      const std::vector<double>& ss, bool accumulate, const int* limit) {
  const int d = sh.d, nx = int(xs.size()), parts = d + 1;
  TK_CHECK(nx >= 1 && nx <= kLincombMax, kErrUnsupported, "MLN sum: too many terms");
  Blob* bl = &pl.blob;
  std::vector<double*> ys;
  std::vector<const double*> xt;
  std::vector<size_t> lens;
  ys.push_back(y.core);
  lens.push_back(ipow_sz(rt, d));
  for (auto& x : xs) xt.push_back(x.core);
  for (int k = 0; k < d; ++k) {
    ys.push_back(y.F[k]);
    lens.push_back(size_t(sh.n[k]) * r);
    for (auto& x : xs) xt.push_back(x.F[k]);
  }
  size_t maxlen = 0;
  for (size_t l : lens) maxlen = std::max(maxlen, l);
  const size_t oy = pl.blob.add(ys), ox = pl.blob.add(xt), oc = pl.blob.add(cs), os = pl.blob.add(ss),
               ol = pl.blob.add(lens);
  const int acc = accumulate ? 1 : 0;
  q.steps.push_back([=](hipStream_t st) {
    lincomb<double>(bl->at<double*>(oy), bl->at<const double*>(ox), bl->at<const double*>(oc), bl->at<double>(os),
                    bl->at<size_t>(ol), parts, nx, maxlen, acc, limit ? *limit : nx, st);
  });
}

// The memory-efficient truncation of a sketch: leading rts^d core entries and
// leading rs factor columns.
void emit_mln_truncate(Seq& q, const Shape& sh, int rt, int r, const MlnSk& src, int rts, int rs, const MlnSk& dst) {
  const int d = sh.d;
  int sd[kMaxD] = {1, 1, 1, 1}, sv[kMaxD] = {1, 1, 1, 1}, dd[kMaxD] = {1, 1, 1, 1};
  for (int k = 0; k < d; ++k) {
    sd[k] = rt;
    sv[k] = rts;
    dd[k] = rts;
  }
  std::array<size_t, kMaxD> fl{};
  for (int k = 0; k < d; ++k) fl[k] = size_t(sh.n[k]) * rs;  // leading columns are contiguous
  (void)r;
  q.steps.push_back([=](hipStream_t st) {
    core_recap<double>(src.core, sd, sv, dst.core, dd, d, st);
    for (int k = 0; k < d; ++k) scale_copy<double>(src.F[k], dst.F[k], fl[k], 1.0, nullptr, nullptr, st);
  });
}

}  // namespace

MlnSk alloc_mln(Arena& ar, const Shape& sh, int r, int rt) {
  MlnSk s;
  s.core = ar.alloc<double>(ipow_sz(rt, sh.d));
  for (int k = 0; k < sh.d; ++k) s.F[k] = ar.alloc<double>(size_t(sh.n[k]) * r);
  return s;
}

void plan_mln_sketch(Seq& q, Planner& pl, const Shape& sh, const Blocks<double>& in,
                     const std::array<const double*, kMaxD>& Psi, int r, int rt, const MlnSk& out, double* diag) {
  const int d = sh.d, nb = in.size();
  TK_CHECK(nb >= 1, kErrInvalidArg, "MLN sketch of an empty sum");
  TK_CHECK(out.core != nullptr, kErrInvalidArg, "MLN sketch: core output is NULL");
  TK_CHECK(r >= 1 && r <= rt && r <= 64, kErrUnsupported, "MLN sketch: need 1 <= r <= min(r + p, 64)");
  Blob* bl = &pl.blob;
  double* coef = pl.ar.alloc<double>(nb);
  const size_t oc = pl.blob.add(in.cptr), os = pl.blob.add(in.cscale);
  q.steps.push_back([=](hipStream_t st) {
    gather_coef(bl->at<const double*>(oc), bl->at<double>(os), nb, coef, st);
  });
  std::array<double*, kMaxD> F{};
  for (int k = 0; k < d; ++k) F[k] = out.F[k];
  // F_k = X_(k) (Khatri-Rao of Psi_j[:, :r], j != k)
  plan_krp_range<double>(q, pl, sh, in, coef, Psi, r, F, nullptr);
  // G_Psi = X x_k Psi_k^T
  plan_core_projection<double>(q, pl, sh, in, coef, Psi, rt, out.core, nullptr);
  if (diag) {
    size_t stride = 0, pw = 1;
    for (int k = 0; k < d; ++k) {
      stride += pw;
      pw *= size_t(rt);
    }
    const double* c = out.core;
    q.steps.push_back([=](hipStream_t st) { strided_gather<double>(c, stride, rt, diag, st); });
  }
}

void plan_mln_recovery(Seq& q, Planner& pl, const Shape& sh, const MlnSk& sk,
                       const std::array<const double*, kMaxD>& Psi, int r, int rt, const TT<double>& out) {
  const int d = sh.d, rc = sh.rc;
  TK_CHECK(r >= 1 && r <= 64 && r <= rc, kErrUnsupported, "MLN recovery: need 1 <= r <= min(64, capacity)");
  TK_CHECK(rt >= r && rt <= 512, kErrUnsupported, "MLN recovery: need r <= r + p <= 512");
  Arena& ar = pl.ar;
  Blob* bl = &pl.blob;
  std::array<double*, kMaxD> A{}, Q1{}, Rt{}, Q2{}, R2{}, M{};
  int* rho = ar.alloc<int>(kMaxD);
  for (int k = 0; k < d; ++k) {
    A[k] = ar.alloc<double>(size_t(rt) * r);
    Q1[k] = ar.alloc<double>(size_t(rt) * r);
    Rt[k] = ar.alloc<double>(size_t(r) * r);
    Q2[k] = ar.alloc<double>(size_t(r) * r);
    R2[k] = ar.alloc<double>(size_t(r) * r);
    M[k] = ar.alloc<double>(size_t(rt) * r);
  }
  const auto groups = group_modes(sh);
  // A_k = Psi_k^T F_k  (rt x r)
  for (auto& modes : groups) {
    const int n = sh.n[modes[0]];
    std::vector<const double*> a, b;
    std::vector<double*> c;
    for (int k : modes) {
      a.push_back(Psi[k]);
      b.push_back(sk.F[k]);
      c.push_back(A[k]);
    }
    plan_gemm_batched<double>(q, pl, true, false, rt, r, n, a, n, b, n, c, rt, 1.0);
  }
  // A_k ~ Q1 Rh (pivoted, rank cut), then Rh^T = Q2 R2
  {
    std::vector<QrPivTask> pt;
    std::vector<QrTask> qt;
    for (int k = 0; k < d; ++k) {
      QrPivTask t{A[k], nullptr, Q1[k], nullptr, nullptr};
      t.Rt = Rt[k];
      t.rank_out = rho + k;
      pt.push_back(t);
      qt.push_back(QrTask{Rt[k], Q2[k], R2[k], rho + k});
    }
    const size_t op = pl.blob.add(pt), oq = pl.blob.add(qt);
    q.steps.push_back([=](hipStream_t st) {
      qr_piv_batched(bl->at<QrPivTask>(op), d, rt, r, kMlnCut, st);
      qr_batched(bl->at<QrTask>(oq), d, r, r, nullptr, st);
    });
  }
  // factors F_k Q2 (n_k x r; columns >= rho are zero)
  for (auto& modes : groups) {
    const int n = sh.n[modes[0]];
    std::vector<const double*> a, b;
    std::vector<double*> c;
    for (int k : modes) {
      a.push_back(sk.F[k]);
      b.push_back(Q2[k]);
      c.push_back(out.U[k]);
    }
    plan_gemm_batched<double>(q, pl, false, false, n, r, r, a, n, b, r, c, n, 1.0);
  }
  // M_k = Q1 R2^{-1} (rt x r)
  {
    std::vector<TrsmTask> tt;
    for (int k = 0; k < d; ++k) tt.push_back(TrsmTask{Q1[k], R2[k], M[k]});
    const size_t ot = pl.blob.add(tt);
    q.steps.push_back([=](hipStream_t st) { trsm_rows(bl->at<TrsmTask>(ot), d, rt, r, nullptr, st); });
  }
  // core G_Psi x_1 M_1^T ... x_d M_d^T (r^d), placed in the capacity layout
  int dims[kMaxD];
  for (int j = 0; j < d; ++j) dims[j] = rt;
  const size_t tl = ipow_sz(rt, d - 1) * size_t(r);
  double* T0 = ar.alloc<double>(tl);
  double* T1 = ar.alloc<double>(tl);
  double* Cr = (r == rc) ? out.core : ar.alloc<double>(ipow_sz(r, d));
  const double* cur = sk.core;
  for (int k = 0; k < d; ++k) {
    double* dst = (k == d - 1) ? Cr : ((k & 1) ? T1 : T0);
    plan_ttm<double>(q, pl, d, dims, k, r, cur, M[k], rt, true, dst);
    dims[k] = r;
    cur = dst;
  }
  std::array<double*, kMaxD> U{};
  std::array<size_t, kMaxD> nl{};
  for (int k = 0; k < d; ++k) {
    U[k] = out.U[k];
    nl[k] = size_t(sh.n[k]);
  }
  int* orank = out.rank;
  double* oc = out.core;
  q.steps.push_back([=](hipStream_t st) {
    if (r < rc) {
      int sd[kMaxD] = {1, 1, 1, 1}, dd[kMaxD] = {1, 1, 1, 1};
      for (int k = 0; k < d; ++k) {
        sd[k] = r;
        dd[k] = rc;
      }
      core_recap<double>(Cr, sd, sd, oc, dd, d, st);
      for (int k = 0; k < d; ++k) fill<double>(U[k] + nl[k] * r, nl[k] * (rc - r), 0.0, st);
    }
    ints_at_least(rho, orank, d, 1, st);
  });
}

// ============================================================ MLN-Tucker sGMRES
// One run of the short-recurrence sketched GMRES with every basis tensor kept
// as an MLN sketch (Sec. 3.3).  Per iteration: W = recover(sketch(L(V_i))),
// whose diag(G_Psi) is the new column of the sketched least-squares matrix;
// h_j = <V_j, W> over the window; the window is subtracted on the sketches;
// W is recovered again, V_{i+1} = W / ||W|| and its sketch is stored.  The
// solution is the recovery of sum_i y_i sketch(V_i).  Every iteration replays
// the plan built for its index; the temporaries of one iteration are reused
// by the next.
//
// Flexible preconditioning (Sec. 3.4): Z_i = recover(sketch(M(V_i))) and L
// acts on Z_i; the sketches of the Z_i (truncated at once in the
// memory-efficient variant) replace those of the V_i in the solution.  The
// 2q + 1 terms of M(V_i) are built in the spectral basis (V_k^T U_k with row
// scalings), where the sketch with Psi_k of a term with factors V_k W_k
// equals the sketch with Psi'_k = V_k^T Psi_k of the term with factors W_k,
// except for the factor sketches, which come out as V_k^T F_k: one GEMM with
// V_k maps them back.  Psi'_k is formed once per solve.
class MlnSolver {
 public:
  Shape sh;
  MlnCfg cfg;
  int r = 0, rt = 0, kt = 1, maxiter = 1, rts = 0, rs = 0;
  Blob blob;
  OpDev<double> op;
  TT<double> b, X;
  std::vector<TT<double>> V;
  std::vector<MlnSk> Sfull;  // full sketches (a ring of kt + 2 with save_memory)
  std::vector<MlnSk> Strunc; // truncated copies of every stored sketch (save_memory)
  MlnSk Wsk, Fsk;
  PrecondT<double> pc;
  std::vector<MlnSk> Zsk;    // sketches of Z_i (truncated with save_memory)
  MlnSk Zfull;               // save_memory: the full sketch of the current Z_i
  TT<double> Z;              // recovered Z_i
  std::array<double*, kMaxD> Psip{};  // V_k^T Psi_k
  double *bnorm2, *beta, *d0, *bs, *bsn2, *bsn, *Mcols, *h, *s2, *omega, *rnorm2;
  double *Hv, *tau, *R, *qtb, *y, *res, *nrmM2, *lam;
  int* flags;
  IterStatus* st_dev;
  IterStatus* st_host = nullptr;
  double* host2 = nullptr;
  double* lam_host = nullptr;
  Seq setup, fin;
  std::vector<Seq> iter;
  int nb_final = 0;
  double conv_tol = 0.0;
  LsState ls{};

  ~MlnSolver() {
    if (st_host) (void)hipHostFree(st_host);
    if (host2) (void)hipHostFree(host2);
    if (lam_host) (void)hipHostFree(lam_host);
  }
  const MlnSk& full(int i) const { return Sfull[cfg.save_memory ? i % (kt + 2) : i]; }
};

void MlnSolverDel::operator()(MlnSolver* s) const { delete s; }

MlnSolverPtr make_mln_solver(Arena& ar, const Shape& sh, const OpDev<double>& op, const TT<double>& b,
                             const MlnCfg& cfg, const std::array<const double*, kMaxD>& Psi, hipStream_t st,
                             const PrecondT<double>& precond) {
  MlnSolverPtr sp(new MlnSolver());
  MlnSolver& s = *sp;
  s.sh = sh;
  s.cfg = cfg;
  s.op = op;
  s.b = b;
  s.r = cfg.r;
  s.rt = cfg.r + cfg.p;
  s.kt = cfg.k_trunc;
  s.maxiter = cfg.maxiter;
  const int d = sh.d, r = s.r, rt = s.rt, mx = s.maxiter, kt = s.kt;
  TK_CHECK(sh.rc == r, kErrInvalidArg, "internal: MLN solver capacity must equal r");
  TK_CHECK(mx >= 1 && mx <= 64, kErrUnsupported, "maxiter must be in [1, 64]");
  TK_CHECK(kt >= 1, kErrInvalidArg, "k_trunc must be >= 1");
  TK_CHECK(rt <= 256, kErrUnsupported, "r + p above 256");
  if (cfg.save_memory) {
    s.rs = cfg.r_sol;
    s.rts = cfg.r_sol + cfg.p_sol;
    TK_CHECK(s.rs >= 1 && s.rs <= r && s.rts >= s.rs && s.rts <= rt, kErrInvalidArg,
             "save_memory needs 1 <= r_sol <= r and r_sol <= r_sol + p_sol <= r + p");
  }
  s.pc = precond;
  const bool flex = precond.q > 0;
  Planner pl(ar, s.blob);
  Blob* bl = &s.blob;

  // ---- persistent state
  for (int i = 0; i <= mx; ++i) s.V.push_back(alloc_tt<double>(ar, sh));
  s.X = alloc_tt<double>(ar, sh);
  const int nfull = cfg.save_memory ? std::min(kt + 2, mx + 1) : mx + 1;
  for (int i = 0; i < nfull; ++i) s.Sfull.push_back(alloc_mln(ar, sh, r, rt));
  if (cfg.save_memory && !flex)
    for (int i = 0; i <= mx; ++i) s.Strunc.push_back(alloc_mln(ar, sh, s.rs, s.rts));
  if (flex) {
    for (int i = 0; i < mx; ++i)
      s.Zsk.push_back(cfg.save_memory ? alloc_mln(ar, sh, s.rs, s.rts) : alloc_mln(ar, sh, r, rt));
    if (cfg.save_memory) s.Zfull = alloc_mln(ar, sh, r, rt);
    s.Z = alloc_tt<double>(ar, sh);
    for (int k = 0; k < d; ++k) s.Psip[k] = ar.alloc<double>(size_t(sh.n[k]) * rt);
  }
  s.Wsk = alloc_mln(ar, sh, r, rt);
  s.Fsk = cfg.save_memory ? alloc_mln(ar, sh, s.rs, s.rts) : alloc_mln(ar, sh, r, rt);
  s.bnorm2 = ar.alloc<double>(1);
  s.beta = ar.alloc<double>(1);
  s.d0 = ar.alloc<double>(rt);
  s.bs = ar.alloc<double>(rt);
  s.bsn2 = ar.alloc<double>(1);
  s.bsn = ar.alloc<double>(1);
  s.Mcols = ar.alloc<double>(size_t(rt) * mx);
  s.h = ar.alloc<double>(size_t(mx) * kt);
  s.s2 = ar.alloc<double>(size_t(mx) * 2);
  s.omega = ar.alloc<double>(mx);
  s.rnorm2 = ar.alloc<double>(1);
  s.Hv = ar.alloc<double>(size_t(rt) * mx);
  s.tau = ar.alloc<double>(mx);
  s.R = ar.alloc<double>(size_t(mx) * mx);
  s.qtb = ar.alloc<double>(rt);
  s.y = ar.alloc<double>(mx);
  s.res = ar.alloc<double>(mx);
  s.nrmM2 = ar.alloc<double>(1);
  s.lam = ar.alloc<double>(mx);
  s.flags = ar.alloc<int>(4);
  s.st_dev = ar.alloc<IterStatus>(1);
  s.ls = LsState{s.Mcols, s.bs, s.Hv, s.tau, s.R, s.qtb, s.y, s.res, s.nrmM2, s.flags, 0.0, s.bsn, s.lam};
  if (!ar.measuring()) {
    TK_HIP(hipHostMalloc(reinterpret_cast<void**>(&s.st_host), sizeof(IterStatus), 0));
    TK_HIP(hipHostMalloc(reinterpret_cast<void**>(&s.host2), 2 * sizeof(double), 0));
    TK_HIP(hipHostMalloc(reinterpret_cast<void**>(&s.lam_host), sizeof(double) * mx, 0));
  }
  const size_t cl = sh.core_len();
  auto store = [&](Seq& q, int i) {
    // sketch of V_i into its slot (and its truncated copy)
    Blocks<double> vb;
    vb.add(s.V[i], nullptr, 1.0);
    plan_mln_sketch(q, pl, sh, vb, Psi, r, rt, s.full(i), i == 0 ? s.d0 : nullptr);
    if (cfg.save_memory && !flex) emit_mln_truncate(q, sh, rt, r, s.full(i), s.rts, s.rs, s.Strunc[i]);
  };
  // Psi'_k = V_k^T Psi_k, one GEMM launch per group of equal mode size
  std::array<const double*, kMaxD> Psip{};
  for (int k = 0; k < d; ++k) Psip[k] = s.Psip[k];
  if (flex)
    for (auto& modes : group_modes(sh)) {
      const int n = sh.n[modes[0]];
      std::vector<const double*> a, bb;
      std::vector<double*> c;
      for (int k : modes) {
        a.push_back(precond.V[k]);
        bb.push_back(Psi[k]);
        c.push_back(s.Psip[k]);
      }
      plan_gemm_batched<double>(s.setup, pl, true, false, n, rt, n, a, n, bb, n, c, n, 1.0);
    }

  // ---- setup: beta = ||b|| (exact), V_1 = b / beta, stored sketch of V_1,
  //      b_s = beta diag(G_Psi(V_1))
  {
    const size_t mk = ar.mark();
    Blocks<double> bb;
    bb.add(b, nullptr, 1.0);
    plan_exact_norm2(s.setup, pl, sh, bb, s.bnorm2);
    const TT<double> v0 = s.V[0];
    double* bn2 = s.bnorm2;
    double* be = s.beta;
    std::array<size_t, kMaxD> fl{};
    for (int k = 0; k < d; ++k) fl[k] = size_t(sh.n[k]) * sh.rc;
    const TT<double> bt = b;
    s.setup.steps.push_back([=](hipStream_t st) {
      vec_sqrt(bn2, be, 1, st);
      scale_copy<double>(bt.core, v0.core, cl, 1.0, nullptr, be, st);
      for (int k = 0; k < d; ++k) scale_copy<double>(bt.U[k], v0.U[k], fl[k], 1.0, nullptr, nullptr, st);
      copy_ints(bt.rank, v0.rank, d, st);
    });
    store(s.setup, 0);
    double* d0 = s.d0;
    double* bsv = s.bs;
    double* n2 = s.bsn2;
    double* n1 = s.bsn;
    LsState lsv = s.ls;
    std::vector<const double*> pv = {bsv};
    const size_t o2 = pl.blob.add(pv);
    s.setup.steps.push_back([=](hipStream_t st) {
      scale_copy<double>(d0, bsv, size_t(rt), 1.0, be, nullptr, st);
      ls_init(lsv, rt, st);
      dot_batched<double>(bl->at<const double*>(o2), bl->at<const double*>(o2), size_t(rt), 1, 1.0, n2, st);
      vec_sqrt(n2, n1, 1, st);
    });
    ar.rewind(mk);
  }

  // ---- iterations
  for (int k = 0; k < mx; ++k) {
    const size_t mk = ar.mark();
    Seq q;
    const TT<double> vn = s.V[k + 1];
    const TT<double>* opnd = &s.V[k];
    if (flex) {
      // sketch of M(V_k): core straight into its slot, factor sketches V_k^T F_k
      // into temporaries mapped back by V_k; then Z_k = recover(sketch)
      const MlnSk zf = cfg.save_memory ? s.Zfull : s.Zsk[k];
      MlnSk zt;
      zt.core = zf.core;
      for (int j = 0; j < d; ++j) zt.F[j] = ar.alloc<double>(size_t(sh.n[j]) * r);
      Blocks<double> mt = plan_precond_terms<double>(q, pl, sh, precond, s.V[k]);
      plan_mln_sketch(q, pl, sh, mt, Psip, r, rt, zt, nullptr);
      for (auto& modes : group_modes(sh)) {
        const int n = sh.n[modes[0]];
        std::vector<const double*> a, bb;
        std::vector<double*> c;
        for (int j : modes) {
          a.push_back(precond.V[j]);
          bb.push_back(zt.F[j]);
          c.push_back(zf.F[j]);
        }
        plan_gemm_batched<double>(q, pl, false, false, n, r, n, a, n, bb, n, c, n, 1.0);
      }
      plan_mln_recovery(q, pl, sh, zf, Psi, r, rt, s.Z);
      if (cfg.save_memory) emit_mln_truncate(q, sh, rt, r, zf, s.rts, s.rs, s.Zsk[k]);
      opnd = &s.Z;
    }
    Blocks<double> LV = plan_apply<double>(q, pl, sh, op, *opnd, false);
    plan_mln_sketch(q, pl, sh, LV, Psi, r, rt, s.Wsk, s.Mcols + size_t(k) * rt);
    plan_mln_recovery(q, pl, sh, s.Wsk, Psi, r, rt, vn);
    Blocks<double> wb;
    wb.add(vn, nullptr, 1.0);
    plan_exact_norm2(q, pl, sh, wb, s.s2 + 2 * k);
    const int j0 = std::max(0, k - kt + 1);
    std::vector<TT<double>> win(s.V.begin() + j0, s.V.begin() + k + 1);
    double* hk = s.h + size_t(k) * kt;
    plan_inner<double>(q, pl, sh, win, wb, hk, 1.0);
    {
      std::vector<MlnSk> xs;
      std::vector<const double*> cs;
      std::vector<double> ss;
      for (int j = j0; j <= k; ++j) {
        xs.push_back(s.full(j));
        cs.push_back(hk + (j - j0));
        ss.push_back(-1.0);
      }
      emit_mln_lincomb(q, pl, sh, rt, r, s.Wsk, xs, cs, ss, true, nullptr);
    }
    plan_mln_recovery(q, pl, sh, s.Wsk, Psi, r, rt, vn);
    plan_exact_norm2(q, pl, sh, wb, s.s2 + 2 * k + 1);
    {
      double* s2k = s.s2 + 2 * k;
      double* om = s.omega + k;
      const double* resk = s.res + k;
      const int* rk = vn.rank;
      double* vc = vn.core;
      LsState lsv = s.ls;
      const double* ctol = &s.conv_tol;
      const double bdt = cfg.bd_tol;
      IterStatus* sd = s.st_dev;
      int* fl = s.flags;
      const bool tik = cfg.tikhonov;
      q.steps.push_back([=](hipStream_t st) {
        ls_add_column(lsv, rt, mx, k, *ctol, bdt, st);
        // regularised y_k and residual (Sec. 4.3)
        if (tik) ls_tikhonov(lsv, rt, mx, k, *ctol, -1.0, st);
        iter_status(s2k, fl, resk, rk, d, bdt, om, sd, st);
        scale_copy<double>(vc, vc, cl, 1.0, nullptr, om, st);
      });
    }
    store(q, k + 1);
    s.iter.push_back(std::move(q));
    ar.rewind(mk);
  }

  // ---- final: X = recover(sum_i y_i sketch(V_i)), true residual ||b - L(X)||^2
  {
    std::vector<MlnSk> xs;
    std::vector<const double*> cs;
    std::vector<double> ss;
    for (int i = 0; i < mx; ++i) {
      xs.push_back(flex ? s.Zsk[i] : cfg.save_memory ? s.Strunc[i] : s.Sfull[i]);
      cs.push_back(s.y + i);
      ss.push_back(1.0);
    }
    const int rr = cfg.save_memory ? s.rs : r, rrt = cfg.save_memory ? s.rts : rt;
    emit_mln_lincomb(s.fin, pl, sh, rrt, rr, s.Fsk, xs, cs, ss, false, &s.nb_final);
    plan_mln_recovery(s.fin, pl, sh, s.Fsk, Psi, rr, rrt, s.X);
    Blocks<double> lx = plan_apply<double>(s.fin, pl, sh, op, s.X, false);
    Blocks<double> rb;
    rb.add(b, nullptr, 1.0);
    for (int j = 0; j < lx.size(); ++j) rb.add(lx.core[j], lx.U[j], lx.rank[j], nullptr, -lx.cscale[j]);
    plan_exact_norm2(s.fin, pl, sh, rb, s.rnorm2);
  }
  // the tables are read by the steps of every scope: place them past all scratch
  ar.seal();
  s.blob.dev = ar.alloc<unsigned char>(std::max<size_t>(s.blob.host.size(), 16));
  if (!ar.measuring())
    TK_HIP(hipMemcpyAsync(s.blob.dev, s.blob.host.data(), s.blob.host.size(), hipMemcpyHostToDevice, st));
  return sp;
}

void mln_solver_run(MlnSolver& s, TT<double>& x_out, MlnInfo& info, hipStream_t st) {
  const auto t0 = std::chrono::steady_clock::now();
  info = MlnInfo{};
  const int d = s.sh.d;
  s.conv_tol = s.cfg.eta * s.cfg.tol;
  s.setup.run(st);
  int status = kNotConverged, kend = s.maxiter;
  for (int k = 0; k < s.maxiter; ++k) {
    s.iter[k].run(st);
    TK_HIP(hipMemcpyAsync(s.st_host, s.st_dev, sizeof(IterStatus), hipMemcpyDeviceToHost, st));
    TK_HIP(hipStreamSynchronize(st));
    const IterStatus v = *s.st_host;
    info.hist.push_back(v.res);
    for (int j = 0; j < d; ++j) info.ranks.push_back(v.rank[j]);
    if (!std::isfinite(v.res) || !std::isfinite(v.omega))
      throw Error{kErrNonFinite, "non-finite sketched residual or basis norm"};
    if (v.breakdown_ls || v.breakdown_w) {
      status = kBreakdown;
      kend = k + 1;
      break;
    }
    if (v.converged) {
      status = kOk;
      kend = k + 1;
      break;
    }
  }
  s.nb_final = kend;
  s.fin.run(st);
  TK_HIP(hipMemcpyAsync(s.host2, s.rnorm2, sizeof(double), hipMemcpyDeviceToHost, st));
  TK_HIP(hipMemcpyAsync(s.host2 + 1, s.bnorm2, sizeof(double), hipMemcpyDeviceToHost, st));
  if (s.cfg.tikhonov) TK_HIP(hipMemcpyAsync(s.lam_host, s.lam, sizeof(double) * kend, hipMemcpyDeviceToHost, st));
  TK_HIP(hipStreamSynchronize(st));
  if (s.cfg.tikhonov) info.lambda.assign(s.lam_host, s.lam_host + kend);
  const double rn = std::sqrt(std::max(s.host2[0], 0.0)), bn = std::sqrt(std::max(s.host2[1], 0.0));
  info.status = status;
  info.iters = kend;
  info.true_relres = bn > 0 ? rn / bn : 0.0;
  x_out = s.X;
  info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace tk
