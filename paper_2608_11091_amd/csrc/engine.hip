// Plans of the Tucker sGMRES hot path: RoundSum (Sec. 3.1), operator apply
// (Eq. (2)), Khatri-Rao sketch (Alg. 2), inner products and the exact norm
// of a block sum.  See engine.hpp for the planning model.
#include "engine.hpp"

#include <algorithm>
#include <cmath>
#include <map>

namespace tk {

namespace {

// ---------------------------------------------------------------- helpers
// Where a product's split-K partials were left for its consumer to sum
// (part = nullptr: the product ran whole and wrote C).  Group g's partials
// start at part + g * splits * stride.
template <typename T>
struct SplitOut {
  const T* part = nullptr;
  int splits = 1;
  size_t stride = 0;  // M * N, one partial
};

template <typename T>
struct GemmDesc {
  bool ta = false, tb = false;
  int M = 0, N = 0, K = 0, lda = 0, ldb = 0, ldc = 0;
  double beta = 0.0;
  std::vector<GemmTerm<T>> terms;
  std::vector<GemmGroup<T>> groups;
  // runtime limits (optional): number of active blocks -> groups / terms
  const int* nb = nullptr;
  std::function<int(int)> ngroups_of;  // active groups as a function of *nb
  bool terms_are_blocks = false;       // clamp each group's terms to *nb
  bool factor_product = false;         // a product with a Tucker factor (BF16 in the BF16-factor form)
  // optional: the only consumer of C sums the split-K partials itself, which
  // saves the reduction launch (C is then not written); needs beta = 0,
  // ldc = M and a fixed group count
  SplitOut<T>* split_out = nullptr;

  void group(T* C, const std::vector<GemmTerm<T>>& ts) {
    GemmGroup<T> g;
    g.C = C;
    g.t0 = int(terms.size());
    for (auto& t : ts) terms.push_back(t);
    g.t1 = int(terms.size());
    groups.push_back(g);
  }
  void group1(T* C, const T* A, const T* B, const double* c1 = nullptr, const double* c2 = nullptr,
              const double* c3 = nullptr, double scale = 1.0) {
    group(C, {GemmTerm<T>{A, B, c1, c2, c3, scale}});
  }
};

template <typename T>
GemmTerm<T> term(const T* A, const T* B, const double* c1 = nullptr, const double* c2 = nullptr,
                 const double* c3 = nullptr, double scale = 1.0) {
  return GemmTerm<T>{A, B, c1, c2, c3, scale};
}

template <typename T>
void emit_gemm(Seq& q, Planner& pl, GemmDesc<T>&& g) {
  if (g.groups.empty()) return;
  const int ng = int(g.groups.size());
  int maxt = 1;
  for (auto& gr : g.groups) maxt = std::max(maxt, gr.t1 - gr.t0);
  const long tiles = long(ceil_div(g.M, 64)) * ceil_div(g.N, 64) * ng;
  const long slabs = long(maxt) * ceil_div(g.K, 16);  // in units of 16 of K
  // Split-K for the path's small, long-K products: about 64 of K (two of the
  // kernel's 32-deep slabs) per workgroup (measured on the path's shapes: a
  // 48 x 53 x 512 product took 44.9 / 16.4 / 12.1 / 11.5 us at 1 / 4 / 8 / 16
  // splits, kernel and reduction); products that already fill the chip or
  // have little K run whole.
  int splits = 1;
  if (tiles < 256 && slabs >= 16) {
    splits = int(std::min<long>(slabs / 4, std::max<long>(1, 512 / tiles)));
    splits = std::max(1, std::min(splits, 32));
  }
  T* partial = splits > 1 ? pl.ar.alloc<T>(size_t(ng) * splits * g.M * g.N) : nullptr;
  const size_t toff = pl.blob.add(g.terms), goff = pl.blob.add(g.groups);
  Blob* bl = &pl.blob;
  GemmLaunch<T> L;
  L.ta = g.ta;
  L.tb = g.tb;
  L.M = g.M;
  L.N = g.N;
  L.K = g.K;
  L.lda = g.lda;
  L.ldb = g.ldb;
  L.ldc = g.ldc;
  L.beta = g.beta;
  L.splits = splits;
  L.partial = partial;
  L.bf16 = std::is_same<T, float>::value && pl.bf16_factors && g.factor_product;
  L.ngroups = ng;
  if (g.split_out) {
    TK_CHECK(g.beta == 0.0 && g.ldc == g.M && g.nb == nullptr, kErrUnsupported,
             "internal: deferred split-K reduction needs beta = 0, ldc = M and fixed groups");
    *g.split_out = SplitOut<T>{};
    if (splits > 1) {
      L.defer_reduce = true;
      *g.split_out = SplitOut<T>{partial, splits, size_t(g.M) * g.N};
    }
  }
  const int* nb = g.nb;
  auto ngf = g.ngroups_of;
  const bool tb = g.terms_are_blocks;
  std::vector<int> nterm;
  for (auto& gr : g.groups) nterm.push_back(gr.t1 - gr.t0);
  const double mnk2 = 2.0 * g.M * g.N * g.K;
  q.steps.push_back([=](hipStream_t st) {
    GemmLaunch<T> l = L;
    l.terms = bl->at<GemmTerm<T>>(toff);
    l.groups = bl->at<GemmGroup<T>>(goff);
    if (nb) {
      if (ngf) l.ngroups = std::min(ng, ngf(*nb));
      if (tb) l.max_terms = *nb;
    }
    if (timer_on(kKcGemm)) {
      double f = 0.0;
      for (int i = 0; i < l.ngroups; ++i) f += mnk2 * std::min(nterm[i], l.max_terms);
      l.flops = f;
    }
    gemm_run(l, st);
  });
}

template <typename X>
size_t blob_ptrs(Blob& b, const std::vector<X>& v) {
  return b.add(v);
}

// Y_b = X_b x_k W_b (mode-k TTM) for a batch.  X dims `dims` (row-major);
// W_b is (newdim x dims[k]) col-major with leading dimension ldw, or, when
// w_transposed, W_b^T is given as (dims[k] x newdim) with leading dim ldw.
// When `sum_into` is set (k == 0 or k == d-1 only) every batch entry is
// accumulated into sum_into with coefficient c1[b] (scaled by cscale).
template <typename T>
void emit_ttm(Seq& q, Planner& pl, int d, const int* dims, int k, int newdim, const std::vector<const T*>& X,
              const std::vector<const T*>& W, int ldw, bool w_transposed, const std::vector<T*>& Y,
              T* sum_into = nullptr, const std::vector<const double*>* c1 = nullptr, double cscale = 1.0,
              const int* nb = nullptr) {
  long pre = 1, post = 1;
  for (int j = 0; j < k; ++j) pre *= dims[j];
  for (int j = k + 1; j < d; ++j) post *= dims[j];
  const int mid = dims[k];
  const int nbat = int(X.size());
  GemmDesc<T> g;
  g.nb = nb;
  if (post == 1) {
    // X is (mid x pre) col-major; Y = W X  (newdim x pre)
    g.ta = w_transposed;
    g.tb = false;
    g.M = newdim;
    g.N = int(pre);
    g.K = mid;
    g.lda = ldw;
    g.ldb = mid;
    g.ldc = newdim;
    if (sum_into) {
      std::vector<GemmTerm<T>> ts;
      for (int b = 0; b < nbat; ++b) ts.push_back(term<T>(W[b], X[b], c1 ? (*c1)[b] : nullptr, nullptr, nullptr, cscale));
      g.group(sum_into, ts);
      g.terms_are_blocks = nb != nullptr;
    } else {
      for (int b = 0; b < nbat; ++b) g.group1(Y[b], W[b], X[b]);
      if (nb) g.ngroups_of = [](int n) { return n; };
    }
  } else {
    // per pre-slice: X_p is (post x mid) col-major; Y_p = X_p W^T  (post x newdim)
    g.ta = false;
    g.tb = !w_transposed;
    g.M = int(post);
    g.N = newdim;
    g.K = mid;
    g.lda = int(post);
    g.ldb = ldw;
    g.ldc = int(post);
    if (sum_into) {
      TK_CHECK(pre == 1, kErrInvalidArg, "internal: summed TTM needs a leading mode");
      std::vector<GemmTerm<T>> ts;
      for (int b = 0; b < nbat; ++b) ts.push_back(term<T>(X[b], W[b], c1 ? (*c1)[b] : nullptr, nullptr, nullptr, cscale));
      g.group(sum_into, ts);
      g.terms_are_blocks = nb != nullptr;
    } else {
      for (int b = 0; b < nbat; ++b)
        for (long p = 0; p < pre; ++p)
          g.group1(Y[b] + size_t(p) * post * newdim, X[b] + size_t(p) * post * mid, W[b]);
      if (nb) {
        const long pr = pre;
        g.ngroups_of = [pr](int n) { return int(n * pr); };
      }
    }
  }
  emit_gemm(q, pl, std::move(g));
}

// G = X_(k) Y_(k)^T (mid x mid, ld ldg) for two tensors of dims `dims`.
template <typename T>
void emit_unfold_gram(Seq& q, Planner& pl, int d, const int* dims, int k, const T* X, const T* Y, T* G, int ldg,
                      double scale = 1.0, SplitOut<T>* split_out = nullptr) {
  long pre = 1, post = 1;
  for (int j = 0; j < k; ++j) pre *= dims[j];
  for (int j = k + 1; j < d; ++j) post *= dims[j];
  const int mid = dims[k];
  GemmDesc<T> g;
  g.M = mid;
  g.N = mid;
  g.ldc = ldg;
  if (post == 1) {
    g.ta = false;
    g.tb = true;
    g.K = int(pre);
    g.lda = mid;
    g.ldb = mid;
    g.group1(G, X, Y, nullptr, nullptr, nullptr, scale);
  } else {
    g.ta = true;
    g.tb = false;
    g.K = int(post);
    g.lda = int(post);
    g.ldb = int(post);
    std::vector<GemmTerm<T>> ts;
    for (long p = 0; p < pre; ++p)
      ts.push_back(term<T>(X + size_t(p) * post * mid, Y + size_t(p) * post * mid, nullptr, nullptr, nullptr, scale));
    g.group(G, ts);
  }
  g.split_out = split_out;
  emit_gemm(q, pl, std::move(g));
}

template <typename T>
std::vector<std::vector<int>> modes_by_n(const Shape& sh) {
  std::map<int, std::vector<int>> m;
  for (int k = 0; k < sh.d; ++k) m[sh.n[k]].push_back(k);
  std::vector<std::vector<int>> out;
  for (auto& kv : m) out.push_back(kv.second);
  return out;
}

template <typename T>
void emit_cast(Seq& q, const T* src, double* dst, size_t len);
template <>
void emit_cast<double>(Seq& q, const double* src, double* dst, size_t len) {
  (void)q; (void)src; (void)dst; (void)len;
}
template <>
void emit_cast<float>(Seq& q, const float* src, double* dst, size_t len) {
  q.steps.push_back([=](hipStream_t st) { cast_copy<float, double>(src, dst, len, st); });
}

// Fork/join of a plan section onto the side stream: the section starts after
// everything issued before it on the caller's stream, and the caller's stream
// waits for the section at the join.  The events live as long as the plan.
struct ForkJoin {
  hipEvent_t fork = nullptr, join = nullptr;
  ForkJoin() {
    TK_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    TK_HIP(hipEventCreateWithFlags(&join, hipEventDisableTiming));
  }
  ~ForkJoin() {
    (void)hipEventSynchronize(join);  // a plan may be dropped right after it was issued
    (void)hipEventDestroy(fork);
    (void)hipEventDestroy(join);
  }
  ForkJoin(const ForkJoin&) = delete;
  ForkJoin& operator=(const ForkJoin&) = delete;
};

}  // namespace

// Moves steps [from, end) of q onto side stream `which` between a fork and the
// join record; the returned step makes the caller's stream wait for them.
std::function<void(hipStream_t)> fork_steps(Seq& q, size_t from, int which) {
  auto fj = std::make_shared<ForkJoin>();
  std::vector<std::function<void(hipStream_t)>> sec(q.steps.begin() + from, q.steps.end());
  q.steps.resize(from);
  q.steps.push_back([fj, sec, which](hipStream_t st) {
    hipStream_t side = side_stream(which);
    TK_HIP(hipEventRecord(fj->fork, st));
    TK_HIP(hipStreamWaitEvent(side, fj->fork, 0));
    for (auto& f : sec) f(side);
    TK_HIP(hipEventRecord(fj->join, side));
  });
  return [fj](hipStream_t st) { TK_HIP(hipStreamWaitEvent(st, fj->join, 0)); };
}

// Khatri-Rao range sketch of a block sum (Sec. 3.1; also the factor sketches
// of the multilinear Nystrom method): for every mode k,
//   Y_k = sum_b coef_b U_bk MTTKRP(G_b; {U_bj^T L_j[:, :w]}_{j != k}, k)   (n_k x w),
// i.e. the mode-k unfolding of the sum times the Khatri-Rao product of the
// other modes' L_j[:, :w] (L_j column-major n_j x >= w).
template <typename T>
void plan_krp_range(Seq& q, Planner& pl, const Shape& sh, const Blocks<T>& in, const double* coef,
                    const std::array<const T*, kMaxD>& L, int w, const std::array<T*, kMaxD>& Y,
                    const int* nb_active) {
  const int d = sh.d, rc = sh.rc, nb = in.size();
  Arena& ar = pl.ar;
  Blob* bl = &pl.blob;
  const size_t P = size_t(ipow(rc, d - 1));
  auto nbA = [nb, nb_active]() { return nb_active ? std::min(nb, *nb_active) : nb; };
  T* Mb = ar.alloc<T>(size_t(nb) * d * rc * w);
  auto Mp = [&](int b, int j) { return Mb + (size_t(b) * d + j) * rc * w; };
  for (auto& modes : modes_by_n<T>(sh)) {  // M_bj = U_bj^T L_j (rc x w)
    const int n = sh.n[modes[0]];
    GemmDesc<T> g;
    g.ta = true;
    g.tb = false;
    g.M = rc;
    g.N = w;
    g.K = n;
    g.lda = n;
    g.ldb = n;
    g.ldc = rc;
    g.nb = nb_active;
    const int nm = int(modes.size());
    g.ngroups_of = [nm](int a) { return a * nm; };
    for (int b = 0; b < nb; ++b)
      for (int j : modes) g.group1(Mp(b, j), in.U[b][j], L[j]);
    g.factor_product = true;
    emit_gemm(q, pl, std::move(g));
  }
  T* Zl = ar.alloc<T>(size_t(nb) * P * w);
  T* Zf = ar.alloc<T>(size_t(nb) * P * w);
  {
    GemmDesc<T> g;  // Zlast_b = G_b x_d M_bd^T : (P x w)
    g.ta = true;
    g.tb = false;
    g.M = int(P);
    g.N = w;
    g.K = rc;
    g.lda = rc;
    g.ldb = rc;
    g.ldc = int(P);
    g.nb = nb_active;
    g.ngroups_of = [](int a) { return a; };
    for (int b = 0; b < nb; ++b) g.group1(Zl + size_t(b) * P * w, in.core[b], Mp(b, d - 1));
    emit_gemm(q, pl, std::move(g));
    GemmDesc<T> h;  // Zfirst_b = G_b x_1 M_b1^T : (P x w)
    h.ta = false;
    h.tb = false;
    h.M = int(P);
    h.N = w;
    h.K = rc;
    h.lda = int(P);
    h.ldb = rc;
    h.ldc = int(P);
    h.nb = nb_active;
    h.ngroups_of = [](int a) { return a; };
    for (int b = 0; b < nb; ++b) h.group1(Zf + size_t(b) * P * w, in.core[b], Mp(b, 0));
    emit_gemm(q, pl, std::move(h));
  }
  T* Tb = ar.alloc<T>(size_t(nb) * d * rc * w);
  auto Tp = [&](int b, int k) { return Tb + (size_t(b) * d + k) * rc * w; };
  {
    std::vector<KrpTask<T>> tasks;
    for (int b = 0; b < nb; ++b)
      for (int k = 0; k < d; ++k) {
        KrpTask<T> t{};
        t.out = Tp(b, k);
        t.scale = 1.0;
        t.ldo = rc;
        if (k < d - 1) {
          t.Z = Zl + size_t(b) * P * w;
          t.f = k;
          for (int j = 0; j < d - 1; ++j) {
            t.Mj[j] = Mp(b, j);
            t.ldm[j] = rc;
          }
        } else {
          t.Z = Zf + size_t(b) * P * w;
          t.f = d - 2;
          for (int j = 0; j < d - 1; ++j) {
            t.Mj[j] = Mp(b, j + 1);
            t.ldm[j] = rc;
          }
        }
        tasks.push_back(t);
      }
    const size_t off = pl.blob.add(tasks);
    std::vector<int> z(d - 1, rc);
    q.steps.push_back([=](hipStream_t st) {
      krp_reduce<T>(bl->at<KrpTask<T>>(off), nbA() * d, d - 1, z.data(), int(P), w, st);
    });
  }
  for (auto& modes : modes_by_n<T>(sh)) {
    const int n = sh.n[modes[0]];
    GemmDesc<T> g;
    g.ta = false;
    g.tb = false;
    g.M = n;
    g.N = w;
    g.K = rc;
    g.lda = n;
    g.ldb = rc;
    g.ldc = n;
    g.nb = nb_active;
    g.terms_are_blocks = nb_active != nullptr;
    for (int k : modes) {
      std::vector<GemmTerm<T>> ts;
      for (int b = 0; b < nb; ++b) ts.push_back(term<T>(in.U[b][k], Tp(b, k), coef + b));
      g.group(Y[k], ts);
    }
    g.factor_product = true;
    emit_gemm(q, pl, std::move(g));
  }
}

// Core projection of a block sum onto per-mode matrices P_k (n_k x >= w,
// column-major): C = sum_b coef_b G_b x_1 (P_1^T U_b1) ... x_d (P_d^T U_bd),
// a w^d row-major core (the RoundSum core of Sec. 3.1 with P_k = the range
// basis; the sketched core of the multilinear Nystrom method with P_k = Psi_k).
template <typename T>
void plan_core_projection(Seq& q, Planner& pl, const Shape& sh, const Blocks<T>& in, const double* coef,
                          const std::array<const T*, kMaxD>& Pm, int w, T* C, const int* nb_active) {
  const int d = sh.d, rc = sh.rc, nb = in.size();
  TK_CHECK(d >= 2, kErrUnsupported, "d = 1");
  Arena& ar = pl.ar;
  T* Wb = ar.alloc<T>(size_t(nb) * d * w * rc);
  auto Wp = [&](int b, int k) { return Wb + (size_t(b) * d + k) * w * rc; };
  for (auto& modes : modes_by_n<T>(sh)) {
    const int n = sh.n[modes[0]];
    GemmDesc<T> g;
    g.ta = true;
    g.tb = false;
    g.M = w;
    g.N = rc;
    g.K = n;
    g.lda = n;
    g.ldb = n;
    g.ldc = w;
    g.nb = nb_active;
    const int nm = int(modes.size());
    g.ngroups_of = [nm](int a) { return a * nm; };
    for (int b = 0; b < nb; ++b)
      for (int k : modes) g.group1(Wp(b, k), Pm[k], in.U[b][k]);
    g.factor_product = true;
    emit_gemm(q, pl, std::move(g));
  }
  // after the TTM of mode k (k = d-1 .. 1) the block tensor has dims
  // (rc^k, w^(d-k)); size the two ping-pong buffers for the largest
  size_t tmplen = 0;
  for (int k = 1; k < d; ++k) tmplen = std::max(tmplen, size_t(ipow(rc, k)) * size_t(ipow(w, d - k)));
  T* X0 = ar.alloc<T>(size_t(nb) * tmplen);
  T* X1 = ar.alloc<T>(size_t(nb) * tmplen);
  int dims[kMaxD];
  for (int j = 0; j < d; ++j) dims[j] = rc;
  std::vector<const T*> Xs, Ws;
  std::vector<T*> Ys;
  std::vector<const double*> cs;
  // mode d-1 from the block cores
  for (int b = 0; b < nb; ++b) {
    Xs.push_back(in.core[b]);
    Ws.push_back(Wp(b, d - 1));
    Ys.push_back(X0 + size_t(b) * tmplen);
    cs.push_back(coef + b);
  }
  emit_ttm<T>(q, pl, d, dims, d - 1, w, Xs, Ws, w, false, Ys, nullptr, nullptr, 1.0, nb_active);
  dims[d - 1] = w;
  T* cur = X0;
  T* nxt = X1;
  for (int k = d - 2; k >= 1; --k) {
    Xs.clear();
    Ws.clear();
    Ys.clear();
    for (int b = 0; b < nb; ++b) {
      Xs.push_back(cur + size_t(b) * tmplen);
      Ws.push_back(Wp(b, k));
      Ys.push_back(nxt + size_t(b) * tmplen);
    }
    emit_ttm<T>(q, pl, d, dims, k, w, Xs, Ws, w, false, Ys, nullptr, nullptr, 1.0, nb_active);
    dims[k] = w;
    std::swap(cur, nxt);
  }
  Xs.clear();
  Ws.clear();
  for (int b = 0; b < nb; ++b) {
    Xs.push_back(cur + size_t(b) * tmplen);
    Ws.push_back(Wp(b, 0));
  }
  emit_ttm<T>(q, pl, d, dims, 0, w, Xs, Ws, w, false, {}, C, &cs, 1.0, nb_active);
}

// ====================================================================== RoundSum
template <typename T>
RoundSumOut<T> plan_roundsum(Seq& q, Planner& pl, const Shape& sh, const Blocks<T>& in, const RoundCfg& cfg,
                             const std::array<const T*, kMaxD>& omega, const TT<T>& out, const int* nb_active) {
  const int d = sh.d, rc = sh.rc, sc = sh.sc(), nb = in.size();
  TK_CHECK(nb >= 1, kErrInvalidArg, "RoundSum of an empty sum");
  TK_CHECK(sc <= 64, kErrUnsupported, "RoundSum: rank cap + oversampling above 64");
  Arena& ar = pl.ar;
  Blob& blob = pl.blob;
  Blob* bl = &blob;
  const size_t P = size_t(ipow(rc, d - 1));       // rc^(d-1)
  const size_t corelen = size_t(ipow(rc, d));
  const size_t sclen = size_t(ipow(sc, d));

  // --- device scalars and tables
  double* coef = ar.alloc<double>(nb);
  double* sumsq = ar.alloc<double>(nb);
  double* w = ar.alloc<double>(nb);
  int* rt = ar.alloc<int>(kMaxD);
  int* s_dev = ar.alloc<int>(1);
  double* total = ar.alloc<double>(1);
  double* zthr = ar.alloc<double>(1);
  const double zero_tol = 16.0 * (std::is_same<T, double>::value ? 1.1102230246251565e-16 : 5.9604644775390625e-08);
  const bool own_eps = cfg.eps_dev == nullptr;
  const double* epsd = own_eps ? ar.alloc<double>(2) : cfg.eps_dev;  // [0] eps, [1] tau
  int* force_dev = ar.alloc<int>(kMaxD);
  const size_t off_cptr = blob.add(in.cptr);
  const size_t off_cscale = blob.add(in.cscale);
  const size_t off_cores = blob.add(in.core);
  const size_t off_ranks = blob.add(in.rank);
  const double eps_v = cfg.eps, tau_v = cfg.tau > 0 ? cfg.tau : cfg.eps;
  auto nbA = [nb, nb_active]() { return nb_active ? std::min(nb, *nb_active) : nb; };
  // Host values copied to device scalars by the first step (pageable source:
  // the copy completes before the call returns).
  struct Params {
    double ev[2];
    int force[kMaxD];
  };
  auto hp = std::make_shared<Params>();
  hp->ev[0] = eps_v;
  hp->ev[1] = tau_v;
  for (int k = 0; k < kMaxD; ++k) hp->force[k] = cfg.force_r[k];
  bool any_force = false;
  for (int k = 0; k < d; ++k) any_force |= cfg.force_r[k] >= 0;

  q.steps.push_back([=](hipStream_t st) {
    if (own_eps) TK_HIP(hipMemcpyAsync(const_cast<double*>(epsd), hp->ev, sizeof(hp->ev), hipMemcpyHostToDevice, st));
    if (any_force) TK_HIP(hipMemcpyAsync(force_dev, hp->force, sizeof(hp->force), hipMemcpyHostToDevice, st));
    dot_batched<T>(bl->at<const T*>(off_cores), bl->at<const T*>(off_cores), corelen, nbA(), 1.0, sumsq, st);
    coef_weights_threshold(bl->at<const double*>(off_cptr), bl->at<double>(off_cscale), sumsq, nbA(), zero_tol, coef,
                           w, zthr, st);
  });

  // --- 1. effective-rank heuristic (Gram eigenvalues) -> sketch width.  With
  //        Cholesky-QR the rule runs on the side stream beside steps 2-3: the
  //        range sketch is formed at the full capacity width sc, and the QR runs
  //        over all sc columns (Cholesky-QR is nested: the leading s columns
  //        of Q only depend on the leading s columns of Y), so only the
  //        zeroing of the columns beyond s waits for the rule.
  const bool rule = cfg.force_s < 0;
  const bool overlap = rule && !cfg.householder;
  const size_t rule_from = q.steps.size();
  // Where the spectrum is expensive (every FP64 Gram; in FP32 the Grams that
  // can exceed the register eigensolver's order) the overlap becomes: Grams
  // on the side stream, and the eigensolves wait on the main stream for the
  // rank certificate after step 3; when it shows r~_k >= cap for some mode
  // the width is cap + p and every eigensolve returns at once.  Elsewhere the
  // eigensolves run on the side stream beside steps 2-3.
  bool big_gram = false;
  for (auto& modes : modes_by_n<T>(sh)) {
    const int n = sh.n[modes[0]];
    big_gram |= n > kEigRegMax && nb * rc > kEigRegMax;
  }
  const bool use_cert = overlap && (std::is_same<T, double>::value || big_gram);
  int* cert_dev = use_cert ? ar.alloc<int>(kMaxD) : nullptr;
  double* fro = use_cert ? ar.alloc<double>(size_t(nb) * d) : nullptr;
  std::vector<std::function<void(hipStream_t)>> eig_steps;
  if (rule) {
    for (auto& modes : modes_by_n<T>(sh)) {
      const int n = sh.n[modes[0]];
      // The Gram goes on the smaller side (n x n, or R x R for the active
      // concatenation; both have the same nonzero spectrum).  Which side is
      // smaller and which eigensolver fits depend on the active ranks, a
      // device value, so wide cases plan both tasks of a pair and the one
      // that does not apply skips itself: the register eigensolver (order
      // <= 160) on the compacted R-side Gram while R <= 160, and the
      // global-memory one (order <= 512) above that, on the R-side Gram while
      // R <= n (capacity permitting) or else on the n-side Gram.
      const int Rp = nb * rc;
      if (use_cert) {
        // squared Frobenius norms of the factors: tr(G_k) for the certificate
        for (int k : modes) {
          std::vector<const T*> xs;
          for (int b = 0; b < nb; ++b) xs.push_back(in.U[b][k]);
          const size_t off = blob.add(xs);
          const size_t len = size_t(n) * rc;
          double* out = fro + size_t(k) * nb;
          q.steps.push_back([=](hipStream_t st) {
            dot_batched<T>(bl->at<const T*>(off), bl->at<const T*>(off), len, nbA(), 1.0, out, st);
          });
        }
      }
      auto nside_gram = [&](int ldg) {
        T* Gn = ar.alloc<T>(size_t(ldg) * n * modes.size());
        GemmDesc<T> g;
        g.ta = false;
        g.tb = true;
        g.M = n;
        g.N = n;
        g.K = rc;
        g.lda = n;
        g.ldb = n;
        g.ldc = ldg;
        g.nb = nb_active;
        g.terms_are_blocks = nb_active != nullptr;
        for (size_t i = 0; i < modes.size(); ++i) {
          const int k = modes[i];
          std::vector<GemmTerm<T>> ts;
          for (int b = 0; b < nb; ++b) ts.push_back(term<T>(in.U[b][k], in.U[b][k], w + b, w + b));
          g.group(Gn + i * size_t(ldg) * n, ts);
        }
        emit_gemm(q, pl, std::move(g));
        return Gn;
      };
      auto eig_launch = [&](std::vector<EigTask<T>> et, int NL) {
        const size_t off_et = blob.add(et);
        const int ne = int(et.size());
        (use_cert ? eig_steps : q.steps).push_back([=](hipStream_t st) {
          jacobi_eig<T>(bl->at<EigTask<T>>(off_et), ne, NL, false, st);
        });
      };
      auto rule_task = [&](T* A, int lda, T* lam, int k) {
        EigTask<T> e{};
        e.A = A;
        e.lda = lda;
        e.lam = lam;
        e.cert = cert_dev;
        e.ncert = use_cert ? d : 0;
        e.rule.kind = 1;
        e.rule.tau = epsd + 1;
        e.rule.delta = cfg.delta;
        e.rule.rank_out = rt + k;
        e.rule.cap1 = sh.cap;  // the width only takes min(r~ + p, cap + p); lam is scratch
        return e;
      };
      if (n <= kEigRegMax) {
        // n-side Gram: sum_b w_b^2 U_b U_b^T, register eigensolver
        T* Gn = nside_gram(n);
        T* lam = ar.alloc<T>(size_t(n) * modes.size());
        std::vector<EigTask<T>> et;
        for (size_t i = 0; i < modes.size(); ++i)
          et.push_back(rule_task(Gn + i * size_t(n) * n, n, lam + i * n, modes[i]));
        eig_launch(et, n);
        continue;
      }
      // R-side Gram of the padded concatenation, compacted to the active ranks
      // (only while they fit the compacted capacity NM; blocks of a disabled
      // mode cost nothing in the GEMM)
      const int NM = std::min(Rp, Rp > n ? kEigRegMax : n);
      const int ldc = NM > kEigRegMax ? (NM + 3) / 4 * 4 : NM;
      double* enable = ar.alloc<double>(kMaxD);
      int* nact = ar.alloc<int>(kMaxD);
      int* skip_reg = ar.alloc<int>(kMaxD);   // R above the register eigensolver's order
      int* skip_gm = ar.alloc<int>(kMaxD);    // R within it
      T* Gp = ar.alloc<T>(size_t(Rp) * Rp * d);
      T* Gc = ar.alloc<T>(size_t(ldc) * NM * d);
      T* lam = ar.alloc<T>(size_t(std::max(NM, n)) * d);
      q.steps.push_back([=](hipStream_t st) {
        // the flags against the register order first, then enable / nact
        // against the compacted capacity (the second call overwrites them)
        gram_prep(bl->at<const int*>(off_ranks), nbA(), d, kEigRegMax, enable, nact, st, skip_reg, skip_gm);
        gram_prep(bl->at<const int*>(off_ranks), nbA(), d, NM, enable, nact, st);
      });
      {
        GemmDesc<T> g;
        g.ta = true;
        g.tb = false;
        g.M = rc;
        g.N = rc;
        g.K = n;
        g.lda = n;
        g.ldb = n;
        g.ldc = Rp;
        g.nb = nb_active;
        const int nmod = int(modes.size());
        g.ngroups_of = [nmod](int a) { return a * (a + 1) / 2 * nmod; };
        for (int b = 0; b < nb; ++b)
          for (int b2 = 0; b2 <= b; ++b2)
            for (int k : modes)
              g.group1(Gp + size_t(k) * Rp * Rp + size_t(b) * rc + size_t(b2) * rc * Rp, in.U[b][k], in.U[b2][k],
                       w + b, w + b2, enable + k);
        emit_gemm(q, pl, std::move(g));
      }
      q.steps.push_back([=](hipStream_t st) {
        gram_compact<T>(Gp, Rp, bl->at<const int*>(off_ranks), nbA(), d, rc, nact, Gc, ldc, size_t(Rp) * Rp,
                        size_t(ldc) * NM, st);
      });
      {
        // register eigensolver on the compacted Gram while R <= 160
        std::vector<EigTask<T>> et;
        for (int k : modes) {
          EigTask<T> e = rule_task(Gc + size_t(k) * ldc * NM, ldc, lam + size_t(k) * std::max(NM, n), k);
          e.ndyn = nact + k;
          e.skip = skip_reg + k;
          et.push_back(e);
        }
        eig_launch(et, std::min(NM, kEigRegMax));
      }
      if (Rp > kEigRegMax) {
        std::vector<EigTask<T>> et;
        if (Rp <= n) {
          // global-memory eigensolver on the compacted Gram (R <= Rp <= n)
          for (int k : modes) {
            EigTask<T> e = rule_task(Gc + size_t(k) * ldc * NM, ldc, lam + size_t(k) * std::max(NM, n), k);
            e.ndyn = nact + k;
            e.skip = skip_gm + k;
            et.push_back(e);
          }
          eig_launch(et, NM);
        } else {
          // global-memory eigensolver on the n-side Gram while R > 160
          const int ldg = (n + 3) / 4 * 4;
          T* Gn = nside_gram(ldg);
          for (size_t i = 0; i < modes.size(); ++i) {
            const int k = modes[i];
            EigTask<T> e = rule_task(Gn + i * size_t(ldg) * n, ldg, lam + size_t(k) * std::max(NM, n), k);
            e.skip = skip_gm + k;
            et.push_back(e);
          }
          eig_launch(et, n);
        }
      }
    }
  }
  std::function<void(hipStream_t)> join;
  const int p_ = sh.p, cap_ = sh.cap, fs_ = cfg.force_s;
  auto emit_width = [&]() {
    q.steps.push_back([=](hipStream_t st) { sketch_width(rt, d, p_, cap_, fs_, s_dev, st); });
  };
  if (overlap)
    join = fork_steps(q, rule_from, 0);
  else
    emit_width();

  // --- 2. Khatri-Rao range sketch Y_k = sum_b c_b U_bk MTTKRP(G_b; U_bj^T Omega_j, k)
  std::array<T*, kMaxD> Y{}, Uh{};
  std::array<double*, kMaxD> Y64{}, Q64{};
  for (int k = 0; k < d; ++k) {
    Y[k] = ar.alloc<T>(size_t(sh.n[k]) * sc);
    Q64[k] = ar.alloc<double>(size_t(sh.n[k]) * sc);
    if (std::is_same<T, double>::value) {
      Y64[k] = reinterpret_cast<double*>(Y[k]);
      Uh[k] = reinterpret_cast<T*>(Q64[k]);
    } else {
      Y64[k] = ar.alloc<double>(size_t(sh.n[k]) * sc);
      Uh[k] = ar.alloc<T>(size_t(sh.n[k]) * sc);
    }
  }
  plan_krp_range<T>(q, pl, sh, in, coef, omega, sc, Y, nb_active);
  // --- 3. orthonormal basis of every range sketch Y_k (FP64): Householder QR
  // when the configuration asks for it, otherwise shifted Cholesky-QR in three
  // passes (Y -> Q -> Y -> Q ping-pong).  Pass 1 is
  // shifted by 11 (m s + s(s+1)) u tr(Y^T Y), so it never breaks down; pass 2
  // drops only columns at the underflow floor; pass 3 sees a nearly
  // orthonormal input, where a pivot below 1/4 can only come from a
  // rounding-noise column of a rank-deficient Y, and zeroes it.  Live columns
  // come out orthonormal to working accuracy and span range(Y) down to
  // rounding level.
  if (cfg.householder) {
    for (auto& modes : modes_by_n<T>(sh)) {
      const int n = sh.n[modes[0]];
      std::vector<QrTask> qt;
      for (int k : modes) {
        emit_cast<T>(q, Y[k], Y64[k], size_t(n) * sc);
        qt.push_back(QrTask{Y64[k], Q64[k], nullptr, nullptr});
      }
      const size_t off = blob.add(qt);
      const int nt = int(qt.size());
      q.steps.push_back([=](hipStream_t st) { qr_batched(bl->at<QrTask>(off), nt, n, sc, s_dev, st); });
      if (!std::is_same<T, double>::value)
        for (int k : modes) {
          double* src = Q64[k];
          T* dst = Uh[k];
          const size_t len = size_t(n) * sc;
          q.steps.push_back([=](hipStream_t st) { cast_copy<double, T>(src, dst, len, st); });
        }
    }
  } else {
    double* Gq = ar.alloc<double>(size_t(d) * sc * sc);
    double* Rq = ar.alloc<double>(size_t(d) * sc * sc);
    for (auto& modes : modes_by_n<T>(sh)) {
      const int n = sh.n[modes[0]];
      if constexpr (!std::is_same<T, double>::value) {
        // the FP32 range sketches of these modes to FP64, one launch
        CastSet<T, double> cs;
        for (int k : modes) {
          cs.x[cs.count] = Y[k];
          cs.y[cs.count] = Y64[k];
          cs.len[cs.count++] = size_t(n) * sc;
        }
        q.steps.push_back([=](hipStream_t st) { cast_multi<T, double>(cs, st); });
      }
      std::vector<CholTask> ct;
      for (int k : modes) ct.push_back(CholTask{Gq + size_t(k) * sc * sc, Rq + size_t(k) * sc * sc});
      const int nt = int(ct.size());
      const double shift1 = 11.0 * (double(n) * sc + double(sc) * (sc + 1)) * 0x1p-53;
      for (int pass = 0; pass < 3; ++pass) {
        std::vector<const double*> src;
        std::vector<double*> dst;
        for (int k : modes) {
          src.push_back(pass == 1 ? Q64[k] : Y64[k]);
          dst.push_back(pass == 1 ? Y64[k] : Q64[k]);
        }
        GemmDesc<double> g;
        g.ta = true;
        g.tb = false;
        g.M = sc;
        g.N = sc;
        g.K = n;
        g.lda = n;
        g.ldb = n;
        g.ldc = sc;
        for (size_t i = 0; i < modes.size(); ++i) g.group1(Gq + size_t(modes[i]) * sc * sc, src[i], src[i]);
        // the Cholesky kernel sums the Gram's split-K partials itself
        SplitOut<double> so;
        g.split_out = &so;
        emit_gemm(q, pl, std::move(g));
        std::vector<CholTask> ctp = ct;
        for (size_t i = 0; i < ctp.size(); ++i)
          if (so.part) {
            ctp[i].part = so.part + i * size_t(so.splits) * so.stride;
            ctp[i].splits = so.splits;
            ctp[i].pstride = so.stride;
          }
        const size_t cpo = blob.add(ctp);
        const double sh_p = pass == 0 ? shift1 : 0.0;
        const double drel = pass == 1 ? 1e-30 : 0.0, dabs = pass == 2 ? 0.25 : 0.0;
        const int* mq = overlap ? nullptr : s_dev;
        q.steps.push_back(
            [=](hipStream_t st) { chol_batched(bl->at<CholTask>(cpo), nt, sc, mq, sh_p, drel, dabs, st); });
        std::vector<TrsmTask> tt;
        for (size_t i = 0; i < modes.size(); ++i) {
          tt.push_back(TrsmTask{src[i], Rq + size_t(modes[i]) * sc * sc, dst[i]});
          // the last pass also writes the FP32 basis of the FP32 form
          if constexpr (!std::is_same<T, double>::value)
            if (pass == 2) tt.back().Qf = Uh[modes[i]];
        }
        const size_t toff = blob.add(tt);
        q.steps.push_back([=](hipStream_t st) { trsm_rows(bl->at<TrsmTask>(toff), nt, n, sc, mq, st); });
      }
    }
  }
  if (use_cert) {
    // Rank certificate (Courant-Fischer): for Q_k' = the first cap columns of
    // the orthonormal range basis, lambda_cap(G_k) >= lambda_min(Q_k'^T G_k Q_k')
    // for the rule's Gram G_k = sum_b w_b^2 U_bk U_bk^T, so a Cholesky
    // factorisation of Q_k'^T G_k Q_k' - theta I settles r~_k >= cap without the
    // spectrum (rank_certificate).  theta covers the rounding of
    // P_bk = w_b Q_k'^T U_bk (inner dimension n) and of sum_b P_bk P_bk^T
    // (inner dimension at most nb rc): 4 (n sqrt(cap) + nb rc) u tr(G_k).
    const int cp_ = sh.cap;
    T* Pm = ar.alloc<T>(size_t(nb) * d * cp_ * rc);
    T* Hc = ar.alloc<T>(size_t(d) * cp_ * cp_);
    for (auto& modes : modes_by_n<T>(sh)) {
      const int n = sh.n[modes[0]];
      {
        // P_bk (cap x rc); groups ordered by block, so the active ones are a prefix
        GemmDesc<T> g;
        g.ta = true;
        g.tb = false;
        g.M = cp_;
        g.N = rc;
        g.K = n;
        g.lda = n;
        g.ldb = n;
        g.ldc = cp_;
        g.nb = nb_active;
        const int nmod = int(modes.size());
        g.ngroups_of = [nmod](int a) { return a * nmod; };
        for (int b = 0; b < nb; ++b)
          for (int k : modes) g.group1(Pm + (size_t(k) * nb + b) * cp_ * rc, Uh[k], in.U[b][k], w + b);
        emit_gemm(q, pl, std::move(g));
      }
      {
        // H_k = sum_b P_bk P_bk^T (cap x cap)
        GemmDesc<T> g;
        g.ta = false;
        g.tb = true;
        g.M = cp_;
        g.N = cp_;
        g.K = rc;
        g.lda = cp_;
        g.ldb = cp_;
        g.ldc = cp_;
        g.nb = nb_active;
        g.terms_are_blocks = nb_active != nullptr;
        for (int k : modes) {
          std::vector<GemmTerm<T>> ts;
          for (int b = 0; b < nb; ++b) {
            const T* P = Pm + (size_t(k) * nb + b) * cp_ * rc;
            ts.push_back(term<T>(P, P));
          }
          g.group(Hc + size_t(k) * cp_ * cp_, ts);
        }
        emit_gemm(q, pl, std::move(g));
      }
    }
    CertParams cpar{};
    cpar.d = d;
    cpar.cap = cp_;
    cpar.nb = nb;
    cpar.delta = cfg.delta;
    const double uT = std::is_same<T, double>::value ? 0x1p-53 : 0x1p-24;
    for (int k = 0; k < d; ++k)
      cpar.rnd[k] = 4.0 * (double(sh.n[k]) * std::sqrt(double(cp_)) + double(nb) * rc) * uT;
    int* rt_ = rt;
    // join the Grams and norms, certify, run the eigensolves that the
    // certificate left, then keep the leading s columns of every basis
    q.steps.push_back(join);
    q.steps.push_back([=](hipStream_t st) {
      rank_certificate<T>(Hc, w, fro, nbA(), epsd + 1, cpar, cert_dev, rt_, st);
    });
    for (auto& f : eig_steps) q.steps.push_back(f);
    WidthZero<T> wz{};
    for (int k = 0; k < d; ++k) {
      wz.U[k] = Uh[k];
      wz.n[k] = sh.n[k];
    }
    q.steps.push_back([=](hipStream_t st) { width_and_zero<T>(wz, d, sc, rt_, p_, cap_, fs_, s_dev, st); });
  }
  // --- 4. core projection C^ = sum_b c_b G_b x_k (U^_k^T U_bk)
  T* Cb[2] = {ar.alloc<T>(sclen), ar.alloc<T>(sclen)};
  T* Bt = ar.alloc<T>(sclen);
  {
    std::array<const T*, kMaxD> Uc{};
    for (int k = 0; k < d; ++k) Uc[k] = Uh[k];
    plan_core_projection<T>(q, pl, sh, in, coef, Uc, sc, Cb[0], nb_active);
  }
  if (!use_cert && overlap) {
    // The rule's eigensolves ran beside steps 2-4: join them, then keep the
    // leading s columns of every basis and the leading s indices of every
    // core mode.  The projection was formed at the full width sc; basis
    // column i only meets core index i of its mode, so zeroing both after
    // the fact gives the same core as projecting onto the zeroed basis.
    q.steps.push_back(join);
    WidthZero<T> wz{};
    for (int k = 0; k < d; ++k) {
      wz.U[k] = Uh[k];
      wz.n[k] = sh.n[k];
    }
    wz.core = Cb[0];
    int* rt_ = rt;
    q.steps.push_back([=](hipStream_t st) { width_and_zero<T>(wz, d, sc, rt_, p_, cap_, fs_, s_dev, st); });
  }
  // --- 5. ST-HOSVD of C^, modes 1..d in order.  Per mode the truncation is
  //        decided by a Jacobi eigen-solve of the Gram of the ROTATED unfolding
  //        V1^T C_(k): for a V1 close to the eigenbasis that Gram is graded, so
  //        small singular values keep their digits and the decision matches a
  //        true SVD of the current (already truncated) core.  V1 only has to be
  //        orthogonal and close: all d of them come from one batched solve on
  //        the unfolding Grams of the untruncated core C^ (exact for mode 1,
  //        close for later modes since truncation removes little energy), so
  //        the d solves of that pass run side by side instead of in sequence.
  {
    // total = ||C^||_F^2
    std::vector<const T*> pc = {Cb[0]};
    const size_t offc = blob.add(pc);
    q.steps.push_back([=](hipStream_t st) {
      dot_batched<T>(bl->at<const T*>(offc), bl->at<const T*>(offc), sclen, 1, 1.0, total, st);
    });
  }
  T* G1 = ar.alloc<T>(size_t(d) * sc * sc);
  T* G2 = ar.alloc<T>(size_t(sc) * sc);
  T* lam1 = ar.alloc<T>(size_t(d) * sc);
  T* lam2 = ar.alloc<T>(sc);
  std::array<T*, kMaxD> V1{}, V2{}, U12{};
  int dims[kMaxD];
  for (int j = 0; j < d; ++j) dims[j] = sc;
  {
    std::vector<EigTask<T>> et(d);
    int in_splits = 1;
    for (int k = 0; k < d; ++k) {
      V1[k] = ar.alloc<T>(size_t(sc) * sc);
      V2[k] = ar.alloc<T>(size_t(sc) * sc);
      U12[k] = ar.alloc<T>(size_t(sc) * sc);
      // the eigensolver sums the Gram's split-K partials itself
      SplitOut<T> so;
      emit_unfold_gram<T>(q, pl, d, dims, k, Cb[0], Cb[0], G1 + size_t(k) * sc * sc, sc, 1.0, &so);
      et[k] = EigTask<T>{};
      et[k].A = G1 + size_t(k) * sc * sc;
      et[k].lda = sc;
      et[k].lam = lam1 + size_t(k) * sc;
      et[k].V = V1[k];
      et[k].part = so.part;
      et[k].splits = so.splits;
      et[k].pstride = so.stride;
      in_splits = std::max(in_splits, so.splits);  // equal for every mode (same K)
    }
    const size_t off = blob.add(et);
    q.steps.push_back([=](hipStream_t st) { jacobi_eig<T>(bl->at<EigTask<T>>(off), d, sc, true, st, in_splits); });
  }
  int cb = 0;
  for (int k = 0; k < d; ++k) {
    emit_ttm<T>(q, pl, d, dims, k, sc, {Cb[cb]}, {V1[k]}, sc, true, {Bt});
    SplitOut<T> so;
    emit_unfold_gram<T>(q, pl, d, dims, k, Bt, Bt, G2, sc, 1.0, &so);
    {
      std::vector<EigTask<T>> et(1);
      et[0] = EigTask<T>{};
      et[0].A = G2;
      et[0].lda = sc;
      et[0].part = so.part;
      et[0].splits = so.splits;
      et[0].pstride = so.stride;
      et[0].lam = lam2;
      et[0].V = V2[k];
      et[0].rule.kind = 2;
      et[0].rule.eps = epsd;
      et[0].rule.d = d;
      et[0].rule.cap = sh.cap;
      et[0].rule.total = total;
      et[0].rule.zthr = zthr;
      et[0].rule.force = (cfg.force_r[k] >= 0) ? force_dev + k : nullptr;
      et[0].rule.rank_out = out.rank + k;
      const size_t off = blob.add(et);
      const int in_splits = std::max(1, so.splits);
      q.steps.push_back([=](hipStream_t st) { jacobi_eig<T>(bl->at<EigTask<T>>(off), 1, sc, true, st, in_splits); });
    }
    emit_ttm<T>(q, pl, d, dims, k, sc, {Bt}, {V2[k]}, sc, true, {Cb[1 - cb]});
    cb = 1 - cb;
  }
  {
    // U12_k = V1_k V2_k for every mode, one grouped launch off the chain
    GemmDesc<T> g;
    g.M = sc;
    g.N = sc;
    g.K = sc;
    g.lda = sc;
    g.ldb = sc;
    g.ldc = sc;
    for (int k = 0; k < d; ++k) g.group1(U12[k], V1[k], V2[k]);
    emit_gemm(q, pl, std::move(g));
  }
  // factors U_k = U^_k U12_k[:, :min(rc, sc)]
  for (auto& modes : modes_by_n<T>(sh)) {
    const int n = sh.n[modes[0]];
    if (rc > sc)
      for (int k : modes) {
        T* u = out.U[k];
        const size_t len = size_t(n) * rc;
        q.steps.push_back([=](hipStream_t st) { fill<T>(u, len, T(0), st); });
      }
    GemmDesc<T> g;
    g.M = n;
    g.N = std::min(rc, sc);
    g.K = sc;
    g.lda = n;
    g.ldb = sc;
    g.ldc = n;
    for (int k : modes) g.group1(out.U[k], Uh[k], U12[k]);
    emit_gemm(q, pl, std::move(g));
  }
  {
    T* src = Cb[cb];
    T* dst = out.core;
    int sd[kMaxD], dd[kMaxD], nn[kMaxD];
    for (int j = 0; j < kMaxD; ++j) {
      sd[j] = sc;
      dd[j] = rc;
      nn[j] = sh.n[j];
    }
    std::array<T*, kMaxD> U = {out.U[0], out.U[1], out.U[2], out.U[3]};
    int* rk = out.rank;
    q.steps.push_back([=](hipStream_t st) {
      core_recap_fixup<T>(src, sd, dst, dd, d, total, zthr, nn, rc, U.data(), rk, st);
    });
  }
  RoundSumOut<T> o;
  o.s_dev = s_dev;
  o.total_dev = total;
  return o;
}

// ====================================================================== apply
template <typename T>
Blocks<T> plan_apply(Seq& q, Planner& pl, const Shape& sh, const OpDev<T>& op, const TT<T>& x, bool transpose,
                     std::vector<T*>* products) {
  const int d = sh.d, rc = sh.rc;
  std::map<std::pair<const T*, int>, T*> prod;
  std::vector<std::pair<const T*, int>> order;
  for (int j = 0; j < op.nterms; ++j)
    for (int k = 0; k < d; ++k) {
      const T* A = op.A[j * d + k];
      if (!A) continue;
      auto key = std::make_pair(A, k);
      if (prod.count(key)) continue;
      prod[key] = pl.ar.alloc<T>(size_t(sh.n[k]) * rc);
      order.push_back(key);
    }
  for (auto& modes : modes_by_n<T>(sh)) {
    const int n = sh.n[modes[0]];
    GemmDesc<T> g;
    g.ta = !transpose;  // row-major A seen column-major is A^T
    g.tb = false;
    g.M = n;
    g.N = rc;
    g.K = n;
    g.lda = n;
    g.ldb = n;
    g.ldc = n;
    for (auto& key : order)
      if (std::find(modes.begin(), modes.end(), key.second) != modes.end())
        g.group1(prod[key], key.first, x.U[key.second]);
    g.factor_product = true;
    emit_gemm(q, pl, std::move(g));
  }
  Blocks<T> out;
  for (int j = 0; j < op.nterms; ++j) {
    std::array<const T*, kMaxD> U{};
    for (int k = 0; k < d; ++k) {
      const T* A = op.A[j * d + k];
      U[k] = A ? prod[std::make_pair(A, k)] : x.U[k];
    }
    out.add(x.core, U, x.rank, nullptr, op.alpha[j]);
  }
  if (products)
    for (auto& key : order) products->push_back(prod[key]);
  return out;
}

// ====================================================================== sketch
template <typename T>
void plan_sketch(Seq& q, Planner& pl, const Shape& sh, const Blocks<T>& in, const std::array<const T*, kMaxD>& S,
                 int s, double* out) {
  const int d = sh.d, rc = sh.rc, nb = in.size();
  Arena& ar = pl.ar;
  Blob* bl = &pl.blob;
  const size_t P = size_t(ipow(rc, d - 1));
  T* Pk = ar.alloc<T>(size_t(nb) * d * rc * s);
  auto Pp = [&](int b, int k) { return Pk + (size_t(b) * d + k) * rc * s; };
  for (auto& modes : modes_by_n<T>(sh)) {
    const int n = sh.n[modes[0]];
    GemmDesc<T> g;
    g.ta = true;
    g.tb = false;
    g.M = rc;
    g.N = s;
    g.K = n;
    g.lda = n;
    g.ldb = n;
    g.ldc = rc;
    for (int b = 0; b < nb; ++b)
      for (int k : modes) g.group1(Pp(b, k), in.U[b][k], S[k]);
    g.factor_product = true;
    emit_gemm(q, pl, std::move(g));
  }
  T* Z = ar.alloc<T>(size_t(nb) * P * s);
  {
    GemmDesc<T> g;
    g.ta = true;
    g.tb = false;
    g.M = int(P);
    g.N = s;
    g.K = rc;
    g.lda = rc;
    g.ldb = rc;
    g.ldc = int(P);
    for (int b = 0; b < nb; ++b) g.group1(Z + size_t(b) * P * s, in.core[b], Pp(b, d - 1));
    emit_gemm(q, pl, std::move(g));
  }
  T* vb = ar.alloc<T>(size_t(nb) * s);
  std::vector<KrpTask<T>> tasks;
  for (int b = 0; b < nb; ++b) {
    KrpTask<T> t{};
    t.Z = Z + size_t(b) * P * s;
    for (int j = 0; j < d - 1; ++j) {
      t.Mj[j] = Pp(b, j);
      t.ldm[j] = rc;
    }
    t.out = vb + size_t(b) * s;
    t.coef = in.cptr[b];
    t.scale = in.cscale[b];
    t.f = -1;
    t.ldo = 1;
    tasks.push_back(t);
  }
  const size_t off = pl.blob.add(tasks);
  std::vector<int> z(d - 1, rc);
  q.steps.push_back([=](hipStream_t st) {
    krp_reduce<T>(bl->at<KrpTask<T>>(off), nb, d - 1, z.data(), int(P), s, st);
    sum_vectors<T>(vb, size_t(s), nb, s, out, st);
  });
}

// ====================================================================== inner products
template <typename T>
void plan_inner(Seq& q, Planner& pl, const Shape& sh, const std::vector<TT<T>>& xs, const Blocks<T>& ys, double* out,
                double scale, std::vector<T*>* grams_out) {
  // pairs i: (xs[i] or xs[0]) with (ys block i or ys block 0)
  const int d = sh.d, rc = sh.rc;
  const int np = std::max<int>(int(xs.size()), ys.size());
  Arena& ar = pl.ar;
  Blob* bl = &pl.blob;
  auto X = [&](int i) { return xs.size() == 1 ? xs[0] : xs[i]; };
  auto Yi = [&](int i) { return ys.size() == 1 ? 0 : i; };
  T* G = ar.alloc<T>(size_t(np) * d * rc * rc);
  auto Gp = [&](int i, int k) { return G + (size_t(i) * d + k) * rc * rc; };
  for (auto& modes : modes_by_n<T>(sh)) {
    const int n = sh.n[modes[0]];
    GemmDesc<T> g;
    g.ta = true;
    g.tb = false;
    g.M = rc;
    g.N = rc;
    g.K = n;
    g.lda = n;
    g.ldb = n;
    g.ldc = rc;
    for (int i = 0; i < np; ++i)
      for (int k : modes) g.group1(Gp(i, k), X(i).U[k], ys.U[Yi(i)][k]);
    emit_gemm(q, pl, std::move(g));
  }
  const size_t corelen = size_t(ipow(rc, d));
  T* H0 = ar.alloc<T>(size_t(np) * corelen);
  T* H1 = ar.alloc<T>(size_t(np) * corelen);
  int dims[kMaxD];
  for (int j = 0; j < d; ++j) dims[j] = rc;
  const T* const* src = nullptr;
  (void)src;
  std::vector<const T*> Xs, Ws;
  std::vector<T*> Ys;
  for (int i = 0; i < np; ++i) {
    Xs.push_back(ys.core[Yi(i)]);
    Ws.push_back(Gp(i, d - 1));
    Ys.push_back(H0 + size_t(i) * corelen);
  }
  emit_ttm<T>(q, pl, d, dims, d - 1, rc, Xs, Ws, rc, false, Ys);
  T* cur = H0;
  T* nxt = H1;
  for (int k = d - 2; k >= 0; --k) {
    Xs.clear();
    Ws.clear();
    Ys.clear();
    for (int i = 0; i < np; ++i) {
      Xs.push_back(cur + size_t(i) * corelen);
      Ws.push_back(Gp(i, k));
      Ys.push_back(nxt + size_t(i) * corelen);
    }
    emit_ttm<T>(q, pl, d, dims, k, rc, Xs, Ws, rc, false, Ys);
    std::swap(cur, nxt);
  }
  std::vector<const T*> a, b;
  for (int i = 0; i < np; ++i) {
    a.push_back(X(i).core);
    b.push_back(cur + size_t(i) * corelen);
  }
  const size_t oa = pl.blob.add(a), ob = pl.blob.add(b);
  q.steps.push_back([=](hipStream_t st) {
    dot_batched<T>(bl->at<const T*>(oa), bl->at<const T*>(ob), corelen, np, scale, out, st);
  });
  if (grams_out)
    for (int i = 0; i < np; ++i)
      for (int k = 0; k < d; ++k) grams_out->push_back(Gp(i, k));
}

// ====================================================================== exact norm
void plan_exact_norm2(Seq& q, Planner& pl, const Shape& sh, const Blocks<double>& in, double* out_norm2) {
  constexpr double kCutTol = 64.0 * 0x1p-53;
  const int d = sh.d, rc = sh.rc, nb = in.size();
  Arena& ar = pl.ar;
  Blob* bl = &pl.blob;
  // distinct factors per mode (first appearance order)
  // The QR of each distinct factor uses its owner's rank as the active column
  // count: padding columns must give zero basis vectors, not unit vectors that
  // would break the orthonormality of the concatenated basis.
  std::vector<std::vector<const double*>> fac(d);
  std::vector<std::vector<const int*>> facr(d);
  std::vector<std::vector<int>> idx(nb, std::vector<int>(d));
  int m = 1;
  for (int k = 0; k < d; ++k) {
    for (int b = 0; b < nb; ++b) {
      auto it = std::find(fac[k].begin(), fac[k].end(), in.U[b][k]);
      if (it == fac[k].end()) {
        fac[k].push_back(in.U[b][k]);
        facr[k].push_back(in.rank[b] + k);
        idx[b][k] = int(fac[k].size()) - 1;
      } else {
        idx[b][k] = int(it - fac[k].begin());
      }
    }
    m = std::max(m, int(fac[k].size()));
  }
  TK_CHECK(rc <= 64, kErrUnsupported, "exact norm: rank capacity above 64");
  const int Md = m * rc;
  std::vector<double*> Qk(d), Rk(d), Xt(d), Ct(d), Rt(d), R2t(d);
  double* coef = ar.alloc<double>(nb);
  const size_t off_cptr = pl.blob.add(in.cptr), off_cs = pl.blob.add(in.cscale);
  q.steps.push_back([=](hipStream_t st) {
    gather_coef(bl->at<const double*>(off_cptr), bl->at<double>(off_cs), nb, coef, st);
  });
  for (int k = 0; k < d; ++k) {
    const int n = sh.n[k];
    Qk[k] = ar.alloc<double>(size_t(n) * Md);
    Rk[k] = ar.alloc<double>(size_t(Md) * Md);
    Xt[k] = ar.alloc<double>(size_t(n) * rc);
    Ct[k] = ar.alloc<double>(size_t(Md) * rc);
    Rt[k] = ar.alloc<double>(size_t(rc) * rc);
    R2t[k] = ar.alloc<double>(size_t(rc) * rc);
    double* R = Rk[k];
    q.steps.push_back([=](hipStream_t st) { fill<double>(R, size_t(Md) * Md, 0.0, st); });
  }
  // Block i of every mode (modes of equal size batched into the same launches):
  // BCGS2 against blocks 0..i-1, rank-revealing QR of the remainder, then one
  // re-orthogonalisation of the new basis block.
  for (auto& modes : modes_by_n<double>(sh)) {
    const int n = sh.n[modes[0]];
    int imax = 0;
    for (int k : modes) imax = std::max(imax, int(fac[k].size()));
    for (int i = 0; i < imax; ++i) {
      std::vector<int> act;
      for (int k : modes)
        if (i < int(fac[k].size())) act.push_back(k);
      const int na = int(act.size());
      auto Rblk = [&](int k) { return Rk[k] + size_t(i) * rc * Md; };  // column block i
      auto Qi = [&](int k) { return Qk[k] + size_t(i) * rc * n; };
      auto Rdiag = [&](int k) { return Rblk(k) + size_t(i) * rc; };
      // GEMM over the active modes: C_k = alpha op(A_k) B_k (+ beta C_k)
      auto gemm = [&](bool ta, int M, int N, int K, int lda, int ldb, int ldc, double beta, double alpha,
                      auto Cf, auto Af, auto Bf) {
        GemmDesc<double> g;
        g.ta = ta;
        g.M = M;
        g.N = N;
        g.K = K;
        g.lda = lda;
        g.ldb = ldb;
        g.ldc = ldc;
        g.beta = beta;
        for (int k : act) g.group1(Cf(k), Af(k), Bf(k), nullptr, nullptr, nullptr, alpha);
        emit_gemm(q, pl, std::move(g));
      };
      std::vector<double*> xs;
      std::vector<const double*> fs;
      for (int k : act) {
        xs.push_back(Xt[k]);
        fs.push_back(fac[k][i]);
      }
      // the first block's QR reads the factors in place (it does not write
      // its input); later blocks are orthogonalised in a working copy
      if (i > 0)
        q.steps.push_back([=](hipStream_t st) {
          for (int a2 = 0; a2 < na; ++a2) mat_recap<double>(fs[a2], n, n, rc, xs[a2], n, n, rc, st);
        });
      if (i > 0) {
        const int Kq = i * rc;
        // C1 = Q^T F -> R[0:Kq, block i];  X -= Q C1;  C2 = Q^T X;  X -= Q C2
        gemm(true, Kq, rc, n, n, n, Md, 0.0, 1.0, Rblk, [&](int k) { return (const double*)Qk[k]; },
             [&](int k) { return fac[k][i]; });
        gemm(false, n, rc, Kq, n, Md, n, 1.0, -1.0, [&](int k) { return Xt[k]; },
             [&](int k) { return (const double*)Qk[k]; }, [&](int k) { return (const double*)Rblk(k); });
        gemm(true, Kq, rc, n, n, n, Md, 0.0, 1.0, [&](int k) { return Ct[k]; },
             [&](int k) { return (const double*)Qk[k]; }, [&](int k) { return (const double*)Xt[k]; });
        gemm(false, n, rc, Kq, n, Md, n, 1.0, -1.0, [&](int k) { return Xt[k]; },
             [&](int k) { return (const double*)Qk[k]; }, [&](int k) { return (const double*)Ct[k]; });
        std::vector<const double*> cts;
        std::vector<double*> rbs;
        for (int k : act) {
          cts.push_back(Ct[k]);
          rbs.push_back(Rblk(k));
        }
        q.steps.push_back([=](hipStream_t st) {
          for (int a2 = 0; a2 < na; ++a2) mat_axpy<double>(cts[a2], Md, rbs[a2], Md, Kq, rc, st);
        });
      }
      // rank-revealing QR of the remainder: columns left with <= 64 u of their
      // norm in the factor lie (numerically) inside the earlier blocks' span
      // and are cut; what is cut is below the rounding of the core sum itself
      // the basis of a mode's last block is needed only when it is re-orthogonalised
      // (blocks after the first) or projected out of later blocks
      // A mode with a single distinct factor needs only R, and with no earlier
      // block there is nothing to cut against: the R of a plain Householder
      // QR gives the same core norm (a column the cut would drop contributes
      // at the 64 u level), at a fraction of the pivoted kernel's cost.
      // With one factor per mode (Md = rc) the first block's R goes straight
      // into its place in R_k.
      const bool direct_r = i == 0 && Md == rc;
      std::vector<QrPivTask> qt;
      std::vector<QrTask> qs;
      for (int k : act) {
        const bool need_q = i > 0 || int(fac[k].size()) > 1;
        const double* y = i == 0 ? fac[k][0] : Xt[k];
        double* r = direct_r ? Rk[k] : Rt[k];
        if (need_q)
          qt.push_back(QrPivTask{y, fac[k][i], Qi(k), r, facr[k][i]});
        else
          qs.push_back(QrTask{y, nullptr, r, facr[k][i]});
      }
      if (!qs.empty()) {
        const size_t off = pl.blob.add(qs);
        const int ns = int(qs.size());
        q.steps.push_back([=](hipStream_t st) { qr_batched(bl->at<QrTask>(off), ns, n, rc, nullptr, st); });
      }
      if (!qt.empty()) {
        const size_t off = pl.blob.add(qt);
        const int np = int(qt.size());
        q.steps.push_back([=](hipStream_t st) { qr_piv_batched(bl->at<QrPivTask>(off), np, n, rc, kCutTol, st); });
      }
      if (i == 0) {
        if (!direct_r) {
          std::vector<const double*> rts;
          std::vector<double*> rds;
          for (int k : act) {
            rts.push_back(Rt[k]);
            rds.push_back(Rdiag(k));
          }
          q.steps.push_back([=](hipStream_t st) {
            for (int a2 = 0; a2 < na; ++a2) mat_recap<double>(rts[a2], rc, rc, rc, rds[a2], Md, rc, rc, st);
          });
        }
        continue;
      }
      // Re-orthogonalise the new block's basis against the previous blocks: a
      // kept column with remainder norm rho comes out of its QR orthogonal to
      // the earlier blocks only to about u / rho.  With T = Q_prev^T Q_i and
      // Q_i - Q_prev T = Q_i' R'': F = Q_prev (C + T R_i) + Q_i' (R'' R_i).
      const int Kq = i * rc;
      gemm(true, Kq, rc, n, n, n, Md, 0.0, 1.0, [&](int k) { return Ct[k]; },
           [&](int k) { return (const double*)Qk[k]; }, [&](int k) { return (const double*)Qi(k); });
      {
        std::vector<const double*> qis;
        for (int k : act) qis.push_back(Qi(k));
        q.steps.push_back([=](hipStream_t st) {
          for (int a2 = 0; a2 < na; ++a2) mat_recap<double>(qis[a2], n, n, rc, xs[a2], n, n, rc, st);
        });
      }
      gemm(false, n, rc, Kq, n, Md, n, 1.0, -1.0, [&](int k) { return Xt[k]; },
           [&](int k) { return (const double*)Qk[k]; }, [&](int k) { return (const double*)Ct[k]; });
      std::vector<QrPivTask> qt2;
      for (int k : act) qt2.push_back(QrPivTask{Xt[k], Qi(k), Qi(k), R2t[k], facr[k][i]});
      const size_t off2 = pl.blob.add(qt2);
      q.steps.push_back([=](hipStream_t st) { qr_piv_batched(bl->at<QrPivTask>(off2), na, n, rc, kCutTol, st); });
      // R[0:Kq, block i] += T R_i;  diagonal block = R'' R_i
      gemm(false, Kq, rc, rc, Md, rc, Md, 1.0, 1.0, Rblk, [&](int k) { return (const double*)Ct[k]; },
           [&](int k) { return (const double*)Rt[k]; });
      gemm(false, rc, rc, rc, rc, rc, Md, 0.0, 1.0, Rdiag, [&](int k) { return (const double*)R2t[k]; },
           [&](int k) { return (const double*)Rt[k]; });
    }
  }
  // core = sum_b c_b G_b x_k R_k[:, block(b, k)]   (Md^d)
  const size_t tl = size_t(rc) * size_t(ipow(Md, d - 1));
  double* T0 = ar.alloc<double>(size_t(nb) * tl);
  double* T1 = ar.alloc<double>(size_t(nb) * tl);
  double* core = ar.alloc<double>(size_t(ipow(Md, d)));
  int dims[kMaxD];
  for (int j = 0; j < d; ++j) dims[j] = rc;
  auto W = [&](int b, int k) { return (const double*)(Rk[k] + size_t(idx[b][k]) * rc * Md); };
  std::vector<const double*> Xs, Ws;
  std::vector<double*> Ys;
  std::vector<const double*> cs;
  for (int b = 0; b < nb; ++b) {
    Xs.push_back(in.core[b]);
    Ws.push_back(W(b, d - 1));
    Ys.push_back(T0 + size_t(b) * tl);
    cs.push_back(coef + b);
  }
  emit_ttm<double>(q, pl, d, dims, d - 1, Md, Xs, Ws, Md, false, Ys);
  dims[d - 1] = Md;
  double* cur = T0;
  double* nxt = T1;
  for (int k = d - 2; k >= 1; --k) {
    Xs.clear();
    Ws.clear();
    Ys.clear();
    for (int b = 0; b < nb; ++b) {
      Xs.push_back(cur + size_t(b) * tl);
      Ws.push_back(W(b, k));
      Ys.push_back(nxt + size_t(b) * tl);
    }
    emit_ttm<double>(q, pl, d, dims, k, Md, Xs, Ws, Md, false, Ys);
    dims[k] = Md;
    std::swap(cur, nxt);
  }
  Xs.clear();
  Ws.clear();
  for (int b = 0; b < nb; ++b) {
    Xs.push_back(cur + size_t(b) * tl);
    Ws.push_back(W(b, 0));
  }
  emit_ttm<double>(q, pl, d, dims, 0, Md, Xs, Ws, Md, false, {}, core, &cs);
  const size_t corelen = size_t(ipow(Md, d));
  std::vector<const double*> pc = {core};
  const size_t offc = pl.blob.add(pc);
  q.steps.push_back([=](hipStream_t st) {
    dot_batched<double>(bl->at<const double*>(offc), bl->at<const double*>(offc), corelen, 1, 1.0, out_norm2, st);
  });
}

template <typename T>
void plan_ttm(Seq& q, Planner& pl, int d, const int* dims, int k, int newdim, const T* X, const T* W, int ldw,
              bool w_transposed, T* Y) {
  emit_ttm<T>(q, pl, d, dims, k, newdim, {X}, {W}, ldw, w_transposed, {Y});
}

template <typename T>
void plan_unfold_gram(Seq& q, Planner& pl, int d, const int* dims, int k, const T* X, const T* Y, T* G, int ldg,
                      double scale) {
  emit_unfold_gram<T>(q, pl, d, dims, k, X, Y, G, ldg, scale);
}

template <typename T>
void plan_gemm(Seq& q, Planner& pl, bool ta, bool tb, int M, int N, int K, const T* A, int lda, const T* B, int ldb,
               T* C, int ldc, double alpha, double beta, bool factor_product) {
  GemmDesc<T> g;
  g.factor_product = factor_product;
  g.ta = ta;
  g.tb = tb;
  g.M = M;
  g.N = N;
  g.K = K;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.beta = beta;
  g.group1(C, A, B, nullptr, nullptr, nullptr, alpha);
  emit_gemm(q, pl, std::move(g));
}

template <typename T>
void plan_gemm_batched(Seq& q, Planner& pl, bool ta, bool tb, int M, int N, int K, const std::vector<const T*>& A,
                       int lda, const std::vector<const T*>& B, int ldb, const std::vector<T*>& C, int ldc,
                       double alpha) {
  TK_CHECK(A.size() == B.size() && A.size() == C.size(), kErrInvalidArg, "batched GEMM: table sizes differ");
  GemmDesc<T> g;
  g.ta = ta;
  g.tb = tb;
  g.M = M;
  g.N = N;
  g.K = K;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  for (size_t i = 0; i < C.size(); ++i) g.group1(C[i], A[i], B[i], nullptr, nullptr, nullptr, alpha);
  emit_gemm(q, pl, std::move(g));
}

// ====================================================================== preconditioner
template <typename T>
Blocks<T> plan_precond_terms(Seq& q, Planner& pl, const Shape& sh, const PrecondT<T>& pc, const TT<T>& x) {
  const int d = sh.d, rc = sh.rc, qn = pc.q, nh = 2 * qn + 1;
  TK_CHECK(qn >= 1, kErrInvalidArg, "preconditioner: q must be >= 1");
  Arena& ar = pl.ar;
  Blob* bl = &pl.blob;
  // spectral factors V_k^T U_k, one GEMM launch per group of equal mode size
  std::array<T*, kMaxD> Ut{};
  for (int k = 0; k < d; ++k) Ut[k] = ar.alloc<T>(size_t(sh.n[k]) * rc);
  for (auto& modes : modes_by_n<T>(sh)) {
    const int n = sh.n[modes[0]];
    std::vector<const T*> a, b;
    std::vector<T*> c;
    for (int k : modes) {
      a.push_back(pc.V[k]);
      b.push_back(x.U[k]);
      c.push_back(Ut[k]);
    }
    plan_gemm_batched<T>(q, pl, true, false, n, rc, n, a, n, b, n, c, n, 1.0);
  }
  // the 2q + 1 terms: row scalings exp(-t_h (lambda - lambda_min)) of every
  // spectral factor (largest entry 1) and device coefficients
  // eta t_h exp(-t_h sum_k lambda_min,k), so that a block's coefficient bounds
  // its size (RoundSum weighs blocks by |coefficient| ||core||)
  const double eta = 3.14159265358979323846 / std::sqrt(double(qn));
  double* lmin = ar.alloc<double>(kMaxD);
  double* coef = ar.alloc<double>(nh);
  {
    std::array<const T*, kMaxD> lam = pc.lam;
    std::array<int, kMaxD> nn{};
    for (int k = 0; k < d; ++k) nn[k] = sh.n[k];
    q.steps.push_back([=](hipStream_t st) { expsum_shift<T>(lam.data(), nn.data(), d, qn, eta, lmin, coef, st); });
  }
  std::vector<std::array<const T*, kMaxD>> fac(nh);
  for (auto& modes : modes_by_n<T>(sh)) {
    const int n = sh.n[modes[0]];
    std::vector<ExpScaleTask<T>> tasks;
    for (int h = 0; h < nh; ++h) {
      const double t = std::exp((h - qn) * eta);
      for (int k : modes) {
        T* o = ar.alloc<T>(size_t(n) * rc);
        tasks.push_back(ExpScaleTask<T>{Ut[k], pc.lam[k], lmin + k, o, t});
        fac[h][k] = o;
      }
    }
    const size_t off = pl.blob.add(tasks);
    const int nt = int(tasks.size());
    q.steps.push_back([=](hipStream_t st) { exp_scale_rows<T>(bl->at<ExpScaleTask<T>>(off), nt, n, rc, st); });
  }
  Blocks<T> terms;
  for (int h = 0; h < nh; ++h) terms.add(x.core, fac[h], x.rank, coef + h, 1.0);
  return terms;
}

template <typename T>
void plan_precond(Seq& q, Planner& pl, const Shape& sh, const PrecondT<T>& pc, const TT<T>& x, const TT<T>& z,
                  const RoundCfg& rcfg, const std::array<const T*, kMaxD>& omega) {
  const int d = sh.d, rc = sh.rc;
  Arena& ar = pl.ar;
  Blocks<T> terms = plan_precond_terms<T>(q, pl, sh, pc, x);
  // rounding in the spectral basis at the full sketch width; the core goes
  // straight into z, the factors into temporaries that are mapped back
  RoundCfg cfg = rcfg;
  cfg.force_s = sh.sc();
  TT<T> zt;
  zt.core = z.core;
  zt.rank = z.rank;
  for (int k = 0; k < d; ++k) zt.U[k] = ar.alloc<T>(size_t(sh.n[k]) * rc);
  plan_roundsum<T>(q, pl, sh, terms, cfg, omega, zt, nullptr);
  for (auto& modes : modes_by_n<T>(sh)) {
    const int n = sh.n[modes[0]];
    std::vector<const T*> a, b;
    std::vector<T*> c;
    for (int k : modes) {
      a.push_back(pc.V[k]);
      b.push_back(zt.U[k]);
      c.push_back(z.U[k]);
    }
    plan_gemm_batched<T>(q, pl, false, false, n, rc, n, a, n, b, n, c, n, 1.0);
  }
}

#define TK_INST(T)                                                                                             \
  template void plan_ttm<T>(Seq&, Planner&, int, const int*, int, int, const T*, const T*, int, bool, T*);     \
  template void plan_unfold_gram<T>(Seq&, Planner&, int, const int*, int, const T*, const T*, T*, int, double); \
  template void plan_gemm<T>(Seq&, Planner&, bool, bool, int, int, int, const T*, int, const T*, int, T*, int,   \
                             double, double, bool);                                                                  \
  template RoundSumOut<T> plan_roundsum<T>(Seq&, Planner&, const Shape&, const Blocks<T>&, const RoundCfg&,   \
                                           const std::array<const T*, kMaxD>&, const TT<T>&, const int*);      \
  template Blocks<T> plan_apply<T>(Seq&, Planner&, const Shape&, const OpDev<T>&, const TT<T>&, bool,         \
                                   std::vector<T*>*);                                                          \
  template void plan_sketch<T>(Seq&, Planner&, const Shape&, const Blocks<T>&, const std::array<const T*, kMaxD>&, \
                               int, double*);                                                                  \
  template void plan_inner<T>(Seq&, Planner&, const Shape&, const std::vector<TT<T>>&, const Blocks<T>&,      \
                              double*, double, std::vector<T*>*);                                              \
  template void plan_gemm_batched<T>(Seq&, Planner&, bool, bool, int, int, int, const std::vector<const T*>&, \
                                     int, const std::vector<const T*>&, int, const std::vector<T*>&, int, double); \
  template void plan_krp_range<T>(Seq&, Planner&, const Shape&, const Blocks<T>&, const double*,              \
                                  const std::array<const T*, kMaxD>&, int, const std::array<T*, kMaxD>&,     \
                                  const int*);                                                                 \
  template void plan_core_projection<T>(Seq&, Planner&, const Shape&, const Blocks<T>&, const double*,        \
                                        const std::array<const T*, kMaxD>&, int, T*, const int*);         \
  template void plan_precond<T>(Seq&, Planner&, const Shape&, const PrecondT<T>&, const TT<T>&, const TT<T>&,  \
                                const RoundCfg&, const std::array<const T*, kMaxD>&);                         \
  template Blocks<T> plan_precond_terms<T>(Seq&, Planner&, const Shape&, const PrecondT<T>&, const TT<T>&);
TK_INST(double)
TK_INST(float)
#undef TK_INST

}  // namespace tk
