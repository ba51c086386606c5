// C ABI of the library (declared in include/tsgmres.h): argument checks,
// import of caller tensors into capacity-padded internal layouts, planning
// (measure-only for the *_workspace queries), execution and export.
#include <algorithm>
#include <cmath>
#include <memory>
#include <mutex>

#include "../../include/tsgmres.h"
#include "engine.hpp"

namespace tk {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
const char* last_error() { return g_err.c_str(); }

template <typename F>
static int guarded(F&& f) {
  try {
    g_err.clear();
    return f();
  } catch (const Error& e) {
    g_err = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    g_err = e.what();
    return kErrInvalidArg;
  } catch (...) {
    g_err = "unknown error";
    return kErrInvalidArg;
  }
}

namespace {

void check_tucker(const tk_tucker* t, const char* name, int d, const int64_t* n) {
  TK_CHECK(t != nullptr, kErrInvalidArg, std::string(name) + " is NULL");
  TK_CHECK(t->d == d, kErrShape, std::string(name) + ": order mismatch");
  TK_CHECK(t->core != nullptr, kErrInvalidArg, std::string(name) + ": core is NULL");
  for (int k = 0; k < d; ++k) {
    TK_CHECK(t->n[k] == n[k], kErrShape, std::string(name) + ": mode size mismatch");
    TK_CHECK(t->r[k] >= 1 && t->r[k] <= t->rcap[k], kErrShape, std::string(name) + ": rank outside [1, rcap]");
    TK_CHECK(t->r[k] <= t->n[k], kErrShape, std::string(name) + ": rank above mode size");
    TK_CHECK(t->U[k] != nullptr, kErrInvalidArg, std::string(name) + ": factor is NULL");
  }
}

void check_dims(int d, const int64_t* n) {
  TK_CHECK(d >= 2 && d <= kMaxD, kErrUnsupported, "order d must be in [2, 4]");
  for (int k = 0; k < d; ++k) {
    TK_CHECK(n[k] >= 1, kErrShape, "mode sizes must be positive");
    TK_CHECK(n[k] <= 512, kErrUnsupported, "mode sizes above 512 are not supported");
  }
}

void check_op(const tk_kron_op* op, int d, const int64_t* n) {
  TK_CHECK(op != nullptr, kErrInvalidArg, "operator is NULL");
  TK_CHECK(op->d == d, kErrShape, "operator order mismatch");
  for (int k = 0; k < d; ++k) TK_CHECK(op->n[k] == n[k], kErrShape, "operator mode size mismatch");
  TK_CHECK(op->nterms >= 1 && op->alpha != nullptr && op->A != nullptr, kErrInvalidArg, "operator has no terms");
}

// Host-side rank staging kept alive by the plan.
struct HostInts {
  int v[kMaxD] = {1, 1, 1, 1};
};

template <typename T>
void emit_import(Seq& q, const Shape& sh, const tk_tucker& u, const TT<T>& t) {
  auto hr = std::make_shared<HostInts>();
  int sd[kMaxD] = {1, 1, 1, 1}, sv[kMaxD] = {1, 1, 1, 1}, dd[kMaxD] = {1, 1, 1, 1};
  std::array<int, kMaxD> rk{}, ncol{};
  const int d = sh.d;
  for (int k = 0; k < d; ++k) {
    hr->v[k] = int(u.r[k]);
    sd[k] = int(u.rcap[k]);
    sv[k] = int(u.r[k]);
    dd[k] = sh.rc;
    rk[k] = int(u.r[k]);
    ncol[k] = sh.n[k];
  }
  const double* core = u.core;
  std::array<const double*, kMaxD> U = {u.U[0], u.U[1], u.U[2], u.U[3]};
  const int rc = sh.rc;
  q.steps.push_back([=](hipStream_t st) {
    core_recap<double>(core, sd, sv, t.core, dd, d, st);
    for (int k = 0; k < d; ++k) mat_recap<double>(U[k], ncol[k], ncol[k], rk[k], t.U[k], ncol[k], ncol[k], rc, st);
    TK_HIP(hipMemcpyAsync(t.rank, hr->v, sizeof(int) * kMaxD, hipMemcpyHostToDevice, st));
  });
}

// Copies an internal tensor out; ranks are read back first.
void export_tt(const Shape& sh, const TT<double>& t, tk_tucker* u, hipStream_t st) {
  int r[kMaxD] = {0, 0, 0, 0};
  TK_HIP(hipMemcpyAsync(r, t.rank, sizeof(int) * kMaxD, hipMemcpyDeviceToHost, st));
  TK_HIP(hipStreamSynchronize(st));
  const int d = sh.d;
  for (int k = 0; k < d; ++k)
    TK_CHECK(r[k] >= 1 && r[k] <= u->rcap[k], kErrCapacity,
             "output rank " + std::to_string(r[k]) + " exceeds the capacity of the output tensor");
  int sd[kMaxD] = {1, 1, 1, 1}, sv[kMaxD] = {1, 1, 1, 1}, dd[kMaxD] = {1, 1, 1, 1};
  for (int k = 0; k < d; ++k) {
    sd[k] = sh.rc;
    sv[k] = r[k];
    dd[k] = int(u->rcap[k]);
  }
  core_recap<double>(t.core, sd, sv, u->core, dd, d, st);
  for (int k = 0; k < d; ++k)
    mat_recap<double>(t.U[k], sh.n[k], sh.n[k], r[k], u->U[k], sh.n[k], sh.n[k], int(u->rcap[k]), st);
  for (int k = 0; k < d; ++k) u->r[k] = r[k];
  TK_HIP(hipStreamSynchronize(st));
}

// Element-type conversion of an internal tensor (capacity layout) and of a
// plain device array, as plan steps.
template <typename S, typename D>
void emit_cast_tt(Seq& q, const Shape& sh, const TT<S>& src, const TT<D>& dst) {
  const size_t cl = sh.core_len();
  const int d = sh.d;
  std::array<size_t, kMaxD> fl{};
  for (int k = 0; k < d; ++k) fl[k] = size_t(sh.n[k]) * sh.rc;
  q.steps.push_back([=](hipStream_t st) {
    cast_copy<S, D>(src.core, dst.core, cl, st);
    for (int k = 0; k < d; ++k) cast_copy<S, D>(src.U[k], dst.U[k], fl[k], st);
    copy_ints(src.rank, dst.rank, d, st);
  });
}
const float* emit_to_f32(Seq& q, Arena& ar, const double* src, size_t len) {
  float* dst = ar.alloc<float>(len);
  q.steps.push_back([=](hipStream_t st) { cast_copy<double, float>(src, dst, len, st); });
  return dst;
}
void check_form(int form) {
  TK_CHECK(form == TK_FORM_FP64 || form == TK_FORM_FP32 || form == TK_FORM_BF16, kErrUnsupported, "unknown form");
}

void finish_blob(Arena& ar, Blob& blob, hipStream_t st) {
  blob.dev = ar.alloc<unsigned char>(std::max<size_t>(blob.host.size(), 16));
  if (!ar.measuring())
    TK_HIP(hipMemcpyAsync(blob.dev, blob.host.data(), blob.host.size(), hipMemcpyHostToDevice, st));
}

Shape shape_of(int d, const int64_t* n, int rc, int cap, int p) {
  Shape sh;
  sh.d = d;
  for (int k = 0; k < d; ++k) sh.n[k] = int(n[k]);
  sh.rc = rc;
  sh.cap = cap;
  sh.p = p;
  return sh;
}

// ---------------------------------------------------------------- apply
int do_apply(const tk_kron_op* op, const tk_tucker* x, int transpose, int form, double* const* AU, Arena& ar,
             hipStream_t st) {
  TK_CHECK(x != nullptr, kErrInvalidArg, "x is NULL");
  check_dims(x->d, x->n);
  check_op(op, x->d, x->n);
  check_tucker(x, "x", x->d, x->n);
  check_form(form);
  const int d = x->d;
  Blob blob;
  Planner pl(ar, blob);
  pl.bf16_factors = form == TK_FORM_BF16;
  const bool f32 = form != TK_FORM_FP64;  // FP32 storage (FP32 and BF16-factor forms)
  Seq q;
  std::array<const float*, kMaxD> U32{};
  if (f32)
    for (int k = 0; k < d; ++k) U32[k] = emit_to_f32(q, ar, x->U[k], size_t(x->n[k]) * x->rcap[k]);
  for (int j = 0; j < op->nterms; ++j)
    for (int k = 0; k < d; ++k) {
      const double* A = op->A[j * d + k];
      if (!A) continue;
      TK_CHECK(AU != nullptr && AU[j * d + k] != nullptr, kErrInvalidArg, "missing output buffer for a factor product");
      const int n = int(x->n[k]), rcap = int(x->rcap[k]);
      if (f32) {
        const float* A32 = emit_to_f32(q, ar, A, size_t(n) * n);
        float* P32 = ar.alloc<float>(size_t(n) * rcap);
        plan_gemm<float>(q, pl, !transpose, false, n, rcap, n, A32, n, U32[k], n, P32, n, 1.0, 0.0, true);
        double* dst = AU[j * d + k];
        const size_t len = size_t(n) * rcap;
        q.steps.push_back([=](hipStream_t st) { cast_copy<float, double>(P32, dst, len, st); });
      } else {
        plan_gemm<double>(q, pl, !transpose, false, n, rcap, n, A, n, x->U[k], n, AU[j * d + k], n, 1.0, 0.0);
      }
    }
  finish_blob(ar, blob, st);
  if (ar.measuring()) return 0;
  q.run(st);
  TK_HIP(hipStreamSynchronize(st));
  return 0;
}

// Finiteness check of the inputs of a solve, run before any other kernel
// reads them: a non-finite entry makes the call fail with TK_ERR_NONFINITE.
// Tensors are checked after their import into the capacity layout, where the
// entries beyond the ranks are zero.
struct FiniteCheck {
  std::vector<const double*> ptr;
  std::vector<size_t> len;
  const double** dptr = nullptr;
  size_t* dlen = nullptr;
  int* count = nullptr;
  void add(const double* p, size_t n) {
    if (p != nullptr && n > 0) {
      ptr.push_back(p);
      len.push_back(n);
    }
  }
  void add_tt(const Shape& sh, const TT<double>& t) {
    add(t.core, sh.core_len());
    for (int k = 0; k < sh.d; ++k) add(t.U[k], size_t(sh.n[k]) * sh.rc);
  }
  void add_inputs(const Shape& sh, const tk_kron_op* op, const double* const* S, int64_t s,
                  const double* const* omega, int wo, const tk_sgmres_params* prm) {
    const int d = sh.d;
    for (int j = 0; j < op->nterms; ++j)
      for (int k = 0; k < d; ++k) add(op->A[j * d + k], size_t(sh.n[k]) * sh.n[k]);
    for (int k = 0; k < d; ++k) {
      if (S) add(S[k], size_t(sh.n[k]) * size_t(s));
      add(omega[k], size_t(sh.n[k]) * size_t(wo));
      if (prm->precond_q > 0 && prm->precond_V && prm->precond_lambda) {
        add(prm->precond_V[k], size_t(sh.n[k]) * sh.n[k]);
        add(prm->precond_lambda[k], size_t(sh.n[k]));
      }
    }
  }
  void alloc(Arena& ar) {
    dptr = ar.alloc<const double*>(std::max<size_t>(ptr.size(), 1));
    dlen = ar.alloc<size_t>(std::max<size_t>(len.size(), 1));
    count = ar.alloc<int>(1);
  }
  void run(hipStream_t st) const {
    if (ptr.empty()) return;
    TK_HIP(hipMemcpyAsync(dptr, ptr.data(), sizeof(const double*) * ptr.size(), hipMemcpyHostToDevice, st));
    TK_HIP(hipMemcpyAsync(dlen, len.data(), sizeof(size_t) * len.size(), hipMemcpyHostToDevice, st));
    size_t mx = 0;
    for (size_t l : len) mx = std::max(mx, l);
    count_nonfinite(dptr, dlen, int(ptr.size()), mx, count, st);
    int h = 0;
    TK_HIP(hipMemcpyAsync(&h, count, sizeof(int), hipMemcpyDeviceToHost, st));
    TK_HIP(hipStreamSynchronize(st));
    TK_CHECK(h == 0, kErrNonFinite,
             std::to_string(h) + " non-finite input entries (right-hand side, initial guess, operator, sketches "
                                 "or preconditioner)");
  }
};

// ---------------------------------------------------------------- block sums
struct Imported {
  Shape sh;
  std::vector<TT<double>> t;
  Blocks<double> blocks;
  std::shared_ptr<std::vector<double>> coef;
};

Imported import_blocks(Seq& q, Arena& ar, const tk_block_sum* in, int cap, int p) {
  TK_CHECK(in != nullptr && in->nblocks >= 1 && in->blocks != nullptr && in->coef != nullptr, kErrInvalidArg,
           "empty block sum");
  const tk_tucker& b0 = in->blocks[0];
  check_dims(b0.d, b0.n);
  int rc = std::max(cap, 1);
  for (int b = 0; b < in->nblocks; ++b) {
    check_tucker(&in->blocks[b], "block", b0.d, b0.n);
    for (int k = 0; k < b0.d; ++k) rc = std::max<int>(rc, int(in->blocks[b].r[k]));
  }
  TK_CHECK(rc <= 128, kErrUnsupported, "ranks above 128 are not supported");
  Imported im;
  im.sh = shape_of(b0.d, b0.n, rc, cap, p);
  im.coef = std::make_shared<std::vector<double>>(in->coef, in->coef + in->nblocks);
  for (int b = 0; b < in->nblocks; ++b) {
    TT<double> t = alloc_tt<double>(ar, im.sh);
    emit_import<double>(q, im.sh, in->blocks[b], t);
    im.t.push_back(t);
    im.blocks.add(t, nullptr, in->coef[b]);
  }
  return im;
}

// The imported blocks rounded to FP32 (same coefficients).
Blocks<float> blocks_f32(Seq& q, Arena& ar, const Imported& im) {
  Blocks<float> out;
  for (size_t b = 0; b < im.t.size(); ++b) {
    TT<float> t = alloc_tt<float>(ar, im.sh);
    emit_cast_tt<double, float>(q, im.sh, im.t[b], t);
    out.add(t, nullptr, im.blocks.cscale[b]);
  }
  return out;
}

int do_sketch(const tk_block_sum* x, const double* const* S, int64_t s, int form, double* out, Arena& ar,
              hipStream_t st) {
  TK_CHECK(S != nullptr && out != nullptr, kErrInvalidArg, "sketch factors or output missing");
  TK_CHECK(s >= 1 && s <= 65535, kErrInvalidArg, "sketch size out of range");
  check_form(form);
  Blob blob;
  Planner pl(ar, blob);
  Seq q;
  Imported im = import_blocks(q, ar, x, 1, 0);
  std::array<const double*, kMaxD> Sk{};
  for (int k = 0; k < im.sh.d; ++k) {
    TK_CHECK(S[k] != nullptr, kErrInvalidArg, "sketch factor is NULL");
    Sk[k] = S[k];
  }
  pl.bf16_factors = form == TK_FORM_BF16;
  if (form != TK_FORM_FP64) {
    std::array<const float*, kMaxD> S32{};
    for (int k = 0; k < im.sh.d; ++k) S32[k] = emit_to_f32(q, ar, Sk[k], size_t(im.sh.n[k]) * s);
    Blocks<float> b32 = blocks_f32(q, ar, im);
    plan_sketch<float>(q, pl, im.sh, b32, S32, int(s), out);
  } else {
    plan_sketch<double>(q, pl, im.sh, im.blocks, Sk, int(s), out);
  }
  finish_blob(ar, blob, st);
  if (ar.measuring()) return 0;
  q.run(st);
  TK_HIP(hipStreamSynchronize(st));
  return 0;
}

int do_rhosvd(const tk_block_sum* in, const tk_round_params* prm, const double* const* omega, tk_tucker* out,
              int32_t* s_out, Arena& ar, hipStream_t st) {
  TK_CHECK(prm != nullptr, kErrInvalidArg, "parameters are NULL");
  TK_CHECK(prm->rank_cap >= 1 && prm->oversample >= 0, kErrInvalidArg, "invalid rank cap / oversampling");
  TK_CHECK(prm->rank_cap + prm->oversample <= 64, kErrUnsupported, "rank_cap + oversample above 64");
  TK_CHECK(prm->eps >= 0.0, kErrInvalidArg, "eps must be >= 0");
  Blob blob;
  Planner pl(ar, blob);
  Seq q;
  Imported im = import_blocks(q, ar, in, prm->rank_cap, prm->oversample);
  const Shape& sh = im.sh;
  TK_CHECK(prm->force_s < 0 || (prm->force_s >= 1 && prm->force_s <= sh.sc()), kErrInvalidArg,
           "force_s outside [1, rank_cap + oversample]");
  RoundCfg cfg;
  cfg.eps = prm->eps;
  cfg.tau = prm->tau;
  cfg.force_s = prm->force_s;
  for (int k = 0; k < sh.d; ++k) {
    cfg.force_r[k] = prm->force_ranks[k];
    TK_CHECK(cfg.force_r[k] <= prm->rank_cap, kErrInvalidArg, "forced rank above rank_cap");
  }
  std::array<const double*, kMaxD> om{};
  TK_CHECK(omega != nullptr, kErrInvalidArg, "omega is NULL");
  for (int k = 0; k < sh.d; ++k) om[k] = omega[k];
  if (out) check_dims(out->d, out->n);
  check_form(prm->form);
  TT<double> o = alloc_tt<double>(ar, sh);
  int* s_dev = nullptr;
  pl.bf16_factors = prm->form == TK_FORM_BF16;
  if (prm->form != TK_FORM_FP64) {
    std::array<const float*, kMaxD> om32{};
    for (int k = 0; k < sh.d; ++k) om32[k] = emit_to_f32(q, ar, om[k], size_t(sh.n[k]) * sh.sc());
    Blocks<float> b32 = blocks_f32(q, ar, im);
    TT<float> o32 = alloc_tt<float>(ar, sh);
    s_dev = plan_roundsum<float>(q, pl, sh, b32, cfg, om32, o32, nullptr).s_dev;
    emit_cast_tt<float, double>(q, sh, o32, o);
  } else {
    s_dev = plan_roundsum<double>(q, pl, sh, im.blocks, cfg, om, o, nullptr).s_dev;
  }
  finish_blob(ar, blob, st);
  if (ar.measuring()) return 0;
  TK_CHECK(out != nullptr && out->d == sh.d, kErrInvalidArg, "output tensor missing or of wrong order");
  for (int k = 0; k < sh.d; ++k) TK_CHECK(out->n[k] == sh.n[k], kErrShape, "output mode size mismatch");
  q.run(st);
  if (s_out) {
    TK_HIP(hipMemcpyAsync(s_out, s_dev, sizeof(int), hipMemcpyDeviceToHost, st));
  }
  export_tt(sh, o, out, st);
  return 0;
}

int do_norm(const tk_block_sum* x, double* out, Arena& ar, hipStream_t st) {
  Blob blob;
  Planner pl(ar, blob);
  Seq q;
  Imported im = import_blocks(q, ar, x, 1, 0);
  TK_CHECK(im.sh.rc <= 64, kErrUnsupported, "exact norm: ranks above 64");
  double* n2 = ar.alloc<double>(1);
  plan_exact_norm2(q, pl, im.sh, im.blocks, n2);
  finish_blob(ar, blob, st);
  if (ar.measuring()) return 0;
  TK_CHECK(out != nullptr, kErrInvalidArg, "output pointer is NULL");
  q.run(st);
  double h = 0.0;
  TK_HIP(hipMemcpyAsync(&h, n2, sizeof(double), hipMemcpyDeviceToHost, st));
  TK_HIP(hipStreamSynchronize(st));
  *out = std::sqrt(std::max(h, 0.0));
  return 0;
}

// ---------------------------------------------------------------- solve
SolveCfg solve_cfg(const tk_sgmres_params* prm) {
  SolveCfg c;
  c.form = prm->form;
  c.tol = prm->tol;
  c.eta = prm->eta;
  c.maxiter = prm->maxiter;
  c.max_restarts = prm->max_restarts;
  c.k_trunc = prm->k_trunc;
  c.s = int(prm->s);
  c.eps_trunc = prm->eps_trunc;
  c.eps_min = prm->eps_min;
  c.tol_inner_floor = prm->tol_inner_floor;
  c.tikhonov = prm->tikhonov != 0;
  c.method = prm->method;
  return c;
}

void check_params(const tk_sgmres_params* prm) {
  TK_CHECK(prm != nullptr, kErrInvalidArg, "parameters are NULL");
  TK_CHECK(prm->form == TK_FORM_FP64 || prm->form == TK_FORM_FP32, kErrUnsupported, "unknown precision form");
  TK_CHECK(prm->tol > 0 && prm->eta > 0 && prm->eta <= 1, kErrInvalidArg, "tol > 0 and 0 < eta <= 1 required");
  TK_CHECK(prm->maxiter >= 1 && prm->maxiter <= 64, kErrUnsupported, "maxiter must be in [1, 64]");
  TK_CHECK(prm->max_restarts >= 0, kErrInvalidArg, "max_restarts must be >= 0");
  TK_CHECK(prm->k_trunc >= 1, kErrInvalidArg, "k_trunc must be >= 1");
  TK_CHECK(prm->rank_cap >= 1 && prm->oversample >= 0 && prm->rank_cap + prm->oversample <= 64, kErrUnsupported,
           "rank_cap + oversample must be in [1, 64]");
  TK_CHECK(prm->method == 0 || prm->method == 1, kErrInvalidArg, "method must be 0 (sGMRES) or 1 (GMRES)");
  TK_CHECK(prm->method == 1 || (prm->s >= prm->maxiter && prm->s <= 256), kErrUnsupported,
           "sketch size must be in [maxiter, 256]");
  TK_CHECK(prm->method == 0 || prm->precond_q == 0, kErrUnsupported,
           "the preconditioner runs with the sketched cycles only (method 0)");
  TK_CHECK(prm->precond_q >= 0 && prm->precond_q <= 400, kErrInvalidArg, "precond_q must be in [0, 400]");
  TK_CHECK(prm->precond_q == 0 || (prm->precond_V != nullptr && prm->precond_lambda != nullptr), kErrInvalidArg,
           "preconditioner eigenpairs missing");
  TK_CHECK(prm->tikhonov == 0 || prm->tikhonov == 1, kErrInvalidArg, "tikhonov must be 0 or 1");
}

PrecondT<double> precond_of(const tk_sgmres_params* prm, int d) {
  PrecondT<double> pc;
  pc.q = prm->precond_q;
  if (pc.q > 0)
    for (int k = 0; k < d; ++k) {
      pc.V[k] = prm->precond_V[k];
      pc.lam[k] = prm->precond_lambda[k];
    }
  return pc;
}

OpDev<double> op_dev(const tk_kron_op* op) {
  OpDev<double> o;
  o.nterms = op->nterms;
  o.alpha.assign(op->alpha, op->alpha + op->nterms);
  for (int i = 0; i < op->nterms * op->d; ++i) o.A.push_back(op->A[i]);
  return o;
}

void fill_info(const SolveInfo& si, tk_sgmres_info* info, int d) {
  if (!info) return;
  info->status = si.status;
  info->iters_total = si.iters;
  info->cycles = si.cycles;
  info->true_relres = si.true_relres;
  info->seconds = si.seconds;
  const int nh = int(si.hist_sketched.size());
  info->hist_len = std::min(nh, std::max(0, info->hist_cap));
  for (int i = 0; i < info->hist_len; ++i) {
    if (info->hist_sketched) info->hist_sketched[i] = si.hist_sketched[i];
    if (info->hist_ranks)
      for (int k = 0; k < TK_MAX_D; ++k) info->hist_ranks[i * TK_MAX_D + k] = k < d ? si.hist_ranks[i * d + k] : 0;
  }
  if (info->hist_true)
    for (int i = 0; i < std::min<int>(int(si.hist_true.size()), info->hist_cap); ++i) info->hist_true[i] = si.hist_true[i];
  if (info->hist_cycle_seconds)
    for (int i = 0; i < std::min<int>(int(si.hist_time.size()), info->hist_cap); ++i)
      info->hist_cycle_seconds[i] = si.hist_time[i];
  if (info->hist_lambda)
    for (int i = 0; i < info->hist_cap; ++i)
      info->hist_lambda[i] = i < int(si.hist_lambda.size()) ? si.hist_lambda[i] : 0.0;
}

int do_solve(const tk_kron_op* op, const tk_tucker* b, const tk_sgmres_params* prm, const double* const* S,
             const double* const* omega, tk_tucker* x, tk_sgmres_info* info, Arena& ar, hipStream_t st) {
  TK_CHECK(b != nullptr, kErrInvalidArg, "b is NULL");
  check_dims(b->d, b->n);
  check_op(op, b->d, b->n);
  check_tucker(b, "b", b->d, b->n);
  check_params(prm);
  TK_CHECK((S != nullptr || prm->method == 1) && omega != nullptr, kErrInvalidArg, "sketch matrices missing");
  const int d = b->d;
  int rc = prm->rank_cap;
  for (int k = 0; k < d; ++k) rc = std::max<int>(rc, int(b->r[k]));
  if (prm->x0) {
    check_tucker(prm->x0, "x0", d, b->n);
    for (int k = 0; k < d; ++k) rc = std::max<int>(rc, int(prm->x0->r[k]));
  }
  TK_CHECK(rc <= 64, kErrUnsupported, "ranks above 64 are not supported by the solver");
  Shape sh = shape_of(d, b->n, rc, prm->rank_cap, prm->oversample);
  Seq imp;
  TT<double> bi = alloc_tt<double>(ar, sh);
  emit_import<double>(imp, sh, *b, bi);
  TT<double> x0i;
  if (prm->x0) {
    x0i = alloc_tt<double>(ar, sh);
    emit_import<double>(imp, sh, *prm->x0, x0i);
  }
  std::array<const double*, kMaxD> Sk{}, Ok{};
  for (int k = 0; k < d; ++k) {
    Sk[k] = S ? S[k] : nullptr;
    Ok[k] = omega[k];
  }
  auto solver = make_solver(ar, sh, op_dev(op), bi, solve_cfg(prm), Sk, Ok, prm->x0 ? &x0i : nullptr, st,
                            precond_of(prm, d));
  FiniteCheck fin;
  fin.add_tt(sh, bi);
  if (prm->x0) fin.add_tt(sh, x0i);
  fin.add_inputs(sh, op, S, prm->s, omega, sh.sc(), prm);
  fin.alloc(ar);
  if (ar.measuring()) return 0;
  TK_CHECK(x != nullptr, kErrInvalidArg, "x is NULL");
  imp.run(st);
  fin.run(st);
  TT<double> xo;
  SolveInfo si;
  solver_run(*solver, xo, si, st);
  export_tt(sh, xo, x, st);
  fill_info(si, info, d);
  return si.status;
}

// ---------------------------------------------------------------- backward
int do_backward(const tk_kron_op* op, const tk_tucker* x, const tk_block_sum* xbar, const tk_sgmres_params* prm,
                const double* const* S, const double* const* omega, tk_tucker* lambda, double* dalpha,
                double* const* dA, tk_sgmres_info* info, Arena& ar, hipStream_t st) {
  TK_CHECK(x != nullptr, kErrInvalidArg, "x is NULL");
  check_dims(x->d, x->n);
  check_op(op, x->d, x->n);
  check_tucker(x, "x", x->d, x->n);
  TK_CHECK(prm == nullptr || prm->tikhonov == 0, kErrUnsupported,
           "the adjoint gradients assume an unregularised solve (tikhonov must be 0)");
  TK_CHECK(prm == nullptr || prm->method == 0, kErrUnsupported, "the adjoint solve runs sGMRES cycles (method 0)");
  check_params(prm);
  TK_CHECK(S != nullptr && omega != nullptr, kErrInvalidArg, "sketch matrices missing");
  const int d = x->d;
  int rc = prm->rank_cap;
  for (int k = 0; k < d; ++k) rc = std::max<int>(rc, int(x->r[k]));
  TK_CHECK(xbar != nullptr && xbar->nblocks >= 1, kErrInvalidArg, "cotangent is empty");
  for (int b = 0; b < xbar->nblocks; ++b) {
    check_tucker(&xbar->blocks[b], "xbar block", d, x->n);
    for (int k = 0; k < d; ++k) rc = std::max<int>(rc, int(xbar->blocks[b].r[k]));
  }
  TK_CHECK(rc <= 64, kErrUnsupported, "ranks above 64 are not supported by the solver");
  Shape sh = shape_of(d, x->n, rc, prm->rank_cap, prm->oversample);
  Blob blob;
  Planner pl(ar, blob);
  Seq imp, pre, post;
  // import x and the cotangent blocks, round the cotangent (FP64)
  TT<double> xi = alloc_tt<double>(ar, sh);
  emit_import<double>(imp, sh, *x, xi);
  FiniteCheck fin;
  fin.add_tt(sh, xi);
  Blocks<double> xb;
  for (int b = 0; b < xbar->nblocks; ++b) {
    TT<double> t = alloc_tt<double>(ar, sh);
    emit_import<double>(imp, sh, xbar->blocks[b], t);
    fin.add_tt(sh, t);
    TK_CHECK(std::isfinite(xbar->coef[b]), kErrNonFinite, "cotangent coefficient is not finite");
    xb.add(t, nullptr, xbar->coef[b]);
  }
  std::array<const double*, kMaxD> Sk{}, Ok{};
  for (int k = 0; k < d; ++k) {
    Sk[k] = S[k];
    Ok[k] = omega[k];
  }
  RoundCfg rc_cfg;
  rc_cfg.eps = 1e-2 * prm->tol;
  TT<double> xbr = alloc_tt<double>(ar, sh);
  plan_roundsum<double>(pre, pl, sh, xb, rc_cfg, Ok, xbr, nullptr);
  // adjoint solve L^T lambda = xbar
  SolveCfg scfg = solve_cfg(prm);
  scfg.transpose = true;
  OpDev<double> od = op_dev(op);
  auto solver = make_solver(ar, sh, od, xbr, scfg, Sk, Ok, nullptr, st, precond_of(prm, d));
  // gradient contractions, planned for every solution slot of the solver
  double* dal = ar.alloc<double>(op->nterms);
  Seq grad[3];
  for (int slot = 0; slot < 3; ++slot) {
    const TT<double> lam = solver_slot(*solver, slot);
    Seq& q = grad[slot];
    Blocks<double> lx = plan_apply<double>(q, pl, sh, od, xi, false);
    std::vector<double*> P;  // P[j*d+l] = U_lam,l^T A_j^(l) U_x,l
    plan_inner<double>(q, pl, sh, {lam}, lx, dal, -1.0, &P);
    if (dA == nullptr) continue;
    for (int j = 0; j < op->nterms; ++j)
      for (int k = 0; k < d; ++k) {
        if (op->A[j * d + k] == nullptr || dA[j * d + k] == nullptr) continue;
        int dims[kMaxD];
        for (int l = 0; l < d; ++l) dims[l] = sh.rc;
        const double* cur = xi.core;
        double* tA = ar.alloc<double>(sh.core_len());
        double* tB = ar.alloc<double>(sh.core_len());
        double* tgt = tA;
        for (int l = d - 1; l >= 0; --l) {
          if (l == k) continue;
          plan_ttm<double>(q, pl, d, dims, l, sh.rc, cur, P[j * d + l], sh.rc, false, tgt);
          cur = tgt;
          tgt = (tgt == tA) ? tB : tA;
        }
        double* Mid = ar.alloc<double>(size_t(sh.rc) * sh.rc);
        plan_unfold_gram<double>(q, pl, d, dims, k, lam.core, cur, Mid, sh.rc, 1.0);
        const int n = sh.n[k];
        double* tmp = ar.alloc<double>(size_t(n) * sh.rc);
        plan_gemm<double>(q, pl, false, true, n, sh.rc, sh.rc, xi.U[k], n, Mid, sh.rc, tmp, n, 1.0, 0.0);
        plan_gemm<double>(q, pl, false, true, n, n, sh.rc, tmp, n, lam.U[k], n, dA[j * d + k], n,
                          -op->alpha[j], 0.0);
      }
  }
  fin.add_inputs(sh, op, S, prm->s, omega, sh.sc(), prm);
  fin.alloc(ar);
  finish_blob(ar, blob, st);
  if (ar.measuring()) return 0;
  imp.run(st);
  fin.run(st);
  pre.run(st);
  TT<double> lam;
  SolveInfo si;
  solver_run(*solver, lam, si, st);
  grad[solver_slot_index(*solver)].run(st);
  if (dalpha) {
    TK_HIP(hipMemcpyAsync(dalpha, dal, sizeof(double) * op->nterms, hipMemcpyDeviceToHost, st));
  }
  TK_HIP(hipStreamSynchronize(st));
  if (lambda) export_tt(sh, lam, lambda, st);
  fill_info(si, info, d);
  return si.status;
}

// ---------------------------------------------------------------- multilinear Nystrom
void check_mln_rank(int r, int p) {
  TK_CHECK(r >= 1 && r <= 64, kErrUnsupported, "MLN target rank r must be in [1, 64]");
  TK_CHECK(p >= 0 && r + p <= 256, kErrUnsupported, "MLN: need p >= 0 and r + p <= 256");
}

std::array<const double*, kMaxD> psi_of(const double* const* Psi, int d) {
  TK_CHECK(Psi != nullptr, kErrInvalidArg, "Psi is NULL");
  std::array<const double*, kMaxD> a{};
  for (int k = 0; k < d; ++k) a[k] = Psi[k];
  return a;
}

int do_mln_sketch(const tk_block_sum* x, const double* const* Psi, int r, int p, double* core, double* const* F,
                  double* diag, Arena& ar, hipStream_t st) {
  check_mln_rank(r, p);
  Blob blob;
  Planner pl(ar, blob);
  Seq q;
  Imported im = import_blocks(q, ar, x, 1, 0);
  const int d = im.sh.d;
  const auto ps = psi_of(Psi, d);
  TK_CHECK(F != nullptr, kErrInvalidArg, "factor sketch outputs missing");
  MlnSk out;
  out.core = core;
  for (int k = 0; k < d; ++k) out.F[k] = F[k];
  plan_mln_sketch(q, pl, im.sh, im.blocks, ps, r, r + p, out, diag);
  finish_blob(ar, blob, st);
  if (ar.measuring()) return 0;
  TK_CHECK(core != nullptr, kErrInvalidArg, "core output is NULL");
  for (int k = 0; k < d; ++k) {
    TK_CHECK(ps[k] != nullptr, kErrInvalidArg, "Psi factor is NULL");
    TK_CHECK(F[k] != nullptr, kErrInvalidArg, "factor sketch output is NULL");
  }
  q.run(st);
  TK_HIP(hipStreamSynchronize(st));
  return 0;
}

int do_mln_recover(const double* core, const double* const* F, const double* const* Psi, int r, int p, int d,
                   const int64_t* n, tk_tucker* out, Arena& ar, hipStream_t st) {
  check_mln_rank(r, p);
  check_dims(d, n);
  TK_CHECK(F != nullptr, kErrInvalidArg, "factor sketches missing");
  const auto ps = psi_of(Psi, d);
  Shape sh = shape_of(d, n, r, r, p);
  Blob blob;
  Planner pl(ar, blob);
  Seq q;
  MlnSk sk;
  sk.core = const_cast<double*>(core);
  for (int k = 0; k < d; ++k) sk.F[k] = const_cast<double*>(F[k]);
  TT<double> o = alloc_tt<double>(ar, sh);
  plan_mln_recovery(q, pl, sh, sk, ps, r, r + p, o);
  finish_blob(ar, blob, st);
  if (ar.measuring()) return 0;
  TK_CHECK(core != nullptr && out != nullptr, kErrInvalidArg, "core or output is NULL");
  for (int k = 0; k < d; ++k) {
    TK_CHECK(ps[k] != nullptr && F[k] != nullptr, kErrInvalidArg, "Psi factor or factor sketch is NULL");
    TK_CHECK(out->rcap[k] >= r, kErrCapacity, "output rank capacity below r");
  }
  q.run(st);
  export_tt(sh, o, out, st);
  return 0;
}

void check_mln_params(const tk_mln_params* prm) {
  TK_CHECK(prm != nullptr, kErrInvalidArg, "parameters are NULL");
  check_mln_rank(prm->r, prm->p);
  TK_CHECK(prm->tol > 0 && prm->eta > 0 && prm->eta <= 1, kErrInvalidArg, "tol > 0 and 0 < eta <= 1 required");
  TK_CHECK(prm->maxiter >= 1 && prm->maxiter <= 64, kErrUnsupported, "maxiter must be in [1, 64]");
  TK_CHECK(prm->k_trunc >= 1, kErrInvalidArg, "k_trunc must be >= 1");
  TK_CHECK(prm->tikhonov == 0 || prm->tikhonov == 1, kErrInvalidArg, "tikhonov must be 0 or 1");
  if (prm->save_memory)
    TK_CHECK(prm->r_sol >= 1 && prm->r_sol <= prm->r && prm->p_sol >= 0 && prm->r_sol + prm->p_sol <= prm->r + prm->p,
             kErrInvalidArg, "save_memory needs 1 <= r_sol <= r and r_sol + p_sol <= r + p");
  TK_CHECK(prm->precond_q >= 0 && prm->precond_q <= 400, kErrInvalidArg, "precond_q must be in [0, 400]");
  TK_CHECK(prm->precond_q == 0 || (prm->precond_V != nullptr && prm->precond_lambda != nullptr), kErrInvalidArg,
           "preconditioner eigenpairs missing");
}

int do_mln_solve(const tk_kron_op* op, const tk_tucker* b, const tk_mln_params* prm, const double* const* Psi,
                 tk_tucker* x, tk_sgmres_info* info, Arena& ar, hipStream_t st) {
  TK_CHECK(b != nullptr, kErrInvalidArg, "b is NULL");
  check_dims(b->d, b->n);
  check_op(op, b->d, b->n);
  check_tucker(b, "b", b->d, b->n);
  check_mln_params(prm);
  const int d = b->d;
  for (int k = 0; k < d; ++k) TK_CHECK(b->r[k] <= prm->r, kErrCapacity, "rank of b above the target rank r");
  const auto ps = psi_of(Psi, d);
  Shape sh = shape_of(d, b->n, prm->r, prm->r, prm->p);
  Seq imp;
  TT<double> bi = alloc_tt<double>(ar, sh);
  emit_import<double>(imp, sh, *b, bi);
  MlnCfg cfg;
  cfg.r = prm->r;
  cfg.p = prm->p;
  cfg.tol = prm->tol;
  cfg.eta = prm->eta;
  cfg.maxiter = prm->maxiter;
  cfg.k_trunc = prm->k_trunc;
  cfg.bd_tol = prm->breakdown_tol > 0 ? prm->breakdown_tol : 1e-14;
  cfg.save_memory = prm->save_memory != 0;
  cfg.r_sol = prm->r_sol;
  cfg.p_sol = prm->p_sol;
  cfg.tikhonov = prm->tikhonov != 0;
  PrecondT<double> pc;
  pc.q = prm->precond_q;
  if (pc.q > 0)
    for (int k = 0; k < d; ++k) {
      pc.V[k] = prm->precond_V[k];
      pc.lam[k] = prm->precond_lambda[k];
      TK_CHECK(ar.measuring() || (pc.V[k] != nullptr && pc.lam[k] != nullptr), kErrInvalidArg,
               "preconditioner eigenpairs missing");
    }
  auto solver = make_mln_solver(ar, sh, op_dev(op), bi, cfg, ps, st, pc);
  if (ar.measuring()) return 0;
  TK_CHECK(x != nullptr, kErrInvalidArg, "x is NULL");
  for (int k = 0; k < d; ++k) TK_CHECK(ps[k] != nullptr, kErrInvalidArg, "Psi factor is NULL");
  imp.run(st);
  TT<double> xo;
  MlnInfo mi;
  mln_solver_run(*solver, xo, mi, st);
  export_tt(sh, xo, x, st);
  if (info) {
    SolveInfo si;
    si.status = mi.status;
    si.iters = mi.iters;
    si.cycles = 1;
    si.true_relres = mi.true_relres;
    si.seconds = mi.seconds;
    si.hist_sketched = mi.hist;
    si.hist_ranks = mi.ranks;
    si.hist_true = {mi.true_relres};
    si.hist_time = {mi.seconds};
    si.hist_lambda = mi.lambda;
    fill_info(si, info, d);
  }
  return mi.status;
}

// ---------------------------------------------------------------- Tikhonov
int do_tikhonov(const double* M, const double* b, int s, int k, double lam_fixed, double* y, double* out, Arena& ar,
                hipStream_t st) {
  TK_CHECK(k >= 1 && k <= 64, kErrUnsupported, "k must be in [1, 64]");
  TK_CHECK(s >= k && s <= 256, kErrUnsupported, "s must be in [k, 256]");
  TK_CHECK(std::isfinite(lam_fixed) || lam_fixed < 0, kErrInvalidArg, "lambda_fixed must be finite");
  LsState ls{};
  ls.Mcol = M;
  ls.bs = b;
  ls.Hv = ar.alloc<double>(size_t(s) * k);
  ls.tau = ar.alloc<double>(k);
  ls.R = ar.alloc<double>(size_t(k) * k);
  ls.qtb = ar.alloc<double>(s);
  ls.y = ar.alloc<double>(k);
  ls.res = ar.alloc<double>(k);
  ls.nrmM2 = ar.alloc<double>(1);
  ls.flags = ar.alloc<int>(4);
  ls.lam = ar.alloc<double>(k);
  double* bn2 = ar.alloc<double>(1);
  double* bn = ar.alloc<double>(1);
  ls.bs_norm = bn;
  const double** tab = ar.alloc<const double*>(1);
  if (ar.measuring()) return 0;
  TK_CHECK(M != nullptr && b != nullptr && y != nullptr && out != nullptr, kErrInvalidArg, "NULL argument");
  TK_HIP(hipMemcpyAsync(tab, &b, sizeof(b), hipMemcpyHostToDevice, st));
  dot_batched<double>(tab, tab, size_t(s), 1, 1.0, bn2, st);
  vec_sqrt(bn2, bn, 1, st);
  ls_init(ls, s, st);
  for (int j = 0; j < k; ++j) ls_add_column(ls, s, k, j, 0.0, 0.0, st);
  ls_tikhonov(ls, s, k, k - 1, 0.0, lam_fixed, st);
  TK_HIP(hipMemcpyAsync(y, ls.y, sizeof(double) * k, hipMemcpyDeviceToDevice, st));
  TK_HIP(hipMemcpyAsync(out, ls.lam + (k - 1), sizeof(double), hipMemcpyDeviceToDevice, st));
  TK_HIP(hipMemcpyAsync(out + 1, ls.res + (k - 1), sizeof(double), hipMemcpyDeviceToDevice, st));
  TK_HIP(hipStreamSynchronize(st));
  return 0;
}

}  // namespace
}  // namespace tk

// ====================================================================== extern "C"
using namespace tk;

static hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Static device scratch of the allocation-free sketch entry point.  Each GPU
// the library runs on holds its own copy of this array until the process
// ends.  In host code the array's name is only a host-side stand-in: kernels
// and copies get the device address that hipGetSymbolAddress returns for the
// current device, looked up once per device and kept.
namespace tk {
namespace {
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

void* noalloc_scratch() {
  int dev = -1;
  TK_HIP(hipGetDevice(&dev));
  TK_CHECK(dev >= 0 && dev < kMaxDevices, kErrUnsupported, "device index outside the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    TK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    TK_CHECK(p != nullptr, kErrHip, "hipGetSymbolAddress returned no address for the static scratch");
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}
}  // namespace
}  // namespace tk

extern "C" {

int tucker_apply_op(const tk_kron_op* op, const tk_tucker* x, int32_t transpose, int32_t form, double* const* AU,
                    void* ws, size_t ws_bytes, void* stream) {
  return guarded([&] {
    TK_CHECK(ws != nullptr || ws_bytes == 0, kErrInvalidArg, "workspace pointer is NULL");
    Arena ar(ws ? ws : reinterpret_cast<void*>(uintptr_t(1)), ws_bytes);
    return do_apply(op, x, transpose, form, AU, ar, as_stream(stream));
  });
}
int tucker_apply_op_workspace(const tk_kron_op* op, const tk_tucker* x, int32_t form, size_t* bytes) {
  return guarded([&] {
    Arena ar(nullptr, 0);
    double* dummy[TK_MAX_D * 64] = {};
    for (auto& p : dummy) p = reinterpret_cast<double*>(uintptr_t(0x1000));
    const int r = do_apply(op, x, 0, form, dummy, ar, nullptr);
    if (bytes) *bytes = ar.used();
    return r;
  });
}

int tucker_sketch(const tk_block_sum* x, const double* const* S, int64_t s, int32_t form, double* out, void* ws,
                  size_t ws_bytes, void* stream) {
  return guarded([&] {
    TK_CHECK(ws != nullptr, kErrInvalidArg, "workspace pointer is NULL");
    Arena ar(ws, ws_bytes);
    return do_sketch(x, S, s, form, out, ar, as_stream(stream));
  });
}
int tucker_sketch_noalloc(const tk_block_sum* x, const double* const* S, int64_t s, int32_t form, double* out,
                          void* stream) {
  return guarded([&] {
    {
      // size check first, so that an oversized call launches nothing
      Arena probe(nullptr, 0);
      do_sketch(x, S, s, form, out, probe, nullptr);
      TK_CHECK(probe.used() <= kNoAllocScratchBytes, kErrWorkspace,
               "tucker_sketch_noalloc: needs " + std::to_string(probe.used()) +
                   " bytes of scratch, above its static maximum of " + std::to_string(kNoAllocScratchBytes));
    }
    Arena ar(noalloc_scratch(), kNoAllocScratchBytes);
    return do_sketch(x, S, s, form, out, ar, as_stream(stream));
  });
}
int tucker_sketch_workspace(const tk_block_sum* x, int64_t s, int32_t form, size_t* bytes) {
  return guarded([&] {
    Arena ar(nullptr, 0);
    const double* S[TK_MAX_D] = {reinterpret_cast<const double*>(uintptr_t(0x1000)),
                                 reinterpret_cast<const double*>(uintptr_t(0x1000)),
                                 reinterpret_cast<const double*>(uintptr_t(0x1000)),
                                 reinterpret_cast<const double*>(uintptr_t(0x1000))};
    const int r = do_sketch(x, S, s, form, reinterpret_cast<double*>(uintptr_t(0x1000)), ar, nullptr);
    if (bytes) *bytes = ar.used();
    return r;
  });
}

int tucker_rhosvd(const tk_block_sum* in, const tk_round_params* prm, const double* const* omega, tk_tucker* out,
                  int32_t* s_out, void* ws, size_t ws_bytes, void* stream) {
  return guarded([&] {
    TK_CHECK(ws != nullptr, kErrInvalidArg, "workspace pointer is NULL");
    Arena ar(ws, ws_bytes);
    return do_rhosvd(in, prm, omega, out, s_out, ar, as_stream(stream));
  });
}
int tucker_rhosvd_workspace(const tk_block_sum* in, const tk_round_params* prm, size_t* bytes) {
  return guarded([&] {
    Arena ar(nullptr, 0);
    const double* om[TK_MAX_D] = {nullptr, nullptr, nullptr, nullptr};
    const int r = do_rhosvd(in, prm, om, nullptr, nullptr, ar, nullptr);
    if (bytes) *bytes = ar.used();
    return r;
  });
}

int tsgmres_solve(const tk_kron_op* op, const tk_tucker* b, const tk_sgmres_params* prm, const double* const* S,
                  const double* const* omega, tk_tucker* x, tk_sgmres_info* info, void* ws, size_t ws_bytes,
                  void* stream) {
  return guarded([&] {
    TK_CHECK(ws != nullptr, kErrInvalidArg, "workspace pointer is NULL");
    Arena ar(ws, ws_bytes);
    return do_solve(op, b, prm, S, omega, x, info, ar, as_stream(stream));
  });
}
int tsgmres_solve_workspace(const tk_kron_op* op, const tk_tucker* b, const tk_sgmres_params* prm, size_t* bytes) {
  return guarded([&] {
    Arena ar(nullptr, 0);
    const double* dummy[TK_MAX_D] = {nullptr, nullptr, nullptr, nullptr};
    const int r = do_solve(op, b, prm, dummy, dummy, nullptr, nullptr, ar, nullptr);
    if (bytes) *bytes = ar.used();
    return r;
  });
}

int tsgmres_backward(const tk_kron_op* op, const tk_tucker* x, const tk_block_sum* xbar,
                     const tk_sgmres_params* prm, const double* const* S, const double* const* omega,
                     tk_tucker* lambda, double* dalpha, double* const* dA, tk_sgmres_info* info, void* ws,
                     size_t ws_bytes, void* stream) {
  return guarded([&] {
    TK_CHECK(ws != nullptr, kErrInvalidArg, "workspace pointer is NULL");
    Arena ar(ws, ws_bytes);
    return do_backward(op, x, xbar, prm, S, omega, lambda, dalpha, dA, info, ar, as_stream(stream));
  });
}
int tsgmres_backward_workspace(const tk_kron_op* op, const tk_tucker* x, const tk_block_sum* xbar,
                               const tk_sgmres_params* prm, size_t* bytes) {
  return guarded([&] {
    Arena ar(nullptr, 0);
    const double* dummy[TK_MAX_D] = {nullptr, nullptr, nullptr, nullptr};
    std::vector<double*> dA(size_t(op ? op->nterms * op->d : 0), reinterpret_cast<double*>(uintptr_t(0x1000)));
    const int r = do_backward(op, x, xbar, prm, dummy, dummy, nullptr, nullptr, dA.data(), nullptr, ar, nullptr);
    if (bytes) *bytes = ar.used();
    return r;
  });
}

int tucker_norm(const tk_block_sum* x, double* out, void* ws, size_t ws_bytes, void* stream) {
  return guarded([&] {
    TK_CHECK(ws != nullptr, kErrInvalidArg, "workspace pointer is NULL");
    Arena ar(ws, ws_bytes);
    return do_norm(x, out, ar, as_stream(stream));
  });
}
int tucker_norm_workspace(const tk_block_sum* x, size_t* bytes) {
  return guarded([&] {
    Arena ar(nullptr, 0);
    const int r = do_norm(x, nullptr, ar, nullptr);
    if (bytes) *bytes = ar.used();
    return r;
  });
}

int tucker_mln_sketch(const tk_block_sum* x, const double* const* Psi, int32_t r, int32_t p, double* core,
                      double* const* F, double* diag, void* ws, size_t ws_bytes, void* stream) {
  return guarded([&] {
    TK_CHECK(ws != nullptr, kErrInvalidArg, "workspace pointer is NULL");
    Arena ar(ws, ws_bytes);
    return do_mln_sketch(x, Psi, r, p, core, F, diag, ar, as_stream(stream));
  });
}
int tucker_mln_sketch_workspace(const tk_block_sum* x, int32_t r, int32_t p, size_t* bytes) {
  return guarded([&] {
    Arena ar(nullptr, 0);
    // stand-in output addresses: planning only records them (a null core
    // would select a different contraction form)
    double* fake = reinterpret_cast<double*>(uintptr_t(0x1000));
    const double* dummy[TK_MAX_D] = {fake, fake, fake, fake};
    double* F[TK_MAX_D] = {fake, fake, fake, fake};
    const int rv = do_mln_sketch(x, dummy, r, p, fake, F, nullptr, ar, nullptr);
    if (bytes) *bytes = ar.used();
    return rv;
  });
}

int tucker_mln_recover(const double* core, const double* const* F, const double* const* Psi, int32_t r, int32_t p,
                       tk_tucker* out, void* ws, size_t ws_bytes, void* stream) {
  return guarded([&] {
    TK_CHECK(ws != nullptr, kErrInvalidArg, "workspace pointer is NULL");
    TK_CHECK(out != nullptr, kErrInvalidArg, "output is NULL");
    Arena ar(ws, ws_bytes);
    return do_mln_recover(core, F, Psi, r, p, out->d, out->n, out, ar, as_stream(stream));
  });
}
int tucker_mln_recover_workspace(int32_t d, const int64_t* n, int32_t r, int32_t p, size_t* bytes) {
  return guarded([&] {
    TK_CHECK(n != nullptr, kErrInvalidArg, "mode sizes are NULL");
    Arena ar(nullptr, 0);
    const double* dummy[TK_MAX_D] = {nullptr, nullptr, nullptr, nullptr};
    const int rv = do_mln_recover(nullptr, dummy, dummy, r, p, d, n, nullptr, ar, nullptr);
    if (bytes) *bytes = ar.used();
    return rv;
  });
}

int tsgmres_mln_solve(const tk_kron_op* op, const tk_tucker* b, const tk_mln_params* prm, const double* const* Psi,
                      tk_tucker* x, tk_sgmres_info* info, void* ws, size_t ws_bytes, void* stream) {
  return guarded([&] {
    TK_CHECK(ws != nullptr, kErrInvalidArg, "workspace pointer is NULL");
    Arena ar(ws, ws_bytes);
    return do_mln_solve(op, b, prm, Psi, x, info, ar, as_stream(stream));
  });
}
int tsgmres_mln_solve_workspace(const tk_kron_op* op, const tk_tucker* b, const tk_mln_params* prm, size_t* bytes) {
  return guarded([&] {
    Arena ar(nullptr, 0);
    const double* dummy[TK_MAX_D] = {nullptr, nullptr, nullptr, nullptr};
    const int rv = do_mln_solve(op, b, prm, dummy, nullptr, nullptr, ar, nullptr);
    if (bytes) *bytes = ar.used();
    return rv;
  });
}

int tsgmres_projected_tikhonov(const double* M, const double* b, int32_t s, int32_t k, double lambda_fixed,
                               double* y, double* out, void* ws, size_t ws_bytes, void* stream) {
  return guarded([&] {
    TK_CHECK(ws != nullptr, kErrInvalidArg, "workspace pointer is NULL");
    Arena ar(ws, ws_bytes);
    return do_tikhonov(M, b, s, k, lambda_fixed, y, out, ar, as_stream(stream));
  });
}
int tsgmres_projected_tikhonov_workspace(int32_t s, int32_t k, size_t* bytes) {
  return guarded([&] {
    Arena ar(nullptr, 0);
    const int rv = do_tikhonov(nullptr, nullptr, s, k, -1.0, nullptr, nullptr, ar, nullptr);
    if (bytes) *bytes = ar.used();
    return rv;
  });
}

int tk_kernel_timer(int32_t kind, int32_t enable) {
  return guarded([&] {
    TK_CHECK(kind >= 0 && kind < kKcCount, kErrInvalidArg, "unknown kernel class");
    timer_enable(kind, enable != 0);
    return 0;
  });
}
int tk_kernel_timer_read(int32_t kind, int64_t* launches, double* total_ms, double* flops, double* bytes) {
  return guarded([&] {
    TK_CHECK(kind >= 0 && kind < kKcCount && launches && total_ms, kErrInvalidArg, "bad timer query");
    double f = 0.0, b = 0.0;
    timer_read(kind, launches, total_ms, &f, &b);
    if (flops) *flops = f;
    if (bytes) *bytes = b;
    return 0;
  });
}

int tk_launch_count(int64_t* count) {
  return guarded([&] {
    TK_CHECK(count != nullptr, kErrInvalidArg, "count is NULL");
    *count = launch_count();
    return 0;
  });
}
int tk_launch_latency(int32_t n, void* stream, double* us_per_launch) {
  return guarded([&] {
    TK_CHECK(n >= 1 && n <= 1000000 && us_per_launch != nullptr, kErrInvalidArg, "bad launch-latency query");
    *us_per_launch = empty_launch_us(n, as_stream(stream));
    return 0;
  });
}

int tk_rank_cert_count(int64_t* tried, int64_t* passed) {
  return guarded([&] {
    TK_CHECK(tried != nullptr && passed != nullptr, kErrInvalidArg, "count pointer is NULL");
    rank_cert_counts(tried, passed);
    return 0;
  });
}

const char* tk_last_error(void) { return tk::last_error(); }
int tk_version(void) { return TK_ABI_VERSION; }

}  // extern "C"
