// Grouped, batched GEMM on CDNA4 matrix cores.
//
// One launch computes, for every group g,
//     C_g = beta * C_g + sum_{t in terms(g)} alpha_t * op(A_t) * op(B_t)
// with column-major operands of uniform shape M x N x K.  alpha_t is
// scale_t * (*c1_t) * (*c2_t) * (*c3_t) with optional device scalars, so
// device-resident coefficients (inner products, least-squares solutions,
// block weights) scale terms without a host round trip.  Term and group
// tables live in device memory and are built once per plan.
#pragma once

#include "common.hpp"

namespace tk {

template <typename T>
struct GemmTerm {
  const T* A;
  const T* B;
  const double* c1;  // optional device scalar (nullptr = 1)
  const double* c2;  // optional device scalar (nullptr = 1)
  const double* c3;  // optional device scalar (nullptr = 1)
  double scale;
};

template <typename T>
struct GemmGroup {
  T* C;
  int t0, t1;  // term range [t0, t1)
};

// Launch descriptor: uniform dims/transposes, device tables.
template <typename T>
struct GemmLaunch {
  bool ta = false, tb = false;
  int M = 0, N = 0, K = 0, lda = 0, ldb = 0, ldc = 0;
  const GemmTerm<T>* terms = nullptr;   // device
  const GemmGroup<T>* groups = nullptr; // device
  int ngroups = 0;
  double beta = 0.0;
  int splits = 1;          // split of the (term x K-slab) space (>1 uses `partial` + a reduction pass)
  T* partial = nullptr;    // ngroups * splits * M * N
  int max_terms = 1 << 30; // clamp every group to its first max_terms terms
  bool bf16 = false;       // FP32 storage: round the operands to bfloat16, BF16 matrix cores, FP32 accumulation
  bool defer_reduce = false;  // splits > 1: leave the partials for the consumer to sum (C is not written)
  double flops = 0.0;      // algorithmic flops of this launch (for the kernel timer)
};

template <typename T>
void gemm_run(const GemmLaunch<T>& g, hipStream_t st);

// Host-side builder: collects the tables of many launches, uploads once.
template <typename T>
struct GemmTables {
  std::vector<GemmTerm<T>> terms;
  std::vector<GemmGroup<T>> groups;
};

}  // namespace tk
