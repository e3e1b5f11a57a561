// Device quartet-list build (f12_k2.hip): parameters and launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "f12_internal.h"

namespace f12 {

constexpr int K2_MAX_GROW = 16;  // undamped growing kernel terms in the estimate

// Per-pair tables (device pointers) and the screening estimate's parameters.
struct K2Params {
  int64_t nb, nk;  // bra and ket shell pairs
  int32_t fold;    // 1: only k <= b (8-fold classes), 0: every (b, k)
  double tol;      // keep when the estimate reaches tol; tol <= 0 keeps all
  const double *Sb, *Sk;      // Q_ab times the pair's extent factor
  const double *bmid, *kmid;  // midpoints (x, y, z) of A and B
  const double *bab, *kab;    // |A - B|
  const int32_t *bcls, *kcls; // l_a (LMAX + 1) + l_b
  const int32_t *bnp, *knp;   // primitive pairs of the shell pair
  const int32_t *bnc, *knc;   // Cartesian components n_a n_b
  int32_t ngrow;              // growing terms |c| r^(alpha - 1) e^{b r}
  double gc[K2_MAX_GROW], ga[K2_MAX_GROW], gb[K2_MAX_GROW];
  double kappa1;              // the growth sum at r = 1
};

// Candidate indices (enumeration order) of the quartets the estimate keeps;
// *d_idx is allocated here (hipMalloc) and freed by the caller.
int k2_select(const K2Params &P, uint64_t ncand, uint64_t **d_idx, int64_t *nkept, hipStream_t st);
// Orders the kept candidates (group, then decreasing primitive count, stable)
// and writes qb, qk (n), qoff, qprim (n + 1) and start[group] (first index of
// each non-empty group; other entries untouched).  Synchronous.
int k2_finalize(const K2Params &P, uint64_t *d_idx, int64_t n, int64_t *qb, int64_t *qk, int64_t *qoff,
                int64_t *qprim, int64_t *start, hipStream_t st);

}  // namespace f12
