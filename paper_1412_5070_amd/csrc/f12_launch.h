// Launchers of the HIP kernels (f12_kernels.hip), called by the host code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "f12_internal.h"

namespace f12 {

int launch_pair_prims(int64_t npp, const int32_t *pp_sa, const int32_t *pp_sb,
                      const int32_t *pp_ia, const int32_t *pp_ib, const int32_t *shell_first,
                      const int32_t *shell_center, const double *xyz, const double *exps,
                      const double *coefs, double *ea, double *eb, double *p, double *Px,
                      double *Py, double *Pz, double *cab, hipStream_t stream);

int launch_aux(const KernelDev *K, const PairsDev &bra, const PairsDev &ket, const int64_t *qb,
               const int64_t *qk, const int64_t *qprim, int64_t qa, int64_t nqc, int64_t p0,
               int64_t np, int L, double *A, hipStream_t stream, int variant);

int launch_contract(const PairsDev &bra, const PairsDev &ket, const int64_t *qb, const int64_t *qk,
                    const int64_t *qoff, const int64_t *qprim, int64_t qa, int64_t nqc, int64_t p0,
                    int64_t np, const double *A, int la, int lb, int lc, int ld, int i5,
                    double *out, int64_t out_base, hipStream_t stream, int64_t grid = 0,
                    int prec = 0, int gdir = -1);

// Device address of the current device's fault word (looked up once per
// device; nullptr if the lookup fails).  Kernels set the word to 1 when they
// produce a non-finite value.
int *fault_word();

// Radial derivatives A_n (n = 0..L) for explicit (p, q, R) triples (diagnostic path).
int launch_aux_points(const KernelDev *K, int64_t n, const double *p, const double *q,
                      const double *R, int L, int route, double *A, hipStream_t stream, int variant);

}  // namespace f12
