// Quartet-list build on the device: enumerate the unique quartets of a class,
// apply the screening estimate, and order them as the public list order
// requires (grouped by (l_a, l_b, l_c, l_d), decreasing primitive count inside
// a group, enumeration order among equals).  Host code (f12_host.cpp) computes
// the per-pair screening factors; everything per quartet runs here.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_select.hpp>
#include <rocprim/iterator/counting_iterator.hpp>

#include "f12_k2.h"

namespace f12 {

namespace {

// Pair indices (b, k) of candidate `idx` in enumeration order: b ascending,
// then k ascending, with k <= b when the bra-ket fold applies.
__device__ __forceinline__ void decode(const K2Params &P, uint64_t idx, int64_t &b, int64_t &k) {
  if (P.fold) {
    double x = floor((sqrt(8.0 * (double)idx + 1.0) - 1.0) * 0.5);
    int64_t bb = (int64_t)x;
    while (bb > 0 && (uint64_t)bb * (bb + 1) / 2 > idx) --bb;
    while ((uint64_t)(bb + 1) * (bb + 2) / 2 <= idx) ++bb;
    b = bb;
    k = (int64_t)(idx - (uint64_t)bb * (bb + 1) / 2);
  } else {
    b = (int64_t)(idx / (uint64_t)P.nk);
    k = (int64_t)(idx - (uint64_t)b * P.nk);
  }
}

struct KeepPred {
  K2Params P;
  __device__ bool operator()(uint64_t idx) const {
    if (!(P.tol > 0.0)) return true;
    int64_t b, k;
    decode(P, idx, b, k);
    double est = P.Sb[b] * P.Sk[k];
    if (est < P.tol && P.ngrow > 0) {
      const double dx = P.bmid[3 * b] - P.kmid[3 * k], dy = P.bmid[3 * b + 1] - P.kmid[3 * k + 1],
                   dz = P.bmid[3 * b + 2] - P.kmid[3 * k + 2];
      const double reff = sqrt(dx * dx + dy * dy + dz * dz) + 0.5 * (P.bab[b] + P.kab[k]);
      if (reff > 1.0) {
        double kap = 0.0;
        for (int t = 0; t < P.ngrow; ++t) kap += P.gc[t] * pow(reff, P.ga[t] - 1.0) * exp(P.gb[t] * reff);
        const double g = kap / P.kappa1;
        if (g > 1.0) est *= g;
      }
    }
    return est >= P.tol;
  }
};

// Sort key: group (one digit of radix LMAX+1 per angular momentum) above the
// complement of the primitive count, so that an ascending stable sort gives
// groups in order and decreasing primitive count inside a group.
constexpr int PRIM_BITS = 17;  // primitive counts up to 16^4 = 65536

__global__ void keys_kernel(K2Params P, const uint64_t *__restrict__ idx, int64_t n, uint32_t *__restrict__ key) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t b, k;
  decode(P, idx[i], b, k);
  const uint32_t grp = (uint32_t)((P.bcls[b] * (LMAX + 1) * (LMAX + 1)) + P.kcls[k]);
  const uint32_t np = (uint32_t)P.bnp[b] * (uint32_t)P.knp[k];
  key[i] = (grp << PRIM_BITS) | ((1u << PRIM_BITS) - 1u - np);
}

__global__ void finalize_kernel(K2Params P, const uint64_t *__restrict__ idx, const uint32_t *__restrict__ key,
                                int64_t n, int64_t *__restrict__ qb, int64_t *__restrict__ qk,
                                int64_t *__restrict__ nout, int64_t *__restrict__ nprim,
                                int64_t *__restrict__ start) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t b, k;
  decode(P, idx[i], b, k);
  qb[i] = b;
  qk[i] = k;
  nout[i] = (int64_t)P.bnc[b] * P.knc[k];
  nprim[i] = (int64_t)P.bnp[b] * P.knp[k];
  const uint32_t g = key[i] >> PRIM_BITS;
  if (i == 0 || (key[i - 1] >> PRIM_BITS) != g) start[g] = i;
}

template <typename F>
int with_temp(F f, hipStream_t st) {
  size_t bytes = 0;
  if (f(nullptr, bytes) != hipSuccess) return -1;
  void *tmp = nullptr;
  if (hipMalloc(&tmp, bytes ? bytes : 1) != hipSuccess) return -1;
  const hipError_t e = f(tmp, bytes);
  const hipError_t s = hipStreamSynchronize(st);
  (void)hipFree(tmp);
  return (e == hipSuccess && s == hipSuccess) ? 0 : -1;
}

}  // namespace

int k2_select(const K2Params &P, uint64_t ncand, uint64_t **d_idx, int64_t *nkept, hipStream_t st) {
  *d_idx = nullptr;
  *nkept = 0;
  uint64_t *out = nullptr, *cnt = nullptr;
  if (hipMalloc((void **)&out, (ncand ? ncand : 1) * sizeof(uint64_t)) != hipSuccess) return -1;
  if (hipMalloc((void **)&cnt, sizeof(uint64_t)) != hipSuccess) {
    (void)hipFree(out);
    return -1;
  }
  KeepPred pred{P};
  rocprim::counting_iterator<uint64_t> first(0);
  int rc = with_temp(
      [&](void *tmp, size_t &bytes) {
        return rocprim::select(tmp, bytes, first, out, cnt, (size_t)ncand, pred, st);
      },
      st);
  uint64_t h = 0;
  if (rc == 0 && hipMemcpy(&h, cnt, sizeof(uint64_t), hipMemcpyDeviceToHost) != hipSuccess) rc = -1;
  (void)hipFree(cnt);
  if (rc != 0) {
    (void)hipFree(out);
    return -1;
  }
  *d_idx = out;
  *nkept = (int64_t)h;
  return 0;
}

int k2_finalize(const K2Params &P, uint64_t *d_idx, int64_t n, int64_t *qb, int64_t *qk, int64_t *qoff,
                int64_t *qprim, int64_t *start, hipStream_t st) {
  if (n == 0) {
    int64_t z = 0;
    if (hipMemcpy(qoff, &z, 8, hipMemcpyHostToDevice) != hipSuccess) return -1;
    if (hipMemcpy(qprim, &z, 8, hipMemcpyHostToDevice) != hipSuccess) return -1;
    return 0;
  }
  uint32_t *key = nullptr, *key2 = nullptr;
  uint64_t *idx2 = nullptr;
  int64_t *sz = nullptr, *pr = nullptr;
  int rc = 0;
  if (hipMalloc((void **)&key, n * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc((void **)&key2, n * sizeof(uint32_t)) != hipSuccess ||
      hipMalloc((void **)&idx2, n * sizeof(uint64_t)) != hipSuccess ||
      hipMalloc((void **)&sz, n * sizeof(int64_t)) != hipSuccess ||
      hipMalloc((void **)&pr, n * sizeof(int64_t)) != hipSuccess)
    rc = -1;
  const unsigned nt = 256;
  const unsigned nblk = (unsigned)((n + nt - 1) / nt);
  if (rc == 0) {
    hipLaunchKernelGGL(keys_kernel, dim3(nblk), dim3(nt), 0, st, P, d_idx, n, key);
    if (hipGetLastError() != hipSuccess) rc = -1;
  }
  constexpr int NGRP = (LMAX + 1) * (LMAX + 1) * (LMAX + 1) * (LMAX + 1);
  static_assert(NGRP <= (1 << (32 - PRIM_BITS)), "group digit fits the sort key");
  int end_bit = PRIM_BITS;
  while ((1 << (end_bit - PRIM_BITS)) < NGRP) ++end_bit;
  if (rc == 0)
    rc = with_temp(
        [&](void *tmp, size_t &bytes) {
          return rocprim::radix_sort_pairs(tmp, bytes, key, key2, d_idx, idx2, (size_t)n, 0, end_bit, st);
        },
        st);
  if (rc == 0) {
    hipLaunchKernelGGL(finalize_kernel, dim3(nblk), dim3(nt), 0, st, P, idx2, key2, n, qb, qk, sz, pr, start);
    if (hipGetLastError() != hipSuccess) rc = -1;
  }
  // offsets: qoff[0] = 0, qoff[i + 1] = qoff[i] + size[i] (same for qprim)
  if (rc == 0) {
    int64_t z = 0;
    if (hipMemcpyAsync(qoff, &z, 8, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(qprim, &z, 8, hipMemcpyHostToDevice, st) != hipSuccess)
      rc = -1;
  }
  if (rc == 0)
    rc = with_temp(
        [&](void *tmp, size_t &bytes) {
          return rocprim::inclusive_scan(tmp, bytes, sz, qoff + 1, (size_t)n, rocprim::plus<int64_t>(), st);
        },
        st);
  if (rc == 0)
    rc = with_temp(
        [&](void *tmp, size_t &bytes) {
          return rocprim::inclusive_scan(tmp, bytes, pr, qprim + 1, (size_t)n, rocprim::plus<int64_t>(), st);
        },
        st);
  if (rc == 0 && hipStreamSynchronize(st) != hipSuccess) rc = -1;
  if (key) (void)hipFree(key);
  if (key2) (void)hipFree(key2);
  if (idx2) (void)hipFree(idx2);
  if (sz) (void)hipFree(sz);
  if (pr) (void)hipFree(pr);
  return rc;
}

}  // namespace f12
