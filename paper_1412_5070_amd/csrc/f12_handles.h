// Opaque handles of the C ABI and small host helpers, shared by the host
// translation units of the library (f12_host.cpp, f12_batch.cpp).  Not part
// of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <vector>

#include "../../include/f12int.h"
#include "f12_internal.h"

namespace f12 {

template <typename T>
struct DevBuf {
  T *ptr = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    n = 0;
  }
  bool alloc(size_t count) {
    release();
    if (count == 0) count = 1;
    if (hipMalloc((void **)&ptr, count * sizeof(T)) != hipSuccess) {
      ptr = nullptr;
      return false;
    }
    n = count;
    return true;
  }
  bool upload(const std::vector<T> &v) {
    if (!alloc(v.size())) return false;
    if (v.empty()) return true;
    return hipMemcpy(ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) == hipSuccess;
  }
};

inline int ncart_host(int l) { return (l + 1) * (l + 2) / 2; }

// One term c r^alpha e^{b r - g r^2}; the coefficient is the double-double
// c + clo (the expansion keeps it to about 32 digits, so that the
// singular parts of terms with negative powers cancel to that precision).
struct HostTerm {
  double c, alpha, b, g;
  double clo = 0.0;
};

struct Bin {
  int la, lb, lc, ld;
  int64_t q0, nq;
};

}  // namespace f12

// ---------------------------------------------------------------- handles ---
using f12::Bin;
using f12::DevBuf;
using f12::HostTerm;
using f12::KernelDev;
using f12::PairsDev;
using f12::LTOT_MAX;

struct f12_basis {
  int32_t ncenter = 0, nshell = 0, nprim = 0;
  std::vector<double> xyz, exps, coefs;
  std::vector<f12_shell> shells;
};

struct f12_pairs {
  int32_t ordered = 0, nshell = 0;
  int64_t nsp = 0, npp = 0;
  // host copies used for enumeration
  std::vector<int32_t> sa, sb, la, lb, ka, kb;
  std::vector<int64_t> pp_off;
  // per shell pair, for the screening estimate: midpoint of A and B, |A - B|,
  // smallest exponent sum a + b and largest exponent over the primitive pairs
  std::vector<double> midx, midy, midz, ablen, pmin, emax;
  DevBuf<int32_t> d_sa, d_sb, d_la, d_lb, d_ka, d_kb;
  DevBuf<int64_t> d_pp_off;
  DevBuf<double> d_ABx, d_ABy, d_ABz;
  DevBuf<double> d_ea, d_eb, d_p, d_Px, d_Py, d_Pz, d_cab;
  PairsDev dev() const {
    PairsDev d;
    d.nsp = nsp;
    d.npp = npp;
    d.nshell = nshell;
    d.ordered = ordered;
    d.sa = d_sa.ptr;
    d.sb = d_sb.ptr;
    d.la = d_la.ptr;
    d.lb = d_lb.ptr;
    d.ka = d_ka.ptr;
    d.kb = d_kb.ptr;
    d.pp_off = d_pp_off.ptr;
    d.ABx = d_ABx.ptr;
    d.ABy = d_ABy.ptr;
    d.ABz = d_ABz.ptr;
    d.ea = d_ea.ptr;
    d.eb = d_eb.ptr;
    d.p = d_p.ptr;
    d.Px = d_Px.ptr;
    d.Py = d_Py.ptr;
    d.Pz = d_Pz.ptr;
    d.cab = d_cab.ptr;
    return d;
  }
};

struct f12_kernel {
  int32_t cls = 0;
  std::vector<HostTerm> terms;
  KernelDev host_desc;  // with device pointers filled in
  DevBuf<KernelDev> d_desc;
  std::vector<std::unique_ptr<DevBuf<double>>> tables;
  DevBuf<double> d_phi;
  int maxL = LTOT_MAX;
};

struct f12_quartets {
  const f12_pairs *bra = nullptr, *ket = nullptr;
  int32_t cls = 0;
  int64_t nq = 0, nout = 0, nprim = 0;
  std::vector<int64_t> qb, qk, qoff, qprim;  // processing (= public) order
  std::vector<Bin> bins;
  DevBuf<int64_t> d_qb, d_qk, d_qoff, d_qprim;
  DevBuf<double> d_A;
  int64_t a_cap_prims = 0;
  int64_t max_qprim = 0;  // largest primitive-quartet count of one quartet
  // range whose radial derivatives sit in d_A after f12_eval_stage(stage 1)
  int64_t stage_qa = -1, stage_qe = -1;
  const f12_kernel *stage_k = nullptr;
};

