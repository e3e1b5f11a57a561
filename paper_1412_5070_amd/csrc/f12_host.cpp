// Host side of the library: C ABI, term tables of the kernels k_i, the
// auxiliary-function tables, shell pairs, quartet lists and evaluation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "../../include/f12int.h"
#include "f12_dd.h"
#include "f12_internal.h"
#include "f12_k2.h"
#include "f12_launch.h"

using namespace f12;

#include "f12_handles.h"

// ============================================================================
// error strings
// ============================================================================
extern "C" const char *f12_strerror(int32_t s) {
  switch (s) {
    case F12_OK: return "ok";
    case F12_EINVAL: return "invalid argument";
    case F12_EPARAM: return "factor parameters rejected or unsupported";
    case F12_ELMAX: return "angular momentum above the supported maximum";
    case F12_ENOMEM: return "out of memory";
    case F12_EDEVICE: return "HIP runtime error";
    case F12_EBUFSIZE: return "output buffer too small";
    case F12_ENONFINITE: return "a kernel produced a non-finite value";
    default: return "unknown status";
  }
}

extern "C" int f12_stream_status(void *stream) {
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return F12_EDEVICE;
  if (hipGetLastError() != hipSuccess) return F12_EDEVICE;
  int *fw = fault_word();
  if (!fw) return F12_EDEVICE;
  int v = 0;
  if (hipMemcpy(&v, fw, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return F12_EDEVICE;
  if (v != 0) {
    const int zero = 0;
    if (hipMemcpy(fw, &zero, sizeof(int), hipMemcpyHostToDevice) != hipSuccess) return F12_EDEVICE;
    return F12_ENONFINITE;
  }
  return F12_OK;
}

// ============================================================================
// basis
// ============================================================================
extern "C" int f12_basis_create(int32_t ncenter, const double *xyz, int32_t nshell,
                                const f12_shell *shells, int32_t nprim_total, const double *exps,
                                const double *coefs, f12_basis **out) {
  if (!out || ncenter <= 0 || nshell <= 0 || nprim_total <= 0 || !xyz || !shells || !exps ||
      !coefs)
    return F12_EINVAL;
  *out = nullptr;
  for (int i = 0; i < 3 * ncenter; ++i)
    if (!std::isfinite(xyz[i])) return F12_EINVAL;
  for (int i = 0; i < nprim_total; ++i)
    if (!(exps[i] > 0.0) || !std::isfinite(exps[i]) || !std::isfinite(coefs[i])) return F12_EINVAL;
  for (int s = 0; s < nshell; ++s) {
    const f12_shell &sh = shells[s];
    if (sh.l < 0) return F12_EINVAL;
    if (sh.l > F12_LMAX) return F12_ELMAX;
    if (sh.nprim <= 0 || sh.nprim > F12_MAX_KPRIM) return F12_EINVAL;
    if (sh.center < 0 || sh.center >= ncenter) return F12_EINVAL;
    if (sh.first_prim < 0 || sh.first_prim + sh.nprim > nprim_total) return F12_EINVAL;
  }
  f12_basis *b = new (std::nothrow) f12_basis;
  if (!b) return F12_ENOMEM;
  b->ncenter = ncenter;
  b->nshell = nshell;
  b->nprim = nprim_total;
  b->xyz.assign(xyz, xyz + 3 * ncenter);
  b->shells.assign(shells, shells + nshell);
  b->exps.assign(exps, exps + nprim_total);
  b->coefs.assign(coefs, coefs + nprim_total);
  *out = b;
  return F12_OK;
}

extern "C" void f12_basis_destroy(f12_basis *b) { delete b; }

// ============================================================================
// pairs
// ============================================================================
extern "C" int f12_pairs_build(const f12_basis *basis, int32_t ordered, void *stream,
                               f12_pairs **out) {
  if (!basis || !out || (ordered != 0 && ordered != 1)) return F12_EINVAL;
  *out = nullptr;
  std::unique_ptr<f12_pairs> P(new (std::nothrow) f12_pairs);
  if (!P) return F12_ENOMEM;
  const int ns = basis->nshell;
  P->ordered = ordered;
  P->nshell = ns;
  std::vector<double> ABx, ABy, ABz;
  std::vector<int32_t> pp_sa, pp_sb, pp_ia, pp_ib;
  int64_t npp = 0;
  for (int i = 0; i < ns; ++i) {
    int jmax = ordered ? ns - 1 : i;
    for (int j = 0; j <= jmax; ++j) {
      const f12_shell &a = basis->shells[i], &b = basis->shells[j];
      P->sa.push_back(i);
      P->sb.push_back(j);
      P->la.push_back(a.l);
      P->lb.push_back(b.l);
      P->ka.push_back(a.nprim);
      P->kb.push_back(b.nprim);
      P->pp_off.push_back(npp);
      const double *A = &basis->xyz[3 * a.center];
      const double *B = &basis->xyz[3 * b.center];
      ABx.push_back(A[0] - B[0]);
      ABy.push_back(A[1] - B[1]);
      ABz.push_back(A[2] - B[2]);
      P->midx.push_back(0.5 * (A[0] + B[0]));
      P->midy.push_back(0.5 * (A[1] + B[1]));
      P->midz.push_back(0.5 * (A[2] + B[2]));
      P->ablen.push_back(std::sqrt((A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) +
                                   (A[2] - B[2]) * (A[2] - B[2])));
      {
        double amin = 1e300, bmin = 1e300, em = 0.0;
        for (int ia = 0; ia < a.nprim; ++ia) {
          amin = std::min(amin, basis->exps[a.first_prim + ia]);
          em = std::max(em, basis->exps[a.first_prim + ia]);
        }
        for (int ib = 0; ib < b.nprim; ++ib) {
          bmin = std::min(bmin, basis->exps[b.first_prim + ib]);
          em = std::max(em, basis->exps[b.first_prim + ib]);
        }
        P->pmin.push_back(amin + bmin);
        P->emax.push_back(em);
      }
      for (int ia = 0; ia < a.nprim; ++ia)
        for (int ib = 0; ib < b.nprim; ++ib) {
          pp_sa.push_back(i);
          pp_sb.push_back(j);
          pp_ia.push_back(ia);
          pp_ib.push_back(ib);
          ++npp;
        }
    }
  }
  P->nsp = (int64_t)P->sa.size();
  P->npp = npp;
  std::vector<int32_t> first(ns), center(ns);
  for (int s = 0; s < ns; ++s) {
    first[s] = basis->shells[s].first_prim;
    center[s] = basis->shells[s].center;
  }
  DevBuf<int32_t> d_ppsa, d_ppsb, d_ppia, d_ppib, d_first, d_center;
  DevBuf<double> d_xyz, d_exps, d_coefs;
  bool ok = P->d_sa.upload(P->sa) && P->d_sb.upload(P->sb) && P->d_la.upload(P->la) &&
            P->d_lb.upload(P->lb) && P->d_ka.upload(P->ka) && P->d_kb.upload(P->kb) &&
            P->d_pp_off.upload(P->pp_off) && P->d_ABx.upload(ABx) && P->d_ABy.upload(ABy) &&
            P->d_ABz.upload(ABz) && d_ppsa.upload(pp_sa) && d_ppsb.upload(pp_sb) &&
            d_ppia.upload(pp_ia) && d_ppib.upload(pp_ib) && d_first.upload(first) &&
            d_center.upload(center) && d_xyz.upload(basis->xyz) && d_exps.upload(basis->exps) &&
            d_coefs.upload(basis->coefs) && P->d_ea.alloc(npp) && P->d_eb.alloc(npp) &&
            P->d_p.alloc(npp) && P->d_Px.alloc(npp) && P->d_Py.alloc(npp) &&
            P->d_Pz.alloc(npp) && P->d_cab.alloc(npp);
  if (!ok) return F12_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  if (launch_pair_prims(npp, d_ppsa.ptr, d_ppsb.ptr, d_ppia.ptr, d_ppib.ptr, d_first.ptr,
                        d_center.ptr, d_xyz.ptr, d_exps.ptr, d_coefs.ptr, P->d_ea.ptr,
                        P->d_eb.ptr, P->d_p.ptr, P->d_Px.ptr, P->d_Py.ptr, P->d_Pz.ptr,
                        P->d_cab.ptr, st) != 0)
    return F12_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return F12_EDEVICE;
  *out = P.release();
  return F12_OK;
}

extern "C" int f12_pairs_count(const f12_pairs *p, int64_t *nsp, int64_t *npp) {
  if (!p) return F12_EINVAL;
  if (nsp) *nsp = p->nsp;
  if (npp) *npp = p->npp;
  return F12_OK;
}

extern "C" void f12_pairs_destroy(f12_pairs *p) { delete p; }

// ============================================================================
// kernel term tables (Eq. (rs12), Eq. (ttdamp), Eqs. (k1)-(k6))
// ============================================================================
namespace {

using Expr = std::vector<HostTerm>;  // sum c r^alpha exp(b r - g r^2)

bool same(double x, double y) { return std::fabs(x - y) <= 1e-12 * (1.0 + std::fabs(x) + std::fabs(y)); }

inline dd tc(const HostTerm &t) { return dd{t.c, t.clo}; }
inline HostTerm term(dd c, double alpha, double b, double g) {
  HostTerm t{c.hi, alpha, b, g};
  t.clo = c.lo;
  return t;
}

void add_term(Expr &e, HostTerm t) {
  if (t.c == 0.0 && t.clo == 0.0) return;
  for (auto &u : e)
    if (same(u.alpha, t.alpha) && same(u.b, t.b) && same(u.g, t.g)) {
      const dd s = dd_add(tc(u), tc(t));
      u.c = s.hi;
      u.clo = s.lo;
      return;
    }
  e.push_back(t);
}

Expr mul(const Expr &x, const Expr &y) {
  Expr r;
  for (auto &a : x)
    for (auto &b : y) add_term(r, term(dd_mul(tc(a), tc(b)), a.alpha + b.alpha, a.b + b.b, a.g + b.g));
  return r;
}

// d/dr [c r^a e^{b r - g r^2}] = c (a r^{a-1} + b r^a - 2 g r^{a+1}) e^{...}
Expr deriv(const Expr &x) {
  Expr r;
  for (auto &t : x) {
    add_term(r, term(dd_mul(tc(t), t.alpha), t.alpha - 1.0, t.b, t.g));
    add_term(r, term(dd_mul(tc(t), t.b), t.alpha, t.b, t.g));
    add_term(r, term(dd_mul(tc(t), -2.0 * t.g), t.alpha + 1.0, t.b, t.g));
  }
  return r;
}

Expr shift_alpha(const Expr &x, double d) {
  Expr r = x;
  for (auto &t : r) t.alpha += d;
  return r;
}

// f(r) = (1 + r/2) e^{-mu r^2} + c0 r^rho e^{B r} - c0 sum_{k<=n} mu^k/k! r^{rho+2k} e^{B r - mu r^2}
Expr factor_expr(const f12_factor &f) {
  Expr e;
  add_term(e, {1.0, 0.0, 0.0, f.mu});
  add_term(e, {0.5, 1.0, 0.0, f.mu});
  if (f.c0 != 0.0) {
    add_term(e, {f.c0, f.rho, f.B, 0.0});
    dd mk = dd_make(1.0);  // mu^k / k!
    for (int k = 0; k <= f.n; ++k) {
      if (k > 0) mk = dd_div(dd_mul(mk, f.mu), (double)k);
      add_term(e, term(dd_mul(mk, -f.c0), f.rho + 2.0 * k, f.B, f.mu));
    }
  }
  return e;
}

int validate_factor(const f12_factor *f) {
  if (!f) return F12_EINVAL;
  if (!std::isfinite(f->c0) || !std::isfinite(f->rho) || !std::isfinite(f->B) ||
      !std::isfinite(f->mu))
    return F12_EPARAM;
  if (!(f->mu > 0.0)) return F12_EPARAM;
  if (f->n < 0 || f->n > 8 || f->reserved != 0) return F12_EPARAM;
  if (f->rho < -2.0 && !(f->n > -f->rho / 2.0 - 1.0)) return F12_EPARAM;
  return F12_OK;
}

// --------------------------------------------------------------- DD Gamma ---
// ln Gamma(z) by Stirling's series for z >= 40 (DD), shifted down by recurrence.
dd dd_lgamma_large(dd z) {
  // Bernoulli numbers B_2k as exact fractions
  static const double num[] = {1, -1, 1, -1, 5, -691, 7, -3617, 43867, -174611, 854513, -236364091};
  static const double den[] = {6, 30, 42, 30, 66, 2730, 6, 510, 798, 330, 138, 2730};
  dd lz = dd_log(z);
  dd r = dd_sub(dd_mul(dd_add(z, -0.5), lz), z);
  // 0.5 ln(2 pi)
  r = dd_add(r, dd{9.189385332046728e-01, -3.8782941580672414e-17});
  dd zi = dd_div(dd_make(1.0), z);
  dd z2 = dd_mul(zi, zi);
  dd pw = zi;
  for (int k = 1; k <= 12; ++k) {
    dd bk = dd_div(dd_make(num[k - 1]), den[k - 1]);
    dd term = dd_div(dd_mul(bk, pw), (double)(2 * k * (2 * k - 1)));
    r = dd_add(r, term);
    pw = dd_mul(pw, z2);
  }
  return r;
}

// Gamma(x) in DD for x > 0 (x given as a binary64 number).
dd dd_gamma(double x) {
  int N = 0;
  dd z = dd_make(x);
  dd prod = dd_make(1.0);
  while (z.hi < 40.0) {
    prod = dd_mul(prod, z);
    z = dd_add(z, 1.0);
    ++N;
  }
  dd lg = dd_lgamma_large(z);
  return dd_div(dd_exp(lg), prod);
}

// Gamma(x) for x possibly <= 0 (non-integer): reflection by the recurrence upward.
dd dd_gamma_any(double x) {
  if (x > 0) return dd_gamma(x);
  // Gamma(x) = Gamma(x + n) / (x (x+1) ... (x+n-1)), x + n > 0
  dd prod = dd_make(1.0);
  double y = x;
  while (y <= 0.0) {
    prod = dd_mul(prod, dd_make(y));
    y += 1.0;
  }
  return dd_div(dd_gamma(y), prod);
}

// ---------------------------------------------------------- W-table builder ---
// W_a(x) = R int_0^inf t^a exp(-(t-x)^2) dt for a = a0 + m, m in [m_lo, m_hi].
//
// Start values at the two regular orders a0 and a0+1 (a0 in [0,1)):
//  * x >= 0: the confluent-hypergeometric form of S(alpha, beta, gamma) valid
//    for either sign of beta (the Tricomi-U form of Eq. (suabz) holds only for
//    beta <= 0): with z = x^2, a' = (a+1)/2,
//      W_a(x) = exp(-z)/2 [Gamma(a') M(a',1/2,z) + 2x Gamma(a'+1/2) M(a'+1/2,3/2,z)],
//    whose series has positive terms (Eq. (msmallz)).
//  * x < 0: double-exponential quadrature of the (regular) integral.
// Ladders by the integration-by-parts relation (Eq. (Srec1) with gamma = 1):
//      W_{a+1} = x W_a + (a/2) W_{a-1}
// run in the direction in which W is the dominant solution (upward for x > 0,
// downward in a for x < 0 above a0 and for |x| small below a0); elsewhere
// Miller's method: a trial solution started far away in the stable direction
// and normalised at a0 (the paper's treatment of T_s for small gamma/beta^2).
typedef long double ld;

ld M_series_scaled(ld a, ld b, ld z) {
  // exp(-z) M(a, b, z), positive terms
  ld term = expl(-z);
  ld sum = term;
  for (int n = 1; n < 20000; ++n) {
    term *= (a + n - 1) * z / ((b + n - 1) * n);
    sum += term;
    if (n > z && term < 1e-24L * sum) break;
  }
  return sum;
}

ld W_pos(ld a, ld x) {
  ld ap = (a + 1) * 0.5L;
  ld z = x * x;
  ld g1 = tgammal(ap), g2 = tgammal(ap + 0.5L);
  return 0.5L * (g1 * M_series_scaled(ap, 0.5L, z) + 2 * x * g2 * M_series_scaled(ap + 0.5L, 1.5L, z));
}

ld W_neg_quad(ld a, ld x) {
  // exp-sinh: t = exp(pi/2 sinh s)
  const ld h = 1.0L / 256;
  const ld pi2 = 1.5707963267948966192313216916397514L;
  ld sum = 0;
  for (int k = -1536; k <= 1536; ++k) {
    ld s = k * h;
    ld t = expl(pi2 * sinhl(s));
    if (t == 0 || !std::isfinite((double)t)) continue;
    ld w = t * pi2 * coshl(s);
    ld v = powl(t, a) * expl(-(t - x) * (t - x)) * w;
    if (std::isfinite((double)v)) sum += v;
  }
  return sum * h;
}

// W_a(x) = exp(-x^2)/2 sum_k Gamma((a+k+1)/2) (2x)^k/k! (Phi_a(y) expanded
// about y = 0 with Phi_a^(k)(0) = Phi_{a+k}(0) = Gamma((a+k+1)/2)/2), in DD.
double w_phi_series_dd(double a, double x) {
  const dd y2 = dd_mul(dd_make(2.0 * x), 2.0 * x);  // (2x)^2
  dd t0 = dd_gamma_any(0.5 * (a + 1.0));              // k = 0 term
  dd t1 = dd_mul(dd_gamma_any(0.5 * (a + 2.0)), 2.0 * x);  // k = 1 term
  dd sum = dd_add(t0, t1);
  const int kmin = (int)(4.0 * x * x) + 40;
  for (int k = 0; k < 4000; k += 2) {
    // t_{k+2} = t_k (a+k+1)/2 (2x)^2 / ((k+1)(k+2))
    t0 = dd_div(dd_mul(dd_mul(t0, 0.5 * (a + k + 1.0)), y2), (double)(k + 1) * (k + 2));
    t1 = dd_div(dd_mul(dd_mul(t1, 0.5 * (a + k + 2.0)), y2), (double)(k + 2) * (k + 3));
    sum = dd_add(sum, dd_add(t0, t1));
    if (k > kmin && std::fabs(t0.hi) + std::fabs(t1.hi) < 1e-34 * std::fabs(sum.hi)) break;
  }
  dd e = dd_exp(dd_neg(dd_mul(dd_make(x), x)));
  return dd_to_double(dd_mul(dd_mul(sum, e), 0.5));
}

// Gauss-Legendre rule of 20 points on [-1, 1] in long double (Newton on P_20).
struct GL20 {
  ld x[20], w[20];
  GL20() {
    const int n = 20;
    for (int k = 0; k < n; ++k) {
      ld z = cosl(3.14159265358979323846264338327950288L * (k + 0.75L) / (n + 0.5L));
      for (int it = 0; it < 100; ++it) {
        ld p0 = 1, p1 = z;
        for (int j = 2; j <= n; ++j) {
          ld p2 = ((2 * j - 1) * z * p1 - (j - 1) * p0) / j;
          p0 = p1;
          p1 = p2;
        }
        ld dp = n * (z * p1 - p0) / (z * z - 1);
        ld dz = p1 / dp;
        z -= dz;
        if (fabsl(dz) < 1e-21L) break;
      }
      ld p0 = 1, p1 = z;
      for (int j = 2; j <= n; ++j) {
        ld p2 = ((2 * j - 1) * z * p1 - (j - 1) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      ld dp = n * (z * p1 - p0) / (z * z - 1);
      x[k] = z;
      w[k] = 2 / ((1 - z * z) * dp * dp);
    }
  }
};

// Finite parts W_{-n}(x) = FP int_0^inf t^{-n} exp(-(t - x)^2) dt, n = 1..nmax
// (Eq. (sila) with beta = 2x, gamma = 1, times exp(-x^2); the finite part
// drops the terms in eps^{j-n+1} and log eps of the integral from eps).  With
// c = 1/(1 + |x|) and H_j the Taylor coefficients of exp(-(t - x)^2) at t = 0,
//   W_{-n} = sum_{j != n-1} H_j c^{j-n+1} / (j - n + 1) + H_{n-1} log c
//            + int_c^inf t^{-n} exp(-(t - x)^2) dt,
// the first sum over all j >= 0 (the part of [0, c] after subtracting the
// singular terms, plus the finite parts of the subtracted terms), the last
// integral by Gauss-Legendre panels: geometric (ratio 1.25) from c to 1, then
// of width 1/4 to max(x, 0) + 12.  H_j = e^{-x^2} Hphys_j(x) / j!.
void w_negint(int nmax, ld x, ld *out) {
  static const GL20 gl;
  const ld c = 1.0L / (1.0L + fabsl(x));
  const ld ex = expl(-x * x);
  // q_j = Hphys_j(x) / j!
  const int J = nmax + 120;
  std::vector<ld> q(J + 1);
  q[0] = 1;
  q[1] = 2 * x;
  for (int j = 1; j < J; ++j) q[j + 1] = (2 * x * q[j] - 2 * q[j - 1]) / (j + 1);
  const ld lc = logl(c);
  for (int n = 1; n <= nmax; ++n) {
    ld s = 0, cp = powl(c, (ld)(1 - n));  // c^{j-n+1} at j = 0
    for (int j = 0; j <= J; ++j) {
      if (j == n - 1)
        s += q[j] * lc;
      else
        s += q[j] * cp / (ld)(j - n + 1);
      cp *= c;
    }
    out[n] = ex * s;
  }
  // tail integrals for every n at once
  std::vector<ld> tail(nmax + 1, 0.0L);
  auto panel = [&](ld a, ld b) {
    const ld h = 0.5L * (b - a), m = 0.5L * (a + b);
    for (int k = 0; k < 20; ++k) {
      const ld t = m + h * gl.x[k];
      const ld g = gl.w[k] * h * expl(-(t - x) * (t - x));
      ld tp = 1.0L / t;
      for (int n = 1; n <= nmax; ++n) {
        tail[n] += g * tp;
        tp /= t;
      }
    }
  };
  ld a = c;
  while (a < 1.0L) {
    const ld b = std::min(1.0L, a * 1.25L);
    panel(a, b);
    a = b;
  }
  const ld top = std::max(x, (ld)0) + 12.0L;
  for (; a < top; a += 0.25L) panel(a, a + 0.25L);
  for (int n = 1; n <= nmax; ++n) out[n] += tail[n];
}

// Finite parts W_{-n}(x), n = 1..nmax, from the series in powers of x:
//   W_a(x) = e^{-x^2} sum_k c_{a+k} (2x)^k / k!,  c_m = FP int_0^inf t^m e^{-t^2} dt,
// c_m = Gamma((m+1)/2)/2, except at m = -(2p+1), where c_m = (-1)^p psi(p+1)/(2 p!)
// (the finite part of the log-divergent integrals).  Terms k >= n (m >= 0)
// by the ratio c_{m+2} = (m+1)/2 c_m; everything in double-double, which
// absorbs the cancellation of the alternating terms k < n.
void w_negint_series_dd(int nmax, double x, ld *out) {
  std::vector<dd> cneg(nmax + 1);  // c_{-n}
  for (int n = 1; n <= nmax; ++n) {
    if (n & 1) {
      const int p = (n - 1) / 2;
      dd psi = dd{-0.5772156649015329, 4.942915152430645e-18};
      dd pf = dd_make(1.0);
      for (int i = 1; i <= p; ++i) {
        psi = dd_add(psi, dd_div(dd_make(1.0), (double)i));
        pf = dd_mul(pf, (double)i);
      }
      dd v = dd_div(dd_mul(psi, 0.5), pf);
      cneg[n] = (p & 1) ? dd_neg(v) : v;
    } else {
      cneg[n] = dd_mul(dd_gamma_any(0.5 - n / 2), 0.5);
    }
  }
  const dd y = dd_make(2.0 * x);
  const dd y2 = dd_mul(y, y);
  const dd ex = dd_exp(dd_neg(dd_mul(dd_make(x), x)));
  const dd c0 = dd_mul(dd_gamma(0.5), 0.5), c1 = dd_make(0.5);  // c_0 = sqrt(pi)/2, c_1 = 1/2
  const int kextra = (int)(4.0 * x * x) + 60;
  for (int n = 1; n <= nmax; ++n) {
    dd sum = dd_make(0.0);
    // k < n: finite-part coefficients
    dd pk = dd_make(1.0);  // (2x)^k / k!
    for (int k = 0; k < n; ++k) {
      sum = dd_add(sum, dd_mul(cneg[n - k], pk));
      pk = dd_div(dd_mul(pk, y), (double)(k + 1));
    }
    // k >= n: t_k = c_{k-n} (2x)^k / k!, two interleaved ratio chains
    dd te = dd_mul(c0, pk);                                        // k = n
    dd to = dd_div(dd_mul(dd_mul(c1, pk), y), (double)(n + 1));    // k = n + 1
    sum = dd_add(sum, dd_add(te, to));
    for (int j = 0; j < kextra; j += 2) {
      const int k = n + j;  // te at k, to at k + 1
      te = dd_div(dd_mul(dd_mul(te, 0.5 * (j + 1)), y2), (double)(k + 1) * (k + 2));
      to = dd_div(dd_mul(dd_mul(to, 0.5 * (j + 2)), y2), (double)(k + 2) * (k + 3));
      sum = dd_add(sum, dd_add(te, to));
      if (j > 4.0 * x * x + 20 && std::fabs(te.hi) + std::fabs(to.hi) < 1e-34 * std::fabs(sum.hi)) break;
    }
    const dd w = dd_mul(sum, ex);
    out[n] = (ld)w.hi + (ld)w.lo;
  }
}

void w_column(double a0, bool is_int, int m_lo, int m_hi, double xd, double *out) {
  const ld x = xd;
  const int n = m_hi - m_lo + 1;
  std::vector<ld> w(n, 0.0L);
  auto at = [&](int m) -> ld & { return w[m - m_lo]; };
  const ld A0 = a0;
  ld w0, w1;
  if (x >= 0) {
    w0 = W_pos(A0, x);
    w1 = W_pos(A0 + 1, x);
  } else {
    w0 = W_neg_quad(A0, x);
    w1 = W_neg_quad(A0 + 1, x);
  }
  // ---- upward (m >= 0)
  if (x > -0.5L) {
    if (0 >= m_lo && 0 <= m_hi) at(0) = w0;
    if (1 >= m_lo && 1 <= m_hi) at(1) = w1;
    ld wm1 = w0, wc = w1;
    for (int m = 1; m < m_hi; ++m) {
      ld a = A0 + m;
      ld wn = x * wc + 0.5L * a * wm1;
      wm1 = wc;
      wc = wn;
      if (m + 1 >= m_lo) at(m + 1) = wn;
    }
  } else {
    // Miller downward (W is the minimal solution as a grows); the ratio of the
    // two solutions per step tends to 1 as x -> 0-, so start further up there.
    int top = std::max(m_hi, 1) + 60 + (int)(600.0L / fabsl(x));
    std::vector<ld> tr(top + 2, 0.0L);
    tr[top + 1] = 0.0L;
    tr[top] = 1e-300L;
    for (int m = top; m >= 1; --m) {
      ld a = A0 + m;  // W_{a-1} = (2 W_{a+1} - 2x W_a)/a
      tr[m - 1] = (2 * tr[m + 1] - 2 * x * tr[m]) / a;
      if (fabsl(tr[m - 1]) > 1e300L) {
        for (int k = m - 1; k <= top + 1; ++k) tr[k] *= 1e-300L;
      }
    }
    ld scale = w0 / tr[0];
    for (int m = std::max(0, m_lo); m <= m_hi; ++m) at(m) = tr[m] * scale;
  }
  // ---- negative integer orders (finite parts)
  if (m_lo < 0 && is_int) {
    const int nmax = -m_lo;
    std::vector<ld> wn(nmax + 1);
    if (x > 16.0L) {
      // the integral is dominated by the peak at t = x: direct formula
      w_negint(nmax, x, wn.data());
    } else if (x > 0.5L) {
      w_negint_series_dd(nmax, (double)x, wn.data());
    } else {
      // W_{-1} = e^{-x^2} [int_0^{1/2} expm1(2xt - t^2)/t dt - log 2]
      //          + int_{1/2}^inf e^{-(t-x)^2}/t dt   (no cancellation for x <= 1/2),
      // then downward: W_{-n-1} = (2x W_{-n} - 2 W_{-n+1} + H_n) / n, the
      // integration-by-parts relation with its boundary term H_n (stable here)
      static const GL20 gl;
      const ld ex = expl(-x * x);
      ld near = 0, far = 0;
      for (int pnl = 0; pnl < 8; ++pnl) {
        const ld a = pnl / 16.0L, h = 1.0L / 32;
        for (int k = 0; k < 20; ++k) {
          const ld t = a + h + h * gl.x[k];
          near += gl.w[k] * h * expm1l(2 * x * t - t * t) / t;
        }
      }
      for (ld a = 0.5L; a < 12.0L; a += 0.25L) {
        const ld h = 0.125L;
        for (int k = 0; k < 20; ++k) {
          const ld t = a + h + h * gl.x[k];
          far += gl.w[k] * h * expl(-(t - x) * (t - x)) / t;
        }
      }
      const ld wm1 = ex * (near - logl(2.0L)) + far;
      ld qm1 = 1, q = 2 * x;  // Hphys_n(x)/n! at n = 0, 1
      ld wprev = w0, wcur = wm1;
      wn[1] = wcur;
      for (int n = 1; n < nmax; ++n) {
        const ld wnext = (2 * x * wcur - 2 * wprev + ex * q) / n;
        wn[n + 1] = wnext;
        wprev = wcur;
        wcur = wnext;
        const ld qn = (2 * x * q - 2 * qm1) / (n + 1);
        qm1 = q;
        q = qn;
      }
    }
    for (int m = m_lo; m < 0; ++m) at(m) = wn[-m];
  }
  // ---- downward (m < 0), non-integer families only
  if (m_lo < 0 && !is_int) {
    if (x > 0.5L && x <= 12.0L) {
      // Below a = -x^2/2 the recurrence is oscillatory (neither direction is
      // stable): sum the Phi-series directly in double-double,
      //   W_a(x) = exp(-x^2)/2 sum_k Gamma((a+k+1)/2) (2x)^k / k!.
      for (int m = m_lo; m < 0; ++m) at(m) = (ld)w_phi_series_dd(a0 + m, (double)x);
    } else if (x > 0.5L) {
      // Miller upward from m_lo - 80 (W dominant as a grows)
      int bot = m_lo - 80;
      int cnt = 1 - bot + 1;
      std::vector<ld> tr(cnt + 1, 0.0L);
      // index k <-> m = bot + k
      tr[0] = 0.0L;
      tr[1] = 1e-300L;
      for (int k = 1; k < cnt; ++k) {
        ld a = A0 + (bot + k);
        tr[k + 1] = x * tr[k] + 0.5L * a * tr[k - 1];
        if (fabsl(tr[k + 1]) > 1e300L)
          for (int j = 0; j <= k + 1; ++j) tr[j] *= 1e-300L;
      }
      ld scale = w0 / tr[0 - bot];
      for (int m = m_lo; m < 0; ++m) at(m) = tr[m - bot] * scale;
    } else {
      ld wp = w1, wc = w0;  // W_{a0+1}, W_{a0}
      for (int m = 0; m > m_lo; --m) {
        ld a = A0 + m;  // W_{a-1} = (2 W_{a+1} - 2x W_a)/a
        ld wn = (2 * wp - 2 * x * wc) / a;
        wp = wc;
        wc = wn;
        at(m - 1) = wn;
      }
    }
  }
  for (int i = 0; i < n; ++i) out[i] = (double)w[i];
}

}  // namespace

// Diagnostic: a column of the W table as built on the host.
extern "C" int f12_aux_w_column(double alpha0, int32_t is_int, int32_t m_lo, int32_t m_hi,
                                double x, double *out) {
  if (!out || m_hi < m_lo || m_hi < 1 || alpha0 < 0 || alpha0 >= 1) return F12_EINVAL;
  if (is_int && m_lo < -64) return F12_EINVAL;
  w_column(alpha0, is_int != 0, m_lo, m_hi, x, out);
  return F12_OK;
}

namespace {
int kernel_from_factors(int32_t cls, const Expr &ef, const Expr &efp, f12_kernel **out);
}  // namespace

extern "C" int f12_kernel_create(int32_t cls, const f12_factor *f, const f12_factor *fp,
                                 f12_kernel **out) {
  if (!out) return F12_EINVAL;
  *out = nullptr;
  if (cls < 1 || cls > 6) return F12_EINVAL;
  if (cls != 1) {
    int s = validate_factor(f);
    if (s) return s;
  }
  if (!fp) fp = f;
  if (cls == 4 || cls == 6) {
    int s = validate_factor(fp);
    if (s) return s;
  }
  Expr ef, efp;
  if (cls != 1) ef = factor_expr(*f);
  if (cls == 4 || cls == 6) efp = factor_expr(*fp);
  return kernel_from_factors(cls, ef, efp, out);
}

extern "C" int f12_kernel_create_terms(int32_t cls, int32_t nf, const double *f_terms, int32_t nfp,
                                       const double *fp_terms, f12_kernel **out) {
  if (!out) return F12_EINVAL;
  *out = nullptr;
  if (cls < 1 || cls > 6) return F12_EINVAL;
  auto read = [](int32_t n, const double *t, Expr &e) -> int {
    if (n <= 0 || n > MAX_TERMS || !t) return F12_EINVAL;
    for (int i = 0; i < n; ++i) {
      const double c = t[4 * i], a = t[4 * i + 1], b = t[4 * i + 2], g = t[4 * i + 3];
      if (!std::isfinite(c) || !std::isfinite(a) || !std::isfinite(b) || !std::isfinite(g)) return F12_EPARAM;
      if (g < 0.0) return F12_EPARAM;
      const bool integer = a == std::floor(a);
      if ((integer && a < 0.0) || (!integer && a <= -1.0)) return F12_EPARAM;
      if (b < 0.0 && !integer) return F12_EPARAM;  // decaying terms: integer powers only
      add_term(e, {c, a, b, g});
    }
    return F12_OK;
  };
  Expr ef, efp;
  if (cls != 1) {
    int s = read(nf, f_terms, ef);
    if (s) return s;
  }
  if (cls == 4 || cls == 6) {
    int s = (nfp == 0 && !fp_terms) ? F12_OK : read(nfp, fp_terms, efp);
    if (s) return s;
    if (nfp == 0 && !fp_terms) efp = ef;
  }
  return kernel_from_factors(cls, ef, efp, out);
}

namespace {
int kernel_from_factors(int32_t cls, const Expr &ef, const Expr &efp, f12_kernel **out) {
  std::unique_ptr<f12_kernel> K(new (std::nothrow) f12_kernel);
  if (!K) return F12_ENOMEM;
  K->cls = cls;
  Expr e;
  switch (cls) {
    case 1: add_term(e, {1.0, 0.0, 0.0, 0.0}); break;
    case 2: e = ef; break;
    case 3:
    case 5: e = shift_alpha(ef, 1.0); break;
    case 4: e = shift_alpha(mul(ef, efp), 1.0); break;
    case 6: e = shift_alpha(mul(deriv(ef), deriv(efp)), 1.0); break;
  }
  // drop exact cancellations
  Expr e2;
  for (auto &t : e)
    if (std::fabs(t.c) > 1e-300) e2.push_back(t);  // exact cancellations
  e = e2;
  K->terms = e;
  // ---- families and chains
  struct Fam {
    double a0;
    bool is_int;
    int m_lo, m_hi;
  };
  std::vector<Fam> fams;
  struct Ch {
    double b, g;
    int fam;
    std::vector<std::pair<int, dd>> tm;
  };
  std::vector<Ch> chains;
  for (auto &t : e) {
    double fl = std::floor(t.alpha + 1e-9);
    double a0 = t.alpha - fl;
    if (a0 < 1e-9 || a0 > 1 - 1e-9) a0 = 0.0;
    int m = (int)std::lround(t.alpha - a0);
    int fi = -1;
    for (size_t i = 0; i < fams.size(); ++i)
      if (std::fabs(fams[i].a0 - a0) < 1e-9) fi = (int)i;
    if (fi < 0) {
      fams.push_back({a0, a0 == 0.0, 1 << 30, -(1 << 30)});
      fi = (int)fams.size() - 1;
    }
    if (m < -NEG_POW_MAX) return F12_EPARAM;  // beyond the tabulated negative orders
    int ci = -1;
    for (size_t i = 0; i < chains.size(); ++i)
      if (chains[i].fam == fi && same(chains[i].b, t.b) && same(chains[i].g, t.g)) ci = (int)i;
    if (ci < 0) {
      chains.push_back({t.b, t.g, fi, {}});
      ci = (int)chains.size() - 1;
    }
    // decaying chains (b < 0) run the downward ladders, written for integer
    // families with non-negative powers
    if (t.b < 0.0 && !(fams[fi].is_int && m >= 0)) return F12_EPARAM;
    chains[ci].tm.push_back({m, dd{t.c, t.clo}});
  }
  if ((int)chains.size() > MAX_CHAINS || (int)e.size() > MAX_TERMS ||
      (int)fams.size() > MAX_FAMILIES)
    return F12_EPARAM;
  KernelDev &D = K->host_desc;
  std::memset(&D, 0, sizeof(D));
  D.cls = cls;
  D.nchains = (int)chains.size();
  D.nfam = (int)fams.size();
  int nt = 0;
  for (size_t c = 0; c < chains.size(); ++c) {
    ChainDesc &cd = D.chains[c];
    cd.b = chains[c].b;
    cd.g = chains[c].g;
    cd.family = chains[c].fam;
    cd.t_begin = nt;
    cd.m_min = 1 << 30;
    cd.m_max = -(1 << 30);
    for (auto &pr : chains[c].tm) {
      D.terms[nt].c = pr.second.hi;
      D.terms[nt].clo = pr.second.lo;
      D.terms[nt].m = pr.first;
      D.terms[nt].chain = (int)c;
      ++nt;
      cd.m_min = std::min(cd.m_min, pr.first);
      cd.m_max = std::max(cd.m_max, pr.first);
    }
    cd.t_end = nt;
    // the large-T route keeps W of orders m_min - L .. m_max per chain
    if (cd.m_max - cd.m_min + LTOT_MAX + 1 > NW_MAX) return F12_EPARAM;
    cd.phi_off = (int)c * 2 * (KPHI + 1);
    Fam &F = fams[cd.family];
    int lo = (F.is_int && cd.m_min >= 0) ? 0 : cd.m_min - LTOT_MAX;
    F.m_lo = std::min(F.m_lo, lo);
    F.m_hi = std::max(F.m_hi, cd.m_max + KT + 1);
  }
  D.nterms = nt;
  D.negint = 0;
  D.heavy = 0;
  D.singular = 0;
  for (int c = 0; c < D.nchains; ++c)
    if (fams[D.chains[c].family].a0 + D.chains[c].m_min <= -1.0 + 1e-9) D.singular = 1;
  for (int c = 0; c < D.nchains; ++c) {
    if (fams[D.chains[c].family].is_int && D.chains[c].m_min < 0) D.negint = 1;
    if (D.chains[c].m_max - D.chains[c].m_min + LTOT_MAX + 1 > NW_LIGHT) D.heavy = 1;
  }
  if (D.negint) D.heavy = 1;
  D.negb = 0;
  for (int c = 0; c < D.nchains; ++c)
    if (D.chains[c].b < 0.0) D.heavy = D.negb = 1;  // the downward ladders live in the heavy kernels
  D.compact = !D.heavy;
  for (int c = 0; c < D.nchains; ++c)
    if (D.chains[c].m_max - D.chains[c].m_min > SPAN_C) D.compact = 0;
  // ---- W tables
  const int nx = (int)std::lround((WX_HI - WX_LO) * WX_INVH) + 1;
  for (size_t fi = 0; fi < fams.size(); ++fi) {
    Fam &F = fams[fi];
    int nm = F.m_hi - F.m_lo + 1;
    std::vector<double> tab((size_t)nx * nm);
    std::vector<double> col(nm);
    for (int ix = 0; ix < nx; ++ix) {
      double x = WX_LO + ix / WX_INVH;
      w_column(F.a0, F.is_int, F.m_lo, F.m_hi, x, col.data());
      std::copy(col.begin(), col.end(), tab.begin() + (size_t)ix * nm);
    }
    auto buf = std::unique_ptr<DevBuf<double>>(new DevBuf<double>);
    if (!buf->upload(tab)) return F12_ENOMEM;
    FamilyDesc &fd = D.fam[fi];
    fd.alpha0 = F.a0;
    fd.is_int = F.is_int;
    fd.m_lo = F.m_lo;
    fd.m_hi = F.m_hi;
    fd.nm = nm;
    fd.nx = nx;
    fd.table = buf->ptr;
    K->tables.push_back(std::move(buf));
  }
  // ---- Phi-series coefficients for the small-T route (DD)
  std::vector<double> phi((size_t)D.nchains * 2 * (KPHI + 1) * 2);
  for (int c = 0; c < D.nchains; ++c) {
    const ChainDesc &cd = D.chains[c];
    double as = fams[cd.family].a0 + cd.m_min + 1;
    for (int s = 0; s < 2; ++s) {
      double a = as + s;
      dd kf = dd_make(1.0);
      for (int k = 0; k <= KPHI; ++k) {
        if (k > 0) kf = dd_mul(kf, (double)k);
        double arg = 0.5 * (a + 1.0 + k);
        dd gval;
        const double pr = -arg;  // a pole of Gamma when a non-negative integer
        if (fams[cd.family].is_int && pr >= 0.0 && pr == std::floor(pr)) {
          // finite part of int_0^inf t^(-2p-1) e^{-t^2} dt = (-1)^p psi(p+1) / (2 p!):
          // the Phi-series coefficient takes (-1)^p psi(p+1) / p! for Gamma(-p)
          const int pp = (int)pr;
          dd psi = dd{-0.5772156649015329, 4.942915152430645e-18};  // -Euler's gamma
          dd pf = dd_make(1.0);
          for (int i = 1; i <= pp; ++i) {
            psi = dd_add(psi, dd_div(dd_make(1.0), (double)i));
            pf = dd_mul(pf, (double)i);
          }
          gval = dd_div(psi, pf);
          if (pp & 1) gval = dd_neg(gval);
        } else {
          gval = dd_gamma_any(arg);
        }
        dd v = dd_div(dd_mul(gval, 0.5), kf);
        size_t o = ((size_t)(c * 2 + s) * (KPHI + 1) + k) * 2;
        phi[o] = v.hi;
        phi[o + 1] = v.lo;
      }
    }
  }
  if (!K->d_phi.upload(phi)) return F12_ENOMEM;
  D.phi = K->d_phi.ptr;
  if (!K->d_desc.alloc(1)) return F12_ENOMEM;
  if (hipMemcpy(K->d_desc.ptr, &D, sizeof(KernelDev), hipMemcpyHostToDevice) != hipSuccess)
    return F12_EDEVICE;
  *out = K.release();
  return F12_OK;
}
}  // namespace

extern "C" int f12_kernel_terms(const f12_kernel *k, int32_t *nterms, double *out, int32_t cap) {
  if (!k || !nterms) return F12_EINVAL;
  *nterms = (int32_t)k->terms.size();
  if (out)
    for (int i = 0; i < (int)k->terms.size() && i < cap; ++i) {
      out[4 * i] = k->terms[i].c;
      out[4 * i + 1] = k->terms[i].alpha;
      out[4 * i + 2] = k->terms[i].b;
      out[4 * i + 3] = k->terms[i].g;
    }
  return F12_OK;
}

extern "C" void f12_kernel_destroy(f12_kernel *k) { delete k; }

// Diagnostic: A_n (n = 0..L) on the device for explicit (p, q, R) triples.
// d_p, d_q, d_R: device double[n]; d_A: device double[(L+1) * n], A[k*n + i].
extern "C" int f12_aux_radial(const f12_kernel *k, int64_t n, const double *d_p, const double *d_q,
                              const double *d_R, int32_t L, int32_t route, double *d_A,
                              void *stream) {
  if (!k || n < 0 || L < 0 || L > LTOT_MAX || route < 0 || route > 3 ||
      (n > 0 && (!d_p || !d_q || !d_R || !d_A)))
    return F12_EINVAL;
  if (launch_aux_points(k->d_desc.ptr, n, d_p, d_q, d_R, L, route, d_A, (hipStream_t)stream,
                        aux_variant(k->host_desc)) != 0)
    return F12_EDEVICE;
  return F12_OK;
}

// ============================================================================
// quartets
// ============================================================================
namespace {

int finish_quartets(f12_quartets *Q, std::vector<int64_t> &qb, std::vector<int64_t> &qk) {
  const f12_pairs *B = Q->bra, *K = Q->ket;
  const int64_t nq = (int64_t)qb.size();
  // bin by (la, lb, lc, ld) with a counting sort (stable); one digit of radix
  // LMAX + 1 per angular momentum
  constexpr int RAD = LMAX + 1, NBIN = RAD * RAD * RAD * RAD;
  static_assert(F12_LMAX == LMAX, "public and internal angular-momentum limits agree");
  auto key = [&](int64_t i) {
    return ((B->la[qb[i]] * RAD + B->lb[qb[i]]) * RAD + K->la[qk[i]]) * RAD + K->lb[qk[i]];
  };
  std::vector<int64_t> cnt(NBIN + 1, 0);
  for (int64_t i = 0; i < nq; ++i) cnt[key(i) + 1]++;
  for (int k = 0; k < NBIN; ++k) cnt[k + 1] += cnt[k];
  std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
  Q->qb.assign(nq, 0);
  Q->qk.assign(nq, 0);
  for (int64_t i = 0; i < nq; ++i) {
    int64_t d = pos[key(i)]++;
    Q->qb[d] = qb[i];
    Q->qk[d] = qk[i];
  }
  qb.clear();
  qb.shrink_to_fit();
  qk.clear();
  qk.shrink_to_fit();
  // inside each group: decreasing primitive-quartet count (stable), so that
  // the longest work-groups of a launch start first
  {
    std::vector<int64_t> idx, tb, tk;
    for (int k = 0; k < NBIN; ++k) {
      const int64_t lo = cnt[k], n = cnt[k + 1] - cnt[k];
      if (n < 2) continue;
      idx.resize(n);
      for (int64_t i = 0; i < n; ++i) idx[i] = lo + i;
      auto np = [&](int64_t i) {
        return (int64_t)B->ka[Q->qb[i]] * B->kb[Q->qb[i]] * (int64_t)K->ka[Q->qk[i]] * K->kb[Q->qk[i]];
      };
      std::stable_sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) { return np(x) > np(y); });
      tb.resize(n);
      tk.resize(n);
      for (int64_t i = 0; i < n; ++i) {
        tb[i] = Q->qb[idx[i]];
        tk[i] = Q->qk[idx[i]];
      }
      std::copy(tb.begin(), tb.end(), Q->qb.begin() + lo);
      std::copy(tk.begin(), tk.end(), Q->qk.begin() + lo);
    }
  }
  Q->bins.clear();
  for (int k = 0; k < NBIN; ++k) {
    int64_t n = cnt[k + 1] - cnt[k];
    if (n == 0) continue;
    Q->bins.push_back({k / (RAD * RAD * RAD), (k / (RAD * RAD)) % RAD, (k / RAD) % RAD, k % RAD, cnt[k], n});
  }
  Q->qoff.assign(nq + 1, 0);
  Q->qprim.assign(nq + 1, 0);
  for (int64_t i = 0; i < nq; ++i) {
    const int64_t b = Q->qb[i], k = Q->qk[i];
    Q->qoff[i + 1] = Q->qoff[i] + (int64_t)ncart_host(B->la[b]) * ncart_host(B->lb[b]) * ncart_host(K->la[k]) *
                                      ncart_host(K->lb[k]);
    Q->qprim[i + 1] =
        Q->qprim[i] + (int64_t)B->ka[b] * B->kb[b] * (int64_t)K->ka[k] * K->kb[k];
  }
  Q->max_qprim = 0;
  for (int64_t i = 0; i < nq; ++i) Q->max_qprim = std::max(Q->max_qprim, Q->qprim[i + 1] - Q->qprim[i]);
  Q->nq = nq;
  Q->nout = Q->qoff[nq];
  Q->nprim = Q->qprim[nq];
  if (!Q->d_qb.upload(Q->qb) || !Q->d_qk.upload(Q->qk) || !Q->d_qoff.upload(Q->qoff) ||
      !Q->d_qprim.upload(Q->qprim))
    return F12_ENOMEM;
  Q->a_cap_prims = std::min<int64_t>(std::max<int64_t>(Q->nprim, 1), (int64_t)1 << 23);
  if (!Q->d_A.alloc((size_t)Q->a_cap_prims * (LTOT_MAX + 1))) return F12_ENOMEM;
  return F12_OK;
}

// Evaluates [q_begin, q_end) with radial-derivative scratch A of cap_prims
// primitive quartets (times LTOT_MAX + 1 doubles), in chunks that fit it.
int eval_range(f12_quartets *Q, const f12_kernel *k, int64_t q_begin, int64_t q_end, double *d_out,
               double *A, int64_t cap_prims, hipStream_t st, int prec = 0, int gdir = -1);

}  // namespace

extern "C" int f12_quartets_from_list(const f12_pairs *bra, const f12_pairs *ket, int32_t cls,
                                      const int32_t *quads, int64_t nq, f12_quartets **out,
                                      int64_t *n_out_doubles) {
  if (!bra || !ket || !out || nq < 0 || (nq > 0 && !quads) || cls < 1 || cls > 6)
    return F12_EINVAL;
  *out = nullptr;
  if (!bra->ordered || !ket->ordered) return F12_EINVAL;
  std::unique_ptr<f12_quartets> Q(new (std::nothrow) f12_quartets);
  if (!Q) return F12_ENOMEM;
  Q->bra = bra;
  Q->ket = ket;
  Q->cls = cls;
  std::vector<int64_t> qb(nq), qk(nq);
  const int64_t ns = bra->nshell;
  for (int64_t i = 0; i < nq; ++i) {
    for (int j = 0; j < 4; ++j)
      if (quads[4 * i + j] < 0 || quads[4 * i + j] >= ns) return F12_EINVAL;
    qb[i] = quads[4 * i] * ns + quads[4 * i + 1];
    qk[i] = quads[4 * i + 2] * ns + quads[4 * i + 3];
  }
  int s = finish_quartets(Q.get(), qb, qk);
  if (s) return s;
  if (n_out_doubles) *n_out_doubles = Q->nout;
  *out = Q.release();
  return F12_OK;
}

namespace {

// Screening estimate of f12_quartets_build.  Q_ab Q_cd alone bounds
// |(ab|k|cd)| only for a positive-definite kernel; the long-range part
// c0 r^rho e^{B r} of Eq. (rs12) grows with r, so the estimate carries the
// growth of the kernel's undamped terms (g = 0, b > 0),
//   kappa(r) = sum |c_t| r^(alpha_t - 1) e^(b_t r),
// from r = 1 to the largest distance R_eff between the primitive-pair
// centres of the two pairs (each P lies on its segment AB), and per pair the
// growth of e^{b |r - P|} over the pair density's extent,
//   exp(b sqrt((l_a + l_b + 1) / (2 p_min)) + b^2 / (4 p_min)).
// I5 = 1/2 (lap_A - lap_B) I3 (Eq. (I5_)) multiplies the bra by up to about
// the largest bra exponent times (2 l + 3).
struct ScreenEst {
  std::vector<double> Sb, Sk;  // Q times the pair's extent factor
  std::vector<HostTerm> grow;
  double kappa1 = 1.0;
  double kappa(double r) const {
    double v = 0.0;
    for (const HostTerm &t : grow) v += std::fabs(t.c) * std::pow(r, t.alpha - 1.0) * std::exp(t.b * r);
    return v;
  }
};

int screen_estimate(const f12_pairs *bra, const f12_pairs *ket, int32_t cls, const f12_kernel *screen_kernel,
                    hipStream_t st, ScreenEst &E) {
  std::vector<double> Qb, Qk;
  // Q_ab = sqrt(max |(ab|k|ab)|) over the diagonal quartets of the pair set
  auto diag = [&](const f12_pairs *P, std::vector<double> &Qv) -> int {
    std::unique_ptr<f12_quartets> D(new (std::nothrow) f12_quartets);
    if (!D) return F12_ENOMEM;
    D->bra = P;
    D->ket = P;
    D->cls = screen_kernel->cls == 5 ? 3 : screen_kernel->cls;
    std::vector<int64_t> qb(P->nsp), qk(P->nsp);
    for (int64_t i = 0; i < P->nsp; ++i) qb[i] = qk[i] = i;
    int s = finish_quartets(D.get(), qb, qk);
    if (s) return s;
    DevBuf<double> dout;
    if (!dout.alloc(D->nout)) return F12_ENOMEM;
    s = eval_range(D.get(), screen_kernel, 0, D->nq, dout.ptr, D->d_A.ptr, D->a_cap_prims, st);
    if (s) return s;
    std::vector<double> h(D->nout);
    if (hipMemcpyAsync(h.data(), dout.ptr, D->nout * sizeof(double), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return F12_EDEVICE;
    Qv.assign(P->nsp, 0.0);
    for (int64_t i = 0; i < D->nq; ++i) {
      double m = 0;
      for (int64_t o = D->qoff[i]; o < D->qoff[i + 1]; ++o) m = std::max(m, std::fabs(h[o]));
      Qv[D->qb[i]] = std::sqrt(m);
    }
    return F12_OK;
  };
  int s = diag(bra, Qb);
  if (s) return s;
  if (ket == bra)
    Qk = Qb;
  else if ((s = diag(ket, Qk)))
    return s;
  double bmax = 0.0;
  E.grow.clear();
  for (const HostTerm &t : screen_kernel->terms)
    if (t.g == 0.0 && t.b > 0.0) {
      E.grow.push_back(t);
      bmax = std::max(bmax, t.b);
    }
  if ((int)E.grow.size() > K2_MAX_GROW) return F12_EPARAM;
  E.kappa1 = E.grow.empty() ? 1.0 : E.kappa(1.0);
  auto pair_factor = [&](const f12_pairs *P, int64_t i, bool i5bra) {
    const double pm = P->pmin[i];
    double f = std::exp(bmax * std::sqrt((P->la[i] + P->lb[i] + 1) / (2.0 * pm)) + bmax * bmax / (4.0 * pm));
    if (i5bra) f *= P->emax[i] * (2 * std::max(P->la[i], P->lb[i]) + 3);
    return f;
  };
  E.Sb.resize(bra->nsp);
  E.Sk.resize(ket->nsp);
  for (int64_t b = 0; b < bra->nsp; ++b) E.Sb[b] = Qb[b] * pair_factor(bra, b, cls == 5);
  for (int64_t k = 0; k < ket->nsp; ++k) E.Sk[k] = Qk[k] * pair_factor(ket, k, false);
  return F12_OK;
}

int check_build_args(const f12_pairs *bra, const f12_pairs *ket, int32_t cls, double screen_tol,
                     const f12_kernel *screen_kernel, f12_quartets **out) {
  if (!bra || !ket || !out || cls < 1 || cls > 6) return F12_EINVAL;
  *out = nullptr;
  if (bra->ordered || ket->ordered) return F12_EINVAL;  // unordered pair sets
  if (bra->nshell != ket->nshell) return F12_EINVAL;
  if (screen_tol > 0 && !screen_kernel) return F12_EINVAL;
  return F12_OK;
}

}  // namespace

extern "C" int f12_quartets_build(const f12_pairs *bra, const f12_pairs *ket, int32_t cls,
                                  double screen_tol, const f12_kernel *screen_kernel, void *stream,
                                  f12_quartets **out, int64_t *n_quartets,
                                  int64_t *n_out_doubles) {
  int s = check_build_args(bra, ket, cls, screen_tol, screen_kernel, out);
  if (s) return s;
  hipStream_t st = (hipStream_t)stream;
  ScreenEst E;
  if (screen_tol > 0 && (s = screen_estimate(bra, ket, cls, screen_kernel, st, E))) return s;
  std::unique_ptr<f12_quartets> Q(new (std::nothrow) f12_quartets);
  if (!Q) return F12_ENOMEM;
  Q->bra = bra;
  Q->ket = ket;
  Q->cls = cls;
  std::vector<int64_t> qb, qk;
  const bool fold = (cls != 5);  // I5 has no bra-ket symmetry
  for (int64_t b = 0; b < bra->nsp; ++b) {
    int64_t kmax = fold ? std::min(b, ket->nsp - 1) : ket->nsp - 1;
    for (int64_t k = 0; k <= kmax; ++k) {
      if (screen_tol > 0) {
        double est = E.Sb[b] * E.Sk[k];
        if (est < screen_tol && !E.grow.empty()) {
          const double dx = bra->midx[b] - ket->midx[k], dy = bra->midy[b] - ket->midy[k],
                       dz = bra->midz[b] - ket->midz[k];
          const double reff = std::sqrt(dx * dx + dy * dy + dz * dz) + 0.5 * (bra->ablen[b] + ket->ablen[k]);
          if (reff > 1.0) {
            const double g = E.kappa(reff) / E.kappa1;
            if (g > 1.0) est *= g;
          }
        }
        if (est < screen_tol) continue;
      }
      qb.push_back(b);
      qk.push_back(k);
    }
  }
  s = finish_quartets(Q.get(), qb, qk);
  if (s) return s;
  if (n_quartets) *n_quartets = Q->nq;
  if (n_out_doubles) *n_out_doubles = Q->nout;
  *out = Q.release();
  return F12_OK;
}

extern "C" int f12_quartets_build_device(const f12_pairs *bra, const f12_pairs *ket, int32_t cls,
                                         double screen_tol, const f12_kernel *screen_kernel, void *stream,
                                         f12_quartets **out, int64_t *n_quartets, int64_t *n_out_doubles) {
  int s = check_build_args(bra, ket, cls, screen_tol, screen_kernel, out);
  if (s) return s;
  hipStream_t st = (hipStream_t)stream;
  ScreenEst E;
  if (screen_tol > 0 && (s = screen_estimate(bra, ket, cls, screen_kernel, st, E))) return s;
  const bool fold = (cls != 5);
  if (fold && bra->nsp != ket->nsp) return F12_EINVAL;
  // per-pair tables on the device
  auto pair_tables = [&](const f12_pairs *P, const std::vector<double> &S, DevBuf<double> &dS,
                         DevBuf<double> &dmid, DevBuf<double> &dab, DevBuf<int32_t> &dcls,
                         DevBuf<int32_t> &dnp, DevBuf<int32_t> &dnc) -> bool {
    std::vector<double> mid(3 * P->nsp);
    std::vector<int32_t> c(P->nsp), np(P->nsp), nc(P->nsp);
    for (int64_t i = 0; i < P->nsp; ++i) {
      mid[3 * i] = P->midx[i];
      mid[3 * i + 1] = P->midy[i];
      mid[3 * i + 2] = P->midz[i];
      c[i] = P->la[i] * (LMAX + 1) + P->lb[i];
      np[i] = P->ka[i] * P->kb[i];
      nc[i] = ncart_host(P->la[i]) * ncart_host(P->lb[i]);
    }
    std::vector<double> Sv = S.empty() ? std::vector<double>(P->nsp, 0.0) : S;
    return dS.upload(Sv) && dmid.upload(mid) && dab.upload(P->ablen) && dcls.upload(c) && dnp.upload(np) &&
           dnc.upload(nc);
  };
  DevBuf<double> bS, bmid, bab, kS, kmid, kab;
  DevBuf<int32_t> bcls, bnp, bnc, kcls, knp, knc;
  if (!pair_tables(bra, E.Sb, bS, bmid, bab, bcls, bnp, bnc) ||
      !pair_tables(ket, E.Sk, kS, kmid, kab, kcls, knp, knc))
    return F12_ENOMEM;
  K2Params P;
  std::memset(&P, 0, sizeof(P));
  P.nb = bra->nsp;
  P.nk = ket->nsp;
  P.fold = fold;
  P.tol = screen_tol;
  P.Sb = bS.ptr;
  P.Sk = kS.ptr;
  P.bmid = bmid.ptr;
  P.kmid = kmid.ptr;
  P.bab = bab.ptr;
  P.kab = kab.ptr;
  P.bcls = bcls.ptr;
  P.kcls = kcls.ptr;
  P.bnp = bnp.ptr;
  P.knp = knp.ptr;
  P.bnc = bnc.ptr;
  P.knc = knc.ptr;
  P.ngrow = screen_tol > 0 ? (int)E.grow.size() : 0;
  for (int t = 0; t < P.ngrow; ++t) {
    P.gc[t] = std::fabs(E.grow[t].c);
    P.ga[t] = E.grow[t].alpha;
    P.gb[t] = E.grow[t].b;
  }
  P.kappa1 = E.kappa1;
  const uint64_t ncand = fold ? (uint64_t)bra->nsp * (bra->nsp + 1) / 2 : (uint64_t)bra->nsp * ket->nsp;
  uint64_t *d_idx = nullptr;
  int64_t n = 0;
  if (k2_select(P, ncand, &d_idx, &n, st) != 0) return F12_EDEVICE;
  std::unique_ptr<f12_quartets> Q(new (std::nothrow) f12_quartets);
  if (!Q) {
    (void)hipFree(d_idx);
    return F12_ENOMEM;
  }
  Q->bra = bra;
  Q->ket = ket;
  Q->cls = cls;
  constexpr int RAD = LMAX + 1, NBIN = RAD * RAD * RAD * RAD;
  DevBuf<int64_t> d_start;
  std::vector<int64_t> start(NBIN, -1);
  bool ok = Q->d_qb.alloc(n) && Q->d_qk.alloc(n) && Q->d_qoff.alloc(n + 1) && Q->d_qprim.alloc(n + 1) &&
            d_start.upload(start);
  if (!ok) {
    (void)hipFree(d_idx);
    return F12_ENOMEM;
  }
  const int rc = k2_finalize(P, d_idx, n, Q->d_qb.ptr, Q->d_qk.ptr, Q->d_qoff.ptr, Q->d_qprim.ptr, d_start.ptr, st);
  (void)hipFree(d_idx);
  if (rc != 0) return F12_EDEVICE;
  // host copies: offsets (chunking, f12_quartet_offsets) and the pair indices
  Q->qb.resize(n);
  Q->qk.resize(n);
  Q->qoff.resize(n + 1);
  Q->qprim.resize(n + 1);
  if ((n > 0 && (hipMemcpy(Q->qb.data(), Q->d_qb.ptr, n * 8, hipMemcpyDeviceToHost) != hipSuccess ||
                 hipMemcpy(Q->qk.data(), Q->d_qk.ptr, n * 8, hipMemcpyDeviceToHost) != hipSuccess)) ||
      hipMemcpy(Q->qoff.data(), Q->d_qoff.ptr, (n + 1) * 8, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(Q->qprim.data(), Q->d_qprim.ptr, (n + 1) * 8, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(start.data(), d_start.ptr, NBIN * 8, hipMemcpyDeviceToHost) != hipSuccess)
    return F12_EDEVICE;
  Q->bins.clear();
  for (int k = 0; k < NBIN; ++k) {
    if (start[k] < 0) continue;
    int64_t e = n;
    for (int j = k + 1; j < NBIN; ++j)
      if (start[j] >= 0) {
        e = start[j];
        break;
      }
    Q->bins.push_back({k / (RAD * RAD * RAD), (k / (RAD * RAD)) % RAD, (k / RAD) % RAD, k % RAD, start[k],
                       e - start[k]});
  }
  Q->nq = n;
  Q->nout = Q->qoff[n];
  Q->nprim = Q->qprim[n];
  Q->max_qprim = 0;
  for (int64_t i = 0; i < n; ++i) Q->max_qprim = std::max(Q->max_qprim, Q->qprim[i + 1] - Q->qprim[i]);
  Q->a_cap_prims = std::min<int64_t>(std::max<int64_t>(Q->nprim, 1), (int64_t)1 << 23);
  if (!Q->d_A.alloc((size_t)Q->a_cap_prims * (LTOT_MAX + 1))) return F12_ENOMEM;
  if (n_quartets) *n_quartets = Q->nq;
  if (n_out_doubles) *n_out_doubles = Q->nout;
  *out = Q.release();
  return F12_OK;
}

extern "C" int f12_quartet_offsets(const f12_quartets *q, int64_t *offsets) {
  if (!q || !offsets) return F12_EINVAL;
  std::copy(q->qoff.begin(), q->qoff.end(), offsets);
  return F12_OK;
}

extern "C" int f12_quartet_list(const f12_quartets *q, int32_t *quads) {
  if (!q || !quads) return F12_EINVAL;
  for (int64_t i = 0; i < q->nq; ++i) {
    quads[4 * i] = q->bra->sa[q->qb[i]];
    quads[4 * i + 1] = q->bra->sb[q->qb[i]];
    quads[4 * i + 2] = q->ket->sa[q->qk[i]];
    quads[4 * i + 3] = q->ket->sb[q->qk[i]];
  }
  return F12_OK;
}

extern "C" int f12_quartet_groups(const f12_quartets *q, int32_t *ngroups, int64_t *starts, int32_t *ls,
                                  int32_t cap) {
  if (!q || !ngroups || cap < 0) return F12_EINVAL;
  const int n = (int)q->bins.size();
  *ngroups = n;
  for (int g = 0; g < n && g < cap; ++g) {
    if (starts) {
      starts[g] = q->bins[g].q0;
      starts[g + 1] = q->bins[g].q0 + q->bins[g].nq;
    }
    if (ls) {
      ls[4 * g] = q->bins[g].la;
      ls[4 * g + 1] = q->bins[g].lb;
      ls[4 * g + 2] = q->bins[g].lc;
      ls[4 * g + 3] = q->bins[g].ld;
    }
  }
  return F12_OK;
}

extern "C" int f12_quartets_prim_count(const f12_quartets *q, int64_t *n) {
  if (!q || !n) return F12_EINVAL;
  *n = q->nprim;
  return F12_OK;
}

extern "C" void f12_quartets_destroy(f12_quartets *q) { delete q; }

// ============================================================================
// evaluation
// ============================================================================
namespace {

int eval_range(f12_quartets *Q, const f12_kernel *k, int64_t q_begin, int64_t q_end, double *d_out,
               double *A, int64_t cap_prims, hipStream_t st, int prec, int gdir) {
  const PairsDev bra = Q->bra->dev(), ket = Q->ket->dev();
  const int i5 = (Q->cls == 5);
  const int64_t out_base = Q->qoff[q_begin];
  for (const Bin &b : Q->bins) {
    int64_t lo = std::max(b.q0, q_begin), hi = std::min(b.q0 + b.nq, q_end);
    if (lo >= hi) continue;
    const int L = b.la + b.lb + b.lc + b.ld + (i5 ? 2 : 0) + (gdir >= 0 ? 1 : 0);
    int64_t qa = lo;
    while (qa < hi) {
      // largest chunk [qa, qe) with at most cap_prims primitive quartets
      int64_t limit = Q->qprim[qa] + cap_prims;
      int64_t qe = std::upper_bound(Q->qprim.begin() + qa + 1, Q->qprim.begin() + hi + 1, limit) -
                   Q->qprim.begin() - 1;
      if (qe <= qa) qe = qa + 1;
      const int64_t p0 = Q->qprim[qa];
      const int64_t np = Q->qprim[qe] - p0;
      if (launch_aux(k->d_desc.ptr, bra, ket, Q->d_qb.ptr, Q->d_qk.ptr, Q->d_qprim.ptr, qa,
                     qe - qa, p0, np, L, A, st, aux_variant(k->host_desc)) != 0)
        return F12_EDEVICE;
      if (launch_contract(bra, ket, Q->d_qb.ptr, Q->d_qk.ptr, Q->d_qoff.ptr, Q->d_qprim.ptr, qa,
                          qe - qa, p0, np, A, b.la, b.lb, b.lc, b.ld, i5, d_out, out_base,
                          st, 0, prec, gdir) != 0)
        return F12_EDEVICE;
      qa = qe;
    }
  }
  return F12_OK;
}

}  // namespace

extern "C" int f12_eval(f12_quartets *q, const f12_kernel *k, int64_t q_begin, int64_t q_end,
                        double *d_out, int64_t out_capacity, void *stream) {
  if (!q || !k || !d_out || q_begin < 0 || q_end > q->nq || q_begin > q_end) return F12_EINVAL;
  if (k->cls != q->cls) return F12_EINVAL;
  if (q->qoff[q_end] - q->qoff[q_begin] > out_capacity) return F12_EBUFSIZE;
  if (q_begin == q_end) return F12_OK;
  q->stage_qa = q->stage_qe = -1;
  return eval_range(q, k, q_begin, q_end, d_out, q->d_A.ptr, q->a_cap_prims, (hipStream_t)stream);
}

extern "C" int f12_eval_sets(f12_quartets *q, const f12_kernel *const *kernels, int32_t nset,
                             int64_t q_begin, int64_t q_end, double *d_out, int64_t out_capacity,
                             void *stream) {
  if (!q || !kernels || nset < 1 || !d_out || q_begin < 0 || q_end > q->nq || q_begin > q_end)
    return F12_EINVAL;
  for (int32_t s = 0; s < nset; ++s)
    if (!kernels[s] || kernels[s]->cls != q->cls) return F12_EINVAL;
  const int64_t n = q->qoff[q_end] - q->qoff[q_begin];
  if (n > 0 && (int64_t)nset > out_capacity / n) return F12_EBUFSIZE;
  if (q_begin == q_end) return F12_OK;
  q->stage_qa = q->stage_qe = -1;
  for (int32_t s = 0; s < nset; ++s) {
    int st = eval_range(q, kernels[s], q_begin, q_end, d_out + (int64_t)s * n, q->d_A.ptr, q->a_cap_prims,
                        (hipStream_t)stream);
    if (st) return st;
  }
  return F12_OK;
}

extern "C" int f12_eval_grad(f12_quartets *q, const f12_kernel *k, int32_t dir, int64_t q_begin,
                             int64_t q_end, double *d_out, int64_t out_capacity, void *stream) {
  if (!q || !k || !d_out || q_begin < 0 || q_end > q->nq || q_begin > q_end) return F12_EINVAL;
  if (k->cls != q->cls || q->cls == 5 || dir < 0 || dir > 2) return F12_EINVAL;
  if (q->qoff[q_end] - q->qoff[q_begin] > out_capacity) return F12_EBUFSIZE;
  if (q_begin == q_end) return F12_OK;
  // every shape of the range must have a derivative form (checked before any launch)
  const PairsDev bra = q->bra->dev(), ket = q->ket->dev();
  for (const Bin &b : q->bins) {
    if (std::max(b.q0, q_begin) >= std::min(b.q0 + b.nq, q_end)) continue;
    const int s = launch_contract(bra, ket, nullptr, nullptr, nullptr, nullptr, 0, 1, 0, 0, nullptr, b.la, b.lb,
                                  b.lc, b.ld, 0, nullptr, 0, (hipStream_t)stream, -1, 0, (int)dir);
    if (s == -3) return F12_ELMAX;
    if (s != 0) return F12_EDEVICE;
  }
  q->stage_qa = q->stage_qe = -1;
  return eval_range(q, k, q_begin, q_end, d_out, q->d_A.ptr, q->a_cap_prims, (hipStream_t)stream, 0, (int)dir);
}

extern "C" int f12_eval_precision(f12_quartets *q, const f12_kernel *k, int64_t q_begin, int64_t q_end,
                                  double *d_out, int64_t out_capacity, int32_t precision, void *stream) {
  if (precision != F12_FP64 && precision != F12_SPLIT_FP32) return F12_EINVAL;
  if (!q || !k || !d_out || q_begin < 0 || q_end > q->nq || q_begin > q_end) return F12_EINVAL;
  if (k->cls != q->cls) return F12_EINVAL;
  if (q->qoff[q_end] - q->qoff[q_begin] > out_capacity) return F12_EBUFSIZE;
  if (q_begin == q_end) return F12_OK;
  q->stage_qa = q->stage_qe = -1;
  return eval_range(q, k, q_begin, q_end, d_out, q->d_A.ptr, q->a_cap_prims, (hipStream_t)stream, precision);
}

extern "C" int f12_eval_stage(f12_quartets *q, const f12_kernel *k, int64_t q_begin, int64_t q_end,
                              double *d_out, int64_t out_capacity, int32_t stage, void *stream) {
  if (!q || !k || q_begin < 0 || q_end > q->nq || q_begin >= q_end) return F12_EINVAL;
  if (k->cls != q->cls || (stage != 1 && stage != 2)) return F12_EINVAL;
  const Bin *bin = nullptr;
  for (const Bin &b : q->bins)
    if (q_begin >= b.q0 && q_begin < b.q0 + b.nq) bin = &b;
  if (!bin || q_end > bin->q0 + bin->nq) return F12_EINVAL;
  const int64_t p0 = q->qprim[q_begin], np = q->qprim[q_end] - p0;
  if (np > q->a_cap_prims) return F12_EBUFSIZE;
  const PairsDev bra = q->bra->dev(), ket = q->ket->dev();
  const int i5 = (q->cls == 5);
  hipStream_t st = (hipStream_t)stream;
  if (stage == 1) {
    const int L = bin->la + bin->lb + bin->lc + bin->ld + (i5 ? 2 : 0);
    if (launch_aux(k->d_desc.ptr, bra, ket, q->d_qb.ptr, q->d_qk.ptr, q->d_qprim.ptr, q_begin,
                   q_end - q_begin, p0, np, L, q->d_A.ptr, st, aux_variant(k->host_desc)) != 0)
      return F12_EDEVICE;
    q->stage_qa = q_begin;
    q->stage_qe = q_end;
    q->stage_k = k;
    return F12_OK;
  }
  if (!d_out) return F12_EINVAL;
  if (q->stage_qa != q_begin || q->stage_qe != q_end || q->stage_k != k) return F12_EINVAL;
  if (q->qoff[q_end] - q->qoff[q_begin] > out_capacity) return F12_EBUFSIZE;
  q->stage_qa = q->stage_qe = -1;
  if (launch_contract(bra, ket, q->d_qb.ptr, q->d_qk.ptr, q->d_qoff.ptr, q->d_qprim.ptr, q_begin,
                      q_end - q_begin, p0, np, q->d_A.ptr, bin->la, bin->lb, bin->lc, bin->ld, i5,
                      d_out, q->qoff[q_begin], st) != 0)
    return F12_EDEVICE;
  return F12_OK;
}

extern "C" int f12_quartets_scratch_prims(const f12_quartets *q, int64_t *n) {
  if (!q || !n) return F12_EINVAL;
  *n = q->a_cap_prims;
  return F12_OK;
}

// ============================================================================
// evaluation without allocation
// ============================================================================
// Radial-derivative scratch for f12_eval_noalloc: a fixed device array, one
// copy per GPU, kept until the process ends.  Host code never passes its name
// to a kernel (in host code the name is only a stand-in); it passes the device
// address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[(size_t)F12_NOALLOC_SCRATCH_PRIMS * (LTOT_MAX + 1)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
int scratch_address(double **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return F12_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return F12_EDEVICE;
    g_scratch_ptr[dev] = (double *)ptr;
  }
  *out = g_scratch_ptr[dev];
  return F12_OK;
}
}  // namespace

extern "C" int f12_eval_noalloc(f12_quartets *q, const f12_kernel *k, int64_t q_begin, int64_t q_end,
                                double *d_out, int64_t out_capacity, void *stream) {
  if (!q || !k || !d_out || q_begin < 0 || q_end > q->nq || q_begin > q_end) return F12_EINVAL;
  if (k->cls != q->cls) return F12_EINVAL;
  if (q->qoff[q_end] - q->qoff[q_begin] > out_capacity) return F12_EBUFSIZE;
  if (q_begin == q_end) return F12_OK;
  // every chunk holds at least one whole quartet: reject a quartet whose
  // primitive quartets exceed the fixed scratch
  if (q->max_qprim > (int64_t)F12_NOALLOC_SCRATCH_PRIMS) return F12_EBUFSIZE;
  double *A = nullptr;
  int s = scratch_address(&A);
  if (s) return s;
  q->stage_qa = q->stage_qe = -1;
  return eval_range(q, k, q_begin, q_end, d_out, A, (int64_t)F12_NOALLOC_SCRATCH_PRIMS,
                    (hipStream_t)stream);
}
