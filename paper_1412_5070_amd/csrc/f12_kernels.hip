// HIP kernels for gfx950: primitive-pair data, radial derivatives of the
// basic integrals (the auxiliary functions), Hermite integrals R_tuv and the
// E.R.E contraction of the McMurchie-Davidson route of arXiv:1412.5070.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>
#include <mutex>
#include <utility>

#include "f12_internal.h"
#include "f12_common.h"
#include "f12_dd.h"
#include "f12_launch.h"

namespace f12 {

#define F12_PI52 17.493418327624862846  // pi^(5/2)
#define F12_SQRTPI 1.7724538509055160273
#define F12_PI 3.14159265358979323846

// Fault word of the device: a kernel that produces a non-finite value (an
// A_n, an output element) sets it to 1 with a plain store from the lane that
// found it; f12_stream_status reads and clears it.
__device__ int fault_word_dev;

namespace {
constexpr int kMaxDev = 64;
std::mutex g_fault_mu;
int *g_fault_ptr[kMaxDev] = {};
}  // namespace

int *fault_word() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return nullptr;
  std::lock_guard<std::mutex> lock(g_fault_mu);
  if (!g_fault_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(fault_word_dev)) != hipSuccess || !ptr) return nullptr;
    g_fault_ptr[dev] = (int *)ptr;
  }
  return g_fault_ptr[dev];
}


// ---------------------------------------------------------------------------
// K1: primitive-pair data.  Gaussian product (Sec. II.B): p = a + b,
// P = (a A + b B)/p; c_a c_b is applied in the contraction.
// ---------------------------------------------------------------------------
__global__ void pair_prims_kernel(int64_t npp, const int32_t *__restrict__ pp_sa,
                                  const int32_t *__restrict__ pp_sb,
                                  const int32_t *__restrict__ pp_ia,
                                  const int32_t *__restrict__ pp_ib,
                                  const int32_t *__restrict__ shell_first,
                                  const int32_t *__restrict__ shell_center,
                                  const double *__restrict__ xyz, const double *__restrict__ exps,
                                  const double *__restrict__ coefs, double *ea, double *eb, double *p,
                                  double *Px, double *Py, double *Pz, double *cab) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npp) return;
  int sa = pp_sa[i], sb = pp_sb[i];
  int ka = shell_first[sa] + pp_ia[i];
  int kb = shell_first[sb] + pp_ib[i];
  double a = exps[ka], b = exps[kb];
  const double *A = xyz + 3 * shell_center[sa];
  const double *B = xyz + 3 * shell_center[sb];
  double pp = a + b;
  ea[i] = a;
  eb[i] = b;
  p[i] = pp;
  Px[i] = (a * A[0] + b * B[0]) / pp;
  Py[i] = (a * A[1] + b * B[1]) / pp;
  Pz[i] = (a * A[2] + b * B[2]) / pp;
  cab[i] = coefs[ka] * coefs[kb];
}

// ---------------------------------------------------------------------------
// Auxiliary functions W_a(X) = R int_0^inf t^a exp(-(t - X)^2) dt, i.e.
// exp(-X^2) S(a, 2X, 1) with S of Eq. (sila).  From the family table by
//   W_a(X_g + d) = exp(-2 X_g d - d^2) sum_k W_{a+k}(X_g) (2d)^k / k!
// (d/dy Phi_a(y) = Phi_{a+1}(y), Phi_a(y) = R int t^a e^{y t - t^2} dt), or for
// X >= WX_HI by the Laplace expansion about the peak t = X:
//   W_a(X) = sqrt(pi) X^a sum_k C(a, 2k) (2k-1)!! / (2 X^2)^k.
// ---------------------------------------------------------------------------
__device__ double w_asym(double a, double X) {
  double inv2x2 = 0.5 / (X * X);
  double term = 1.0, sum = 1.0;
  for (int k = 0; k < 80; ++k) {
    term *= (a - 2 * k) * (a - 2 * k - 1) / (2.0 * k + 2.0) * inv2x2;
    sum += term;
    if (fabs(term) < 1e-18 * fabs(sum)) break;
  }
  return F12_SQRTPI * pow(X, a) * sum;
}


// ---------------------------------------------------------------------------
// Radial derivatives A_n = D^n B_i / N', D = R^-1 d/dR, n = 0..L.
//
// Large-T route (binary64).  For one kernel term c r^alpha e^{b r - g r^2},
// completing the square in Eq. (bfinal) gives
//   B_t / N' = c [F(R) - F(-R)] / R,  F(x) = E(x) Omega_alpha(kappa x + c_s),
//   E(x) = exp(b^2/(4 gam) + b kappa x - (xi g/gam) x^2),
//   Omega_a(y) = R int_0^inf r^a e^{-gam (r - y)^2} dr = gam^{-(a+1)/2} W_a(sqrt(gam) y),
// gam = xi + g, kappa = xi/gam, c_s = b/(2 gam).  The R-derivatives are taken
// on the kernel side: integrating by parts, Omega_a' = a Omega_{a-1} (the
// finite part drops the boundary term for non-integer a; for an integer a >= 0
// Omega_a^(a+1) = a! exp(-gam y^2)).  This lowering form has no cancellation
// at large T, unlike raising the derivative onto the Gaussian (the split
// H-recursion of Eq. (finalrec), which cancels like (2T)^n/(2n-1)!! in
// binary64).  D^n(phi/R) is then formed from the R-jet of phi.
// ---------------------------------------------------------------------------

// W~_m(X) = e^{X^2} W_m(X), m = mlo..mhi (integer m >= 0), for X < WX_LO, the
// region below the tables that decaying chains (b < 0) reach: their F(+-R)
// is e^{-T} W~ there, since E(x) e^{-gam y^2} = e^{-xi x^2} exactly.  W_m is
// the minimal solution of W_{m+1} = X W_m + (m/2) W_{m-1} for X < 0 (the
// other solution integrates over (-inf, 0] and is larger by ~e^{X^2}); the
// recurrence runs downward from mhi + 40, where the ratio of the two
// solutions changes by ~2 X^2 / m > 4 per order, and W~_0 =
// sqrt(pi)/2 erfcx(-X) fixes the scale.  Om[m - mlo] = gp isq^(m - mlo) W~_m.
__device__ inline void w_far_scaled(double X, int mlo, int mhi, double gp, double isq, double *Om) {
  double wa = 0.0, wb = 1.0;  // W~_{m+1}, W~_m at m = top (up to a common scale)
  for (int m = mhi + 40; m >= 1; --m) {
    if (m <= mhi && m >= mlo) Om[m - mlo] = wb;
    const double wn = (2.0 / m) * (wa - X * wb);  // W~_{m-1}
    wa = wb;
    wb = wn;
    const double sc = fabs(wb) > 1e200 ? 1e-200 : (fabs(wb) < 1e-200 ? 1e200 : 1.0);
    if (sc != 1.0) {
      wa *= sc;
      wb *= sc;
      for (int k = m - 1 < mlo ? mlo : m - 1; k <= mhi; ++k)
        if (k >= m) Om[k - mlo] *= sc;
    }
  }
  if (mlo == 0) Om[0] = wb;
  const double lam = 0.5 * F12_SQRTPI * erfcx(-X) / wb;
  double g = gp * lam;
  for (int m = mlo; m <= mhi; ++m) {
    Om[m - mlo] *= g;
    g *= isq;
  }
}

// H ("heavy"): the kernel has negative integer powers (finite parts with log
// terms) or chains whose orders span more than NW_LIGHT; a uniform property
// of the kernel, so each launch takes one instantiation, and the common
// kernels carry neither that code nor its larger private arrays.
template <bool H>
__device__ void aux_large(const KernelDev *__restrict__ K, double xi, double R, int L,
                          double mbudget, double *A) {
  double phi[LTOT_MAX + 1];
  for (int m = 0; m <= L; ++m) phi[m] = 0.0;
  const int nchains = K->nchains;
  // minus sides: per chain, or, for a kernel with finite parts, for every
  // chain once any needs it (the pieces at r ~ 0 cancel only across chains)
  const double T = xi * R * R;
  bool any_minus = false;
  if (K->singular)
    for (int c = 0; c < nchains; ++c) any_minus |= T * (xi / (xi + K->chains[c].g)) < mbudget;
  for (int c = 0; c < nchains; ++c) {
    const ChainDesc ch = K->chains[c];
    const FamilyDesc F = K->fam[ch.family];
    const double g = ch.g, b = ch.b;
    const double gam = xi + g;
    const double kap = xi / gam;
    const double cs = b / (2.0 * gam);
    const double a1 = b * kap;
    const double a2 = xi * g / gam;
    const double e0 = b * b / (4.0 * gam);
    const double sqg = sqrt(gam);
    const double isq = 1.0 / sqg;
    const double g0 = pow(gam, -0.5 * (F.alpha0 + 1.0));
    int mlo = ch.m_min - L;
    if (F.is_int && ch.m_min >= 0 && mlo < 0) mlo = 0;
    const int mhi = ch.m_max;
    // negative integer powers: finite parts in r, Omega_{-n}(y) =
    // gam^{(n-1)/2} W_{-n}(sqrt(gam) y) - (1/2) log(gam) h_{n-1}(y), with
    // h_m(y) = [r^m] e^{-gam (r - y)^2} = gam^{m/2} e^{-X^2} Hphys_m(X) / m!
    const bool negint = H && F.is_int && ch.m_min < 0;
    const double hlg = negint ? 0.5 * log(gam) : 0.0;
    // a decaying chain's sides compare as exp(-X_+^2), X_+ = sqrt(gam) (kappa R + c_s),
    // and are alike once X_+ < 0 (the pair Gaussian's centre inside the decay length)
    const double Xp = sqg * (kap * R + cs);
    const bool do_minus = K->singular ? any_minus
                          : (H && b < 0.0 ? (Xp < 0.0 || Xp * Xp < mbudget) : kap * T < mbudget);
    for (int sgn = 1; sgn >= -1; sgn -= 2) {
      if (sgn < 0 && !do_minus) break;
      const double x = sgn * R;
      const double y = kap * x + cs;
      const double X = sqg * y;
      const bool far = H && b < 0.0 && X < WX_LO;  // decaying chain below the tables
      if (sgn < 0 && X < WX_LO && !far) break;     // below exp(-110) of this chain's F(R)
      const double E = far ? exp(-xi * x * x) : exp(e0 + a1 * x - a2 * x * x);
      double Om[H ? NW_MAX : NW_LIGHT];
      {
        // gam^{-(alpha0+m+1)/2} = g0 * isq^m
        double gp = g0;
        if (mlo >= 0) {
          for (int i = 0; i < mlo; ++i) gp *= isq;
        } else {
          for (int i = 0; i < -mlo; ++i) gp *= sqg;
        }
        if (far) {
          w_far_scaled(X, mlo, mhi, gp, isq, Om);
        } else if (X >= WX_HI) {
          for (int m = mlo; m <= mhi; ++m) {
            Om[m - mlo] = gp * w_asym(F.alpha0 + m, X);
            gp *= isq;
          }
        } else {
          // one grid point and one exp factor for every order m
          const double xs = (X - WX_LO) * WX_INVH;
          int ix = (int)rint(xs);
          ix = ix < 0 ? 0 : (ix >= F.nx ? F.nx - 1 : ix);
          const double Xg = WX_LO + ix * (1.0 / WX_INVH);
          const double d = X - Xg;
          const double ef = exp(-d * (2.0 * Xg + d));
          const double td = 2.0 * d;
          const double *row = F.table + (int64_t)ix * F.nm - F.m_lo;
          // a window of KT + 1 entries slides along the row: each entry is
          // read once (order m takes entries m .. m + KT)
          double w[KT + 1];
#pragma unroll
          for (int k = 0; k <= KT; ++k) w[k] = row[mlo + k];
          for (int m = mlo; m <= mhi; ++m) {
            double sm = w[KT];
#pragma unroll
            for (int k = KT; k >= 1; --k) sm = fma(sm, td * (1.0 / k), w[k - 1]);
            Om[m - mlo] = gp * ef * sm;
            gp *= isq;
            if (m < mhi) {
#pragma unroll
              for (int k = 0; k < KT; ++k) w[k] = w[k + 1];
              w[KT] = row[m + 1 + KT];
            }
          }
        }
      }
      // h_m(y), m = 0..-mlo (negative integer powers only)
      double hh[H ? NW_MAX + 1 : 1];
      if (negint) {
        const double eX = exp(-X * X);
        double q0 = 1.0, q1 = 2.0 * X, gpw = 1.0;
        const double sg = sqrt(gam);
        for (int m = 0; m <= -mlo; ++m) {
          const double qm = m == 0 ? q0 : q1;
          hh[m] = gpw * eX * qm;
          if (m >= 1) {
            const double q2 = (2.0 * X * q1 - 2.0 * q0) / (m + 1);
            q0 = q1;
            q1 = q2;
          }
          gpw *= sg;
        }
        for (int m = mlo; m < 0 && m <= mhi; ++m) Om[m - mlo] -= hlg * hh[-m - 1];
      }
      double Z[LTOT_MAX + 1];
      for (int k = 0; k <= L; ++k) Z[k] = 0.0;
      for (int t = ch.t_begin; t < ch.t_end; ++t) {
        const double ct = K->terms[t].c;
        const int mt = K->terms[t].m;
        const double al = F.alpha0 + mt;
        if (H && F.is_int && mt < 0) {
          // d^k/dy^k Omega_{-n} = (-1)^k (n+k-1)!/(n-1)! [Omega_{-n-k}
          //   - (sum_{j<k} 1/(n+j)) h_{n+k-1}]  (Omega'_{-n} = -n Omega_{-n-1} + h_n,
          // h_m' = -(m+1) h_{m+1})
          const int n = -mt;
          double pf = 1.0, hs = 0.0;
          for (int k = 0; k <= L; ++k) {
            Z[k] += ct * pf * (Om[mt - k - mlo] - hs * hh[n + k - 1]);
            pf *= -(double)(n + k);
            hs += 1.0 / (n + k);
          }
          continue;
        }
        double ff = 1.0;
        int klow = L;
        if (F.is_int && mt < L) klow = mt;
        for (int k = 0; k <= klow; ++k) {
          Z[k] += ct * ff * Om[mt - k - mlo];
          ff *= (al - k);
        }
        if (F.is_int && mt < L) {
          // Omega_mt^(mt+1+j)(y) = mt! d^j/dy^j exp(-gam y^2) = mt! e^{-gam y^2} Q_j(y)
          double fact = 1.0;
          for (int i = 2; i <= mt; ++i) fact *= i;
          const double eg = ct * fact * (far ? 1.0 : exp(-gam * y * y));  // far: scaled by e^{X^2}
          double q0 = 1.0, q1 = -2.0 * gam * y;
          for (int k = mt + 1; k <= L; ++k) {
            const int j = k - mt - 1;
            double qj;
            if (j == 0) {
              qj = q0;
            } else if (j == 1) {
              qj = q1;
            } else {
              double q2 = -2.0 * gam * y * q1 - 2.0 * gam * (j - 1) * q0;
              q0 = q1;
              q1 = q2;
              qj = q2;
            }
            Z[k] += eg * qj;
          }
        }
      }
      // E^(j)(x) = E P_j(x): P_{j+1} = (a1 - 2 a2 x) P_j - 2 a2 j P_{j-1}
      double P[LTOT_MAX + 1], kp[LTOT_MAX + 1];
      P[0] = 1.0;
      kp[0] = 1.0;
      const double slope = a1 - 2.0 * a2 * x;
      if (L >= 1) {
        P[1] = slope;
        kp[1] = kap;
      }
      for (int j = 1; j < L; ++j) {
        P[j + 1] = slope * P[j] - 2.0 * a2 * j * P[j - 1];
        kp[j + 1] = kp[j] * kap;
      }
      for (int m = 0; m <= L; ++m) {
        double G = 0.0, binom = 1.0;
        for (int j = 0; j <= m; ++j) {
          G += binom * P[j] * kp[m - j] * Z[m - j];
          binom = binom * (m - j) / (j + 1);
        }
        G *= E;
        if (sgn > 0)
          phi[m] += G;
        else
          phi[m] -= (m & 1) ? -G : G;
      }
    }
  }
  // D^n (phi / R) from the R-jet f_k = phi^(k)/k!:  g = f/(R + h), then
  // repeatedly differentiate the jet and divide by (R + h).
  double gj[LTOT_MAX + 1];
  double fk = 1.0;
  double prev = 0.0;
  const double iR = 1.0 / R;
  for (int k = 0; k <= L; ++k) {
    if (k > 0) fk /= k;
    prev = (phi[k] * fk - prev) * iR;
    gj[k] = prev;
  }
  A[0] = gj[0];
  for (int n = 1; n <= L; ++n) {
    double pv = 0.0;
    for (int k = 0; k <= L - n; ++k) {
      double d = (k + 1) * gj[k + 1];
      pv = (d - pv) * iR;
      gj[k] = pv;
    }
    A[n] = gj[0];
  }
}

// The large-T route of the common kernels (compact: not heavy, every chain
// spanning at most SPAN_C orders) with L fixed at compile time: the same
// formulas as aux_large<false>, arranged so that every array index is a
// compile-time constant once the loops are unrolled, and the W orders, the
// E-polynomials, phi and the R-jet stay in registers.  Orders are held for
// m = m_min - L .. m_min - L + NO - 1 of each chain; those a chain does not
// use are left at zero.
__device__ __noinline__ double w_asym_call(double a, double X) { return w_asym(a, X); }

template <int L>
__device__ __forceinline__ void aux_large_c(const KernelDev *__restrict__ K, double xi, double R,
                                            double mbudget, double (&A)[L + 1]) {
  constexpr int NO = L + SPAN_C + 1;
  double phi[L + 1];
#pragma unroll
  for (int m = 0; m <= L; ++m) phi[m] = 0.0;
  const int nchains = K->nchains;
  const double T = xi * R * R;
  bool any_minus = false;
  if (K->singular)
    for (int c = 0; c < nchains; ++c) any_minus |= T * (xi / (xi + K->chains[c].g)) < mbudget;
  for (int c = 0; c < nchains; ++c) {
    const ChainDesc ch = K->chains[c];
    const FamilyDesc F = K->fam[ch.family];
    const double g = ch.g, b = ch.b;
    const double gam = xi + g;
    const double kap = xi / gam;
    const double cs = b / (2.0 * gam);
    const double a1 = b * kap;
    const double a2 = xi * g / gam;
    const double e0 = b * b / (4.0 * gam);
    const double sqg = sqrt(gam);
    const double isq = 1.0 / sqg;
    const double g0 = pow(gam, -0.5 * (F.alpha0 + 1.0));
    const int m0 = ch.m_min - L;  // order held in Om[0]
    // orders below zero of an integer family with m_min >= 0 are not needed
    const int ilo = (F.is_int && ch.m_min >= 0 && m0 < 0) ? -m0 : 0;
    const int ihi = ch.m_max - m0;
    // gam^{-(alpha0 + m + 1)/2} at m = m0
    double gp0 = g0;
    if (m0 >= 0) {
      for (int i = 0; i < m0; ++i) gp0 *= isq;
    } else {
      for (int i = 0; i < -m0; ++i) gp0 *= sqg;
    }
    const bool do_minus = K->singular ? any_minus : kap * T < mbudget;
    for (int sgn = 1; sgn >= -1; sgn -= 2) {
      if (sgn < 0 && !do_minus) break;
      const double x = sgn * R;
      const double y = kap * x + cs;
      const double X = sqg * y;
      if (sgn < 0 && X < WX_LO) break;  // below exp(-110) of this chain's F(R)
      const double E = exp(e0 + a1 * x - a2 * x * x);
      double Om[NO];
      {
        double gp = gp0;
        if (X >= WX_HI) {
#pragma unroll
          for (int i = 0; i < NO; ++i) {
            Om[i] = (i >= ilo && i <= ihi) ? gp * w_asym_call(F.alpha0 + m0 + i, X) : 0.0;
            gp *= isq;
          }
        } else {
          const double xs = (X - WX_LO) * WX_INVH;
          int ix = (int)rint(xs);
          ix = ix < 0 ? 0 : (ix >= F.nx ? F.nx - 1 : ix);
          const double Xg = WX_LO + ix * (1.0 / WX_INVH);
          const double d = X - Xg;
          const double ef = exp(-d * (2.0 * Xg + d));
          const double td = 2.0 * d;
          const double *row = F.table + (int64_t)ix * F.nm - F.m_lo + m0;
          // each table entry of the row is read once (order i takes entries
          // i .. i + KT, so neighbouring orders share all but one)
          double seg[NO + KT];
#pragma unroll
          for (int j = 0; j < NO + KT; ++j) seg[j] = (j >= ilo && j <= ihi + KT) ? row[j] : 0.0;
#pragma unroll
          for (int i = 0; i < NO; ++i) {
            double v = 0.0;
            if (i >= ilo && i <= ihi) {
              double sm = seg[i + KT];
#pragma unroll
              for (int k = KT; k >= 1; --k) sm = fma(sm, td * (1.0 / k), seg[i + k - 1]);
              v = gp * ef * sm;
            }
            Om[i] = v;
            gp *= isq;
          }
        }
      }
      // Z_k = sum_t c_t d^k/dy^k Omega_{alpha_t}(y), each term's orders picked
      // by its offset d_t = m_t - m_min through a uniform branch
      double Z[L + 1];
#pragma unroll
      for (int k = 0; k <= L; ++k) Z[k] = 0.0;
      for (int t = ch.t_begin; t < ch.t_end; ++t) {
        const double ct = K->terms[t].c;
        const int mt = K->terms[t].m;
        const int dt = mt - ch.m_min;
        const double al = F.alpha0 + mt;
        const int klow = (F.is_int && mt < L) ? mt : L;
#pragma unroll
        for (int dd = 0; dd <= SPAN_C; ++dd) {
          if (dd == dt) {
            double ff = 1.0;
#pragma unroll
            for (int k = 0; k <= L; ++k) {
              if (k <= klow) Z[k] += ct * ff * Om[dd + L - k];
              ff *= (al - k);
            }
          }
        }
        if (F.is_int && mt < L) {
          // Omega_mt^(mt+1+j)(y) = mt! e^{-gam y^2} Q_j(y)
          double fact = 1.0;
          for (int i = 2; i <= mt; ++i) fact *= i;
          const double eg = ct * fact * exp(-gam * y * y);
          double q0 = 1.0, q1 = -2.0 * gam * y;
#pragma unroll
          for (int k = 1; k <= L; ++k) {
            if (k > mt) {
              const int j = k - mt - 1;
              double qj;
              if (j == 0) {
                qj = q0;
              } else if (j == 1) {
                qj = q1;
              } else {
                const double q2 = -2.0 * gam * y * q1 - 2.0 * gam * (j - 1) * q0;
                q0 = q1;
                q1 = q2;
                qj = q2;
              }
              Z[k] += eg * qj;
            }
          }
        }
      }
      // kappa^k Z_k, and E^(j)(x) = E P_j(x): P_{j+1} = (a1 - 2 a2 x) P_j - 2 a2 j P_{j-1}
      {
        double kp = 1.0;
#pragma unroll
        for (int k = 1; k <= L; ++k) {
          kp *= kap;
          Z[k] *= kp;
        }
      }
      double P[L + 1];
      P[0] = 1.0;
      const double slope = a1 - 2.0 * a2 * x;
      if constexpr (L >= 1) P[1] = slope;
#pragma unroll
      for (int j = 1; j < L; ++j) P[j + 1] = slope * P[j] - 2.0 * a2 * j * P[j - 1];
#pragma unroll
      for (int m = 0; m <= L; ++m) {
        double G = 0.0, binom = 1.0;
#pragma unroll
        for (int j = 0; j <= m; ++j) {
          G += binom * P[j] * Z[m - j];
          binom = binom * (m - j) / (j + 1);
        }
        G *= E;
        if (sgn > 0)
          phi[m] += G;
        else
          phi[m] -= (m & 1) ? -G : G;
      }
    }
  }
  // D^n (phi / R) from the R-jet, as in aux_large
  double gj[L + 1];
  double fk = 1.0;
  double prev = 0.0;
  const double iR = 1.0 / R;
#pragma unroll
  for (int k = 0; k <= L; ++k) {
    if (k > 0) fk /= k;
    prev = (phi[k] * fk - prev) * iR;
    gj[k] = prev;
  }
  A[0] = gj[0];
#pragma unroll
  for (int n = 1; n <= L; ++n) {
    double pv = 0.0;
#pragma unroll
    for (int k = 0; k <= L - n; ++k) {
      const double d = (k + 1) * gj[k + 1];
      pv = (d - pv) * iR;
      gj[k] = pv;
    }
    A[n] = gj[0];
  }
}

// ---------------------------------------------------------------------------
// Small-T route (double-double).  The corrected series of Eq. (biqsmall)
// (factor 4 pi, not 2 pi):
//   B_i / N' = 4 xi exp(-xi u) sum_j (4 xi^2)^j / (2j+1)! M_j,  u = R^2,
//   M_j = int_0^inf k_i(r) r^(2j+2) e^{-xi r^2} dr = sum_t c_t S(alpha_t + 2j + 1, b_t, g_t + xi),
// A_n = D^n B = 2^n d^n B / du^n from the u-jet of P(u) = sum_j a_j u^j
// (Horner Taylor shift) times the jet of exp(-xi u).  The S ladder of each
// chain starts from S(a_s), S(a_s + 1), a_s = alpha0 + m_min + 1 > -1, with
// S(a, b, gam) = gam^{-(a+1)/2} Phi_a(b / sqrt(gam)),
// Phi_a(y) = sum_k Gamma((a+k+1)/2)/(2 k!) y^k, and rises by the integration-
// by-parts relation of Eq. (Srec1): 2 gam S(a+1) = a S(a-1) + b S(a)
// (stable upward for b >= 0).  DD absorbs the exp(2T)-scale cancellation.
// ---------------------------------------------------------------------------
// terms of the u-series: L + 24 + 4T, at most 112 (heavy kernels, T < 14) or
// 64 (the others, T < 6)
constexpr int JMAX_HEAVY = 112, JMAX_LIGHT = 64;

// Decaying chains (b < 0, integer alpha family with m_min >= 0).  With b < 0,
// S(a, b, gam) is the minimal solution of 2 gam S(a+2) = (a+1) S(a) + b S(a+1):
// the other solution, the integral over (-inf, 0], is (-1)^a S(a, -b, gam),
// larger by ~exp(2 |b| r*) at the integrand's peak r*.  Upward the ladder
// then loses a factor of up to exp(y^2/2) (y = b/sqrt(gam)), and the Phi
// series of its start values, whose sum is only ~|y|^-(a+1) for y < 0, keeps
// a truncation tail ~|y|^KPHI / Gamma(KPHI/2) relative to terms of order
// one.  Up to |y| = Y_UPWARD both stay far below 1e-20 and the upward ladder
// of the other chains is used.  Beyond it the ladder runs downward (Miller): first
// from an order far above the top with arbitrary start values down to order
// 0, where S(0) = 1/2 sqrt(pi/gam) erfcx(|y|/2) fixes the scale (the Miller
// ratios converge like exp(-|y| / sqrt(2a)) per order at order a), then
// from the top with the normalised values, adding each S to the M_j it
// belongs to.  The normalisation is one factor for the whole chain, so its
// binary64 accuracy is not amplified by the cancellation of the u-series.
constexpr double Y_UPWARD = 3.0;

__device__ inline void small_ladder_down(const KernelDev *__restrict__ K, const ChainDesc &ch, double b,
                                         dd gam, dd y, double as, int kmax, int J, dd *M) {
  const int ks = (int)as;  // a_s = m_min + 1 >= 1 (integer family)
  const double ay = -y.hi;
  int extra = (int)(48.0 * sqrt(2.0 * (ks + kmax + 1)) / ay) + 8;
  if (extra > 600) extra = 600;
  // pass 1: orders ks + kmax + extra + 1 .. 0
  const double big = 0x1p600, small = 0x1p-600;
  dd sa = dd_make(0.0), sb = dd_make(1.0);  // S(o + 1), S(o) at o = top
  dd rec0 = dd_make(0.0), rec1 = dd_make(0.0);  // S(ks + kmax), S(ks + kmax + 1)
  const dd g2 = dd_mul(gam, 2.0);
  for (int o = ks + kmax + extra; o >= 1; --o) {
    if (o == ks + kmax + 1) rec1 = sb;
    if (o == ks + kmax) rec0 = sb;
    // S(o - 1) = (2 gam S(o + 1) - b S(o)) / o
    const dd sn = dd_div(dd_sub(dd_mul(g2, sa), dd_mul(sb, b)), (double)o);
    sa = sb;
    sb = sn;
    const double sc = fabs(sb.hi) > big ? small : (fabs(sb.hi) < small && sb.hi != 0.0 ? big : 1.0);
    if (sc != 1.0) {
      sa = dd_mul(sa, sc);
      sb = dd_mul(sb, sc);
      rec0 = dd_mul(rec0, sc);
      rec1 = dd_mul(rec1, sc);
    }
  }
  // sb = S(0) up to the common scale
  const double z = 0.5 * ay;
  const dd s0 = dd_mul(dd_div(dd_sqrt(dd_div(dd_make(F12_PI), gam)), 2.0), erfcx(z));
  const dd lam = dd_div(s0, sb);
  dd Sk = dd_mul(rec0, lam), Snext = dd_mul(rec1, lam);  // S(a_s + k), S(a_s + k + 1) at k = kmax
  // pass 2: k = kmax .. 0, each S(a_s + k) into the M_j of its terms
  for (int k = kmax; k >= 0; --k) {
    for (int t = ch.t_begin; t < ch.t_end; ++t) {
      const int dk = k - (K->terms[t].m - ch.m_min);
      if (dk >= 0 && !(dk & 1) && (dk >> 1) <= J)
        M[dk >> 1] = dd_add(M[dk >> 1], dd_mul(Sk, dd{K->terms[t].c, K->terms[t].clo}));
    }
    const dd sp = dd_div(dd_sub(dd_mul(g2, Snext), dd_mul(Sk, b)), as + k);  // S(a_s + k - 1)
    Snext = Sk;
    Sk = sp;
  }
}

template <bool H>
__device__ void aux_small(const KernelDev *__restrict__ K, double xi, double u, int L, double T,
                          double *A, int Jset = 0) {
  constexpr int JM = H ? JMAX_HEAVY : JMAX_LIGHT;
  int J = Jset > 0 ? Jset : L + 24 + (int)(4.0 * T);
  if (J > JM) J = JM;
  dd M[JM + 1];
  for (int j = 0; j <= J; ++j) M[j] = dd{0.0, 0.0};
  const int nchains = K->nchains;
  for (int c = 0; c < nchains; ++c) {
    const ChainDesc ch = K->chains[c];
    const FamilyDesc F = K->fam[ch.family];
    const double b = ch.b;
    const dd gam = two_sum(xi, ch.g);
    const dd sg = dd_sqrt(gam);
    const dd y = (b == 0.0) ? dd{0.0, 0.0} : dd_div(dd_make(b), sg);
    const double as = F.alpha0 + ch.m_min + 1;
    const dd lg = dd_log(gam);
    const dd p0 = dd_exp(dd_mul(lg, -0.5 * (as + 1.0)));
    const dd p1 = dd_div(p0, sg);
    const double *ph = K->phi + 2 * (ch.phi_off);
    dd f0 = dd{ph[2 * KPHI], ph[2 * KPHI + 1]};
    dd f1 = dd{ph[2 * (KPHI + 1) + 2 * KPHI], ph[2 * (KPHI + 1) + 2 * KPHI + 1]};
    if (b != 0.0) {
      for (int k = KPHI - 1; k >= 0; --k) {
        f0 = dd_add(dd_mul(f0, y), dd{ph[2 * k], ph[2 * k + 1]});
        f1 = dd_add(dd_mul(f1, y), dd{ph[2 * (KPHI + 1) + 2 * k], ph[2 * (KPHI + 1) + 2 * k + 1]});
      }
    } else {
      f0 = dd{ph[0], ph[1]};
      f1 = dd{ph[2 * (KPHI + 1)], ph[2 * (KPHI + 1) + 1]};
    }
    dd Sm1 = dd_mul(p0, f0);  // S(a_s)
    dd S0 = dd_mul(p1, f1);   // S(a_s + 1)
    // integer a_s <= -1 (negative powers): finite parts in r, with the
    // Taylor coefficients f_m = [r^m] e^{b r - gam r^2},
    // (m+1) f_{m+1} = b f_m - 2 gam f_{m-1}:
    //   S(-n) = gam^{(n-1)/2} Phi_{-n}(b / sqrt(gam)) - (1/2) log(gam) f_{n-1},
    // and the ladder gains + f_{-a} at every integer a <= 0 (the boundary term
    // of the integration by parts)
    const bool negint = H && F.is_int && ch.m_min < 0;
    const int nneg = negint ? -(ch.m_min + 1) : -1;  // -a_s
    dd fm[H ? NEG_POW_MAX + 2 : 1];
    if (negint) {
      fm[0] = dd_make(1.0);
      if (nneg + 1 >= 1) fm[1] = dd_make(b);
      for (int m = 1; m < nneg + 1; ++m)
        fm[m + 1] = dd_div(dd_sub(dd_mul(fm[m], b), dd_mul(dd_mul(fm[m - 1], gam), 2.0)), (double)(m + 1));
      const dd hl = dd_mul(lg, 0.5);
      if (nneg >= 1) Sm1 = dd_sub(Sm1, dd_mul(hl, fm[nneg - 1]));
      if (nneg >= 2) S0 = dd_sub(S0, dd_mul(hl, fm[nneg - 2]));
    }
    const dd inv2g = dd_div(dd_make(0.5), gam);
    const int span = ch.m_max - ch.m_min;
    const int kmax = span + 2 * J;
    if (H && b < 0.0 && -y.hi > Y_UPWARD) {
      small_ladder_down(K, ch, b, gam, y, as, kmax, J, M);
      continue;
    }
    dd Sk = Sm1, Snext = S0;
    for (int k = 0; k <= kmax; ++k) {
      // Sk = S(a_s + k)
      for (int t = ch.t_begin; t < ch.t_end; ++t) {
        const int off = K->terms[t].m - ch.m_min;
        const int dk = k - off;
        if (dk >= 0 && !(dk & 1)) {
          const int j = dk >> 1;
          if (j <= J) {
            // double-double coefficients where finite parts cancel between chains
            if constexpr (H)
              M[j] = dd_add(M[j], dd_mul(Sk, dd{K->terms[t].c, K->terms[t].clo}));
            else
              M[j] = dd_add(M[j], dd_mul(Sk, K->terms[t].c));
          }
        }
      }
      // advance: S(a_s + k + 2) = ((a_s + k + 1) S(a_s + k) + b S(a_s + k + 1)) / (2 gam)
      dd num = dd_add(dd_mul(Sk, as + k + 1), dd_mul(Snext, b));
      if (negint && nneg - k - 1 >= 0) num = dd_add(num, fm[nneg - k - 1]);
      dd Snn = dd_mul(num, inv2g);
      Sk = Snext;
      Snext = Snn;
    }
  }
  // a_j = (4 xi^2)^j / (2j+1)! M_j
  {
    const dd x4 = dd_mul(dd_mul(dd_make(xi), xi), 4.0);
    dd cj = dd{1.0, 0.0};
    for (int j = 0; j <= J; ++j) {
      M[j] = dd_mul(M[j], cj);
      cj = dd_div(dd_mul(cj, x4), (double)((2 * j + 2) * (2 * j + 3)));
    }
  }
  dd jet[LTOT_MAX + 1];
  for (int k = 0; k <= L; ++k) jet[k] = dd{0.0, 0.0};
  for (int j = J; j >= 0; --j) {
    for (int k = L; k >= 1; --k) jet[k] = dd_add(dd_mul(jet[k], u), jet[k - 1]);
    jet[0] = dd_add(dd_mul(jet[0], u), M[j]);
  }
  // times exp(-xi (u + d)) = e^{-xi u} sum_i (-xi d)^i / i!
  const dd eu = dd_exp(dd_neg(two_prod(xi, u)));
  dd ej[LTOT_MAX + 1];
  ej[0] = eu;
  for (int i = 1; i <= L; ++i) ej[i] = dd_div(dd_mul(ej[i - 1], -xi), (double)i);
  double scale = 4.0 * xi;
  for (int n = 0; n <= L; ++n) {
    dd s = dd{0.0, 0.0};
    for (int i = 0; i <= n; ++i) s = dd_add(s, dd_mul(ej[i], jet[n - i]));
    A[n] = scale * dd_to_double(s);
    scale *= 2.0 * (n + 1);
  }
}

// The same series in binary64, for T < 2 and L <= 5, where the cancellation
// (about e^{2T} and the alternating u-jet product) leaves ~1e-14 of the
// scaled envelope; the S ladders, M_j and the u-jet as in aux_small.
template <bool H>
__device__ void aux_small_f64(const KernelDev *__restrict__ K, double xi, double u, int L,
                              double T, double *A) {
  constexpr int JM = H ? JMAX_HEAVY : JMAX_LIGHT;
  int J = L + 20 + (int)(4.0 * T);
  if (J > JM) J = JM;
  double M[JM + 1];
  for (int j = 0; j <= J; ++j) M[j] = 0.0;
  const int nchains = K->nchains;
  for (int c = 0; c < nchains; ++c) {
    const ChainDesc ch = K->chains[c];
    const FamilyDesc F = K->fam[ch.family];
    const double b = ch.b;
    const double gam = xi + ch.g;
    const double sg = sqrt(gam);
    const double y = b / sg;
    const double as = F.alpha0 + ch.m_min + 1;
    const double p0 = pow(gam, -0.5 * (as + 1.0));
    const double p1 = p0 / sg;
    const double *ph = K->phi + 2 * (ch.phi_off);
    double f0 = ph[2 * KPHI], f1 = ph[2 * (KPHI + 1) + 2 * KPHI];
    if (b != 0.0) {
      for (int k = KPHI - 1; k >= 0; --k) {
        f0 = fma(f0, y, ph[2 * k]);
        f1 = fma(f1, y, ph[2 * (KPHI + 1) + 2 * k]);
      }
    } else {
      f0 = ph[0];
      f1 = ph[2 * (KPHI + 1)];
    }
    double Sk = p0 * f0, Snext = p1 * f1;
    // negative integer powers: finite parts as in aux_small
    const bool negint = H && F.is_int && ch.m_min < 0;
    const int nneg = negint ? -(ch.m_min + 1) : -1;
    double fm[H ? NEG_POW_MAX + 2 : 1];
    if (negint) {
      fm[0] = 1.0;
      if (nneg + 1 >= 1) fm[1] = b;
      for (int m = 1; m < nneg + 1; ++m) fm[m + 1] = (b * fm[m] - 2.0 * gam * fm[m - 1]) / (m + 1);
      const double hl = 0.5 * log(gam);
      if (nneg >= 1) Sk -= hl * fm[nneg - 1];
      if (nneg >= 2) Snext -= hl * fm[nneg - 2];
    }
    const double inv2g = 0.5 / gam;
    const int kmax = ch.m_max - ch.m_min + 2 * J;
    for (int k = 0; k <= kmax; ++k) {
      for (int t = ch.t_begin; t < ch.t_end; ++t) {
        const int dk = k - (K->terms[t].m - ch.m_min);
        if (dk >= 0 && !(dk & 1) && (dk >> 1) <= J) M[dk >> 1] = fma(Sk, K->terms[t].c, M[dk >> 1]);
      }
      double num = (as + k + 1) * Sk + b * Snext;
      if (negint && nneg - k - 1 >= 0) num += fm[nneg - k - 1];
      const double Snn = num * inv2g;
      Sk = Snext;
      Snext = Snn;
    }
  }
  {
    const double x4 = 4.0 * xi * xi;
    double cj = 1.0;
    for (int j = 0; j <= J; ++j) {
      M[j] *= cj;
      cj = cj * x4 / (double)((2 * j + 2) * (2 * j + 3));
    }
  }
  double jet[LTOT_MAX + 1];
  for (int k = 0; k <= L; ++k) jet[k] = 0.0;
  for (int j = J; j >= 0; --j) {
    for (int k = L; k >= 1; --k) jet[k] = fma(jet[k], u, jet[k - 1]);
    jet[0] = fma(jet[0], u, M[j]);
  }
  double ej[LTOT_MAX + 1];
  ej[0] = exp(-xi * u);
  for (int i = 1; i <= L; ++i) ej[i] = ej[i - 1] * (-xi) / (double)i;
  double scale = 4.0 * xi;
  for (int n = 0; n <= L; ++n) {
    double sacc = 0.0;
    for (int i = 0; i <= n; ++i) sacc = fma(ej[i], jet[n - i], sacc);
    A[n] = scale * sacc;
    scale *= 2.0 * (n + 1);
  }
}

// Small-T / large-T switch and the cut for the exp(-xi (r+R)^2) side.
// The lowering route holds ~1e-14 of the (2 xi)^n-scaled envelope of A_n from
// T = 1 (L <= 3), 1.5 (L = 4), 2 (L = 5, 6), 2.5, 3, 3.5, 4, 4.5, 5 (L = 7..12)
// and 6 (L = 13, 14), measured against the DD series, which holds to
// T = 14; below those T the DD series runs.
__device__ __forceinline__ double t_switch(int L) {
  constexpr double sw[LTOT_MAX + 1] = {1.0, 1.0, 1.0, 1.0, 1.5, 2.0, 2.0, 2.5,
                                       3.0, 3.5, 4.0, 4.5, 5.0, 6.0, 6.0};
  return sw[L < 0 ? 0 : (L > LTOT_MAX ? LTOT_MAX : L)];
}
// Kernels with negative integer powers: the finite parts of single terms
// cancel between chains, and the pieces grow like gam^{(n-1)/2} for a power
// r^{-n}; in the lowering route (binary64) that cancellation is damped by
// e^{-T} only, so the double-double series (exact to T = 14, with the
// double-double term coefficients) runs up to T = 14.
// Kernels with decaying chains (b < 0): while the pair Gaussian's centre lies
// inside a chain's decay length (X_+ < 0, 2 xi R < |b|), F(R) and F(-R) are
// both ~e^{-T} and the lowering form's terms b^j Omega^(m-j) exceed their
// sum by up to (|b| / (2 xi R))^m; the double-double series, which needs few
// terms for such short-ranged kernels, runs up to T = 14 for them as well.
constexpr double TSW_NEGINT = 14.0;
__device__ __forceinline__ double t_switch_k(const KernelDev *K, int L) {
  const double sw = t_switch(L);
  return ((K->negint || K->negb) && sw < TSW_NEGINT) ? TSW_NEGINT : sw;
}

// Short-ranged kernels past the switch.  When every chain decays faster than
// the pair Gaussian spreads, the u-series of the small-T route converges at
// any T: for a chain e^{b r} (g = 0, b < 0) its terms fall like
// (2j+2) rho^j, rho = (2 xi R / b)^2 = 4 xi T / b^2; for a chain with a
// Gaussian (g > 0) like (kappa T)^j / j!, kappa = xi / (xi + g).  The sum is
// then O(1) against e^{-T}, so the double-double jet keeps its accuracy.
// This is the regime (2 xi R < |b|) where the lowering form of a decaying
// chain cancels.  Returns the number of series terms, or 0 when a chain is
// long-ranged (g = 0, b >= 0), rho > 1/2, or more than 70 terms would be
// needed (M_j stays within the double range up to there).
__device__ inline int short_range_terms(const KernelDev *__restrict__ K, double xi, double T, int L) {
  double jm = 0.0;
  for (int c = 0; c < K->nchains; ++c) {
    const double g = K->chains[c].g, b = K->chains[c].b;
    double jc;
    if (g == 0.0) {
      if (b >= 0.0) return 0;
      const double rho = 4.0 * xi * T / (b * b);
      if (rho > 0.5) return 0;
      jc = rho > 0.0 ? 46.0 / -log(rho) : 0.0;
    } else {
      const double m = T * xi / (xi + g);
      jc = m + 10.0 * sqrt(m) + 20.0;
    }
    jm = fmax(jm, jc);
  }
  const int J = L + 10 + (int)ceil(jm);
  return J <= 70 ? J : 0;
}

// The F(-R) side of the large-T route.  Against F(R) of its own chain it is
// damped by exp(-kappa T - b kappa R - b^2/(4 gam)) <= exp(-kappa T),
// kappa = xi / (xi + g): the far side of the pair Gaussian meets the kernel
// at r ~ 0, the near side at r ~ kappa R.  For g = 0 (kappa = 1) the plus
// side's A_n can fall like (2n-1)!!/(2T)^n, so a chain keeps its minus side
// while exp(-kappa T) (2T)^L / (2L-1)!! > 1e-19, i.e. kappa T < minus_budget;
// and never where the minus-side argument lies below the W tables, where the
// side is below exp(-110) of its plus side.  Terms r^a with a <= -1 are
// finite parts: a chain's side then holds pieces of size exp(-T) (2 xi R)^k
// from r ~ 0 that cancel only in the sum over chains, so such a kernel takes
// the minus side of every chain or of none.
__device__ __forceinline__ double minus_budget(double T, int L) {
  double lg = 43.7;
  if (L > 0) {
    lg += L * log(2.0 * T);
    for (int k = 3; k <= 2 * L - 1; k += 2) lg -= log((double)k);
  }
  return lg;
}

// ---------------------------------------------------------------------------
// K3/K4: A[n * np + t] = A_n for the primitive quartets of a chunk.  Each
// work-group takes F12_NT_AUX consecutive primitive quartets, computes their
// geometry and T, and hands them out again ordered by route and by octave of
// T (a counting sort in LDS), so that the lanes of a wave mostly take the
// same branch.  Each result is still written to its own slot and does not
// depend on which thread computes it.
// ---------------------------------------------------------------------------
#ifndef F12_NT_AUX
#define F12_NT_AUX 512
#endif
constexpr int AUX_BINS = 16;

__device__ __forceinline__ int aux_bin(double T, int L, double sw) {
  if (T < sw) return (L <= 5 && T < 2.0) ? 0 : 1;
  int e = ilogb(T / sw);  // octave above the switch; NaN and inf are clamped
  e = e < 0 ? 0 : (e > AUX_BINS - 3 ? AUX_BINS - 3 : e);
  return 2 + e;
}

// LC >= 0: the compact kernels with L = LC fixed at compile time (H false).
// Those are held to at most 168 VGPRs (the register budget of three waves per
// SIMD).  A 512-thread work-group still runs two waves per SIMD either way;
// the cap is kept because it was measured faster: with all 256 registers the
// launches take 1.5-1.9x as long, capped at 128 (spilling more) 1.1x.
template <bool H, int LC>
__global__ void __launch_bounds__(F12_NT_AUX) __attribute__((amdgpu_waves_per_eu(LC >= 0 ? 3 : 1)))
aux_kernel(const KernelDev *__restrict__ K, PairsDev bra,
                                                  PairsDev ket, const int64_t *__restrict__ qb,
                                                  const int64_t *__restrict__ qk,
                                                  const int64_t *__restrict__ qprim, int64_t qa,
                                                  int64_t nqc, int64_t p0, int64_t np, int L,
                                                  double *__restrict__ A, int *fault) {
  __shared__ double s_xi[F12_NT_AUX], s_u[F12_NT_AUX], s_np[F12_NT_AUX];
  __shared__ int s_perm[F12_NT_AUX];
  __shared__ int s_cnt[AUX_BINS], s_off[AUX_BINS];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * F12_NT_AUX;
  const int64_t t = base + tid;
  const double sw = t_switch_k(K, L);
  if (tid < AUX_BINS) s_cnt[tid] = 0;
  __syncthreads();
  int bin = AUX_BINS - 1;
  if (t < np) {
    const int64_t gidx = p0 + t;
    int64_t lo = qa, hi = qa + nqc;
    while (hi - lo > 1) {
      int64_t mid = (lo + hi) >> 1;
      if (qprim[mid] <= gidx)
        lo = mid;
      else
        hi = mid;
    }
    const int64_t q = lo;
    const int64_t local = gidx - qprim[q];
    const int64_t bp = qb[q], kp = qk[q];
    const int64_t nk = (int64_t)ket.ka[kp] * ket.kb[kp];
    const int64_t i = local / nk;
    const int64_t j = local - i * nk;
    const int64_t ib = bra.pp_off[bp] + i;
    const int64_t ik = ket.pp_off[kp] + j;
    const double p = bra.p[ib], qq = ket.p[ik];
    const double X = ket.Px[ik] - bra.Px[ib];
    const double Y = ket.Py[ik] - bra.Py[ib];
    const double Z = ket.Pz[ik] - bra.Pz[ib];
    const double u = X * X + Y * Y + Z * Z;
    const double xi = p * qq / (p + qq);
    s_xi[tid] = xi;
    s_u[tid] = u;
    s_np[tid] = F12_PI52 / (sqrt(p + qq) * p * qq);
    bin = aux_bin(xi * u, L, sw);
  }
  const int rank = atomicAdd(&s_cnt[bin], 1);
  __syncthreads();
  if (tid == 0) {
    int s = 0;
    for (int b = 0; b < AUX_BINS; ++b) {
      s_off[b] = s;
      s += s_cnt[b];
    }
  }
  __syncthreads();
  s_perm[s_off[bin] + rank] = tid;
  __syncthreads();
  const int me = s_perm[tid];
  if (base + me >= np) return;
  const double xi = s_xi[me], u = s_u[me], Np = s_np[me];
  const double T = xi * u;
  if constexpr (LC >= 0) {
    double a[LC + 1];
    if (T < sw) {
      double as[LTOT_MAX + 1];
      if (LC <= 5 && T < 2.0)
        aux_small_f64<false>(K, xi, u, LC, T, as);
      else
        aux_small<false>(K, xi, u, LC, T, as);
#pragma unroll
      for (int n = 0; n <= LC; ++n) a[n] = as[n];
    } else {
      aux_large_c<LC>(K, xi, sqrt(u), minus_budget(T, LC), a);
    }
    bool bad = false;
#pragma unroll
    for (int n = 0; n <= LC; ++n) {
      const double v = a[n] * Np;
      bad |= !isfinite(v);
      A[n * np + base + me] = v;
    }
    if (bad) *fault = 1;
    return;
  }
  double a[LTOT_MAX + 1];
  const int Jsr = (H && T >= sw && K->negb) ? short_range_terms(K, xi, T, L) : 0;
  if (T < sw) {
    if (!H && L <= 5 && T < 2.0)
      aux_small_f64<H>(K, xi, u, L, T, a);
    else
      aux_small<H>(K, xi, u, L, T, a);
  } else if (Jsr > 0) {
    aux_small<H>(K, xi, u, L, T, a, Jsr);
  } else {
    aux_large<H>(K, xi, sqrt(u), L, minus_budget(T, L), a);
  }
  bool bad = false;
  for (int n = 0; n <= L; ++n) {
    const double v = a[n] * Np;
    bad |= !isfinite(v);
    A[n * np + base + me] = v;
  }
  if (bad) *fault = 1;
}


// ---------------------------------------------------------------------------
// K5/K6: the Hermite integrals and the E.R.E contraction run in the
// shape-specialised kernels of f12_big.h (instantiated by f12_big_unit.hip).
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
int launch_pair_prims(int64_t npp, const int32_t *pp_sa, const int32_t *pp_sb,
                      const int32_t *pp_ia, const int32_t *pp_ib, const int32_t *shell_first,
                      const int32_t *shell_center, const double *xyz, const double *exps,
                      const double *coefs, double *ea, double *eb, double *p, double *Px,
                      double *Py, double *Pz, double *cab, hipStream_t stream) {
  if (npp <= 0) return 0;
  int nt = 256;
  int64_t nbk = (npp + nt - 1) / nt;
  hipLaunchKernelGGL(pair_prims_kernel, dim3((unsigned)nbk), dim3(nt), 0, stream, npp, pp_sa,
                     pp_sb, pp_ia, pp_ib, shell_first, shell_center, xyz, exps, coefs, ea, eb, p,
                     Px, Py, Pz, cab);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// The compact kernels, one per L, reached through a table of launchers.
using AuxLaunch = void (*)(dim3, hipStream_t, const KernelDev *, PairsDev, PairsDev, const int64_t *,
                           const int64_t *, const int64_t *, int64_t, int64_t, int64_t, int64_t, int, double *,
                           int *);
template <int LC>
static void launch_aux_c(dim3 grid, hipStream_t st, const KernelDev *K, PairsDev bra, PairsDev ket,
                         const int64_t *qb, const int64_t *qk, const int64_t *qprim, int64_t qa, int64_t nqc,
                         int64_t p0, int64_t np, int L, double *A, int *fw) {
  hipLaunchKernelGGL((aux_kernel<false, LC>), grid, dim3(F12_NT_AUX), 0, st, K, bra, ket, qb, qk, qprim, qa, nqc,
                     p0, np, L, A, fw);
}
template <int... Ls>
static const AuxLaunch *aux_table_of(std::integer_sequence<int, Ls...>) {
  static const AuxLaunch t[] = {&launch_aux_c<Ls>...};
  return t;
}
static const AuxLaunch *compact_aux_table() {
  return aux_table_of(std::make_integer_sequence<int, LTOT_MAX + 1>{});
}

int launch_aux(const KernelDev *K, const PairsDev &bra, const PairsDev &ket, const int64_t *qb,
               const int64_t *qk, const int64_t *qprim, int64_t qa, int64_t nqc, int64_t p0,
               int64_t np, int L, double *A, hipStream_t stream, int variant) {
  if (np <= 0) return 0;
  int *fw = fault_word();
  if (!fw) return -1;
  const int64_t nbk = (np + F12_NT_AUX - 1) / F12_NT_AUX;
  if (variant == 2 && L >= 0 && L <= LTOT_MAX) {
    compact_aux_table()[L](dim3((unsigned)nbk), stream, K, bra, ket, qb, qk, qprim, qa, nqc, p0, np, L, A, fw);
  } else if (variant == 1) {
    hipLaunchKernelGGL((aux_kernel<true, -1>), dim3((unsigned)nbk), dim3(F12_NT_AUX), 0, stream, K, bra, ket,
                       qb, qk, qprim, qa, nqc, p0, np, L, A, fw);
  } else {
    hipLaunchKernelGGL((aux_kernel<false, -1>), dim3((unsigned)nbk), dim3(F12_NT_AUX), 0, stream, K, bra, ket,
                       qb, qk, qprim, qa, nqc, p0, np, L, A, fw);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// One launcher per (l_a + l_b, ket precision), each built in a translation
// unit of its own from f12_big_unit.hip.
template <int LAB, int PREC>
int launch_big_unit(int lcd, int i5, const ContractArgs &a, unsigned nblocks, hipStream_t st);
#define F12_UNIT(L)                                                                             \
  template <> int launch_big_unit<L, 0>(int, int, const ContractArgs &, unsigned, hipStream_t); \
  template <> int launch_big_unit<L, 1>(int, int, const ContractArgs &, unsigned, hipStream_t);
F12_UNIT(0) F12_UNIT(1) F12_UNIT(2) F12_UNIT(3) F12_UNIT(4) F12_UNIT(5) F12_UNIT(6)
#undef F12_UNIT

template <int PREC>
static int launch_big_p(int lab, int lcd, int i5, const ContractArgs &a, unsigned nb, hipStream_t st) {
  switch (lab) {
    case 0: return launch_big_unit<0, PREC>(lcd, i5, a, nb, st);
    case 1: return launch_big_unit<1, PREC>(lcd, i5, a, nb, st);
    case 2: return launch_big_unit<2, PREC>(lcd, i5, a, nb, st);
    case 3: return launch_big_unit<3, PREC>(lcd, i5, a, nb, st);
    case 4: return launch_big_unit<4, PREC>(lcd, i5, a, nb, st);
    case 5: return launch_big_unit<5, PREC>(lcd, i5, a, nb, st);
    case 6: return launch_big_unit<6, PREC>(lcd, i5, a, nb, st);
    default: return -1;
  }
}

static int launch_big(int lab, int lcd, int i5, const ContractArgs &a, unsigned nb, hipStream_t st) {
  return a.prec == 1 ? launch_big_p<1>(lab, lcd, i5, a, nb, st) : launch_big_p<0>(lab, lcd, i5, a, nb, st);
}

int launch_contract(const PairsDev &bra, const PairsDev &ket, const int64_t *qb, const int64_t *qk,
                    const int64_t *qoff, const int64_t *qprim, int64_t qa, int64_t nqc, int64_t p0,
                    int64_t np, const double *A, int la, int lb, int lc, int ld, int i5,
                    double *out, int64_t out_base, hipStream_t stream, int64_t grid, int prec,
                    int gdir) {
  if (nqc <= 0) return 0;
  ContractArgs a;
  a.gdir = gdir;
  a.fault = fault_word();
  if (!a.fault) return -1;
  a.bra = bra;
  a.ket = ket;
  a.qb = qb;
  a.qk = qk;
  a.qoff = qoff;
  a.qprim = qprim;
  a.qa = qa;
  a.nqc = nqc;
  a.p0 = p0;
  a.np = np;
  a.A = A;
  a.la = la;
  a.lb = lb;
  a.lc = lc;
  a.ld = ld;
  a.i5 = i5;
  a.out = out;
  a.out_base = out_base;
  a.prec = prec;
  // grid > 0: persistent work-groups (at most grid of them); grid == 0: one
  // work-group per quartet; grid < 0: set the kernel's attributes only
  const int64_t nb = grid < 0 ? 0 : (grid == 0 ? nqc : (grid < nqc ? grid : nqc));
  return launch_big(la + lb, lc + ld, i5, a, (unsigned)nb, stream);
}

// Diagnostic: A_n for explicit (p, q, R) triples (one thread each), R along z.
__global__ void aux_points_kernel(const KernelDev *__restrict__ K, int64_t n,
                                  const double *__restrict__ pp, const double *__restrict__ qq,
                                  const double *__restrict__ RR, int L, int route,
                                  double *__restrict__ A) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double p = pp[t], q = qq[t], R = RR[t];
  const double u = R * R;
  const double xi = p * q / (p + q);
  const double T = xi * u;
  const double Np = F12_PI52 / (sqrt(p + q) * p * q);
  double a[LTOT_MAX + 1];
  if (route == 3) {
    aux_small_f64<true>(K, xi, u, L, T, a);
    for (int k = 0; k <= L; ++k) A[k * n + t] = a[k] * Np;
    return;
  }
  if (route == 0) {
    // the production dispatch of aux_kernel
    if (K->heavy) {
      const int Jsr = K->negb ? short_range_terms(K, xi, T, L) : 0;
      if (T < t_switch_k(K, L))
        aux_small<true>(K, xi, u, L, T, a);
      else if (Jsr > 0)
        aux_small<true>(K, xi, u, L, T, a, Jsr);
      else
        aux_large<true>(K, xi, R, L, minus_budget(T, L), a);
    } else {
      if (T < t_switch_k(K, L)) {
        if (L <= 5 && T < 2.0)
          aux_small_f64<false>(K, xi, u, L, T, a);
        else
          aux_small<false>(K, xi, u, L, T, a);
      } else {
        aux_large<false>(K, xi, R, L, minus_budget(T, L), a);
      }
    }
    for (int k = 0; k <= L; ++k) A[k * n + t] = a[k] * Np;
    return;
  }
  const bool small = (route == 1) || (route == 0 && T < t_switch_k(K, L));
  // routes 1, 2: one formula forced, with the large arrays
  if (small)
    aux_small<true>(K, xi, u, L, T, a);
  else
    aux_large<true>(K, xi, R, L, 1e300, a);
  for (int k = 0; k <= L; ++k) A[k * n + t] = a[k] * Np;
}

// route 0 of a compact kernel: the dispatch of aux_kernel<false, LC>.
template <int LC>
__global__ void aux_points_c_kernel(const KernelDev *__restrict__ K, int64_t n, const double *__restrict__ pp,
                                    const double *__restrict__ qq, const double *__restrict__ RR,
                                    double *__restrict__ A) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double p = pp[t], q = qq[t], R = RR[t];
  const double u = R * R;
  const double xi = p * q / (p + q);
  const double T = xi * u;
  const double Np = F12_PI52 / (sqrt(p + q) * p * q);
  double a[LC + 1];
  if (T < t_switch_k(K, LC)) {
    double as[LTOT_MAX + 1];
    if (LC <= 5 && T < 2.0)
      aux_small_f64<false>(K, xi, u, LC, T, as);
    else
      aux_small<false>(K, xi, u, LC, T, as);
#pragma unroll
    for (int k = 0; k <= LC; ++k) a[k] = as[k];
  } else {
    aux_large_c<LC>(K, xi, R, minus_budget(T, LC), a);
  }
#pragma unroll
  for (int k = 0; k <= LC; ++k) A[k * n + t] = a[k] * Np;
}

using AuxPointsLaunch = void (*)(dim3, hipStream_t, const KernelDev *, int64_t, const double *, const double *,
                                 const double *, double *);
template <int LC>
static void launch_points_c(dim3 grid, hipStream_t st, const KernelDev *K, int64_t n, const double *p,
                            const double *q, const double *R, double *A) {
  hipLaunchKernelGGL((aux_points_c_kernel<LC>), grid, dim3(128), 0, st, K, n, p, q, R, A);
}
template <int... Ls>
static const AuxPointsLaunch *points_table_of(std::integer_sequence<int, Ls...>) {
  static const AuxPointsLaunch t[] = {&launch_points_c<Ls>...};
  return t;
}

int launch_aux_points(const KernelDev *K, int64_t n, const double *p, const double *q,
                      const double *R, int L, int route, double *A, hipStream_t stream, int variant) {
  if (n <= 0) return 0;
  int nt = 128;
  int64_t nbk = (n + nt - 1) / nt;
  if (route == 0 && variant == 2 && L >= 0 && L <= LTOT_MAX)
    points_table_of(std::make_integer_sequence<int, LTOT_MAX + 1>{})[L](dim3((unsigned)nbk), stream, K, n, p, q,
                                                                         R, A);
  else
    hipLaunchKernelGGL(aux_points_kernel, dim3((unsigned)nbk), dim3(nt), 0, stream, K, n, p, q, R,
                       L, route, A);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace f12
