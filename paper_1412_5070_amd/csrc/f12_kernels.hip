// HIP kernels for gfx950: primitive-pair data, radial derivatives of the
// basic integrals (the auxiliary functions), Hermite integrals R_tuv and the
// E.R.E contraction of the McMurchie-Davidson route of arXiv:1412.5070.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#include "f12_internal.h"
#include "f12_dd.h"
#include "f12_launch.h"

namespace f12 {

#define F12_PI52 17.493418327624862846  // pi^(5/2)
#define F12_SQRTPI 1.7724538509055160273

__device__ __forceinline__ int hsize(int L) { return (L + 1) * (L + 2) * (L + 3) / 6; }
// Hermite index of (t,u,v): by total N = t+u+v, then t descending, then u descending.
__device__ __forceinline__ int ridx(int t, int u, int v) {
  int N = t + u + v;
  int s = N - t;
  return N * (N + 1) * (N + 2) / 6 + s * (s + 1) / 2 + (s - u);
}
__device__ __forceinline__ int ncart(int l) { return (l + 1) * (l + 2) / 2; }
// Canonical Cartesian component c of angular momentum l: (i,k,m), i from l
// down to 0, then k from l-i down to 0.
__device__ __forceinline__ void cart_comp(int l, int c, int &i, int &k, int &m) {
  int ii = l, base = 0;
  while (c >= base + (l - ii + 1)) {
    base += l - ii + 1;
    --ii;
  }
  int kk = (l - ii) - (c - base);
  i = ii;
  k = kk;
  m = l - ii - kk;
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

__device__ __forceinline__ double w_eval(const FamilyDesc &F, int m, double X) {
  if (X >= WX_HI) return w_asym(F.alpha0 + m, X);
  double xs = (X - WX_LO) * WX_INVH;
  int ix = (int)rint(xs);
  ix = ix < 0 ? 0 : (ix >= F.nx ? F.nx - 1 : ix);
  double Xg = WX_LO + ix * (1.0 / WX_INVH);
  double d = X - Xg;
  const double *row = F.table + (int64_t)ix * F.nm + (m - F.m_lo);
  double td = 2.0 * d;
  double s = row[KT];
#pragma unroll
  for (int k = KT; k >= 1; --k) s = fma(s, td * (1.0 / k), row[k - 1]);
  return exp(-d * (2.0 * Xg + d)) * s;
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
#define F12_NW 64

__device__ void aux_large(const KernelDev *__restrict__ K, double xi, double R, int L,
                          bool do_minus, double *A) {
  double phi[LTOT_MAX + 1];
  for (int m = 0; m <= L; ++m) phi[m] = 0.0;
  const int nchains = K->nchains;
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
    if (F.is_int && mlo < 0) mlo = 0;
    const int mhi = ch.m_max;
    for (int sgn = 1; sgn >= -1; sgn -= 2) {
      if (sgn < 0 && !do_minus) break;
      const double x = sgn * R;
      const double y = kap * x + cs;
      const double X = sqg * y;
      const double E = exp(e0 + a1 * x - a2 * x * x);
      double Om[F12_NW];
      {
        // gam^{-(alpha0+m+1)/2} = g0 * isq^m
        double gp = g0;
        if (mlo >= 0) {
          for (int i = 0; i < mlo; ++i) gp *= isq;
        } else {
          for (int i = 0; i < -mlo; ++i) gp *= sqg;
        }
        for (int m = mlo; m <= mhi; ++m) {
          Om[m - mlo] = gp * w_eval(F, m, X);
          gp *= isq;
        }
      }
      double Z[LTOT_MAX + 1];
      for (int k = 0; k <= L; ++k) Z[k] = 0.0;
      for (int t = ch.t_begin; t < ch.t_end; ++t) {
        const double ct = K->terms[t].c;
        const int mt = K->terms[t].m;
        const double al = F.alpha0 + mt;
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
          const double eg = ct * fact * exp(-gam * y * y);
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
#define F12_JMAX 112

__device__ void aux_small(const KernelDev *__restrict__ K, double xi, double u, int L, double T,
                          double *A) {
  int J = L + 24 + (int)(4.0 * T);
  if (J > F12_JMAX) J = F12_JMAX;
  dd M[F12_JMAX + 1];
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
    const dd inv2g = dd_div(dd_make(0.5), gam);
    const int span = ch.m_max - ch.m_min;
    const int kmax = span + 2 * J;
    dd Sk = Sm1, Snext = S0;
    for (int k = 0; k <= kmax; ++k) {
      // Sk = S(a_s + k)
      for (int t = ch.t_begin; t < ch.t_end; ++t) {
        const int off = K->terms[t].m - ch.m_min;
        const int dk = k - off;
        if (dk >= 0 && !(dk & 1)) {
          const int j = dk >> 1;
          if (j <= J) M[j] = dd_add(M[j], dd_mul(Sk, K->terms[t].c));
        }
      }
      // advance: S(a_s + k + 2) = ((a_s + k + 1) S(a_s + k) + b S(a_s + k + 1)) / (2 gam)
      dd Snn = dd_mul(dd_add(dd_mul(Sk, as + k + 1), dd_mul(Snext, b)), inv2g);
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

// Small-T / large-T switch and the cut for the exp(-xi (r+R)^2) side.
// Both routes reach ~1e-15 of the (2 xi)^n-scaled envelope of A_n in an
// overlap: the DD series for T <= 14, the lowering route for T >= 4 (T >= 2
// when L <= 4).  The switch sits inside it.
__device__ __forceinline__ double t_switch(int L) { return L <= 4 ? 2.5 : (L <= 8 ? 4.5 : 6.0); }
__device__ __forceinline__ bool minus_side_needed(double T, int L) {
  // keep the F(-R) branch while exp(-T) (2T)^L / (2L-1)!! > 1e-19
  double lg = -T;
  if (L > 0) {
    lg += L * log(2.0 * T);
    for (int k = 3; k <= 2 * L - 1; k += 2) lg -= log((double)k);
  }
  return lg > -43.7 && T < 108.0;
}

// ---------------------------------------------------------------------------
// K3/K4: one thread per primitive quartet of a chunk; A[n * np + t] = A_n.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(128) aux_kernel(const KernelDev *__restrict__ K, PairsDev bra,
                                                  PairsDev ket, const int64_t *__restrict__ qb,
                                                  const int64_t *__restrict__ qk,
                                                  const int64_t *__restrict__ qprim, int64_t qa,
                                                  int64_t nqc, int64_t p0, int64_t np, int L,
                                                  double *__restrict__ A) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= np) return;
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
  const double T = xi * u;
  const double Np = F12_PI52 / (sqrt(p + qq) * p * qq);
  double a[LTOT_MAX + 1];
  if (T < t_switch(L)) {
    aux_small(K, xi, u, L, T, a);
  } else {
    aux_large(K, xi, sqrt(u), L, minus_side_needed(T, L), a);
  }
  for (int n = 0; n <= L; ++n) A[n * np + t] = a[n] * Np;
}

// ---------------------------------------------------------------------------
// E_t^{ij} (and F_t^{ij} = dE_t^{ij}/dAB_x) along one direction by the
// recursions of Eqs. (Erec0)-(Erect) (with the stray "E_0" of (Erecj) read as
// a typo) and their AB-derivatives:
//   E_0^{00} = exp(-(ab/p) AB^2),       F_0^{00} = -(2ab/p) AB E_0^{00}
//   E_0^{i+1,j} = -(b/p) AB E_0^{ij} + E_1^{ij}
//   F_0^{i+1,j} = -(b/p) AB F_0^{ij} + F_1^{ij} - (b/p) E_0^{ij}
//   E_0^{i,j+1} =  (a/p) AB E_0^{ij} + E_1^{ij}
//   F_0^{i,j+1} =  (a/p) AB F_0^{ij} + F_1^{ij} + (a/p) E_0^{ij}
//   E_t^{ij} = (i E_{t-1}^{i-1,j} + j E_{t-1}^{i,j-1}) / (2 p t), same for F.
// Layout E[(i * 4 + j) * 7 + t].
// ---------------------------------------------------------------------------
#define EIDX(i, j, t) (((i) * (LMAX + 1) + (j)) * (2 * LMAX + 1) + (t))
constexpr int E1D = (LMAX + 1) * (LMAX + 1) * (2 * LMAX + 1);

__device__ void e_table(double a, double b, double AB, int la, int lb, double *E, double *Fd) {
  for (int k = 0; k < E1D; ++k) {
    E[k] = 0.0;
    if (Fd) Fd[k] = 0.0;
  }
  const double p = a + b;
  const double mu = a * b / p;
  const double i2p = 0.5 / p;
  E[EIDX(0, 0, 0)] = exp(-mu * AB * AB);
  if (Fd) Fd[EIDX(0, 0, 0)] = -2.0 * mu * AB * E[EIDX(0, 0, 0)];
  for (int N = 1; N <= la + lb; ++N) {
    for (int i = (N - lb > 0 ? N - lb : 0); i <= (la < N ? la : N); ++i) {
      const int j = N - i;
      for (int t = 1; t <= N; ++t) {
        double v = 0.0, w = 0.0;
        if (i > 0) {
          v += i * E[EIDX(i - 1, j, t - 1)];
          if (Fd) w += i * Fd[EIDX(i - 1, j, t - 1)];
        }
        if (j > 0) {
          v += j * E[EIDX(i, j - 1, t - 1)];
          if (Fd) w += j * Fd[EIDX(i, j - 1, t - 1)];
        }
        E[EIDX(i, j, t)] = v * i2p / t;
        if (Fd) Fd[EIDX(i, j, t)] = w * i2p / t;
      }
      if (i > 0) {
        const double c = -(b / p) * AB;
        E[EIDX(i, j, 0)] = c * E[EIDX(i - 1, j, 0)] + E[EIDX(i - 1, j, 1)];
        if (Fd)
          Fd[EIDX(i, j, 0)] = c * Fd[EIDX(i - 1, j, 0)] + Fd[EIDX(i - 1, j, 1)] -
                              (b / p) * E[EIDX(i - 1, j, 0)];
      } else {
        const double c = (a / p) * AB;
        E[EIDX(i, j, 0)] = c * E[EIDX(i, j - 1, 0)] + E[EIDX(i, j - 1, 1)];
        if (Fd)
          Fd[EIDX(i, j, 0)] = c * Fd[EIDX(i, j - 1, 0)] + Fd[EIDX(i, j - 1, 1)] +
                              (a / p) * E[EIDX(i, j - 1, 0)];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// K5/K6: one workgroup per contracted quartet.  For each bra primitive pair:
//   R^(0)_tuv from A_n by the MD recurrence (X = Q - P)
//     R^(n)_{t+1,u,v} = t R^(n+1)_{t-1,u,v} + X_x R^(n+1)_{tuv}   (Eq. (ri))
//   W[h][cd] += c_c c_d sum_{h' in box(cd)} E^cd_h' R_{h+h'}     (ket, Eq. (ii))
// then I[ab][cd] += c_a c_b sum_h (-1)^|h| E^ab_h W[h][cd]        (bra, Eq. (ii)).
// I5 (Eq. (I5byI3_) with the gradient coefficient -1, which is what
// 1/2(lap_A - lap_B) = (a-b)/(2p) lap_Q - grad_Q . grad_AB gives):
//   comp 0: (a-b)/(2p) E^ab_h  with  R_{h+h'+2x} + R_{h+h'+2y} + R_{h+h'+2z}
//   comp d: -F^ab_{h,d}        with  R_{h+h'+e_d}
// ---------------------------------------------------------------------------
template <int NT, int MAXE>
__global__ void __launch_bounds__(NT)
    contract_kernel(PairsDev bra, PairsDev ket, const int64_t *__restrict__ qb,
                    const int64_t *__restrict__ qk, const int64_t *__restrict__ qoff,
                    const int64_t *__restrict__ qprim, int64_t qa, int64_t p0, int64_t np,
                    const double *__restrict__ A, int la, int lb, int lc, int ld, int i5,
                    double *__restrict__ out, int64_t out_base) {
  extern __shared__ double lds[];
  const int tid = threadIdx.x;
  const int64_t q = qa + blockIdx.x;
  const int Lab = la + lb, Lcd = lc + ld;
  const int L = Lab + Lcd + (i5 ? 2 : 0);
  const int nb = ncart(lb), nd = ncart(ld);
  const int nab = ncart(la) * nb, ncd = ncart(lc) * nd;
  const int HL = hsize(L), Hab = hsize(Lab);
  double *Rc = lds;
  double *Rn = Rc + HL;
  double *W = Rn + HL;
  double *Eb = W + Hab * ncd;  // 3 directions
  double *Fb = Eb + 3 * E1D;
  double *Ek = Fb + 3 * E1D;
  int *tuv = (int *)(Ek + 3 * E1D);
  for (int idx = tid; idx < HL; idx += NT) {
    // invert ridx
    int N = 0;
    while (hsize(N) <= idx) ++N;
    int r = idx - (N > 0 ? hsize(N - 1) : 0);
    int s = 0;
    while ((s + 1) * (s + 2) / 2 <= r) ++s;
    int u = s - (r - s * (s + 1) / 2);
    int t = N - s;
    int v = N - t - u;
    tuv[idx] = t | (u << 8) | (v << 16);
  }
  const int64_t bp = qb[q], kp = qk[q];
  const int nbra = bra.ka[bp] * bra.kb[bp];
  const int nket = ket.ka[kp] * ket.kb[kp];
  const double ABb[3] = {bra.ABx[bp], bra.ABy[bp], bra.ABz[bp]};
  const double ABk[3] = {ket.ABx[kp], ket.ABy[kp], ket.ABz[kp]};
  const int64_t qp0 = qprim[q] - p0;
  double Iacc[MAXE];
#pragma unroll
  for (int k = 0; k < MAXE; ++k) Iacc[k] = 0.0;
  const int ncomp = i5 ? 4 : 1;
  for (int comp = 0; comp < ncomp; ++comp) {
    for (int ib = 0; ib < nbra; ++ib) {
      const int64_t ppb = bra.pp_off[bp] + ib;
      const double ea = bra.ea[ppb], eb = bra.eb[ppb], pb = bra.p[ppb];
      const double Pb[3] = {bra.Px[ppb], bra.Py[ppb], bra.Pz[ppb]};
      if (tid < 3) e_table(ea, eb, ABb[tid], la, lb, Eb + tid * E1D, i5 ? Fb + tid * E1D : nullptr);
      for (int e = tid; e < Hab * ncd; e += NT) W[e] = 0.0;
      for (int jk = 0; jk < nket; ++jk) {
        const int64_t ppk = ket.pp_off[kp] + jk;
        __syncthreads();  // previous users of Ek / Rc are done
        if (tid < 3) e_table(ket.ea[ppk], ket.eb[ppk], ABk[tid], lc, ld, Ek + tid * E1D, nullptr);
        const double Xq[3] = {ket.Px[ppk] - Pb[0], ket.Py[ppk] - Pb[1], ket.Pz[ppk] - Pb[2]};
        const int64_t pl = qp0 + (int64_t)ib * nket + jk;
        double *rc = Rc, *rn = Rn;
        for (int n = L; n >= 0; --n) {
          const int cnt = hsize(L - n);
          for (int idx = tid; idx < cnt; idx += NT) {
            const int code = tuv[idx];
            const int t = code & 255, u = (code >> 8) & 255, v = code >> 16;
            double val;
            if (idx == 0) {
              val = A[(int64_t)n * np + pl];
            } else if (t > 0) {
              val = Xq[0] * rc[ridx(t - 1, u, v)];
              if (t > 1) val += (t - 1) * rc[ridx(t - 2, u, v)];
            } else if (u > 0) {
              val = Xq[1] * rc[ridx(t, u - 1, v)];
              if (u > 1) val += (u - 1) * rc[ridx(t, u - 2, v)];
            } else {
              val = Xq[2] * rc[ridx(t, u, v - 1)];
              if (v > 1) val += (v - 1) * rc[ridx(t, u, v - 2)];
            }
            rn[idx] = val;
          }
          __syncthreads();
          double *tmp = rc;
          rc = rn;
          rn = tmp;
        }
        // ket transform
        const double ckd = ket.cab[ppk];
        const int dt = (comp == 1), du = (comp == 2), dv = (comp == 3);
        for (int e = tid; e < Hab * ncd; e += NT) {
          const int h = e / ncd, cd = e - h * ncd;
          const int code = tuv[h];
          const int t = code & 255, u = (code >> 8) & 255, v = code >> 16;
          int cx, cy, cz, dx, dy, dz;
          cart_comp(lc, cd / nd, cx, cy, cz);
          cart_comp(ld, cd % nd, dx, dy, dz);
          const double *ex = Ek + EIDX(cx, dx, 0);
          const double *ey = Ek + E1D + EIDX(cy, dy, 0);
          const double *ez = Ek + 2 * E1D + EIDX(cz, dz, 0);
          double s = 0.0;
          for (int tp = 0; tp <= cx + dx; ++tp) {
            for (int up = 0; up <= cy + dy; ++up) {
              const double exy = ex[tp] * ey[up];
              for (int vp = 0; vp <= cz + dz; ++vp) {
                const int T = t + tp, U = u + up, V = v + vp;
                double r;
                if (i5 && comp == 0)
                  r = rc[ridx(T + 2, U, V)] + rc[ridx(T, U + 2, V)] + rc[ridx(T, U, V + 2)];
                else
                  r = rc[ridx(T + dt, U + du, V + dv)];
                s += exy * ez[vp] * r;
              }
            }
          }
          W[e] += ckd * s;
        }
      }
      __syncthreads();  // W complete
      // bra transform
      const double cb = bra.cab[ppb];
      const double wlap = i5 ? (ea - eb) / (2.0 * pb) : 1.0;
#pragma unroll
      for (int k = 0; k < MAXE; ++k) {
        const int e = tid + k * NT;
        if (e < nab * ncd) {
          const int ab = e / ncd, cd = e - ab * ncd;
          int ax, ay, az, bx, by, bz;
          cart_comp(la, ab / nb, ax, ay, az);
          cart_comp(lb, ab % nb, bx, by, bz);
          const double *ex = ((i5 && comp == 1) ? Fb : Eb) + EIDX(ax, bx, 0);
          const double *ey = ((i5 && comp == 2) ? Fb : Eb) + E1D + EIDX(ay, by, 0);
          const double *ez = ((i5 && comp == 3) ? Fb : Eb) + 2 * E1D + EIDX(az, bz, 0);
          double s = 0.0;
          for (int t = 0; t <= ax + bx; ++t) {
            for (int u = 0; u <= ay + by; ++u) {
              const double exy = ex[t] * ey[u];
              for (int v = 0; v <= az + bz; ++v) {
                const double term = exy * ez[v] * W[ridx(t, u, v) * ncd + cd];
                s += ((t + u + v) & 1) ? -term : term;
              }
            }
          }
          Iacc[k] += cb * ((comp == 0) ? wlap : -1.0) * s;
        }
      }
      __syncthreads();  // before Eb / W are overwritten
    }
  }
  const int64_t o = qoff[q] - out_base;
#pragma unroll
  for (int k = 0; k < MAXE; ++k) {
    const int e = tid + k * NT;
    if (e < nab * ncd) out[o + e] = Iacc[k];
  }
}

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

int launch_aux(const KernelDev *K, const PairsDev &bra, const PairsDev &ket, const int64_t *qb,
               const int64_t *qk, const int64_t *qprim, int64_t qa, int64_t nqc, int64_t p0,
               int64_t np, int L, double *A, hipStream_t stream) {
  if (np <= 0) return 0;
  int nt = 128;
  int64_t nbk = (np + nt - 1) / nt;
  hipLaunchKernelGGL(aux_kernel, dim3((unsigned)nbk), dim3(nt), 0, stream, K, bra, ket, qb, qk,
                     qprim, qa, nqc, p0, np, L, A);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

static size_t contract_lds_bytes(int la, int lb, int lc, int ld, int i5) {
  auto hs = [](int L) { return (L + 1) * (L + 2) * (L + 3) / 6; };
  auto nc = [](int l) { return (l + 1) * (l + 2) / 2; };
  int L = la + lb + lc + ld + (i5 ? 2 : 0);
  size_t d = 2 * (size_t)hs(L) + (size_t)hs(la + lb) * nc(lc) * nc(ld) + 9 * (size_t)E1D;
  return d * sizeof(double) + hs(L) * sizeof(int);
}

int launch_contract(const PairsDev &bra, const PairsDev &ket, const int64_t *qb, const int64_t *qk,
                    const int64_t *qoff, const int64_t *qprim, int64_t qa, int64_t nqc, int64_t p0,
                    int64_t np, const double *A, int la, int lb, int lc, int ld, int i5,
                    double *out, int64_t out_base, hipStream_t stream) {
  if (nqc <= 0) return 0;
  size_t lds = contract_lds_bytes(la, lb, lc, ld, i5);
  auto nc = [](int l) { return (l + 1) * (l + 2) / 2; };
  int nel = nc(la) * nc(lb) * nc(lc) * nc(ld);
  if (nel <= 64 * 4) {
    hipLaunchKernelGGL((contract_kernel<64, 4>), dim3((unsigned)nqc), dim3(64), lds, stream, bra,
                       ket, qb, qk, qoff, qprim, qa, p0, np, A, la, lb, lc, ld, i5, out, out_base);
  } else {
    static bool attr_set = false;
    if (!attr_set) {
      hipFuncSetAttribute((const void *)contract_kernel<256, 40>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
      attr_set = true;
    }
    hipLaunchKernelGGL((contract_kernel<256, 40>), dim3((unsigned)nqc), dim3(256), lds, stream,
                       bra, ket, qb, qk, qoff, qprim, qa, p0, np, A, la, lb, lc, ld, i5, out,
                       out_base);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
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
  const bool small = (route == 1) || (route == 0 && T < t_switch(L));
  if (small)
    aux_small(K, xi, u, L, T, a);
  else
    aux_large(K, xi, R, L, route == 2 ? true : minus_side_needed(T, L), a);
  for (int k = 0; k <= L; ++k) A[k * n + t] = a[k] * Np;
}

int launch_aux_points(const KernelDev *K, int64_t n, const double *p, const double *q,
                      const double *R, int L, int route, double *A, hipStream_t stream) {
  if (n <= 0) return 0;
  int nt = 128;
  int64_t nbk = (n + nt - 1) / nt;
  hipLaunchKernelGGL(aux_points_kernel, dim3((unsigned)nbk), dim3(nt), 0, stream, K, n, p, q, R,
                     L, route, A);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace f12
