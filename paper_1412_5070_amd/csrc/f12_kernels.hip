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
// Layout E[(i * (lb+1) + j) * (la+lb+1) + t].
// ---------------------------------------------------------------------------

__device__ void e_table(double a, double b, double AB, int la, int lb, double *E, double *Fd) {
  const int nj = lb + 1, ntt = la + lb + 1;
#define EI(i, j, t) (((i) * nj + (j)) * ntt + (t))
  const int ne = (la + 1) * nj * ntt;
  for (int k = 0; k < ne; ++k) {
    E[k] = 0.0;
    if (Fd) Fd[k] = 0.0;
  }
  const double p = a + b;
  const double mu = a * b / p;
  const double i2p = 0.5 / p;
  E[EI(0, 0, 0)] = exp(-mu * AB * AB);
  if (Fd) Fd[EI(0, 0, 0)] = -2.0 * mu * AB * E[EI(0, 0, 0)];
  for (int N = 1; N <= la + lb; ++N) {
    for (int i = (N - lb > 0 ? N - lb : 0); i <= (la < N ? la : N); ++i) {
      const int j = N - i;
      for (int t = 1; t <= N; ++t) {
        double v = 0.0, w = 0.0;
        if (i > 0) {
          v += i * E[EI(i - 1, j, t - 1)];
          if (Fd) w += i * Fd[EI(i - 1, j, t - 1)];
        }
        if (j > 0) {
          v += j * E[EI(i, j - 1, t - 1)];
          if (Fd) w += j * Fd[EI(i, j - 1, t - 1)];
        }
        E[EI(i, j, t)] = v * i2p / t;
        if (Fd) Fd[EI(i, j, t)] = w * i2p / t;
      }
      if (i > 0) {
        const double c = -(b / p) * AB;
        E[EI(i, j, 0)] = c * E[EI(i - 1, j, 0)] + E[EI(i - 1, j, 1)];
        if (Fd)
          Fd[EI(i, j, 0)] = c * Fd[EI(i - 1, j, 0)] + Fd[EI(i - 1, j, 1)] -
                              (b / p) * E[EI(i - 1, j, 0)];
      } else {
        const double c = (a / p) * AB;
        E[EI(i, j, 0)] = c * E[EI(i, j - 1, 0)] + E[EI(i, j - 1, 1)];
        if (Fd)
          Fd[EI(i, j, 0)] = c * Fd[EI(i, j - 1, 0)] + Fd[EI(i, j - 1, 1)] +
                              (a / p) * E[EI(i, j - 1, 0)];
      }
    }
  }
}
#undef EI

// ---------------------------------------------------------------------------
// K5/K6: E.R.E contraction, one workgroup (256 threads) per contracted
// quartet.  The threads form NG = 256/GS groups of GS lanes inside one
// wavefront (so a group needs only wave-level synchronisation); group g
// takes the ket primitive pairs j = g, g+NG, ...  For each bra primitive
// pair i and each of its ket pairs j a group
//   * builds R_ij: R^(n)_{t+1,u,v} = t R^(n+1)_{t-1,u,v} + X_x R^(n+1)_{tuv}
//     (Eq. (ri), X = Q - P), the last level stored as lines along v;
//   * does the ket transform (Eq. (ii))
//       W[t,u,v][cd] += c_c c_d sum_{t'u'} Ex[t'] Ey[u'] sum_{v'} Ez[v'] R[t+t',u+u',v+v']
//     as 1-D convolutions of R lines held in registers: a task is one
//     (t,u) line and one cd, with accumulators W[t,u,0..Lab-t-u] in
//     registers across all of the group's j.
// The group partials are then summed in LDS and the bra transform
//   I[ab][cd] += c_a c_b sum_h (-1)^|h| E^ab_h W[h][cd]
// runs over (ab, cd) elements.  Large classes walk cd in chunks so that
// tasks fit TPT per lane.
// I5 (Eq. (I5byI3_) with gradient coefficient -1, the value of
// 1/2 (lap_A - lap_B) = (a-b)/(2p) lap_Q - grad_Q . grad_AB):
//   comp 0: (a-b)/(2p) E^ab  with lines R[T+2,U,.] + R[T,U+2,.] + R[T,U,.+2]
//   comp d: -F^ab_d           with lines shifted by one along d.
// ---------------------------------------------------------------------------
constexpr int LINEMAX = 2 * (2 * LMAX) + 3;  // Lv + Z + 2 + 1

__device__ __forceinline__ void group_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

struct ContractArgs {
  PairsDev bra, ket;
  const int64_t *qb, *qk, *qoff, *qprim;
  int64_t qa, p0, np;
  const double *A;
  int la, lb, lc, ld, i5;
  int cd_chunk, nchunks;
  double *out;
  int64_t out_base;
};

constexpr int MAXI = 8;

template <int GS, int TPT>
__global__ void __launch_bounds__(256) contract_kernel(ContractArgs a) {
  constexpr int NT = 256;
  constexpr int NG = NT / GS;
  extern __shared__ double lds[];
  const int tid = threadIdx.x;
  const int g = tid / GS, lt = tid % GS;
  const int64_t q = a.qa + blockIdx.x;
  const int la = a.la, lb = a.lb, lc = a.lc, ld = a.ld, i5 = a.i5;
  const int Lab = la + lb, Lcd = lc + ld;
  const int L = Lab + Lcd + (i5 ? 2 : 0);
  const int nb = ncart(lb), nd = ncart(ld);
  const int nab = ncart(la) * nb, ncd = ncart(lc) * nd;
  const int HL = hsize(L), Hab = hsize(Lab);
  const int nlines = (Lab + 1) * (Lab + 2) / 2;
  const int cdc = a.cd_chunk;
  // E tables: [i][j][t] with runtime strides per pair
  const int Eab1 = (la + 1) * (lb + 1) * (Lab + 1);  // one direction, bra
  const int Ecd1 = (lc + 1) * (ld + 1) * (Lcd + 1);  // one direction, ket
  // LDS layout
  double *Eb = lds;               // 3 * Eab1
  double *Fb = Eb + 3 * Eab1;     // 3 * Eab1
  double *Gr = Fb + 3 * Eab1;     // per group: R0[HL], R1[HL], Ek[3*Ecd1]
  const int gstride = 2 * HL + 3 * Ecd1;
  double *Wp = Gr + NG * gstride; // NG * Hab * cdc
  int *tuv = (int *)(Wp + (size_t)NG * Hab * cdc);  // HL
  int *lineoff = tuv + HL;                           // (L+1)^2
  int *linetu = lineoff + (L + 1) * (L + 1);         // nlines
  for (int idx = tid; idx < HL; idx += NT) {
    int N = 0;
    while (hsize(N) <= idx) ++N;
    int r = idx - (N > 0 ? hsize(N - 1) : 0);
    int s = 0;
    while ((s + 1) * (s + 2) / 2 <= r) ++s;
    int u = s - (r - s * (s + 1) / 2);
    int t = N - s;
    tuv[idx] = t | (u << 8) | ((N - t - u) << 16);
  }
  if (tid == 0) {
    int off = 0;
    for (int T = 0; T <= L; ++T)
      for (int U = 0; U <= L - T; ++U) {
        lineoff[T * (L + 1) + U] = off;
        off += L - T - U + 1;
      }
    int k = 0;
    for (int t = 0; t <= Lab; ++t)
      for (int u = 0; u <= Lab - t; ++u) linetu[k++] = t | (u << 8);
  }
  __syncthreads();
  const int64_t bp = a.qb[q], kp = a.qk[q];
  const PairsDev &bra = a.bra, &ket = a.ket;
  const int nbra = bra.ka[bp] * bra.kb[bp];
  const int nket = ket.ka[kp] * ket.kb[kp];
  const double ABb[3] = {bra.ABx[bp], bra.ABy[bp], bra.ABz[bp]};
  const double ABk[3] = {ket.ABx[kp], ket.ABy[kp], ket.ABz[kp]};
  const int64_t qp0 = a.qprim[q] - a.p0;
  const int64_t o = a.qoff[q] - a.out_base;
  double *R0 = Gr + g * gstride;
  double *R1 = R0 + HL;
  double *Ek = R1 + HL;
  const int ncomp = i5 ? 4 : 1;
  for (int chunk = 0; chunk < a.nchunks; ++chunk) {
    const int cd0 = chunk * cdc;
    const int ncdc = (ncd - cd0 < cdc) ? (ncd - cd0) : cdc;
    const int ntask = nlines * ncdc;
    double Iacc[MAXI];
#pragma unroll
    for (int k = 0; k < MAXI; ++k) Iacc[k] = 0.0;
    for (int comp = 0; comp < ncomp; ++comp) {
      const int dt = (comp == 1), du = (comp == 2), dv = (comp == 3);
      for (int ib = 0; ib < nbra; ++ib) {
        const int64_t ppb = bra.pp_off[bp] + ib;
        const double ea = bra.ea[ppb], eb = bra.eb[ppb], pb = bra.p[ppb];
        const double Pb0 = bra.Px[ppb], Pb1 = bra.Py[ppb], Pb2 = bra.Pz[ppb];
        if (tid < 3) e_table(ea, eb, ABb[tid], la, lb, Eb + tid * Eab1, i5 ? Fb + tid * Eab1 : nullptr);
        double acc[TPT][2 * LMAX + 1];
#pragma unroll
        for (int s = 0; s < TPT; ++s)
#pragma unroll
          for (int v = 0; v <= 2 * LMAX; ++v) acc[s][v] = 0.0;
        for (int jk = g; jk < nket; jk += NG) {
          const int64_t ppk = ket.pp_off[kp] + jk;
          for (int dir = lt; dir < 3; dir += GS)
            e_table(ket.ea[ppk], ket.eb[ppk], ABk[dir], lc, ld, Ek + dir * Ecd1, nullptr);
          const double X0 = ket.Px[ppk] - Pb0, X1 = ket.Py[ppk] - Pb1, X2 = ket.Pz[ppk] - Pb2;
          const int64_t pl = qp0 + (int64_t)ib * nket + jk;
          double *rc = R0, *rn = R1;
          for (int n = L; n >= 0; --n) {
            const int cnt = hsize(L - n);
            for (int idx = lt; idx < cnt; idx += GS) {
              const int code = tuv[idx];
              const int t = code & 255, u = (code >> 8) & 255, v = code >> 16;
              double val;
              if (idx == 0) {
                val = a.A[(int64_t)n * a.np + pl];
              } else if (t > 0) {
                val = X0 * rc[ridx(t - 1, u, v)];
                if (t > 1) val += (t - 1) * rc[ridx(t - 2, u, v)];
              } else if (u > 0) {
                val = X1 * rc[ridx(t, u - 1, v)];
                if (u > 1) val += (u - 1) * rc[ridx(t, u - 2, v)];
              } else {
                val = X2 * rc[ridx(t, u, v - 1)];
                if (v > 1) val += (v - 1) * rc[ridx(t, u, v - 2)];
              }
              if (n == 0)
                rn[lineoff[t * (L + 1) + u] + v] = val;
              else
                rn[idx] = val;
            }
            group_sync();
            double *tmp = rc;
            rc = rn;
            rn = tmp;
          }
          const double *Rl = rc;  // lines along v
          const double ckd = ket.cab[ppk];
#pragma unroll
          for (int s = 0; s < TPT; ++s) {
            const int k = lt + s * GS;
            if (k < ntask) {
              const int line = k / ncdc;
              const int cd = cd0 + (k - line * ncdc);
              const int tu = linetu[line];
              const int t = tu & 255, u = tu >> 8;
              const int Lv = Lab - t - u;
              int cx, cy, cz, dx, dy, dz;
              cart_comp(lc, cd / nd, cx, cy, cz);
              cart_comp(ld, cd % nd, dx, dy, dz);
              const double *ex = Ek + (cx * (ld + 1) + dx) * (Lcd + 1);
              const double *ey = Ek + Ecd1 + (cy * (ld + 1) + dy) * (Lcd + 1);
              const double *ez = Ek + 2 * Ecd1 + (cz * (ld + 1) + dz) * (Lcd + 1);
              const int Z = cz + dz;
              const int nlv = Lv + Z + 1;
              for (int tp = 0; tp <= cx + dx; ++tp) {
                const double wx = ex[tp] * ckd;
                for (int up = 0; up <= cy + dy; ++up) {
                  const double c = wx * ey[up];
                  const int T = t + tp, U = u + up;
                  double lbuf[LINEMAX];
                  if (i5 && comp == 0) {
                    const double *l1 = Rl + lineoff[(T + 2) * (L + 1) + U];
                    const double *l2 = Rl + lineoff[T * (L + 1) + U + 2];
                    const double *l3 = Rl + lineoff[T * (L + 1) + U] + 2;
                    for (int v = 0; v < nlv; ++v) lbuf[v] = l1[v] + l2[v] + l3[v];
                  } else {
                    const double *l1 = Rl + lineoff[(T + dt) * (L + 1) + U + du] + dv;
                    for (int v = 0; v < nlv; ++v) lbuf[v] = l1[v];
                  }
                  for (int vp = 0; vp <= Z; ++vp) {
                    const double cz2 = c * ez[vp];
#pragma unroll
                    for (int v = 0; v <= 2 * LMAX; ++v)
                      if (v <= Lv) acc[s][v] = fma(cz2, lbuf[v + vp], acc[s][v]);
                  }
                }
              }
            }
          }
          group_sync();  // R / Ek reused by the next j of this group
        }
        // group partials -> Wp[g][h][cd]
        double *Wg = Wp + (size_t)g * Hab * cdc;
        for (int e = lt; e < Hab * cdc; e += GS) Wg[e] = 0.0;
        group_sync();
#pragma unroll
        for (int s = 0; s < TPT; ++s) {
          const int k = lt + s * GS;
          if (k < ntask) {
            const int line = k / ncdc;
            const int cdl = k - line * ncdc;
            const int tu = linetu[line];
            const int t = tu & 255, u = tu >> 8;
            for (int v = 0; v <= Lab - t - u; ++v) Wg[ridx(t, u, v) * cdc + cdl] = acc[s][v];
          }
        }
        __syncthreads();
        for (int e = tid; e < Hab * cdc; e += NT) {
          double sum = Wp[e];
          for (int gg = 1; gg < NG; ++gg) sum += Wp[(size_t)gg * Hab * cdc + e];
          Wp[e] = sum;
        }
        __syncthreads();
        // bra transform
        const double cb = bra.cab[ppb];
        const double wlap = i5 ? (ea - eb) / (2.0 * pb) : 1.0;
        const double cw = cb * ((comp == 0) ? wlap : -1.0);
#pragma unroll
        for (int k = 0; k < MAXI; ++k) {
          const int e = tid + k * NT;
          if (e < nab * ncdc) {
            const int ab = e / ncdc, cdl = e - ab * ncdc;
            int ax, ay, az, bx, by, bz;
            cart_comp(la, ab / nb, ax, ay, az);
            cart_comp(lb, ab % nb, bx, by, bz);
            const double *ex = ((i5 && comp == 1) ? Fb : Eb) + (ax * (lb + 1) + bx) * (Lab + 1);
            const double *ey = ((i5 && comp == 2) ? Fb : Eb) + Eab1 + (ay * (lb + 1) + by) * (Lab + 1);
            const double *ez = ((i5 && comp == 3) ? Fb : Eb) + 2 * Eab1 + (az * (lb + 1) + bz) * (Lab + 1);
            double sacc = 0.0;
            for (int t = 0; t <= ax + bx; ++t) {
              for (int u = 0; u <= ay + by; ++u) {
                const double exy = ex[t] * ey[u];
                for (int v = 0; v <= az + bz; ++v) {
                  const double term = exy * ez[v] * Wp[ridx(t, u, v) * cdc + cdl];
                  sacc += ((t + u + v) & 1) ? -term : term;
                }
              }
            }
            Iacc[k] += cw * sacc;
          }
        }
        __syncthreads();  // before Eb / Wp are overwritten
      }
    }
#pragma unroll
    for (int k = 0; k < MAXI; ++k) {
      const int e = tid + k * NT;
      if (e < nab * ncdc) {
        const int ab = e / ncdc, cdl = e - ab * ncdc;
        a.out[o + (int64_t)ab * ncd + cd0 + cdl] = Iacc[k];
      }
    }
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

// Launch shape per class: GS lanes per group (a power of two <= 64), TPT
// tasks per lane, cd chunk size; returns the LDS bytes.
struct ContractShape {
  int gs, tpt, cd_chunk, nchunks;
  size_t lds;
};

static ContractShape contract_shape(int la, int lb, int lc, int ld, int i5) {
  auto hs = [](int L) { return (L + 1) * (L + 2) * (L + 3) / 6; };
  auto nc = [](int l) { return (l + 1) * (l + 2) / 2; };
  const int Lab = la + lb;
  const int L = la + lb + lc + ld + (i5 ? 2 : 0);
  const int nlines = (Lab + 1) * (Lab + 2) / 2;
  const int ncd = nc(lc) * nc(ld);
  const int nab = nc(la) * nc(lb);
  ContractShape sh;
  const int ntask = nlines * ncd;
  if (ntask <= 64 * 4) {
    int need = (ntask + 3) / 4;
    int gs = 1;
    while (gs < need) gs *= 2;
    sh.gs = gs;
    sh.tpt = 4;
    sh.cd_chunk = ncd;
  } else {
    sh.gs = 64;
    sh.tpt = 8;
    sh.cd_chunk = (64 * 8) / nlines;
    if (sh.cd_chunk > ncd) sh.cd_chunk = ncd;
  }
  // the bra transform keeps MAXI elements per thread
  while ((size_t)nab * sh.cd_chunk > (size_t)256 * MAXI) --sh.cd_chunk;
  sh.nchunks = (ncd + sh.cd_chunk - 1) / sh.cd_chunk;
  const int NG = 256 / sh.gs;
  const int HL = hs(L);
  const int Eab1 = (la + 1) * (lb + 1) * (Lab + 1);
  const int Ecd1 = (lc + 1) * (ld + 1) * (lc + ld + 1);
  size_t d = 6 * (size_t)Eab1 + (size_t)NG * (2 * HL + 3 * Ecd1) + (size_t)NG * hs(Lab) * sh.cd_chunk;
  size_t ints = HL + (size_t)(L + 1) * (L + 1) + nlines;
  sh.lds = d * sizeof(double) + ints * sizeof(int);
  return sh;
}

template <int GS, int TPT>
static void launch_contract_t(const ContractArgs &a, unsigned nblocks, size_t lds, hipStream_t st) {
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void *)contract_kernel<GS, TPT>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr = true;
  }
  hipLaunchKernelGGL((contract_kernel<GS, TPT>), dim3(nblocks), dim3(256), lds, st, a);
}

int launch_contract(const PairsDev &bra, const PairsDev &ket, const int64_t *qb, const int64_t *qk,
                    const int64_t *qoff, const int64_t *qprim, int64_t qa, int64_t nqc, int64_t p0,
                    int64_t np, const double *A, int la, int lb, int lc, int ld, int i5,
                    double *out, int64_t out_base, hipStream_t stream) {
  if (nqc <= 0) return 0;
  ContractShape sh = contract_shape(la, lb, lc, ld, i5);
  if (sh.lds > 160 * 1024) return -1;
  ContractArgs a;
  a.bra = bra;
  a.ket = ket;
  a.qb = qb;
  a.qk = qk;
  a.qoff = qoff;
  a.qprim = qprim;
  a.qa = qa;
  a.p0 = p0;
  a.np = np;
  a.A = A;
  a.la = la;
  a.lb = lb;
  a.lc = lc;
  a.ld = ld;
  a.i5 = i5;
  a.cd_chunk = sh.cd_chunk;
  a.nchunks = sh.nchunks;
  a.out = out;
  a.out_base = out_base;
  const unsigned nb = (unsigned)nqc;
  switch (sh.gs * 10 + sh.tpt) {
    case 14: launch_contract_t<1, 4>(a, nb, sh.lds, stream); break;
    case 24: launch_contract_t<2, 4>(a, nb, sh.lds, stream); break;
    case 44: launch_contract_t<4, 4>(a, nb, sh.lds, stream); break;
    case 84: launch_contract_t<8, 4>(a, nb, sh.lds, stream); break;
    case 164: launch_contract_t<16, 4>(a, nb, sh.lds, stream); break;
    case 324: launch_contract_t<32, 4>(a, nb, sh.lds, stream); break;
    case 644: launch_contract_t<64, 4>(a, nb, sh.lds, stream); break;
    case 648: launch_contract_t<64, 8>(a, nb, sh.lds, stream); break;
    default: return -1;
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
