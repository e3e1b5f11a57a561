// E.R.E contraction specialised on the class shape (L_ab = l_a + l_b,
// L_cd = l_c + l_d, I5 or not).
//
// One work-group of 256 threads per contracted quartet; all threads work on
// one primitive quartet at a time.  Per primitive quartet (bra i, ket j):
//   R     R^(n)_{t+1,u,v} = t R^(n+1)_{t-1,u,v} + X_x R^(n+1)_{tuv} from
//         R^(n)_000 = A_n (Eq. (ri) in MD form, X = Q - P), level by level;
//         the last level is stored as lines along v.
//   z     Z[T,U][v][fz] = sum_phi E^fz_phi R[T,U,v+phi]
//   y     Y[T][u,v][fy,fz] = sum_nu E^fy_nu Z[T,u+nu][v][fz]
//   x     V[t,u,v][f] = sum_tau E^fx_tau Y[t+tau][u,v][fy,fz]
// with the one-centre ket expansion x_C^f exp(-q x_Q^2) = sum E^f_phi
// Lambda_phi(x_Q).  V is summed over ket primitives in registers: thread
// slot s owns a fixed V element whose f_x is known at compile time, so the
// x sums run unrolled on E coefficients held in registers.  Per bra
// primitive the bra transform I[ab][f] += c_a c_b sum_h (-1)^{|h|} E^ab_h V[h][f]
// (Eq. (ii)) accumulates in registers, and the exponent-free transfer
// x_D^d = sum_k C(d,k) (C_x - D_x)^(d-k) x_C^k gives (ab|cd) at the end.
// I5 has two forms.  MODE 2 (the default where LDS and registers allow):
// I5 = 1/2 (lap_A - lap_B) I3 (Eq. (I5_)) with the one-dimensional Laplacian
// of x_A^i exp(-a x_A^2), i(i-1) x^(i-2) - 2a(2i+1) x^i + 4a^2 x^(i+2), folded
// into the bra coefficients: one ket transform over bra Hermite indices up to
// l_a + l_b + 2 and, per direction d, D^{ij}_t = 1/2 [i(i-1) E^{i-2,j} -
// 2a(2i+1) E^{ij} + 4a^2 E^{i+2,j} - j(j-1) E^{i,j-2} + 2b(2j+1) E^{ij} -
// 4b^2 E^{i,j+2}]_t in place of E along d.  MODE 1 (Eq. (I5byI3_) with
// gradient coefficient -1) runs four ket transforms:
//   comp 0: (a-b)/(2p) E^ab with R_lap = R_{t+2,u,v} + R_{t,u+2,v} + R_{t,u,v+2},
//   comp d: -F^ab_d with R shifted by one along d.
// MODE 3: the first derivative of I1-I4, I6 with respect to the bra's first
// centre along direction d = a.gdir.  With P = (a A + b B)/p and the Hermite
// Gaussians Lambda_t(x - P_x) = (d/dP_x)^t e^{-p (x - P_x)^2},
//   d/dA_x sum_t E_t Lambda_t = sum_t [F_t + (a/p) E_{t-1}] Lambda_t,
// F = dE/d(A_x - B_x) (Sec. II.B): the bra coefficients along d become
// G_t = F_t + (a/p) E_{t-1}, t <= i + j + 1, over one ket transform with the
// bra Hermite range l_a + l_b + 1.
#pragma once
#include <type_traits>

#include "f12_common.h"

namespace f12 {

constexpr int hs3c(int L) { return (L + 1) * (L + 2) * (L + 3) / 6; }
constexpr int nc2c(int l) { return (l + 1) * (l + 2) / 2; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }

constexpr int max_nab(int lab) {
  int m = 0;
  for (int la = 0; la <= LMAX; ++la) {
    const int lb = lab - la;
    if (lb >= 0 && lb <= LMAX) m = cmax(m, nc2c(la) * nc2c(lb));
  }
  return m;
}
constexpr int max_eab(int lab) {
  int m = 0;
  for (int la = 0; la <= LMAX; ++la) {
    const int lb = lab - la;
    if (lb >= 0 && lb <= LMAX) m = cmax(m, (la + 1) * (lb + 1) * (lab + 1));
  }
  return m;
}
constexpr int max_nf(int lcd) {
  const int lcmin = lcd > LMAX ? lcd - LMAX : 0;
  return hs3c(lcd) - hs3c(lcmin - 1);
}

// MODE 3: the G table of one direction, t <= l_a + l_b + 1.
constexpr int max_eabg(int lab) {
  int m = 0;
  for (int la = 0; la <= LMAX; ++la) {
    const int lb = lab - la;
    if (lb >= 0 && lb <= LMAX) m = cmax(m, (la + 1) * (lb + 1) * (lab + 2));
  }
  return m;
}

// Bra E tables up to (l_a + 2, l_b + 2) and the D tables of MODE 2.
constexpr int max_eab2(int lab) {
  int m = 0;
  for (int la = 0; la <= LMAX; ++la) {
    const int lb = lab - la;
    if (lb >= 0 && lb <= LMAX) m = cmax(m, 3 * (la + 3) * (lb + 3) * (lab + 5) + 3 * (la + 1) * (lb + 1) * (lab + 3));
  }
  return m;
}

// MODE: 0 = I1-I4, I6; 1 = I5 by four components; 2 = I5 by the Laplacian
// form, with LAB = l_a + l_b + 2 (the bra Hermite range of the ket transform);
// 3 = first derivative along a.gdir with respect to the bra's first centre,
// LAB = l_a + l_b + 1.
template <int LAB, int LCD, int MODE, int NJ>
struct BigShape {
  static constexpr bool I5 = MODE == 1;
  static constexpr int BLAB = MODE == 2 ? LAB - 2 : (MODE == 3 ? LAB - 1 : LAB);  // l_a + l_b
  static constexpr int NT = 256;
  static constexpr int LP = LAB + LCD;
  static constexpr int L = LP + (I5 ? 2 : 0);
  static constexpr int HL = hs3c(L);
  static constexpr int HAB = hs3c(LAB);
  static constexpr int NE = nc2c(LCD);   // E^f_phi per direction; also (fy, fz) pairs
  static constexpr int NUV = nc2c(LAB);  // (u, v) pairs with u + v <= LAB
  static constexpr int NF0 = hs3c(LCD);  // one-centre components with |f| <= LCD
  static constexpr int NLL = nc2c(L);    // R lines (T, U), T + U <= L
  static constexpr int RLS = L + 1;
  static constexpr int NLP = nc2c(LP);   // z-pass lines
  static constexpr int ZST = (LAB + 1) * (LCD + 1);
  static constexpr int YST = NUV * NE;
  static constexpr int NZT = NLP * (LAB + 1);
  static constexpr int NYT = (LP + 1) * (LAB + 1) * (LCD + 1);
  static constexpr int NEB = MODE == 2 ? max_eab2(BLAB)
                             : (MODE == 3 ? 6 * max_eab(BLAB) + max_eabg(BLAB) : (I5 ? 6 : 3) * max_eab(LAB));
  // LDS (doubles)
  // per ket primitive of a pass: G rows, Z, Y, one-centre E
  static constexpr int jG = 0;
  static constexpr int jZ = jG + (L + 1) * (L + 1) + 2;
  static constexpr int jY = jZ + NLP * ZST;
  static constexpr int jEk = jY + (LP + 1) * YST;
  static constexpr int PJ = jEk + 3 * NE;
  // ket primitives staged at a time: centre Q, q, d exponent, weight; A_0..A_L
  static constexpr int KC = 32;
  static constexpr int KDW = 6;
  static constexpr int oHC = NEB;                         // c(T, i) table
  static constexpr int oKD = oHC + (LTOT_MAX + 1) * (LTOT_MAX / 2 + 1);
  static constexpr int oAS = oKD + KC * KDW;
  static constexpr int oRp = oAS + KC * (L + 1);
  static constexpr int DBL = oRp + NJ * PJ + 8;  // + pad: loads past a line end stay inside
  static constexpr int INTS = HL + NLP;
  static constexpr size_t BYTES = (size_t)DBL * 8 + (size_t)INTS * 4;
  // V slots: for each f_x, HAB * (#(fy,fz) with fy + fz <= LCD - fx) elements
  static constexpr int cnt_fx(int fx) { return HAB * nc2c(LCD - fx); }
  static constexpr int slots_fx(int fx) { return (cnt_fx(fx) + NT - 1) / NT; }
  static constexpr int off_fx(int fx) {
    int s = 0;
    for (int k = 0; k < fx; ++k) s += slots_fx(k);
    return s;
  }
  static constexpr int MAXW = off_fx(LCD + 1);
  static constexpr int MAXU = (max_nab(BLAB) * max_nf(LCD) + NT - 1) / NT;
  static_assert(HAB * NF0 <= DBL - oRp, "V staging must fit");
  static_assert(max_nab(BLAB) * max_nf(LCD) <= DBL - oRp, "(ab|f) staging must fit");
};

template <int NCOL, int STRIDE, typename T>
__device__ __forceinline__ void load_col(const T *p, int last, T (&c)[NCOL]) {
#pragma unroll
  for (int w = 0; w < NCOL; ++w) c[w] = (w <= last) ? p[w * STRIDE] : T{};
}

// ---------------------------------------------------------------------------
// Split-FP32 ("float-float") arithmetic for the ket transform of PREC = 1: a
// value is hi + lo with two floats (about 48 significant bits).  A product is
// made exact with one fma (Dekker's two-product), sums by Knuth's two-sum,
// then renormalised.  Contraction of a*b + c into fma is switched off so that
// the error-free transforms hold.
// ---------------------------------------------------------------------------
struct ff {
  float hi, lo;
};

__device__ __forceinline__ ff ff_from(double x) {
  const float h = (float)x;
  return ff{h, (float)(x - (double)h)};
}

__device__ __forceinline__ double ff_to(ff a) { return (double)a.hi + (double)a.lo; }

// c + a b
__device__ __forceinline__ ff ff_fma(ff a, ff b, ff c) {
#pragma clang fp contract(off)
  const float p = a.hi * b.hi;
  float e = __builtin_fmaf(a.hi, b.hi, -p);
  e = __builtin_fmaf(a.hi, b.lo, e);
  e = __builtin_fmaf(a.lo, b.hi, e);
  const float s = c.hi + p;
  const float bb = s - c.hi;
  float t = (c.hi - (s - bb)) + (p - bb);
  t = t + (c.lo + e);
  const float h = s + t;
  return ff{h, t - (h - s)};
}

// 2^-e with e the binary exponent of max_n |A_n|, n = 0..L: the power-of-two
// scale that brings one primitive quartet's Hermite integrals into float range
// (exact, so it changes no digit).
template <int L>
__device__ __forceinline__ double pq_scale(const double *A) {
  double m = 0.0;
#pragma unroll
  for (int n = 0; n <= L; ++n) m = fmax(m, fabs(A[n]));
  return m > 0.0 ? ldexp(1.0, -ilogb(m)) : 1.0;
}

// c(T, i) = T! / (i! (T - 2i)! 2^i): the coefficient of X^(T-2i) D^(T-i) in
// d^T/dX^T of a function of |X|^2/2 (D = R^-1 d/dR); table [T][i], T <= 14.
constexpr int HC_T = LTOT_MAX + 1, HC_I = LTOT_MAX / 2 + 1;

// X-direction partial sums of the closed form below, one row per T:
//   G_T[n] = sum_i c(T,i) X^(T-2i) A_{T-i+n},  n = 0..L-T  (row stride L+1,
// entries past L-T are 0).  One entry per call, so that a work-group spreads
// the rows over (T, n).
template <int L>
__device__ __forceinline__ double g_entry(int T, int n, double X, const double *A, const double *hc) {
  constexpr int H = L / 2;
  double hx[H + 1];
  {
    double px = (T & 1) ? X : 1.0;
    const double X2 = X * X;
#pragma unroll
    for (int i = H; i >= 0; --i) {
      hx[i] = 0.0;
      if (2 * i <= T) {
        hx[i] = hc[T * HC_I + i] * px;
        px *= X2;
      }
    }
  }
  double g = 0.0;
  if (n <= L - T) {
#pragma unroll
    for (int i = 0; i <= H; ++i) {
      if (2 * i > T) continue;
      g = fma(hx[i], A[T - i + n], g);
    }
  }
  return g;
}

// One Hermite line R_{T,U,w+SH}, w = 0..NW-1, of the primitive quartet, from
//   R_{T,U,W} = sum_{i,j,k} c(T,i) X^(T-2i) c(U,j) Y^(U-2j) c(W,k) Z^(W-2k) A_{T+U+W-i-j-k},
// the closed form of the recurrence R^(n)_{t+1,u,v} = t R^(n+1)_{t-1,u,v} +
// X R^(n+1)_{tuv} (each d/dX of a radial function is X D), with the X sum
// taken from the row G_T.  Entries past the line end (T + U + W > L) are 0.
template <int L, int NW, int SH>
__device__ __forceinline__ void r_line(int T, int U, double Y, double Z, const double *GT,
                                       const double *hc, double (&R)[NW]) {
  constexpr int H = L / 2;
  double hy[H + 1];
  {
    double py = (U & 1) ? Y : 1.0;
    const double Y2 = Y * Y;
#pragma unroll
    for (int i = H; i >= 0; --i) {
      hy[i] = 0.0;
      if (2 * i <= U) {
        hy[i] = hc[U * HC_I + i] * py;
        py *= Y2;
      }
    }
  }
  // col[m] = sum_j c(U,j) Y^(U-2j) G_T[U-j+m]
  const int rem = L - T - U;
  double col[L + 1];
#pragma unroll
  for (int m = 0; m <= L; ++m) col[m] = 0.0;
#pragma unroll
  for (int j = 0; j <= H; ++j) {
    if (2 * j > U) continue;
    const double *Gp = GT + (U - j);
#pragma unroll
    for (int m = 0; m <= L; ++m)
      if (m <= rem) col[m] = fma(hy[j], Gp[m], col[m]);
  }
  double zp[L + 1];
  zp[0] = 1.0;
#pragma unroll
  for (int k = 1; k <= L; ++k) zp[k] = zp[k - 1] * Z;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const int W = w + SH;
    double r = 0.0;
    if (W <= L) {
      double c = 1.0;  // c(W, 0)
#pragma unroll
      for (int k = 0; 2 * k <= W; ++k) {
        r = fma(c * zp[W - 2 * k], col[W - k], r);
        c = c * (W - 2 * k) * (W - 2 * k - 1) / (2.0 * (k + 1));
      }
    }
    R[w] = (W <= rem) ? r : 0.0;
  }
}

// PREC: 0 = FP64 throughout; 1 = the ket transform (z, y, x passes, one per
// primitive quartet) in split FP32 on power-of-two-scaled Hermite integrals,
// with the Hermite integrals themselves, the E coefficients, the bra transform
// and every accumulation over primitives in FP64.
template <int LAB, int LCD, int MODE, int NJ, int PREC>
__global__ void __launch_bounds__(256) big_kernel(ContractArgs a) {
  using S = BigShape<LAB, LCD, MODE, NJ>;
  using VT = typename std::conditional<PREC == 1, ff, double>::type;
  constexpr int NT = S::NT, LP = S::LP, L = S::L, NE = S::NE;
  constexpr bool I5 = S::I5;
  constexpr int BLAB = S::BLAB;
  extern __shared__ double lds[];
  const int tid = threadIdx.x;
  const int la = a.la, lb = a.lb, lc = a.lc, ld = a.ld;
  // bra tables: MODE 0/1 E (and F) up to (l_a, l_b); MODE 2 E up to
  // (l_a + 2, l_b + 2) with stride ES, then D up to (l_a, l_b) with stride DS
  const int ESb = MODE == 2 ? lb + 3 : lb + 1, ESt = MODE == 2 ? BLAB + 5 : BLAB + 1;
  const int Eab1 = (MODE == 2 ? la + 3 : la + 1) * ESb * ESt;
  const int DSt = BLAB + 3, Dab1 = (la + 1) * (lb + 1) * DSt;
  double *Eb = lds, *Fb = lds + 3 * Eab1;
  int *tuv = (int *)(lds + S::DBL);
  int *linetu = tuv + S::HL;
  for (int idx = tid; idx < S::HL; idx += NT) {
    int N = 0;
    while (hs3c(N) <= idx) ++N;
    const int r = idx - hs3c(N - 1);
    int s = 0;
    while ((s + 1) * (s + 2) / 2 <= r) ++s;
    const int u = s - (r - s * (s + 1) / 2);
    const int t = N - s;
    tuv[idx] = t | (u << 8) | ((N - t - u) << 16);
  }
  // line tasks ordered by T + U, longest-first groups of equal length, so
  // that a wave's lanes share their line length (dead code is skipped whole)
  for (int line = tid; line < S::NLP; line += NT) {
    int Ssum = LP, base = 0;
    while (base + (Ssum + 1) <= line) {
      base += Ssum + 1;
      --Ssum;
    }
    const int T = line - base;
    linetu[line] = T | ((Ssum - T) << 8);
  }
  double *hc = lds + S::oHC;
  for (int w = tid; w < HC_T * HC_I; w += NT) {
    const int T = w / HC_I, i = w - T * HC_I;
    double c = 0.0;
    if (2 * i <= T) {
      c = 1.0;
      for (int k = 2; k <= T; ++k) c *= k;
      for (int k = 2; k <= i; ++k) c /= k;
      for (int k = 2; k <= T - 2 * i; ++k) c /= k;
      for (int k = 0; k < i; ++k) c *= 0.5;
    }
    hc[w] = c;
  }
  __syncthreads();

  // V slot descriptors: Y offset of the slot's element (t, u, v, fy, fz), or -1
  int ybase[S::MAXW];
  double wacc[S::MAXW];
#pragma unroll
  for (int fx = 0; fx <= LCD; ++fx) {
    const int M = LCD - fx;
    const int nyz = (M + 1) * (M + 2) / 2;
#pragma unroll
    for (int k = 0; k < S::slots_fx(fx); ++k) {
      const int slot = S::off_fx(fx) + k;
      const int e = tid + NT * k;
      ybase[slot] = -1;
      if (e < S::cnt_fx(fx)) {
        const int h = e / nyz, r = e - h * nyz;
        int fy = 0, rr = r;
        while (rr > M - fy) {
          rr -= M - fy + 1;
          ++fy;
        }
        const int fz = rr;
        const int code = tuv[h];
        const int t = code & 255, u = (code >> 8) & 255, v = code >> 16;
        if (fx + fy + fz >= lc) {
          const int uvi = u * (LAB + 1) - u * (u - 1) / 2 + v;
          const int fyz = fy * (LCD + 1) - fy * (fy - 1) / 2 + fz;
          ybase[slot] = t * S::YST + uvi * NE + fyz;
        }
      }
    }
  }

  // one contracted quartet per pass; a grid smaller than the range makes the
  // work-groups persistent (quartet blockIdx.x, then + gridDim.x, ...), and the
  // set-up above is paid once per work-group
  for (int64_t qi = blockIdx.x; qi < a.nqc; qi += gridDim.x) {
  const int64_t q = a.qa + qi;
  const int64_t bp = a.qb[q], kp = a.qk[q];
  const PairsDev &bra = a.bra, &ket = a.ket;
  const int nbra = bra.ka[bp] * bra.kb[bp];
  const int nket = ket.ka[kp] * ket.kb[kp];
  const double ABb[3] = {bra.ABx[bp], bra.ABy[bp], bra.ABz[bp]};
  const double CD[3] = {ket.ABx[kp], ket.ABy[kp], ket.ABz[kp]};
  const double CD2 = CD[0] * CD[0] + CD[1] * CD[1] + CD[2] * CD[2];
  const int64_t qp0 = a.qprim[q] - a.p0;
  const int64_t o = a.qoff[q] - a.out_base;
  const int nb = ncart(lb);
  const int nf = hs3(LCD) - hs3(lc - 1);
  const int foff = hs3(lc - 1);
  const int nu = ncart(la) * nb * nf;

  double uacc[S::MAXU];
#pragma unroll
  for (int k = 0; k < S::MAXU; ++k) uacc[k] = 0.0;

  for (int ib = 0; ib < nbra; ++ib) {
    const int64_t ppb = bra.pp_off[bp] + ib;
    const double ea = bra.ea[ppb], eb = bra.eb[ppb], pb = bra.p[ppb];
    const double Pb0 = bra.Px[ppb], Pb1 = bra.Py[ppb], Pb2 = bra.Pz[ppb];
    const double cab = bra.cab[ppb];
    // bra tables of this primitive pair, built by the whole work-group (the
    // previous pair's bra transform ended with a barrier)
    if constexpr (MODE == 2) {
      e_tables_wg(ea, eb, ABb[0], ABb[1], ABb[2], la + 2, lb + 2, Eb, nullptr, Eab1, tid, NT);
      // D^{ij}_t of the Laplacian form, one entry per thread, t <= i + j + 2
      const int nd1 = (la + 1) * (lb + 1) * DSt;
      for (int k = tid; k < 3 * nd1; k += NT) {
        const int d = k / nd1;
        const int r = k - d * nd1;
        const int t = r % DSt, ij = r / DSt;
        const int i = ij / (lb + 1), j = ij - (ij / (lb + 1)) * (lb + 1);
        if (t > i + j + 2) continue;
        const double *E = Eb + d * Eab1;
        const double e0 = E[(i * ESb + j) * ESt + t];
        double v = (2.0 * eb * (2 * j + 1) - 2.0 * ea * (2 * i + 1)) * e0 +
                   4.0 * ea * ea * E[((i + 2) * ESb + j) * ESt + t] -
                   4.0 * eb * eb * E[(i * ESb + j + 2) * ESt + t];
        if (i >= 2) v += i * (i - 1) * E[((i - 2) * ESb + j) * ESt + t];
        if (j >= 2) v -= j * (j - 1) * E[(i * ESb + j - 2) * ESt + t];
        Fb[d * Dab1 + (i * (lb + 1) + j) * DSt + t] = 0.5 * v;
      }
    } else if constexpr (MODE == 3) {
      // E and F = dE/dAB up to (l_a, l_b), then G = F + (a/p) E_{t-1} along gdir
      e_tables_wg(ea, eb, ABb[0], ABb[1], ABb[2], la, lb, Eb, Fb, Eab1, tid, NT);
      const int GSt = BLAB + 2, ng = (la + 1) * (lb + 1) * GSt;
      const double *E = Eb + a.gdir * Eab1, *F = Fb + a.gdir * Eab1;
      double *G = Fb + 3 * Eab1;
      const double ap = ea / pb;
      for (int k = tid; k < ng; k += NT) {
        const int t = k % GSt, ij = k / GSt;
        const int i = ij / (lb + 1), j = ij - i * (lb + 1);
        double v = 0.0;
        if (t <= i + j) v = F[(i * (lb + 1) + j) * ESt + t];
        if (t >= 1 && t - 1 <= i + j) v += ap * E[(i * (lb + 1) + j) * ESt + t - 1];
        G[k] = v;
      }
    } else {
      e_tables_wg(ea, eb, ABb[0], ABb[1], ABb[2], la, lb, Eb, I5 ? Fb : nullptr, Eab1, tid, NT);
    }
#pragma unroll 1
    for (int comp = 0; comp < (I5 ? 4 : 1); ++comp) {
#pragma unroll
      for (int s = 0; s < S::MAXW; ++s) wacc[s] = 0.0;
      const bool lap = I5 && comp == 0;
      const int dt = comp == 1, du = comp == 2, dv = comp == 3;
      double *KD = lds + S::oKD, *AS = lds + S::oAS;
      for (int kc0 = 0; kc0 < nket; kc0 += S::KC) {
      const int nkc = nket - kc0 < S::KC ? nket - kc0 : S::KC;
      // stage the chunk's ket primitive data and radial derivatives (one
      // round of global loads instead of one per R level); the ket data does
      // not depend on the bra primitive, so a single chunk is staged once
      const bool stage_kd = nket > S::KC || (ib == 0 && comp == 0);
      for (int w = tid; stage_kd && w < nkc; w += NT) {
        const int64_t ppk = ket.pp_off[kp] + kc0 + w;
        const double qk = ket.p[ppk], ed = ket.eb[ppk];
        KD[w * S::KDW + 0] = ket.Px[ppk];
        KD[w * S::KDW + 1] = ket.Py[ppk];
        KD[w * S::KDW + 2] = ket.Pz[ppk];
        KD[w * S::KDW + 3] = qk;
        KD[w * S::KDW + 4] = ed;
        KD[w * S::KDW + 5] = ket.cab[ppk] * exp(-(ket.ea[ppk] * ed / qk) * CD2);
      }
      for (int w = tid; w < nkc * (L + 1); w += NT) {
        const int j = w / (L + 1), n = w - j * (L + 1);
        AS[w] = a.A[(int64_t)n * a.np + qp0 + (int64_t)ib * nket + kc0 + j];
      }
      __syncthreads();
      for (int jk0 = 0; jk0 < nkc; jk0 += NJ) {
        // NJ ket primitives per pass; a missing one (past the chunk) repeats
        // jk0 with weight 0
        double Xj0[NJ], Xj1[NJ], Xj2[NJ], ckdj[NJ];
        int ajj[NJ];
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
          const bool ok = jk0 + jj < nkc;
          const int jk = ok ? jk0 + jj : jk0;
          Xj0[jj] = KD[jk * S::KDW + 0] - Pb0;
          Xj1[jj] = KD[jk * S::KDW + 1] - Pb1;
          Xj2[jj] = KD[jk * S::KDW + 2] - Pb2;
          ckdj[jj] = ok ? KD[jk * S::KDW + 5] : 0.0;
          if constexpr (PREC == 1) ckdj[jj] /= pq_scale<L>(AS + jk * (L + 1));  // undo the ket scale
          ajj[jj] = jk * (L + 1);
        }
        if (tid < 3 * NJ) {
          const int jj = tid / 3, d = tid - 3 * jj;
          const int jk = jk0 + jj < nkc ? jk0 + jj : jk0;
          const double qk = KD[jk * S::KDW + 3], ed = KD[jk * S::KDW + 4];
          const double cdd = d == 0 ? CD[0] : (d == 1 ? CD[1] : CD[2]);
          e_onecentre(qk, -(ed / qk) * cdd, LCD, lds + S::oRp + jj * S::PJ + S::jEk + d * NE);
        }
        // R lines from the closed form and the z pass, one (jj, line) per
        // thread: Z[T,U][v][fz] = sum_phi E^fz_phi R_{T',U',v+phi+sh}, with
        // (T', U', sh) = (T, U, 0), the shifted line of an I5 component, or
        // the three terms of R_lap.
        const int nvj = nkc - jk0 < NJ ? nkc - jk0 : NJ;  // ket primitives in this pass
        // rows G_T[n] of the NJ ket primitives, one entry (jj, T, n) per thread
        for (int k = tid; k < nvj * (L + 1) * (L + 1); k += NT) {
          const int jj = k / ((L + 1) * (L + 1));
          const int r = k - jj * ((L + 1) * (L + 1));
          const int T = r / (L + 1), n = r - (r / (L + 1)) * (L + 1);
          const int jk = jk0 + jj;
          double gv = g_entry<L>(T, n, KD[jk * S::KDW + 0] - Pb0, AS + jk * (L + 1), hc);
          if constexpr (PREC == 1) gv *= pq_scale<L>(AS + jk * (L + 1));
          lds[S::oRp + jj * S::PJ + S::jG + T * (L + 1) + n] = gv;
        }
        __syncthreads();
        for (int k = tid; k < nvj * S::NLP; k += NT) {
          const int jj = k / S::NLP, line = k - jj * S::NLP;
          const int jk = jk0 + jj < nkc ? jk0 + jj : jk0;
          const double Y = KD[jk * S::KDW + 1] - Pb1, Zc = KD[jk * S::KDW + 2] - Pb2;
          double *base = lds + S::oRp + jj * S::PJ;
          const double *G = base + S::jG;
          const int tu = linetu[line];
          const int T = tu & 255, U = tu >> 8;
          const int zline = T * (LP + 1) - T * (T - 1) / 2 + U;  // storage order: T, then U
          double rl[LP + 1];
          if (lap) {
            double r1[LP + 1], r2[LP + 1], r3[LP + 1];
            r_line<L, LP + 1, 0>(T + 2, U, Y, Zc, G + (T + 2) * (L + 1), hc, r1);
            r_line<L, LP + 1, 0>(T, U + 2, Y, Zc, G + T * (L + 1), hc, r2);
            r_line<L, LP + 1, 2>(T, U, Y, Zc, G + T * (L + 1), hc, r3);
#pragma unroll
            for (int w = 0; w <= LP; ++w) rl[w] = r1[w] + r2[w] + r3[w];
          } else if (dv) {
            r_line<L, LP + 1, 1>(T, U, Y, Zc, G + T * (L + 1), hc, rl);
          } else {
            r_line<L, LP + 1, 0>(T + dt, U + du, Y, Zc, G + (T + dt) * (L + 1), hc, rl);
          }
          const double *ez = base + S::jEk + 2 * NE;
          if constexpr (PREC == 1) {
            ff ezr[NE], rlf[LP + 1];
#pragma unroll
            for (int e = 0; e < NE; ++e) ezr[e] = ff_from(ez[e]);
#pragma unroll
            for (int w = 0; w <= LP; ++w) rlf[w] = ff_from(rl[w]);
            ff *zo = (ff *)(base + S::jZ + zline * S::ZST);
#pragma unroll
            for (int v = 0; v <= LAB; ++v) {
#pragma unroll
              for (int fz = 0; fz <= LCD; ++fz) {
                ff acc{0.f, 0.f};
#pragma unroll
                for (int ph = 0; ph <= fz; ++ph)
                  if (v + ph <= LP) acc = ff_fma(ezr[fz * (fz + 1) / 2 + ph], rlf[v + ph], acc);
                zo[v * (LCD + 1) + fz] = acc;
              }
            }
          } else {
          double ezr[NE];
#pragma unroll
          for (int e = 0; e < NE; ++e) ezr[e] = ez[e];
          double *zo = base + S::jZ + zline * S::ZST;
#pragma unroll
          for (int v = 0; v <= LAB; ++v) {
#pragma unroll
            for (int fz = 0; fz <= LCD; ++fz) {
              double acc = 0.0;
#pragma unroll
              for (int ph = 0; ph <= fz; ++ph)
                if (v + ph <= LP) acc = fma(ezr[fz * (fz + 1) / 2 + ph], rl[v + ph], acc);
              zo[v * (LCD + 1) + fz] = acc;
            }
          }
          }
        }
        __syncthreads();
        // y pass
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
          if (jj >= nvj) break;
          double *base = lds + S::oRp + jj * S::PJ;
          VT ey[NE];
#pragma unroll
          for (int k = 0; k < NE; ++k) {
            if constexpr (PREC == 1)
              ey[k] = ff_from(base[S::jEk + NE + k]);
            else
              ey[k] = base[S::jEk + NE + k];
          }
          VT *zb = (VT *)(base + S::jZ);
          for (int k = tid; k < S::NYT; k += NT) {
            // T fastest: the lanes of a wave share (v, fz) in runs
            const int T = k % (LP + 1);
            const int r1 = k / (LP + 1);
            const int v = r1 % (LAB + 1), fz = r1 / (LAB + 1);
            if (T + v + fz > LP) continue;
            const int line0 = T * (LP + 1) - T * (T - 1) / 2;
            VT col[LP + 1];
            load_col<LP + 1, S::ZST>(zb + line0 * S::ZST + v * (LCD + 1) + fz, LP - T, col);
            VT *yo = (VT *)(base + S::jY) + T * S::YST + v * NE + fz;
#pragma unroll
            for (int u = 0; u <= LAB; ++u) {
              if (u + v > LAB) continue;
              const int uo = (u * (LAB + 1) - u * (u - 1) / 2) * NE;
#pragma unroll
              for (int fy = 0; fy <= LCD; ++fy) {
                if (fy + fz > LCD) continue;
                VT acc{};
#pragma unroll
                for (int nu = 0; nu <= fy; ++nu) {
                  if constexpr (PREC == 1)
                    acc = ff_fma(ey[fy * (fy + 1) / 2 + nu], col[u + nu], acc);
                  else
                    acc = fma(ey[fy * (fy + 1) / 2 + nu], col[u + nu], acc);
                }
                yo[uo + fy * (LCD + 1) - fy * (fy - 1) / 2] = acc;
              }
            }
          }
        }
        __syncthreads();
        // x pass into the register slots
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
          if (jj >= nvj) break;
          const double *base = lds + S::oRp + jj * S::PJ;
          const VT *Yb = (const VT *)(base + S::jY);
          VT ex[NE];
#pragma unroll
          for (int k = 0; k < NE; ++k) {
            if constexpr (PREC == 1)
              ex[k] = ff_from(base[S::jEk + k]);
            else
              ex[k] = base[S::jEk + k];
          }
#pragma unroll
          for (int fx = 0; fx <= LCD; ++fx) {
#pragma unroll
            for (int k = 0; k < S::slots_fx(fx); ++k) {
              const int slot = S::off_fx(fx) + k;
              const int yb = ybase[slot];
              if (yb >= 0) {
                VT acc{};
#pragma unroll
                for (int ta = 0; ta <= fx; ++ta) {
                  if constexpr (PREC == 1)
                    acc = ff_fma(ex[fx * (fx + 1) / 2 + ta], Yb[yb + ta * S::YST], acc);
                  else
                    acc = fma(ex[fx * (fx + 1) / 2 + ta], Yb[yb + ta * S::YST], acc);
                }
                if constexpr (PREC == 1)
                  wacc[slot] = fma(ckdj[jj], ff_to(acc), wacc[slot]);
                else
                  wacc[slot] = fma(ckdj[jj], acc, wacc[slot]);
              }
            }
          }
        }
        __syncthreads();  // Ek, Y and R are rewritten for the next ket primitives
      }
      }
      // stage V[t,u,v][f] (dense f over |f| <= LCD) for the bra transform,
      // lines (t,u) in order, v contiguous: row vline(t,u) + v
      double *Vs = lds + S::oRp;
      auto vline = [](int t, int u) {
        return hs3(LAB) - hs3(LAB - t) + u * (LAB - t + 1) - u * (u - 1) / 2;
      };
#pragma unroll
      for (int fx = 0; fx <= LCD; ++fx) {
        const int M = LCD - fx;
        const int nyz = (M + 1) * (M + 2) / 2;
#pragma unroll
        for (int k = 0; k < S::slots_fx(fx); ++k) {
          const int slot = S::off_fx(fx) + k;
          if (ybase[slot] >= 0) {
            const int e = tid + NT * k;
            const int h = e / nyz, r = e - h * nyz;
            int fy = 0, rr = r;
            while (rr > M - fy) {
              rr -= M - fy + 1;
              ++fy;
            }
            const int fz = rr;
            const int n = fx + fy + fz, s2 = fy + fz;
            const int code = tuv[h];
            const int t = code & 255, u = (code >> 8) & 255, v = code >> 16;
            Vs[(vline(t, u) + v) * S::NF0 + hs3(n - 1) + s2 * (s2 + 1) / 2 + fz] = wacc[slot];
          }
        }
      }
      __syncthreads();
      const double cw = cab * (I5 ? (comp == 0 ? (ea - eb) / (2.0 * pb) : -1.0) : 1.0);
      // sum over t <= nx, u <= ny, v <= nz of (-1)^(t+u+v) ex[t] ey[u] ez[v] V[t,u,v][f]; the
      // signed z coefficients are held in registers over the shape's whole v range
      auto box = [&](const double *exr, const double *eyr, const double *ezr, int nx, int ny, int nz,
                     int f) {
        double ez[LAB + 1];
#pragma unroll
        for (int v = 0; v <= LAB; ++v) ez[v] = v <= nz ? ((v & 1) ? -ezr[v] : ezr[v]) : 0.0;
        double sb = 0.0;
        for (int t = 0; t <= nx; ++t)
          for (int u = 0; u <= ny; ++u) {
            const double exy = ((t + u) & 1) ? -exr[t] * eyr[u] : exr[t] * eyr[u];
            const double *vr = Vs + vline(t, u) * S::NF0 + f;
            double sv = 0.0;
#pragma unroll
            for (int v = 0; v <= LAB; ++v)
              if (v <= nz) sv = fma(ez[v], vr[v * S::NF0], sv);
            sb = fma(exy, sv, sb);
          }
        return sb;
      };
#pragma unroll
      for (int k = 0; k < S::MAXU; ++k) {
        const int e = tid + NT * k;
        if (e < nu) {
          const int ab = e / nf, f = e - ab * nf + foff;
          int ax, ay, az, bx, by, bz;
          cart_comp(la, ab / nb, ax, ay, az);
          cart_comp(lb, ab % nb, bx, by, bz);
          double sacc = 0.0;
          if constexpr (MODE == 3) {
            // E along the other directions (stride l_a + l_b + 1), G along gdir
            const int GSt = BLAB + 2, g = a.gdir;
            const double *Gb = Fb + 3 * Eab1;
            const int ia[3] = {ax, ay, az}, ib[3] = {bx, by, bz};
            const double *er[3];
            int nn[3];
            for (int d = 0; d < 3; ++d) {
              er[d] = d == g ? Gb + (ia[d] * (lb + 1) + ib[d]) * GSt : Eb + d * Eab1 + (ia[d] * (lb + 1) + ib[d]) * ESt;
              nn[d] = ia[d] + ib[d] + (d == g ? 1 : 0);
            }
            sacc = box(er[0], er[1], er[2], nn[0], nn[1], nn[2], f);
          } else if constexpr (MODE == 2) {
            const double *er[3] = {Eb + (ax * ESb + bx) * ESt, Eb + Eab1 + (ay * ESb + by) * ESt,
                                   Eb + 2 * Eab1 + (az * ESb + bz) * ESt};
            const double *dr[3] = {Fb + (ax * (lb + 1) + bx) * DSt, Fb + Dab1 + (ay * (lb + 1) + by) * DSt,
                                   Fb + 2 * Dab1 + (az * (lb + 1) + bz) * DSt};
            for (int d = 0; d < 3; ++d) {
              const double *exr = d == 0 ? dr[0] : er[0];
              const double *eyr = d == 1 ? dr[1] : er[1];
              const double *ezr = d == 2 ? dr[2] : er[2];
              const int nx = ax + bx + (d == 0 ? 2 : 0), ny = ay + by + (d == 1 ? 2 : 0),
                        nz = az + bz + (d == 2 ? 2 : 0);
              sacc += box(exr, eyr, ezr, nx, ny, nz, f);
            }
          } else {
            const double *exr = (comp == 1 ? Fb : Eb) + (ax * (lb + 1) + bx) * (LAB + 1);
            const double *eyr = (comp == 2 ? Fb : Eb) + Eab1 + (ay * (lb + 1) + by) * (LAB + 1);
            const double *ezr = (comp == 3 ? Fb : Eb) + 2 * Eab1 + (az * (lb + 1) + bz) * (LAB + 1);
            sacc = box(exr, eyr, ezr, ax + bx, ay + by, az + bz, f);
          }
          uacc[k] = fma(cw, sacc, uacc[k]);
        }
      }
      __syncthreads();  // before V staging / E tables are overwritten
    }
  }
  double *Uf = lds + S::oRp;
#pragma unroll
  for (int k = 0; k < S::MAXU; ++k) {
    const int e = tid + NT * k;
    if (e < nu) Uf[e] = uacc[k];
  }
  __syncthreads();
  hrr_store(Uf, la, lb, lc, ld, nf, CD, a.out + o, tid, NT, a.fault);
  __syncthreads();  // Uf is rewritten by the next quartet
  }
}

// Ket primitives per pass: more when the shape's LDS is small, so that
// several work-groups still share a CU.
template <int LAB, int LCD, int MODE>
constexpr int pick_nj() {
  if (BigShape<LAB, LCD, MODE, 8>::BYTES <= 40 * 1024) return 8;
  if (BigShape<LAB, LCD, MODE, 4>::BYTES <= 40 * 1024) return 4;
  if (BigShape<LAB, LCD, MODE, 2>::BYTES <= 64 * 1024) return 2;
  return 1;
}

template <int LAB, int LCD, int MODE, int PREC>
inline int launch_big_t(const ContractArgs &a, unsigned nblocks, hipStream_t st) {
  constexpr int NJ = pick_nj<LAB, LCD, MODE>();
  using S = BigShape<LAB, LCD, MODE, NJ>;
  static_assert(S::BYTES <= 160 * 1024, "LDS per work-group");
  static bool attr = false;
  if (!attr) {
    if (hipFuncSetAttribute((const void *)big_kernel<LAB, LCD, MODE, NJ, PREC>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)S::BYTES) != hipSuccess)
      return -1;
    attr = true;
  }
  if (nblocks == 0) return 0;  // set-up only (before a graph capture)
  hipLaunchKernelGGL((big_kernel<LAB, LCD, MODE, NJ, PREC>), dim3(nblocks), dim3(256), S::BYTES, st, a);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// The Laplacian form of I5 is used where its LDS and register slots fit.
template <int LAB, int LCD>
constexpr bool lap_fits() {
  using S = BigShape<LAB + 2, LCD, 2, 1>;
  return S::BYTES <= 160 * 1024 && S::MAXW <= 40 && S::MAXU <= 32;
}

// The derivative form (MODE 3) where its LDS and register slots fit: every
// shape but those with l_a + l_b = 6 and l_c + l_d = 6.
template <int LAB, int LCD>
constexpr bool grad_fits() {
  using S = BigShape<LAB + 1, LCD, 3, 1>;
  return S::BYTES <= 160 * 1024 && S::MAXW <= 40 && S::MAXU <= 32;
}

// -3: the shape has no derivative form (F12_ELMAX at the boundary)
template <int LAB, int LCD, int PREC>
inline int launch_big_grad(const ContractArgs &a, unsigned nblocks, hipStream_t st) {
  if constexpr (PREC == 0 && grad_fits<LAB, LCD>())
    return launch_big_t<LAB + 1, LCD, 3, PREC>(a, nblocks, st);
  else
    return -3;
}

template <int LAB, int PREC>
inline int launch_big_lab(int lcd, int i5, const ContractArgs &a, unsigned nblocks, hipStream_t st) {
#define F12_BIG_CASE(LCD)                                                                       \
  case LCD:                                                                                     \
    if (a.gdir >= 0) return launch_big_grad<LAB, LCD, PREC>(a, nblocks, st);                    \
    if (!i5) return launch_big_t<LAB, LCD, 0, PREC>(a, nblocks, st);                            \
    if constexpr (lap_fits<LAB, LCD>()) return launch_big_t<LAB + 2, LCD, 2, PREC>(a, nblocks, st); \
    else return launch_big_t<LAB, LCD, 1, PREC>(a, nblocks, st);
  switch (lcd) {
    F12_BIG_CASE(0)
    F12_BIG_CASE(1)
    F12_BIG_CASE(2)
    F12_BIG_CASE(3)
    F12_BIG_CASE(4)
    F12_BIG_CASE(5)
    F12_BIG_CASE(6)
    default:
      return -1;
  }
#undef F12_BIG_CASE
}

}  // namespace f12
