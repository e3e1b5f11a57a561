// Device helpers shared by the contraction kernels (f12_kernels.hip and the
// per-shape kernels of f12_big.h): Hermite index maps, Cartesian
// component order, E coefficients and the launch argument block.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#include "f12_internal.h"

namespace f12 {

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

__host__ __device__ inline int hs3(int L) { return (L + 1) * (L + 2) * (L + 3) / 6; }
__host__ __device__ inline int nc2(int l) { return (l + 1) * (l + 2) / 2; }

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

#define EI(i, j, t) (((i) * nj + (j)) * ntt + (t))

// The tables of the three directions are built by a whole work-group: the
// entries of one level N = i + j depend only on level N - 1, so each level is
// computed in parallel over (direction, i, t), with one barrier per level.
// Direction d is at E + d * stride (and Fd + d * stride).  Every thread of the
// work-group must call it.
__device__ inline void e_tables_wg(double a, double b, double ABx, double ABy, double ABz, int la,
                                   int lb, double *E, double *Fd, int stride, int tid, int nt) {
  const int nj = lb + 1, ntt = la + lb + 1;
  const int ne = (la + 1) * nj * ntt;
  for (int k = tid; k < 3 * ne; k += nt) {
    const int d = k / ne, r = k - d * ne;
    E[d * stride + r] = 0.0;
    if (Fd) Fd[d * stride + r] = 0.0;
  }
  __syncthreads();
  const double p = a + b;
  const double mu = a * b / p;
  const double i2p = 0.5 / p;
  if (tid < 3) {
    const double ab = tid == 0 ? ABx : (tid == 1 ? ABy : ABz);
    const double e0 = exp(-mu * ab * ab);
    E[tid * stride + EI(0, 0, 0)] = e0;
    if (Fd) Fd[tid * stride + EI(0, 0, 0)] = -2.0 * mu * ab * e0;
  }
  __syncthreads();
  for (int N = 1; N <= la + lb; ++N) {
    const int i0 = N - lb > 0 ? N - lb : 0, i1 = la < N ? la : N;
    const int per = (i1 - i0 + 1) * (N + 1);  // (i, t) entries of one direction
    for (int k = tid; k < 3 * per; k += nt) {
      const int d = k / per, r = k - d * per;
      const int i = i0 + r / (N + 1), t = r - (r / (N + 1)) * (N + 1);
      const int j = N - i;
      double *Ed = E + d * stride;
      double *Fdd = Fd ? Fd + d * stride : nullptr;
      if (t >= 1) {
        double v = 0.0, w = 0.0;
        if (i > 0) {
          v += i * Ed[EI(i - 1, j, t - 1)];
          if (Fd) w += i * Fdd[EI(i - 1, j, t - 1)];
        }
        if (j > 0) {
          v += j * Ed[EI(i, j - 1, t - 1)];
          if (Fd) w += j * Fdd[EI(i, j - 1, t - 1)];
        }
        Ed[EI(i, j, t)] = v * i2p / t;
        if (Fd) Fdd[EI(i, j, t)] = w * i2p / t;
      } else {
        const double ab = d == 0 ? ABx : (d == 1 ? ABy : ABz);
        if (i > 0) {
          const double c = -(b / p) * ab;
          Ed[EI(i, j, 0)] = c * Ed[EI(i - 1, j, 0)] + Ed[EI(i - 1, j, 1)];
          if (Fd)
            Fdd[EI(i, j, 0)] = c * Fdd[EI(i - 1, j, 0)] + Fdd[EI(i - 1, j, 1)] -
                               (b / p) * Ed[EI(i - 1, j, 0)];
        } else {
          const double c = (a / p) * ab;
          Ed[EI(i, j, 0)] = c * Ed[EI(i, j - 1, 0)] + Ed[EI(i, j - 1, 1)];
          if (Fd)
            Fdd[EI(i, j, 0)] = c * Fdd[EI(i, j - 1, 0)] + Fdd[EI(i, j - 1, 1)] +
                               (a / p) * Ed[EI(i, j - 1, 0)];
        }
      }
    }
    __syncthreads();
  }
}
#undef EI


struct ContractArgs {
  PairsDev bra, ket;
  const int64_t *qb, *qk, *qoff, *qprim;
  int64_t qa, nqc, p0, np;  // quartets [qa, qa + nqc)
  const double *A;
  int la, lb, lc, ld, i5;
  double *out;
  int64_t out_base;
  int prec;    // 0: FP64; 1: ket transform in split FP32
  int *fault;  // the device's fault word (set on a non-finite output element)
  int gdir;    // -1: the integrals; 0, 1, 2: d/dA_x, d/dA_y, d/dA_z of them
};

// Position of one-centre component (fx, fy, fz) among |f| = l_c .. l_c+l_d.
__device__ __forceinline__ int findex(int fx, int fy, int fz, int lc) {
  const int n = fx + fy + fz, s = fy + fz;
  return hs3(n - 1) - hs3(lc - 1) + s * (s + 1) / 2 + fz;
}

__device__ __forceinline__ int binom3(int d, int k) {
  return (k == 0 || k == d) ? 1 : (d == 2 ? 2 : 3);
}

__device__ __forceinline__ double ipow(double x, int n) {
  double r = 1.0;
  for (int i = 0; i < n; ++i) r *= x;
  return r;
}


// Ket one-centre E^f_phi, f <= Lcd, at E[f(f+1)/2 + phi].
__device__ inline void e_onecentre(double q, double XQC, int Lcd, double *E) {
  const double i2q = 0.5 / q;
  E[0] = 1.0;
  for (int f = 0; f < Lcd; ++f) {
    const double *e = E + f * (f + 1) / 2;
    double *en = E + (f + 1) * (f + 2) / 2;
    for (int ph = 0; ph <= f + 1; ++ph) {
      double v = 0.0;
      if (ph > 0) v += i2q * e[ph - 1];
      if (ph <= f) v += XQC * e[ph];
      if (ph + 1 <= f) v += (ph + 1) * e[ph + 1];
      en[ph] = v;
    }
  }
}

// (ab|f) -> (ab|cd) by x_D^d = sum_k C(d,k) (C_x - D_x)^(d-k) x_C^k (and y, z),
// then the store of the contracted block; U[ab * nf + f] in LDS.  A non-finite
// element sets the device's fault word.
__device__ inline void hrr_store(const double *U, int la, int lb, int lc, int ld, int nf,
                                 const double CD[3], double *out, int tid, int nt, int *fault) {
  const int nd = ncart(ld), ncd = ncart(lc) * nd;
  const int nab = ncart(la) * ncart(lb);
  for (int e = tid; e < nab * ncd; e += nt) {
    const int ab = e / ncd, cd = e - ab * ncd;
    int cx, cy, cz, dx, dy, dz;
    cart_comp(lc, cd / nd, cx, cy, cz);
    cart_comp(ld, cd % nd, dx, dy, dz);
    const double *u = U + ab * nf;
    double s = 0.0;
    for (int kx = 0; kx <= dx; ++kx) {
      const double wx = binom3(dx, kx) * ipow(CD[0], dx - kx);
      for (int ky = 0; ky <= dy; ++ky) {
        const double wy = wx * binom3(dy, ky) * ipow(CD[1], dy - ky);
        for (int kz = 0; kz <= dz; ++kz) {
          const double wz = wy * binom3(dz, kz) * ipow(CD[2], dz - kz);
          s = fma(wz, u[findex(cx + kx, cy + ky, cz + kz, lc)], s);
        }
      }
    }
    if (!isfinite(s)) *fault = 1;
    out[e] = s;
  }
}

}  // namespace f12
