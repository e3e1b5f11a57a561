// Output over real solid harmonics: the Cartesian blocks that f12_eval writes,
// transformed index by index to the regular solid harmonics S_lm
// (m = -l..l), the basis in which the paper's spherical tensor gradient
// operators Y_lm(nabla) of Eq. (Ylm) are written (Sec. II.D).  The real forms
// take the combinations of m and -m; the normalisation is Racah's:
//   S_lm(r) = sqrt(4 pi / (2l + 1)) r^l Y_lm(r^),  S_l0 = z^l + ...,
// so that S_11 = x, S_1-1 = y, S_10 = z, S_22 = sqrt(3)/2 (x^2 - y^2).
// A contracted shell of unnormalised primitives, phi_i = x^a y^b z^c e^{-e r^2}
// over its Cartesian components, becomes sum_i C_lm,i phi_i = S_lm e^{-e r^2}.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <vector>

#include "../../include/f12int.h"
#include "f12_handles.h"

namespace f12 {

constexpr int SPH_NF = (LMAX + 1) * (LMAX + 1);  // functions S_lm, l <= LMAX
constexpr int SPH_NNZ = 4;                        // monomials of one S_lm, l <= 3

struct SphTable {
  int32_t n[SPH_NF];
  int32_t idx[SPH_NF][SPH_NNZ];  // Cartesian component (canonical order of degree l)
  double c[SPH_NF][SPH_NNZ];
};

namespace {

// Index of (i, j, k), i + j + k = l, in the canonical Cartesian order: i from
// l down to 0, then j from l - i down to 0.
int cart_index(int l, int i, int j) {
  int base = 0;
  for (int ii = l; ii > i; --ii) base += l - ii + 1;
  return base + (l - i - j);
}

// Polynomials in x, y, z as dense coefficient arrays P[i][j][k] (degree <= LMAX + 2).
constexpr int PD = LMAX + 3;
struct Poly {
  double a[PD][PD][PD] = {};
};

Poly times(const Poly &p, int di, int dj, int dk, double s) {
  Poly r;
  for (int i = 0; i < PD; ++i)
    for (int j = 0; j < PD; ++j)
      for (int k = 0; k < PD; ++k)
        if (p.a[i][j][k] != 0.0 && i + di < PD && j + dj < PD && k + dk < PD)
          r.a[i + di][j + dj][k + dk] += s * p.a[i][j][k];
  return r;
}

void axpy(Poly &r, const Poly &p, double s) {
  for (int i = 0; i < PD; ++i)
    for (int j = 0; j < PD; ++j)
      for (int k = 0; k < PD; ++k) r.a[i][j][k] += s * p.a[i][j][k];
}

// S_lm by the standard recurrences of the real solid harmonics in Racah's
// normalisation (raising l along the diagonal m = +-l, then in z):
//   S_{l+1,l+1}  = sqrt(2^d (2l+1)/(2l+2)) (x S_ll - [l > 0] y S_l,-l)
//   S_{l+1,-l-1} = sqrt(2^d (2l+1)/(2l+2)) (y S_ll + [l > 0] x S_l,-l),  d = [l = 0]
//   S_{l+1,m} = ((2l+1) z S_lm - sqrt((l+m)(l-m)) r^2 S_{l-1,m}) / sqrt((l+m+1)(l-m+1))
std::vector<Poly> solid_harmonics() {
  std::vector<Poly> S((LMAX + 1) * (LMAX + 1));
  auto at = [&](int l, int m) -> Poly & { return S[l * l + m + l]; };
  at(0, 0).a[0][0][0] = 1.0;
  for (int l = 0; l < LMAX; ++l) {
    const double s = std::sqrt((l == 0 ? 2.0 : 1.0) * (2 * l + 1) / (2.0 * l + 2.0));
    Poly top = times(at(l, l), 1, 0, 0, s), bot = times(at(l, l), 0, 1, 0, s);
    if (l > 0) {
      axpy(top, times(at(l, -l), 0, 1, 0, s), -1.0);
      axpy(bot, times(at(l, -l), 1, 0, 0, s), 1.0);
    }
    for (int m = -l; m <= l; ++m) {
      Poly p = times(at(l, m), 0, 0, 1, 2 * l + 1);
      if (std::abs(m) <= l - 1) {
        const double w = -std::sqrt((double)(l + m) * (l - m));
        axpy(p, times(at(l - 1, m), 2, 0, 0, w), 1.0);
        axpy(p, times(at(l - 1, m), 0, 2, 0, w), 1.0);
        axpy(p, times(at(l - 1, m), 0, 0, 2, w), 1.0);
      }
      at(l + 1, m) = times(p, 0, 0, 0, 1.0 / std::sqrt((double)(l + m + 1) * (l - m + 1)));
    }
    at(l + 1, l + 1) = top;
    at(l + 1, -l - 1) = bot;
  }
  return S;
}

std::once_flag g_sph_once;
SphTable g_sph;
std::vector<std::vector<double>> g_sph_dense;  // per l: (2l+1) x ncart(l), row-major

void build_tables() {
  const std::vector<Poly> S = solid_harmonics();
  g_sph = SphTable{};
  g_sph_dense.assign(LMAX + 1, {});
  for (int l = 0; l <= LMAX; ++l) {
    const int nc = (l + 1) * (l + 2) / 2;
    g_sph_dense[l].assign((size_t)(2 * l + 1) * nc, 0.0);
    for (int m = -l; m <= l; ++m) {
      const int f = l * l + m + l;
      int n = 0;
      for (int i = l; i >= 0; --i)
        for (int j = l - i; j >= 0; --j) {
          const double v = S[f].a[i][j][l - i - j];
          if (std::fabs(v) < 1e-14) continue;
          g_sph.idx[f][n] = cart_index(l, i, j);
          g_sph.c[f][n] = v;
          g_sph_dense[l][(size_t)(m + l) * nc + cart_index(l, i, j)] = v;
          ++n;
        }
      g_sph.n[f] = n;
    }
  }
}

// the list's bins in public order (ascending first quartet)
std::vector<Bin> bins_in_order(const f12_quartets *q) {
  std::vector<Bin> b = q->bins;
  std::sort(b.begin(), b.end(), [](const Bin &x, const Bin &y) { return x.q0 < y.q0; });
  return b;
}

}  // namespace

// One work-group per quartet of a bin (equal l_a..l_d), one thread per
// spherical element; each element sums the few Cartesian elements that its
// four S_lm contain (at most 4 per index).
__global__ void __launch_bounds__(128) cart_to_sph_kernel(const double *__restrict__ cart,
                                                         double *__restrict__ sph,
                                                         const int64_t *__restrict__ qoff, int64_t q0,
                                                         int64_t nq, int64_t cart_base, int64_t sph0,
                                                         int la, int lb, int lc, int ld, SphTable T) {
  const int nb = (lb + 1) * (lb + 2) / 2;
  const int nc = (lc + 1) * (lc + 2) / 2, nd = (ld + 1) * (ld + 2) / 2;
  const int sa = 2 * la + 1, sb = 2 * lb + 1, sc = 2 * lc + 1, sd = 2 * ld + 1;
  const int nsph = sa * sb * sc * sd;
  for (int64_t qi = blockIdx.x; qi < nq; qi += gridDim.x) {
    const double *in = cart + (qoff[q0 + qi] - cart_base);
    double *out = sph + sph0 + qi * nsph;
    for (int e = threadIdx.x; e < nsph; e += blockDim.x) {
      const int md = e % sd, r1 = e / sd;
      const int mc = r1 % sc, r2 = r1 / sc;
      const int mb = r2 % sb, ma = r2 / sb;
      const int fa = la * la + ma, fb = lb * lb + mb, fc = lc * lc + mc, fd = ld * ld + md;
      double s = 0.0;
      for (int ia = 0; ia < T.n[fa]; ++ia)
        for (int ib = 0; ib < T.n[fb]; ++ib) {
          const double cab = T.c[fa][ia] * T.c[fb][ib];
          const int64_t oab = ((int64_t)T.idx[fa][ia] * nb + T.idx[fb][ib]) * nc;
          for (int ic = 0; ic < T.n[fc]; ++ic) {
            const double cabc = cab * T.c[fc][ic];
            const double *row = in + (oab + T.idx[fc][ic]) * nd;
            for (int id = 0; id < T.n[fd]; ++id) s = fma(cabc * T.c[fd][id], row[T.idx[fd][id]], s);
          }
        }
      out[e] = s;
    }
  }
}

}  // namespace f12

using namespace f12;

extern "C" int f12_sph_coefficients(int32_t l, double *out) {
  if (l < 0 || l > LMAX || !out) return F12_EINVAL;
  std::call_once(g_sph_once, build_tables);
  std::copy(g_sph_dense[l].begin(), g_sph_dense[l].end(), out);
  return F12_OK;
}

extern "C" int f12_quartet_offsets_sph(const f12_quartets *q, int64_t *offsets) {
  if (!q || !offsets) return F12_EINVAL;
  offsets[0] = 0;
  int64_t pos = 0;
  for (const Bin &b : bins_in_order(q)) {
    const int64_t n = (int64_t)(2 * b.la + 1) * (2 * b.lb + 1) * (2 * b.lc + 1) * (2 * b.ld + 1);
    for (int64_t i = 0; i < b.nq; ++i) {
      pos += n;
      offsets[b.q0 + i + 1] = pos;
    }
  }
  return F12_OK;
}

extern "C" int f12_cart_to_sph(const f12_quartets *q, int64_t q_begin, int64_t q_end, const double *d_cart,
                               double *d_sph, int64_t sph_capacity, void *stream) {
  if (!q || !d_cart || !d_sph || q_begin < 0 || q_end > q->nq || q_begin > q_end) return F12_EINVAL;
  std::call_once(g_sph_once, build_tables);
  // spherical offsets of the range, bin by bin (a bin's blocks have one size)
  const std::vector<Bin> bins = bins_in_order(q);
  int64_t need = 0;
  for (const Bin &b : bins) {
    const int64_t lo = std::max(b.q0, q_begin), hi = std::min(b.q0 + b.nq, q_end);
    if (lo < hi) need += (hi - lo) * (2 * b.la + 1) * (2 * b.lb + 1) * (2 * b.lc + 1) * (2 * b.ld + 1);
  }
  if (need > sph_capacity) return F12_EBUFSIZE;
  if (q_begin == q_end) return F12_OK;
  const int64_t cart_base = q->qoff[q_begin];
  int64_t sph0 = 0;
  for (const Bin &b : bins) {
    const int64_t lo = std::max(b.q0, q_begin), hi = std::min(b.q0 + b.nq, q_end);
    if (lo >= hi) continue;
    const int64_t nq = hi - lo;
    const unsigned grid = (unsigned)std::min<int64_t>(nq, 65536);
    hipLaunchKernelGGL(cart_to_sph_kernel, dim3(grid), dim3(128), 0, (hipStream_t)stream, d_cart, d_sph,
                       q->d_qoff.ptr, lo, nq, cart_base, sph0, b.la, b.lb, b.lc, b.ld, g_sph);
    if (hipGetLastError() != hipSuccess) return F12_EDEVICE;
    sph0 += nq * (2 * b.la + 1) * (2 * b.lb + 1) * (2 * b.lc + 1) * (2 * b.ld + 1);
  }
  return F12_OK;
}
