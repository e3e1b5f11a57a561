// The Hobson / spherical-tensor route to the Hermite integrals (Sec. II.D),
// an alternative to the MD recurrence of the contraction kernels:
//   Eq. (Ylm):  Y_lm(nabla) g(Q) = [D^l g](Q) Q^l Y_lm(Q^),  D = Q^-1 d/dQ,
// in real form with the solid harmonics S_lm of f12_sph.hip.  A Cartesian
// derivative d^t_x d^u_y d^v_z is the operator of the monomial x^t y^u z^v
// with x, y, z replaced by the derivatives; that monomial decomposes as
//   x^t y^u z^v = sum_{l = N, N-2, ...} r^(N-l) sum_m c_{tuv,lm} S_lm,  N = t+u+v,
// so d^{tuv} = sum c_{tuv,lm} (nabla^2)^k S_lm(nabla), k = (N - l)/2.  The
// powers of the Laplacian are the correction that Eq. (QxQyQz) leaves out;
// on a radial function nabla^2 h = 3 D h + Q^2 D^2 h, and nabla^2 commutes
// with S_lm(nabla), so
//   R_tuv = sum_{l,m} c_{tuv,lm} S_lm(X) [D^l (3D + Q^2 D^2)^k B](X),
// which with D Q^2 = Q^2 D + 2 is a polynomial sum_{i,j} e_ij Q^(2i) A_j in
// the radial derivatives A_j = D^j B.  The coefficients c come from sphere
// moments (the S_lm are orthogonal on the sphere with norm 4 pi / (2l+1)).
// Diagnostic entry point: R_tuv for given A_n and X, one thread per (point,
// Hermite index), tables in device memory.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#include <algorithm>
#include <cstdlib>
#include <map>
#include <tuple>
#include <mutex>
#include <vector>

#include "../../include/f12int.h"
#include "f12_internal.h"

namespace f12 {
namespace {

constexpr int HMAX = LTOT_MAX;  // Hermite order up to 14

inline int ncart_(int l) { return (l + 1) * (l + 2) / 2; }
// canonical index of (i, j, k = l - i - j): i from l down, then j from l - i down
inline int cidx(int l, int i, int j) { return (l - i) * (l - i + 1) / 2 + (l - i - j); }
inline int hidx(int t, int u, int v) {  // Hermite order: by N, then t descending, then u descending
  const int N = t + u + v, s = N - t;
  return N * (N + 1) * (N + 2) / 6 + s * (s + 1) / 2 + (s - u);
}

using Poly = std::vector<double>;  // homogeneous of degree l, ncart(l) coefficients

Poly mul_axis(const Poly &p, int l, int axis) {  // times x, y or z
  Poly r(ncart_(l + 1), 0.0);
  for (int i = 0; i <= l; ++i)
    for (int j = 0; i + j <= l; ++j) {
      const double c = p[cidx(l, i, j)];
      if (c == 0.0) continue;
      const int ii = i + (axis == 0), jj = j + (axis == 1);
      r[cidx(l + 1, ii, jj)] += c;
    }
  return r;
}

Poly mul_r2(const Poly &p, int l) {
  Poly r(ncart_(l + 2), 0.0);
  for (int a = 0; a < 3; ++a) {
    Poly q = mul_axis(mul_axis(p, l, a), l + 1, a);
    for (size_t n = 0; n < r.size(); ++n) r[n] += q[n];
  }
  return r;
}

// real solid harmonics, Racah's normalisation, l <= HMAX (recurrences as in f12_sph.hip)
std::vector<std::vector<Poly>> solid(int lmax) {
  std::vector<std::vector<Poly>> S(lmax + 1);
  S[0] = {Poly{1.0}};
  for (int l = 0; l < lmax; ++l) {
    S[l + 1].assign(2 * l + 3, Poly());
    auto at = [&](int m) -> const Poly & { return S[l][m + l]; };
    const double s = std::sqrt((l == 0 ? 2.0 : 1.0) * (2 * l + 1) / (2.0 * l + 2.0));
    Poly top = mul_axis(at(l), l, 0), bot = mul_axis(at(l), l, 1);
    if (l > 0) {
      Poly yl = mul_axis(at(-l), l, 1), xl = mul_axis(at(-l), l, 0);
      for (size_t n = 0; n < top.size(); ++n) {
        top[n] -= yl[n];
        bot[n] += xl[n];
      }
    }
    for (auto &v : top) v *= s;
    for (auto &v : bot) v *= s;
    for (int m = -l; m <= l; ++m) {
      Poly p = mul_axis(at(m), l, 2);
      for (auto &v : p) v *= (2 * l + 1);
      if (std::abs(m) <= l - 1) {
        Poly q = mul_r2(S[l - 1][m + l - 1], l - 1);
        const double w = std::sqrt((double)(l + m) * (l - m));
        for (size_t n = 0; n < p.size(); ++n) p[n] -= w * q[n];
      }
      const double d = 1.0 / std::sqrt((double)(l + m + 1) * (l - m + 1));
      for (auto &v : p) v *= d;
      S[l + 1][m + l + 1] = p;
    }
    S[l + 1][2 * l + 2] = top;
    S[l + 1][0] = bot;
  }
  return S;
}

double sphere_moment(int a, int b, int c) {  // int over the unit sphere of x^a y^b z^c
  if ((a | b | c) & 1) return 0.0;
  return 2.0 * std::tgamma(0.5 * (a + 1)) * std::tgamma(0.5 * (b + 1)) * std::tgamma(0.5 * (c + 1)) /
         std::tgamma(0.5 * (a + b + c + 3));
}

// D^l (3D + u D^2)^k as sum_{i,j} e_ij u^i D^j (u = Q^2, D u = u D + 2)
std::map<std::pair<int, int>, double> radial_op(int l, int k) {
  std::map<std::pair<int, int>, double> P{{{0, 0}, 1.0}};
  auto applyD = [](const std::map<std::pair<int, int>, double> &A) {
    std::map<std::pair<int, int>, double> r;
    for (auto &[key, c] : A) {
      const int i = key.first, j = key.second;
      r[{i, j + 1}] += c;                    // u^i D (D^j)
      if (i > 0) r[{i - 1, j}] += 2.0 * i * c;  // D u^i = u^i D + 2 i u^(i-1)
    }
    return r;
  };
  auto applyU = [](const std::map<std::pair<int, int>, double> &A) {
    std::map<std::pair<int, int>, double> r;
    for (auto &[key, c] : A) r[{key.first + 1, key.second}] += c;
    return r;
  };
  // operators act to the right: build (3D + u D^2)^k first, then D^l on the left
  for (int s = 0; s < k; ++s) {
    auto d1 = applyD(P);
    auto d2 = applyU(applyD(d1));
    std::map<std::pair<int, int>, double> r;
    for (auto &[key, c] : d1) r[key] += 3.0 * c;
    for (auto &[key, c] : d2) r[key] += c;
    P = r;
  }
  for (int s = 0; s < l; ++s) P = applyD(P);
  return P;
}

struct HobsonTables {
  // per Hermite index h: terms [toff[h], toff[h+1]) of (l, m, k, c)
  std::vector<int32_t> toff, tl, tm;
  std::vector<double> tc;
  // per (l, m): monomials [soff, soff + n) of (i, j, coef)
  std::vector<int32_t> soff, si, sj;
  std::vector<double> sc;
  // per (l, k): radial terms of (i, j, e)
  std::vector<int32_t> roff, ri, rj;
  std::vector<double> re;
};

HobsonTables build_tables() {
  HobsonTables T;
  const auto S = solid(HMAX);
  // solid harmonics, flat over (l, m) with index l^2 + m + l
  T.soff.push_back(0);
  for (int l = 0; l <= HMAX; ++l)
    for (int m = -l; m <= l; ++m) {
      const Poly &p = S[l][m + l];
      for (int i = 0; i <= l; ++i)
        for (int j = 0; i + j <= l; ++j) {
          const double c = p[cidx(l, i, j)];
          if (std::fabs(c) < 1e-300) continue;
          T.si.push_back(i);
          T.sj.push_back(j);
          T.sc.push_back(c);
        }
      T.soff.push_back((int32_t)T.sc.size());
    }
  // radial operators, flat over (l, k) with l + 2k <= HMAX: index l * (HMAX/2 + 1) + k
  const int KW = HMAX / 2 + 1;
  T.roff.assign((HMAX + 1) * KW + 1, 0);
  for (int l = 0; l <= HMAX; ++l)
    for (int k = 0; k < KW; ++k) {
      T.roff[l * KW + k] = (int32_t)T.re.size();
      if (l + 2 * k <= HMAX)
        for (auto &[key, e] : radial_op(l, k)) {
          T.ri.push_back(key.first);
          T.rj.push_back(key.second);
          T.re.push_back(e);
        }
    }
  T.roff[(HMAX + 1) * KW] = (int32_t)T.re.size();
  // monomial decomposition per Hermite index
  const int HLn = (HMAX + 1) * (HMAX + 2) * (HMAX + 3) / 6;
  std::vector<std::vector<std::tuple<int, int, double>>> per(HLn);
  for (int N = 0; N <= HMAX; ++N)
    for (int t = N; t >= 0; --t)
      for (int u = N - t; u >= 0; --u) {
        const int v = N - t - u;
        auto &out = per[hidx(t, u, v)];
        for (int l = N % 2; l <= N; l += 2)
          for (int m = -l; m <= l; ++m) {
            const Poly &p = S[l][m + l];
            double s = 0.0;
            for (int i = 0; i <= l; ++i)
              for (int j = 0; i + j <= l; ++j) {
                const double c = p[cidx(l, i, j)];
                if (c != 0.0) s += c * sphere_moment(t + i, u + j, v + (l - i - j));
              }
            const double c = s * (2 * l + 1) / (4.0 * M_PI);
            if (std::fabs(c) > 1e-13) out.emplace_back(l, m, c);
          }
      }
  T.toff.push_back(0);
  for (int h = 0; h < HLn; ++h) {
    for (auto &[l, m, c] : per[h]) {
      T.tl.push_back(l);
      T.tm.push_back(m);
      T.tc.push_back(c);
    }
    T.toff.push_back((int32_t)T.tc.size());
  }
  return T;
}

struct DevTables {
  int32_t *toff, *tl, *tm, *soff, *si, *sj, *roff, *ri, *rj;
  double *tc, *sc, *re;
};

std::mutex g_mu;
DevTables g_dev[64];
bool g_have[64] = {};

template <typename T>
T *upload(const std::vector<T> &v) {
  T *p = nullptr;
  if (hipMalloc((void **)&p, std::max<size_t>(v.size(), 1) * sizeof(T)) != hipSuccess) return nullptr;
  if (!v.empty() && hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
  return p;
}

int device_tables(DevTables *out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return F12_EDEVICE;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_have[dev]) {
    static const HobsonTables T = build_tables();
    DevTables d{upload(T.toff), upload(T.tl), upload(T.tm), upload(T.soff), upload(T.si), upload(T.sj),
                upload(T.roff), upload(T.ri), upload(T.rj), upload(T.tc), upload(T.sc), upload(T.re)};
    if (!d.toff || !d.tl || !d.tm || !d.soff || !d.si || !d.sj || !d.roff || !d.ri || !d.rj || !d.tc || !d.sc ||
        !d.re)
      return F12_ENOMEM;
    g_dev[dev] = d;
    g_have[dev] = true;
  }
  *out = g_dev[dev];
  return F12_OK;
}

}  // namespace

__global__ void hobson_r_kernel(DevTables T, const double *__restrict__ A, const double *__restrict__ X,
                                int64_t np, int L, double *__restrict__ R) {
  const int HLn = (L + 1) * (L + 2) * (L + 3) / 6;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= np * HLn) return;
  const int64_t p = g / HLn;
  const int h = (int)(g - p * HLn);
  const double x = X[3 * p], y = X[3 * p + 1], z = X[3 * p + 2];
  const double u = x * x + y * y + z * z;
  const double *a = A + p * (L + 1);
  const int KW = HMAX / 2 + 1;
  int Nh = 0;  // the order N = t + u + v of Hermite index h; N = l + 2k
  while ((Nh + 1) * (Nh + 2) * (Nh + 3) / 6 <= h) ++Nh;
  double r = 0.0;
  for (int q = T.toff[h]; q < T.toff[h + 1]; ++q) {
    const int l = T.tl[q], m = T.tm[q];
    // S_lm(X)
    const int f = l * l + m + l;
    double s = 0.0;
    for (int w = T.soff[f]; w < T.soff[f + 1]; ++w) {
      const int i = T.si[w], j = T.sj[w], k = l - i - j;
      s += T.sc[w] * pow(x, i) * pow(y, j) * pow(z, k);
    }
    const int k = (Nh - l) / 2;
    double rad = 0.0;
    for (int w = T.roff[l * KW + k]; w < T.roff[l * KW + k + 1]; ++w) rad += T.re[w] * pow(u, T.ri[w]) * a[T.rj[w]];
    r += T.tc[q] * s * rad;
  }
  R[p * HLn + h] = r;
}

}  // namespace f12

using namespace f12;

extern "C" int f12_hermite_hobson(const double *d_A, const double *d_X, int64_t np, int32_t L, double *d_R,
                                  void *stream) {
  if (!d_A || !d_X || !d_R || np < 0 || L < 0 || L > HMAX) return F12_EINVAL;
  if (np == 0) return F12_OK;
  DevTables T;
  const int s = device_tables(&T);
  if (s) return s;
  const int64_t HLn = (int64_t)(L + 1) * (L + 2) * (L + 3) / 6;
  const int64_t n = np * HLn;
  const int nt = 128;
  hipLaunchKernelGGL(hobson_r_kernel, dim3((unsigned)((n + nt - 1) / nt)), dim3(nt), 0, (hipStream_t)stream, T,
                     d_A, d_X, np, (int)L, d_R);
  return hipGetLastError() == hipSuccess ? F12_OK : F12_EDEVICE;
}
