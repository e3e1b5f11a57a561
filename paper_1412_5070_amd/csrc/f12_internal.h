// Internal data layouts shared by the host code (f12_host.cpp) and the HIP
// kernels (f12_kernels.hip).  Not part of the public ABI.
#pragma once
#include <stdint.h>

namespace f12 {

constexpr int LMAX = 3;                 // f shells
constexpr int LTOT_MAX = 4 * LMAX + 2;  // I5 (ff|ff): 14
constexpr int MAX_CHAINS = 16;
constexpr int MAX_TERMS = 96;
constexpr int MAX_FAMILIES = 4;
constexpr int NEG_POW_MAX = 12;        // most negative integer power of a kernel term
constexpr int KT = 16;                  // Taylor terms of the W-table interpolation
constexpr int KPHI = 96;                // terms of the DD Phi-series (small-T route)
constexpr int NW_LIGHT = 32;            // the same bound for the common kernels
constexpr int NW_MAX = 64;              // orders of W per chain in the large-T route:
                                        // (m_max - m_min) + LTOT_MAX + 1 must not exceed it
constexpr int SPAN_C = 6;               // widest chain (m_max - m_min) of the register-resident
                                        // large-T path (kernels that are not heavy)
constexpr double WX_LO = -10.5;         // W-table abscissa range
constexpr double WX_HI = 36.0;
constexpr double WX_INVH = 64.0;        // grid step 1/64

// One term c * r^alpha * exp(b r - g r^2) of K_i(r) = r k_i(r); alpha = alpha0(chain) + m.
struct TermDesc {
  double c, clo;  // coefficient as a double-double c + clo
  int32_t m;
  int32_t chain;
};

// A chain: terms sharing (b, g, alpha mod 1).
struct ChainDesc {
  double b, g;
  int32_t family;      // index into KernelDev::fam
  int32_t t_begin, t_end;
  int32_t m_min, m_max;
  int32_t phi_off;     // offset (in DD pairs) of this chain's Phi-series coefficients
};

// Table W_a(x) for a = alpha0 + m, m in [m_lo, m_hi]; layout [ix][m - m_lo].
struct FamilyDesc {
  double alpha0;
  int32_t is_int;
  int32_t m_lo, m_hi, nm;
  int32_t nx;
  const double *table;
};

struct KernelDev {
  int32_t cls;
  int32_t nchains, nterms, nfam;
  int32_t negint;  // 1 if an integer family has negative powers (finite parts with log terms)
  int32_t heavy;   // negint, or a chain spanning more than NW_LIGHT orders in the large-T route
  int32_t singular;  // a term r^a with a <= -1 (finite parts; their singular pieces cancel across chains)
  int32_t negb;      // a decaying chain (b < 0)
  int32_t compact;   // not heavy, and every chain spans at most SPAN_C orders
  ChainDesc chains[MAX_CHAINS];
  TermDesc terms[MAX_TERMS];
  FamilyDesc fam[MAX_FAMILIES];
  // Phi-series coefficients for the small-T route, DD pairs (hi, lo):
  // for chain c, start index s in {0,1}: F((a_s + 1 + k)/2) / (2 k!),
  // a_s = alpha0 + m_min + 1 + s, k = 0..KPHI, with F = Gamma, except at its
  // poles -p (p = 0, 1, ...), where the finite part of int t^(-2p-1) e^{-t^2}
  // takes its place: F = (-1)^p psi(p + 1) / p!.
  const double *phi;
};

// Which radial-derivative kernel a launch takes: 1 heavy, 2 compact (orders
// and arrays fixed at compile time per L), 0 the other light kernels.
inline int aux_variant(const KernelDev &K) { return K.heavy ? 1 : (K.compact ? 2 : 0); }

// Device-side pair data (structure of arrays).
struct PairsDev {
  int64_t nsp, npp;
  int32_t nshell, ordered;
  // shell pairs
  const int32_t *sa, *sb;
  const int32_t *la, *lb, *ka, *kb;
  const int64_t *pp_off;
  const double *ABx, *ABy, *ABz;  // A - B
  // primitive pairs
  const double *ea, *eb, *p, *Px, *Py, *Pz, *cab;
};

// One bin of quartets with equal (la, lb, lc, ld), in processing order.
struct BinDev {
  int32_t la, lb, lc, ld;
  int64_t q0, nq;  // range in the processing-order arrays
};

}  // namespace f12
