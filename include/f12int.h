/*
 * f12int.h - C ABI of the MI355X (gfx950) library that evaluates, in batches,
 * the two-electron integral classes of explicitly correlated (F12) methods
 * with the range-separated correlation factor of Silkowski, Lesiuk and
 * Moszynski (arXiv:1412.5070), over contracted Cartesian Gaussian shells.
 *
 *   I1 = (ab| 1/r12 |cd)            Eq. (I1)
 *   I2 = (ab| f/r12 |cd)            Eq. (I2)
 *   I3 = (ab| f |cd)                Eq. (I3)
 *   I4 = (ab| f f' |cd)             Eq. (I4)
 *   I5 = (ab| [f, T1] |cd)          Eq. (I5), evaluated as 1/2 (lap_A - lap_B) I3, Eq. (I5_)
 *   I6 = (ab| [[f, T1], f'] |cd)    Eq. (I6), evaluated as (ab| f_r f'_r |cd), Eq. (I6_)
 *
 * with f(r) = (1 + r/2) exp(-mu r^2) + S_n(mu r^2) c0 r^rho exp(B r)   Eq. (rs12)
 * and  S_n(x) = 1 - exp(-x) sum_{k<=n} x^k / k!                        Eq. (ttdamp).
 *
 * Orbitals are unnormalised primitive Cartesian Gaussians x_A^i y_A^k z_A^m
 * exp(-a r_A^2) (Eq. (basis)); contraction coefficients are used as given.
 * Cartesian components of a shell of angular momentum l are ordered (i,k,m)
 * with i from l down to 0, then k from l-i down to 0.  Coordinates in bohr.
 *
 * Conventions for every function:
 *  - return an int status: F12_OK (0) or a negative f12_status; nothing is
 *    thrown across the ABI.  Argument validation happens before any launch.
 *  - host pointers are read during the call only (the library copies what it
 *    keeps); device pointers ("d_") must stay valid until the work enqueued
 *    on the given HIP stream has completed.
 *  - handles are owned by the library and freed by the matching *_destroy.
 *  - stream arguments are hipStream_t passed as void* (NULL = default stream).
 */
#ifndef F12INT_H
#define F12INT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  F12_OK = 0,
  F12_EINVAL = -1,    /* bad argument (null pointer, out-of-range index, ...)   */
  F12_EPARAM = -2,    /* factor parameters rejected (mu <= 0, non-finite, n   */
                      /* violating n > -rho/2 - 1 for rho < -2, or a kernel     */
                      /* term the library does not support: a negative integer  */
                      /* power, a power <= -2, b < 0 with a non-integer power,  */
                      /* or too many terms/chains                              */
                      /* or too wide a range of powers in one chain)           */
  F12_ELMAX = -3,     /* angular momentum above the supported maximum           */
  F12_ENOMEM = -4,    /* host or device allocation failed                       */
  F12_EDEVICE = -5,   /* a HIP runtime call failed                              */
  F12_EBUFSIZE = -6,  /* output buffer too small for the requested range        */
  F12_ENONFINITE = -7 /* a kernel produced a non-finite value (f12_stream_status) */
} f12_status;

typedef enum {
  F12_I1_COULOMB = 1,
  F12_I2_F_OVER_R = 2,
  F12_I3_F = 3,
  F12_I4_FFP = 4,
  F12_I5_COMM_T1 = 5,
  F12_I6_DF_DFP = 6
} f12_class;

/* Parameters of one range-separated factor, Eq. (rs12) and Eq. (ttdamp).
 * c0, rho, B: any finite reals; mu > 0; n >= 0 integer, and n > -rho/2 - 1
 * when rho < -2 (the paper's condition for a regular factor at r = 0). */
typedef struct {
  double c0, rho, B, mu;
  int32_t n;
  int32_t reserved; /* must be 0 */
} f12_factor;

/* One contracted shell: angular momentum l (0..F12_LMAX), nprim primitives
 * whose exponents/coefficients are exps/coefs[first_prim .. first_prim+nprim),
 * centred on centre index `center`. */
typedef struct {
  int32_t l, nprim, center, first_prim;
} f12_shell;

#define F12_LMAX 3         /* s, p, d, f shells                                  */
#define F12_MAX_KPRIM 16   /* primitives per shell                               */

typedef struct f12_basis f12_basis;
typedef struct f12_pairs f12_pairs;
typedef struct f12_kernel f12_kernel;
typedef struct f12_quartets f12_quartets;
typedef struct f12_batch f12_batch;

/* ---------------------------------------------------------------- basis ---- */
/* Copies the geometry and shells.  xyz: ncenter*3 doubles; shells: nshell
 * entries; exps/coefs: nprim_total doubles each (exponents > 0). */
int f12_basis_create(int32_t ncenter, const double *xyz, int32_t nshell,
                     const f12_shell *shells, int32_t nprim_total,
                     const double *exps, const double *coefs, f12_basis **out);
void f12_basis_destroy(f12_basis *basis);

/* ---------------------------------------------------------------- pairs ---- */
/* Shell-pair and primitive-pair data on the device (McMurchie-Davidson
 * Gaussian product, Sec. II.B: p = a + b, P = (aA + bB)/p, c_a c_b).
 * ordered = 0: pairs (i, j) with i >= j (for f12_quartets_build);
 * ordered = 1: all pairs (i, j) (for explicit quartet lists).
 * Pair index of (i, j): ordered ? i*nshell + j : i*(i+1)/2 + j.
 * The kernels are enqueued on `stream`; the call returns after they finish. */
int f12_pairs_build(const f12_basis *basis, int32_t ordered, void *stream, f12_pairs **out);
int f12_pairs_count(const f12_pairs *pairs, int64_t *n_shell_pairs, int64_t *n_prim_pairs);
void f12_pairs_destroy(f12_pairs *pairs);

/* -------------------------------------------------------------- kernel ---- */
/* Kernel function k_i for class `cls` with factors f and fp (fp may be NULL,
 * meaning fp = f; only I4 and I6 use fp).  Builds the term table of
 * r*k_i(r) = sum_t c_t r^alpha_t exp(b_t r - g_t r^2) by expanding
 * Eq. (rs12)/(ttdamp) (and d/dr of it for I6), groups the terms into chains of
 * equal (b, g, alpha mod 1), and builds the auxiliary-function tables
 * W_a(x) = R int_0^inf t^a exp(-(t-x)^2) dt (Eq. (sila) with gamma = 1) for the
 * chains' alpha families; uploads everything to the current device. */
int f12_kernel_create(int32_t cls, const f12_factor *f, const f12_factor *fp, f12_kernel **out);
/* Kernel of class `cls` for factors given by their terms instead of the
 * parameters of Eq. (rs12): f(r) = sum_t c_t r^alpha_t exp(b_t r - g_t r^2)
 * (f_terms: host double[4 nf] of (c, alpha, b, g); the same for f' with
 * nfp = 0 and fp_terms = NULL meaning f' = f; f' is used by I4 and I6).  Any
 * such factor goes through the same term tables and kernels as Eq. (rs12):
 * Gaussian geminals sum_i c_i exp(-g_i r^2) (the Gaussian fits of Ten-no's
 * exponential), their products with powers of r, growing exponentials,
 * and decaying ones: Ten-no's exponential exp(-gamma r) is the single term
 * (1, 0, -gamma, 0).  The kernels k_i are formed from f as for Eq. (rs12):
 * I2 f/r, I3 and I5 f, I4 f f', I6 f_r f'_r.  Each term needs g >= 0 and
 * either an integer alpha >= 0 or a non-integer alpha > -1, and a term with
 * b < 0 an integer alpha (else F12_EPARAM; a kernel whose decaying terms
 * share a power family with non-integer powers is rejected the same way);
 * 1 <= nf <= 96 (else F12_EINVAL). */
int f12_kernel_create_terms(int32_t cls, int32_t nf, const double *f_terms, int32_t nfp,
                            const double *fp_terms, f12_kernel **out);
/* Copies up to `cap` terms as (c, alpha, b, g) quadruples into out[4*k..]. */
int f12_kernel_terms(const f12_kernel *k, int32_t *nterms, double *out, int32_t cap);
void f12_kernel_destroy(f12_kernel *k);

/* ------------------------------------------------------------ quartets ---- */
/* All unique quartets of class `cls` over bra and ket pairs built from the
 * same basis with unordered pair sets (ordered = 0): for I1-I4 and I6 the
 * bra pair index >= the ket pair index (8-fold symmetry); for I5 every
 * (bra, ket) combination (no bra-ket symmetry; (ba|cd) = -(ab|cd) and
 * (ab|dc) = (ab|cd) give the remaining blocks).
 * If screen_tol > 0 a quartet is kept when its size estimate reaches
 * screen_tol.  The estimate is Q_ab Q_cd, Q_ab = sqrt(max |(ab|k|ab)|)
 * evaluated with `screen_kernel` (the class's kernel; an I3 kernel for I5),
 * times the growth of the kernel's undamped terms c r^alpha e^{b r} (b > 0,
 * the long-range part of Eq. (rs12)) from r = 1 to the largest distance
 * between the pairs' product centres, times exp(b sqrt((l_a+l_b+1)/(2 p_min))
 * + b^2/(4 p_min)) per pair for the extent of its density (p_min the
 * smallest exponent sum of the pair); for I5 the bra factor also carries the
 * largest bra exponent times (2 l_max + 3) (Eq. (I5_)).  It is an estimate,
 * not a proven bound: Schwarz's inequality does not hold for a kernel that
 * grows with r.  screen_kernel may be NULL when screen_tol <= 0.
 * The public order (offsets, output, f12_quartet_list) groups the quartets
 * by (l_a, l_b, l_c, l_d) and, inside a group, orders them by decreasing
 * number of primitive quartets (enumeration order among equal counts). */
int f12_quartets_build(const f12_pairs *bra, const f12_pairs *ket, int32_t cls,
                       double screen_tol, const f12_kernel *screen_kernel, void *stream,
                       f12_quartets **out, int64_t *n_quartets, int64_t *n_out_doubles);
/* The same list as f12_quartets_build (same arguments, same quartets in the
 * same public order), built on the device: candidate quartets are generated
 * from their enumeration index, screened with the same estimate (per-pair
 * factors from the host, the per-quartet growth term on the device, so a
 * quartet whose estimate lies within rounding of screen_tol may be decided
 * the other way), compacted, and ordered by a stable radix sort on
 * (l_a, l_b, l_c, l_d) and decreasing primitive count; offsets by prefix
 * sums.  The call returns when the list is complete.  Memory: about 64 bytes
 * of device memory per kept quartet during the build. */
int f12_quartets_build_device(const f12_pairs *bra, const f12_pairs *ket, int32_t cls,
                              double screen_tol, const f12_kernel *screen_kernel, void *stream,
                              f12_quartets **out, int64_t *n_quartets, int64_t *n_out_doubles);
/* An explicit list of nq shell quadruples (a, b, c, d) (host int32[4*nq]);
 * bra and ket must be ordered pair sets.  The public order groups the list
 * by (l_a, l_b, l_c, l_d) and by decreasing primitive count inside a group
 * (stable): read it back with f12_quartet_list. */
int f12_quartets_from_list(const f12_pairs *bra, const f12_pairs *ket, int32_t cls,
                           const int32_t *shell_quads, int64_t nq, f12_quartets **out,
                           int64_t *n_out_doubles);
/* offsets: host int64[n_quartets + 1]; block q occupies
 * [offsets[q], offsets[q+1]) doubles, row-major [a][b][c][d]. */
int f12_quartet_offsets(const f12_quartets *q, int64_t *offsets);
/* shell_quads: host int32[4 * n_quartets] in public order. */
int f12_quartet_list(const f12_quartets *q, int32_t *shell_quads);
/* Shape groups of the public order: group g holds quartets
 * [starts[g], starts[g+1]) of angular momenta ls[4g .. 4g+3] = (l_a, l_b,
 * l_c, l_d).  *ngroups receives the number of groups; up to cap groups are
 * written (starts: host int64[cap + 1], ls: host int32[4 cap]; either may be
 * NULL to query the count). */
int f12_quartet_groups(const f12_quartets *q, int32_t *ngroups, int64_t *starts, int32_t *ls, int32_t cap);
/* Number of primitive quartets in the list (work measure). */
int f12_quartets_prim_count(const f12_quartets *q, int64_t *n_prim_quartets);
void f12_quartets_destroy(f12_quartets *q);

/* ---------------------------------------------------------------- eval ---- */
/* Enqueues on `stream` the evaluation of quartets [q_begin, q_end) (public
 * order) with kernel `k` (its class must match the list's).  Block q is
 * written to d_out + offsets[q] - offsets[q_begin]; out_capacity is the
 * number of doubles available at d_out.  Asynchronous: returns after the
 * launches; device-side problems are reported by f12_stream_status.
 * Scratch memory is owned by the quartet list (one eval at a time per list). */
int f12_eval(f12_quartets *q, const f12_kernel *k, int64_t q_begin, int64_t q_end,
             double *d_out, int64_t out_capacity, void *stream);

/* Arithmetic of the E.R.E contraction (Eq. (ii)). */
typedef enum {
  F12_FP64 = 0,       /* every step in binary64                                   */
  F12_SPLIT_FP32 = 1  /* the ket transform (the one-centre z, y, x passes applied   */
                      /* to each primitive quartet's Hermite integrals) in split     */
                      /* FP32: each value a float pair hi + lo (about 48 bits),      */
                      /* products made exact by fma, sums by two-sum; the integrals  */
                      /* R_tuv are scaled by an exact power of two per primitive     */
                      /* quartet to stay in float range.  Radial derivatives, R_tuv, */
                      /* E coefficients, the bra transform and every sum over        */
                      /* primitives stay in binary64.                                */
} f12_precision;

/* Several factor sets in one call: f12_eval of the range with each of
 * kernels[0..nset) (all of the list's class), set s written at
 * d_out + s * n, n = offsets[q_end] - offsets[q_begin] (layout
 * [set][quartet block]); out_capacity must hold nset * n doubles (else
 * F12_EBUFSIZE).  The sets run one after the other on `stream` and share the
 * list's radial-derivative buffer.  F12_EINVAL for nset < 1, a null kernel
 * or a class mismatch; otherwise as f12_eval. */
int f12_eval_sets(f12_quartets *q, const f12_kernel *const *kernels, int32_t nset, int64_t q_begin,
                  int64_t q_end, double *d_out, int64_t out_capacity, void *stream);

/* First derivatives (Sec. II.B: E and F = dE/d(A - B), and the shift of the
 * Hermite Gaussians with P = (aA + bB)/p): blocks of d/dA_dir (ab|k|cd),
 * A the centre of the bra's first shell, dir 0/1/2 = x/y/z, laid out as
 * f12_eval lays out the integrals.  The other centres follow from the
 * symmetries of I1-I4 and I6: d/dB of (ab|cd) is d/dA of (ba|cd) (block
 * transposed in a, b), d/dC and d/dD are d/dA and d/dB of (cd|ab), and
 * d/dA + d/dB + d/dC + d/dD = 0.  I1-I4 and I6 (else F12_EINVAL, as for a bad
 * dir); F12_ELMAX for a range holding shapes with l_a + l_b = 6 and
 * l_c + l_d = 6, whose derivative form does not fit the LDS; otherwise as
 * f12_eval. */
int f12_eval_grad(f12_quartets *q, const f12_kernel *k, int32_t dir, int64_t q_begin, int64_t q_end,
                  double *d_out, int64_t out_capacity, void *stream);

/* f12_eval with the contraction arithmetic chosen by `precision`
 * (F12_FP64 gives exactly f12_eval's result).  F12_EINVAL for an unknown
 * precision; otherwise as f12_eval. */
int f12_eval_precision(f12_quartets *q, const f12_kernel *k, int64_t q_begin, int64_t q_end,
                       double *d_out, int64_t out_capacity, int32_t precision, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation as f12_eval, with the same arguments and output, but the radial-
 * derivative scratch is a fixed device array inside the library instead of
 * the list's own buffer.  It holds the radial derivatives A_0..A_14 of
 * F12_NOALLOC_SCRATCH_PRIMS primitive quartets (15 doubles each, 31.5 MiB),
 * one copy per GPU kept until the process ends; ranges with more primitive quartets run in
 * chunks that fit it.  The call performs no hipMalloc/hipFree; its first call
 * on a device looks the array's address up once.  Errors: as f12_eval, plus
 * F12_EBUFSIZE if one quartet of the list has more primitive quartets than
 * the array holds.  Every call on a GPU shares that GPU's array and it keeps
 * the previous call's contents (every value read is written first by the same
 * call), so calls that overlap in time on one GPU (two streams, two threads)
 * race: serialise them. */
#define F12_NOALLOC_SCRATCH_PRIMS 262144
int f12_eval_noalloc(f12_quartets *q, const f12_kernel *k, int64_t q_begin, int64_t q_end,
                     double *d_out, int64_t out_capacity, void *stream);

/* The two launches of f12_eval, separately, for timing them one by one.
 * [q_begin, q_end) must lie inside one (l_a, l_b, l_c, l_d) group of the
 * public order and hold at most f12_quartets_scratch_prims primitive
 * quartets (else F12_EBUFSIZE).  stage 1 enqueues the radial derivatives
 * A_n (Eq. (bfinal), D^n) into the list's scratch; stage 2 enqueues the
 * Hermite integrals and the E.R.E contraction (Eq. (ri), Eq. (ii)) of the
 * same range with the same kernel, writing d_out as f12_eval does (F12_EINVAL
 * if stage 1 of that range and kernel did not come first).  Together they
 * give the same result as f12_eval on the range. */
int f12_eval_stage(f12_quartets *q, const f12_kernel *k, int64_t q_begin, int64_t q_end,
                   double *d_out, int64_t out_capacity, int32_t stage, void *stream);
/* Primitive quartets the list's scratch holds (bound for f12_eval_stage). */
int f12_quartets_scratch_prims(const f12_quartets *q, int64_t *n_prim_quartets);

/* -------------------------------------------------------------- batches ---- */
/* One class's quartets of every (l_a l_b|l_c l_d) shape, from nlists quartet
 * lists (ranges [q_begin[i], q_end[i]) of list i, written to d_outs[i] as
 * f12_eval writes them: block q at d_outs[i] + offsets[q] - offsets[q_begin[i]]),
 * evaluated by one launch of a captured HIP graph (the E.R.E route of
 * Eq. (ii) with A_n of Eq. (bfinal), as f12_eval computes it; results are
 * identical).  The graph forks into nbranch (1..16) concurrent branches, each
 * with its own radial-derivative scratch (2^21 primitive quartets x 15
 * doubles, 252 MiB) and a chain of chunks; chunks are dealt longest-first to
 * the least-loaded branch.  Contraction launches run persistent grids of G
 * work-groups where that is faster: with tune = 1 the contraction of one
 * sample chunk per shape is timed for G in {one work-group per quartet, 256,
 * 512, 1024, 2048, 4096} (this writes that chunk's output range once, which
 * the graph rewrites); with tune = 0 every shape uses one work-group per
 * quartet.  tune_path (may be NULL): a text file of "L_ab L_cd i5 G" lines
 * read first (shapes found there are not timed) and rewritten with what was
 * learned.  The lists, the kernel and the outputs must outlive the batch.
 * Synchronous (uses `stream` for the tuning and set-up).  Errors: F12_EINVAL
 * (arguments, class mismatch, unwritable tune_path), F12_EBUFSIZE (an output
 * capacity too small), F12_ENOMEM, F12_EDEVICE. */
int f12_batch_create(int32_t nlists, f12_quartets *const *lists, const int64_t *q_begin,
                     const int64_t *q_end, const f12_kernel *k, double *const *d_outs,
                     const int64_t *out_caps, int32_t nbranch, int32_t tune, const char *tune_path,
                     void *stream, f12_batch **out);
/* Enqueues one replay of the batch's graph on `stream` (asynchronous).  A
 * batch's replays share its scratch: do not overlap two replays of one batch. */
int f12_batch_launch(f12_batch *b, void *stream);
/* Quartets, primitive quartets and chunks of the batch. */
int f12_batch_info(const f12_batch *b, int64_t *n_quartets, int64_t *n_prim_quartets, int64_t *n_chunks);
/* The contraction grid chosen for shape (L_ab, L_cd, i5): 0 = one work-group
 * per quartet, G > 0 = persistent; F12_EINVAL if the batch has no such shape. */
int f12_batch_grid(const f12_batch *b, int32_t lab, int32_t lcd, int32_t i5, int64_t *grid);
void f12_batch_destroy(f12_batch *b);

/* ------------------------------------------------------------ diagnostics -- */
/* Radial derivatives A_n = (R^-1 d/dR)^n B_i (Eq. (bfinal), n = 0..L) of the
 * kernel's basic integral, computed by the same device code as f12_eval,
 * for n primitive quartets given by exponent sums p, q and distance R.
 * d_p, d_q, d_R: device double[n]; d_A: device double[(L+1) n] with A_k of
 * point i at d_A[k*n + i].  route: 0 = the switch f12_eval uses (small-T
 * series below T = xi R^2 = 1 for L <= 3, 1.5, 2, 2, 2.5, 3, 3.5, 4, 4.5, 5
 * for L = 4..12 and 6 for L = 13, 14, in binary64 where L <= 5 and T < 2 and
 * in double-double otherwise; the large-T lowering route above);
 * 1 = small-T series in double-double; 2 = large-T route with the
 * exp(-xi (r+R)^2) side kept; 3 = small-T series in binary64.
 * Asynchronous on `stream`. */
int f12_aux_radial(const f12_kernel *k, int64_t n, const double *d_p, const double *d_q,
                   const double *d_R, int32_t L, int32_t route, double *d_A, void *stream);
/* ------------------------------------------------- solid harmonics ---- */
/* Output over real solid harmonics, the basis of the spherical tensor
 * gradient operators Y_lm(nabla) of Eq. (Ylm) (Sec. II.D): each index of a
 * Cartesian block [a][b][c][d] goes over to S_lm, m = -l..l, with
 * S_lm(r) = sqrt(4 pi/(2l+1)) r^l Y_lm(r^) in real form (Racah's
 * normalisation: S_l0 = z^l + ..., S_11 = x, S_1-1 = y, S_22 =
 * sqrt(3)/2 (x^2 - y^2)), so a shell of unnormalised primitives
 * x^i y^j z^k exp(-e r^2) becomes S_lm(r) exp(-e r^2).
 * f12_sph_coefficients: host double[(2l+1) * (l+1)(l+2)/2], row m + l, column
 * the Cartesian component in canonical order (i from l down, then j from
 * l - i down); 0 <= l <= 3 (else F12_EINVAL). */
int f12_sph_coefficients(int32_t l, double *out);
/* Offsets of the spherical blocks in the list's public order: host
 * int64[n_quartets + 1], block q of (2l_a+1)(2l_b+1)(2l_c+1)(2l_d+1) doubles. */
int f12_quartet_offsets_sph(const f12_quartets *q, int64_t *offsets);
/* Enqueues on `stream` the transform of the Cartesian blocks [q_begin, q_end)
 * at d_cart (laid out as f12_eval writes the range: block q at
 * d_cart + offsets[q] - offsets[q_begin]) into spherical blocks at
 * d_sph + sph_offsets[q] - sph_offsets[q_begin], [ma][mb][mc][md] with m
 * ascending.  Device pointers; the two buffers must not overlap.
 * F12_EBUFSIZE if sph_capacity cannot hold the range; F12_EINVAL for bad
 * arguments. */
int f12_cart_to_sph(const f12_quartets *q, int64_t q_begin, int64_t q_end, const double *d_cart,
                    double *d_sph, int64_t sph_capacity, void *stream);

/* Checksum of output chunks for streamed runs (the integrals of a long run
 * are written to a ring buffer chunk by chunk and cannot all be kept; each
 * chunk's quartet range and digest are logged instead, so that two runs can be
 * compared and a run restarted at a chunk).  Adds to *d_digest, modulo 2^64,
 *   D = sum_e mix(bits(x_e) + G (e0 + e + 1)),
 * over the doubles x_e of blocks [q_begin, q_end) at d_out (laid out as
 * f12_eval writes the range), e0 = offsets[q_begin] the global element index
 * of the first one (f12_quartet_offsets), bits() the IEEE-754 bit pattern,
 * G = 0x9E3779B97F4A7C15 and mix the SplitMix64 output function (Steele, Lea
 * and Flood, OOPSLA 2014).  The sum does not depend on the order of
 * reduction, and the digests of the parts of a split range add up to the
 * digest of the whole.  d_digest: device uint64, set by the caller (to 0 for a
 * fresh digest); d_out may be NULL for an empty range.  Enqueued on `stream`;
 * F12_EINVAL for a bad range. */
int f12_digest(const f12_quartets *q, int64_t q_begin, int64_t q_end, const double *d_out, uint64_t *d_digest,
               void *stream);

/* Hermite integrals R_tuv by the Hobson / spherical-tensor route of
 * Sec. II.D, Eq. (Ylm), with the powers of the Laplacian that Eq. (QxQyQz)
 * leaves out restored: R_tuv = sum c_{tuv,lm} S_lm(X) [D^l (nabla^2)^k B](X),
 * N = t+u+v = l + 2k, nabla^2 = 3D + |X|^2 D^2 on radial functions; an
 * alternative to the MD recurrence that the contraction kernels use (a
 * diagnostic path).  Device arrays: d_A[np][L+1] radial derivatives
 * A_n = D^n B, d_X[np][3] the vectors X = Q - P, d_R[np][(L+1)(L+2)(L+3)/6]
 * in the Hermite order (by N, then t descending, then u descending).
 * 0 <= L <= 14 (else F12_EINVAL). */
int f12_hermite_hobson(const double *d_A, const double *d_X, int64_t np, int32_t L, double *d_R,
                       void *stream);

/* Host-side table builder: W_a(x) = R int_0^inf t^a exp(-(t-x)^2) dt
 * (Eq. (sila) with beta = 2x, gamma = 1, times exp(-x^2)) for
 * a = alpha0 + m, m = m_lo..m_hi (alpha0 in [0,1); is_int = 1 for alpha0 = 0
 * requires m_lo >= 0).  out: host double[m_hi - m_lo + 1]. */
int f12_aux_w_column(double alpha0, int32_t is_int, int32_t m_lo, int32_t m_hi, double x,
                     double *out);

/* Synchronises `stream` and reports what the device saw: F12_EDEVICE if a
 * HIP call or launch failed; F12_ENONFINITE if, since the last call on this
 * device, a kernel of the library produced a non-finite value (a radial
 * derivative A_n of Eq. (bfinal) or an output element; for example from
 * contraction coefficients so large that their products overflow).  The
 * device keeps one such fault word, shared by every stream and handle on it;
 * this call reads it and clears it.  F12_OK otherwise. */
int f12_stream_status(void *stream);
const char *f12_strerror(int32_t status);

#ifdef __cplusplus
}
#endif
#endif /* F12INT_H */
