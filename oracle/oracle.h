/*
 * oracle.h -- plain, slow, FP64 CPU reference for the spherical harmonic
 * transforms of Szydlarski et al., "Parallel Spherical Harmonic Transforms on
 * heterogeneous architectures".
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * Conventions (shared with the product only as an interface):
 *   a_lm  complex128 interleaved (re, im), m-major packed over m >= 0:
 *         index(l, m) = m*(2*lmax+1-m)/2 + l,  m <= l <= lmax.
 *   map   float64, ring r occupies map[ofs[r] .. ofs[r]+nphi[r]-1], pixel j at
 *         longitude phi0[r] + 2*pi*j/nphi[r].
 *   Delta complex128 [count][mmax+1] for the requested rings (synthesis) or
 *         [nrings][count_m] for the requested m (analysis).
 *
 * All functions return 0 on success and -1 on invalid arguments.
 */
#ifndef SHT_ORACLE_H
#define SHT_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* Thread count used by the OpenMP loops (<= 0: the OpenMP default). */
void oracle_set_threads(int n);
int oracle_get_threads(void);

/* Normalised associated Legendre functions lambda_lm(cos theta), l = m..lmax,
 * as mant[l-m] * 2^exp2[l-m] (mant in [0.5,1) or 0), never under/overflowing.
 * Sec. 2.1 eqs. assLegRec, betaDef, pmm, pm1m (with the readings in the
 * source file's header). */
int oracle_plm_ext(int lmax, int m, double theta, double *mant, int32_t *exp2);

/* Same values rounded into IEEE doubles (gradual underflow). */
int oracle_plm(int lmax, int m, double theta, double *out);

/* Delta^A_m(r) = sum_{l=m}^{lmax} a_lm lambda_lm(cos theta_r), m = 0..mmax
 * (Sec. 2.2 eq. DeltaDef), for the listed rings (ring_sel == NULL: all rings,
 * nsel = nrings).  out: complex128 [nsel][mmax+1]. */
int oracle_delta_syn(int lmax, int mmax, int nrings, const double *theta,
                     const double *alm, int nsel, const int32_t *ring_sel,
                     double *out);

/* Ring synthesis (Sec. 2.2 eq. Delta2map, read with phi_j for phi_0):
 * s_{r,j} = Re Delta_0(r) + 2 Re sum_{m=1}^{mmax} Delta_m(r) e^{i m phi_j},
 * as a plain DFT.  delta: complex128 [nsel][mmax+1] for the listed rings;
 * writes only those rings' pixels of map. */
int oracle_delta2map(int mmax, int nrings, const int32_t *nphi,
                     const double *phi0, const int64_t *ofs, const double *delta,
                     int nsel, const int32_t *ring_sel, double *map);

/* alm2map (Sec. 3, Alg. 2): delta_syn followed by delta2map on the listed rings. */
int oracle_alm2map(int lmax, int mmax, int nrings, const double *theta,
                   const int32_t *nphi, const double *phi0, const int64_t *ofs,
                   const double *alm, int nsel, const int32_t *ring_sel,
                   double *map);

/* Ring analysis (Sec. 2.2 eq. almfftdef, with phi_j and e^{-i m phi}):
 * Delta^S_m(r) = w_r sum_j s_{r,j} e^{-i m phi_j} for every ring and the
 * listed m (m_sel == NULL: all m = 0..mmax, nm = mmax+1).
 * out: complex128 [nrings][nm]. */
int oracle_map2delta(int mmax, int nrings, const int32_t *nphi,
                     const double *phi0, const double *weight,
                     const int64_t *ofs, const double *map, int nm,
                     const int32_t *m_sel, double *out);

/* a_lm = sum_r Delta^S_m(r) lambda_lm(cos theta_r) (Sec. 2.2 eq. almdef) for
 * the listed m; delta: complex128 [nrings][nm] as produced above.  Writes
 * only the a_lm entries of the listed m; Im a_l0 is written as 0. */
int oracle_delta2alm(int lmax, int mmax, int nrings, const double *theta,
                     const double *delta, int nm, const int32_t *m_sel,
                     double *alm);

/* map2alm (Sec. 3, Alg. 1): map2delta followed by delta2alm for the listed m. */
int oracle_map2alm(int lmax, int mmax, int nrings, const double *theta,
                   const int32_t *nphi, const double *phi0,
                   const double *weight, const int64_t *ofs, const double *map,
                   int nm, const int32_t *m_sel, double *alm);

#ifdef __cplusplus
}
#endif
#endif
