/*
 * oracle.c -- plain, slow FP64 CPU reference for the spherical harmonic
 * transforms (Szydlarski et al., "Parallel Spherical Harmonic Transforms on
 * heterogeneous architectures").  Interface in oracle.h.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product library.
 *
 * What is computed is the plain definition of the discrete transforms
 * (Sec. 2.1 eqs. map2almDef, alm2mapDef), split as the paper does into the
 * Legendre stage (Sec. 2.2 eqs. DeltaDef, almdef) and the azimuthal sums
 * (eqs. Delta2map, almfftdef), with the azimuthal sums done as plain DFTs
 * (no FFT) and every loop in ascending index order.  Arithmetic is plain
 * double precision (built with -ffp-contract=off, so no fused operations);
 * long double is used only to build phase factors and the mu_m seeds.
 *
 * Readings of the paper's formulas used here:
 *  R1 (eq. assLegRec) the recurrence is
 *       P_{l,m} = beta_{l,m} x P_{l-1,m} - (beta_{l,m}/beta_{l-1,m}) P_{l-2,m};
 *     the printed '+' sign does not reproduce P_20 = sqrt(5/4pi)(3x^2-1)/2.
 *  R2 (eq. pmm) the seed is P_mm = (-1)^m mu_m (1-x^2)^{m/2} = (-1)^m mu_m
 *     sin^m(theta): exponent m/2, with the Condon-Shortley phase that the
 *     symmetry Y_{l,-m} = (-1)^m conj(Y_lm) of Sec. 2.1 presumes.
 *  R3 (eq. pm1m) P_{m+1,m} = beta_{m+1,m} x P_mm, beta_{m+1,m} = sqrt(2m+3).
 *  R4 (eqs. Delta2map, almfftdef) the phase is e^{+-i m phi_j} with
 *     phi_j = phi0 + 2 pi j / N_phi; analysis uses the conjugate harmonic
 *     (eq. invers_continous), i.e. e^{-i m phi}, and the per-pixel weight w_r.
 *  R5 (real maps) s = Re Delta_0 + 2 Re sum_{m>=1} Delta_m e^{i m phi}: the
 *     m < 0 half of eq. Delta2map is the complex conjugate of the m > 0 half
 *     (eq. DeltaDef, third case).  Im a_l0 is ignored on input and written as
 *     0 on output.
 *  R6 (rescaling, Sec. 2.1, algorithm not given in the paper) a value is kept
 *     as f * 2^(256 k) with k <= 0; after each step, when |P_l| >= 2^256 both
 *     live values are multiplied by 2^-256 and k incremented.  No downward
 *     rescaling is needed: while k < 0 the recurrence is before its turning
 *     point, where lambda_lm only grows with l.  Power-of-two scaling is
 *     exact, so each term equals the infinite-exponent-range recurrence; it is
 *     converted to a double with ldexp (gradual underflow).
 */
#include "oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define SCALE_BITS 256
static const double BIG = 0x1p256;
static const double SMALL = 0x1p-256;
static const long double PI_L = 3.141592653589793238462643383279502884L;

typedef struct {
    double f; /* mantissa carrier */
    int k;    /* value = f * 2^(SCALE_BITS*k) */
} xdbl;

static int g_threads = 0;

void oracle_set_threads(int n) { g_threads = n; }

int oracle_get_threads(void) {
    return g_threads > 0 ? g_threads : omp_get_max_threads();
}

static int64_t alm_idx(int l, int m, int lmax) {
    return (int64_t)m * (2 * lmax + 1 - m) / 2 + l;
}

static int64_t nalm_of(int lmax, int mmax) {
    return (int64_t)(mmax + 1) * (2 * lmax + 2 - mmax) / 2;
}

/* mu_m of eq. pmm, mu_m = sqrt((2m+1)!/(4 pi)) / (2^m m!), built from
 * mu_0 = 1/sqrt(4 pi) and mu_m / mu_{m-1} = sqrt((2m+1)/(2m)). */
static void mu_table(int mmax, double *mu) {
    long double v = 1.0L / sqrtl(4.0L * PI_L);
    mu[0] = (double)v;
    for (int m = 1; m <= mmax; ++m) {
        v *= sqrtl((long double)(2 * m + 1) / (long double)(2 * m));
        mu[m] = (double)v;
    }
}

/* beta_lm of eq. betaDef and the ratio beta_lm / beta_{l-1,m} of eq.
 * assLegRec for one m, stored at [l - m] for l = m..lmax (entry l = m
 * unused; the ratio is used from l = m+2 on). */
static void beta_column(int lmax, int m, double *beta, double *ratio) {
    for (int l = m; l <= lmax; ++l) {
        double ll = (double)l, mm = (double)m;
        if (l == m) {
            beta[0] = 0.0;
            ratio[0] = 0.0;
            continue;
        }
        beta[l - m] = sqrt((4.0 * ll * ll - 1.0) / (ll * ll - mm * mm));
        ratio[l - m] = (l >= m + 2) ? beta[l - m] / beta[l - m - 1] : 0.0;
    }
}

/* The same for every m <= mmax, at the packed (l, m) index. */
static void beta_tables(int lmax, int mmax, double *beta, double *ratio) {
    for (int m = 0; m <= mmax; ++m) {
        int64_t b = alm_idx(m, m, lmax);
        beta_column(lmax, m, beta + b, ratio + b);
    }
}

/* Seeds P_mm(cos theta) = (-1)^m mu_m sin^m(theta) for m = 0..mmax as
 * extended-range numbers; sin^m by repeated multiplication, renormalised
 * with frexp after every factor. */
static void seed_row(int mmax, double s, const double *mu, xdbl *seed) {
    double pf = 1.0; /* sin^m = pf * 2^pe */
    long pe = 0;
    for (int m = 0; m <= mmax; ++m) {
        if (m > 0) {
            int e;
            pf = frexp(pf * s, &e);
            pe += e;
        }
        double f = ((m & 1) ? -mu[m] : mu[m]) * pf;
        /* value = f * 2^pe with pe <= 1; k = -floor(-pe / 256) keeps the
         * carrier f * 2^(pe - 256k) within [2^-260, 2^4]. */
        long k = (pe >= 0) ? 0 : -((-pe) / SCALE_BITS);
        seed[m].f = (f == 0.0) ? 0.0 : ldexp(f, (int)(pe - (long)SCALE_BITS * k));
        seed[m].k = (f == 0.0) ? 0 : (int)k;
    }
}

static inline double xval(double f, int k) {
    return k == 0 ? f : ldexp(f, SCALE_BITS * k);
}

/* Runs the l-recurrence for one (m, x) from its seed, with beta and ratio
 * the column of that m (index l - m).  Writes, for l = m..lmax, the carrier
 * f and scale index k of lambda_lm(x). */
static void plm_run(int lmax, int m, double x, xdbl seed, const double *beta,
                    const double *ratio, double *f_out, int *k_out) {
    double p2 = seed.f; /* P_{l-2} */
    int k = seed.k;
    f_out[0] = p2;
    k_out[0] = k;
    if (lmax == m) return;
    double p1 = beta[1] * x * p2; /* eq. pm1m */
    f_out[1] = p1;
    k_out[1] = k;
    for (int l = m + 2; l <= lmax; ++l) {
        double p = beta[l - m] * x * p1 - ratio[l - m] * p2; /* eq. assLegRec (R1) */
        p2 = p1;
        p1 = p;
        if (fabs(p1) >= BIG) {
            p1 *= SMALL;
            p2 *= SMALL;
            k += 1;
        }
        f_out[l - m] = p1;
        k_out[l - m] = k;
    }
}

int oracle_plm_ext(int lmax, int m, double theta, double *mant, int32_t *exp2) {
    if (lmax < 0 || m < 0 || m > lmax || !mant || !exp2) return -1;
    if (!(theta >= 0.0 && theta <= M_PI)) return -1;
    double *beta = malloc(sizeof(double) * (lmax - m + 1));
    double *ratio = malloc(sizeof(double) * (lmax - m + 1));
    double *mu = malloc(sizeof(double) * (m + 1));
    xdbl *seed = malloc(sizeof(xdbl) * (m + 1));
    double *f = malloc(sizeof(double) * (lmax - m + 1));
    int *k = malloc(sizeof(int) * (lmax - m + 1));
    beta_column(lmax, m, beta, ratio);
    mu_table(m, mu);
    seed_row(m, sin(theta), mu, seed);
    plm_run(lmax, m, cos(theta), seed[m], beta, ratio, f, k);
    for (int l = m; l <= lmax; ++l) {
        int e = 0;
        double fr = frexp(f[l - m], &e);
        mant[l - m] = fr;
        exp2[l - m] = (fr == 0.0) ? 0 : e + SCALE_BITS * k[l - m];
    }
    free(beta); free(ratio); free(mu); free(seed); free(f); free(k);
    return 0;
}

int oracle_plm(int lmax, int m, double theta, double *out) {
    if (lmax < 0 || m < 0 || m > lmax || !out) return -1;
    double *mant = malloc(sizeof(double) * (lmax - m + 1));
    int32_t *e = malloc(sizeof(int32_t) * (lmax - m + 1));
    int rc = oracle_plm_ext(lmax, m, theta, mant, e);
    if (rc == 0)
        for (int l = m; l <= lmax; ++l) out[l - m] = ldexp(mant[l - m], e[l - m]);
    free(mant); free(e);
    return rc;
}

static int check_rings(int nrings, const double *theta) {
    if (nrings < 1 || !theta) return -1;
    for (int r = 0; r < nrings; ++r)
        if (!(theta[r] >= 0.0 && theta[r] <= M_PI)) return -1;
    return 0;
}

int oracle_delta_syn(int lmax, int mmax, int nrings, const double *theta,
                     const double *alm, int nsel, const int32_t *ring_sel,
                     double *out) {
    if (lmax < 0 || mmax < 0 || mmax > lmax || !alm || !out) return -1;
    if (check_rings(nrings, theta)) return -1;
    if (!ring_sel) nsel = nrings;
    if (nsel < 0) return -1;
    for (int i = 0; ring_sel && i < nsel; ++i)
        if (ring_sel[i] < 0 || ring_sel[i] >= nrings) return -1;
    int64_t na = nalm_of(lmax, mmax);
    double *beta = malloc(sizeof(double) * na), *ratio = malloc(sizeof(double) * na);
    double *mu = malloc(sizeof(double) * (mmax + 1));
    beta_tables(lmax, mmax, beta, ratio);
    mu_table(mmax, mu);
#pragma omp parallel num_threads(oracle_get_threads())
    {
        xdbl *seed = malloc(sizeof(xdbl) * (mmax + 1));
        double *f = malloc(sizeof(double) * (lmax + 1));
        int *k = malloc(sizeof(int) * (lmax + 1));
#pragma omp for schedule(dynamic, 1)
        for (int i = 0; i < nsel; ++i) {
            int r = ring_sel ? ring_sel[i] : i;
            double x = cos(theta[r]);
            seed_row(mmax, sin(theta[r]), mu, seed);
            for (int m = 0; m <= mmax; ++m) {
                int64_t b = alm_idx(m, m, lmax);
                plm_run(lmax, m, x, seed[m], beta + b, ratio + b, f, k);
                const double *a = alm + 2 * alm_idx(0, m, lmax);
                double dre = 0.0, dim = 0.0;
                for (int l = m; l <= lmax; ++l) {
                    double v = xval(f[l - m], k[l - m]);
                    dre += a[2 * l] * v;
                    if (m > 0) dim += a[2 * l + 1] * v; /* R5: Im a_l0 ignored */
                }
                out[2 * ((int64_t)i * (mmax + 1) + m)] = dre;
                out[2 * ((int64_t)i * (mmax + 1) + m) + 1] = dim;
            }
        }
        free(seed); free(f); free(k);
    }
    free(beta); free(ratio); free(mu);
    return 0;
}

/* e^{2 pi i t / n} for t = 0..n-1, built in long double. */
static void unit_roots(int n, double *re, double *im) {
    for (int t = 0; t < n; ++t) {
        long double a = 2.0L * PI_L * (long double)t / (long double)n;
        re[t] = (double)cosl(a);
        im[t] = (double)sinl(a);
    }
}

static int check_layout(int nrings, const int32_t *nphi, const double *phi0,
                        const int64_t *ofs) {
    if (nrings < 1 || !nphi || !phi0 || !ofs) return -1;
    for (int r = 0; r < nrings; ++r)
        if (nphi[r] < 1 || ofs[r] < 0 || !isfinite(phi0[r])) return -1;
    return 0;
}

int oracle_delta2map(int mmax, int nrings, const int32_t *nphi,
                     const double *phi0, const int64_t *ofs, const double *delta,
                     int nsel, const int32_t *ring_sel, double *map) {
    if (mmax < 0 || !delta || !map) return -1;
    if (check_layout(nrings, nphi, phi0, ofs)) return -1;
    if (!ring_sel) nsel = nrings;
    for (int i = 0; ring_sel && i < nsel; ++i)
        if (ring_sel[i] < 0 || ring_sel[i] >= nrings) return -1;
#pragma omp parallel num_threads(oracle_get_threads())
    {
        double *cre = malloc(sizeof(double) * (mmax + 1));
        double *cim = malloc(sizeof(double) * (mmax + 1));
        double *wre = NULL, *wim = NULL;
        int wn = 0;
#pragma omp for schedule(dynamic, 1)
        for (int i = 0; i < nsel; ++i) {
            int r = ring_sel ? ring_sel[i] : i;
            int n = nphi[r];
            if (n != wn) {
                free(wre); free(wim);
                wre = malloc(sizeof(double) * n);
                wim = malloc(sizeof(double) * n);
                unit_roots(n, wre, wim);
                wn = n;
            }
            const double *d = delta + 2 * (int64_t)i * (mmax + 1);
            /* c_m = Delta_m e^{i m phi0}  (R4) */
            for (int m = 0; m <= mmax; ++m) {
                long double a = (long double)m * (long double)phi0[r];
                double pr = (double)cosl(a), pi = (double)sinl(a);
                cre[m] = d[2 * m] * pr - d[2 * m + 1] * pi;
                cim[m] = d[2 * m] * pi + d[2 * m + 1] * pr;
            }
            for (int j = 0; j < n; ++j) {
                /* s_j = Re Delta_0 + 2 sum_m Re(c_m e^{2 pi i m j / n})  (R5) */
                double acc = 0.0;
                int64_t t = 0; /* (m j) mod n */
                for (int m = 1; m <= mmax; ++m) {
                    t += j;
                    if (t >= n) t %= n;
                    acc += cre[m] * wre[t] - cim[m] * wim[t];
                }
                map[ofs[r] + j] = d[0] + 2.0 * acc;
            }
        }
        free(cre); free(cim); free(wre); free(wim);
    }
    return 0;
}

int oracle_alm2map(int lmax, int mmax, int nrings, const double *theta,
                   const int32_t *nphi, const double *phi0, const int64_t *ofs,
                   const double *alm, int nsel, const int32_t *ring_sel,
                   double *map) {
    if (check_layout(nrings, nphi, phi0, ofs)) return -1;
    int cnt = ring_sel ? nsel : nrings;
    if (cnt < 0) return -1;
    double *delta = malloc(sizeof(double) * 2 * (size_t)(cnt ? cnt : 1) * (mmax + 1));
    int rc = oracle_delta_syn(lmax, mmax, nrings, theta, alm, nsel, ring_sel, delta);
    if (rc == 0)
        rc = oracle_delta2map(mmax, nrings, nphi, phi0, ofs, delta, nsel, ring_sel, map);
    free(delta);
    return rc;
}

int oracle_map2delta(int mmax, int nrings, const int32_t *nphi,
                     const double *phi0, const double *weight,
                     const int64_t *ofs, const double *map, int nm,
                     const int32_t *m_sel, double *out) {
    if (mmax < 0 || !weight || !map || !out) return -1;
    if (check_layout(nrings, nphi, phi0, ofs)) return -1;
    if (!m_sel) nm = mmax + 1;
    if (nm < 0) return -1;
    for (int i = 0; m_sel && i < nm; ++i)
        if (m_sel[i] < 0 || m_sel[i] > mmax) return -1;
#pragma omp parallel num_threads(oracle_get_threads())
    {
        double *wre = NULL, *wim = NULL;
        int wn = 0;
#pragma omp for schedule(dynamic, 1)
        for (int r = 0; r < nrings; ++r) {
            int n = nphi[r];
            if (n != wn) {
                free(wre); free(wim);
                wre = malloc(sizeof(double) * n);
                wim = malloc(sizeof(double) * n);
                unit_roots(n, wre, wim);
                wn = n;
            }
            const double *s = map + ofs[r];
            for (int i = 0; i < nm; ++i) {
                int m = m_sel ? m_sel[i] : i;
                /* sum_j s_j e^{-2 pi i m j / n} */
                double sre = 0.0, sim = 0.0;
                int64_t t = 0, mm = m % n;
                for (int j = 0; j < n; ++j) {
                    sre += s[j] * wre[t];
                    sim -= s[j] * wim[t];
                    t += mm;
                    if (t >= n) t -= n;
                }
                /* times w_r e^{-i m phi0}  (R4) */
                long double a = (long double)m * (long double)phi0[r];
                double pr = (double)cosl(a), pi = -(double)sinl(a);
                out[2 * ((int64_t)r * nm + i)] = weight[r] * (sre * pr - sim * pi);
                out[2 * ((int64_t)r * nm + i) + 1] = weight[r] * (sre * pi + sim * pr);
            }
        }
        free(wre); free(wim);
    }
    return 0;
}

int oracle_delta2alm(int lmax, int mmax, int nrings, const double *theta,
                     const double *delta, int nm, const int32_t *m_sel,
                     double *alm) {
    if (lmax < 0 || mmax < 0 || mmax > lmax || !delta || !alm) return -1;
    if (check_rings(nrings, theta)) return -1;
    if (!m_sel) nm = mmax + 1;
    if (nm < 0) return -1;
    int mtop = 0;
    for (int i = 0; i < nm; ++i) {
        int m = m_sel ? m_sel[i] : i;
        if (m < 0 || m > mmax) return -1;
        if (m > mtop) mtop = m;
    }
    int64_t na = nalm_of(lmax, mmax);
    double *beta = malloc(sizeof(double) * na), *ratio = malloc(sizeof(double) * na);
    double *mu = malloc(sizeof(double) * (mmax + 1));
    beta_tables(lmax, mmax, beta, ratio);
    mu_table(mmax, mu);
    /* seeds for every ring and m <= mtop */
    xdbl *seeds = malloc(sizeof(xdbl) * (size_t)nrings * (mtop + 1));
    double *xs = malloc(sizeof(double) * nrings);
#pragma omp parallel for num_threads(oracle_get_threads()) schedule(static)
    for (int r = 0; r < nrings; ++r) {
        xs[r] = cos(theta[r]);
        seed_row(mtop, sin(theta[r]), mu, seeds + (size_t)r * (mtop + 1));
    }
#pragma omp parallel num_threads(oracle_get_threads())
    {
        double *f = malloc(sizeof(double) * (lmax + 1));
        int *k = malloc(sizeof(int) * (lmax + 1));
        double *acc = malloc(sizeof(double) * 2 * (lmax + 1));
#pragma omp for schedule(dynamic, 1)
        for (int i = 0; i < nm; ++i) {
            int m = m_sel ? m_sel[i] : i;
            int nl = lmax - m + 1;
            memset(acc, 0, sizeof(double) * 2 * nl);
            for (int r = 0; r < nrings; ++r) { /* ascending r */
                plm_run(lmax, m, xs[r], seeds[(size_t)r * (mtop + 1) + m], beta + alm_idx(m, m, lmax),
                        ratio + alm_idx(m, m, lmax), f, k);
                double dre = delta[2 * ((int64_t)r * nm + i)];
                double dim = delta[2 * ((int64_t)r * nm + i) + 1];
                for (int l = m; l <= lmax; ++l) {
                    double v = xval(f[l - m], k[l - m]);
                    acc[2 * (l - m)] += dre * v;
                    acc[2 * (l - m) + 1] += dim * v;
                }
            }
            double *a = alm + 2 * alm_idx(0, m, lmax);
            for (int l = m; l <= lmax; ++l) {
                a[2 * l] = acc[2 * (l - m)];
                a[2 * l + 1] = (m == 0) ? 0.0 : acc[2 * (l - m) + 1]; /* R5 */
            }
        }
        free(f); free(k); free(acc);
    }
    free(seeds); free(xs); free(beta); free(ratio); free(mu);
    return 0;
}

int oracle_map2alm(int lmax, int mmax, int nrings, const double *theta,
                   const int32_t *nphi, const double *phi0,
                   const double *weight, const int64_t *ofs, const double *map,
                   int nm, const int32_t *m_sel, double *alm) {
    if (lmax < 0 || mmax < 0 || mmax > lmax) return -1;
    if (check_layout(nrings, nphi, phi0, ofs)) return -1;
    int cnt = m_sel ? nm : mmax + 1;
    if (cnt < 0) return -1;
    double *delta = malloc(sizeof(double) * 2 * (size_t)nrings * (cnt ? cnt : 1));
    int rc = oracle_map2delta(mmax, nrings, nphi, phi0, weight, ofs, map, nm, m_sel, delta);
    if (rc == 0)
        rc = oracle_delta2alm(lmax, mmax, nrings, theta, delta, nm, m_sel, alm);
    free(delta);
    return rc;
}
