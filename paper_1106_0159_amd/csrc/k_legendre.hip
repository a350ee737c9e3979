// Legendre-stage kernels for gfx950 (FP64 VALU).
//
// Synthesis computes Delta^A_m(r) = sum_l a_lm lambda_lm(cos theta_r)
// (Sec. 2.2 eq. DeltaDef); analysis computes a_lm = sum_r Delta^S_m(r)
// lambda_lm(cos theta_r) (eq. almdef).  lambda_lm comes from the l-recurrence
// (eqs. assLegRec, betaDef) seeded by lambda_mm = (-1)^m mu_m sin^m(theta)
// (eq. pmm, with the exponent m/2 and the Condon-Shortley phase) and
// lambda_{m+1,m} = sqrt(2m+3) x lambda_mm (eq. pm1m).
//
// The recurrence runs in a rescaled variable q_l = lambda_l / c_l for which
// the coefficient of q_{l-2} is -1 (q_l = alpha_l x q_{l-1} - q_{l-2}); the
// plan tabulates alpha and c.  Synthesis folds c into a_lm once per call
// (k_prescale); analysis multiplies each finished a_lm by c.
//
// One recurrence serves a ring and its mirror image (x -> -x) because
// lambda_lm(-x) = (-1)^(l+m) lambda_lm(x): even and odd (l+m) partial sums
// are kept apart and combined as E+O (north) and E-O (south).
//
// Work mapping (the paper's GPU design assigns one ring per thread and the
// rings loop outermost; here a workgroup owns one m for a tile of ring
// pairs, so the m-dependent loop length is uniform across the workgroup and
// a_lm, alpha are wave-uniform scalar loads):
//   synthesis  grid.x = (m, 256-slot tile) with m ascending (longest first),
//              grid.y = map; one slot per lane, no reduction needed.
//   analysis   grid.x = m (ascending), grid.y = map; a workgroup owns every
//              slot of its m (T slots per lane), sums over its lanes in LDS
//              in a fixed order: no atomics, bitwise deterministic.
//
// Underflow near the poles (Sec. 2.1, rescaling; the paper leaves the
// algorithm to its references): a value is held as q * 2^(600 sc), sc <= 0.
// While sc < 0 the value is below 2^-660 and its term is dropped; when the
// carrier exceeds 2^-60 it is scaled by 2^-600 and sc incremented (checked
// every second step).  Waves run three loops: (A0) every lane negligible:
// recurrence only; (A) some lane still rescaling: terms weighted by 0/1;
// (B) all lanes in range: no checks.
#include "sht_internal.h"

namespace sht {
namespace {

constexpr double kDown = 0x1p-600;       // 2^-kScaleBits
constexpr double kThresh = 0x1p-60;
static_assert(kScaleBits == 600, "kDown must equal 2^-kScaleBits");

// lambda_mm = (-1)^m mu_m s^m as carrier * 2^(600 sc).  s^m by binary
// powering with frexp renormalisation (about 2 log2(m) roundings).
__device__ __forceinline__ double seed_carrier(int m, double s, double mu_m, int &sc) {
    int eb;
    double b = frexp(s, &eb);
    double r = 1.0;
    int E = 0;
    for (int k = m; k; k >>= 1) {
        if (k & 1) {
            int e;
            r = frexp(r * b, &e);
            E += e + eb;
        }
        if (k > 1) {
            int e2;
            b = frexp(b * b, &e2);
            eb = 2 * eb + e2;
        }
    }
    const double v = ((m & 1) ? -mu_m : mu_m) * r;
    if (v == 0.0) {
        sc = 0;
        return 0.0;
    }
    // keep the carrier exponent in (-660, -60] when sc < 0
    const int ns = (E >= -60) ? 0 : (-E - 60) / kScaleBits;
    sc = -ns;
    return ldexp(v, E + kScaleBits * ns);
}

__global__ __launch_bounds__(kBlock) void k_prescale(int64_t nalm, int lmax, int nmaps,
                                                     const double2 *__restrict__ alm,
                                                     const double *__restrict__ cfac,
                                                     double2 *__restrict__ out) {
    const int64_t total = nalm * nmaps;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * kBlock) {
        const int64_t k = i % nalm;
        const double c = cfac[k];
        const double2 a = alm[i];
        // entries k <= lmax are m = 0: Im a_l0 is ignored
        out[i] = make_double2(a.x * c, k <= lmax ? 0.0 : a.y * c);
    }
}

__global__ __launch_bounds__(kBlock) void k_leg_syn(int lmax, int mmax, int nslots, int tiles,
                                                    int nrings, int64_t nalm,
                                                    const double2 *__restrict__ ap,
                                                    const double *__restrict__ alpha,
                                                    const double *__restrict__ mu,
                                                    const double *__restrict__ sx,
                                                    const double *__restrict__ ss,
                                                    const int32_t *__restrict__ rn,
                                                    const int32_t *__restrict__ rsouth,
                                                    double2 *__restrict__ delta) {
    const int m = blockIdx.x / tiles;
    const int slot = (blockIdx.x - m * tiles) * kBlock + threadIdx.x;
    const int map = blockIdx.y;
    const bool active = slot < nslots;
    const double x = active ? sx[slot] : 0.0;
    const double s = active ? ss[slot] : 1.0;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;  // (l, m) lives at base + l
    const double2 *__restrict__ a = ap + (int64_t)map * nalm + base;
    const double *__restrict__ al = alpha + base;

    int sc;
    const double seed = seed_carrier(m, s, mu[m], sc);
    // state (q_{l-2}, q_{l-1}) before step l; (-seed, 0) makes step l = m yield the seed
    double q2 = -seed, q1 = 0.0;
    double cf = (sc == 0) ? 1.0 : 0.0;
    double er = 0.0, ei = 0.0, orr = 0.0, oi = 0.0;

#define SHT_REC(L)                               \
    {                                            \
        const double t_ = al[(L)] * x;           \
        const double q_ = fma(t_, q1, -q2);      \
        q2 = q1;                                 \
        q1 = q_;                                 \
    }
#define SHT_RESCALE()                            \
    if (sc < 0 && fabs(q1) > kThresh) {          \
        q1 *= kDown;                             \
        q2 *= kDown;                             \
        ++sc;                                    \
        cf = (sc == 0) ? 1.0 : 0.0;              \
    }

    int l = m;
    // (A0) all lanes below range: recurrence only
    while (l + 1 <= lmax && __all(sc < 0)) {
        SHT_REC(l);
        SHT_REC(l + 1);
        SHT_RESCALE();
        l += 2;
    }
    // (A) mixed: weight terms by cf
    while (l + 1 <= lmax && __any(sc < 0)) {
        SHT_REC(l);
        {
            const double p = cf * q1;
            const double2 c = a[l];
            er = fma(c.x, p, er);
            ei = fma(c.y, p, ei);
        }
        SHT_REC(l + 1);
        {
            const double p = cf * q1;
            const double2 c = a[l + 1];
            orr = fma(c.x, p, orr);
            oi = fma(c.y, p, oi);
        }
        SHT_RESCALE();
        l += 2;
    }
    // (B) all lanes in range
    for (; l + 1 <= lmax; l += 2) {
        SHT_REC(l);
        const double2 c0 = a[l];
        er = fma(c0.x, q1, er);
        ei = fma(c0.y, q1, ei);
        SHT_REC(l + 1);
        const double2 c1 = a[l + 1];
        orr = fma(c1.x, q1, orr);
        oi = fma(c1.y, q1, oi);
    }
    if (l == lmax) {  // one trailing step with even (l - m)
        SHT_REC(l);
        const double p = cf * q1;
        const double2 c = a[l];
        er = fma(c.x, p, er);
        ei = fma(c.y, p, ei);
    }
#undef SHT_REC
#undef SHT_RESCALE

    if (active) {
        double2 *d = delta + (int64_t)map * nrings * (mmax + 1);
        d[(int64_t)rn[slot] * (mmax + 1) + m] = make_double2(er + orr, ei + oi);
        const int r2 = rsouth[slot];
        if (r2 >= 0) d[(int64_t)r2 * (mmax + 1) + m] = make_double2(er - orr, ei - oi);
    }
}

constexpr int kChunk = 16;  // l values per reduction round in analysis

template <int T>
__global__ __launch_bounds__(kBlock) void k_leg_ana(int lmax, int mmax, int nslots, int nrings,
                                                    int64_t nalm, const double2 *__restrict__ delta,
                                                    const double *__restrict__ alpha,
                                                    const double *__restrict__ cfac,
                                                    const double *__restrict__ mu,
                                                    const double *__restrict__ sx,
                                                    const double *__restrict__ ss,
                                                    const int32_t *__restrict__ rn,
                                                    const int32_t *__restrict__ rsouth,
                                                    double2 *__restrict__ alm) {
    __shared__ double red_re[kChunk][kBlock];
    __shared__ double red_im[kChunk][kBlock];
    const int m = blockIdx.x;
    const int map = blockIdx.y;
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
    const double *__restrict__ al = alpha + base;
    const double2 *__restrict__ d = delta + (int64_t)map * nrings * (mmax + 1);

    double x[T], q1[T], q2[T], cf[T], pr[T], pi[T], mr[T], mi[T];
    int sc[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int slot = tid * T + t;
        const bool act = slot < nslots;
        x[t] = act ? sx[slot] : 0.0;
        const double s = act ? ss[slot] : 1.0;
        double2 dn = make_double2(0.0, 0.0), ds = make_double2(0.0, 0.0);
        if (act) {
            dn = d[(int64_t)rn[slot] * (mmax + 1) + m];
            const int r2 = rsouth[slot];
            if (r2 >= 0) ds = d[(int64_t)r2 * (mmax + 1) + m];
        }
        // even (l+m): north + south; odd: north - south
        pr[t] = dn.x + ds.x;
        pi[t] = dn.y + ds.y;
        mr[t] = dn.x - ds.x;
        mi[t] = dn.y - ds.y;
        const double seed = seed_carrier(m, s, mu[m], sc[t]);
        q2[t] = -seed;
        q1[t] = 0.0;
        cf[t] = (sc[t] == 0) ? 1.0 : 0.0;
    }

    for (int l0 = m; l0 <= lmax; l0 += kChunk) {
        double accr[kChunk], acci[kChunk];
        bool slow = false;
#pragma unroll
        for (int t = 0; t < T; ++t) slow |= (sc[t] < 0);
        slow = __any(slow);
        const bool full = (l0 + kChunk - 1 <= lmax);
#pragma unroll
        for (int i = 0; i < kChunk; ++i) {
            accr[i] = 0.0;
            acci[i] = 0.0;
            const int l = l0 + i;
            if (full || l <= lmax) {
                const double a_l = al[l];
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    const double q = fma(a_l * x[t], q1[t], -q2[t]);
                    q2[t] = q1[t];
                    q1[t] = q;
                    const double p = slow ? cf[t] * q : q;
                    const double dr = (i & 1) ? mr[t] : pr[t];
                    const double di = (i & 1) ? mi[t] : pi[t];
                    accr[i] = fma(p, dr, accr[i]);
                    acci[i] = fma(p, di, acci[i]);
                }
                if (slow && (i & 1)) {
#pragma unroll
                    for (int t = 0; t < T; ++t) {
                        if (sc[t] < 0 && fabs(q1[t]) > kThresh) {
                            q1[t] *= kDown;
                            q2[t] *= kDown;
                            ++sc[t];
                            cf[t] = (sc[t] == 0) ? 1.0 : 0.0;
                        }
                    }
                }
            }
        }
        // a slot left mid-rescale at an odd chunk end is checked next chunk
#pragma unroll
        for (int i = 0; i < kChunk; ++i) {
            red_re[i][tid] = accr[i];
            red_im[i][tid] = acci[i];
        }
        __syncthreads();
        // thread (li = tid/16, g = tid%16) sums lanes g, g+16, ..., g+240 of row li,
        // then the 16 lanes of the group combine with xor shuffles
        {
            const int li = tid >> 4, g = tid & 15;
            double sr = 0.0, si = 0.0;
#pragma unroll
            for (int j = 0; j < kBlock / 16; ++j) {
                sr += red_re[li][j * 16 + g];
                si += red_im[li][j * 16 + g];
            }
#pragma unroll
            for (int off = 8; off >= 1; off >>= 1) {
                sr += __shfl_xor(sr, off, 16);
                si += __shfl_xor(si, off, 16);
            }
            const int l = l0 + li;
            if (g == 0 && l <= lmax) {
                const double c = cfac[base + l];
                alm[(int64_t)map * nalm + base + l] = make_double2(sr * c, m == 0 ? 0.0 : si * c);
            }
        }
        __syncthreads();
    }
}

}  // namespace

static int grid_ok(int64_t n) { return n > 0 && n < (int64_t)INT32_MAX; }

int launch_prescale(const CoefTables &c, const void *alm, void *aprime, int nmaps, hipStream_t st) {
    const int64_t total = c.nalm * nmaps;
    const int64_t blocks = std::min<int64_t>((total + kBlock - 1) / kBlock, 1 << 16);
    hipLaunchKernelGGL(k_prescale, dim3((unsigned)blocks), dim3(kBlock), 0, st, c.nalm, c.lmax, nmaps,
                       static_cast<const double2 *>(alm), c.cfac, static_cast<double2 *>(aprime));
    SHT_HIP(hipGetLastError());
    return SHT_OK;
}

int launch_leg_syn(const CoefTables &c, const GeomPlan &p, const void *aprime, void *delta, int nmaps,
                   hipStream_t st) {
    const int tiles = (p.nslots + kBlock - 1) / kBlock;
    const int64_t gx = (int64_t)tiles * (c.mmax + 1);
    if (!grid_ok(gx) || nmaps > 65535) return SHT_EUNSUPPORTED;
    hipLaunchKernelGGL(k_leg_syn, dim3((unsigned)gx, (unsigned)nmaps), dim3(kBlock), 0, st, c.lmax,
                       c.mmax, p.nslots, tiles, p.nrings, c.nalm, static_cast<const double2 *>(aprime),
                       c.alpha, c.mu, p.slot_x, p.slot_s, p.slot_north, p.slot_south,
                       static_cast<double2 *>(delta));
    SHT_HIP(hipGetLastError());
    return SHT_OK;
}

template <int T>
static void launch_ana_t(const CoefTables &c, const GeomPlan &p, const void *delta, void *alm, int nmaps,
                         hipStream_t st) {
    hipLaunchKernelGGL(k_leg_ana<T>, dim3((unsigned)(c.mmax + 1), (unsigned)nmaps), dim3(kBlock), 0, st,
                       c.lmax, c.mmax, p.nslots, p.nrings, c.nalm, static_cast<const double2 *>(delta),
                       c.alpha, c.cfac, c.mu, p.slot_x, p.slot_s, p.slot_north, p.slot_south,
                       static_cast<double2 *>(alm));
}

int launch_leg_ana(const CoefTables &c, const GeomPlan &p, const void *delta, void *alm, int nmaps,
                   hipStream_t st) {
    if (nmaps > 65535) return SHT_EUNSUPPORTED;
    const int per = (p.nslots + kBlock - 1) / kBlock;
    if (per <= 1) launch_ana_t<1>(c, p, delta, alm, nmaps, st);
    else if (per <= 2) launch_ana_t<2>(c, p, delta, alm, nmaps, st);
    else if (per <= 4) launch_ana_t<4>(c, p, delta, alm, nmaps, st);
    else if (per <= 8) launch_ana_t<8>(c, p, delta, alm, nmaps, st);
    else if (per <= kAnaMaxSlotsPerThread) launch_ana_t<16>(c, p, delta, alm, nmaps, st);
    else return SHT_EUNSUPPORTED;
    SHT_HIP(hipGetLastError());
    return SHT_OK;
}

}  // namespace sht
