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
//   synthesis  grid.x = (m, 512-slot tile) with m ascending (longest first),
//              grid.y = map; two slots per lane, no reduction needed.
//   analysis   grid.x = (m ascending, slot group), grid.y = map; a workgroup
//              owns up to 1024 slots of its m (T slots per lane); each wave sums
//              its lanes through its own LDS rows, the four waves are added in
//              wave order every 64 l, and groups are summed in order by a
//              second small kernel: no atomics, bitwise deterministic.
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

// Synthesis: lane i of tile t owns slots t*256*T + i + 256*u, u < T.
template <int T>
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
    const int tile = blockIdx.x - m * tiles;
    const int map = blockIdx.y;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;  // (l, m) lives at base + l
    const double2 *__restrict__ a = ap + (int64_t)map * nalm + base;
    const double *__restrict__ al = alpha + base;
    const double mu_m = mu[m];

    double x[T], q1[T], q2[T], cf[T], er[T], ei[T], orr[T], oi[T];
    int sc[T];
#pragma unroll
    for (int u = 0; u < T; ++u) {
        const int slot = tile * kBlock * T + u * kBlock + threadIdx.x;
        const bool act = slot < nslots;
        x[u] = act ? sx[slot] : 0.0;
        const double s = act ? ss[slot] : 1.0;
        const double seed = seed_carrier(m, s, mu_m, sc[u]);
        // state (q_{l-2}, q_{l-1}) before step l; (-seed, 0) makes step l = m yield the seed
        q2[u] = -seed;
        q1[u] = 0.0;
        cf[u] = (sc[u] == 0) ? 1.0 : 0.0;
        er[u] = ei[u] = orr[u] = oi[u] = 0.0;
    }
    auto any_scaled = [&]() {
        bool b = false;
#pragma unroll
        for (int u = 0; u < T; ++u) b |= (sc[u] < 0);
        return b;
    };
    auto all_scaled = [&]() {
        bool b = true;
#pragma unroll
        for (int u = 0; u < T; ++u) b &= (sc[u] < 0);
        return b;
    };
    auto rec = [&](double av) {
#pragma unroll
        for (int u = 0; u < T; ++u) {
            const double q = fma(av * x[u], q1[u], -q2[u]);
            q2[u] = q1[u];
            q1[u] = q;
        }
    };
    auto rescale = [&]() {
#pragma unroll
        for (int u = 0; u < T; ++u) {
            if (sc[u] < 0 && fabs(q1[u]) > kThresh) {
                q1[u] *= kDown;
                q2[u] *= kDown;
                ++sc[u];
                cf[u] = (sc[u] == 0) ? 1.0 : 0.0;
            }
        }
    };

    int l = m;
    // (A0) every value below range: recurrence only
    while (l + 1 <= lmax && __all(all_scaled())) {
        rec(al[l]);
        rec(al[l + 1]);
        rescale();
        l += 2;
    }
    // (A) some value below range: terms weighted by cf (0 or 1)
    while (l + 1 <= lmax && __any(any_scaled())) {
        const double2 c0 = a[l], c1 = a[l + 1];
        rec(al[l]);
#pragma unroll
        for (int u = 0; u < T; ++u) {
            const double p = cf[u] * q1[u];
            er[u] = fma(c0.x, p, er[u]);
            ei[u] = fma(c0.y, p, ei[u]);
        }
        rec(al[l + 1]);
#pragma unroll
        for (int u = 0; u < T; ++u) {
            const double p = cf[u] * q1[u];
            orr[u] = fma(c1.x, p, orr[u]);
            oi[u] = fma(c1.y, p, oi[u]);
        }
        rescale();
        l += 2;
    }
    // (B) all values in range: four steps per iteration, next block's
    // coefficients loaded one iteration ahead
    if (l + 3 <= lmax) {
        double a0 = al[l], a1 = al[l + 1], a2 = al[l + 2], a3 = al[l + 3];
        double2 c0 = a[l], c1 = a[l + 1], c2 = a[l + 2], c3 = a[l + 3];
        for (;;) {
            const bool more = (l + 7 <= lmax);
            double n0 = 0, n1 = 0, n2 = 0, n3 = 0;
            double2 d0 = c0, d1 = c1, d2 = c2, d3 = c3;
            if (more) {
                n0 = al[l + 4]; n1 = al[l + 5]; n2 = al[l + 6]; n3 = al[l + 7];
                d0 = a[l + 4]; d1 = a[l + 5]; d2 = a[l + 6]; d3 = a[l + 7];
            }
            rec(a0);
#pragma unroll
            for (int u = 0; u < T; ++u) { er[u] = fma(c0.x, q1[u], er[u]); ei[u] = fma(c0.y, q1[u], ei[u]); }
            rec(a1);
#pragma unroll
            for (int u = 0; u < T; ++u) { orr[u] = fma(c1.x, q1[u], orr[u]); oi[u] = fma(c1.y, q1[u], oi[u]); }
            rec(a2);
#pragma unroll
            for (int u = 0; u < T; ++u) { er[u] = fma(c2.x, q1[u], er[u]); ei[u] = fma(c2.y, q1[u], ei[u]); }
            rec(a3);
#pragma unroll
            for (int u = 0; u < T; ++u) { orr[u] = fma(c3.x, q1[u], orr[u]); oi[u] = fma(c3.y, q1[u], oi[u]); }
            l += 4;
            if (!more) break;
            a0 = n0; a1 = n1; a2 = n2; a3 = n3;
            c0 = d0; c1 = d1; c2 = d2; c3 = d3;
        }
    }
    // remaining steps (fewer than four), weighted by cf in case phase (A) ran out of l
    for (; l + 1 <= lmax; l += 2) {
        const double2 c0 = a[l], c1 = a[l + 1];
        rec(al[l]);
#pragma unroll
        for (int u = 0; u < T; ++u) {
            const double p = cf[u] * q1[u];
            er[u] = fma(c0.x, p, er[u]);
            ei[u] = fma(c0.y, p, ei[u]);
        }
        rec(al[l + 1]);
#pragma unroll
        for (int u = 0; u < T; ++u) {
            const double p = cf[u] * q1[u];
            orr[u] = fma(c1.x, p, orr[u]);
            oi[u] = fma(c1.y, p, oi[u]);
        }
    }
    if (l == lmax) {  // one trailing step with even (l - m)
        const double2 c0 = a[l];
        rec(al[l]);
#pragma unroll
        for (int u = 0; u < T; ++u) {
            const double p = cf[u] * q1[u];
            er[u] = fma(c0.x, p, er[u]);
            ei[u] = fma(c0.y, p, ei[u]);
        }
    }

    double2 *d = delta + (int64_t)map * nrings * (mmax + 1);
#pragma unroll
    for (int u = 0; u < T; ++u) {
        const int slot = tile * kBlock * T + u * kBlock + threadIdx.x;
        if (slot < nslots) {
            d[(int64_t)rn[slot] * (mmax + 1) + m] = make_double2(er[u] + orr[u], ei[u] + oi[u]);
            const int r2 = rsouth[slot];
            if (r2 >= 0) d[(int64_t)r2 * (mmax + 1) + m] = make_double2(er[u] - orr[u], ei[u] - oi[u]);
        }
    }
}

constexpr int kChunk = 8;   // l values per in-wave reduction in analysis
constexpr int kFlush = 8;   // chunks between cross-wave flushes (one barrier each)
constexpr int kTPad = 65;   // padded row (doubles) of the wave-private transpose buffer

// One chunk of kChunk recurrence steps for the T slots of a lane, accumulating
// sum_slots q_l * D(parity) per l, with the chunk's alpha_l in av.  SLOW:
// terms of slots still below range (sc < 0) are dropped and carriers rescaled;
// FULL: no l <= lmax guard.
template <int T, bool SLOW, bool FULL>
__device__ __forceinline__ void ana_chunk(int l0, int lmax, const double (&av)[kChunk],
                                          const double (&x)[T], double (&q1)[T], double (&q2)[T],
                                          int (&sc)[T], const double (&pr)[T], const double (&pi)[T],
                                          const double (&mr)[T], const double (&mi)[T],
                                          double (&accr)[kChunk], double (&acci)[kChunk]) {
#pragma unroll
    for (int i = 0; i < kChunk; ++i) {
        accr[i] = 0.0;
        acci[i] = 0.0;
        if (FULL || l0 + i <= lmax) {
#pragma unroll
            for (int t = 0; t < T; ++t) {
                // alpha * (x q_{l-1}): keeps the product on the dependency chain
                const double q = fma(av[i], x[t] * q1[t], -q2[t]);
                q2[t] = q1[t];
                q1[t] = q;
                const double p = SLOW ? (sc[t] == 0 ? q : 0.0) : q;
                accr[i] = fma(p, (i & 1) ? mr[t] : pr[t], accr[i]);
                acci[i] = fma(p, (i & 1) ? mi[t] : pi[t], acci[i]);
            }
            if (SLOW && (i & 1)) {
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    if (sc[t] < 0 && fabs(q1[t]) > kThresh) {
                        q1[t] *= kDown;
                        q2[t] *= kDown;
                        ++sc[t];
                    }
                }
            }
        }
    }
}

// quad all-reduce (lanes l, l^1, l^2, l^3) of a double through DPP moves
__device__ __forceinline__ double quad_sum(double v) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    double w = __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, 0xB1, 0xf, 0xf, false),
                                __builtin_amdgcn_update_dpp(0, lo, 0xB1, 0xf, 0xf, false));  // quad_perm [1,0,3,2]
    v += w;
    lo = __double2loint(v);
    hi = __double2hiint(v);
    w = __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, 0x4E, 0xf, 0xf, false),
                         __builtin_amdgcn_update_dpp(0, lo, 0x4E, 0xf, 0xf, false));  // quad_perm [2,3,0,1]
    return v + w;
}

// Analysis: workgroups of 4 waves; wave w of group g of m owns slots
// (g*4 + w) * 64T + lane*T + t.  Per chunk of kChunk l values each lane sums
// its T slots; the wave sums its 64 lanes through its own LDS rows (no
// barrier); every kFlush chunks the 4 wave sums are added in wave order after
// one barrier.  With one group the finished a_lm (times c_lm) is written;
// otherwise the group's partial goes to part[(map * groups + group) * nalm + idx]
// for k_ana_combine.
template <int T>
__global__ __launch_bounds__(kBlock) void k_leg_ana(int lmax, int mmax, int nslots, int nrings,
                                                    int64_t nalm, int groups,
                                                    const double2 *__restrict__ delta,
                                                    const double *__restrict__ alpha,
                                                    const double *__restrict__ cfac,
                                                    const double *__restrict__ mu,
                                                    const double *__restrict__ sx,
                                                    const double *__restrict__ ss,
                                                    const int32_t *__restrict__ rn,
                                                    const int32_t *__restrict__ rsouth,
                                                    double2 *__restrict__ alm,
                                                    double2 *__restrict__ part) {
    constexpr int kVals = 2 * kChunk;                 // (l, re/im) values per chunk
    constexpr int kWaves = kBlock / 64;
    __shared__ double tbuf[kWaves][kVals][kTPad];     // wave-private transpose rows
    __shared__ double ring[2][kFlush][kWaves][kVals]; // per-wave chunk sums awaiting the flush
    static_assert(kFlush * kVals <= kBlock, "one thread per flushed value");
    const int m = blockIdx.x / groups;
    const int grp = blockIdx.x - m * groups;
    const int map = blockIdx.y;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
    const double *__restrict__ al = alpha + base;
    const double2 *__restrict__ d = delta + (int64_t)map * nrings * (mmax + 1);

    double x[T], q1[T], q2[T], pr[T], pi[T], mr[T], mi[T];
    int sc[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int slot = (grp * kWaves + wave) * 64 * T + lane * T + t;
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
    }

    // flush bookkeeping: thread f < kFlush*kVals owns value (chunk f/kVals, j = f%kVals)
    const int fk = tid / kVals, fj = tid - fk * kVals;
    auto flush_out = [&](int lbase, int par, int nchunks, double cval) {
        if (tid < nchunks * kVals) {
            double v = 0.0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) v += ring[par][fk][w][fj];
            const int l = lbase + fk * kChunk + (fj >> 1);
            if (l <= lmax) {
                double *dst;
                if (groups == 1) {
                    dst = reinterpret_cast<double *>(alm + (int64_t)map * nalm + base + l) + (fj & 1);
                    v = (m == 0 && (fj & 1)) ? 0.0 : v * cval;
                } else {
                    dst = reinterpret_cast<double *>(part + ((int64_t)map * groups + grp) * nalm + base + l) + (fj & 1);
                }
                *dst = v;
            }
        }
    };
    auto cfac_for = [&](int lbase) {
        const int l = lbase + fk * kChunk + (fj >> 1);
        return (groups == 1 && tid < kFlush * kVals && l <= lmax) ? cfac[base + l] : 0.0;
    };

    double av[kChunk];
#pragma unroll
    for (int i = 0; i < kChunk; ++i) av[i] = (m + i <= lmax) ? al[m + i] : 0.0;
    int par = 0, kc = 0, lbase = m;
    double cval = cfac_for(lbase);
    for (int l0 = m; l0 <= lmax; l0 += kChunk) {
        double avn[kChunk];  // next chunk's alpha, loaded while this one computes
#pragma unroll
        for (int i = 0; i < kChunk; ++i) avn[i] = (l0 + kChunk + i <= lmax) ? al[l0 + kChunk + i] : 0.0;
        double accr[kChunk], acci[kChunk];
        bool scaled = false;
#pragma unroll
        for (int t = 0; t < T; ++t) scaled |= (sc[t] < 0);
        const bool slow = __any(scaled);
        const bool full = (l0 + kChunk - 1 <= lmax);
        if (full && !slow)
            ana_chunk<T, false, true>(l0, lmax, av, x, q1, q2, sc, pr, pi, mr, mi, accr, acci);
        else if (full)
            ana_chunk<T, true, true>(l0, lmax, av, x, q1, q2, sc, pr, pi, mr, mi, accr, acci);
        else
            ana_chunk<T, true, false>(l0, lmax, av, x, q1, q2, sc, pr, pi, mr, mi, accr, acci);
        // wave sum: each lane writes its 16 values as one column of the wave's
        // rows; lane (j = lane/4, q = lane%4) adds lanes 16q..16q+15 of row j,
        // and the quad of lanes 4j..4j+3 combines by DPP (lane 4j holds the sum)
#pragma unroll
        for (int i = 0; i < kChunk; ++i) {
            tbuf[wave][2 * i][lane] = accr[i];
            tbuf[wave][2 * i + 1][lane] = acci[i];
            av[i] = avn[i];
        }
        __builtin_amdgcn_wave_barrier();
        {
            const int j = lane >> 2, q = lane & 3;
            double v = 0.0;
#pragma unroll
            for (int k = 0; k < 16; ++k) v += tbuf[wave][j][q * 16 + k];
            v = quad_sum(v);
            if (q == 0) ring[par][kc][wave][j] = v;
        }
        __builtin_amdgcn_wave_barrier();
        ++kc;
        if (kc == kFlush || l0 + kChunk > lmax) {
            __syncthreads();
            flush_out(lbase, par, kc, cval);
            lbase += kFlush * kChunk;
            cval = cfac_for(lbase);
            par ^= 1;
            kc = 0;
        }
    }
}

// a_lm = c_lm * sum_{g < groups} part[map][g][idx], groups summed in order.
__global__ __launch_bounds__(kBlock) void k_ana_combine(int64_t nalm, int lmax, int nmaps, int groups,
                                                        const double2 *__restrict__ part,
                                                        const double *__restrict__ cfac,
                                                        double2 *__restrict__ alm) {
    const int64_t total = nalm * nmaps;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * kBlock) {
        const int64_t map = i / nalm, k = i - map * nalm;
        const double2 *src = part + map * groups * nalm + k;
        double sr = 0.0, si = 0.0;
        for (int g = 0; g < groups; ++g) {
            const double2 v = src[(int64_t)g * nalm];
            sr += v.x;
            si += v.y;
        }
        const double c = cfac[k];
        alm[i] = make_double2(sr * c, k <= lmax ? 0.0 : si * c);
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

constexpr int kSynSlotsPerLane = 2;

int launch_leg_syn(const CoefTables &c, const GeomPlan &p, const void *aprime, void *delta, int nmaps,
                   hipStream_t st) {
    constexpr int T = kSynSlotsPerLane;
    const int tiles = (p.nslots + kBlock * T - 1) / (kBlock * T);
    const int64_t gx = (int64_t)tiles * (c.mmax + 1);
    if (!grid_ok(gx) || nmaps > 65535) return SHT_EUNSUPPORTED;
    hipLaunchKernelGGL(k_leg_syn<T>, dim3((unsigned)gx, (unsigned)nmaps), dim3(kBlock), 0, st, c.lmax,
                       c.mmax, p.nslots, tiles, p.nrings, c.nalm, static_cast<const double2 *>(aprime),
                       c.alpha, c.mu, p.slot_x, p.slot_s, p.slot_north, p.slot_south,
                       static_cast<double2 *>(delta));
    SHT_HIP(hipGetLastError());
    return SHT_OK;
}

template <int T>
static void launch_ana_t(const CoefTables &c, const GeomPlan &p, int groups, const void *delta, void *alm,
                         void *part, int nmaps, hipStream_t st) {
    hipLaunchKernelGGL(k_leg_ana<T>, dim3((unsigned)((c.mmax + 1) * groups), (unsigned)nmaps), dim3(kBlock),
                       0, st, c.lmax, c.mmax, p.nslots, p.nrings, c.nalm, groups,
                       static_cast<const double2 *>(delta), c.alpha, c.cfac, c.mu, p.slot_x, p.slot_s,
                       p.slot_north, p.slot_south, static_cast<double2 *>(alm), static_cast<double2 *>(part));
}

int launch_leg_ana(const CoefTables &c, const GeomPlan &p, const void *delta, void *alm, int nmaps,
                   void *partials, hipStream_t st) {
    if (nmaps > 65535) return SHT_EUNSUPPORTED;
    const int T = ana_slots_per_thread(p.nslots);
    const int groups = ana_groups(p.nslots);
    if (!grid_ok((int64_t)(c.mmax + 1) * groups)) return SHT_EUNSUPPORTED;
    if (groups > 1 && !partials) return SHT_EWORKSPACE;
    switch (T) {
        case 1: launch_ana_t<1>(c, p, groups, delta, alm, partials, nmaps, st); break;
        case 2: launch_ana_t<2>(c, p, groups, delta, alm, partials, nmaps, st); break;
        default: launch_ana_t<kAnaSlotsPerThread>(c, p, groups, delta, alm, partials, nmaps, st); break;
    }
    SHT_HIP(hipGetLastError());
    if (groups > 1) {
        const int64_t total = c.nalm * nmaps;
        const int64_t blocks = std::min<int64_t>((total + kBlock - 1) / kBlock, 1 << 16);
        hipLaunchKernelGGL(k_ana_combine, dim3((unsigned)blocks), dim3(kBlock), 0, st, c.nalm, c.lmax, nmaps,
                           groups, static_cast<const double2 *>(partials), c.cfac, static_cast<double2 *>(alm));
        SHT_HIP(hipGetLastError());
    }
    return SHT_OK;
}

}  // namespace sht
