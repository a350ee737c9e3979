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
// plan tabulates alpha and c (0.16 < c < 1.13).  Synthesis folds c into a_lm
// once per call (k_prescale); analysis multiplies each finished a_lm by c.
//
// One recurrence serves a ring and its mirror image (x -> -x) because
// lambda_lm(-x) = (-1)^(l+m) lambda_lm(x): even and odd (l+m) partial sums
// are kept apart and combined as E+O (north) and E-O (south).
//
// Underflow near the poles (Sec. 2.1 asks for rescaling and leaves the
// algorithm to its references).  Once per plan, k_leg_start runs every
// (m, slot) recurrence from its seed with exponent tracking (a value held as
// q * 2^(600 sc), sc <= 0) until |q| first reaches 2^-100, and stores the l
// that opens the block of kStep steps (counted from m) holding that step,
// with the two recurrence values before it.  The transform kernels start
// each slot there: every term they leave out has |lambda| < 1.13 * 2^-100,
// and from its start on a slot's values stay in normal double range, so the
// hot loops have no rescaling.  A slot whose values stay below 2^-100 up to
// lmax is not started at all.
//
// Work mapping (the paper's GPU design assigns one ring per thread and the
// rings loop outermost; here a workgroup owns one m for a tile of ring
// pairs, so the loop over l is uniform across a wave and a_lm, alpha are
// wave-uniform scalar operands):
//   synthesis  grid.x = (m, 1024-slot tile), m ascending (longest first),
//              grid.y = map; four adjacent slots per lane, no reduction.
//   analysis   grid.x = (m, slot group), grid.y = map; a workgroup owns up
//              to 256T slots of its m (T adjacent slots per lane); each wave
//              sums its lanes through its own LDS rows, the four waves are
//              added in wave order every 64 l, and groups are summed in
//              order by a second small kernel: no atomics, deterministic.
#include "k_device.h"

namespace sht {
namespace {

constexpr double kDown = 0x1p-600;   // 2^-kScaleBits
constexpr double kThresh = 0x1p-60;  // carrier bound that triggers rescaling
constexpr double kStart = 0x1p-100;  // a slot starts once |q| reaches this
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

// Plan kernel: one thread per (m, slot); grid.x covers slots, grid.y = m.
// Writes lstart[m * nslots + slot] (lmax + 1 when never reached) and
// state[m * nslots + slot] = (q_{l-2}, q_{l-1}) before step l = lstart.
__global__ __launch_bounds__(kBlock) void k_leg_start(int lmax, int nslots, const double *__restrict__ alpha,
                                                      const double *__restrict__ mu,
                                                      const double *__restrict__ sx,
                                                      const double *__restrict__ ss,
                                                      int32_t *__restrict__ lstart,
                                                      double2 *__restrict__ state) {
    const int slot = blockIdx.x * kBlock + threadIdx.x;
    const int m = blockIdx.y;
    if (slot >= nslots) return;
    const double x = sx[slot];
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
    const double *__restrict__ al = alpha + base;
    int sc;
    const double seed = seed_carrier(m, ss[slot], mu[m], sc);
    // (q_{l-2}, q_{l-1}) before step l; (-seed, 0) makes step l = m yield the seed
    double q2 = -seed, q1 = 0.0;
    int found = lmax + 1;
    double s2 = 0.0, s1 = 0.0;
    for (int l0 = m; l0 <= lmax && found > lmax; l0 += kStartStep) {
        const double b2 = q2, b1 = q1;
        const int bsc = sc;
        bool hit = false;
        for (int i = 0; i < kStartStep && l0 + i <= lmax; ++i) {
            const double q = fma(al[l0 + i] * x, q1, -q2);
            q2 = q1;
            q1 = q;
            hit |= (sc == 0 && fabs(q) >= kStart);
            if ((i & 1) && sc < 0 && fabs(q1) > kThresh) {
                q1 *= kDown;
                q2 *= kDown;
                ++sc;
            }
        }
        if (hit) {
            found = l0;
            // a value leaves sc < 0 near 2^-660 and cannot grow past 2^-100
            // within one block, so bsc is 0 here in practice
            s2 = ldexp(b2, kScaleBits * bsc);
            s1 = ldexp(b1, kScaleBits * bsc);
        }
    }
    lstart[(int64_t)m * nslots + slot] = found;
    state[(int64_t)m * nslots + slot] = make_double2(s2, s1);
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

// One load from each of the first kBlock 128-byte lines of p[stride * i],
// i0 <= i <= i1 (addresses clamped to i1, so every load is in bounds).  The
// workgroup's pass over a coefficient column brings it into this XCD's L2
// ahead of the wave-uniform loads that use it; the value is only handed to an
// empty asm at the end of the kernel, so nothing waits for it before then.
__device__ __forceinline__ double warm_l2(const double *p, int stride, int i0, int i1) {
    const int per_line = 16 / stride;  // entries per 128 bytes
    const int i = min(i0 + per_line * (int)threadIdx.x, i1);
    return p[(int64_t)stride * i];
}

// Synthesis of one m of M maps over a tile of slots: thread li of the
// threads sharing the tile owns slots slot0 + li*T + u, u < T, for maps
// map0 .. map0 + M - 1 (those past nmaps repeat the last map and are not
// stored).  Each recurrence value serves the M maps, so a slot and l cost
// 2 + 2M operations instead of 4M; per map the arithmetic (the same fused
// multiply-adds in the same order) does not depend on M, so results are the
// same bits for any M.  The wave works on its own (no cross-wave step), so a
// tile may be one wave's (li = lane) or a workgroup's (li = thread index).
template <int T, int M = 1>
__device__ __forceinline__ void syn_tile(const SynArgs &A, int m, int map0, int nmaps, int slot0, int li) {
    const int lmax = A.lmax, mmax = A.mmax, nslots = A.nslots, nrings = A.nrings;
    const double *__restrict__ sx = A.sx;
    const int32_t *__restrict__ lstart = A.lstart;
    const double2 *__restrict__ state = A.state;
    const int32_t *__restrict__ rn = A.rn;
    const int32_t *__restrict__ rsouth = A.rsouth;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;  // (l, m) lives at base + l
    ConstC a[M];
#pragma unroll
    for (int k = 0; k < M; ++k) a[k] = ro(A.ap + (int64_t)min(map0 + k, nmaps - 1) * A.nalm + base);
    const const_ptr<double> al = ro(A.alpha + base);

    double x[T], q1[T], q2[T], er[T][M], ei[T][M], orr[T][M], oi[T][M];
    int ls[T];
    double2 st[T];
    int lo = lmax + 1, hi = m;
#pragma unroll
    for (int u = 0; u < T; ++u) {
        const int slot = slot0 + li * T + u;
        const bool act = slot < nslots;
        x[u] = act ? sx[slot] : 0.0;
        ls[u] = act ? lstart[(int64_t)m * nslots + slot] : lmax + 1;
        st[u] = act ? state[(int64_t)m * nslots + slot] : make_double2(0.0, 0.0);
        q1[u] = q2[u] = 0.0;  // a slot carries zeros until it starts
#pragma unroll
        for (int k = 0; k < M; ++k) er[u][k] = ei[u][k] = orr[u][k] = oi[u][k] = 0.0;
        lo = min(lo, ls[u]);
        if (ls[u] <= lmax) hi = max(hi, ls[u]);
    }
    lo = wave_min(lo);
    hi = wave_max(hi);

    auto rec = [&](double av) {
#pragma unroll
        for (int u = 0; u < T; ++u) {
            const double q = fma(av * x[u], q1[u], -q2[u]);
            q2[u] = q1[u];
            q1[u] = q;
        }
    };
    auto acc_e = [&](const double2 (&c)[M]) {
#pragma unroll
        for (int k = 0; k < M; ++k)
#pragma unroll
            for (int u = 0; u < T; ++u) {
                er[u][k] = fma(c[k].x, q1[u], er[u][k]);
                ei[u][k] = fma(c[k].y, q1[u], ei[u][k]);
            }
    };
    auto acc_o = [&](const double2 (&c)[M]) {
#pragma unroll
        for (int k = 0; k < M; ++k)
#pragma unroll
            for (int u = 0; u < T; ++u) {
                orr[u][k] = fma(c[k].x, q1[u], orr[u][k]);
                oi[u][k] = fma(c[k].y, q1[u], oi[u][k]);
            }
    };
    auto coef = [&](int l, double2 (&c)[M]) {
#pragma unroll
        for (int k = 0; k < M; ++k) c[k] = a[k][l];
    };
    auto step2 = [&](int l) {  // steps l (even l - m) and l + 1 (odd)
        double2 c[M];
        rec(al[l]);
        coef(l, c);
        acc_e(c);
        rec(al[l + 1]);
        coef(l + 1, c);
        acc_o(c);
    };
    auto inject = [&](int l) {
#pragma unroll
        for (int u = 0; u < T; ++u) {
            if (ls[u] == l) {
                q2[u] = st[u].x;
                q1[u] = st[u].y;
            }
        }
    };

    // start positions are m + kStartStep k: walk whole blocks while lanes join
    int l = lo;
    for (; l <= hi && l + kStartStep - 1 <= lmax; l += kStartStep) {
        inject(l);
#pragma unroll
        for (int i = 0; i < kStartStep; i += 2) step2(l + i);
    }
    if (l <= hi) inject(l);  // the last start lies in the ragged tail
    // l is uniform; restate it so that the compiler does not carry the lane
    // value it equals inside inject() into the loops below
    l = __builtin_amdgcn_readfirstlane(l);
    // every started slot is running: pairs of four-step halves with two
    // coefficient sets in turn, each loaded one half ahead (a and alpha are
    // padded, so the loads past lmax stay in bounds); the trip count is fixed
    // up front so that no exit separates a load from its use
    if (l + 7 <= lmax) {
        auto load4 = [&](int l4, double (&av)[4], double2 (&cv)[4][M]) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                av[i] = al[l4 + i];
                coef(l4 + i, cv[i]);
            }
            // compiler-only fence: keeps the loads here instead of letting
            // them sink to their first use in the next half
            asm volatile("" ::: "memory");
        };
        auto step4 = [&](const double (&av)[4], const double2 (&cv)[4][M]) {
            rec(av[0]);
            acc_e(cv[0]);
            rec(av[1]);
            acc_o(cv[1]);
            rec(av[2]);
            acc_e(cv[2]);
            rec(av[3]);
            acc_o(cv[3]);
        };
        const int npairs = (lmax + 1 - l) / 8;
        double avA[4], avB[4];
        double2 cvA[4][M], cvB[4][M];
        load4(l, avA, cvA);
        for (int b = 0; b < npairs; ++b) {
            load4(l + 4, avB, cvB);
            step4(avA, cvA);
            load4(l + 8, avA, cvA);
            step4(avB, cvB);
            l += 8;
        }
    }
    for (; l + 1 <= lmax; l += 2) step2(l);
    if (l == lmax) {  // one trailing step with even (l - m)
        double2 c[M];
        rec(al[l]);
        coef(l, c);
        acc_e(c);
    }

#pragma unroll
    for (int k = 0; k < M; ++k) {
        if (map0 + k >= nmaps) break;
        double2 *d = A.delta + (int64_t)(map0 + k) * nrings * (mmax + 1);
#pragma unroll
        for (int u = 0; u < T; ++u) {
            const int slot = slot0 + li * T + u;
            if (slot < nslots) {
                d[(int64_t)rn[slot] * (mmax + 1) + m] = make_double2(er[u][k] + orr[u][k], ei[u][k] + oi[u][k]);
                const int r2 = rsouth[slot];
                if (r2 >= 0)
                    d[(int64_t)r2 * (mmax + 1) + m] = make_double2(er[u][k] - orr[u][k], ei[u][k] - oi[u][k]);
            }
        }
    }
}

// Synthesis of M maps per workgroup (grid.y = map group of M), T slots per
// lane: the recurrence shared by the M maps (syn_tile).
template <int T, int M>
__global__ __launch_bounds__(kBlock, 2) void k_leg_syn_mm(SynArgs A, int tiles, int nmaps) {
    const MPart mp = xcd_m_part(tiles);
    const int m = mp.m, tile = mp.part;
    if (m > A.mmax) return;  // padding of the m range
    const int map0 = blockIdx.y * M;
    const int64_t base = (int64_t)m * (2 * A.lmax + 1 - m) / 2;
    const double warm_a = warm_l2(reinterpret_cast<const double *>(A.ap + (int64_t)map0 * A.nalm + base), 2, m, A.lmax);
    const double warm_al = warm_l2(A.alpha + base, 1, m, A.lmax);
    syn_tile<T, M>(A, m, map0, nmaps, tile * kBlock * T, (int)threadIdx.x);
    asm volatile("" ::"v"(warm_a), "v"(warm_al));  // the warming loads are waited for only here
}

// Synthesis kernel: grid.x = (m, 256T-slot tile) in the XCD-aware order,
// grid.y = map; thread i of tile t owns slots (t*256 + i)*T + u, u < T.
template <int T>
__global__ __launch_bounds__(kBlock, 4) void k_leg_syn(SynArgs A, int tiles) {
    const MPart mp = xcd_m_part(tiles);
    const int m = mp.m, tile = mp.part;
    if (m > A.mmax) return;  // padding of the m range
    const int64_t base = (int64_t)m * (2 * A.lmax + 1 - m) / 2;
    const double warm_a = warm_l2(reinterpret_cast<const double *>(A.ap + (int64_t)blockIdx.y * A.nalm + base), 2,
                                  m, A.lmax);
    const double warm_al = warm_l2(A.alpha + base, 1, m, A.lmax);
    syn_tile<T>(A, m, (int)blockIdx.y, (int)gridDim.y, tile * kBlock * T, (int)threadIdx.x);
    asm volatile("" ::"v"(warm_a), "v"(warm_al));  // the warming loads are waited for only here
}

constexpr int kChunk = kStartStep;  // l values per in-wave reduction in analysis
// chunks between cross-wave flushes (one barrier each); one thread per flushed value
constexpr int kFlush = kAnaThreads / (2 * kChunk) < 8 ? kAnaThreads / (2 * kChunk) : 8;
// Wave-private transpose rows: lane i stores its value at (i/16)*kQStride + i%16;
// lane (j, q) then reads 16 doubles from row j at q*kQStride.  With these
// strides the 16 lanes of each 64-bit LDS pass touch 16 distinct bank pairs
// on both the write and the read side.
constexpr int kQStride = 20;
constexpr int kTRow = 4 * kQStride + 1;

// One chunk of kChunk recurrence steps for the T slots of a lane, accumulating
// sum_slots q_l * D(parity) per l, with the chunk's alpha_l in av.  FULL: no
// l <= lmax guard.
template <int T, bool FULL>
__device__ __forceinline__ void ana_chunk(int l0, int lmax, const double (&av)[kChunk],
                                          const double (&x)[T], double (&q1)[T], double (&q2)[T],
                                          const double (&pr)[T], const double (&pi)[T],
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
                accr[i] = fma(q, (i & 1) ? mr[t] : pr[t], accr[i]);
                acci[i] = fma(q, (i & 1) ? mi[t] : pi[t], acci[i]);
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


constexpr int kVals = 2 * kChunk;            // (l, re/im) values per chunk
constexpr int kAnaWaves = kAnaThreads / 64;
// LDS of the analysis tiles: wave-private transpose rows, the per-wave chunk
// sums awaiting a cross-wave flush, and the waves' first starts.
struct AnaLds {
    double tbuf[kAnaWaves][kVals][kTRow];
    double ring[2][kFlush][kAnaWaves][kVals];
    int wstart[kAnaWaves];
};
static_assert(kFlush * kVals <= kAnaThreads, "one thread per flushed value");

// The slot operands of one lane: x, start, start state and the pair sums
// D+ = north + south (even l+m) and D- = north - south (odd) of Delta_m.
template <int T>
struct AnaSlots {
    double x[T], q1[T], q2[T], pr[T], pi[T], mr[T], mi[T];
    int ls[T];
    double2 st[T];
    int lo, hi;  // wave-uniform: earliest start, latest start (m if none)

    __device__ __forceinline__ void load(const AnaArgs &A, int m, const double2 *__restrict__ d, int slot0) {
        const int lmax = A.lmax, nslots = A.nslots;
        lo = lmax + 1;
        hi = m;
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const int slot = slot0 + t;
            const bool act = slot < nslots;
            x[t] = act ? A.sx[slot] : 0.0;
            ls[t] = act ? A.lstart[(int64_t)m * nslots + slot] : lmax + 1;
            st[t] = act ? A.state[(int64_t)m * nslots + slot] : make_double2(0.0, 0.0);
            double2 dn = make_double2(0.0, 0.0), ds = make_double2(0.0, 0.0);
            if (ls[t] <= lmax) {
                dn = d[(int64_t)A.rn[slot] * (A.mmax + 1) + m];
                const int r2 = A.rsouth[slot];
                if (r2 >= 0) ds = d[(int64_t)r2 * (A.mmax + 1) + m];
            }
            // even (l+m): north + south; odd: north - south
            pr[t] = dn.x + ds.x;
            pi[t] = dn.y + ds.y;
            mr[t] = dn.x - ds.x;
            mi[t] = dn.y - ds.y;
            q1[t] = q2[t] = 0.0;  // a slot carries zeros until it starts
            lo = min(lo, ls[t]);
            if (ls[t] <= lmax) hi = max(hi, ls[t]);
        }
        lo = wave_min(lo);
        hi = wave_max(hi);
    }
    __device__ __forceinline__ void inject(int l0) {
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const bool now = (ls[t] == l0);
            q2[t] = now ? st[t].x : q2[t];
            q1[t] = now ? st[t].y : q1[t];
        }
    }
};

// Wave sum of one chunk: each lane writes its 16 values as one column of the
// wave's rows; lane (j = lane/4, q = lane%4) adds lanes 16q..16q+15 of row j,
// and the quad of lanes 4j..4j+3 combines by DPP.  Returns the sum of value
// j in lanes with q == 0 (j = 2i + part: l = l0 + i, part 0 re / 1 im).
__device__ __forceinline__ double wave_sum16(double (*tb)[kTRow], const double (&accr)[kChunk],
                                             const double (&acci)[kChunk]) {
    const int lane = threadIdx.x & 63;
    const int lane_w = (lane >> 4) * kQStride + (lane & 15);  // this lane's column
#pragma unroll
    for (int i = 0; i < kChunk; ++i) {
        tb[2 * i][lane_w] = accr[i];
        tb[2 * i + 1][lane_w] = acci[i];
    }
    __builtin_amdgcn_wave_barrier();
    const int j = lane >> 2, q = lane & 3;
    const double *row = &tb[j][q * kQStride];
    double v = row[0];
#pragma unroll
    for (int k = 1; k < 16; ++k) v += row[k];
    v = quad_sum(v);
    __builtin_amdgcn_wave_barrier();
    return v;
}

// Analysis of one m of one map by a workgroup of 4 waves: wave w of group g
// owns slots ((g*4 + w) * 64 + lane) * T + t.  Per chunk of kChunk l values
// each lane sums its T slots; the wave sums its 64 lanes through its own LDS
// rows (no barrier); every kFlush chunks the 4 wave sums are added in wave
// order after one barrier.  The workgroup starts at the earliest start of
// its slots (a_lm before it get no term); a wave adds zeros until its own
// first start.  With one group the finished a_lm (times c_lm) is written;
// otherwise the group's partial goes to part[(map * groups + group) * nalm +
// idx] for k_ana_combine.  Every thread of the workgroup must call it.
template <int T>
__device__ __forceinline__ void ana_group(const AnaArgs &A, int m, int grp, int map, int groups, AnaLds &L) {
    const int lmax = A.lmax;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
    const const_ptr<double> al = ro(A.alpha + base);
    const double2 *__restrict__ d = A.delta + (int64_t)map * A.nrings * (A.mmax + 1);
    double2 *__restrict__ dst = (groups == 1) ? A.alm + (int64_t)map * A.nalm + base
                                              : A.part + ((int64_t)map * groups + grp) * A.nalm + base;
    AnaSlots<T> S;
    S.load(A, m, d, ((grp * kAnaWaves + wave) * 64 + lane) * T);
    const int lo = S.lo, hi = S.hi;
    if (lane == 0) L.wstart[wave] = lo;
    __syncthreads();
    int l0s = lmax + 1;
#pragma unroll
    for (int w = 0; w < kAnaWaves; ++w) l0s = min(l0s, L.wstart[w]);
    l0s = __builtin_amdgcn_readfirstlane(l0s);  // the same in every lane

    for (int l = m + tid; l < l0s; l += kAnaThreads) dst[l] = make_double2(0.0, 0.0);

    // flush bookkeeping: thread f < kFlush*kVals owns value (chunk f/kVals, j = f%kVals)
    const int fk = tid / kVals, fj = tid - fk * kVals;
    auto flush_out = [&](int lbase, int par, int nchunks, double cval) {
        if (tid < nchunks * kVals) {
            double v = 0.0;
#pragma unroll
            for (int w = 0; w < kAnaWaves; ++w) v += L.ring[par][fk][w][fj];
            const int l = lbase + fk * kChunk + (fj >> 1);
            if (l <= lmax) {
                if (groups == 1) v = (m == 0 && (fj & 1)) ? 0.0 : v * cval;
                reinterpret_cast<double *>(dst + l)[fj & 1] = v;
            }
        }
    };
    auto cfac_for = [&](int lbase) {
        const int l = lbase + fk * kChunk + (fj >> 1);
        return (groups == 1 && tid < kFlush * kVals && l <= lmax) ? A.cfac[base + l] : 0.0;
    };

    // alpha is read in whole chunks: entries past lmax belong to the next
    // column or the padding and are never used.  The chunk after next is
    // loaded once the wave's LDS traffic of a chunk is done, so that waiting
    // for that traffic never waits for the load as well.
    static_assert(3 * kChunk <= kCoefPad, "alpha padding too short");
    double av[kChunk], avn[kChunk];
#pragma unroll
    for (int i = 0; i < kChunk; ++i) {
        av[i] = al[l0s + i];
        avn[i] = al[l0s + kChunk + i];
    }
    int par = 0, kc = 0, lbase = l0s;
    double cval = cfac_for(lbase);

    // After each chunk: the wave's sums go to the ring buffer, the alpha
    // registers advance, and every kFlush chunks (or at the last) the four
    // waves' sums are added and written.  Every wave runs this once per chunk
    // from l0s on, whichever phase below it is in, so the barriers match.
    auto next_chunk = [&](int l0) {
#pragma unroll
        for (int i = 0; i < kChunk; ++i) {
            av[i] = avn[i];
            avn[i] = al[l0 + 2 * kChunk + i];
        }
        ++kc;
        if (kc == kFlush || l0 + kChunk > lmax) {
            __syncthreads();
            flush_out(lbase, par, kc, cval);
            lbase += kFlush * kChunk;
            cval = cfac_for(lbase);
            par ^= 1;
            kc = 0;
        }
    };
    auto to_ring = [&](const double (&accr)[kChunk], const double (&acci)[kChunk]) {
        const double v = wave_sum16(L.tbuf[wave], accr, acci);
        if ((lane & 3) == 0) L.ring[par][kc][wave][lane >> 2] = v;
    };

    // Three phases, each a loop without branches between chunk kinds, so the
    // recurrence registers stay in place from chunk to chunk:
    // (1) no slot of this wave has started: zero sums, no transpose
    int l0 = l0s;
#pragma unroll 1
    for (; l0 < lo && l0 <= lmax; l0 += kChunk) {
        if ((lane & 3) == 0) L.ring[par][kc][wave][lane >> 2] = 0.0;
        next_chunk(l0);
    }
    // (2) whole chunks; slots join at their tabulated start
#pragma unroll 1
    for (; l0 + kChunk - 1 <= lmax; l0 += kChunk) {
        if (l0 <= hi) S.inject(l0);
        double accr[kChunk], acci[kChunk];
        ana_chunk<T, true>(l0, lmax, av, S.x, S.q1, S.q2, S.pr, S.pi, S.mr, S.mi, accr, acci);
        to_ring(accr, acci);
        next_chunk(l0);
    }
    // (3) the ragged last chunk
    if (l0 <= lmax) {
        if (l0 <= hi) S.inject(l0);
        double accr[kChunk], acci[kChunk];
        ana_chunk<T, false>(l0, lmax, av, S.x, S.q1, S.q2, S.pr, S.pi, S.mr, S.mi, accr, acci);
        to_ring(accr, acci);
        next_chunk(l0);
    }
}

// Analysis of one m of one map by one wave holding every slot (nslots <=
// 64 T; lane i owns slots i*T + t): per chunk the wave's sum goes straight
// to a_lm (times c_lm), with no step across waves, so the four waves of a
// workgroup may each work on their own m.  tb: the wave's transpose rows.
template <int T>
__device__ __forceinline__ void ana_wave(const AnaArgs &A, int m, int map, double (*tb)[kTRow]) {
    const int lmax = A.lmax;
    const int lane = threadIdx.x & 63;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
    const const_ptr<double> al = ro(A.alpha + base);
    const double2 *__restrict__ d = A.delta + (int64_t)map * A.nrings * (A.mmax + 1);
    double2 *__restrict__ dst = A.alm + (int64_t)map * A.nalm + base;
    AnaSlots<T> S;
    S.load(A, m, d, lane * T);
    const int lo = S.lo, hi = S.hi;
    for (int l = m + lane; l < lo && l <= lmax; l += 64) dst[l] = make_double2(0.0, 0.0);
    if (lo > lmax) return;
    double av[kChunk], avn[kChunk];
#pragma unroll
    for (int i = 0; i < kChunk; ++i) {
        av[i] = al[lo + i];
        avn[i] = al[lo + kChunk + i];
    }
    const int j = lane >> 2;
    auto out = [&](int l0, const double (&accr)[kChunk], const double (&acci)[kChunk]) {
        const double v = wave_sum16(tb, accr, acci);
        const int l = l0 + (j >> 1);
        if ((lane & 3) == 0 && l <= lmax)
            reinterpret_cast<double *>(dst + l)[j & 1] = (m == 0 && (j & 1)) ? 0.0 : v * A.cfac[base + l];
#pragma unroll
        for (int i = 0; i < kChunk; ++i) {
            av[i] = avn[i];
            avn[i] = al[l0 + 2 * kChunk + i];
        }
    };
    int l0 = lo;
#pragma unroll 1
    for (; l0 + kChunk - 1 <= lmax; l0 += kChunk) {
        if (l0 <= hi) S.inject(l0);
        double accr[kChunk], acci[kChunk];
        ana_chunk<T, true>(l0, lmax, av, S.x, S.q1, S.q2, S.pr, S.pi, S.mr, S.mi, accr, acci);
        out(l0, accr, acci);
    }
    if (l0 <= lmax) {
        if (l0 <= hi) S.inject(l0);
        double accr[kChunk], acci[kChunk];
        ana_chunk<T, false>(l0, lmax, av, S.x, S.q1, S.q2, S.pr, S.pi, S.mr, S.mi, accr, acci);
        out(l0, accr, acci);
    }
}

// Analysis kernel: grid.x = (m, slot group) in the XCD-aware order, grid.y = map.
template <int T>
__global__ __launch_bounds__(kAnaThreads) void k_leg_ana(AnaArgs A, int groups) {
    __shared__ AnaLds L;
    const MPart mp = xcd_m_part(groups);
    if (mp.m > A.mmax) return;  // padding of the m range (whole workgroup, before any barrier)
    ana_group<T>(A, mp.m, mp.part, (int)blockIdx.y, groups, L);
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

// ---------------------------------------------------------------- uneven batches
// The Legendre stage of a whole batch of requests (any lmax and geometry, both
// directions) in one persistent launch.  Each workgroup takes the next item of
// a device work queue (one atomic add by one thread, broadcast through LDS)
// until the queue is empty, then exits; the host lists the items longest
// first, so that the cheap ones (high m, small requests) fill the end of the
// run on every CU.  Every item's work is that of the ordinary kernels, so
// which workgroup takes it does not change a result.
__global__ __launch_bounds__(kBlock, 3) void k_leg_batch(const BatchReq *__restrict__ reqs,
                                                       const BatchItem *__restrict__ items, int nitems,
                                                       int *__restrict__ head) {
    __shared__ AnaLds L;
    __shared__ int s_idx;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    for (;;) {
        if (threadIdx.x == 0) s_idx = atomicAdd(head, 1);
        __syncthreads();
        const int idx = __builtin_amdgcn_readfirstlane(s_idx);
        __syncthreads();  // every thread has read s_idx before it is written again
        if (idx >= nitems) return;  // the whole workgroup: the queue is empty
        const BatchItem it = items[idx];
        const BatchReq &R = reqs[it.req];
        const int T = R.T;
        if (R.kind == 0) {
            const int u = it.u0 + wave;
            if (u < R.nunits) {
                const int m = __builtin_amdgcn_readfirstlane(u / R.tiles);
                const int slot0 = (u - m * R.tiles) * 64 * T;
                if (T == 1) syn_tile<1>(R.syn, m, 0, 1, slot0, lane);
                else if (T == 2) syn_tile<2>(R.syn, m, 0, 1, slot0, lane);
                else syn_tile<4>(R.syn, m, 0, 1, slot0, lane);
            }
        } else if (R.shape == 0) {
            const int m = it.u0 + wave;
            if (m <= R.ana.mmax) {
                if (T == 1) ana_wave<1>(R.ana, m, 0, L.tbuf[wave]);
                else if (T == 2) ana_wave<2>(R.ana, m, 0, L.tbuf[wave]);
                else ana_wave<4>(R.ana, m, 0, L.tbuf[wave]);
            }
        } else {
            const int m = it.u0 / R.groups, grp = it.u0 - m * R.groups;
            if (T == 1) ana_group<1>(R.ana, m, grp, 0, R.groups, L);
            else if (T == 2) ana_group<2>(R.ana, m, grp, 0, R.groups, L);
            else ana_group<4>(R.ana, m, grp, 0, R.groups, L);
        }
        __syncthreads();  // the item's LDS use is over before the next one starts
    }
}

__global__ void k_batch_reset(int *head) { *head = 0; }

// c-scaled a_lm of every synthesis request of a batch: grid.y = request (of
// the list), grid.x strides over its a_lm.
__global__ __launch_bounds__(kBlock) void k_prescale_batch(const BatchReq *__restrict__ reqs,
                                                            const int32_t *__restrict__ list) {
    const BatchReq &R = reqs[list[blockIdx.y]];
    const int64_t nalm = R.syn.nalm;
    const int lmax = R.syn.lmax;
    const double *__restrict__ cfac = R.ana.cfac;
    double2 *out = const_cast<double2 *>(R.syn.ap);
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < nalm; k += (int64_t)gridDim.x * kBlock) {
        const double c = cfac[k];
        const double2 a = R.alm_in[k];
        out[k] = make_double2(a.x * c, k <= lmax ? 0.0 : a.y * c);  // Im a_l0 is ignored
    }
}

// a_lm = c_lm * sum of the group partials (groups in order) for every
// analysis request of the list that has several groups.
__global__ __launch_bounds__(kBlock) void k_combine_batch(const BatchReq *__restrict__ reqs,
                                                           const int32_t *__restrict__ list) {
    const BatchReq &R = reqs[list[blockIdx.y]];
    const int64_t nalm = R.ana.nalm;
    const int lmax = R.ana.lmax, groups = R.groups;
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < nalm; k += (int64_t)gridDim.x * kBlock) {
        double sr = 0.0, si = 0.0;
        for (int g = 0; g < groups; ++g) {
            const double2 v = R.ana.part[(int64_t)g * nalm + k];
            sr += v.x;
            si += v.y;
        }
        const double c = R.ana.cfac[k];
        R.ana.alm[k] = make_double2(sr * c, k <= lmax ? 0.0 : si * c);
    }
}

}  // namespace

int leg_batch_grid(int *grid) {
    int dev = 0, per_cu = 0;
    SHT_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    SHT_HIP(hipGetDeviceProperties(&prop, dev));
    SHT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_leg_batch, kBlock, 0));
    *grid = std::max(1, per_cu) * prop.multiProcessorCount;
    return SHT_OK;
}

int launch_leg_batch(const BatchReq *reqs, const BatchItem *items, int nitems, int *head, int grid, hipStream_t st) {
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, st, head);
    SHT_HIP(hipGetLastError());
    if (nitems <= 0) return SHT_OK;
    hipLaunchKernelGGL(k_leg_batch, dim3((unsigned)std::min(grid, nitems)), dim3(kBlock), 0, st, reqs, items, nitems,
                       head);
    SHT_HIP(hipGetLastError());
    return SHT_OK;
}

int launch_prescale_batch(const BatchReq *reqs, const int32_t *syn_reqs, int nsyn, int max_chunks, hipStream_t st) {
    if (nsyn <= 0) return SHT_OK;
    if (nsyn > 65535) return SHT_EUNSUPPORTED;
    hipLaunchKernelGGL(k_prescale_batch, dim3((unsigned)std::max(1, std::min(max_chunks, 4096)), (unsigned)nsyn),
                       dim3(kBlock), 0, st, reqs, syn_reqs);
    SHT_HIP(hipGetLastError());
    return SHT_OK;
}

int launch_combine_batch(const BatchReq *reqs, const int32_t *comb_reqs, int ncomb, int max_chunks, hipStream_t st) {
    if (ncomb <= 0) return SHT_OK;
    if (ncomb > 65535) return SHT_EUNSUPPORTED;
    hipLaunchKernelGGL(k_combine_batch, dim3((unsigned)std::max(1, std::min(max_chunks, 4096)), (unsigned)ncomb),
                       dim3(kBlock), 0, st, reqs, comb_reqs);
    SHT_HIP(hipGetLastError());
    return SHT_OK;
}

int launch_leg_start(const CoefTables &c, const GeomPlan &p, int32_t *lstart, void *state, hipStream_t st) {
    const int tiles = (p.nslots + kBlock - 1) / kBlock;
    if (c.mmax + 1 > 65535) return SHT_EUNSUPPORTED;
    hipLaunchKernelGGL(k_leg_start, dim3((unsigned)tiles, (unsigned)(c.mmax + 1)), dim3(kBlock), 0, st, c.lmax,
                       p.nslots, c.alpha, c.mu, p.slot_x, p.slot_s, lstart, static_cast<double2 *>(state));
    SHT_HIP(hipGetLastError());
    return SHT_OK;
}

int launch_prescale(const CoefTables &c, const void *alm, void *aprime, int nmaps, hipStream_t st) {
    const int64_t total = c.nalm * nmaps;
    const int64_t blocks = std::min<int64_t>((total + kBlock - 1) / kBlock, 1 << 16);
    hipLaunchKernelGGL(k_prescale, dim3((unsigned)blocks), dim3(kBlock), 0, st, c.nalm, c.lmax, nmaps,
                       static_cast<const double2 *>(alm), c.cfac, static_cast<double2 *>(aprime));
    SHT_HIP(hipGetLastError());
    return SHT_OK;
}

constexpr int kSynSlotsPerLane = 4;

template <int T, int M>
static int launch_syn_mm(const SynArgs &A, int nslots, int mmax, int nmaps, hipStream_t st) {
    const int tiles = (nslots + kBlock * T - 1) / (kBlock * T);
    const int64_t gx = (int64_t)tiles * padded_m(mmax);
    if (!grid_ok(gx)) return SHT_EUNSUPPORTED;
    hipLaunchKernelGGL((k_leg_syn_mm<T, M>), dim3((unsigned)gx, (unsigned)((nmaps + M - 1) / M)), dim3(kBlock), 0, st,
                       A, tiles, nmaps);
    SHT_HIP(hipGetLastError());
    return SHT_OK;
}

int launch_leg_syn(const CoefTables &c, const GeomPlan &p, const StartTable &s, const void *aprime, void *delta,
                   int nmaps, hipStream_t st) {
    const SynArgs A{c.lmax, c.mmax, p.nslots, p.nrings, c.nalm, static_cast<const double2 *>(aprime), c.alpha,
                    s.lstart, s.state, p.slot_x, p.slot_north, p.slot_south, static_cast<double2 *>(delta)};
    if (nmaps > 65535) return SHT_EUNSUPPORTED;
    // Slots per lane: kSynSlotsPerLane for large geometries, else the fewest
    // of 1 to 3 that put every slot of an m in one workgroup.  With few slots
    // a tile of kSynSlotsPerLane per lane would leave lanes and waves of the
    // workgroup idle while the others walk the l-recurrences of their slots in
    // turn; small transforms are bound by that sequential walk of the longest
    // m (at lmax 256 on 129 slots, 17.7 -> 8.5 us for the kernel with one slot
    // per lane), and on 513 slots (Gauss-Legendre at lmax 1024) three per lane
    // fill three waves with 9 slot-units of work where four per lane take 12.
    const int T = p.nslots <= kBlock         ? 1
                  : p.nslots <= 2 * kBlock   ? 2
                  : p.nslots <= 3 * kBlock   ? 3
                                             : kSynSlotsPerLane;
    // several maps share each recurrence: 2 maps per workgroup (at 4 slots per
    // lane faster than 4 maps and 2 slots: 29.7 against 30.6 ms for 64 maps at
    // HEALPix 1024 / lmax 2048)
    if (nmaps >= 2) {
        switch (T) {
            case 1: return launch_syn_mm<1, 2>(A, p.nslots, c.mmax, nmaps, st);
            case 2: return launch_syn_mm<2, 2>(A, p.nslots, c.mmax, nmaps, st);
            case 3: return launch_syn_mm<3, 2>(A, p.nslots, c.mmax, nmaps, st);
            default: return launch_syn_mm<kSynSlotsPerLane, 2>(A, p.nslots, c.mmax, nmaps, st);
        }
    }
    const int tiles = (p.nslots + kBlock * T - 1) / (kBlock * T);
    const int64_t gx = (int64_t)tiles * padded_m(c.mmax);
    if (!grid_ok(gx)) return SHT_EUNSUPPORTED;
    const dim3 grid((unsigned)gx, (unsigned)nmaps);
    switch (T) {
        case 1: hipLaunchKernelGGL(k_leg_syn<1>, grid, dim3(kBlock), 0, st, A, tiles); break;
        case 2: hipLaunchKernelGGL(k_leg_syn<2>, grid, dim3(kBlock), 0, st, A, tiles); break;
        case 3: hipLaunchKernelGGL(k_leg_syn<3>, grid, dim3(kBlock), 0, st, A, tiles); break;
        default: hipLaunchKernelGGL(k_leg_syn<kSynSlotsPerLane>, grid, dim3(kBlock), 0, st, A, tiles); break;
    }
    SHT_HIP(hipGetLastError());
    return SHT_OK;
}

template <int T>
static void launch_ana_t(const CoefTables &c, const GeomPlan &p, const StartTable &s, int groups,
                         const void *delta, void *alm, void *part, int nmaps, hipStream_t st) {
    const AnaArgs A{c.lmax, c.mmax, p.nslots, p.nrings, c.nalm, static_cast<const double2 *>(delta), c.alpha,
                    c.cfac, s.lstart, s.state, p.slot_x, p.slot_north, p.slot_south, static_cast<double2 *>(alm),
                    static_cast<double2 *>(part)};
    hipLaunchKernelGGL(k_leg_ana<T>, dim3((unsigned)(padded_m(c.mmax) * groups), (unsigned)nmaps), dim3(kAnaThreads), 0,
                       st, A, groups);
}

int launch_leg_ana(const CoefTables &c, const GeomPlan &p, const StartTable &s, const void *delta, void *alm,
                   int nmaps, void *partials, hipStream_t st) {
    if (nmaps > 65535) return SHT_EUNSUPPORTED;
    const int T = ana_slots_per_thread(p.nslots);
    const int groups = ana_groups(p.nslots);
    if (!grid_ok((int64_t)padded_m(c.mmax) * groups)) return SHT_EUNSUPPORTED;
    if (groups > 1 && !partials) return SHT_EWORKSPACE;
    switch (T) {
        case 1: launch_ana_t<1>(c, p, s, groups, delta, alm, partials, nmaps, st); break;
        case 2: launch_ana_t<2>(c, p, s, groups, delta, alm, partials, nmaps, st); break;
        case 3: launch_ana_t<3>(c, p, s, groups, delta, alm, partials, nmaps, st); break;
        case 4: launch_ana_t<4>(c, p, s, groups, delta, alm, partials, nmaps, st); break;
        default: launch_ana_t<kAnaSlotsPerThread>(c, p, s, groups, delta, alm, partials, nmaps, st); break;
    }
    SHT_HIP(hipGetLastError());
    return groups > 1 ? launch_ana_combine(c, nmaps, groups, partials, alm, st) : SHT_OK;
}

int launch_ana_combine(const CoefTables &c, int nmaps, int groups, const void *partials, void *alm,
                       hipStream_t st) {
    const int64_t total = c.nalm * nmaps;
    const int64_t blocks = std::min<int64_t>((total + kBlock - 1) / kBlock, 1 << 16);
    hipLaunchKernelGGL(k_ana_combine, dim3((unsigned)blocks), dim3(kBlock), 0, st, c.nalm, c.lmax, nmaps, groups,
                       static_cast<const double2 *>(partials), c.cfac, static_cast<double2 *>(alm));
    SHT_HIP(hipGetLastError());
    return SHT_OK;
}

}  // namespace sht
