// Ring Fourier stage for gfx950: one workgroup per job, two real sequences of
// one length transformed as one complex sequence held in LDS (the two rings
// of a mirror pair of one map, or with map-minor Delta one ring of two
// adjacent maps).  Jobs are launched in classes of transform length (<= 1024,
// 2048, 4096, 8192 points) so that LDS and the per-thread register arrays are
// sized for the class, with four or eight points per thread.
//
// Synthesis (Sec. 2.2 eq. Delta2map, with phi_j = phi0 + 2 pi j/N): for a
// real map the m < 0 half is the conjugate of the m > 0 half (eq. DeltaDef),
// so s_j = Re sum_{k<N} c_k e^{2 pi i k j/N} with
//   c_k = sum_{m = k mod N, m <= mmax} w_m Delta_m e^{i m phi0},  w_0 = 1 (real part), w_m = 2.
// Folding m mod N is exact aliasing for rings with N < 2 mmax + 1.  Since
// Re(z) = Re(conj z), s = Re FFT_forward(conj c).
//
// Analysis (eq. almfftdef with e^{-i m phi_j} and the ring's pixel weight):
//   Delta^S_m = w_r e^{-i m phi0} S_{m mod N},  S = FFT_forward(s).
//
// The FFT is an in-place Stockham decimation-in-time over the radices of the
// length (8, 4, 2, 3, 5, then any larger prime as a direct R-term stage); each
// stage reads its butterflies into registers, synchronises, and writes them
// back.  Lengths whose larger prime factors would make those direct stages
// costly use Bluestein's chirp-z identity instead (when 2N-1 rounds up to a
// 5-smooth length that fits)
//   X_k = conj(b_k) sum_n (x_n conj(b_n)) b_{k-n},  b_t = e^{i pi t^2/N},
// as a cyclic convolution of 5-smooth length L >= 2N-1 done with two forward
// transforms (the filter spectrum, scaled by 1/L, is a plan table).
#include <type_traits>

#include "k_device.h"

namespace sht {
namespace {

// plan descriptors are read through the constant address space (scalar loads)
using DescP = const_ptr<FftDesc>;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 conj2(double2 a) { return make_double2(a.x, -a.y); }

// sin and cos of r for |r| <= 4: quadrant reduction by pi/2 (two-term pi/2,
// fused multiply-adds), then Taylor series on |t| <= pi/4 with coefficients
// 1/n! up to t^19 (sin) and t^20 (cos); the truncation error is below 1e-19.
__device__ __forceinline__ void sincos_small(double r, double &sn, double &cs) {
    const double kPio2Hi = 1.5707963267948966;       // double(pi/2)
    const double kPio2Lo = 6.123233995736766e-17;    // pi/2 - kPio2Hi
    const double q = rint(r * 0.63661977236758138);  // r / (pi/2)
    double t = fma(-q, kPio2Hi, r);
    t = fma(-q, kPio2Lo, t);
    const double t2 = t * t;
    // sin t = t - t^3/3! + t^5/5! - ...
    double ps = -8.2206352466243295e-18;
    ps = fma(ps, t2, 2.8114572543455206e-15);
    ps = fma(ps, t2, -7.6471637318198164e-13);
    ps = fma(ps, t2, 1.6059043836821613e-10);
    ps = fma(ps, t2, -2.505210838544172e-08);
    ps = fma(ps, t2, 2.7557319223985893e-06);
    ps = fma(ps, t2, -0.00019841269841269841);
    ps = fma(ps, t2, 0.0083333333333333332);
    ps = fma(ps, t2, -0.16666666666666666);
    const double sv = fma(ps * t2, t, t);
    double pc = 4.1103176233121648e-19;
    pc = fma(pc, t2, -1.5619206968586225e-16);
    pc = fma(pc, t2, 4.7794773323873853e-14);
    pc = fma(pc, t2, -1.1470745597729725e-11);
    pc = fma(pc, t2, 2.08767569878681e-09);
    pc = fma(pc, t2, -2.7557319223985888e-07);
    pc = fma(pc, t2, 2.4801587301587302e-05);
    pc = fma(pc, t2, -0.0013888888888888889);
    pc = fma(pc, t2, 0.041666666666666664);
    pc = fma(pc, t2, -0.5);
    const double cv = fma(pc, t2, 1.0);
    const int iq = ((int)q) & 3;
    const double s0 = (iq & 1) ? cv : sv;
    const double c0 = (iq & 1) ? sv : cv;
    sn = (iq & 2) ? -s0 : s0;
    cs = ((iq + 1) & 2) ? -c0 : c0;
}

// e^{i m phi0} with the product m*phi0 split exactly (fma) and reduced
// modulo 2 pi with a two-term 2 pi, so the phase error is ~1 ulp of pi
// instead of ~1 ulp of m*phi0.
__device__ __forceinline__ double2 phase_exp(int m, double phi0) {
    const double kTwoPiHi = 6.283185307179586232;        // double(2 pi)
    const double kTwoPiLo = 2.4492935982947064e-16;      // 2 pi - kTwoPiHi
    const double kInvTwoPi = 0.15915494309189535;
    const double dm = (double)m;
    const double hi = dm * phi0;
    const double lo = fma(dm, phi0, -hi);
    const double n = rint(hi * kInvTwoPi);
    double r = fma(-n, kTwoPiHi, hi);
    r = fma(-n, kTwoPiLo, r);
    r += lo;
    double sn, cs;
    sincos_small(r, sn, cs);
    return make_double2(cs, sn);
}

// e^{i m phi0} of one ring from two LDS tables filled per workgroup with
// phase_exp: lo[b] = e^{i b phi0} (b < 64) and hi[h] = e^{i 64 h phi0}, so
// e^{i m phi0} = hi[m / 64] lo[m % 64] (one complex product, about one more
// rounding than phase_exp) for m < 64 * kPhHiMax.  With hi == nullptr the
// phase is evaluated directly.
constexpr int kPhLo = 64;
constexpr int kPhHiMax = 64;
__host__ __device__ constexpr int phase_hi_entries(int mmax) { return mmax / kPhLo + 1; }
struct Phase {
    const double2 *lo, *hi;
    double phi0;
    __device__ __forceinline__ double2 operator()(int m) const {
        if (!hi) return phase_exp(m, phi0);
        const double2 a = hi[m / kPhLo], b = lo[m % kPhLo];
        return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
    }
};
template <int NT>
__device__ __forceinline__ Phase load_phases(double2 *tab, int mmax, double phi0) {
    const int nh = phase_hi_entries(mmax);
    for (int t = threadIdx.x; t < kPhLo + nh; t += NT)
        tab[t] = phase_exp(t < kPhLo ? t : (t - kPhLo) * kPhLo, phi0);
    return Phase{tab, tab + kPhLo, phi0};
}

// Forward-sign butterflies of radix 2, 3, 4, 5, 8 in registers, with the
// roots of unity as constants: cos(2pi/5) = (sqrt5-1)/4, cos(4pi/5) =
// -(sqrt5+1)/4, sin(2pi/5), sin(4pi/5), sqrt(3)/2 and 1/sqrt(2), each rounded
// to double.
__device__ __forceinline__ double2 add2(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 sub2(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// a - i b and a + i b
__device__ __forceinline__ double2 sub_i(double2 a, double2 b) { return make_double2(a.x + b.y, a.y - b.x); }
__device__ __forceinline__ double2 add_i(double2 a, double2 b) { return make_double2(a.x - b.y, a.y + b.x); }

template <int R>
__device__ __forceinline__ void butterfly(double2 (&v)[R]) {
    if constexpr (R == 2) {
        const double2 a = v[0], b = v[1];
        v[0] = add2(a, b);
        v[1] = sub2(a, b);
    } else if constexpr (R == 3) {
        const double kH3 = 0.8660254037844386;
        const double2 a = v[0], s = add2(v[1], v[2]), d = sub2(v[1], v[2]);
        const double2 m = make_double2(fma(-0.5, s.x, a.x), fma(-0.5, s.y, a.y));
        const double2 u = make_double2(kH3 * d.x, kH3 * d.y);
        v[0] = add2(a, s);
        v[1] = sub_i(m, u);
        v[2] = add_i(m, u);
    } else if constexpr (R == 4) {
        const double2 a = v[0], b = v[1], c = v[2], d = v[3];
        const double2 s0 = add2(a, c), s1 = sub2(a, c), s2 = add2(b, d), s3 = sub2(b, d);
        v[0] = add2(s0, s2);
        v[2] = sub2(s0, s2);
        v[1] = sub_i(s1, s3);
        v[3] = add_i(s1, s3);
    } else if constexpr (R == 8) {
        // pairs (n, n+4), then the odd half turned by W8^n, then two radix-4 DFTs
        const double kR = 0.70710678118654752;  // 1/sqrt(2)
        double2 a[4], b[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            a[n] = add2(v[n], v[n + 4]);
            b[n] = sub2(v[n], v[n + 4]);
        }
        b[1] = make_double2((b[1].x + b[1].y) * kR, (b[1].y - b[1].x) * kR);
        b[2] = make_double2(b[2].y, -b[2].x);
        b[3] = make_double2((b[3].y - b[3].x) * kR, -(b[3].x + b[3].y) * kR);
        butterfly<4>(a);
        butterfly<4>(b);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[2 * k] = a[k];
            v[2 * k + 1] = b[k];
        }
    } else if constexpr (R == 5) {
        const double kC1 = 0.30901699437494745, kC2 = -0.8090169943749475;
        const double kS1 = 0.9510565162951535, kS2 = 0.5877852522924731;
        const double2 a = v[0];
        const double2 p1 = add2(v[1], v[4]), q1 = sub2(v[1], v[4]);
        const double2 p2 = add2(v[2], v[3]), q2 = sub2(v[2], v[3]);
        const double2 r1 = make_double2(fma(kC1, p1.x, fma(kC2, p2.x, a.x)), fma(kC1, p1.y, fma(kC2, p2.y, a.y)));
        const double2 r2 = make_double2(fma(kC2, p1.x, fma(kC1, p2.x, a.x)), fma(kC2, p1.y, fma(kC1, p2.y, a.y)));
        const double2 i1 = make_double2(fma(kS1, q1.x, kS2 * q2.x), fma(kS1, q1.y, kS2 * q2.y));
        const double2 i2 = make_double2(fma(kS2, q1.x, -kS1 * q2.x), fma(kS2, q1.y, -kS1 * q2.y));
        v[0] = add2(a, add2(p1, p2));
        v[1] = sub_i(r1, i1);
        v[4] = add_i(r1, i1);
        v[2] = sub_i(r2, i2);
        v[3] = add_i(r2, i2);
    }
}

// Twiddles W_L^t = e^{-2 pi i t / L} come from two small LDS tables,
// W_L^t = hi[t / 64] * lo[t % 64] with hi[h] = W_L^{64 h} and lo[u] = W_L^u,
// both copied from the plan's correctly rounded table once per workgroup:
// one extra complex product per twiddle (about one more rounding) instead of
// a global load in every stage.  A radix-R butterfly takes W^{k tstep} from
// the tables and its other twiddles as powers of it (at most R - 2 further
// products, a few ulp for R <= 8).
constexpr int kTwLo = 64;
// LDS index of point x (unpadded: a slot after every 8 points, meant to
// spread the strided Stockham writes over the banks, timed slower on gfx950)
__device__ __forceinline__ int pd(int x) { return x; }
template <int L>
constexpr int padded_len() { return L; }
template <int MAXL>
constexpr int tw_entries() { return kTwLo + (MAXL + kTwLo - 1) / kTwLo; }

struct TwLds {
    const double2 *lo, *hi;
    __device__ __forceinline__ double2 operator()(int t) const { return cmul(hi[t / kTwLo], lo[t % kTwLo]); }
};

// fills the two tables for length L from the plan table tw (caller synchronises)
template <int NT>
__device__ __forceinline__ void load_twiddles(double2 *lo, double2 *hi, const double2 *__restrict__ tw, int L) {
    const int nhi = (L + kTwLo - 1) / kTwLo;
    for (int t = threadIdx.x; t < kTwLo + nhi; t += NT) {
        if (t < kTwLo)
            lo[t] = t < L ? tw[t] : make_double2(1.0, 0.0);
        else
            hi[t - kTwLo] = tw[(t - kTwLo) * kTwLo];
    }
}

// One Stockham stage of radix R on buf[0..L), L <= MAXL, Ns = product of
// earlier radices.  Each thread holds up to kMaxB twiddled butterflies in
// registers (NT threads) and writes them back after the barrier.
// Point access of a stage: LDS (the default), or a caller's function that
// supplies the first stage's input points / takes the last stage's output
// points in registers (no LDS pass and no barrier for them).
struct LdsIn {
    const double2 *buf;
    __device__ __forceinline__ double2 operator()(int t) const { return buf[pd(t)]; }
};
struct LdsOut {
    double2 *buf;
    __device__ __forceinline__ void operator()(int t, double2 v) const { buf[pd(t)] = v; }
};

// FIRST: the first stage (Ns = 1, all twiddles 1); a stage with register
// input is always the first.
template <int R, int MAXL, int NT, bool FIRST = false, class In = LdsIn, class Out = LdsOut>
__device__ __forceinline__ void fft_stage(double2 *buf, int L, int Ns_, TwLds tw, In in = In{}, Out out = Out{}) {
    constexpr bool kLdsIn = std::is_same<In, LdsIn>::value, kLdsOut = std::is_same<Out, LdsOut>::value;
    constexpr bool kFirst = FIRST || !kLdsIn;
    const int Ns = kFirst ? 1 : Ns_;
    constexpr int kMaxB = (MAXL / R + NT - 1) / NT;
    const int nbf = L / R;
    const int tstep = L / (Ns * R);
    // j / Ns from a float reciprocal: (j + 0.5) / Ns stays at least 0.5/Ns away
    // from an integer, far beyond the float rounding for j, Ns <= 8192
    const float inv_ns = 1.0f / (float)Ns;
    double2 v[kMaxB][R];
#pragma unroll
    for (int b = 0; b < kMaxB; ++b) {
        const int j = threadIdx.x + b * NT;
        if (j < nbf) {
            const int jq = (int)(((float)j + 0.5f) * inv_ns);
            const int k = j - jq * Ns;
            // twiddles W^{r k tstep} as powers of W^{k tstep}
            const double2 w1 = tw(k * tstep);
            double2 wr = w1;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double2 xv = kLdsIn ? buf[pd(j + r * nbf)] : in(j + r * nbf);
                if (r == 0 || kFirst) {
                    v[b][r] = xv;
                } else {
                    v[b][r] = cmul(xv, wr);
                    if (r + 1 < R) wr = cmul(wr, w1);
                }
            }
            butterfly<R>(v[b]);
        }
    }
    if (kLdsIn) __syncthreads();  // in place: every read is done before the writes
#pragma unroll
    for (int b = 0; b < kMaxB; ++b) {
        const int j = threadIdx.x + b * NT;
        if (j < nbf) {
            const int jq = (int)(((float)j + 0.5f) * inv_ns);
            const int k = j - jq * Ns;
            const int o = jq * Ns * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (kLdsOut)
                    buf[pd(o + r * Ns)] = v[b][r];
                else
                    out(o + r * Ns, v[b][r]);
            }
        }
    }
    if (kLdsOut) __syncthreads();
}

// One Stockham stage of a prime radix R > 5 (a direct R-term DFT per
// butterfly).  Butterfly j (k = j mod Ns) takes x_q = buf[j + q L/R] twiddled
// to x'_q = x_q W_L^{q k tstep}; its outputs y_s = sum_q x'_q W_R^{q s} go to
// o + s Ns.  With W_R^{q s} = cos t - i sin t (t = 2 pi q s / R) and the
// inputs paired with their mirrors, P_q = x'_q + x'_{R-q} and M_q = x'_q -
// x'_{R-q} (q = 1 .. h, h = (R-1)/2),
//   y_s = A_s - i B_s,  y_{R-s} = A_s + i B_s,
//   A_s = x'_0 + sum_q P_q cos t,  B_s = sum_q M_q sin t,
// so an output pair costs 4 real multiply-adds per q instead of 8 per term
// of each output.  Pass 1 forms P and M in place (q in slot q, M in slot R-q);
// pass 2 gives each thread items of two output pairs (s, s+1) of one
// butterfly, holds the outputs until every thread has read its inputs, then
// writes them.  W_R^{q s} is carried in registers (w <- w W_R^s) and taken
// afresh from the table, at the exact integer exponent q s mod R, every
// kAnchor terms (a recurrence error of at most kAnchor roundings).
template <int MAXL, int NT>
__device__ __forceinline__ void fft_stage_generic(double2 *buf, int L, int Ns, int R, TwLds tw) {
    constexpr int kAnchor = 16;
    constexpr int kPairs = 2;  // output pairs per item
    // pass 2 has (L / R) floor((R + 3) / 4) items; over the primes R >= 7 that
    // is at most 0.31 L (R = 13), so 0.31 MAXL / NT items per thread
    constexpr int kMaxItems = (4 * MAXL / NT + 12) / 13;
    const int nbf = L / R, h = (R - 1) / 2;
    const int tstep = L / (Ns * R);
    const float inv_nbf = 1.0f / (float)nbf, inv_ns = 1.0f / (float)Ns;
    // pass 1: P_q, M_q for q = 1 .. h of every butterfly, in place
    for (int i = threadIdx.x; i < nbf * h; i += NT) {
        const int q = 1 + (int)(((float)i + 0.5f) * inv_nbf);  // (i + 0.5) / nbf is 0.5/nbf from an integer
        const int j = i - (q - 1) * nbf;
        const int jq = (int)(((float)j + 0.5f) * inv_ns);
        const int kt = (j - jq * Ns) * tstep;  // k tstep < L / R: q kt < L
        const double2 a = cmul(buf[pd(j + q * nbf)], tw(q * kt));
        const double2 b = cmul(buf[pd(j + (R - q) * nbf)], tw((R - q) * kt));
        buf[pd(j + q * nbf)] = add2(a, b);
        buf[pd(j + (R - q) * nbf)] = sub2(a, b);
    }
    __syncthreads();
    // pass 2: item i = (group g, butterfly j); group g holds s = 2 g, 2 g + 1 (<= h)
    const int ng = (h + kPairs) / kPairs;
    double2 y[kMaxItems][2 * kPairs];
#pragma unroll
    for (int it = 0; it < kMaxItems; ++it) {
        const int i = threadIdx.x + it * NT;
        if (i >= nbf * ng) break;
        const int g = (int)(((float)i + 0.5f) * inv_nbf);
        const int j = i - g * nbf;
        const double2 x0 = buf[pd(j)];
        double2 A[kPairs], Bp[kPairs], w[kPairs], ws[kPairs];
#pragma unroll
        for (int u = 0; u < kPairs; ++u) {
            const int sv = min(kPairs * g + u, h);
            A[u] = x0;
            Bp[u] = make_double2(0.0, 0.0);
            ws[u] = tw(sv * nbf);  // W_R^s
        }
        for (int q0 = 1; q0 <= h; q0 += kAnchor) {
#pragma unroll
            for (int u = 0; u < kPairs; ++u) {
                const int sv = min(kPairs * g + u, h);
                w[u] = tw(((q0 * sv) % R) * nbf);  // W_R^{q0 s}, exact exponent
            }
            const int qe = min(h, q0 + kAnchor - 1);
            for (int q = q0; q <= qe; ++q) {
                const double2 P = buf[pd(j + q * nbf)], M = buf[pd(j + (R - q) * nbf)];
#pragma unroll
                for (int u = 0; u < kPairs; ++u) {
                    // A += cos t P, B' += -sin t M = w.y M  (so B = -B')
                    A[u].x = fma(w[u].x, P.x, A[u].x);
                    A[u].y = fma(w[u].x, P.y, A[u].y);
                    Bp[u].x = fma(w[u].y, M.x, Bp[u].x);
                    Bp[u].y = fma(w[u].y, M.y, Bp[u].y);
                    w[u] = cmul(w[u], ws[u]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kPairs; ++u) {
            // y_s = A - i B = A + i B', y_{R-s} = A + i B = A - i B'
            y[it][2 * u] = make_double2(A[u].x - Bp[u].y, A[u].y + Bp[u].x);
            y[it][2 * u + 1] = make_double2(A[u].x + Bp[u].y, A[u].y - Bp[u].x);
        }
    }
    __syncthreads();  // in place: every input is read before the outputs land
#pragma unroll
    for (int it = 0; it < kMaxItems; ++it) {
        const int i = threadIdx.x + it * NT;
        if (i >= nbf * ng) break;
        const int g = (int)(((float)i + 0.5f) * inv_nbf);
        const int j = i - g * nbf;
        const int jq = (int)(((float)j + 0.5f) * inv_ns);
        const int o = jq * Ns * R + (j - jq * Ns);
#pragma unroll
        for (int u = 0; u < kPairs; ++u) {
            const int sv = kPairs * g + u;
            if (sv > h) break;
            buf[pd(o + sv * Ns)] = y[it][2 * u];
            if (sv > 0) buf[pd(o + (R - sv) * Ns)] = y[it][2 * u + 1];
        }
    }
    __syncthreads();
}

// Whether the first (last) stage of the transform of d can take its input
// (give its output) in registers: a radix-4 or radix-8 stage of a direct
// transform with more than one stage.  (Not under Bluestein: evaluating the
// chirp inside the unrolled stage costs more registers than the LDS pass.)
__device__ __forceinline__ bool reg_stage_ok(int R) { return R == 8 || R == 4; }
__device__ __forceinline__ bool reg_first(DescP d) { return !d->bluestein && d->nrad > 1 && reg_stage_ok(d->rad[0]); }
__device__ __forceinline__ bool reg_last(DescP d) {
    return !d->bluestein && d->nrad > 1 && reg_stage_ok(d->rad[d->nrad - 1]);
}

// Stages s0 .. s1-1 of the forward FFT of length d->L (<= MAXL) in LDS, Ns0
// the product of the radices before s0 (all stages: natural order in and out).
template <int MAXL, int NT>
__device__ __forceinline__ void fft_stages(double2 *buf, DescP d, TwLds tw, int s0, int s1, int Ns0) {
    const int L = d->L;
    int Ns = Ns0;
    for (int s = s0; s < s1; ++s) {
        const int R = d->rad[s];
        switch (Ns == 1 ? -R : R) {
            case -8: fft_stage<8, MAXL, NT, true>(buf, L, 1, tw); break;
            case -4: fft_stage<4, MAXL, NT, true>(buf, L, 1, tw); break;
            case -2: case 2: fft_stage<2, MAXL, NT>(buf, L, Ns, tw); break;
            case -3: case 3: fft_stage<3, MAXL, NT>(buf, L, Ns, tw); break;
            case -5: case 5: fft_stage<5, MAXL, NT>(buf, L, Ns, tw); break;
            case 8: fft_stage<8, MAXL, NT>(buf, L, Ns, tw); break;
            case 4: fft_stage<4, MAXL, NT>(buf, L, Ns, tw); break;
            default: fft_stage_generic<MAXL, NT>(buf, L, Ns, R, tw); break;
        }
        Ns *= R;
    }
}

// DFT of n points: afterwards X_k is result_at(buf, d, k).  The points are those
// already placed in buf[0..n) (pre-multiplied by conj(chirp) when Bluestein),
// or, when in_reg and reg_first(d), in(t) for t < L = n, read by the first
// stage.  With out_reg and reg_last(d) the last stage hands X_t to out(t, X_t)
// instead (t < n), and buf holds no result.  (The register stages sit outside
// the stage loop, so that the compiler keeps none of their addresses live
// across it.)
template <int MAXL, int NT, class In = LdsIn, class Out = LdsOut>
__device__ __forceinline__ void transform(double2 *buf, DescP d, TwLds tw, In in = In{}, bool in_reg = false,
                                          Out out = Out{}, bool out_reg = false) {
    constexpr bool kRegIn = !std::is_same<In, LdsIn>::value, kRegOut = !std::is_same<Out, LdsOut>::value;
    const int L = d->L, nrad = d->nrad, passes = d->bluestein ? 2 : 1;
    in_reg = kRegIn && in_reg && reg_first(d);
    out_reg = kRegOut && out_reg && reg_last(d);
    int s0 = 0, Ns0 = 1;
    if constexpr (kRegIn) {
        if (in_reg) {
            s0 = 1;
            Ns0 = d->rad[0];
            if (Ns0 == 8)
                fft_stage<8, MAXL, NT, true, In, LdsOut>(buf, L, 1, tw, in, LdsOut{buf});
            else
                fft_stage<4, MAXL, NT, true, In, LdsOut>(buf, L, 1, tw, in, LdsOut{buf});
        }
    }
    const int s1 = out_reg ? nrad - 1 : nrad;
    // Bluestein (no register stages): zero padding, then two transforms with
    // one copy of the stage code (the kernels are otherwise large enough to
    // thrash the instruction cache)
    const double2 *__restrict__ kern = d->kern;
    if (passes == 2) {
        for (int t = d->n + threadIdx.x; t < L; t += NT) buf[pd(t)] = make_double2(0.0, 0.0);
        __syncthreads();
    }
#pragma unroll 1
    for (int pass = 0; pass < passes; ++pass) {
        if (pass == 1) {
            for (int t = threadIdx.x; t < L; t += NT) buf[pd(t)] = conj2(cmul(buf[pd(t)], kern[t]));
            __syncthreads();
        }
        fft_stages<MAXL, NT>(buf, d, tw, pass == 0 ? s0 : 0, pass == passes - 1 ? s1 : nrad, pass == 0 ? Ns0 : 1);
    }
    if constexpr (kRegOut) {
        if (out_reg) {
            const int R = d->rad[nrad - 1];
            if (R == 8)
                fft_stage<8, MAXL, NT, false, LdsIn, Out>(buf, L, L / 8, tw, LdsIn{buf}, out);
            else
                fft_stage<4, MAXL, NT, false, LdsIn, Out>(buf, L, L / 4, tw, LdsIn{buf}, out);
        }
    }
}

// Bluestein chirp b_t = e^{i pi t^2 / n}.  The angle's numerator q = t^2
// mod 2n is an exact integer; b_t = hi[q / 64] lo[q % 64] from two LDS tables
// filled per workgroup, lo[u] = e^{i pi u / n} (u < 64) and hi[h] = e^{i pi
// 64 h / n} (64 h < 2n), each entry from the reduced-range sin/cos at pi r / n
// with r = its numerator taken exactly into (-n, n]: one complex product per
// point (about one more rounding) instead of a sin/cos evaluation, and no
// per-length table in memory.
constexpr int kChLo = 64;
template <int MAXL>
constexpr int chirp_entries() { return kChLo + MAXL / kChLo + 1; }  // 2n <= L + 2 <= MAXL + 2
__device__ __forceinline__ double2 e_pi_over(int r, int n) {
    const int n2 = 2 * n;
    r %= n2;
    if (r > n) r -= n2;
    double sn, cs;
    sincos_small(3.141592653589793 * (double)r / (double)n, sn, cs);
    return make_double2(cs, sn);
}
struct Chirp {
    const double2 *lo, *hi;
    int n;
    double inv2n;  // 1 / (2n)
    __device__ __forceinline__ double2 operator()(int t) const {
        // t^2 < 2^27 (t < 8192); the quotient from the double reciprocal is
        // off by at most one, corrected below
        const int n2 = 2 * n, tt = t * t;
        int q = tt - (int)((double)tt * inv2n) * n2;
        q = q < 0 ? q + n2 : (q >= n2 ? q - n2 : q);
        return cmul(hi[q / kChLo], lo[q % kChLo]);
    }
};
// fills the chirp tables of length n (caller synchronises)
template <int NT>
__device__ __forceinline__ Chirp load_chirp(double2 *lo, double2 *hi, int n) {
    const int nhi = (2 * n - 1) / kChLo + 1;
    for (int t = threadIdx.x; t < kChLo + nhi; t += NT) {
        if (t < kChLo)
            lo[t] = e_pi_over(t, n);
        else
            hi[t - kChLo] = e_pi_over((t - kChLo) * kChLo, n);
    }
    return Chirp{lo, hi, n, 1.0 / (2.0 * (double)n)};
}

__device__ __forceinline__ double2 result_at(const double2 *buf, DescP d, const Chirp &ch, int k) {
    if (!d->bluestein) return buf[pd(k)];
    // X_k = conj(b_k) * conj(y_k), y = conj(second transform)
    return conj2(cmul(ch(k), buf[pd(k)]));
}

__device__ __forceinline__ double2 input_point(double2 v, DescP d, const Chirp &ch, int t) {
    return d->bluestein ? cmul(v, conj2(ch(t))) : v;
}

// The analysis input point t of a job (direct transform), read from the
// rings' pixels by the first stage: s_a(t) + i s_b(t).
struct PixelsIn {
    const double *a, *b;
    bool two;
    __device__ __forceinline__ double2 operator()(int t) const {
        const double vb = b[t];  // b = a for a single ring
        return make_double2(a[t], two ? vb : 0.0);
    }
};
// The synthesis output point t of a job (direct transform), written to the
// rings' pixels by the last stage: z = FFT(conj g)_t, s_a(t) = Re z,
// s_b(t) = -Im z.
struct PixelsOut {
    double *a, *b;
    bool two;
    __device__ __forceinline__ void operator()(int t, double2 v) const {
        a[t] = v.x;
        if (two) b[t] = -v.y;
    }
};

// ---------------------------------------------------------------- ring jobs
// A job is one ring or two rings of the same length n, transformed together
// as the real and imaginary parts of one complex sequence.
//
// Synthesis of a job (a, b): per ring, the folded and phased spectrum c is
// made Hermitian, h_k = (c_k + conj c_{-k}) / 2, so that its inverse DFT is the
// real ring; g = h_a + i h_b, z = IDFT(g) = conj(FFT(conj g)), and
// s_a = Re z, s_b = Im z.  Analysis: z = s_a + i s_b, Z = FFT(z),
// S_a,k = (Z_k + conj Z_{-k}) / 2, S_b,k = (Z_k - conj Z_{-k}) / (2i).

// w_m Delta_m e^{i m phi0} (w_0 = 1, real part only; w_m = 2)
__device__ __forceinline__ double2 bin_term(double2 dv, int m, const Phase &ph) {
    if (m == 0) return make_double2(dv.x, 0.0);
    const double2 e = ph(m);
    return make_double2(2.0 * fma(dv.x, e.x, -dv.y * e.y), 2.0 * fma(dv.x, e.y, dv.y * e.x));
}

// c_k of one ring: sum over m = k mod n (m <= mmax) of w_m Delta_m e^{i m phi0},
// in increasing m, given the term of m = k (first, zero if k > mmax)
__device__ __forceinline__ double2 fold_bin(double2 first, const double2 *__restrict__ D, int64_t sm, int k, int n,
                                            int mmax, const Phase &ph) {
    double cr = first.x, ci = first.y;
    for (int m = k + n; m <= mmax; m += n) {
        const double2 t = bin_term(D[m * sm], m, ph);
        cr += t.x;
        ci += t.y;
    }
    return make_double2(cr, ci);
}

// phased terms of one ring for m = tid, tid+NT, ...: w_m Delta_m e^{i m phi0}
template <int NT>
__device__ __forceinline__ void phased_terms(const double2 *__restrict__ D, int64_t sm, int mmax, const Phase &ph,
                                             double2 *__restrict__ out) {
    for (int m = threadIdx.x; m <= mmax; m += NT) {
        const double2 dv = D[m * sm];
        if (m == 0) {
            out[0] = make_double2(dv.x, 0.0);
        } else {
            const double2 e = ph(m);
            out[m] = make_double2(2.0 * fma(dv.x, e.x, -dv.y * e.y), 2.0 * fma(dv.x, e.y, dv.y * e.x));
        }
    }
}

// sum_{m = k mod n, m <= lim} t_m, in increasing m
__device__ __forceinline__ double2 fold_terms(const double2 *__restrict__ t, int k, int n, int lim) {
    double cr = 0.0, ci = 0.0;
    for (int m = k; m <= lim; m += n) {
        cr += t[m].x;
        ci += t[m].y;
    }
    return make_double2(cr, ci);
}

// In-place column sums for a short ring (n <= NT): with S = n * floor(NT / n),
// thread u < S replaces t_u by sum_{j >= 0} t_{u + jS}.  As S is a multiple of
// n, the bin sum c_k is then sum_{i < S/n} t_{k + in}: two short sums instead
// of one of (mmax+1)/n terms.  Only thread u reads t_u for u < S, so the
// update needs no extra buffer.  Returns the last index to fold.
template <int NT>
__device__ __forceinline__ int fold_columns(double2 *__restrict__ t, int n, int mmax) {
    const int S = n * (NT / n);
    const int u = threadIdx.x;
    if (u < S && u <= mmax) {
        double cr = 0.0, ci = 0.0;
        for (int m = u; m <= mmax; m += S) {
            cr += t[m].x;
            ci += t[m].y;
        }
        t[u] = make_double2(cr, ci);
    }
    return min(S - 1, mmax);
}

// The two real sequences a workgroup transforms as one complex sequence:
// ring ra of map ma and ring rb of map mb (rings of equal length).
struct JobSeqs {
    int ra, rb, ma, mb;
    bool two;  // false: only sequence a
};
// Workgroup -> sequences.  Ring-major Delta: a job (a mirror pair or two
// rings of equal length) of one map, the maps of one job in consecutive
// workgroups (they share the job's tables through L2).  Map-minor Delta: one
// ring of two adjacent maps, whose Delta entries are adjacent (32 bytes per m);
// units of (job, ring of the job, 8 maps), whose entries share 128-byte lines,
// go to the XCDs in turn (workgroup b runs on XCD b mod 8) and a unit's 4
// workgroups run back to back on its XCD, so that each line is fetched (or
// completed) once in that XCD's L2.  Returns false for the padding of the
// grid and for the missing second ring of a single-ring job (whole workgroups).
__device__ __forceinline__ bool job_seqs(int njobs, int nmaps, int map_minor, const int2 *__restrict__ jobs,
                                         JobSeqs &js) {
    if (!map_minor) {
        const int2 job = jobs[blockIdx.x / nmaps];
        const int mp = blockIdx.x % nmaps;
        js = JobSeqs{job.x, job.y >= 0 ? job.y : job.x, mp, mp, job.y >= 0};
        return true;
    }
    const int groups = (nmaps + 7) / 8;
    const int x = blockIdx.x % 8, k = blockIdx.x / 8;
    const int unit = (k / 4) * 8 + x;
    const int ji = unit / (2 * groups), rem = unit % (2 * groups);
    const int ma = (rem % groups) * 8 + 2 * (k % 4);
    if (ji >= njobs || ma >= nmaps) return false;
    const int2 job = jobs[ji];
    const int r = rem / groups ? job.y : job.x;
    if (r < 0) return false;
    js = JobSeqs{r, r, ma, ma + 1 < nmaps ? ma + 1 : ma, ma + 1 < nmaps};
    return true;
}
// The plan entry and sequences of this workgroup.  BATCH: workgroup b takes
// entry bjobs[b] = (plan, job) of a batch table (one map; the entry is read
// with scalar loads); otherwise the kernel argument's plan, with the grid over
// its jobs and maps as job_seqs.  False: nothing to do.
template <bool BATCH>
__device__ __forceinline__ bool ring_task(const RingPlan &one, const RingPlan *plans, const int2 *bjobs,
                                          RingPlan &P, JobSeqs &js) {
    if constexpr (BATCH) {
        const const_ptr<int> bj = ro(reinterpret_cast<const int *>(bjobs)) + 2 * (int64_t)blockIdx.x;
        const const_ptr<RingPlan> q = ro(plans) + bj[0];
        P.mmax = q->mmax;
        P.nmaps = 1;
        P.njobs = q->njobs;
        P.fold_rows = q->fold_rows;
        P.ph_tab = q->ph_tab;
        P.npix = q->npix;
        P.dl.s_map = q->dl.s_map;
        P.dl.s_ring = q->dl.s_ring;
        P.dl.s_m = q->dl.s_m;
        P.dl.map_minor = 0;
        P.jobs = q->jobs;
        P.ring_desc = q->ring_desc;
        P.descs = q->descs;
        P.phi0 = q->phi0;
        P.weight = q->weight;
        P.ofs = q->ofs;
        P.din = q->din;
        P.mout = q->mout;
        P.min = q->min;
        P.dout = q->dout;
        const const_ptr<int> job = ro(reinterpret_cast<const int *>(P.jobs)) + 2 * (int64_t)bj[1];
        const int a = job[0], b = job[1];
        js = JobSeqs{a, b >= 0 ? b : a, 0, 0, b >= 0};
        return true;
    } else {
        P = one;
        return job_seqs(P.njobs, P.nmaps, P.dl.map_minor, P.jobs, js);
    }
}
// workgroups of one class launch: njobs * nmaps, or for map-minor Delta 32 per
// 8 units of (job, ring of the job, 8 maps)
inline int64_t fft_grid(int njobs, int nmaps, int map_minor) {
    if (!map_minor) return (int64_t)njobs * nmaps;
    const int64_t units = (int64_t)njobs * 2 * ((nmaps + 7) / 8);
    return (units + 7) / 8 * 32;
}

// Synthesis.  LDS: the twiddle tables, buf[L], plus (fold_rows != 0) two
// rows of mmax+1 phased terms used when the ring folds many m per bin,
// n < (mmax+1)/2.
template <int MAXL, int NT, bool BATCH>
__global__ __launch_bounds__(NT, 4) void k_fft_syn(RingPlan one, const RingPlan *__restrict__ plans,
                                                   const int2 *__restrict__ bjobs) {
    extern __shared__ double2 lds[];
    double2 *tlo = lds, *thi = lds + kTwLo, *clo = lds + tw_entries<MAXL>(), *chi = clo + kChLo;
    double2 *buf = clo + chirp_entries<MAXL>();
    RingPlan P;
    JobSeqs js;
    if (!ring_task<BATCH>(one, plans, bjobs, P, js)) return;  // whole workgroup
    const int mmax = P.mmax, fold_rows = P.fold_rows;
    const DeltaLayout dl = P.dl;
    const bool two = js.two;
    const DescP d = ro(P.descs) + P.ring_desc[js.ra];
    const int N = d->n, L = d->L;
    const double2 *__restrict__ Da = P.din + js.ma * dl.s_map + js.ra * dl.s_ring;
    const double2 *__restrict__ Db = P.din + js.mb * dl.s_map + js.rb * dl.s_ring;
    const bool lds_fold = fold_rows && (2 * N < mmax + 1);
    const double2 z = make_double2(0.0, 0.0);
    // Delta at m = k of every bin k = threadIdx.x + u NT of this thread (both
    // rings): all in flight while the tables are set up
    constexpr int U = MAXL / (2 * NT);
    double2 fa[U + 1], fb[U + 1];
#pragma unroll
    for (int u = 0; u <= U; ++u) {
        const int k = threadIdx.x + u * NT;
        const bool ok = !lds_fold && 2 * k <= N && k <= mmax;
        fa[u] = ok ? Da[k * dl.s_m] : z;
        fb[u] = (ok && two) ? Db[k * dl.s_m] : z;
    }
    load_twiddles<NT>(tlo, thi, d->tw, L);
    const bool blue = d->bluestein != 0;
    Chirp ch{clo, chi, N, 0.0};
    if (blue) ch = load_chirp<NT>(clo, chi, N);
    const double pa = P.phi0[js.ra], pb = P.phi0[js.rb];
    Phase pha{nullptr, nullptr, pa}, phb{nullptr, nullptr, pb};
    if (P.ph_tab) {
        double2 *tab = buf + padded_len<MAXL>() + (fold_rows ? 2 * (mmax + 1) : 0);
        pha = load_phases<NT>(tab, mmax, pa);
        phb = pha;
        if (two && js.rb != js.ra) phb = load_phases<NT>(tab + kPhLo + phase_hi_entries(mmax), mmax, pb);
    }
    if (P.ph_tab || blue) __syncthreads();  // phase and chirp tables visible
    int lim = mmax;  // last index of the phased-term rows that the bins fold
    if (lds_fold) {
        // all threads evaluate phases; short rings first sum the rows in columns
        double2 *ta = buf + pd(L), *tb = buf + pd(L) + (mmax + 1);
        phased_terms<NT>(Da, dl.s_m, mmax, pha, ta);
        if (two) phased_terms<NT>(Db, dl.s_m, mmax, phb, tb);
        __syncthreads();
        if (N <= NT) {
            lim = fold_columns<NT>(ta, N, mmax);
            if (two) fold_columns<NT>(tb, N, mmax);
            __syncthreads();
        }
    }
    // thread handles the bin pairs (k, n-k), k = threadIdx.x + u NT <= n/2:
    // u < U for every thread, and k = U NT (only when n = MAXL) by thread 0
    auto put = [&](int k, double2 a0, double2 a1, double2 b0, double2 b1) {
        const int kn = k ? N - k : 0;  // (n - k) mod n, k < n
        // h_k = (c_k + conj c_{n-k}) / 2, h_{n-k} = conj h_k
        const double2 ha = make_double2(0.5 * (a0.x + a1.x), 0.5 * (a0.y - a1.y));
        const double2 hb = make_double2(0.5 * (b0.x + b1.x), 0.5 * (b0.y - b1.y));
        // g = h_a + i h_b; the transform input is conj(g)
        const double2 gk = make_double2(ha.x - hb.y, ha.y + hb.x);
        const double2 gn = make_double2(ha.x + hb.y, -ha.y + hb.x);  // h_a* + i h_b* at n-k
        buf[pd(k)] = input_point(conj2(gk), d, ch, k);
        if (kn != k) buf[pd(kn)] = input_point(conj2(gn), d, ch, kn);
    };
    // the four folded bins of one k: c_a(k), c_a(n-k), c_b(k), c_b(n-k)
    auto bins = [&](int k, double2 &a0, double2 &a1, double2 &b0, double2 &b1) {
        const int kn = k ? N - k : 0;  // (n - k) mod n, k < n
        if (lds_fold) {
            const double2 *ta = buf + pd(L), *tb = buf + pd(L) + (mmax + 1);
            a0 = fold_terms(ta, k, N, lim);
            a1 = fold_terms(ta, kn, N, lim);
            b0 = two ? fold_terms(tb, k, N, lim) : z;
            b1 = two ? fold_terms(tb, kn, N, lim) : z;
        } else {
            // a0..b1 hold the first Delta of each bin (m = k, m = n-k) on entry
            a0 = fold_bin(k <= mmax ? bin_term(a0, k, pha) : z, Da, dl.s_m, k, N, mmax, pha);
            a1 = fold_bin(kn <= mmax ? bin_term(a1, kn, pha) : z, Da, dl.s_m, kn, N, mmax, pha);
            b0 = two ? fold_bin(k <= mmax ? bin_term(b0, k, phb) : z, Db, dl.s_m, k, N, mmax, phb) : z;
            b1 = two ? fold_bin(kn <= mmax ? bin_term(b1, kn, phb) : z, Db, dl.s_m, kn, N, mmax, phb) : z;
        }
    };
    // bins k = threadIdx.x + u NT, u = 0 .. U (k = U NT only for thread 0 when
    // n = MAXL); the second Delta of a bin pair (m = n - k) exists only for
    // rings shorter than 2 mmax + 1, and aliases m + n <= mmax are loaded by
    // the fold
#pragma unroll
    for (int u = 0; u <= U; ++u) {
        const int k = threadIdx.x + u * NT;
        const int kn = k ? N - k : 0;  // (n - k) mod n, k < n
        const bool ok = !lds_fold && 2 * k <= N && kn <= mmax;
        double2 a0 = fa[u], b0 = fb[u];
        double2 a1 = ok ? Da[kn * dl.s_m] : z;
        double2 b1 = (ok && two) ? Db[kn * dl.s_m] : z;
        if (2 * k <= N) {
            bins(k, a0, a1, b0, b1);
            put(k, a0, a1, b0, b1);
        }
    }
    __syncthreads();
    double *outa = P.mout + (int64_t)js.ma * P.npix + P.ofs[js.ra];
    double *outb = P.mout + (int64_t)js.mb * P.npix + P.ofs[js.rb];
    // the last stage writes the pixels when it can (radix 4 or 8)
    const bool reg_out = reg_last(d);
    transform<MAXL, NT, LdsIn, PixelsOut>(buf, d, TwLds{tlo, thi}, LdsIn{buf}, false,
                                          PixelsOut{outa, outb, two}, true);
    if (reg_out) return;
    for (int j = threadIdx.x; j < N; j += NT) {
        const double2 z = result_at(buf, d, ch, j);  // FFT(conj g)_j; IDFT(g)_j = conj of it
        outa[j] = z.x;
        if (two) outb[j] = -z.y;
    }
}

template <int MAXL, int NT, bool BATCH>
__global__ __launch_bounds__(NT, 4) void k_fft_ana(RingPlan one, const RingPlan *__restrict__ plans,
                                                   const int2 *__restrict__ bjobs) {
    extern __shared__ double2 lds[];
    double2 *tlo = lds, *thi = lds + kTwLo, *clo = lds + tw_entries<MAXL>(), *chi = clo + kChLo;
    double2 *buf = clo + chirp_entries<MAXL>();
    RingPlan P;
    JobSeqs js;
    if (!ring_task<BATCH>(one, plans, bjobs, P, js)) return;  // whole workgroup
    const int mmax = P.mmax;
    const DeltaLayout dl = P.dl;
    const bool two = js.two;
    const DescP d = ro(P.descs) + P.ring_desc[js.ra];
    const int N = d->n;
    load_twiddles<NT>(tlo, thi, d->tw, d->L);
    Chirp ch{clo, chi, N, 0.0};
    if (d->bluestein) {
        ch = load_chirp<NT>(clo, chi, N);
        __syncthreads();  // the input points below take the chirp
    }
    const double pa = P.phi0[js.ra], wa = P.weight[js.ra];
    const double pb = P.phi0[js.rb], wb = P.weight[js.rb];
    // phase tables: visible after the barrier that follows the input below
    Phase pha{nullptr, nullptr, pa}, phb{nullptr, nullptr, pb};
    if (P.ph_tab) {
        double2 *tab = buf + padded_len<MAXL>();
        pha = load_phases<NT>(tab, mmax, pa);
        phb = pha;
        if (two && js.rb != js.ra) phb = load_phases<NT>(tab + kPhLo + phase_hi_entries(mmax), mmax, pb);
    }
    const double *ina = P.min + (int64_t)js.ma * P.npix + P.ofs[js.ra];
    const double *inb = P.min + (int64_t)js.mb * P.npix + P.ofs[js.rb];
    // the first stage reads the pixels when it can (radix 4 or 8)
    const bool reg_in = reg_first(d);
    if (!reg_in) {
        // every pixel of this thread is loaded before any is used (N <= MAXL)
        constexpr int U = MAXL / NT;
        double va[U], vb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = threadIdx.x + u * NT;
            va[u] = j < N ? ina[j] : 0.0;
            vb[u] = (two && j < N) ? inb[j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = threadIdx.x + u * NT;
            if (j < N) buf[pd(j)] = input_point(make_double2(va[u], vb[u]), d, ch, j);
        }
    }
    __syncthreads();  // twiddle and phase tables (and the points) visible
    transform<MAXL, NT, PixelsIn>(buf, d, TwLds{tlo, thi}, PixelsIn{ina, inb, two}, true);
    double2 *Da = P.dout + js.ma * dl.s_map + js.ra * dl.s_ring;
    double2 *Db = P.dout + js.mb * dl.s_map + js.rb * dl.s_ring;
    for (int m = threadIdx.x; m <= mmax; m += NT) {
        const int k = m < N ? m : m % N, kn = k ? N - k : 0;  // m mod n, (n - k) mod n
        const double2 Z = result_at(buf, d, ch, k), Zn = result_at(buf, d, ch, kn);
        // S_a = (Z_k + conj Z_{n-k}) / 2, S_b = (Z_k - conj Z_{n-k}) / (2i)
        const double2 Sa = make_double2(0.5 * (Z.x + Zn.x), 0.5 * (Z.y - Zn.y));
        const double2 Sb = make_double2(0.5 * (Z.y + Zn.y), -0.5 * (Z.x - Zn.x));
        const double2 ea = pha(m);
        // w * conj(e) * S
        Da[m * dl.s_m] = make_double2(wa * fma(Sa.x, ea.x, Sa.y * ea.y), wa * fma(Sa.y, ea.x, -Sa.x * ea.y));
        if (two) {
            const double2 eb = phb(m);
            Db[m * dl.s_m] = make_double2(wb * fma(Sb.x, eb.x, Sb.y * eb.y), wb * fma(Sb.y, eb.x, -Sb.x * eb.y));
        }
    }
}

// threads per workgroup for each length class: four points per thread up to
// 2048 points, eight (one radix-8 butterfly) above, so that two 4096-point
// workgroups fit a CU's registers
template <int MAXL>
constexpr int fft_threads() { return MAXL <= 2048 ? MAXL / 4 : MAXL / 8; }

constexpr int kMaxLds = 160 * 1024;  // LDS bytes per workgroup on gfx950

template <int MAXL>
int allow_max_lds() {
    constexpr int NT = fft_threads<MAXL>();
    const void *fns[] = {reinterpret_cast<const void *>(&k_fft_syn<MAXL, NT, false>),
                         reinterpret_cast<const void *>(&k_fft_ana<MAXL, NT, false>),
                         reinterpret_cast<const void *>(&k_fft_syn<MAXL, NT, true>),
                         reinterpret_cast<const void *>(&k_fft_ana<MAXL, NT, true>)};
    for (const void *f : fns) SHT_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLds));
    return SHT_OK;
}

// every class may use up to the whole LDS (the 4096 class needs more than the
// 64 KB default: twiddle tables plus 4096 points); set once per device
int set_lds_attr() {
    static std::mutex mu;
    static uint64_t done = 0;  // bit d: device d
    int dev = 0;
    SHT_HIP(hipGetDevice(&dev));
    const uint64_t bit = dev < 64 ? (uint64_t)1 << dev : 0;
    std::lock_guard<std::mutex> lk(mu);
    if (bit && (done & bit)) return SHT_OK;
    int rc;
    if ((rc = allow_max_lds<1024>()) || (rc = allow_max_lds<2048>()) || (rc = allow_max_lds<4096>()) ||
        (rc = allow_max_lds<8192>()))
        return rc;
    done |= bit;
    return SHT_OK;
}

static_assert((tw_entries<kMaxFftLen>() + chirp_entries<kMaxFftLen>() + padded_len<kMaxFftLen>()) * sizeof(double2) <= kMaxLds,
              "largest class fits LDS");

// the phase tables of a job's two rings; used for mmax < 64 kPhHiMax when
// they fit next to the other LDS data
size_t phase_table_bytes(int mmax) { return 2 * (size_t)(kPhLo + phase_hi_entries(mmax)) * sizeof(double2); }
int phase_tables_fit(int mmax, size_t lds) {
    return phase_hi_entries(mmax) <= kPhHiMax && lds + phase_table_bytes(mmax) <= (size_t)kMaxLds;
}

// LDS bytes and layout flags of class MAXL for a plan of this mmax
template <int MAXL>
size_t class_lds(int mmax, bool synthesis, int *fold_rows, int *ph_tab) {
    const size_t base = (size_t)(tw_entries<MAXL>() + chirp_entries<MAXL>() + padded_len<MAXL>()) * sizeof(double2);
    const size_t rows = 2 * (size_t)(mmax + 1) * sizeof(double2);
    // the small-length class of synthesis keeps the phased terms in LDS when they fit
    *fold_rows = (synthesis && MAXL <= 1024 && base + rows <= kMaxLds) ? 1 : 0;
    size_t lds = base + (*fold_rows ? rows : 0);
    *ph_tab = phase_tables_fit(mmax, lds);
    if (*ph_tab) lds += phase_table_bytes(mmax);
    return lds;
}

template <int MAXL>
void launch_class(const RingPlan &P, int64_t grid, size_t lds, bool synthesis, const RingPlan *plans,
                  const int2 *bjobs, hipStream_t st) {
    constexpr int NT = fft_threads<MAXL>();
    if (plans && synthesis)
        hipLaunchKernelGGL((k_fft_syn<MAXL, NT, true>), dim3((unsigned)grid), dim3(NT), lds, st, P, plans, bjobs);
    else if (plans)
        hipLaunchKernelGGL((k_fft_ana<MAXL, NT, true>), dim3((unsigned)grid), dim3(NT), lds, st, P, plans, bjobs);
    else if (synthesis)
        hipLaunchKernelGGL((k_fft_syn<MAXL, NT, false>), dim3((unsigned)grid), dim3(NT), lds, st, P, plans, bjobs);
    else
        hipLaunchKernelGGL((k_fft_ana<MAXL, NT, false>), dim3((unsigned)grid), dim3(NT), lds, st, P, plans, bjobs);
}
void launch_class_any(int c, const RingPlan &P, int64_t grid, size_t lds, bool synthesis, const RingPlan *plans,
                      const int2 *bjobs, hipStream_t st) {
    switch (c) {
        case 0: launch_class<1024>(P, grid, lds, synthesis, plans, bjobs, st); break;
        case 1: launch_class<2048>(P, grid, lds, synthesis, plans, bjobs, st); break;
        case 2: launch_class<4096>(P, grid, lds, synthesis, plans, bjobs, st); break;
        default: launch_class<8192>(P, grid, lds, synthesis, plans, bjobs, st); break;
    }
}

static_assert(kFftClasses == 4 && kFftClassLen[0] == 1024 && kFftClassLen[3] == kMaxFftLen,
              "launch table below follows kFftClassLen");

}  // namespace

// one workgroup per (job, map) of a class
static bool grid_fits(const GeomPlan &p, int nmaps, int map_minor) {
    for (int c = 0; c < kFftClasses; ++c)
        if (fft_grid(p.class_count[c], nmaps, map_minor) >= (int64_t)INT32_MAX) return false;
    return true;
}

RingPlan ring_plan(const GeomPlan &p, int c, int mmax, int nmaps, DeltaLayout dl, bool synthesis, size_t *lds) {
    RingPlan P{};
    P.mmax = mmax;
    P.nmaps = nmaps;
    P.njobs = p.class_count[c];
    P.npix = p.npix;
    P.dl = dl;
    P.jobs = p.class_jobs[c];
    P.ring_desc = p.ring_desc;
    P.descs = p.descs;
    P.phi0 = p.phi0;
    P.weight = p.weight;
    P.ofs = p.ofs;
    switch (c) {
        case 0: *lds = class_lds<1024>(mmax, synthesis, &P.fold_rows, &P.ph_tab); break;
        case 1: *lds = class_lds<2048>(mmax, synthesis, &P.fold_rows, &P.ph_tab); break;
        case 2: *lds = class_lds<4096>(mmax, synthesis, &P.fold_rows, &P.ph_tab); break;
        default: *lds = class_lds<8192>(mmax, synthesis, &P.fold_rows, &P.ph_tab); break;
    }
    return P;
}

// Runs launch(i, stream) for the n classes: concurrently through fork_join
// (the largest on the caller's stream, the others on side streams), or one
// after another on st.
static int each_class(hipStream_t st, int n, bool fork, const std::function<int(int, hipStream_t)> &launch) {
    if (fork) return fork_join(st, n, launch);
    int rc = SHT_OK;
    for (int i = 0; i < n && rc == SHT_OK; ++i) rc = launch(i, st);
    return rc;
}

static int launch_fft(const GeomPlan &p, int mmax, const void *din, double *mout, const double *min, void *dout,
                      DeltaLayout dl, int nmaps, bool synthesis, hipStream_t st, bool fork) {
    if (nmaps > 65535 || !grid_fits(p, nmaps, dl.map_minor)) return SHT_EUNSUPPORTED;
    if (!synthesis && !p.weight) return SHT_EINVAL;
    int rc = set_lds_attr();
    if (rc) return rc;
    int cls[kFftClasses], n = 0;
    for (int c = kFftClasses - 1; c >= 0; --c)
        if (p.class_count[c]) cls[n++] = c;
    return each_class(st, n, fork, [&](int i, hipStream_t s) {
        const int c = cls[i];
        size_t lds = 0;
        RingPlan P = ring_plan(p, c, mmax, nmaps, dl, synthesis, &lds);
        P.din = static_cast<const double2 *>(din);
        P.mout = mout;
        P.min = min;
        P.dout = static_cast<double2 *>(dout);
        launch_class_any(c, P, fft_grid(P.njobs, nmaps, dl.map_minor), lds, synthesis, nullptr, nullptr, s);
        SHT_HIP(hipGetLastError());
        return SHT_OK;
    });
}

int launch_fft_syn(const GeomPlan &p, int mmax, const void *delta, DeltaLayout dl, double *map, int nmaps,
                   hipStream_t st, bool fork) {
    return launch_fft(p, mmax, delta, map, nullptr, nullptr, dl, nmaps, true, st, fork);
}

int launch_fft_ana(const GeomPlan &p, int mmax, const double *map, void *delta, DeltaLayout dl, int nmaps,
                   hipStream_t st, bool fork) {
    return launch_fft(p, mmax, nullptr, nullptr, map, delta, dl, nmaps, false, st, fork);
}

static int launch_batch(const RingBatch &b, bool synthesis, hipStream_t st) {
    int rc = set_lds_attr();
    if (rc) return rc;
    for (int c = kFftClasses - 1; c >= 0; --c) {
        if (!b.njobs[c]) continue;
        launch_class_any(c, RingPlan{}, b.njobs[c], b.lds[c], synthesis, b.plans, b.jobs[c], st);
        SHT_HIP(hipGetLastError());
    }
    return SHT_OK;
}
int launch_fft_syn_batch(const RingBatch &b, hipStream_t st) { return launch_batch(b, true, st); }
int launch_fft_ana_batch(const RingBatch &b, hipStream_t st) { return launch_batch(b, false, st); }

}  // namespace sht
