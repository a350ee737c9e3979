// Ring Fourier stage for gfx950: one workgroup per ring (and map), the
// ring's transform held in LDS.  Rings are launched in classes of transform
// length (<= 1024, 2048, 4096, 8192 points) so that LDS and the per-thread
// register arrays are sized for the class, with about four points per thread.
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
// length (4, 2, 3, 5); each stage reads its butterflies into registers,
// synchronises, and writes them back.  Lengths with a larger prime factor use
// Bluestein's chirp-z identity
//   X_k = conj(b_k) sum_n (x_n conj(b_n)) b_{k-n},  b_t = e^{i pi t^2/N},
// as a cyclic convolution of 5-smooth length L >= 2N-1 done with two forward
// transforms (the filter spectrum, scaled by 1/L, is a plan table).
#include "sht_internal.h"

namespace sht {
namespace {

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

// Forward-sign butterflies of radix 2, 3, 4, 5 in registers, with the roots
// of unity as constants: cos(2pi/5) = (sqrt5-1)/4, cos(4pi/5) = -(sqrt5+1)/4,
// sin(2pi/5), sin(4pi/5) and sqrt(3)/2, each rounded to double.
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

// One Stockham stage of radix R on buf[0..L), L <= MAXL, Ns = product of
// earlier radices.  Each thread holds up to kMaxB twiddled butterflies in
// registers (NT threads) and writes them back after the barrier.
template <int R, int MAXL, int NT>
__device__ void fft_stage(double2 *buf, int L, int Ns, const double2 *__restrict__ tw) {
    constexpr int kMaxB = (MAXL / R + NT - 1) / NT;
    const int nbf = L / R;
    const int tstep = L / (Ns * R);
    double2 v[kMaxB][R];
#pragma unroll
    for (int b = 0; b < kMaxB; ++b) {
        const int j = threadIdx.x + b * NT;
        if (j < nbf) {
            const int k = j % Ns;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double2 xv = buf[j + r * nbf];
                v[b][r] = (r == 0) ? xv : cmul(xv, tw[r * k * tstep]);
            }
            butterfly<R>(v[b]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < kMaxB; ++b) {
        const int j = threadIdx.x + b * NT;
        if (j < nbf) {
            const int k = j % Ns;
            const int o = (j / Ns) * Ns * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[o + r * Ns] = v[b][r];
        }
    }
    __syncthreads();
}

// Forward FFT of length d->L (<= MAXL) in LDS (natural order in and out).
template <int MAXL, int NT>
__device__ void fft_forward(double2 *buf, const FftDesc *__restrict__ d) {
    const int L = d->L, nrad = d->nrad;
    const double2 *tw = d->tw;
    int Ns = 1;
    for (int s = 0; s < nrad; ++s) {
        const int R = d->rad[s];
        switch (R) {
            case 4: fft_stage<4, MAXL, NT>(buf, L, Ns, tw); break;
            case 2: fft_stage<2, MAXL, NT>(buf, L, Ns, tw); break;
            case 3: fft_stage<3, MAXL, NT>(buf, L, Ns, tw); break;
            default: fft_stage<5, MAXL, NT>(buf, L, Ns, tw); break;
        }
        Ns *= R;
    }
}

// DFT of the n points already placed in buf[0..n) (pre-multiplied by
// conj(chirp) when Bluestein): afterwards X_k is at_k(buf, d, k).
template <int MAXL, int NT>
__device__ void transform(double2 *buf, const FftDesc *__restrict__ d) {
    if (!d->bluestein) {
        fft_forward<MAXL, NT>(buf, d);
        return;
    }
    const int L = d->L;
    const double2 *kern = d->kern;
    for (int t = d->n + threadIdx.x; t < L; t += NT) buf[t] = make_double2(0.0, 0.0);
    __syncthreads();
    fft_forward<MAXL, NT>(buf, d);
    for (int t = threadIdx.x; t < L; t += NT) buf[t] = conj2(cmul(buf[t], kern[t]));
    __syncthreads();
    fft_forward<MAXL, NT>(buf, d);
}

__device__ __forceinline__ double2 result_at(const double2 *buf, const FftDesc *__restrict__ d, int k) {
    if (!d->bluestein) return buf[k];
    // X_k = conj(b_k) * conj(y_k), y = conj(second transform)
    return conj2(cmul(d->chirp[k], buf[k]));
}

__device__ __forceinline__ double2 input_point(double2 v, const FftDesc *__restrict__ d, int t) {
    return d->bluestein ? cmul(v, conj2(d->chirp[t])) : v;
}

template <int MAXL, int NT>
__global__ __launch_bounds__(NT) void k_fft_syn(int mmax, int nrings, int64_t npix,
                                                    const int32_t *__restrict__ rings,
                                                    const int32_t *__restrict__ ring_desc,
                                                    const FftDesc *__restrict__ descs,
                                                    const double *__restrict__ phi0,
                                                    const int64_t *__restrict__ ofs,
                                                    const double2 *__restrict__ delta,
                                                    double *__restrict__ map) {
    extern __shared__ double2 buf[];
    const int r = rings[blockIdx.x];
    const int mp = blockIdx.y;
    const FftDesc *d = descs + ring_desc[r];
    const int N = d->n;
    const double ph0 = phi0[r];
    const double2 *__restrict__ D = delta + ((int64_t)mp * nrings + r) * (mmax + 1);
    for (int k = threadIdx.x; k < N; k += NT) {
        double cr = 0.0, ci = 0.0;
        for (int m = k; m <= mmax; m += N) {
            const double2 dv = D[m];
            if (m == 0) {
                cr += dv.x;
            } else {
                const double2 e = phase_exp(m, ph0);
                cr += 2.0 * fma(dv.x, e.x, -dv.y * e.y);
                ci += 2.0 * fma(dv.x, e.y, dv.y * e.x);
            }
        }
        buf[k] = input_point(make_double2(cr, -ci), d, k);
    }
    __syncthreads();
    transform<MAXL, NT>(buf, d);
    double *out = map + (int64_t)mp * npix + ofs[r];
    for (int j = threadIdx.x; j < N; j += NT) out[j] = result_at(buf, d, j).x;
}

template <int MAXL, int NT>
__global__ __launch_bounds__(NT) void k_fft_ana(int mmax, int nrings, int64_t npix,
                                                    const int32_t *__restrict__ rings,
                                                    const int32_t *__restrict__ ring_desc,
                                                    const FftDesc *__restrict__ descs,
                                                    const double *__restrict__ phi0,
                                                    const double *__restrict__ weight,
                                                    const int64_t *__restrict__ ofs,
                                                    const double *__restrict__ map,
                                                    double2 *__restrict__ delta) {
    extern __shared__ double2 buf[];
    const int r = rings[blockIdx.x];
    const int mp = blockIdx.y;
    const FftDesc *d = descs + ring_desc[r];
    const int N = d->n;
    const double *in = map + (int64_t)mp * npix + ofs[r];
    for (int j = threadIdx.x; j < N; j += NT) buf[j] = input_point(make_double2(in[j], 0.0), d, j);
    __syncthreads();
    transform<MAXL, NT>(buf, d);
    const double ph0 = phi0[r], w = weight[r];
    double2 *D = delta + ((int64_t)mp * nrings + r) * (mmax + 1);
    for (int m = threadIdx.x; m <= mmax; m += NT) {
        const double2 X = result_at(buf, d, m % N);
        const double2 e = phase_exp(m, ph0);
        // w * conj(e) * X
        D[m] = make_double2(w * fma(X.x, e.x, X.y * e.y), w * fma(X.y, e.x, -X.x * e.y));
    }
}

// threads per workgroup for each length class: about four points per thread
template <int MAXL>
constexpr int fft_threads() { return MAXL / 4 < 1024 ? MAXL / 4 : 1024; }

bool g_attr_set = false;

int set_lds_attr() {
    if (g_attr_set) return SHT_OK;
    const int bytes = kMaxFftLen * (int)sizeof(double2);
    SHT_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft_syn<8192, fft_threads<8192>()>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    SHT_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft_ana<8192, fft_threads<8192>()>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    g_attr_set = true;
    return SHT_OK;
}

template <int MAXL>
void launch_syn_class(const GeomPlan &p, int c, int mmax, const void *delta, double *map, int nmaps,
                      hipStream_t st) {
    constexpr int NT = fft_threads<MAXL>();
    const size_t lds = (size_t)std::min(MAXL, p.max_L) * sizeof(double2);
    hipLaunchKernelGGL((k_fft_syn<MAXL, NT>), dim3((unsigned)p.class_count[c], (unsigned)nmaps), dim3(NT), lds,
                       st, mmax, p.nrings, p.npix, p.class_rings[c], p.ring_desc, p.descs, p.phi0, p.ofs,
                       static_cast<const double2 *>(delta), map);
}

template <int MAXL>
void launch_ana_class(const GeomPlan &p, int c, int mmax, const double *map, void *delta, int nmaps,
                      hipStream_t st) {
    constexpr int NT = fft_threads<MAXL>();
    const size_t lds = (size_t)std::min(MAXL, p.max_L) * sizeof(double2);
    hipLaunchKernelGGL((k_fft_ana<MAXL, NT>), dim3((unsigned)p.class_count[c], (unsigned)nmaps), dim3(NT), lds,
                       st, mmax, p.nrings, p.npix, p.class_rings[c], p.ring_desc, p.descs, p.phi0, p.weight,
                       p.ofs, map, static_cast<double2 *>(delta));
}

static_assert(kFftClasses == 4 && kFftClassLen[0] == 1024 && kFftClassLen[3] == kMaxFftLen,
              "launch table below follows kFftClassLen");

}  // namespace

int launch_fft_syn(const GeomPlan &p, int mmax, const void *delta, double *map, int nmaps, hipStream_t st) {
    if (nmaps > 65535) return SHT_EUNSUPPORTED;
    int rc = set_lds_attr();
    if (rc) return rc;
    if (p.class_count[0]) launch_syn_class<1024>(p, 0, mmax, delta, map, nmaps, st);
    if (p.class_count[1]) launch_syn_class<2048>(p, 1, mmax, delta, map, nmaps, st);
    if (p.class_count[2]) launch_syn_class<4096>(p, 2, mmax, delta, map, nmaps, st);
    if (p.class_count[3]) launch_syn_class<8192>(p, 3, mmax, delta, map, nmaps, st);
    SHT_HIP(hipGetLastError());
    return SHT_OK;
}

int launch_fft_ana(const GeomPlan &p, int mmax, const double *map, void *delta, int nmaps, hipStream_t st) {
    if (nmaps > 65535) return SHT_EUNSUPPORTED;
    if (!p.weight) return SHT_EINVAL;
    int rc = set_lds_attr();
    if (rc) return rc;
    if (p.class_count[0]) launch_ana_class<1024>(p, 0, mmax, map, delta, nmaps, st);
    if (p.class_count[1]) launch_ana_class<2048>(p, 1, mmax, map, delta, nmaps, st);
    if (p.class_count[2]) launch_ana_class<4096>(p, 2, mmax, map, delta, nmaps, st);
    if (p.class_count[3]) launch_ana_class<8192>(p, 3, mmax, map, delta, nmaps, st);
    SHT_HIP(hipGetLastError());
    return SHT_OK;
}

}  // namespace sht
