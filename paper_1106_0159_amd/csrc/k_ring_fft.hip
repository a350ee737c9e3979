// Ring Fourier stage for gfx950: one workgroup per ring (and map), the
// ring's transform held in LDS.
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
// length (4, 2, 3, 5, 7, 11, 13); each stage reads its butterflies into
// registers, synchronises, and writes them back.  Lengths with a larger
// prime factor use Bluestein's chirp-z identity
//   X_k = conj(b_k) sum_n (x_n conj(b_n)) b_{k-n},  b_t = e^{i pi t^2/N},
// as a cyclic convolution of power-of-two length L >= 2N-1 done with two
// forward transforms (the filter spectrum, scaled by 1/L, is a plan table).
#include "sht_internal.h"

namespace sht {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 conj2(double2 a) { return make_double2(a.x, -a.y); }

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
    sincos(r, &sn, &cs);
    return make_double2(cs, sn);
}

// Small DFT of size R with the forward sign, roots read from W_L.
template <int R>
__device__ __forceinline__ void dft_small(double2 (&v)[R], const double2 *__restrict__ tw, int L) {
    if constexpr (R == 2) {
        const double2 a = v[0], b = v[1];
        v[0] = make_double2(a.x + b.x, a.y + b.y);
        v[1] = make_double2(a.x - b.x, a.y - b.y);
    } else if constexpr (R == 4) {
        const double2 a = v[0], b = v[1], c = v[2], d = v[3];
        const double2 s0 = make_double2(a.x + c.x, a.y + c.y), s1 = make_double2(a.x - c.x, a.y - c.y);
        const double2 s2 = make_double2(b.x + d.x, b.y + d.y), s3 = make_double2(b.x - d.x, b.y - d.y);
        // -i * s3 = (s3.y, -s3.x)
        v[0] = make_double2(s0.x + s2.x, s0.y + s2.y);
        v[2] = make_double2(s0.x - s2.x, s0.y - s2.y);
        v[1] = make_double2(s1.x + s3.y, s1.y - s3.x);
        v[3] = make_double2(s1.x - s3.y, s1.y + s3.x);
    } else {
        double2 w[R];
#pragma unroll
        for (int t = 0; t < R; ++t) w[t] = tw[t * (L / R)];
        double2 y[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            double2 acc = v[0];
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const double2 z = cmul(v[r], w[(r * q) % R]);
                acc.x += z.x;
                acc.y += z.y;
            }
            y[q] = acc;
        }
#pragma unroll
        for (int q = 0; q < R; ++q) v[q] = y[q];
    }
}

// One Stockham stage of radix R on buf[0..L), Ns = product of earlier radices.
template <int R>
__device__ void fft_stage(double2 *buf, int L, int Ns, const double2 *__restrict__ tw) {
    constexpr int kMaxB = (kMaxFftLen / R + kBlock - 1) / kBlock;
    const int nbf = L / R;
    const int tstep = L / (Ns * R);
    double2 v[kMaxB][R];
#pragma unroll
    for (int b = 0; b < kMaxB; ++b) {
        const int j = threadIdx.x + b * kBlock;
        if (j < nbf) {
            const int k = j % Ns;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double2 xv = buf[j + r * nbf];
                v[b][r] = (r == 0) ? xv : cmul(xv, tw[r * k * tstep]);
            }
            dft_small<R>(v[b], tw, L);
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < kMaxB; ++b) {
        const int j = threadIdx.x + b * kBlock;
        if (j < nbf) {
            const int k = j % Ns;
            const int o = (j / Ns) * Ns * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[o + r * Ns] = v[b][r];
        }
    }
    __syncthreads();
}

// Forward FFT of length d.L in LDS (natural order in and out).
__device__ void fft_forward(double2 *buf, const FftDesc &d) {
    int Ns = 1;
    for (int s = 0; s < d.nrad; ++s) {
        const int R = d.rad[s];
        switch (R) {
            case 4: fft_stage<4>(buf, d.L, Ns, d.tw); break;
            case 2: fft_stage<2>(buf, d.L, Ns, d.tw); break;
            case 3: fft_stage<3>(buf, d.L, Ns, d.tw); break;
            case 5: fft_stage<5>(buf, d.L, Ns, d.tw); break;
            case 7: fft_stage<7>(buf, d.L, Ns, d.tw); break;
            case 11: fft_stage<11>(buf, d.L, Ns, d.tw); break;
            default: fft_stage<13>(buf, d.L, Ns, d.tw); break;
        }
        Ns *= R;
    }
}

// DFT of the n points already placed in buf[0..n) (pre-multiplied by
// conj(chirp) when Bluestein): afterwards X_k is at_k(buf, d, k).
__device__ void transform(double2 *buf, const FftDesc &d) {
    if (!d.bluestein) {
        fft_forward(buf, d);
        return;
    }
    for (int t = d.n + threadIdx.x; t < d.L; t += kBlock) buf[t] = make_double2(0.0, 0.0);
    __syncthreads();
    fft_forward(buf, d);
    for (int t = threadIdx.x; t < d.L; t += kBlock) buf[t] = conj2(cmul(buf[t], d.kern[t]));
    __syncthreads();
    fft_forward(buf, d);
}

__device__ __forceinline__ double2 result_at(const double2 *buf, const FftDesc &d, int k) {
    if (!d.bluestein) return buf[k];
    // X_k = conj(b_k) * conj(y_k), y = conj(second transform)
    return conj2(cmul(d.chirp[k], buf[k]));
}

__device__ __forceinline__ double2 input_point(double2 v, const FftDesc &d, int t) {
    return d.bluestein ? cmul(v, conj2(d.chirp[t])) : v;
}

__global__ __launch_bounds__(kBlock) void k_fft_syn(int mmax, int nrings, int64_t npix,
                                                    const int32_t *__restrict__ ring_desc,
                                                    const FftDesc *__restrict__ descs,
                                                    const double *__restrict__ phi0,
                                                    const int64_t *__restrict__ ofs,
                                                    const double2 *__restrict__ delta,
                                                    double *__restrict__ map) {
    extern __shared__ double2 buf[];
    const int r = blockIdx.x;
    const int mp = blockIdx.y;
    const FftDesc d = descs[ring_desc[r]];
    const int N = d.n;
    const double ph0 = phi0[r];
    const double2 *__restrict__ D = delta + ((int64_t)mp * nrings + r) * (mmax + 1);
    for (int k = threadIdx.x; k < N; k += kBlock) {
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
    transform(buf, d);
    double *out = map + (int64_t)mp * npix + ofs[r];
    for (int j = threadIdx.x; j < N; j += kBlock) out[j] = result_at(buf, d, j).x;
}

__global__ __launch_bounds__(kBlock) void k_fft_ana(int mmax, int nrings, int64_t npix,
                                                    const int32_t *__restrict__ ring_desc,
                                                    const FftDesc *__restrict__ descs,
                                                    const double *__restrict__ phi0,
                                                    const double *__restrict__ weight,
                                                    const int64_t *__restrict__ ofs,
                                                    const double *__restrict__ map,
                                                    double2 *__restrict__ delta) {
    extern __shared__ double2 buf[];
    const int r = blockIdx.x;
    const int mp = blockIdx.y;
    const FftDesc d = descs[ring_desc[r]];
    const int N = d.n;
    const double *in = map + (int64_t)mp * npix + ofs[r];
    for (int j = threadIdx.x; j < N; j += kBlock) buf[j] = input_point(make_double2(in[j], 0.0), d, j);
    __syncthreads();
    transform(buf, d);
    const double ph0 = phi0[r], w = weight[r];
    double2 *D = delta + ((int64_t)mp * nrings + r) * (mmax + 1);
    for (int m = threadIdx.x; m <= mmax; m += kBlock) {
        const double2 X = result_at(buf, d, m % N);
        const double2 e = phase_exp(m, ph0);
        // w * conj(e) * X
        D[m] = make_double2(w * fma(X.x, e.x, X.y * e.y), w * fma(X.y, e.x, -X.x * e.y));
    }
}

bool g_attr_set = false;

int set_lds_attr() {
    if (g_attr_set) return SHT_OK;
    const int bytes = kMaxFftLen * (int)sizeof(double2);
    SHT_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft_syn),
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    SHT_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_fft_ana),
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    g_attr_set = true;
    return SHT_OK;
}

}  // namespace

int launch_fft_syn(const GeomPlan &p, int mmax, const void *delta, double *map, int nmaps, hipStream_t st) {
    if (nmaps > 65535) return SHT_EUNSUPPORTED;
    int rc = set_lds_attr();
    if (rc) return rc;
    const size_t lds = (size_t)p.max_L * sizeof(double2);
    hipLaunchKernelGGL(k_fft_syn, dim3((unsigned)p.nrings, (unsigned)nmaps), dim3(kBlock), lds, st, mmax,
                       p.nrings, p.npix, p.ring_desc, p.descs, p.phi0, p.ofs,
                       static_cast<const double2 *>(delta), map);
    SHT_HIP(hipGetLastError());
    return SHT_OK;
}

int launch_fft_ana(const GeomPlan &p, int mmax, const double *map, void *delta, int nmaps, hipStream_t st) {
    if (nmaps > 65535) return SHT_EUNSUPPORTED;
    if (!p.weight) return SHT_EINVAL;
    int rc = set_lds_attr();
    if (rc) return rc;
    const size_t lds = (size_t)p.max_L * sizeof(double2);
    hipLaunchKernelGGL(k_fft_ana, dim3((unsigned)p.nrings, (unsigned)nmaps), dim3(kBlock), lds, st, mmax,
                       p.nrings, p.npix, p.ring_desc, p.descs, p.phi0, p.weight, p.ofs, map,
                       static_cast<double2 *>(delta));
    SHT_HIP(hipGetLastError());
    return SHT_OK;
}

}  // namespace sht
