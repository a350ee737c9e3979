// Legendre synthesis with the contraction on FP32 matrix cores (mixed
// precision, for batches of maps).
//
// For one m the paper writes Delta^A_m of a map as the matrix of
// lambda_lm(cos theta_r) (rings by l) times the vector of its a_lm (Sec. 3,
// eq. matrix_vec); for a batch the vector becomes an l-by-maps matrix, so each
// m is one matrix product.  As in the FP64 kernels, the recurrence runs in
// q_lm = lambda_lm / c_lm with c_lm folded into a_lm, one recurrence serves a
// ring pair, and the sum is split by the parity of l - m:
//   E[col][slot] = sum_{l-m even} a'_lm[col] q_lm(x_slot),  O likewise,
//   north ring = E + O, south ring = E - O,
// with col = 2 map + (0: real part, 1: imaginary part).
//
// Precision: the recurrence, its seeds, the start table and the coefficients
// are those of the FP64 kernels and run in FP64.  Each q_lm and each
// a'_lm = c_lm a_lm is rounded to FP32 once, and the products are summed in
// FP32 over l by v_mfma_f32_16x16x4_f32.  The ring FFTs stay FP64.
//
// Tiling: a wave owns 64 ring pairs (one recurrence per lane) and 16 NCF
// columns of one m; a workgroup holds four such waves on 256 consecutive
// pairs with the same columns, and the pair tiles of one m share one XCD's L2
// (the mapping of the FP64 kernels).  l advances in blocks of kMxL = 32: each
// lane runs 32 recurrence steps and writes its 16 even and 16 odd q (FP32) to
// its row of the wave's LDS tile; the wave reads them back in the matrix-core
// operand layout and issues 2 (parities) x 4 (16-pair groups) x NCF
// (16-column groups) x 4 (k steps) matrix instructions per block.  Within a
// block, k step j of lane l takes k = 4 (l / 16) + j for both operands (any
// one-to-one assignment of k to (lane group, step) gives the same sum), so
// each operand of four steps is one 16-byte load; k_prescale_mx stores a'
// tiled to match: [col group][l-block of column m][parity][col][k].
#include "k_device.h"

namespace sht {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kMxHalf = kMxL / 2;  // k values (l of one parity) per block
constexpr int kPRow = 5;           // 16-byte words per LDS row: 16 k + 4 floats of padding (conflict-free reads)
constexpr int kWaves = kBlock / 64;

// a'_lm = c_lm a_lm rounded to FP32, in the block-tiled operand layout.  One
// workgroup per (l-block, m, column group); entries with l > lmax or with a
// map index >= nmaps are zero, and Im a_l0 is ignored.
template <int NCF>
__global__ __launch_bounds__(kBlock) void k_prescale_mx(int lmax, int nmaps, int64_t nalm, int64_t mxblocks,
                                                      const int64_t *__restrict__ mxofs,
                                                      const double2 *__restrict__ alm,
                                                      const double *__restrict__ cfac,
                                                      float *__restrict__ out) {
    constexpr int NC = 16 * NCF;
    constexpr int kTile = 2 * NC * kMxHalf;
    const int kb = blockIdx.x, m = blockIdx.y, cg = blockIdx.z;
    if (kb >= mx_blocks(lmax, m)) return;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
    float *__restrict__ o = out + ((int64_t)cg * mxblocks + mxofs[m] + kb) * kTile;
    for (int e = threadIdx.x; e < kTile; e += kBlock) {
        const int p = e / (NC * kMxHalf), col = (e / kMxHalf) % NC, k = e % kMxHalf;
        const int l = m + kMxL * kb + 2 * k + p;
        const int map = cg * (NC / 2) + col / 2;
        double v = 0.0;
        if (l <= lmax && map < nmaps) {
            const double2 a = alm[(int64_t)map * nalm + base + l];
            v = (col & 1) ? (m == 0 ? 0.0 : a.y) : a.x;
            v *= cfac[base + l];
        }
        o[e] = (float)v;
    }
}

template <int NCF>
__global__ __launch_bounds__(kBlock, 2) void k_leg_syn_mx(int lmax, int mmax, int nslots, int tiles, int nrings,
                                                        int nmaps, int64_t mxblocks,
                                                        const int64_t *__restrict__ mxofs,
                                                        const float *__restrict__ ap,
                                                        const double *__restrict__ alpha,
                                                        const int32_t *__restrict__ lstart,
                                                        const double2 *__restrict__ state,
                                                        const double *__restrict__ sx,
                                                        const int32_t *__restrict__ rn,
                                                        const int32_t *__restrict__ rsouth,
                                                        double2 *__restrict__ delta) {
    constexpr int NC = 16 * NCF;
    constexpr int kTile = 2 * NC * kMxHalf;
    __shared__ floatx4 pt[kWaves][2][64][kPRow];

    const MPart mp = xcd_m_part(tiles);
    const int m = mp.m, tile = mp.part;
    if (m > mmax) return;  // padding of the m range
    const int cg = blockIdx.y;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int c16 = lane & 15, kq = lane >> 4;
    const int slot = tile * kBlock + (int)threadIdx.x;
    const bool act = slot < nslots;
    const double x = act ? sx[slot] : 0.0;
    const int ls = act ? lstart[(int64_t)m * nslots + slot] : lmax + 1;
    const double2 stv = act ? state[(int64_t)m * nslots + slot] : make_double2(0.0, 0.0);
    const int lo = wave_min(ls);
    const int hi = wave_max(ls <= lmax ? ls : m);

    const int64_t base = uniform64((int64_t)m * (2 * lmax + 1 - m) / 2);  // (l, m) lives at base + l
    const double *__restrict__ al = alpha + base;
    const float *__restrict__ apm = ap + ((int64_t)cg * mxblocks + mxofs[m]) * kTile;
    const int nb = mx_blocks(lmax, m);

    floatx4 acc[2][4][NCF];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int rf = 0; rf < 4; ++rf)
#pragma unroll
            for (int cf = 0; cf < NCF; ++cf) acc[p][rf][cf] = floatx4{0.f, 0.f, 0.f, 0.f};

    double q1 = 0.0, q2 = 0.0;  // a pair carries zeros until it starts
    const int kb0 = lo <= lmax ? (lo - m) / kMxL : nb;
    for (int kb = kb0; kb < nb; ++kb) {
        // uniform; restated so that the compiler keeps alpha on scalar loads
        // (inside the injection branch it may otherwise use the equal lane
        // value ls in its place)
        const int l0 = __builtin_amdgcn_readfirstlane(m + kMxL * kb);
        // a' operands of this block (issued first, used after the recurrence)
        floatx4 av[2][NCF];
        const float *__restrict__ t = apm + (int64_t)kb * kTile;
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int cf = 0; cf < NCF; ++cf)
                av[p][cf] = *reinterpret_cast<const floatx4 *>(t + p * NC * kMxHalf + (cf * 16 + c16) * kMxHalf + kq * 4);

        // 32 recurrence steps, written as FP32 to this lane's LDS rows; starts
        // lie at m + kStartStep j, so only the four 8-step boundaries inject
        const bool inj = l0 <= hi;
        const bool tail = l0 + kMxL - 1 > lmax;
#pragma unroll
        for (int g = 0; g < kMxL / 8; ++g) {
            if (inj && ls == l0 + 8 * g) {
                q2 = stv.x;
                q1 = stv.y;
            }
            float pe[4], po[4];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int l = l0 + 8 * g + i;
                const double q = fma(al[l] * x, q1, -q2);
                q2 = q1;
                q1 = q;
                // past lmax alpha runs into the next column: those q are not used
                const float f = (tail && l > lmax) ? 0.f : (float)q;
                if (i & 1)
                    po[i >> 1] = f;
                else
                    pe[i >> 1] = f;
            }
            pt[w][0][lane][g] = floatx4{pe[0], pe[1], pe[2], pe[3]};
            pt[w][1][lane][g] = floatx4{po[0], po[1], po[2], po[3]};
        }
        // LDS operations of one wave complete in order: the reads below see
        // the writes above, and the next block's writes follow these reads
        floatx4 bv[2][4];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int rf = 0; rf < 4; ++rf)
                bv[p][rf] = pt[w][p][rf * 16 + c16][kq];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int rf = 0; rf < 4; ++rf)
#pragma unroll
                    for (int cf = 0; cf < NCF; ++cf)
                        acc[p][rf][cf] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[p][cf][j], bv[p][rf][j],
                                                                              acc[p][rf][cf], 0, 0, 0);
    }

    // lane l holds rows (columns of the batch) 4 (l / 16) + r, r < 4, i.e. two
    // whole complex values, of ring pair 16 rf + l % 16 in each 16 x 16 tile
#pragma unroll
    for (int rf = 0; rf < 4; ++rf) {
        const int s = tile * kBlock + w * 64 + rf * 16 + c16;
        if (s >= nslots) continue;
        const int64_t rN = rn[s], rS = rsouth[s];
#pragma unroll
        for (int cf = 0; cf < NCF; ++cf)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int map = cg * (NC / 2) + cf * 8 + 2 * kq + h;
                if (map >= nmaps) continue;
                const double er = acc[0][rf][cf][2 * h], ei = acc[0][rf][cf][2 * h + 1];
                const double orr = acc[1][rf][cf][2 * h], oi = acc[1][rf][cf][2 * h + 1];
                double2 *d = delta + (int64_t)map * nrings * (mmax + 1) + m;
                d[rN * (mmax + 1)] = make_double2(er + orr, ei + oi);
                if (rS >= 0) d[rS * (mmax + 1)] = make_double2(er - orr, ei - oi);
            }
    }
}

template <int NCF>
int launch_syn_mx_t(const CoefTables &c, const GeomPlan &p, const StartTable &s, const void *alm, void *aprime,
                    void *delta, int nmaps, hipStream_t st) {
    constexpr int NC = 16 * NCF;
    const int ncg = (nmaps + NC / 2 - 1) / (NC / 2);
    const int tiles = (p.nslots + kBlock - 1) / kBlock;
    const int64_t gx = (int64_t)tiles * padded_m(c.mmax);
    if (!grid_ok(gx) || c.mmax + 1 > 65535 || ncg > 65535) return SHT_EUNSUPPORTED;
    hipLaunchKernelGGL(k_prescale_mx<NCF>, dim3((unsigned)mx_blocks(c.lmax, 0), (unsigned)(c.mmax + 1), (unsigned)ncg),
                       dim3(kBlock), 0, st, c.lmax, nmaps, c.nalm, c.mxblocks, c.mxofs,
                       static_cast<const double2 *>(alm), c.cfac, static_cast<float *>(aprime));
    SHT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_leg_syn_mx<NCF>, dim3((unsigned)gx, (unsigned)ncg), dim3(kBlock), 0, st, c.lmax, c.mmax,
                       p.nslots, tiles, p.nrings, nmaps, c.mxblocks, c.mxofs, static_cast<const float *>(aprime),
                       c.alpha, s.lstart, s.state, p.slot_x, p.slot_north, p.slot_south,
                       static_cast<double2 *>(delta));
    SHT_HIP(hipGetLastError());
    return SHT_OK;
}

}  // namespace

int mx_col_frags(int nmaps) { return nmaps <= 8 ? 1 : nmaps <= 16 ? 2 : 4; }

size_t mx_aprime_bytes(int lmax, int mmax, int nmaps) {
    int64_t blocks = 0;
    for (int m = 0; m <= mmax; ++m) blocks += mx_blocks(lmax, m);
    const int nc = 16 * mx_col_frags(nmaps);
    const int64_t ncg = (nmaps + nc / 2 - 1) / (nc / 2);
    return (size_t)(ncg * blocks * 2 * nc * kMxHalf) * sizeof(float);
}

int launch_leg_syn_mx(const CoefTables &c, const GeomPlan &p, const StartTable &s, const void *alm, void *aprime,
                      void *delta, int nmaps, hipStream_t st) {
    switch (mx_col_frags(nmaps)) {
        case 1: return launch_syn_mx_t<1>(c, p, s, alm, aprime, delta, nmaps, st);
        case 2: return launch_syn_mx_t<2>(c, p, s, alm, aprime, delta, nmaps, st);
        default: return launch_syn_mx_t<4>(c, p, s, alm, aprime, delta, nmaps, st);
    }
}

}  // namespace sht
