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
// FP32 by v_mfma_f32_16x16x4_f32: over all l (one FP32 chain), or, with
// block sums in FP64 (F64S), over the 32 l of one block in a fresh FP32
// accumulator whose sum is then added to FP64 totals -- the compensated form
// of the l-sum, whose error no longer grows with the number of blocks.  In
// the split form (SPLIT) each FP32 operand is cut exactly into three bf16
// parts and each product is formed from the six part products above 2^-24
// of it by v_mfma_f32_16x16x16_bf16, again summed in FP32.  The ring FFTs
// stay FP64.
//
// Tiling: a wave owns 64 ring pairs (one recurrence per lane) and 16 NCF
// columns (NCF = 1, 2, 4) of one m; a workgroup holds four such waves on 256 consecutive
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
#include <type_traits>

#include "k_device.h"

namespace sht {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));  // four bf16 matrix-core operands

// Split of an FP32 value f into three bf16 parts by truncation: hi keeps the
// sign, exponent and top 7 fraction bits of f; r = f - hi is exact in FP32
// and has at most 16 significant bits, mid is its top 8, and lo = r - mid
// has at most 8, so f = hi + mid + lo exactly (unless lo falls below the
// normal FP32 range).  Each part is returned in the upper half of an FP32
// bit pattern whose lower half is zero.
struct Split3 {
    uint32_t hi, mid, lo;
};
__device__ __forceinline__ Split3 split3(float f) {
    Split3 s;
    s.hi = __float_as_uint(f) & 0xffff0000u;
    const float r = f - __uint_as_float(s.hi);
    s.mid = __float_as_uint(r) & 0xffff0000u;
    s.lo = __float_as_uint(r - __uint_as_float(s.mid));
    return s;
}
// bf16 pair (a, b) from the upper halves of two such bit patterns (a in the
// lower 16 bits)
__device__ __forceinline__ uint32_t bf16_pair(uint32_t a, uint32_t b) { return __builtin_amdgcn_perm(b, a, 0x07060302u); }
// the six products of the split operands that carry more than 2^-24 of the
// whole, smallest first, added to acc
__device__ __forceinline__ floatx4 mfma_split3(const shortx4 (&a)[3], const shortx4 (&b)[3], floatx4 acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[2], b[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[1], b[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[0], b[2], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[1], b[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[0], b[1], acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[0], b[0], acc, 0, 0, 0);
}

constexpr int kMxHalf = kMxL / 2;  // k values (l of one parity) per block
constexpr int kPRow = 5;           // 16-byte words per LDS row: 16 k + 4 floats of padding (conflict-free reads)
constexpr int kWaves = kBlock / 64;

// a'_lm = c_lm a_lm rounded to FP32, in the block-tiled operand layout.  One
// workgroup per (l-block, m, column group); a thread takes one complex a_lm
// (consecutive threads: consecutive l of one map, so the reads are
// contiguous) and writes its two columns into the workgroup's tile.  Entries
// with l > lmax or with a map index >= nmaps are zero, and Im a_l0 is ignored.
// SPLIT: the tile holds three bf16 planes (hi, mid, lo of split3) of the same
// layout instead of one FP32 plane.
template <int NCF, bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_prescale_mx(int lmax, int nmaps, int64_t nalm, int64_t mxblocks,
                                                      const int64_t *__restrict__ mxofs,
                                                      const double2 *__restrict__ alm,
                                                      const double *__restrict__ cfac,
                                                      void *__restrict__ out) {
    constexpr int NC = 16 * NCF;
    constexpr int kPlane = 2 * NC * kMxHalf;
    constexpr int kTile = (SPLIT ? 3 : 1) * kPlane;
    const int kb = blockIdx.x, m = blockIdx.y, cg = blockIdx.z;
    if (kb >= mx_blocks(lmax, m)) return;
    const int64_t base = (int64_t)m * (2 * lmax + 1 - m) / 2;
    const int64_t tile = ((int64_t)cg * mxblocks + mxofs[m] + kb) * kTile;
    for (int e = threadIdx.x; e < kMxL * (NC / 2); e += kBlock) {
        const int lt = e % kMxL, mm = e / kMxL;  // l offset in the block, map in the group
        const int l = m + kMxL * kb + lt, map = cg * (NC / 2) + mm;
        double re = 0.0, im = 0.0;
        if (l <= lmax && map < nmaps) {
            const double2 a = alm[(int64_t)map * nalm + base + l];
            const double c = cfac[base + l];
            re = a.x * c;
            im = m == 0 ? 0.0 : a.y * c;
        }
        const int at = ((lt & 1) * NC + 2 * mm) * kMxHalf + (lt >> 1);
        if constexpr (SPLIT) {
            uint16_t *__restrict__ t = static_cast<uint16_t *>(out) + tile + at;
            const Split3 r = split3((float)re), i = split3((float)im);
            t[0] = (uint16_t)(r.hi >> 16);
            t[kPlane] = (uint16_t)(r.mid >> 16);
            t[2 * kPlane] = (uint16_t)(r.lo >> 16);
            t[kMxHalf] = (uint16_t)(i.hi >> 16);
            t[kPlane + kMxHalf] = (uint16_t)(i.mid >> 16);
            t[2 * kPlane + kMxHalf] = (uint16_t)(i.lo >> 16);
        } else {
            float *__restrict__ t = static_cast<float *>(out) + tile + at;
            t[0] = (float)re;
            t[kMxHalf] = (float)im;
        }
    }
}

// LDS q tiles of one workgroup: per wave, parity and lane row, the four
// 4-k words of a block as FP32, or (SPLIT) as bf16 in three planes (8-byte
// words; a row of 5 words keeps the row writes and the operand reads free of
// bank conflicts, as kPRow does for the 16-byte words)
struct QTileF32 {
    floatx4 v[kWaves][2][64][kPRow];
};
struct QTileSplit {
    uint2 v[kWaves][3][2][64][kPRow];
};

template <int NCF, bool F64S, bool SPLIT>
__global__ __launch_bounds__(kBlock, 2) void k_leg_syn_mx(int lmax, int mmax, int nslots, int tiles, DeltaLayout dl,
                                                        int nmaps, int64_t mxblocks,
                                                        const int64_t *__restrict__ mxofs,
                                                        const void *__restrict__ ap,
                                                        const double *__restrict__ alpha,
                                                        const int32_t *__restrict__ lstart,
                                                        const double2 *__restrict__ state,
                                                        const double *__restrict__ sx,
                                                        const int32_t *__restrict__ rn,
                                                        const int32_t *__restrict__ rsouth,
                                                        double2 *__restrict__ delta) {
    constexpr int NC = 16 * NCF;
    constexpr int kPlane = 2 * NC * kMxHalf;
    constexpr int kTile = (SPLIT ? 3 : 1) * kPlane;
    __shared__ typename std::conditional<SPLIT, QTileSplit, QTileF32>::type pt;

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
    const int64_t apm = ((int64_t)cg * mxblocks + mxofs[m]) * kTile;  // this m's tiles (elements)
    const int nb = mx_blocks(lmax, m);

    // FP32 accumulators of the matrix instructions; with F64S they hold one
    // block's sum, added to the FP64 totals dsum after the block
    floatx4 acc[2][4][NCF];
    double dsum[2][4][F64S ? NCF : 1][4];  // (unused without F64S)
    auto zero_acc = [&]() {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int rf = 0; rf < 4; ++rf)
#pragma unroll
                for (int cf = 0; cf < NCF; ++cf) acc[p][rf][cf] = floatx4{0.f, 0.f, 0.f, 0.f};
    };
    zero_acc();
    if constexpr (F64S) {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int rf = 0; rf < 4; ++rf)
#pragma unroll
                for (int cf = 0; cf < NCF; ++cf)
#pragma unroll
                    for (int r = 0; r < 4; ++r) dsum[p][rf][cf][r] = 0.0;
    }

    double q1 = 0.0, q2 = 0.0;  // a pair carries zeros until it starts
    const int kb0 = lo <= lmax ? (lo - m) / kMxL : nb;
    // a' operands: FP32 one block ahead, those of block kb loaded while block
    // kb - 1 runs (the index is clamped, so the load after the last block
    // re-reads it and stays in bounds); SPLIT (three times the registers) at
    // the start of their own block, in flight during its recurrence steps
    floatx4 an[2][NCF];
    shortx4 ans[2][NCF][3];  // SPLIT: hi, mid, lo
    auto load_a = [&](int kb) {
        const int64_t t = apm + (int64_t)min(kb, nb - 1) * kTile;
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int cf = 0; cf < NCF; ++cf) {
                const int at = p * NC * kMxHalf + (cf * 16 + c16) * kMxHalf + kq * 4;
                if constexpr (SPLIT) {
#pragma unroll
                    for (int h = 0; h < 3; ++h)
                        ans[p][cf][h] =
                            *reinterpret_cast<const shortx4 *>(static_cast<const uint16_t *>(ap) + t + h * kPlane + at);
                } else {
                    an[p][cf] = *reinterpret_cast<const floatx4 *>(static_cast<const float *>(ap) + t + at);
                }
            }
    };
    if constexpr (!SPLIT) {
        if (kb0 < nb) load_a(kb0);
    }
    for (int kb = kb0; kb < nb; ++kb) {
        // uniform; restated so that the compiler keeps alpha on scalar loads
        // (inside the injection branch it may otherwise use the equal lane
        // value ls in its place)
        const int l0 = __builtin_amdgcn_readfirstlane(m + kMxL * kb);
        floatx4 av[2][NCF];
        if constexpr (SPLIT) {
            load_a(kb);
        } else {
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int cf = 0; cf < NCF; ++cf) av[p][cf] = an[p][cf];
            load_a(kb + 1);
        }
        // compiler-only fence: the loads stay here, ahead of this block's work
        asm volatile("" ::: "memory");

        // 32 recurrence steps, written as FP32 to this lane's LDS rows; starts
        // lie at m + kStartStep j, so only the four 8-step boundaries inject
        // blocks where pairs start (injection) or that pass lmax take the
        // general path, all others the one without selects
        auto steps = [&](auto general) {
#pragma unroll
            for (int g = 0; g < kMxL / 8; ++g) {
                if constexpr (decltype(general)::value) {
                    if (ls == l0 + 8 * g) {
                        q2 = stv.x;
                        q1 = stv.y;
                    }
                }
                float pe[4], po[4];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int l = l0 + 8 * g + i;
                    const double q = fma(al[l] * x, q1, -q2);
                    q2 = q1;
                    q1 = q;
                    // past lmax alpha runs into the next column: those q are not used
                    float f = (float)q;
                    if constexpr (decltype(general)::value) f = l > lmax ? 0.f : f;
                    if (i & 1)
                        po[i >> 1] = f;
                    else
                        pe[i >> 1] = f;
                }
                if constexpr (SPLIT) {
                    Split3 e[4], o[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        e[i] = split3(pe[i]);
                        o[i] = split3(po[i]);
                    }
                    pt.v[w][0][0][lane][g] = make_uint2(bf16_pair(e[0].hi, e[1].hi), bf16_pair(e[2].hi, e[3].hi));
                    pt.v[w][1][0][lane][g] = make_uint2(bf16_pair(e[0].mid, e[1].mid), bf16_pair(e[2].mid, e[3].mid));
                    pt.v[w][2][0][lane][g] = make_uint2(bf16_pair(e[0].lo, e[1].lo), bf16_pair(e[2].lo, e[3].lo));
                    pt.v[w][0][1][lane][g] = make_uint2(bf16_pair(o[0].hi, o[1].hi), bf16_pair(o[2].hi, o[3].hi));
                    pt.v[w][1][1][lane][g] = make_uint2(bf16_pair(o[0].mid, o[1].mid), bf16_pair(o[2].mid, o[3].mid));
                    pt.v[w][2][1][lane][g] = make_uint2(bf16_pair(o[0].lo, o[1].lo), bf16_pair(o[2].lo, o[3].lo));
                } else {
                    pt.v[w][0][lane][g] = floatx4{pe[0], pe[1], pe[2], pe[3]};
                    pt.v[w][1][lane][g] = floatx4{po[0], po[1], po[2], po[3]};
                }
            }
        };
        if (l0 <= hi || l0 + kMxL - 1 > lmax)
            steps(std::true_type{});
        else
            steps(std::false_type{});
        // LDS operations of one wave complete in order: the reads below see
        // the writes above, and the next block's writes follow these reads
        if constexpr (SPLIT) {
            // one 16 x 16 x 16 bf16 instruction covers the 16 k of a parity
            // (lane l: k = 4 (l / 16) + i, the k of the FP32 steps j = i);
            // the q planes of one 16-pair tile are read just before its products
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int rf = 0; rf < 4; ++rf) {
                    shortx4 b3[3];
#pragma unroll
                    for (int h = 0; h < 3; ++h) b3[h] = __builtin_bit_cast(shortx4, pt.v[w][h][p][rf * 16 + c16][kq]);
#pragma unroll
                    for (int cf = 0; cf < NCF; ++cf) acc[p][rf][cf] = mfma_split3(ans[p][cf], b3, acc[p][rf][cf]);
                }
        } else {
            floatx4 bv[2][4];
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int rf = 0; rf < 4; ++rf)
                    bv[p][rf] = pt.v[w][p][rf * 16 + c16][kq];
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
        if constexpr (F64S) {
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int rf = 0; rf < 4; ++rf)
#pragma unroll
                    for (int cf = 0; cf < NCF; ++cf)
#pragma unroll
                        for (int r = 0; r < 4; ++r) dsum[p][rf][cf][r] += (double)acc[p][rf][cf][r];
            zero_acc();
        }
    }
    // the l-sum of (parity p, tile rf, column group cf, row r)
    auto total = [&](int p, int rf, int cf, int r) -> double {
        if constexpr (F64S)
            return dsum[p][rf][cf][r];
        else
            return (double)acc[p][rf][cf][r];
    };

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
                const double er = total(0, rf, cf, 2 * h), ei = total(0, rf, cf, 2 * h + 1);
                const double orr = total(1, rf, cf, 2 * h), oi = total(1, rf, cf, 2 * h + 1);
                double2 *d = delta + map * dl.s_map + m * dl.s_m;
                d[rN * dl.s_ring] = make_double2(er + orr, ei + oi);
                if (rS >= 0) d[rS * dl.s_ring] = make_double2(er - orr, ei - oi);
            }
    }
}

// Analysis: a_lm[col] = c_lm sum_pairs D[pair][col] q_lm(x_pair) with
// D = D+ = north + south for even l - m and D- = north - south for odd (the
// mirror identity used by the FP64 kernels), col = 2 map + (re, im).  One
// workgroup of kAnaMxWaves waves holds kAnaMxGroup ring pairs of one m (a
// group; more pairs take several groups whose partial sums k_ana_combine
// adds) and kAnaMxMaps maps.  Wave w owns kAnaMxTiles tiles of 64 pairs,
// spread over the group's latitudes; its
// D+ and D- operands stay in registers for the whole kernel (rounded to FP32
// once).  Per l-block each wave runs the recurrences of its tiles (one pair
// per lane), stages q (FP32) in its LDS tile k-major, and contracts over its
// pairs on the matrix cores with a fresh FP32 accumulator: rows are the 16 l
// of one parity, columns the 16 columns, K the pairs (in k step j of tile t,
// lane l takes pair 16 (l / 16) + 4 u + j of the tile for its u-th operand
// load).  The waves' sums of two consecutive blocks are added in wave order in
// FP64 after one barrier (two LDS buffers in turn), scaled by c_lm and written.
constexpr int kAnaMxTiles = 4;
constexpr int kAnaMxMaps = 8;   // 16 columns
constexpr int kQRow = 64 + 4;   // floats per k row of a q tile (padding: conflict-free operand reads)
static_assert(kAnaMxGroup == 8 * kAnaMxTiles * 64, "pairs per analysis group of the widest workgroup");
constexpr int kAnaMxOut = 2 * 2 * kMxHalf * kAnaMxMaps;  // finished (block, parity, k, map) per two blocks

// WAVES waves per workgroup (kAnaMxTiles * 64 * WAVES ring pairs): 8 for large
// geometries, 4 or 2 where the pairs fill no more than that, so that a
// workgroup's waves carry whole tiles and, with less LDS each, two or four
// workgroups share a CU (two waves per SIMD in every case: the Delta operands
// take 128 VGPRs)
template <int WAVES>
__global__ __launch_bounds__(64 * WAVES, WAVES == 8 ? 1 : 2) void k_leg_ana_mx(int lmax, int mmax, int nslots, DeltaLayout dl,
                                                              int nmaps, int64_t nalm, int groups,
                                                              const double2 *__restrict__ delta,
                                                              const double *__restrict__ alpha,
                                                              const double *__restrict__ cfac,
                                                              const int32_t *__restrict__ lstart,
                                                              const double2 *__restrict__ state,
                                                              const double *__restrict__ sx,
                                                              const int32_t *__restrict__ rn,
                                                              const int32_t *__restrict__ rsouth,
                                                              double2 *__restrict__ alm,
                                                              double2 *__restrict__ part) {
    constexpr int kThreads = 64 * WAVES, kGroup = WAVES * kAnaMxTiles * 64;
    __shared__ float qs[WAVES][2][kMxHalf][kQRow];
    __shared__ float red[2][2][WAVES][2][kMxHalf][16];  // [buffer][block of the pair]...
    __shared__ int wlo[WAVES];

    const MPart mp = xcd_m_part(groups);
    const int m = mp.m, grp = mp.part;
    if (m > mmax) return;  // padding of the m range (whole workgroup, before any barrier)
    const int cg = blockIdx.y;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int c16 = lane & 15, kq = lane >> 4;
    const int map_c = cg * kAnaMxMaps + (c16 >> 1);  // this lane's column: map and part
    const bool col_ok = map_c < nmaps;
    // tile t of wave w holds pairs from (t * WAVES + w) * 64 on: pairs are
    // sorted by latitude and start late near the poles, so every wave gets
    // tiles from the whole range and the waves' work per block stays even
    auto tile0 = [&](int t) { return grp * kGroup + (t * WAVES + w) * 64; };

    double x[kAnaMxTiles], q1[kAnaMxTiles], q2[kAnaMxTiles];
    double2 stv[kAnaMxTiles];
    int ls[kAnaMxTiles], tlo[kAnaMxTiles], thi[kAnaMxTiles];
    float dp[kAnaMxTiles][16], dm[kAnaMxTiles][16];
    const double *__restrict__ dcol = reinterpret_cast<const double *>(delta) +
                                      2 * ((col_ok ? map_c : 0) * dl.s_map + m * dl.s_m) + (c16 & 1);
    int mylo = lmax + 1;
#pragma unroll
    for (int t = 0; t < kAnaMxTiles; ++t) {
        const int slot = tile0(t) + lane;
        const bool act = slot < nslots;
        x[t] = act ? sx[slot] : 0.0;
        ls[t] = act ? lstart[(int64_t)m * nslots + slot] : lmax + 1;
        stv[t] = act ? state[(int64_t)m * nslots + slot] : make_double2(0.0, 0.0);
        q1[t] = q2[t] = 0.0;
        tlo[t] = wave_min(ls[t]);
        thi[t] = wave_max(ls[t] <= lmax ? ls[t] : m);
        mylo = min(mylo, tlo[t]);
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            // branch-free: indices clamped into range, unused values selected away
            const int sl = tile0(t) + 16 * kq + s;
            const bool ok = sl < nslots && col_ok;
            const int slc = min(sl, nslots - 1);
            const int r2 = rsouth[slc];
            const double vn = dcol[2 * rn[slc] * dl.s_ring];
            const double vs = dcol[2 * max(r2, 0) * dl.s_ring];
            const double dn = ok ? vn : 0.0, ds = (ok && r2 >= 0) ? vs : 0.0;
            dp[t][s] = (float)(dn + ds);
            dm[t][s] = (float)(dn - ds);
            // the FP32 operands exist here, before the barrier below: keeping
            // the FP64 values live past it instead would need 256 registers
            asm volatile("" ::"v"(dp[t][s]), "v"(dm[t][s]));
        }
    }
    if (lane == 0) wlo[w] = mylo;
    __syncthreads();
    int lo = lmax + 1;
#pragma unroll
    for (int i = 0; i < WAVES; ++i) lo = min(lo, wlo[i]);
    lo = __builtin_amdgcn_readfirstlane(lo);

    const int64_t base = uniform64((int64_t)m * (2 * lmax + 1 - m) / 2);  // (l, m) lives at base + l
    const double *__restrict__ al = alpha + base;
    const int nb = mx_blocks(lmax, m);
    const int kb0 = lo <= lmax ? (lo - m) / kMxL : nb;
    auto out_at = [&](int map, int l) -> double2 * {
        return groups == 1 ? alm + (int64_t)map * nalm + base + l
                           : part + ((int64_t)map * groups + grp) * nalm + base + l;
    };
    // no pair of the group has started before block kb0: those a_lm get no term
    for (int i = threadIdx.x; i < kb0 * kMxL * kAnaMxMaps; i += kThreads) {
        const int l = m + i / kAnaMxMaps, map = cg * kAnaMxMaps + i % kAnaMxMaps;
        if (l <= lmax && map < nmaps) *out_at(map, l) = make_double2(0.0, 0.0);
    }

    // the wave sums of two consecutive blocks are kept (slot b of the pair)
    // and added across the waves together: one barrier per two blocks
    floatx4 acc2[2][2];
#pragma unroll
    for (int b = 0; b < 2; ++b) acc2[b][0] = acc2[b][1] = floatx4{0.f, 0.f, 0.f, 0.f};
    int buf = 0;
    for (int kb = kb0; kb < nb; ++kb) {
        const int l0 = __builtin_amdgcn_readfirstlane(m + kMxL * kb);
        const bool tail = l0 + kMxL - 1 > lmax;
        const int slot = (kb - kb0) & 1;
#pragma unroll
        for (int t = 0; t < kAnaMxTiles; ++t) {
            if (tlo[t] > l0 + kMxL - 1) continue;  // no pair of the tile has started: all q are 0
            // 32 steps; blocks where pairs start (injection) or that pass lmax
            // take the general path, all others the one without selects
            auto steps = [&](auto general) {
#pragma unroll
                for (int g = 0; g < kMxL / 8; ++g) {
                    if constexpr (decltype(general)::value) {
                        if (ls[t] == l0 + 8 * g) {
                            q2[t] = stv[t].x;
                            q1[t] = stv[t].y;
                        }
                    }
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const int l = l0 + 8 * g + i;
                        const double q = fma(al[l] * x[t], q1[t], -q2[t]);
                        q2[t] = q1[t];
                        q1[t] = q;
                        float f = (float)q;
                        if constexpr (decltype(general)::value) f = l > lmax ? 0.f : f;
                        qs[w][i & 1][4 * g + (i >> 1)][lane] = f;
                    }
                }
            };
            if (tail || l0 <= thi[t])
                steps(std::true_type{});
            else
                steps(std::false_type{});
            // LDS operations of one wave complete in order (no barrier needed)
            auto mma = [&](floatx4 (&acc)[2]) {
#pragma unroll
                for (int p = 0; p < 2; ++p) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const floatx4 a4 = *reinterpret_cast<const floatx4 *>(&qs[w][p][c16][16 * kq + 4 * u]);
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            acc[p] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                                a4[j], p ? dm[t][4 * u + j] : dp[t][4 * u + j], acc[p], 0, 0, 0);
                    }
                }
            };
            if (slot == 0)
                mma(acc2[0]);
            else
                mma(acc2[1]);
        }
        if (slot == 0 && kb + 1 < nb) continue;  // the pair's second block comes first
        // lane l holds rows (k) 4 (l / 16) + r of column l % 16
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int r = 0; r < 4; ++r) red[buf][b][w][p][4 * kq + r][c16] = acc2[b][p][r];
        __syncthreads();
        for (int e = threadIdx.x; e < kAnaMxOut; e += kThreads) {
            const int b = e / (2 * kMxHalf * kAnaMxMaps);
            const int p = (e / (kMxHalf * kAnaMxMaps)) % 2;
            const int k = (e / kAnaMxMaps) % kMxHalf, mm = e % kAnaMxMaps;
            const int l = m + kMxL * (kb - slot + b) + 2 * k + p, map = cg * kAnaMxMaps + mm;
            if (b <= slot && l <= lmax && map < nmaps) {
                double sr = 0.0, si = 0.0;
#pragma unroll
                for (int v = 0; v < WAVES; ++v) {
                    sr += red[buf][b][v][p][k][2 * mm];
                    si += red[buf][b][v][p][k][2 * mm + 1];
                }
                if (groups == 1) {
                    const double c = cfac[base + l];
                    *out_at(map, l) = make_double2(sr * c, m == 0 ? 0.0 : si * c);
                } else {
                    *out_at(map, l) = make_double2(sr, si);  // scaled and Im a_l0 cleared by k_ana_combine
                }
            }
        }
#pragma unroll
        for (int b = 0; b < 2; ++b) acc2[b][0] = acc2[b][1] = floatx4{0.f, 0.f, 0.f, 0.f};
        buf ^= 1;  // the next pair writes the other buffer while this one may still be read
    }
}

template <int NCF, bool F64S, bool SPLIT>
int launch_syn_mx_t(const CoefTables &c, const GeomPlan &p, const StartTable &s, const void *alm, void *aprime,
                    void *delta, DeltaLayout dl, int nmaps, hipStream_t st) {
    constexpr int NC = 16 * NCF;
    const int ncg = (nmaps + NC / 2 - 1) / (NC / 2);
    const int tiles = (p.nslots + kBlock - 1) / kBlock;
    const int64_t gx = (int64_t)tiles * padded_m(c.mmax);
    if (!grid_ok(gx) || c.mmax + 1 > 65535 || ncg > 65535) return SHT_EUNSUPPORTED;
    hipLaunchKernelGGL((k_prescale_mx<NCF, SPLIT>), dim3((unsigned)mx_blocks(c.lmax, 0), (unsigned)(c.mmax + 1), (unsigned)ncg),
                       dim3(kBlock), 0, st, c.lmax, nmaps, c.nalm, c.mxblocks, c.mxofs,
                       static_cast<const double2 *>(alm), c.cfac, aprime);
    SHT_HIP(hipGetLastError());
    hipLaunchKernelGGL((k_leg_syn_mx<NCF, F64S, SPLIT>), dim3((unsigned)gx, (unsigned)ncg), dim3(kBlock), 0, st, c.lmax, c.mmax,
                       p.nslots, tiles, dl, nmaps, c.mxblocks, c.mxofs, static_cast<const void *>(aprime),
                       c.alpha, s.lstart, s.state, p.slot_x, p.slot_north, p.slot_south,
                       static_cast<double2 *>(delta));
    SHT_HIP(hipGetLastError());
    return SHT_OK;
}

template <int WAVES>
int launch_ana_mx_t(const CoefTables &c, const GeomPlan &p, const StartTable &s, const void *delta,
                    DeltaLayout dl, void *alm, int nmaps, void *partials, hipStream_t st) {
    constexpr int kGroup = WAVES * kAnaMxTiles * 64;
    const int groups = (p.nslots + kGroup - 1) / kGroup;
    const int ncg = (nmaps + kAnaMxMaps - 1) / kAnaMxMaps;
    const int64_t gx = (int64_t)groups * padded_m(c.mmax);
    if (!grid_ok(gx) || ncg > 65535) return SHT_EUNSUPPORTED;
    if (groups > 1 && !partials) return SHT_EWORKSPACE;
    hipLaunchKernelGGL(k_leg_ana_mx<WAVES>, dim3((unsigned)gx, (unsigned)ncg), dim3(64 * WAVES), 0, st, c.lmax,
                       c.mmax, p.nslots, dl, nmaps, c.nalm, groups, static_cast<const double2 *>(delta), c.alpha,
                       c.cfac, s.lstart, s.state, p.slot_x, p.slot_north, p.slot_south, static_cast<double2 *>(alm),
                       static_cast<double2 *>(partials));
    SHT_HIP(hipGetLastError());
    return groups > 1 ? launch_ana_combine(c, nmaps, groups, partials, alm, st) : SHT_OK;
}

}  // namespace

int launch_leg_ana_mx(const CoefTables &c, const GeomPlan &p, const StartTable &s, const void *delta,
                      DeltaLayout dl, void *alm, int nmaps, void *partials, hipStream_t st) {
    if (p.nslots <= 2 * kAnaMxTiles * 64) return launch_ana_mx_t<2>(c, p, s, delta, dl, alm, nmaps, partials, st);
    if (p.nslots <= 4 * kAnaMxTiles * 64) return launch_ana_mx_t<4>(c, p, s, delta, dl, alm, nmaps, partials, st);
    return launch_ana_mx_t<8>(c, p, s, delta, dl, alm, nmaps, partials, st);
}

// Block sums in FP64 (the compensated l-sum) with SHT_MIXED_FP64_SUMS, and
// always above kMxOneChainLmax, where one FP32 chain over the l range would
// pass the 1e-6 target.  The FP64 totals take the registers of three more
// column groups, so such a wave covers 8 maps.
constexpr int kMxOneChainLmax = 2048;
bool mx_f64_sums(int lmax, uint32_t flags) { return lmax > kMxOneChainLmax || (flags & SHT_MIXED_FP64_SUMS); }
// 16-column groups per wave
int mx_col_frags(int nmaps, int lmax, uint32_t flags) {
    if (mx_f64_sums(lmax, flags)) return 1;
    return nmaps <= 8 ? 1 : nmaps <= 16 ? 2 : 4;
}

size_t mx_aprime_bytes(int lmax, int mmax, int nmaps, uint32_t flags) {
    int64_t blocks = 0;
    for (int m = 0; m <= mmax; ++m) blocks += mx_blocks(lmax, m);
    const int nc = 16 * mx_col_frags(nmaps, lmax, flags);
    const int64_t ncg = (nmaps + nc / 2 - 1) / (nc / 2);
    const size_t elem = (flags & SHT_MIXED_SPLIT_BF16) ? 3 * sizeof(uint16_t) : sizeof(float);
    return (size_t)(ncg * blocks * 2 * nc * kMxHalf) * elem;
}

int launch_leg_syn_mx(const CoefTables &c, const GeomPlan &p, const StartTable &s, const void *alm, void *aprime,
                      void *delta, DeltaLayout dl, int nmaps, uint32_t flags, hipStream_t st) {
    const bool f64s = mx_f64_sums(c.lmax, flags);
    if (flags & SHT_MIXED_SPLIT_BF16) {
        if (f64s) return launch_syn_mx_t<1, true, true>(c, p, s, alm, aprime, delta, dl, nmaps, st);
        switch (mx_col_frags(nmaps, c.lmax, flags)) {
            case 1: return launch_syn_mx_t<1, false, true>(c, p, s, alm, aprime, delta, dl, nmaps, st);
            case 2: return launch_syn_mx_t<2, false, true>(c, p, s, alm, aprime, delta, dl, nmaps, st);
            default: return launch_syn_mx_t<4, false, true>(c, p, s, alm, aprime, delta, dl, nmaps, st);
        }
    }
    if (f64s) return launch_syn_mx_t<1, true, false>(c, p, s, alm, aprime, delta, dl, nmaps, st);
    switch (mx_col_frags(nmaps, c.lmax, flags)) {
        case 1: return launch_syn_mx_t<1, false, false>(c, p, s, alm, aprime, delta, dl, nmaps, st);
        case 2: return launch_syn_mx_t<2, false, false>(c, p, s, alm, aprime, delta, dl, nmaps, st);
        default: return launch_syn_mx_t<4, false, false>(c, p, s, alm, aprime, delta, dl, nmaps, st);
    }
}

}  // namespace sht
