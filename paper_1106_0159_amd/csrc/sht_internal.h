// Internal declarations shared by the host plan code and the HIP kernels of
// libsht.so.  Nothing here is part of the public ABI (include/sht.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <initializer_list>
#include <mutex>
#include <memory>
#include <string>
#include <vector>

#include "sht.h"

namespace sht {

constexpr int kBlock = 256;          // threads per workgroup of every kernel
constexpr int kMaxFftLen = 8192;     // complex points one workgroup holds in LDS
constexpr int kMaxRadices = 16;
constexpr int kFftClasses = 4;
constexpr int kFftClassLen[kFftClasses] = {1024, 2048, 4096, 8192};
// Analysis: a workgroup of kAnaThreads threads holds up to kAnaSlotsPerThread
// ring slots per thread; an m whose slots need several workgroups writes one
// partial a_lm per group to the workspace, summed afterwards in group order.
constexpr int kAnaThreads = 256;
constexpr int kAnaSlotsPerThread = 8;

// Slots per lane: the fewest of 1 to 4 that put every slot in one workgroup,
// else kAnaSlotsPerThread.  (At 513 slots, Gauss-Legendre at lmax 1024, three
// per lane fill three waves with 9 slot-units of work where four per lane
// would take 12.)
inline int ana_slots_per_thread(int nslots) {
    return nslots <= kAnaThreads         ? 1
           : nslots <= 2 * kAnaThreads   ? 2
           : nslots <= 3 * kAnaThreads   ? 3
           : nslots <= 4 * kAnaThreads   ? 4
                                         : kAnaSlotsPerThread;
}
inline int ana_groups(int nslots) {
    const int per = kAnaThreads * ana_slots_per_thread(nslots);
    return (nslots + per - 1) / per;
}

// Rescaling of the Legendre recurrence (exponent tracking) in the plan
// kernel that finds where each recurrence enters double range.  A value is
// kept as q * 2^(kScaleBits * sc) with sc <= 0; when the carrier of a scaled
// value exceeds 2^-60 it is multiplied by 2^-kScaleBits and sc incremented.
// At sc == 0 the carrier is the value itself.
constexpr int kScaleBits = 600;
// Recurrence start positions are l = m + kStartStep * k.
constexpr int kStartStep = 8;

// Entries after the last column of alpha (zeros) and of the c-scaled a_lm in
// the workspace: kernels read blocks of coefficients up to 3 kStartStep - 1
// entries past lmax of a column without a guard.
constexpr int kCoefPad = 32;

// Mixed-precision Legendre stage: l runs in blocks of kMxL values counted
// from m (kMxL / 2 of each parity of l - m); column m has mx_blocks(lmax, m).
constexpr int kMxL = 32;
constexpr int kAnaMxGroup = 2048;  // ring pairs per workgroup of the mixed analysis
__host__ __device__ inline int mx_blocks(int lmax, int m) { return (lmax - m + kMxL) / kMxL; }

// Streams that enqueued work reading a cached table.  Each transform call,
// after enqueuing its kernels, re-records one event per (device, stream)
// and notes that stream on every table it used; a table that is evicted is
// freed once the host has waited for that event of each stream that used it
// (no device-wide synchronisation).
struct StreamUse {
    int dev;
    hipStream_t stream;
    hipEvent_t ev;
};
struct Fenced {
    mutable std::mutex fence_mu;
    mutable std::vector<StreamUse *> users;
    void note_use(StreamUse *u) const;
    void wait_users() const;  // host waits for the last recorded use on each stream
};

// Coefficient tables for one (lmax, mmax) on one device.  Packed (l, m)
// index as for a_lm.  p_lm = cfac_lm * q_lm, q_lm = alpha_lm x q_{l-1,m} - q_{l-2,m}.
struct CoefTables : Fenced {
    int dev = -1;             // device holding the tables
    int lmax = -1, mmax = -1;
    int64_t nalm = 0;
    double *alpha = nullptr;  // [nalm + kCoefPad]; alpha at l = m is 0, at l = m+1 sqrt(2m+3)
    double *cfac = nullptr;   // [nalm]
    double *mu = nullptr;     // [mmax+1]
    int64_t *mxofs = nullptr; // [mmax+2] first l-block of column m, blocks counted over m
    int64_t mxblocks = 0;     // sum over m of mx_blocks(lmax, m)
    std::vector<void *> owned;
    CoefTables() = default;
    CoefTables(const CoefTables &) = delete;
    CoefTables &operator=(const CoefTables &) = delete;
    ~CoefTables();            // waits for the streams that used it, then frees
};

// One FFT length (device view).  Points of length n are transformed in LDS
// either directly (L == n, radices of n) or by Bluestein's chirp-z method
// with the shortest 5-smooth length L >= 2n - 2.
struct FftDesc {
    int n;
    int L;
    int nrad;
    int bluestein;
    int rad[kMaxRadices];
    const double2 *tw;     // W_L[t] = exp(-2 pi i t / L), t < L
    const double2 *kern;   // Bluestein: FFT_L of the extended chirp b_t = exp(i pi t^2 / n)
                           // (b_{L-t} = b_t, zero between), divided by L
};

// Where each (m, slot) recurrence starts, for one coefficient set on one
// geometry plan: lstart[m * nslots + slot] is the first l of the block of
// kStartStep steps in which |q_lm| first reaches 2^-100 (lmax + 1 if it never
// does) and state[m * nslots + slot] = (q_{l-2}, q_{l-1}) before that step.
// A table built for (lmax', mmax') serves every lmax <= lmax', mmax <= mmax'.
struct StartTable : Fenced {
    int dev = -1;
    int lmax = -1, mmax = -1;
    int32_t *lstart = nullptr;
    double2 *state = nullptr;
    uint64_t last_use = 0;    // guarded by the cache lock
    int pins = 0;             // guarded by the cache lock; pinned tables are never evicted
    StartTable() = default;
    StartTable(const StartTable &) = delete;
    StartTable &operator=(const StartTable &) = delete;
    ~StartTable();            // waits for the streams that used it, then frees
};

// Geometry plan for one (ring set) on one device.
struct GeomPlan : Fenced {
    int dev = -1;
    int nrings = 0;
    int nslots = 0;
    int64_t npix = 0;
    int max_L = 1;
    int all_nphi_max = 1;
    // slots: ring pairs (north, south) sharing one recurrence, sorted by sin(theta)
    double *slot_x = nullptr;
    double *slot_s = nullptr;
    int32_t *slot_north = nullptr;
    int32_t *slot_south = nullptr;   // -1 when unpaired
    // rings
    double *phi0 = nullptr;
    double *weight = nullptr;        // null when the geometry has no weights
    int64_t *ofs = nullptr;
    int32_t *ring_desc = nullptr;    // index into descs
    FftDesc *descs = nullptr;
    // FFT jobs (one ring, or two rings of equal length: mirror pairs first),
    // grouped by transform-length class (L <= kFftClassLen[c]), one launch per class
    int class_count[4] = {0, 0, 0, 0};
    int2 *class_jobs[4] = {nullptr, nullptr, nullptr, nullptr};
    std::vector<void *> owned;       // device allocations to free
    // start tables built on first use by get_start; guarded by the cache lock
    mutable std::vector<std::shared_ptr<StartTable>> starts;
    GeomPlan() = default;
    GeomPlan(const GeomPlan &) = delete;
    GeomPlan &operator=(const GeomPlan &) = delete;
    ~GeomPlan();                     // waits for the streams that used it, then frees
};

// Element (map, ring, m) of a Delta array lies at
// map * s_map + ring * s_ring + m * s_m (complex entries).  Ring-major (the
// default) is [nmaps][nrings][mmax+1]; map-minor (SHT_DELTA_MAP_MINOR) is
// [nrings][mmax+1][nmaps], where the 8 maps that share a 128-byte line for one
// (ring, m) are written or read together by the mixed Legendre kernels.
struct DeltaLayout {
    int64_t s_map, s_ring, s_m;
    int map_minor;
};
inline DeltaLayout delta_layout(int nrings, int mmax, int nmaps, bool map_minor) {
    const int64_t nm = mmax + 1;
    if (map_minor) return DeltaLayout{1, nm * nmaps, (int64_t)nmaps, 1};
    return DeltaLayout{(int64_t)nrings * nm, nm, 1, 0};
}

// The mixed-precision kernels pay from kMxMinMaps maps on (a wave's
// matrix-core columns hold 8 maps, and FP32 vector arithmetic runs no faster
// than FP64 here); with fewer maps SHT_MIXED runs the FP64 kernels, faster
// there and at least as accurate.  Map-minor Delta in the stage calls always
// takes the mixed kernels (the FP64 Legendre kernels use ring-major Delta).
constexpr int kMxMinMaps = 8;
inline bool use_mx(uint32_t flags, int nmaps) {
    return (flags & SHT_MIXED) && (nmaps >= kMxMinMaps || (flags & SHT_DELTA_MAP_MINOR));
}

// Delta layout of sht_alm2map's workspace: with SHT_MIXED map-minor from 8
// maps on (the matrix-core kernel then stores whole 128-byte lines per (ring,
// m), which saves more than the ring FFT loses on its strided reads; with
// fewer maps there are no whole lines to gain, and the ring-major FFT
// transforms a mirror pair per workgroup instead of one ring).
inline DeltaLayout alm2map_layout(int nrings, int mmax, int nmaps, uint32_t flags) {
    return delta_layout(nrings, mmax, nmaps, use_mx(flags & ~SHT_DELTA_MAP_MINOR, nmaps));
}

// One length class of one plan's ring stage as the ring kernels read it: a
// kernel argument for a single call, or an entry of a batch's device table
// (the jobs of every request and class in one launch per class).  Ring-major
// Delta unless dl.map_minor; nmaps maps per job (1 in batches).  fold_rows
// and ph_tab: the LDS layout of this entry (rows of phased terms, phase tables).
struct RingPlan {
    int mmax, nmaps, njobs, fold_rows, ph_tab;
    int64_t npix;
    DeltaLayout dl;
    const int2 *jobs;          // [njobs] (ring a, ring b or -1) of this class
    const int32_t *ring_desc;  // [nrings] index into descs
    const FftDesc *descs;
    const double *phi0, *weight;
    const int64_t *ofs;
    const double2 *din;  // synthesis: Delta read
    double *mout;        // synthesis: map written
    const double *min;   // analysis: map read
    double2 *dout;       // analysis: Delta written
};

// Validated, normalised copy of the caller's geometry.
struct HostGeom {
    int nrings = 0;
    std::vector<double> theta, phi0, weight;
    std::vector<int32_t> nphi;
    std::vector<int64_t> ofs;
    bool has_weight = false;
    int64_t npix = 0;
};

int validate_geom(const sht_geom *g, bool need_weight, HostGeom *out);
// Number of recurrence slots (mirror pairs plus unpaired rings) of a geometry.
int count_slots(const HostGeom &h);
int validate_sizes(int lmax, int mmax, int nmaps);

// Plan lookup (builds on first use, outside the cache lock).  Thread safe.
// A call holds the references for as long as it uses the tables: an entry
// evicted from a cache meanwhile is freed only when its last reference goes,
// after the host has waited for the last recorded use of each stream that
// enqueued work reading it (note_uses), so kernels already enqueued with it
// finish first.  Pinned entries (pin_plan) are never evicted.
using CoefRef = std::shared_ptr<const CoefTables>;
using GeomRef = std::shared_ptr<const GeomPlan>;
using StartRef = std::shared_ptr<const StartTable>;
int get_coef(int lmax, int mmax, CoefRef *out);
int get_geom(const HostGeom &hg, int mmax_for_fft, GeomRef *out);
// Start table of (c, p), built on the stream st and waited for on first use.
int get_start(const CoefTables &c, const GeomRef &p, hipStream_t st, StartRef *out);
// Records the use event of stream st (re-recorded per call) and notes st on
// the given tables; nothing is recorded while st is capturing a graph (a
// captured graph needs its plan pinned instead).
int note_uses(hipStream_t st, std::initializer_list<const Fenced *> tables);
// Adds delta (+1 or -1) to the pin counts of the resident tables of
// (lmax, mmax, geometry); SHT_ENOPLAN if they are not resident (or, for -1,
// not pinned).
int pin_plan(int lmax, int mmax, const HostGeom &hg, int delta);
// The pinned resident tables of (lmax, mmax, geometry), looked up without
// building, evicting or allocating anything; SHT_ENOPLAN if there are none.
int find_pinned(int lmax, int mmax, const HostGeom &hg, CoefRef *c, GeomRef *p, StartRef *s);

// Runs launch(i, stream_i) for i < n (n <= kSideStreams + 1): piece 0 on st,
// the others on the library's side streams of the current device (default
// priority), each ordered after the work already enqueued on st; st then
// waits for all of them, so the caller sees one ordered stream.
constexpr int kSideStreams = 3;
int fork_join(hipStream_t st, int n, const std::function<int(int, hipStream_t)> &launch);

void set_hip_error(hipError_t e, const char *where);
#define SHT_HIP(call)                                        \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) {                              \
            ::sht::set_hip_error(e_, #call);                 \
            return SHT_EDEVICE;                              \
        }                                                    \
    } while (0)

// Arguments of the FP64 Legendre tiles (k_legendre.hip) for one (lmax, mmax,
// geometry): synthesis reads the c-scaled a_lm (ap) and writes ring-major
// Delta; analysis reads Delta and writes a_lm (or per-group partials).
struct SynArgs {
    int lmax, mmax, nslots, nrings;
    int64_t nalm;
    const double2 *__restrict__ ap;
    const double *__restrict__ alpha;
    const int32_t *__restrict__ lstart;
    const double2 *__restrict__ state;
    const double *__restrict__ sx;
    const int32_t *__restrict__ rn;
    const int32_t *__restrict__ rsouth;
    double2 *__restrict__ delta;
};

struct AnaArgs {
    int lmax, mmax, nslots, nrings;
    int64_t nalm;
    const double2 *__restrict__ delta;
    const double *__restrict__ alpha;
    const double *__restrict__ cfac;
    const int32_t *__restrict__ lstart;
    const double2 *__restrict__ state;
    const double *__restrict__ sx;
    const int32_t *__restrict__ rn;
    const int32_t *__restrict__ rsouth;
    double2 *__restrict__ alm;
    double2 *__restrict__ part;
};

// One request of an uneven batch (sht_batch_*), as the persistent Legendre
// kernel reads it.  kind 0: synthesis, in wave units (m, tile of 64 T
// slots), nunits = (mmax+1) * tiles; kind 1: analysis, shape 0 one wave per
// m holding every slot (nslots <= 64 T), shape 1 one workgroup per (m, group
// of 256 T slots), groups > 1 writing partials summed by a combine kernel.
struct BatchReq {
    SynArgs syn;
    AnaArgs ana;
    const double2 *alm_in;  // synthesis: the caller's a_lm (prescaled into syn.ap)
    int kind, shape, T, tiles, nunits, groups;
};
// One work item: request `req`, first unit u0 (wave units: the item's four
// waves take u0 .. u0+3; group shape: u0 = m * groups + group).
struct BatchItem {
    int32_t req, u0;
};

// Kernel launchers (k_legendre.hip, k_ring_fft.hip).  They enqueue only.
int launch_leg_start(const CoefTables &c, const GeomPlan &p, int32_t *lstart, void *state, hipStream_t st);
int launch_prescale(const CoefTables &c, const void *alm, void *aprime, int nmaps, hipStream_t st);
int launch_leg_syn(const CoefTables &c, const GeomPlan &p, const StartTable &s, const void *aprime,
                   void *delta, int nmaps, hipStream_t st);
int launch_leg_ana(const CoefTables &c, const GeomPlan &p, const StartTable &s, const void *delta,
                   void *alm, int nmaps, void *partials, hipStream_t st);
// Mixed precision (SHT_MIXED, k_legendre_mx.hip): prescale of a_lm into FP32
// block tiles of mx_aprime_bytes(...) bytes, then the synthesis contraction.
int mx_col_frags(int nmaps, int lmax, uint32_t flags);
size_t mx_aprime_bytes(int lmax, int mmax, int nmaps, uint32_t flags);
int launch_leg_syn_mx(const CoefTables &c, const GeomPlan &p, const StartTable &s, const void *alm,
                      void *aprime, void *delta, DeltaLayout dl, int nmaps, uint32_t flags, hipStream_t st);
int launch_leg_ana_mx(const CoefTables &c, const GeomPlan &p, const StartTable &s, const void *delta,
                      DeltaLayout dl, void *alm, int nmaps, void *partials, hipStream_t st);
// Uneven batches: the persistent Legendre kernel over the items (queue head
// *head reset to 0 first, in the same launch sequence), the prescale of
// every synthesis request, and the combine of analysis requests with
// several groups.  leg_batch_grid: resident workgroups of the persistent
// kernel on the current device.
int leg_batch_grid(int *grid);
int launch_leg_batch(const BatchReq *reqs, const BatchItem *items, int nitems, int *head, int grid, hipStream_t st);
int launch_prescale_batch(const BatchReq *reqs, const int32_t *syn_reqs, int nsyn, int max_chunks, hipStream_t st);
int launch_combine_batch(const BatchReq *reqs, const int32_t *comb_reqs, int ncomb, int max_chunks, hipStream_t st);
constexpr int kBatchMaxSynT = 4, kBatchMaxAnaT = 4;

// a_lm = c_lm * (sum of the per-group partials, groups in order); Im a_l0 = 0.
int launch_ana_combine(const CoefTables &c, int nmaps, int groups, const void *partials, void *alm,
                       hipStream_t st);
// Ring stages: the length classes run concurrently on side streams of st
// (fork_join), or with fork = false one after another on st (no side streams).
int launch_fft_syn(const GeomPlan &p, int mmax, const void *delta, DeltaLayout dl, double *map, int nmaps,
                   hipStream_t st, bool fork = true);
int launch_fft_ana(const GeomPlan &p, int mmax, const double *map, void *delta, DeltaLayout dl, int nmaps,
                   hipStream_t st, bool fork = true);

// Ring stages of a batch: for each length class c, one launch over the
// entries `jobs[c]` = (plan index into `plans`, job index of that plan),
// with the LDS bytes the largest entry of the class needs.
struct RingBatch {
    const RingPlan *plans = nullptr;  // device table
    const int2 *jobs[kFftClasses] = {nullptr, nullptr, nullptr, nullptr};
    int njobs[kFftClasses] = {0, 0, 0, 0};
    size_t lds[kFftClasses] = {0, 0, 0, 0};
};
// Host side: the RingPlan of class c of plan p for a call (din/mout or
// min/dout filled by the caller), and the LDS bytes it needs.
RingPlan ring_plan(const GeomPlan &p, int c, int mmax, int nmaps, DeltaLayout dl, bool synthesis, size_t *lds);
int launch_fft_syn_batch(const RingBatch &b, hipStream_t st);
int launch_fft_ana_batch(const RingBatch &b, hipStream_t st);

// sht_alm2map's host-side validation (sizes, flags, geometry, alm and map
// pointers); sets the workspace bytes the call needs.
int check_alm2map(int lmax, int mmax, const sht_geom *g, const void *alm, const double *map, int nmaps,
                  uint32_t flags, HostGeom *h, size_t *ws_bytes_needed);
// The kernels of sht_alm2map on stream st: Legendre synthesis into the
// workspace Delta (aprime: the workspace's aux part), then the ring FFTs,
// their length classes on side streams of st (fork) or one after another on st.
int enqueue_alm2map(const CoefTables &c, const GeomPlan &p, const StartTable &s, const void *alm, void *aprime,
                    void *delta, DeltaLayout dl, double *map, int nmaps, uint32_t flags, hipStream_t st, bool fork);
// Workspace offset of the aux part (after Delta), for the layout [Delta][aux].
size_t ws_aux_offset(int nrings, int mmax, int nmaps);

inline int64_t nalm_of(int lmax, int mmax) {
    return (int64_t)(mmax + 1) * (2 * (int64_t)lmax + 2 - mmax) / 2;
}

}  // namespace sht
