// Host side of libsht.so: argument validation, recurrence-coefficient tables,
// ring pairing, FFT plans and the per-device plan caches.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <unordered_map>
#include <tuple>

#include "sht_internal.h"

namespace sht {

static thread_local std::string g_last_hip_error;

void set_hip_error(hipError_t e, const char *where) {
    g_last_hip_error = std::string(hipGetErrorString(e)) + " (" + where + ")";
}

const char *last_hip_error() { return g_last_hip_error.c_str(); }

int validate_sizes(int lmax, int mmax, int nmaps) {
    if (lmax < 0 || mmax < 0 || mmax > lmax || nmaps < 1) return SHT_EINVAL;
    // kernels index l in int and a_lm in int64; keep l*l and the LDS-resident
    // FFT comfortably in range
    if (lmax > 32768) return SHT_EUNSUPPORTED;
    return SHT_OK;
}

int validate_geom(const sht_geom *g, bool need_weight, HostGeom *out) {
    if (!g || g->nrings < 1 || !g->theta || !g->nphi || !g->phi0) return SHT_EINVAL;
    if (need_weight && !g->weight) return SHT_EINVAL;
    const int n = g->nrings;
    HostGeom h;
    h.nrings = n;
    h.theta.assign(g->theta, g->theta + n);
    h.nphi.assign(g->nphi, g->nphi + n);
    h.phi0.assign(g->phi0, g->phi0 + n);
    h.has_weight = g->weight != nullptr;
    if (h.has_weight) h.weight.assign(g->weight, g->weight + n);
    h.ofs.resize(n);
    int64_t acc = 0;
    for (int r = 0; r < n; ++r) {
        const double t = h.theta[r];
        if (!(t >= 0.0 && t <= M_PI)) return SHT_EINVAL;  // also rejects NaN
        if (h.nphi[r] < 1 || !std::isfinite(h.phi0[r])) return SHT_EINVAL;
        if (h.has_weight && !std::isfinite(h.weight[r])) return SHT_EINVAL;
        if (g->ofs) {
            h.ofs[r] = g->ofs[r];
            if (h.ofs[r] < 0) return SHT_EINVAL;
        } else {
            h.ofs[r] = acc;
            acc += h.nphi[r];
        }
    }
    // ring pixel ranges must not overlap (checked in offset order; rings are
    // usually given in that order already, which needs no sort)
    std::vector<int> ord(n);
    for (int r = 0; r < n; ++r) ord[r] = r;
    if (!std::is_sorted(h.ofs.begin(), h.ofs.end()))
        std::sort(ord.begin(), ord.end(), [&](int a, int b) { return h.ofs[a] < h.ofs[b]; });
    int64_t npix = 0;
    for (int i = 0; i < n; ++i) {
        const int r = ord[i];
        if (i > 0) {
            const int q = ord[i - 1];
            if (h.ofs[q] + h.nphi[q] > h.ofs[r]) return SHT_EINVAL;
        }
        npix = std::max<int64_t>(npix, h.ofs[r] + h.nphi[r]);
    }
    h.npix = npix;
    *out = std::move(h);
    return SHT_OK;
}

// ------------------------------------------------------------------ device memory helpers
// Every plan-table allocation goes through dev_alloc / dev_free, which keep
// the bytes the caches hold on the devices (sht_plan_cache_bytes).
static std::mutex g_bytes_mu;
static auto &g_sizes = *new std::unordered_map<void *, size_t>();
static size_t g_plan_bytes = 0;

// Test hook for the failure paths of plan builds: with SHT_TEST_FAIL_ALLOC=n
// in the environment, the n-th plan-table allocation counted from when that
// value was first seen fails as if the device were out of memory.  Read only
// here, during plan builds.
static bool injected_failure() {
    static std::mutex mu;
    static std::string seen;
    static long count = 0;
    const char *v = std::getenv("SHT_TEST_FAIL_ALLOC");
    std::lock_guard<std::mutex> lk(mu);
    if (!v || !*v) {
        seen.clear();
        count = 0;
        return false;
    }
    if (seen != v) {
        seen = v;
        count = 0;
    }
    return ++count == std::strtol(v, nullptr, 10);
}

static bool dev_alloc(void **p, size_t bytes) {
    if (injected_failure()) return false;
    if (hipMalloc(p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    std::lock_guard<std::mutex> lk(g_bytes_mu);
    g_sizes[*p] = bytes;
    g_plan_bytes += bytes;
    return true;
}

static void dev_free(void *p) {
    {
        std::lock_guard<std::mutex> lk(g_bytes_mu);
        auto it = g_sizes.find(p);
        if (it != g_sizes.end()) {
            g_plan_bytes -= it->second;
            g_sizes.erase(it);
        }
    }
    (void)hipFree(p);
}

size_t plan_cache_bytes() {
    std::lock_guard<std::mutex> lk(g_bytes_mu);
    return g_plan_bytes;
}

template <class T>
static int upload(const std::vector<T> &v, T **dst, std::vector<void *> &owned) {
    void *p = nullptr;
    const size_t bytes = std::max<size_t>(1, v.size()) * sizeof(T);
    if (!dev_alloc(&p, bytes)) return SHT_ENOMEM;
    owned.push_back(p);
    *dst = static_cast<T *>(p);  // set before the copy: a failed copy still hands the allocation back
    if (!v.empty()) SHT_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return SHT_OK;
}

static int current_device(int *dev) {
    SHT_HIP(hipGetDevice(dev));
    return SHT_OK;
}

// ------------------------------------------------------------------ use fences
static std::mutex g_use_mu;
static auto &g_uses = *new std::map<std::pair<int, hipStream_t>, StreamUse *>();

void Fenced::note_use(StreamUse *u) const {
    std::lock_guard<std::mutex> lk(fence_mu);
    for (StreamUse *v : users)
        if (v == u) return;
    users.push_back(u);
}

void Fenced::wait_users() const {
    std::lock_guard<std::mutex> lk(fence_mu);
    for (StreamUse *u : users) (void)hipEventSynchronize(u->ev);
    users.clear();
}

int note_uses(hipStream_t st, std::initializer_list<const Fenced *> tables) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    SHT_HIP(hipStreamIsCapturing(st, &cs));
    if (cs != hipStreamCaptureStatusNone) return SHT_OK;  // captured graphs pin their plans
    int dev = 0;
    SHT_HIP(hipGetDevice(&dev));
    StreamUse *u = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_use_mu);
        auto &slot = g_uses[std::make_pair(dev, st)];
        if (!slot) {
            hipEvent_t ev = nullptr;
            SHT_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            slot = new StreamUse{dev, st, ev};
        }
        u = slot;
        SHT_HIP(hipEventRecord(u->ev, st));
    }
    for (const Fenced *t : tables)
        if (t) t->note_use(u);
    return SHT_OK;
}

// Frees device allocations of a table on its device once the work that used
// it is done (see Fenced).
static void release_device(int dev, const Fenced &f, std::vector<void *> &ptrs) {
    f.wait_users();
    if (ptrs.empty()) return;
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (dev >= 0 && cur != dev) (void)hipSetDevice(dev);
    for (void *q : ptrs) dev_free(q);
    ptrs.clear();
    if (dev >= 0 && cur >= 0 && cur != dev) (void)hipSetDevice(cur);
}

CoefTables::~CoefTables() { release_device(dev, *this, owned); }

StartTable::~StartTable() {
    std::vector<void *> v;
    if (lstart) v.push_back(lstart);
    if (state) v.push_back(state);
    release_device(dev, *this, v);
}

GeomPlan::~GeomPlan() {
    starts.clear();  // each start table frees itself when its last user is done
    release_device(dev, *this, owned);
}

// ------------------------------------------------------------------ coefficient tables
// For one m: beta_l = sqrt((4l^2-1)/(l^2-m^2)) (eq. betaDef), c_m = c_{m+1} = 1,
// c_l = (beta_l/beta_{l-1}) c_{l-2}, alpha_l = beta_l c_{l-1}/c_l.  Then
// p_l = c_l q_l turns eq. assLegRec into q_l = alpha_l x q_{l-1} - q_{l-2}.
// alpha is derived from the stored (rounded) c so that the effective
// recurrence coefficients carry only their own rounding.
static void coef_column(int lmax, int m, double *alpha, double *cfac) {
    const int n = lmax - m + 1;
    std::vector<long double> beta(n + 1, 0.0L);
    for (int l = m + 1; l <= lmax; ++l) {
        const long double L = l, M = m;
        beta[l - m] = sqrtl((4.0L * L * L - 1.0L) / (L * L - M * M));
    }
    cfac[0] = 1.0;
    alpha[0] = 0.0;
    if (lmax >= m + 1) {
        cfac[1] = 1.0;
        alpha[1] = (double)beta[1];  // sqrt(2m+3), eq. pm1m
    }
    for (int l = m + 2; l <= lmax; ++l) {
        const int i = l - m;
        const long double c = beta[i] / beta[i - 1] * (long double)cfac[i - 2];
        cfac[i] = (double)c;
        alpha[i] = (double)(beta[i] * (long double)cfac[i - 1] / (long double)cfac[i]);
    }
}

// The caches are created on first use and never destroyed at process exit
// (their destructors would call into the HIP runtime after it has gone);
// sht_shutdown empties them.  Tables are built outside the cache lock (a
// concurrent build of the same key keeps the first one inserted), and
// evicted entries are dropped after the lock is released, so that no call
// waits on another's build or free.
struct CoefEntry {
    std::shared_ptr<CoefTables> t;
    uint64_t last_use = 0;
    int pins = 0;
};
static std::mutex g_mu;
static uint64_t g_clock = 0;
static auto &g_coef = *new std::map<std::tuple<int, int, int>, CoefEntry>();
// cache capacities (entries per process); sht_plan_cache_limits changes them
static size_t g_max_coef = 8;
static size_t g_max_geom = 32;

static int build_coef(int dev, int lmax, int mmax, std::shared_ptr<CoefTables> *out) {
    auto t = std::make_shared<CoefTables>();
    t->dev = dev;
    const int64_t na = nalm_of(lmax, mmax);
    std::vector<double> alpha(na), cfac(na), mu(mmax + 1);
    for (int m = 0; m <= mmax; ++m) {
        const int64_t b = (int64_t)m * (2 * (int64_t)lmax + 1 - m) / 2 + m;
        coef_column(lmax, m, alpha.data() + b, cfac.data() + b);
    }
    // mu_m of eq. pmm: mu_0 = 1/sqrt(4 pi), mu_m = mu_{m-1} sqrt((2m+1)/(2m))
    long double v = 1.0L / sqrtl(4.0L * 3.141592653589793238462643383279502884L);
    mu[0] = (double)v;
    for (int m = 1; m <= mmax; ++m) {
        v *= sqrtl((long double)(2 * m + 1) / (long double)(2 * m));
        mu[m] = (double)v;
    }
    t->lmax = lmax;
    t->mmax = mmax;
    t->nalm = na;
    alpha.resize(na + kCoefPad, 0.0);  // kernels may read past the last column
    std::vector<int64_t> mxofs(mmax + 2, 0);
    for (int m = 0; m <= mmax; ++m) mxofs[m + 1] = mxofs[m] + mx_blocks(lmax, m);
    t->mxblocks = mxofs[mmax + 1];
    int rc;
    if ((rc = upload(alpha, &t->alpha, t->owned)) || (rc = upload(cfac, &t->cfac, t->owned)) ||
        (rc = upload(mu, &t->mu, t->owned)) || (rc = upload(mxofs, &t->mxofs, t->owned)))
        return rc;  // t frees what was uploaded
    *out = std::move(t);
    return SHT_OK;
}

int get_coef(int lmax, int mmax, CoefRef *out) {
    int dev = 0;
    int rc = current_device(&dev);
    if (rc) return rc;
    const auto key = std::make_tuple(dev, lmax, mmax);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_coef.find(key);
        if (it != g_coef.end()) {
            it->second.last_use = ++g_clock;
            *out = it->second.t;
            return SHT_OK;
        }
    }
    std::shared_ptr<CoefTables> t;
    if ((rc = build_coef(dev, lmax, mmax, &t))) return rc;
    std::vector<std::shared_ptr<CoefTables>> dropped;  // freed after the lock is released
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_coef.find(key);
    if (it != g_coef.end()) {  // built meanwhile by another call: keep that one
        it->second.last_use = ++g_clock;
        *out = it->second.t;
        dropped.push_back(std::move(t));
        return SHT_OK;
    }
    // make room: least recently used unpinned entries first
    while (g_coef.size() >= g_max_coef) {
        auto lru = g_coef.end();
        for (auto e = g_coef.begin(); e != g_coef.end(); ++e)
            if (e->second.pins == 0 && (lru == g_coef.end() || e->second.last_use < lru->second.last_use)) lru = e;
        if (lru == g_coef.end()) break;  // all pinned
        dropped.push_back(std::move(lru->second.t));
        g_coef.erase(lru);
    }
    g_coef[key] = CoefEntry{t, ++g_clock, 0};
    *out = t;
    return SHT_OK;
}

// ------------------------------------------------------------------ FFT plans
using cld = std::complex<long double>;
static const long double kPiL = 3.141592653589793238462643383279502884L;

static bool factor_small(int n, std::vector<int> &rad) {
    rad.clear();
    while (n % 8 == 0) { rad.push_back(8); n /= 8; }
    while (n % 4 == 0) { rad.push_back(4); n /= 4; }
    while (n % 2 == 0) { rad.push_back(2); n /= 2; }
    for (int p : {3, 5}) {
        while (n % p == 0) { rad.push_back(p); n /= p; }
    }
    return n == 1 && (int)rad.size() <= kMaxRadices;
}

// All prime factors: 8, 4, 2, 3, 5 first (the fixed-radix stages), then the
// other primes ascending (direct R-term stages).
static bool factor_all(int n, std::vector<int> &rad) {
    factor_small(n, rad);
    int r = n;
    for (int f : rad) r /= f;
    for (int p = 7; (long long)p * p <= r; p += 2)
        while (r % p == 0) { rad.push_back(p); r /= p; }
    if (r > 1) rad.push_back(r);
    return (int)rad.size() <= kMaxRadices;
}

// Cost of a prime-radix stage in flops per point and unit of R, against 400
// per point of Bluestein's length: of the weights 12, 6, 4 and 3 the last
// timed best with the mirror-paired stage (ring stages at HEALPix 1024,
// one map and 64 maps).
constexpr double kPrimeCost = 3.0;

static bool smooth5(int n) {
    for (int p : {2, 3, 5})
        while (n % p == 0) n /= p;
    return n == 1;
}

// Forward DFT (sign -1) of a 5-smooth length in long double, by recursive
// decimation in time over the factors 2, 3, 5.
static void host_fft_smooth(std::vector<cld> &a) {
    const size_t n = a.size();
    if (n == 1) return;
    size_t p = (n % 2 == 0) ? 2 : (n % 3 == 0) ? 3 : 5;
    const size_t m = n / p;
    std::vector<std::vector<cld>> sub(p, std::vector<cld>(m));
    for (size_t j = 0; j < m; ++j)
        for (size_t r = 0; r < p; ++r) sub[r][j] = a[j * p + r];
    for (auto &v : sub) host_fft_smooth(v);
    for (size_t k = 0; k < n; ++k) {
        cld acc(0, 0);
        for (size_t r = 0; r < p; ++r) {
            const long double ang = -2.0L * kPiL * (long double)((r * k) % n) / (long double)n;
            acc += sub[r][k % m] * cld(cosl(ang), sinl(ang));
        }
        a[k] = acc;
    }
}

struct FftCache {
    std::map<int, double2 *> twiddles;      // by L
    std::map<int, FftDesc> descs;           // by n
    std::vector<void *> owned;
};
static auto &g_fft = *new std::map<int, std::unique_ptr<FftCache>>();  // by device
static std::mutex g_fft_mu;  // guards g_fft and its entries

// What one geometry build added to an FftCache, so that a failed build can
// take it all out again (the cache then holds only complete entries).
struct FftAdded {
    std::vector<int> lengths, twiddle_L;
    std::vector<void *> ptrs;
};
static void fft_rollback(FftCache &fc, FftAdded &a) {
    for (int n : a.lengths) fc.descs.erase(n);
    for (int L : a.twiddle_L) fc.twiddles.erase(L);
    for (void *p : a.ptrs) {
        fc.owned.erase(std::remove(fc.owned.begin(), fc.owned.end(), p), fc.owned.end());
        dev_free(p);
    }
    a = FftAdded{};
}

static int twiddle_table(FftCache &fc, int L, const double2 **out, FftAdded &added) {
    auto it = fc.twiddles.find(L);
    if (it != fc.twiddles.end()) {
        *out = it->second;
        return SHT_OK;
    }
    std::vector<double2> w(L);
    for (int t = 0; t < L; ++t) {
        const long double a = -2.0L * kPiL * (long double)t / (long double)L;
        w[t] = make_double2((double)cosl(a), (double)sinl(a));
    }
    double2 *d = nullptr;
    const size_t before = fc.owned.size();
    int rc = upload(w, &d, fc.owned);
    if (fc.owned.size() > before) added.ptrs.push_back(fc.owned.back());
    if (rc) return rc;
    fc.twiddles[L] = d;
    added.twiddle_L.push_back(L);
    *out = d;
    return SHT_OK;
}

static int fft_desc(FftCache &fc, int n, FftDesc *out, FftAdded &added) {
    auto it = fc.descs.find(n);
    if (it != fc.descs.end()) {
        *out = it->second;
        return SHT_OK;
    }
    FftDesc d;
    std::memset(&d, 0, sizeof(d));
    d.n = n;
    std::vector<int> rad;
    int rc;
    // Direct transform of length n when it is 5-smooth, or when its direct
    // R-term stages (with the mirror-paired inputs about kPrimeCost R flops
    // per point each) cost less than Bluestein's two transforms of length L
    // (taken as 400 flops per point of L), or when Bluestein's L would not
    // fit the largest class.
    // Bluestein's cyclic convolution takes the chirp at offsets -(n-1) ..
    // n-1.  The chirp is even in its offset, so the one pair of offsets that
    // share an index modulo L = 2n - 2, +-(n-1), needs the same value there:
    // L >= 2n - 2 is exact (L = 4096 for n = 2049 = 2 lmax + 1 at lmax 1024,
    // where L >= 2n - 1 would take 4320 and the 8192 class).
    int Lb = n > 1 ? 2 * n - 2 : 1;
    while (!smooth5(Lb)) ++Lb;
    std::vector<int> all;
    const bool all_ok = factor_all(n, all);
    double direct = 0.0;
    for (int f : all) direct += f > 5 ? kPrimeCost * f * n : 0.0;
    if (factor_small(n, rad)) {
        d.L = n;
        d.bluestein = 0;
    } else if (all_ok && (Lb > kMaxFftLen || direct <= 400.0 * Lb)) {
        rad = all;
        d.L = n;
        d.bluestein = 0;
    } else {
        const int L = Lb;
        d.L = L;
        d.bluestein = 1;
        factor_small(L, rad);
        // chirp b_t = exp(i pi t^2 / n), angle reduced exactly: t^2 mod 2n
        // (the kernels compute b_t themselves; the plan keeps the spectrum of
        // its extension to length L: b at t and at L - t, which are one index
        // for t = n - 1 when L = 2n - 2, with the same value)
        std::vector<cld> ext(L, cld(0, 0));
        for (int t = 0; t < n; ++t) {
            const long long q = (long long)t * t % (2LL * n);
            const long double a = kPiL * (long double)q / (long double)n;
            const cld v(cosl(a), sinl(a));
            ext[t] = v;
            if (t > 0) ext[L - t] = v;
        }
        host_fft_smooth(ext);
        std::vector<double2> k(L);
        for (int t = 0; t < L; ++t)
            k[t] = make_double2((double)(ext[t].real() / L), (double)(ext[t].imag() / L));
        double2 *dk = nullptr;
        rc = upload(k, &dk, fc.owned);
        if (dk) added.ptrs.push_back(dk);
        if (rc) return rc;
        d.kern = dk;
    }
    if (d.L > kMaxFftLen) return SHT_EUNSUPPORTED;
    // Stockham stages may come in any order: with two radix-8/4 factors or
    // more, one of them goes last, so that both the first and the last stage
    // can move their points through registers (pixels in, pixels out)
    // instead of LDS.
    {
        int n84 = 0, last84 = -1;
        for (int i = 0; i < (int)rad.size(); ++i)
            if (rad[i] == 8 || rad[i] == 4) ++n84, last84 = i;
        if (n84 >= 2 && last84 != (int)rad.size() - 1) {
            const int r = rad[last84];
            rad.erase(rad.begin() + last84);
            rad.push_back(r);
        }
    }
    d.nrad = (int)rad.size();
    for (int i = 0; i < d.nrad; ++i) d.rad[i] = rad[i];
    if ((rc = twiddle_table(fc, d.L, &d.tw, added))) return rc;
    fc.descs[n] = d;
    added.lengths.push_back(n);
    *out = d;
    return SHT_OK;
}

// ------------------------------------------------------------------ geometry plans
struct GeomEntry {
    int dev;
    HostGeom key;
    std::shared_ptr<GeomPlan> plan;
    uint64_t last_use;
    int pins;
};
static auto &g_geom = *new std::vector<GeomEntry>();

static bool same_geom(const HostGeom &a, const HostGeom &b) {
    return a.nrings == b.nrings && a.has_weight == b.has_weight && a.theta == b.theta &&
           a.nphi == b.nphi && a.phi0 == b.phi0 && a.ofs == b.ofs && a.weight == b.weight;
}

// Mirror pairs: rings r, r' with |theta_r + theta_r' - pi| <= kMirrorTol,
// the sum taken exactly in long double, share one recurrence
// (lambda_lm(-x) = (-1)^(l+m) lambda_lm(x)); the northern ring's cos and sin
// are used for both.  Two ulp of pi: a southern colatitude rounded from
// pi - theta_n (once, or as double(pi) - theta_n) is within it, and a ring any
// further off mirror is its own slot, evaluated at its own colatitude.
constexpr long double kMirrorTol = 0x1p-50L;  // 2 ulp of pi = 8.9e-16 rad
static void build_slots(const HostGeom &h, std::vector<double> &sx, std::vector<double> &ss,
                        std::vector<int32_t> &sn, std::vector<int32_t> &sso) {
    const int n = h.nrings;
    std::vector<int> ord(n);
    for (int r = 0; r < n; ++r) ord[r] = r;
    std::sort(ord.begin(), ord.end(), [&](int a, int b) {
        return h.theta[a] < h.theta[b] || (h.theta[a] == h.theta[b] && a < b);
    });
    struct S { double x, s; int n, so; };
    std::vector<S> slots;
    int i = 0, j = n - 1;
    while (i <= j) {
        const int a = ord[i], b = ord[j];
        if (i == j) {
            slots.push_back({std::cos(h.theta[a]), std::sin(h.theta[a]), a, -1});
            break;
        }
        const long double d = ((long double)h.theta[a] + (long double)h.theta[b]) - kPiL;
        if (fabsl(d) <= kMirrorTol) {
            slots.push_back({std::cos(h.theta[a]), std::sin(h.theta[a]), a, b});
            ++i;
            --j;
        } else if (d < 0) {
            slots.push_back({std::cos(h.theta[a]), std::sin(h.theta[a]), a, -1});
            ++i;
        } else {
            slots.push_back({std::cos(h.theta[b]), std::sin(h.theta[b]), b, -1});
            --j;
        }
    }
    // polar slots first: neighbouring lanes then leave the rescaled regime together
    std::stable_sort(slots.begin(), slots.end(), [](const S &p, const S &q) { return p.s < q.s; });
    for (const S &s : slots) {
        sx.push_back(s.x);
        ss.push_back(s.s);
        sn.push_back(s.n);
        sso.push_back(s.so);
    }
}

// The slot count depends on the colatitudes only; the last few results are
// remembered so that sizing the workspace does not pair the rings each call.
int count_slots(const HostGeom &h) {
    static std::mutex mu;
    static auto &memo = *new std::vector<std::pair<std::vector<double>, int>>();
    {
        std::lock_guard<std::mutex> lk(mu);
        for (const auto &e : memo)
            if (e.first == h.theta) return e.second;
    }
    std::vector<double> sx, ss;
    std::vector<int32_t> sn, sso;
    build_slots(h, sx, ss, sn, sso);
    const int n = (int)sx.size();
    std::lock_guard<std::mutex> lk(mu);
    if (memo.size() >= 256) memo.erase(memo.begin());
    memo.emplace_back(h.theta, n);
    return n;
}

static GeomEntry *find_geom_locked(int dev, const HostGeom &hg) {
    for (auto &e : g_geom)
        if (e.dev == dev && same_geom(e.key, hg)) return &e;
    return nullptr;
}

static int build_geom(int dev, const HostGeom &hg, std::shared_ptr<GeomPlan> *out);

int get_geom(const HostGeom &hg, int /*mmax_for_fft*/, GeomRef *out) {
    int dev = 0;
    int rc = current_device(&dev);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (GeomEntry *e = find_geom_locked(dev, hg)) {
            e->last_use = ++g_clock;
            *out = e->plan;
            return SHT_OK;
        }
    }
    std::shared_ptr<GeomPlan> plan;
    if ((rc = build_geom(dev, hg, &plan))) return rc;
    std::vector<std::shared_ptr<GeomPlan>> dropped;  // freed after the lock is released
    std::lock_guard<std::mutex> lk(g_mu);
    if (GeomEntry *e = find_geom_locked(dev, hg)) {  // built meanwhile by another call
        e->last_use = ++g_clock;
        *out = e->plan;
        dropped.push_back(std::move(plan));
        return SHT_OK;
    }
    while (g_geom.size() >= g_max_geom) {
        // the least recently used unpinned plan goes; it is freed when its last user is done
        auto lru = g_geom.end();
        for (auto e = g_geom.begin(); e != g_geom.end(); ++e)
            if (e->pins == 0 && (lru == g_geom.end() || e->last_use < lru->last_use)) lru = e;
        if (lru == g_geom.end()) break;  // all pinned
        dropped.push_back(std::move(lru->plan));
        g_geom.erase(lru);
    }
    g_geom.push_back(GeomEntry{dev, hg, plan, ++g_clock, 0});
    *out = plan;
    return SHT_OK;
}

static int build_geom(int dev, const HostGeom &hg, std::shared_ptr<GeomPlan> *out) {
    int rc;
    auto plan = std::make_shared<GeomPlan>();
    GeomPlan &p = *plan;  // on an error return below, plan frees what was uploaded
    p.dev = dev;
    p.nrings = hg.nrings;
    p.npix = hg.npix;
    std::vector<double> sx, ss;
    std::vector<int32_t> sn, sso;
    build_slots(hg, sx, ss, sn, sso);
    p.nslots = (int)sx.size();
    std::vector<FftDesc> descs;
    std::map<int, int> desc_index;
    std::vector<int32_t> ring_desc(hg.nrings);
    int maxL = 1, maxn = 1;
    std::unique_lock<std::mutex> fft_lk(g_fft_mu);  // held until the plan is complete (or rolled back)
    auto &fcp = g_fft[dev];
    if (!fcp) fcp = std::make_unique<FftCache>();
    FftAdded added;
    struct Rollback {
        FftCache &fc;
        FftAdded &a;
        bool done = false;
        ~Rollback() {
            if (!done) fft_rollback(fc, a);
        }
    } rollback{*fcp, added};
    {
        for (int r = 0; r < hg.nrings; ++r) {
            const int n = hg.nphi[r];
            auto it = desc_index.find(n);
            if (it == desc_index.end()) {
                FftDesc d;
                rc = fft_desc(*fcp, n, &d, added);
                if (rc) return rc;
                desc_index[n] = (int)descs.size();
                descs.push_back(d);
                it = desc_index.find(n);
            }
            ring_desc[r] = it->second;
            maxL = std::max(maxL, descs[it->second].L);
            maxn = std::max(maxn, n);
        }
    }
    p.max_L = maxL;
    p.all_nphi_max = maxn;
    // FFT jobs: mirror pairs with equal nphi, then leftover rings paired by length
    std::vector<int2> jobs;
    std::vector<char> used(hg.nrings, 0);
    for (size_t i = 0; i < sn.size(); ++i) {
        const int a = sn[i], b = sso[i];
        if (b >= 0 && hg.nphi[a] == hg.nphi[b]) {
            jobs.push_back(make_int2(a, b));
            used[a] = used[b] = 1;
        }
    }
    std::map<int, int> waiting;  // nphi -> ring without a partner yet
    for (int r = 0; r < hg.nrings; ++r) {
        if (used[r]) continue;
        auto it = waiting.find(hg.nphi[r]);
        if (it == waiting.end()) {
            waiting[hg.nphi[r]] = r;
        } else {
            jobs.push_back(make_int2(it->second, r));
            waiting.erase(it);
        }
    }
    for (auto &kv : waiting) jobs.push_back(make_int2(kv.second, -1));
    std::vector<int2> cls[kFftClasses];
    for (const int2 &j : jobs) {
        const int L = descs[ring_desc[j.x]].L;
        int c = 0;
        while (c < kFftClasses - 1 && L > kFftClassLen[c]) ++c;
        cls[c].push_back(j);
    }
    for (int c = 0; c < kFftClasses; ++c) {
        p.class_count[c] = (int)cls[c].size();
        if (cls[c].empty()) continue;
        if ((rc = upload(cls[c], &p.class_jobs[c], p.owned))) return rc;
    }
    if ((rc = upload(sx, &p.slot_x, p.owned)) || (rc = upload(ss, &p.slot_s, p.owned)) ||
        (rc = upload(sn, &p.slot_north, p.owned)) || (rc = upload(sso, &p.slot_south, p.owned)) ||
        (rc = upload(hg.phi0, &p.phi0, p.owned)) || (rc = upload(hg.ofs, &p.ofs, p.owned)) ||
        (rc = upload(ring_desc, &p.ring_desc, p.owned)) || (rc = upload(descs, &p.descs, p.owned)))
        return rc;
    if (hg.has_weight && (rc = upload(hg.weight, &p.weight, p.owned))) return rc;
    rollback.done = true;  // the new FFT lengths stay cached for every plan that needs them
    *out = std::move(plan);
    return SHT_OK;
}

constexpr size_t kMaxStartTables = 4;  // per geometry plan (unpinned ones may go beyond it)

// a start table of p that serves (lmax, mmax); with pinned_only, a pinned one
static std::shared_ptr<StartTable> find_start_locked(const GeomPlan &p, int lmax, int mmax, bool pinned_only) {
    for (const auto &t : p.starts)
        if (t->lmax >= lmax && t->mmax >= mmax && (!pinned_only || t->pins > 0)) return t;
    return nullptr;
}

int get_start(const CoefTables &c, const GeomRef &pref, hipStream_t st, StartRef *out) {
    const GeomPlan &p = *pref;  // its start list is only touched under the cache lock
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (auto t = find_start_locked(p, c.lmax, c.mmax, false)) {
            t->last_use = ++g_clock;
            *out = t;
            return SHT_OK;
        }
    }
    // built and waited for outside the cache lock
    auto t = std::make_shared<StartTable>();
    t->dev = p.dev;
    t->lmax = c.lmax;
    t->mmax = c.mmax;
    const size_t n = (size_t)(c.mmax + 1) * (size_t)p.nslots;
    void *a = nullptr, *b = nullptr;
    if (!dev_alloc(&a, n * sizeof(int32_t))) return SHT_ENOMEM;
    t->lstart = static_cast<int32_t *>(a);
    if (!dev_alloc(&b, n * sizeof(double2))) return SHT_ENOMEM;  // t frees lstart
    t->state = static_cast<double2 *>(b);
    int rc = launch_leg_start(c, p, t->lstart, t->state, st);
    if (rc == SHT_OK && hipStreamSynchronize(st) != hipSuccess) rc = SHT_EDEVICE;
    if (rc) return rc;
    std::vector<std::shared_ptr<StartTable>> dropped;  // freed after the lock is released
    std::lock_guard<std::mutex> lk(g_mu);
    if (auto u = find_start_locked(p, c.lmax, c.mmax, false)) {  // built meanwhile by another call
        u->last_use = ++g_clock;
        *out = u;
        dropped.push_back(std::move(t));
        return SHT_OK;
    }
    while (p.starts.size() >= kMaxStartTables) {
        // the least recently used unpinned table goes; it is freed when its last user is done
        auto lru = p.starts.end();
        for (auto e = p.starts.begin(); e != p.starts.end(); ++e)
            if ((*e)->pins == 0 && (lru == p.starts.end() || (*e)->last_use < (*lru)->last_use)) lru = e;
        if (lru == p.starts.end()) break;  // all pinned
        dropped.push_back(std::move(*lru));
        p.starts.erase(lru);
    }
    t->last_use = ++g_clock;
    p.starts.push_back(t);
    *out = t;
    return SHT_OK;
}

int pin_plan(int lmax, int mmax, const HostGeom &hg, int delta) {
    int dev = 0;
    int rc = current_device(&dev);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    auto ce = g_coef.find(std::make_tuple(dev, lmax, mmax));
    GeomEntry *ge = find_geom_locked(dev, hg);
    if (ce == g_coef.end() || !ge) return SHT_ENOPLAN;
    auto st = find_start_locked(*ge->plan, lmax, mmax, delta < 0);
    if (!st) return SHT_ENOPLAN;
    if (delta < 0 && (ce->second.pins <= 0 || ge->pins <= 0)) return SHT_ENOPLAN;
    ce->second.pins += delta;
    ge->pins += delta;
    st->pins += delta;
    return SHT_OK;
}

int find_pinned(int lmax, int mmax, const HostGeom &hg, CoefRef *c, GeomRef *p, StartRef *s) {
    int dev = 0;
    int rc = current_device(&dev);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    auto ce = g_coef.find(std::make_tuple(dev, lmax, mmax));
    GeomEntry *ge = find_geom_locked(dev, hg);
    if (ce == g_coef.end() || ce->second.pins <= 0 || !ge || ge->pins <= 0) return SHT_ENOPLAN;
    auto st = find_start_locked(*ge->plan, lmax, mmax, true);
    if (!st) return SHT_ENOPLAN;
    *c = ce->second.t;
    *p = ge->plan;
    *s = st;
    return SHT_OK;
}

// ------------------------------------------------------------------ side streams
// Each calling stream has its own side streams and fork/join events, so that
// calls on different streams never share them: they neither serialise on a
// lock nor join each other's graph captures.
struct SideStreams {
    hipStream_t s[kSideStreams] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kSideStreams] = {};
    std::mutex mu;  // one call at a time per calling stream
};
static std::mutex g_side_mu;
static auto &g_side = *new std::map<std::pair<int, hipStream_t>, std::unique_ptr<SideStreams>>();

static void free_side(SideStreams &p) {
    for (int i = 0; i < kSideStreams; ++i) {
        if (p.s[i]) (void)hipStreamDestroy(p.s[i]);
        if (p.join[i]) (void)hipEventDestroy(p.join[i]);
    }
    if (p.fork) (void)hipEventDestroy(p.fork);
}

int fork_join(hipStream_t st, int n, const std::function<int(int, hipStream_t)> &launch) {
    if (n <= 1) return n == 1 ? launch(0, st) : SHT_OK;
    if (n > kSideStreams + 1) return SHT_EUNSUPPORTED;
    int dev = 0;
    int rc = current_device(&dev);
    if (rc) return rc;
    SideStreams *p = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_side_mu);
        auto &slot = g_side[std::make_pair(dev, st)];
        if (!slot) {
            auto q = std::make_unique<SideStreams>();
            // the events only order kernels of one device: a device-scope release
            // suffices (no system-scope fence, which would write back for the host)
            const unsigned ef = hipEventDisableTiming | hipEventDisableSystemFence;
            bool ok = hipEventCreateWithFlags(&q->fork, ef) == hipSuccess;
            for (int i = 0; ok && i < kSideStreams; ++i)
                ok = hipStreamCreateWithFlags(&q->s[i], hipStreamNonBlocking) == hipSuccess &&
                     hipEventCreateWithFlags(&q->join[i], ef) == hipSuccess;
            if (!ok) {
                free_side(*q);
                g_side.erase(std::make_pair(dev, st));
                return SHT_EDEVICE;
            }
            slot = std::move(q);
        }
        p = slot.get();
    }
    std::lock_guard<std::mutex> lk(p->mu);
    SHT_HIP(hipEventRecord(p->fork, st));
    for (int i = 1; i < n; ++i) SHT_HIP(hipStreamWaitEvent(p->s[i - 1], p->fork, 0));
    for (int i = 0; i < n && rc == SHT_OK; ++i) rc = launch(i, i == 0 ? st : p->s[i - 1]);
    // join even after a failed launch, so that st never runs ahead of side work
    for (int i = 1; i < n; ++i) {
        SHT_HIP(hipEventRecord(p->join[i - 1], p->s[i - 1]));
        SHT_HIP(hipStreamWaitEvent(st, p->join[i - 1], 0));
    }
    return rc;
}

int set_cache_limits(int max_coef, int max_geom) {
    if (max_coef < 1 || max_geom < 1) return SHT_EINVAL;
    std::vector<std::shared_ptr<CoefTables>> dc;  // freed after the lock is released
    std::vector<std::shared_ptr<GeomPlan>> dg;
    std::lock_guard<std::mutex> lk(g_mu);
    g_max_coef = (size_t)max_coef;
    g_max_geom = (size_t)max_geom;
    // unpinned entries beyond the new limits go now, least recently used
    // first; each is freed when its last user is done
    while (g_coef.size() > g_max_coef) {
        auto lru = g_coef.end();
        for (auto e = g_coef.begin(); e != g_coef.end(); ++e)
            if (e->second.pins == 0 && (lru == g_coef.end() || e->second.last_use < lru->second.last_use)) lru = e;
        if (lru == g_coef.end()) break;
        dc.push_back(std::move(lru->second.t));
        g_coef.erase(lru);
    }
    while (g_geom.size() > g_max_geom) {
        auto lru = g_geom.end();
        for (auto e = g_geom.begin(); e != g_geom.end(); ++e)
            if (e->pins == 0 && (lru == g_geom.end() || e->last_use < lru->last_use)) lru = e;
        if (lru == g_geom.end()) break;
        dg.push_back(std::move(lru->plan));
        g_geom.erase(lru);
    }
    return SHT_OK;
}

void shutdown_all() {
    std::vector<GeomEntry> geoms;
    std::map<std::tuple<int, int, int>, CoefEntry> coefs;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        geoms.swap(g_geom);
        coefs.swap(g_coef);
    }
    (void)hipDeviceSynchronize();  // calls in flight must have completed; this is the last check
    geoms.clear();  // plans and their start tables free themselves
    coefs.clear();
    {
        std::lock_guard<std::mutex> lk(g_fft_mu);
        for (auto &kv : g_fft)
            for (void *p : kv.second->owned) dev_free(p);
        g_fft.clear();
    }
    {
        std::lock_guard<std::mutex> lk(g_side_mu);
        for (auto &kv : g_side) free_side(*kv.second);
        g_side.clear();
    }
    std::lock_guard<std::mutex> lk(g_use_mu);
    for (auto &kv : g_uses) {
        (void)hipEventDestroy(kv.second->ev);
        delete kv.second;
    }
    g_uses.clear();
}

}  // namespace sht
