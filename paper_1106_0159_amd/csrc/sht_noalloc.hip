// sht_alm2map_noalloc: the synthesis of sht_alm2map for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  Its workspace -- the Delta_m(r) array and
// the c-scaled a_lm that the Legendre kernels read -- lives in a fixed device
// array of this library instead of a caller-supplied buffer, and its plan
// tables must already be resident and pinned, so that the call enqueues
// kernels and nothing else.
#include <array>
#include <atomic>
#include <mutex>

#include "sht_internal.h"
#include "sht_noalloc.h"

using namespace sht;

namespace {

constexpr size_t kScratchBytes = SHT_NOALLOC_SCRATCH_BYTES;

// One copy per GPU, at its own device address; host code never uses this
// name as an address (it is a host-side stand-in there), only the pointer
// that hipGetSymbolAddress returns for the current device.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::array<std::atomic<void *>, kMaxDevices> g_scratch{};  // device address of `scratch`, per device
std::mutex g_scratch_mu;

// The device address of `scratch` on device dev (current), looked up once.
int scratch_ptr(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return SHT_EUNSUPPORTED;
    void *p = g_scratch[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        p = g_scratch[dev].load(std::memory_order_relaxed);
        if (!p) {
            SHT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
            if (!p) return SHT_EDEVICE;
            g_scratch[dev].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return SHT_OK;
}

}  // namespace

extern "C" {

int sht_alm2map_noalloc(int lmax, int mmax, const sht_geom *g, const void *alm, double *map, int nmaps,
                        uint32_t flags, void *stream) {
    HostGeom h;
    size_t need = 0;
    int rc = check_alm2map(lmax, mmax, g, alm, map, nmaps, flags, &h, &need);
    if (rc) return rc;
    if (need > kScratchBytes) return SHT_EWORKSPACE;  // beyond the fixed array
    int dev = 0;
    SHT_HIP(hipGetDevice(&dev));
    void *ws = nullptr;
    if ((rc = scratch_ptr(dev, &ws))) return rc;
    // pinned tables are never evicted, so no stream use needs recording
    CoefRef c;
    GeomRef p;
    StartRef s;
    if ((rc = find_pinned(lmax, mmax, h, &c, &p, &s))) return rc;
    char *w = static_cast<char *>(ws);
    void *delta = w, *aprime = w + ws_aux_offset(h.nrings, mmax, nmaps);
    const DeltaLayout dl = alm2map_layout(h.nrings, mmax, nmaps, flags);
    // ring stages one length class after another on `stream`: no side streams
    return enqueue_alm2map(*c, *p, *s, alm, aprime, delta, dl, map, nmaps, flags,
                           reinterpret_cast<hipStream_t>(stream), false);
}

}  // extern "C"
