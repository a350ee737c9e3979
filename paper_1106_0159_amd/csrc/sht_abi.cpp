// extern "C" entry points of libsht.so (declared in include/sht.h).
#include <algorithm>
#include <cstring>

#include "sht_internal.h"

namespace sht {
const char *last_hip_error();
void shutdown_all();
int set_cache_limits(int max_coef, int max_geom);
size_t plan_cache_bytes();
}  // namespace sht

using namespace sht;

namespace {

constexpr uint32_t kKnownFlags = SHT_MIXED | SHT_DELTA_MAP_MINOR | SHT_MIXED_FP64_SUMS | SHT_MIXED_SPLIT_BF16;

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

size_t alm_bytes(int lmax, int mmax, int nmaps) {
    return (size_t)nalm_of(lmax, mmax) * 16u * (size_t)nmaps;
}
size_t delta_bytes(int nrings, int mmax, int nmaps) {
    return (size_t)nrings * (size_t)(mmax + 1) * 16u * (size_t)nmaps;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// Workspace layout: [Delta (synthesis/analysis)][aux], aux holding the
// c-scaled a_lm of synthesis (followed by kCoefPad entries that the synthesis
// kernel may read ahead; with SHT_MIXED the FP32 block tiles instead) or the
// per-group partial a_lm of analysis.
size_t partial_bytes(int lmax, int mmax, int nslots, int nmaps) {
    const int G = ana_groups(nslots);
    return G > 1 ? (size_t)G * alm_bytes(lmax, mmax, nmaps) : 0;
}
size_t aux_bytes(int lmax, int mmax, int nslots, int nmaps, uint32_t flags) {
    // with SHT_MIXED either kernel set may run (use_mx), so room for both
    const size_t f64 = alm_bytes(lmax, mmax, nmaps) + 16u * kCoefPad;
    const size_t syn = (flags & SHT_MIXED) ? std::max(f64, mx_aprime_bytes(lmax, mmax, nmaps, flags)) : f64;
    return std::max(round256(syn), round256(partial_bytes(lmax, mmax, nslots, nmaps)));
}
size_t ws_need(int lmax, int mmax, const HostGeom &h, int nmaps, uint32_t flags) {
    return round256(delta_bytes(h.nrings, mmax, nmaps)) + aux_bytes(lmax, mmax, count_slots(h), nmaps, flags);
}

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// After a call has enqueued its kernels (status rc): notes the stream's use
// of the tables, so that an eviction waits for this work before freeing them.
int fenced(int rc, hipStream_t st, std::initializer_list<const Fenced *> tables) {
    const int rf = note_uses(st, tables);
    return rc ? rc : rf;
}

// Delta layout of a stage call; the FP64 Legendre kernels take ring-major only
DeltaLayout stage_layout(const HostGeom &h, int mmax, int nmaps, uint32_t flags) {
    return delta_layout(h.nrings, mmax, nmaps, (flags & SHT_DELTA_MAP_MINOR) != 0);
}
bool legendre_layout_ok(uint32_t flags) { return !(flags & SHT_DELTA_MAP_MINOR) || (flags & SHT_MIXED); }

// Common checks for the transforms; fills the validated geometry.
int check_common(int lmax, int mmax, const sht_geom *g, int nmaps, uint32_t flags, bool need_weight,
                 HostGeom *h) {
    int rc = validate_sizes(lmax, mmax, nmaps);
    if (rc) return rc;
    if (flags & ~kKnownFlags) return SHT_EUNSUPPORTED;
    if ((flags & (SHT_MIXED_FP64_SUMS | SHT_MIXED_SPLIT_BF16)) && !(flags & SHT_MIXED)) return SHT_EUNSUPPORTED;
    return validate_geom(g, need_weight, h);
}

}  // namespace

namespace sht {

size_t ws_aux_offset(int nrings, int mmax, int nmaps) { return round256(delta_bytes(nrings, mmax, nmaps)); }

int check_alm2map(int lmax, int mmax, const sht_geom *g, const void *alm, const double *map, int nmaps,
                  uint32_t flags, HostGeom *h, size_t *ws_bytes_needed) {
    int rc = check_common(lmax, mmax, g, nmaps, flags, false, h);
    if (rc) return rc;
    if (!alm || !map || !aligned(alm, 16) || !aligned(map, 8)) return SHT_EINVAL;
    const size_t ab = alm_bytes(lmax, mmax, nmaps), mb = (size_t)h->npix * 8u * nmaps;
    if (overlap(alm, ab, map, mb)) return SHT_EINVAL;
    *ws_bytes_needed = ws_need(lmax, mmax, *h, nmaps, flags);
    return SHT_OK;
}

int enqueue_alm2map(const CoefTables &c, const GeomPlan &p, const StartTable &s, const void *alm, void *aprime,
                    void *delta, DeltaLayout dl, double *map, int nmaps, uint32_t flags, hipStream_t st, bool fork) {
    int rc;
    if (use_mx(flags & ~SHT_DELTA_MAP_MINOR, nmaps)) {
        if ((rc = launch_leg_syn_mx(c, p, s, alm, aprime, delta, dl, nmaps, flags, st))) return rc;
    } else {
        if ((rc = launch_prescale(c, alm, aprime, nmaps, st))) return rc;
        if ((rc = launch_leg_syn(c, p, s, aprime, delta, nmaps, st))) return rc;
    }
    return launch_fft_syn(p, c.mmax, delta, dl, map, nmaps, st, fork);
}

}  // namespace sht

extern "C" {

size_t sht_workspace_bytes(int lmax, int mmax, const sht_geom *g, int nmaps, uint32_t flags) {
    HostGeom h;
    if (check_common(lmax, mmax, g, nmaps, flags, false, &h)) return 0;
    return ws_need(lmax, mmax, h, nmaps, flags);
}

int sht_alm2delta(int lmax, int mmax, const sht_geom *g, const void *alm, void *delta, int nmaps,
                  void *workspace, size_t ws_bytes, uint32_t flags, void *stream) {
    HostGeom h;
    int rc = check_common(lmax, mmax, g, nmaps, flags, false, &h);
    if (rc) return rc;
    if (!legendre_layout_ok(flags)) return SHT_EUNSUPPORTED;
    if (!alm || !delta || !aligned(alm, 16) || !aligned(delta, 16)) return SHT_EINVAL;
    const size_t ab = alm_bytes(lmax, mmax, nmaps), db = delta_bytes(h.nrings, mmax, nmaps);
    if (!workspace || !aligned(workspace, 16) || ws_bytes < ws_need(lmax, mmax, h, nmaps, flags))
        return SHT_EWORKSPACE;
    if (overlap(alm, ab, delta, db) || overlap(workspace, ws_bytes, alm, ab) ||
        overlap(workspace, ws_bytes, delta, db))
        return SHT_EINVAL;
    CoefRef c;
    GeomRef p;
    StartRef s;
    if ((rc = get_coef(lmax, mmax, &c)) || (rc = get_geom(h, mmax, &p)) ||
        (rc = get_start(*c, p, as_stream(stream), &s)))
        return rc;
    if (use_mx(flags, nmaps))
        rc = launch_leg_syn_mx(*c, *p, *s, alm, workspace, delta, stage_layout(h, mmax, nmaps, flags), nmaps, flags,
                               as_stream(stream));
    else if (!(rc = launch_prescale(*c, alm, workspace, nmaps, as_stream(stream))))
        rc = launch_leg_syn(*c, *p, *s, workspace, delta, nmaps, as_stream(stream));
    return fenced(rc, as_stream(stream), {c.get(), p.get(), s.get()});
}

int sht_delta2map(int mmax, const sht_geom *g, const void *delta, double *map, int nmaps,
                  uint32_t flags, void *stream) {
    HostGeom h;
    int rc = check_common(mmax, mmax, g, nmaps, flags, false, &h);
    if (rc) return rc;
    if (!delta || !map || !aligned(delta, 16) || !aligned(map, 8)) return SHT_EINVAL;
    if (overlap(delta, delta_bytes(h.nrings, mmax, nmaps), map, (size_t)h.npix * 8u * nmaps))
        return SHT_EINVAL;
    GeomRef p;
    if ((rc = get_geom(h, mmax, &p))) return rc;
    rc = launch_fft_syn(*p, mmax, delta, stage_layout(h, mmax, nmaps, flags), map, nmaps, as_stream(stream));
    return fenced(rc, as_stream(stream), {p.get()});
}

int sht_map2delta(int mmax, const sht_geom *g, const double *map, void *delta, int nmaps,
                  uint32_t flags, void *stream) {
    HostGeom h;
    int rc = check_common(mmax, mmax, g, nmaps, flags, true, &h);
    if (rc) return rc;
    if (!delta || !map || !aligned(delta, 16) || !aligned(map, 8)) return SHT_EINVAL;
    if (overlap(delta, delta_bytes(h.nrings, mmax, nmaps), map, (size_t)h.npix * 8u * nmaps))
        return SHT_EINVAL;
    GeomRef p;
    if ((rc = get_geom(h, mmax, &p))) return rc;
    rc = launch_fft_ana(*p, mmax, map, delta, stage_layout(h, mmax, nmaps, flags), nmaps, as_stream(stream));
    return fenced(rc, as_stream(stream), {p.get()});
}

int sht_delta2alm(int lmax, int mmax, const sht_geom *g, const void *delta, void *alm, int nmaps,
                  void *workspace, size_t ws_bytes, uint32_t flags, void *stream) {
    HostGeom h;
    int rc = check_common(lmax, mmax, g, nmaps, flags, false, &h);
    if (rc) return rc;
    if (!legendre_layout_ok(flags) || (flags & SHT_MIXED_SPLIT_BF16)) return SHT_EUNSUPPORTED;
    if (!delta || !alm || !aligned(delta, 16) || !aligned(alm, 16)) return SHT_EINVAL;
    const size_t ab = alm_bytes(lmax, mmax, nmaps), db = delta_bytes(h.nrings, mmax, nmaps);
    if (!workspace || !aligned(workspace, 16) || ws_bytes < ws_need(lmax, mmax, h, nmaps, flags))
        return SHT_EWORKSPACE;
    if (overlap(delta, db, alm, ab) || overlap(workspace, ws_bytes, alm, ab) ||
        overlap(workspace, ws_bytes, delta, db))
        return SHT_EINVAL;
    CoefRef c;
    GeomRef p;
    StartRef s;
    if ((rc = get_coef(lmax, mmax, &c)) || (rc = get_geom(h, mmax, &p)) ||
        (rc = get_start(*c, p, as_stream(stream), &s)))
        return rc;
    if (use_mx(flags, nmaps))
        rc = launch_leg_ana_mx(*c, *p, *s, delta, stage_layout(h, mmax, nmaps, flags), alm, nmaps, workspace,
                               as_stream(stream));
    else
        rc = launch_leg_ana(*c, *p, *s, delta, alm, nmaps, workspace, as_stream(stream));
    return fenced(rc, as_stream(stream), {c.get(), p.get(), s.get()});
}

int sht_alm2map(int lmax, int mmax, const sht_geom *g, const void *alm, double *map, int nmaps,
                void *workspace, size_t ws_bytes, uint32_t flags, void *stream) {
    HostGeom h;
    size_t need = 0;
    int rc = check_alm2map(lmax, mmax, g, alm, map, nmaps, flags, &h, &need);
    if (rc) return rc;
    const size_t ab = alm_bytes(lmax, mmax, nmaps), db = delta_bytes(h.nrings, mmax, nmaps);
    const size_t mb = (size_t)h.npix * 8u * nmaps;
    if (!workspace || !aligned(workspace, 16) || ws_bytes < need) return SHT_EWORKSPACE;
    if (overlap(workspace, ws_bytes, alm, ab) || overlap(workspace, ws_bytes, map, mb)) return SHT_EINVAL;
    hipStream_t st = as_stream(stream);
    CoefRef c;
    GeomRef p;
    StartRef s;
    if ((rc = get_coef(lmax, mmax, &c)) || (rc = get_geom(h, mmax, &p)) || (rc = get_start(*c, p, st, &s)))
        return rc;
    char *ws = static_cast<char *>(workspace);
    void *delta = ws, *aprime = ws + round256(db);
    const DeltaLayout dl = alm2map_layout(h.nrings, mmax, nmaps, flags);
    rc = enqueue_alm2map(*c, *p, *s, alm, aprime, delta, dl, map, nmaps, flags, st, true);
    return fenced(rc, st, {c.get(), p.get(), s.get()});
}

int sht_map2alm(int lmax, int mmax, const sht_geom *g, const double *map, void *alm, int nmaps,
                void *workspace, size_t ws_bytes, uint32_t flags, void *stream) {
    HostGeom h;
    int rc = check_common(lmax, mmax, g, nmaps, flags, true, &h);
    if (rc) return rc;
    if (flags & SHT_MIXED_SPLIT_BF16) return SHT_EUNSUPPORTED;  // a synthesis variant
    if (!alm || !map || !aligned(alm, 16) || !aligned(map, 8)) return SHT_EINVAL;
    const size_t ab = alm_bytes(lmax, mmax, nmaps), db = delta_bytes(h.nrings, mmax, nmaps);
    const size_t mb = (size_t)h.npix * 8u * nmaps;
    if (!workspace || !aligned(workspace, 16) || ws_bytes < ws_need(lmax, mmax, h, nmaps, flags))
        return SHT_EWORKSPACE;
    if (overlap(alm, ab, map, mb) || overlap(workspace, ws_bytes, alm, ab) ||
        overlap(workspace, ws_bytes, map, mb))
        return SHT_EINVAL;
    hipStream_t st = as_stream(stream);
    CoefRef c;
    GeomRef p;
    StartRef s;
    if ((rc = get_coef(lmax, mmax, &c)) || (rc = get_geom(h, mmax, &p)) || (rc = get_start(*c, p, st, &s)))
        return rc;
    char *ws = static_cast<char *>(workspace);
    void *delta = ws, *partials = ws + round256(db);
    // ring-major here also with SHT_MIXED: with map-minor Delta the ring FFT
    // loses about what the analysis kernel gains on its reads
    const DeltaLayout dl = delta_layout(h.nrings, mmax, nmaps, false);
    if (!(rc = launch_fft_ana(*p, mmax, map, delta, dl, nmaps, st))) {
        if (use_mx(flags & ~SHT_DELTA_MAP_MINOR, nmaps))
            rc = launch_leg_ana_mx(*c, *p, *s, delta, dl, alm, nmaps, partials, st);
        else
            rc = launch_leg_ana(*c, *p, *s, delta, alm, nmaps, partials, st);
    }
    return fenced(rc, st, {c.get(), p.get(), s.get()});
}

int sht_prepare(int lmax, int mmax, const sht_geom *g, uint32_t flags, void *stream) {
    HostGeom h;
    int rc = check_common(lmax, mmax, g, 1, flags & ~SHT_PIN, false, &h);
    if (rc) return rc;
    CoefRef c;
    GeomRef p;
    StartRef s;
    if ((rc = get_coef(lmax, mmax, &c)) || (rc = get_geom(h, mmax, &p)) ||
        (rc = get_start(*c, p, as_stream(stream), &s)))
        return rc;
    // pinned by key: if another call evicted these entries between the
    // lookups above and here, they are built again
    for (int tries = 0; (flags & SHT_PIN) && tries < 4; ++tries) {
        if ((rc = pin_plan(lmax, mmax, h, +1)) != SHT_ENOPLAN) return rc;
        if ((rc = get_coef(lmax, mmax, &c)) || (rc = get_geom(h, mmax, &p)) ||
            (rc = get_start(*c, p, as_stream(stream), &s)))
            return rc;
    }
    return (flags & SHT_PIN) ? SHT_ENOMEM : SHT_OK;
}

int sht_unpin(int lmax, int mmax, const sht_geom *g) {
    HostGeom h;
    int rc = check_common(lmax, mmax, g, 1, 0, false, &h);
    if (rc) return rc;
    return pin_plan(lmax, mmax, h, -1);
}

int sht_plan_cache_limits(int max_coef_tables, int max_geom_plans) {
    return set_cache_limits(max_coef_tables, max_geom_plans);
}

size_t sht_plan_cache_bytes(void) { return plan_cache_bytes(); }

const char *sht_strerror(int code) {
    switch (code) {
        case SHT_OK: return "success";
        case SHT_EINVAL: return "invalid argument";
        case SHT_EWORKSPACE: return "workspace missing or too small";
        case SHT_EDEVICE: {
            const char *s = last_hip_error();
            return (s && *s) ? s : "HIP runtime error";
        }
        case SHT_ENOMEM: return "out of memory for plan tables";
        case SHT_EUNSUPPORTED: return "unsupported flag or size";
        case SHT_ENOPLAN: return "plan tables not resident and pinned (sht_prepare with SHT_PIN first)";
        default: return "unknown status code";
    }
}

void sht_shutdown(void) { shutdown_all(); }

}  // extern "C"
