/*
 * sht_noalloc.h -- an allocation-free variant of sht_alm2map (libsht.so).
 *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 */
#ifndef SHT_NOALLOC_H
#define SHT_NOALLOC_H

#include "sht.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Size of the library's fixed device scratch array (64 MiB): each GPU the
 * library runs on holds one copy from the library's load until the process
 * ends. */
#define SHT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* sht_alm2map without a caller workspace and without any allocation: the
 * workspace (Delta_m(r) and the c-scaled a_lm, sht_workspace_bytes(...)
 * bytes) is the library's fixed scratch array on the current device.  The
 * call enqueues kernels on `stream` and nothing else: no hipMalloc, hipFree,
 * memset, copy, synchronisation, event or stream creation, and no plan
 * building.  Arguments, layouts and results as for sht_alm2map (the same
 * kernels; the ring stages run their length classes one after another on
 * `stream`, which gives the same bits).
 *
 * The plan tables of (lmax, mmax, g) must be resident and pinned on the
 * current device: sht_prepare(lmax, mmax, g, SHT_PIN, stream) first, with the
 * same geometry (weights included or not, as here).
 *
 * Errors: as sht_alm2map's validation, plus SHT_EWORKSPACE when
 * sht_workspace_bytes(lmax, mmax, g, nmaps, flags) exceeds
 * SHT_NOALLOC_SCRATCH_BYTES (nothing is enqueued), SHT_ENOPLAN when the plan
 * is not resident and pinned, SHT_EDEVICE for a HIP error.
 *
 * Every call on one GPU shares that GPU's scratch array, which keeps the last
 * call's contents (the kernels write every entry they read, so nothing needs
 * clearing): calls that overlap on one GPU -- on different streams, or from
 * several host threads -- race on it and must be serialised by the caller. */
int sht_alm2map_noalloc(int lmax, int mmax, const sht_geom *g, const void *alm, double *map, int nmaps,
                        uint32_t flags, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SHT_NOALLOC_H */
