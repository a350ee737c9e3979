/*
 * sht.h -- C ABI of the MI355X (gfx950) spherical harmonic transform library
 * (libsht.so): the Legendre stage and ring FFTs of the transforms described
 * in Szydlarski et al., "Parallel Spherical Harmonic Transforms on
 * heterogeneous architectures".
 *
 * Problem statement (Sec. 2.1, eqs. map2almDef and alm2mapDef):
 *   synthesis  s(theta_n, phi_n) = sum_{l<=lmax} sum_{|m|<=min(l,mmax)} a_lm Y_lm(theta_n, phi_n)
 *   analysis   a_lm = sum_n w_n s_n conj(Y_lm(theta_n, phi_n))
 * with Y_lm = lambda_lm(cos theta) e^{i m phi} (eq. YlmDef, Condon-Shortley
 * phase), real maps and therefore a_{l,-m} = (-1)^m conj(a_lm) (the symmetry
 * stated after eq. YlmDef), so only m >= 0 is stored.
 *
 * Geometry (Sec. 2.2, iso-latitude rings): ring r has colatitude theta[r],
 * nphi[r] equidistant pixels at phi_j = phi0[r] + 2 pi j / nphi[r], and one
 * per-pixel quadrature weight weight[r]; its pixels are map[ofs[r] + j].
 *
 * Data layouts (all device buffers are caller-owned; the library never
 * keeps a pointer to them after a call returns):
 *   a_lm   complex128 (re, im interleaved, 16-byte aligned), [nmaps][nalm],
 *          m-major packed: index(l, m) = m*(2*lmax+1-m)/2 + l, m <= l <= lmax,
 *          nalm = (mmax+1)*(2*lmax+2-mmax)/2.
 *   map    float64, [nmaps][npix], npix = max_r(ofs[r] + nphi[r]).
 *   delta  complex128, [nmaps][nrings][mmax+1]: Delta_m(r) of Sec. 2.2
 *          (eq. DeltaDef for synthesis, eq. almfftdef for analysis);
 *          [nrings][mmax+1][nmaps] with SHT_DELTA_MAP_MINOR.
 *
 * Conventions: Im a_l0 is ignored on input and written as exactly 0 on
 * output.  Rings r, r' whose colatitudes satisfy |theta_r + theta_r' - pi|
 * <= 2^-50 (8.9e-16 rad, two ulp of pi; the sum taken exactly) are treated as
 * mirror images (cos theta_r' = -cos theta_r, evaluated from the northern
 * ring) and share one Legendre recurrence; any other ring is evaluated at its
 * own colatitude.
 *
 * Execution: every compute call validates its arguments on the host, then
 * enqueues kernels on `stream` (a hipStream_t; NULL = the null stream) and
 * returns without waiting.  A failed validation returns an error before
 * anything is enqueued and leaves all outputs untouched.  Kernel faults
 * surface at the caller's next synchronisation of the stream.  The first call
 * for a (lmax, mmax, geometry) builds and caches device tables (recurrence
 * coefficients, FFT plans, and for the Legendre stage the start table: where
 * each (m, ring pair) recurrence enters double range, 20 bytes per (m, pair),
 * built by a kernel on `stream`); that call waits for `stream`.  The
 * library owns these tables and frees them on eviction or sht_shutdown().
 *
 * Thread safety: all functions may be called from several host threads.
 * Buffers passed to concurrent calls must not overlap (outputs), and inputs
 * must not be written while a call that reads them is in flight.
 */
#ifndef SHT_H
#define SHT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Ring geometry, HOST memory, read only during the call. */
typedef struct sht_geom {
    int32_t nrings;         /* >= 1 */
    const double *theta;    /* [nrings] colatitude in [0, pi] */
    const int32_t *nphi;    /* [nrings] pixels per ring, >= 1 */
    const double *phi0;     /* [nrings] longitude of pixel j = 0 (finite) */
    const double *weight;   /* [nrings] per-pixel quadrature weight; required by
                               analysis, may be NULL for synthesis */
    const int64_t *ofs;     /* [nrings] first-pixel offset; NULL = rings packed
                               in order from 0.  Ring ranges must not overlap. */
} sht_geom;

enum sht_status {
    SHT_OK = 0,
    SHT_EINVAL = -1,        /* invalid argument (sizes, geometry, pointers) */
    SHT_EWORKSPACE = -2,    /* workspace NULL or smaller than required */
    SHT_EDEVICE = -3,       /* a HIP runtime call failed (see sht_strerror) */
    SHT_ENOMEM = -4,        /* device or host allocation for plan tables failed */
    SHT_EUNSUPPORTED = -5,  /* unknown flag bit, or a size beyond the kernels' limits
                               (a ring of more than 8192 pixels, mmax >= 65535,
                               nmaps > 65535, grids beyond 2^31 workgroups) */
    SHT_ENOPLAN = -6        /* the plan tables of this (lmax, mmax, geometry) are not
                               resident and pinned (sht_prepare with SHT_PIN), where a
                               call requires that (sht_unpin) */
};

/* Flag bits of the `flags` arguments. */
enum sht_flags {
    /* Mixed precision for the Legendre contraction (sht_alm2map,
     * sht_alm2delta, sht_map2alm, sht_delta2alm; the ring-FFT calls ignore
     * it).  The recurrence, its seeds, start table and coefficients stay FP64
     * (Sec. 2.1).  Each lambda_lm (in the rescaled form q_lm = lambda_lm / c_lm)
     * is rounded to FP32 once, as is each c_lm a_lm (synthesis) or each
     * north +- south Delta_m of a ring pair (analysis), and the per-m matrix
     * products of Sec. 3 (eq. matrix_vec and its transpose, one column per
     * map and real/imaginary part) run on the FP32 matrix cores: synthesis
     * sums over l in FP32 (with SHT_MIXED_FP64_SUMS, and above lmax 2048,
     * 32 l at a time, those block sums added in FP64); analysis sums 32 l at
     * a time over up to 256 ring pairs in FP32 and adds those sums in FP64.  The
     * Delta and FFT stages stay FP64.  Expected relative RMS error against
     * the FP64 transform: about 1e-7 to 1e-6.  Built for batches: a wave
     * covers 8 to 32 maps in synthesis (8 with FP64 block sums) and 8 in
     * analysis.  With fewer than 8 maps the FP64 kernels run instead (a
     * single map would leave most matrix-core columns idle, and FP32 vector
     * arithmetic is no faster than FP64 on this part), except in the stage
     * calls with SHT_DELTA_MAP_MINOR, which always take the mixed kernels.
     * sht_alm2map with this flag and nmaps >= 8 keeps its workspace Delta
     * map-minor (as SHT_DELTA_MAP_MINOR below), ring-major with fewer maps;
     * sht_map2alm keeps it ring-major. */
    SHT_MIXED = 1u,
    /* Layout of the `delta` argument of the stage calls: [nrings][mmax+1][nmaps]
     * (map index fastest) instead of [nmaps][nrings][mmax+1].  Accepted by
     * sht_delta2map and sht_map2delta, and by sht_alm2delta and sht_delta2alm
     * together with SHT_MIXED (otherwise SHT_EUNSUPPORTED); no effect on
     * sht_alm2map, sht_map2alm and sht_workspace_bytes.  The Legendre stages
     * give the same bits in either layout; the ring stages then transform two
     * adjacent maps of one ring together instead of the two rings of a mirror
     * pair, which changes their results by rounding only. */
    SHT_DELTA_MAP_MINOR = 2u,
    /* sht_prepare only: pin the plan's tables (one more pin per call) so that
     * no eviction (LRU or sht_plan_cache_limits) frees them until as many
     * sht_unpin calls have removed the pins; only sht_shutdown frees pinned
     * tables.  A pinned cache may hold more entries than its limits.  The
     * transforms reject this bit (SHT_EUNSUPPORTED). */
    SHT_PIN = 4u,
    /* With SHT_MIXED only (alone: SHT_EUNSUPPORTED): the synthesis sums each
     * 32-l block on the matrix cores in a fresh FP32 accumulator and adds the
     * block sums in FP64 (a compensated l-sum; analysis always does so), so
     * the FP32 rounding no longer accumulates over the whole l range.  A wave
     * then covers 8 maps.  Always in effect above lmax 2048. */
    SHT_MIXED_FP64_SUMS = 8u,
    /* With SHT_MIXED only (alone: SHT_EUNSUPPORTED), and for synthesis only
     * (sht_alm2map, sht_alm2delta; the analysis calls return
     * SHT_EUNSUPPORTED): the split low-precision form of the synthesis
     * matrix products (Sec. 3, eq. matrix_vec).  Each FP32 operand (q_lm and
     * c_lm a_lm, rounded to FP32 as with SHT_MIXED alone) is split exactly
     * into three bf16 parts, hi + mid + lo, and each product is the sum of the
     * six bf16 matrix-core products whose terms exceed 2^-24 of it (hi*hi,
     * hi*mid, mid*hi, hi*lo, mid*mid, lo*hi), accumulated in FP32.  Combines
     * with SHT_MIXED_FP64_SUMS.  A wave covers 8 to 32 maps as with
     * SHT_MIXED alone (8 with FP64 block sums).  No effect where SHT_MIXED
     * runs the FP64 kernels (fewer than 8 maps). */
    SHT_MIXED_SPLIT_BF16 = 16u
};

/* Bytes of device workspace needed by sht_alm2map, sht_map2alm,
 * sht_alm2delta and sht_delta2alm for these arguments, flags included (a
 * multiple of 256; for given flags the same value serves all four).  Returns
 * 0 if the arguments are invalid. */
size_t sht_workspace_bytes(int lmax, int mmax, const sht_geom *g, int nmaps, uint32_t flags);

/* Synthesis (Sec. 3, Alg. 2): Delta^A_m(r) by the l-recurrence contracted
 * with a_lm (eqs. assLegRec, pmm, pm1m, DeltaDef), then one Fourier sum per
 * ring (eq. Delta2map, phase e^{i m phi_j}).
 *   alm        DEVICE complex128 [nmaps][nalm], read only
 *   map        DEVICE float64   [nmaps][npix], written (pixels outside the
 *              rings are left untouched)
 *   workspace  DEVICE, >= sht_workspace_bytes(...) bytes, 256-byte aligned,
 *              must not alias alm or map; contents undefined afterwards
 *   flags      0 (FP64) or SHT_MIXED, optionally with SHT_MIXED_FP64_SUMS
 *              and SHT_MIXED_SPLIT_BF16 (SHT_DELTA_MAP_MINOR has no effect).
 *              Any other bit: SHT_EUNSUPPORTED. */
int sht_alm2map(int lmax, int mmax, const sht_geom *g, const void *alm, double *map,
                int nmaps, void *workspace, size_t ws_bytes, uint32_t flags, void *stream);

/* Analysis (Sec. 3, Alg. 1): Delta^S_m(r) = w_r sum_j s_rj e^{-i m phi_j}
 * per ring (eq. almfftdef), then a_lm = sum_r Delta^S_m(r) lambda_lm(cos theta_r)
 * (eq. almdef), a reduction over rings done in a fixed order (deterministic).
 * Requires g->weight.
 *   map        DEVICE float64   [nmaps][npix], read only
 *   alm        DEVICE complex128 [nmaps][nalm], fully written
 *   workspace  as for sht_alm2map
 *   flags      as for sht_alm2map, except SHT_MIXED_SPLIT_BF16 (a synthesis
 *              variant): SHT_EUNSUPPORTED. */
int sht_map2alm(int lmax, int mmax, const sht_geom *g, const double *map, void *alm,
                int nmaps, void *workspace, size_t ws_bytes, uint32_t flags, void *stream);

/* The two stages of each transform, for callers that keep Delta
 * themselves (and for per-stage timing).  sht_alm2map = sht_alm2delta then
 * sht_delta2map; sht_map2alm = sht_map2delta then sht_delta2alm.
 *   delta      DEVICE complex128 [nmaps][nrings][mmax+1] ([nrings][mmax+1][nmaps]
 *              with SHT_DELTA_MAP_MINOR)
 * sht_alm2delta and sht_delta2alm need a workspace of sht_workspace_bytes(...)
 * bytes (it must not alias their other buffers); the two ring stages need none. */
int sht_alm2delta(int lmax, int mmax, const sht_geom *g, const void *alm, void *delta,
                  int nmaps, void *workspace, size_t ws_bytes, uint32_t flags, void *stream);
int sht_delta2map(int mmax, const sht_geom *g, const void *delta, double *map, int nmaps,
                  uint32_t flags, void *stream);
int sht_map2delta(int mmax, const sht_geom *g, const double *map, void *delta, int nmaps,
                  uint32_t flags, void *stream);
int sht_delta2alm(int lmax, int mmax, const sht_geom *g, const void *delta, void *alm,
                  int nmaps, void *workspace, size_t ws_bytes, uint32_t flags, void *stream);

/* ---- uneven batches: many requests, one persistent Legendre launch ----
 *
 * A batch is a fixed set of transforms, each with its own lmax, mmax,
 * geometry and direction (one map each), whose Legendre stage (Sec. 3,
 * Algs. 1 and 2) runs in ONE persistent launch: every workgroup takes the
 * next work item -- (request, m-block, ring tile) -- from a device queue
 * until it is empty.  The items are listed longest first, the dynamic
 * counterpart of the paper's min-max balancing of m (Sec. 4.2.1, where
 * pairs m' + m'' = mmax cost the same): the cheap items of every request
 * fill the end of the run on each CU.  Around it: the ring analysis of the
 * map2alm requests before, the ring synthesis of the alm2map requests after.
 * Precision: FP64 (flags 0).  Results equal those of sht_alm2map /
 * sht_map2alm to rounding (the same arithmetic; analysis tiles may sum ring
 * pairs in another order). */
enum sht_kind { SHT_ALM2MAP = 0, SHT_MAP2ALM = 1 };
typedef struct sht_request {
    int32_t kind;          /* SHT_ALM2MAP or SHT_MAP2ALM */
    int32_t lmax, mmax;    /* 0 <= mmax <= lmax */
    const sht_geom *geom;  /* HOST, read during sht_batch_create only; map2alm needs weights */
    const void *in;        /* DEVICE: a_lm complex128 [nalm] (alm2map) or map float64 [npix] (map2alm) */
    void *out;             /* DEVICE: map (alm2map) or a_lm (map2alm), written by every sht_batch_run */
    int32_t tile;          /* Legendre tile: 0 = the library's choice, else 16 * shape + T with T in {1, 2, 4}:
                              shape 0 = one wave per (m, 64 T ring slots), four such units per item
                              (analysis: every slot of m in one wave, so 64 T >= slots); shape 1
                              (analysis only) = one workgroup per (m, group of 256 T slots), groups
                              added by a combine kernel.  A slot is a mirror ring pair or a ring. */
} sht_request;
typedef struct sht_batch sht_batch;

/* Device workspace bytes of a batch (a multiple of 256; 0 if a request is
 * invalid).  It holds the queue head and every request's Delta and aux. */
size_t sht_batch_workspace_bytes(int nreq, const sht_request *reqs, uint32_t flags);

/* Builds a batch: validates every request (SHT_EINVAL / SHT_EUNSUPPORTED as
 * for the single transforms; flags must be 0), builds and pins each plan
 * (start tables by kernels on `stream`, waited for), and uploads the request
 * table and the item list.  `workspace` (DEVICE, 256-byte aligned, at least
 * sht_batch_workspace_bytes, not aliasing any request's buffers) and every
 * request's in/out pointers are bound to the batch: they must stay valid until
 * sht_batch_destroy.  On success *out owns the batch; on failure *out is NULL. */
int sht_batch_create(int nreq, const sht_request *reqs, void *workspace, size_t ws_bytes, uint32_t flags,
                     void *stream, sht_batch **out);

/* Enqueues every transform of the batch on `stream` (a fixed launch
 * sequence: no allocation, copy or synchronisation, so it may be captured
 * in a HIP graph and replayed; the queue is reset by a kernel at its start).
 * Runs of one batch must not overlap (they share its workspace).  Returns
 * SHT_OK, SHT_EINVAL (NULL batch, or another device current than at
 * creation) or SHT_EDEVICE. */
int sht_batch_run(sht_batch *b, void *stream);

/* Frees the batch's device tables and unpins its plans.  No run of it may be
 * in flight. */
void sht_batch_destroy(sht_batch *b);

/* ---- plan residency, for callers that serve requests of many sizes ----
 *
 * The plan tables of a (lmax, mmax, geometry) are what the paper's memory
 * model (Sec. 4.1.2) counts beside the maps and a_lm: per-ring geometry and
 * FFT plans (proportional to R_N and the ring lengths), recurrence
 * coefficients (2 lmax mmax terms) and the start table (mmax x ring pairs).
 * A server that keeps them resident on the device pays for them once, not
 * per request. */

/* Builds every table that a transform of this (lmax, mmax, geometry) needs
 * and keeps it in the plan cache, so that later calls find it resident.  The
 * start table is built by a kernel on `stream`; the call returns after it has
 * completed.  Validation as for sht_alm2map (weights may be NULL; a geometry
 * with weights and one without are distinct cache keys, so a caller that
 * runs both directions passes the weights to both).  `flags`: SHT_MIXED is
 * validated only (both precision modes use the same tables); SHT_PIN pins the
 * tables (see sht_flags).  Returns SHT_OK, SHT_EINVAL, SHT_EUNSUPPORTED,
 * SHT_ENOMEM or SHT_EDEVICE.
 *
 * HIP graph capture: once its plan is resident, a transform call enqueues
 * kernels and stream-ordering events only (no allocation, copy, memset or
 * synchronisation), so it may be captured.  A captured graph holds the
 * tables' device addresses: it is valid only while the plan stays pinned
 * (SHT_PIN) and until sht_shutdown.  Under capture the ring stages fork onto
 * side streams that belong to the capturing stream, so captures on
 * different streams, and eager calls on other streams, do not interfere. */
int sht_prepare(int lmax, int mmax, const sht_geom *g, uint32_t flags, void *stream);

/* Removes one pin that sht_prepare(..., SHT_PIN) put on the tables of this
 * (lmax, mmax, geometry); they become evictable when no pin is left.
 * Returns SHT_OK, SHT_EINVAL (invalid arguments) or SHT_ENOPLAN (no pinned
 * tables for these arguments). */
int sht_unpin(int lmax, int mmax, const sht_geom *g);

/* Sets how many coefficient tables (one per (device, lmax, mmax)) and how
 * many geometry plans (one per (device, geometry), each holding up to four
 * start tables) the cache keeps before it evicts the least recently used
 * unpinned one (defaults 8 and 32).  Lowering a limit evicts at once.  An
 * evicted table is freed when the last call holding it has returned, after
 * the host has waited for the work that each stream enqueued with it (an
 * event per stream, re-recorded by every call), so kernels in flight never
 * lose it; no device-wide synchronisation is involved.  Returns SHT_OK, or
 * SHT_EINVAL if either limit is below 1. */
int sht_plan_cache_limits(int max_coef_tables, int max_geom_plans);

/* Device bytes held by the plan cache over all devices (coefficient tables,
 * geometry and FFT plans, start tables). */
size_t sht_plan_cache_bytes(void);

/* Static description of a status code.  For SHT_EDEVICE the text of the
 * last HIP error seen by the calling thread is returned instead. */
const char *sht_strerror(int code);

/* Frees every cached plan table on every device.  Calls in flight must have
 * completed.  Later calls rebuild the tables. */
void sht_shutdown(void);

#ifdef __cplusplus
}
#endif
#endif /* SHT_H */
