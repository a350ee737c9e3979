// Uneven batches (sht_batch_*): many alm2map / map2alm requests, each with
// its own lmax and geometry, whose Legendre stage runs in one persistent
// launch over a device work queue (k_leg_batch).
//
// Paper Sec. 4.2.1 balances the m-loop by pairing m' and m'' with m' + m'' =
// mmax, whose costs add to a constant.  Over an uneven batch the costs of
// the work units differ by orders of magnitude across requests, so the
// units are dealt out dynamically instead: the queue lists them longest
// first, and each workgroup takes the next one when it finishes its last
// (greedy longest-processing-time scheduling), so the cheapest units fill
// the end of the run on every CU.
#include <algorithm>
#include <cstring>
#include <numeric>

#include "sht_internal.h"

using namespace sht;

namespace {

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }
bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// Tile codes of sht_request.tile: 16 * shape + T.
constexpr int kShapeWave = 0, kShapeGroup = 1;

struct ReqPlan {
    sht_request r;
    HostGeom h;
    CoefRef c;
    GeomRef p;
    StartRef s;
    int shape = 0, T = 1;
    bool pinned = false;
    size_t delta_off = 0, aux_off = 0, aux_bytes = 0;
};

// The default tile of a request: the smallest wave tile that holds every
// slot of one m (analysis: up to 256 slots), else a workgroup per m in groups
// of 1024 slots; synthesis tiles of 64 T slots, T up to 4.
void default_tile(int kind, int nslots, int *shape, int *T) {
    if (kind == SHT_ALM2MAP) {
        *shape = kShapeWave;
        *T = nslots <= 64 ? 1 : nslots <= 128 ? 2 : 4;
        return;
    }
    if (nslots <= 64 * kBatchMaxAnaT) {
        *shape = kShapeWave;
        *T = nslots <= 64 ? 1 : nslots <= 128 ? 2 : 4;
    } else {
        *shape = kShapeGroup;
        *T = nslots <= 256 ? 1 : nslots <= 512 ? 2 : 4;
    }
}

int decode_tile(int kind, int tile, int nslots, int *shape, int *T) {
    if (tile == 0) {
        default_tile(kind, nslots, shape, T);
        return SHT_OK;
    }
    *shape = tile / 16;
    *T = tile % 16;
    if (*T != 1 && *T != 2 && *T != 4) return SHT_EINVAL;
    if (kind == SHT_ALM2MAP) return *shape == kShapeWave ? SHT_OK : SHT_EINVAL;
    if (*shape == kShapeWave) return nslots <= 64 * *T ? SHT_OK : SHT_EINVAL;
    return *shape == kShapeGroup ? SHT_OK : SHT_EINVAL;
}

int ana_groups_of(int nslots, int T) { return (nslots + kAnaThreads * T - 1) / (kAnaThreads * T); }

// Validates one request and fills its host-side plan (no device work).
int check_request(const sht_request &r, ReqPlan *q) {
    if (r.kind != SHT_ALM2MAP && r.kind != SHT_MAP2ALM) return SHT_EINVAL;
    int rc = validate_sizes(r.lmax, r.mmax, 1);
    if (rc) return rc;
    if ((rc = validate_geom(r.geom, r.kind == SHT_MAP2ALM, &q->h))) return rc;
    if (!r.in || !r.out) return SHT_EINVAL;
    if (!aligned(r.kind == SHT_ALM2MAP ? r.in : r.out, 16) || !aligned(r.kind == SHT_ALM2MAP ? r.out : r.in, 8))
        return SHT_EINVAL;
    q->r = r;
    q->r.geom = nullptr;  // the geometry is read during the call only
    const int ns = count_slots(q->h);
    if ((rc = decode_tile(r.kind, r.tile, ns, &q->shape, &q->T))) return rc;
    if (r.kind == SHT_MAP2ALM && q->shape == kShapeGroup && (int64_t)ana_groups_of(ns, q->T) * (r.mmax + 1) >= INT32_MAX)
        return SHT_EUNSUPPORTED;
    return SHT_OK;
}

// Workspace layout: [queue head, 256 B][per request: Delta][aux], aux the
// c-scaled a_lm (synthesis, with the padding the kernels may read ahead) or
// the group partials (analysis with several groups).
size_t layout(std::vector<ReqPlan> &qs) {
    size_t off = 256;
    for (ReqPlan &q : qs) {
        const sht_request &r = q.r;
        const int64_t na = nalm_of(r.lmax, r.mmax);
        q.delta_off = off;
        off += round256((size_t)q.h.nrings * (size_t)(r.mmax + 1) * 16u);
        q.aux_off = off;
        if (r.kind == SHT_ALM2MAP) {
            q.aux_bytes = round256((size_t)(na + kCoefPad) * 16u);
        } else {
            const int g = q.shape == kShapeGroup ? ana_groups_of(count_slots(q.h), q.T) : 1;
            q.aux_bytes = g > 1 ? round256((size_t)g * (size_t)na * 16u) : 0;
        }
        off += q.aux_bytes;
    }
    return off;
}

int check_all(int nreq, const sht_request *reqs, uint32_t flags, std::vector<ReqPlan> *qs) {
    if (nreq < 1 || !reqs) return SHT_EINVAL;
    if (flags != 0) return SHT_EUNSUPPORTED;
    qs->assign(nreq, ReqPlan{});
    for (int i = 0; i < nreq; ++i) {
        const int rc = check_request(reqs[i], &(*qs)[i]);
        if (rc) return rc;
    }
    return SHT_OK;
}

}  // namespace

struct sht_batch {
    int dev = -1;
    std::vector<ReqPlan> q;
    std::vector<void *> owned;  // device arrays of the batch
    BatchReq *reqs = nullptr;
    BatchItem *items = nullptr;
    int32_t *syn_list = nullptr, *comb_list = nullptr;
    int nitems = 0, nsyn = 0, ncomb = 0, grid = 1;
    int syn_chunks = 1, comb_chunks = 1;
    int *head = nullptr;
    char *ws = nullptr;
    // ring stages of all requests: one launch per length class and direction
    RingBatch ring_ana, ring_syn;
    ~sht_batch() {
        for (void *p : owned) (void)hipFree(p);
        for (ReqPlan &r : q)
            if (r.pinned) (void)pin_plan(r.r.lmax, r.r.mmax, r.h, -1);
    }
};

template <class T>
static int upload_vec(sht_batch *b, const std::vector<T> &v, T **out) {
    void *p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(1, v.size()) * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return SHT_ENOMEM;
    }
    b->owned.push_back(p);
    if (!v.empty()) SHT_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    *out = static_cast<T *>(p);
    return SHT_OK;
}

extern "C" {

size_t sht_batch_workspace_bytes(int nreq, const sht_request *reqs, uint32_t flags) {
    std::vector<ReqPlan> qs;
    if (check_all(nreq, reqs, flags, &qs)) return 0;
    return layout(qs);
}

int sht_batch_create(int nreq, const sht_request *reqs, void *workspace, size_t ws_bytes, uint32_t flags,
                     void *stream, sht_batch **out) {
    if (!out) return SHT_EINVAL;
    *out = nullptr;
    std::vector<ReqPlan> qs;
    int rc = check_all(nreq, reqs, flags, &qs);
    if (rc) return rc;
    const size_t need = layout(qs);
    if (!workspace || !aligned(workspace, 256) || ws_bytes < need) return SHT_EWORKSPACE;
    auto b = std::make_unique<sht_batch>();
    SHT_HIP(hipGetDevice(&b->dev));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    // plans: built (or found) and pinned, so that they stay for the batch's life
    for (ReqPlan &q : qs) {
        const sht_request &r = q.r;
        if ((rc = get_coef(r.lmax, r.mmax, &q.c)) || (rc = get_geom(q.h, r.mmax, &q.p)) ||
            (rc = get_start(*q.c, q.p, st, &q.s)))
            break;
        if ((rc = pin_plan(r.lmax, r.mmax, q.h, +1))) break;
        q.pinned = true;
    }
    b->q = std::move(qs);
    if (rc) return rc;  // ~sht_batch unpins what was pinned
    char *ws = static_cast<char *>(workspace);
    b->ws = ws;
    b->head = reinterpret_cast<int *>(ws);
    std::vector<BatchReq> R(b->q.size());
    struct Work {
        double cost;
        BatchItem it;
    };
    std::vector<Work> work;
    std::vector<int32_t> syn_list, comb_list;
    int64_t max_nalm = 1;
    for (size_t i = 0; i < b->q.size(); ++i) {
        ReqPlan &q = b->q[i];
        const sht_request &r = q.r;
        const CoefTables &c = *q.c;
        const GeomPlan &p = *q.p;
        const StartTable &s = *q.s;
        BatchReq &d = R[i];
        std::memset(&d, 0, sizeof(d));
        double2 *delta = reinterpret_cast<double2 *>(ws + q.delta_off);
        double2 *aux = reinterpret_cast<double2 *>(ws + q.aux_off);
        d.kind = r.kind == SHT_ALM2MAP ? 0 : 1;
        d.shape = q.shape;
        d.T = q.T;
        d.syn = SynArgs{r.lmax, r.mmax, p.nslots, p.nrings, c.nalm, aux, c.alpha, s.lstart, s.state, p.slot_x,
                        p.slot_north, p.slot_south, delta};
        d.ana = AnaArgs{r.lmax, r.mmax, p.nslots, p.nrings, c.nalm, delta, c.alpha, c.cfac, s.lstart, s.state,
                        p.slot_x, p.slot_north, p.slot_south, static_cast<double2 *>(r.out), aux};
        d.alm_in = static_cast<const double2 *>(r.in);
        max_nalm = std::max<int64_t>(max_nalm, c.nalm);
        const int lmax = r.lmax;
        // the cost of a unit: slot-recurrence steps of its busiest wave
        auto steps = [&](int m) { return (double)(lmax - m + 1); };
        if (d.kind == 0) {
            d.tiles = (p.nslots + 64 * q.T - 1) / (64 * q.T);
            d.nunits = (r.mmax + 1) * d.tiles;
            d.groups = 1;
            for (int u0 = 0; u0 < d.nunits; u0 += kBlock / 64)
                work.push_back(Work{steps(u0 / d.tiles) * q.T, BatchItem{(int32_t)i, u0}});
            syn_list.push_back((int32_t)i);
        } else if (q.shape == kShapeWave) {
            d.tiles = 1;
            d.nunits = r.mmax + 1;
            d.groups = 1;
            for (int m0 = 0; m0 <= r.mmax; m0 += kBlock / 64)
                work.push_back(Work{steps(m0) * q.T, BatchItem{(int32_t)i, m0}});
        } else {
            d.groups = ana_groups_of(p.nslots, q.T);
            d.tiles = d.groups;
            d.nunits = (r.mmax + 1) * d.groups;
            for (int m = 0; m <= r.mmax; ++m)
                for (int g = 0; g < d.groups; ++g)
                    work.push_back(Work{steps(m) * q.T, BatchItem{(int32_t)i, m * d.groups + g}});
            if (d.groups > 1) comb_list.push_back((int32_t)i);
            else d.ana.part = nullptr;
        }
    }
    // longest first; equal costs keep request order (deterministic queue)
    std::stable_sort(work.begin(), work.end(), [](const Work &a, const Work &b2) { return a.cost > b2.cost; });
    std::vector<BatchItem> items(work.size());
    for (size_t k = 0; k < work.size(); ++k) items[k] = work[k].it;
    if (items.size() >= (size_t)INT32_MAX) return SHT_EUNSUPPORTED;
    b->nitems = (int)items.size();
    b->nsyn = (int)syn_list.size();
    b->ncomb = (int)comb_list.size();
    b->syn_chunks = b->comb_chunks = (int)std::min<int64_t>(4096, (max_nalm + kBlock - 1) / kBlock);
    if ((rc = upload_vec(b.get(), R, &b->reqs)) || (rc = upload_vec(b.get(), items, &b->items)) ||
        (rc = upload_vec(b.get(), syn_list, &b->syn_list)) || (rc = upload_vec(b.get(), comb_list, &b->comb_list)) ||
        (rc = leg_batch_grid(&b->grid)))
        return rc;
    // ring stages: a plan entry per (request, length class), and per class and
    // direction the list of (entry, job) of every request
    std::vector<RingPlan> rplans;
    std::vector<int2> rjobs[2][kFftClasses];  // [0] analysis, [1] synthesis
    size_t rlds[2][kFftClasses] = {};
    for (size_t i = 0; i < b->q.size(); ++i) {
        const ReqPlan &q = b->q[i];
        const bool syn = q.r.kind == SHT_ALM2MAP;
        const DeltaLayout dl = delta_layout(q.h.nrings, q.r.mmax, 1, false);
        for (int c = 0; c < kFftClasses; ++c) {
            if (!q.p->class_count[c]) continue;
            size_t lds = 0;
            RingPlan P = ring_plan(*q.p, c, q.r.mmax, 1, dl, syn, &lds);
            if (syn) {
                P.din = reinterpret_cast<const double2 *>(b->ws + q.delta_off);
                P.mout = static_cast<double *>(q.r.out);
            } else {
                P.min = static_cast<const double *>(q.r.in);
                P.dout = reinterpret_cast<double2 *>(b->ws + q.delta_off);
            }
            const int e = (int)rplans.size();
            rplans.push_back(P);
            rlds[syn][c] = std::max(rlds[syn][c], lds);
            for (int j = 0; j < q.p->class_count[c]; ++j) rjobs[syn][c].push_back(make_int2(e, j));
        }
    }
    RingPlan *dplans = nullptr;
    if ((rc = upload_vec(b.get(), rplans, &dplans))) return rc;
    for (int dir = 0; dir < 2; ++dir) {
        RingBatch &rb = dir ? b->ring_syn : b->ring_ana;
        rb.plans = dplans;
        for (int c = 0; c < kFftClasses; ++c) {
            if (rjobs[dir][c].size() >= (size_t)INT32_MAX) return SHT_EUNSUPPORTED;
            rb.njobs[c] = (int)rjobs[dir][c].size();
            rb.lds[c] = rlds[dir][c];
            int2 *dj = nullptr;
            if (rb.njobs[c] && (rc = upload_vec(b.get(), rjobs[dir][c], &dj))) return rc;
            rb.jobs[c] = dj;
        }
    }
    *out = b.release();
    return SHT_OK;
}

int sht_batch_run(sht_batch *b, void *stream) {
    if (!b) return SHT_EINVAL;
    int dev = -1;
    SHT_HIP(hipGetDevice(&dev));
    if (dev != b->dev) return SHT_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int rc;
    // ring analysis of the map2alm requests (Delta^S), then the Legendre stage
    // of every request in one persistent launch, then the ring synthesis of
    // the alm2map requests; each ring stage one launch per length class over
    // the jobs of every request
    if ((rc = launch_fft_ana_batch(b->ring_ana, st)) ||
        (rc = launch_prescale_batch(b->reqs, b->syn_list, b->nsyn, b->syn_chunks, st)) ||
        (rc = launch_leg_batch(b->reqs, b->items, b->nitems, b->head, b->grid, st)) ||
        (rc = launch_combine_batch(b->reqs, b->comb_list, b->ncomb, b->comb_chunks, st)) ||
        (rc = launch_fft_syn_batch(b->ring_syn, st)))
        return rc;
    return SHT_OK;
}

void sht_batch_destroy(sht_batch *b) { delete b; }

}  // extern "C"
