// batch.cpp -- batched plans: many independent grids in one graph launch.
//
// Problems are grouped into size classes by their largest interior edge
// (<= 64, then buckets of 32).  Each class gets one form and launch shape
// (tuned by timing the class's own work list over all its problems, or the
// defaults) and a work list of (problem, tile) items.  A run is one hipGraph: the halo copies,
// then per class a chain of T work-list launches (classes are
// parallel branches of the graph), then the odd-T tail copies.  The graph is
// captured at the first run with a given (T, field pointers) and replayed
// afterwards.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/stencil.h"
#include "internal.hpp"
#include "plan.hpp"
#include "tune.hpp"

namespace stn {

stencil_status fail(stencil_status st, const char *fmt, ...);
void logf(const char *fmt, ...);
stencil_status hip_fail(hipError_t e, const char *what);
stencil_status validate_desc(const stencil_desc *d, Geom &g, int &rz);
void free_plan(stencil_plan_s *p);

namespace {

// Blocks of a work-list launch (at most).  One block per item: the hardware
// dispatcher then overlaps one item's priming with another's sweep, which a
// block walking its items in turn cannot (2048 looping blocks measured 8 %
// slower for the single-sweep classes, 1 % for the two-sweep ones).
constexpr int kBatchGrid = 1 << 20;
// Work lists at least this long are dealt to the XCDs in contiguous chunks.
constexpr int kXcdChunkItems = 2048;

int size_class(const Geom &g) {
    const int m = std::max(g.nx, std::max(g.ny, g.nz));
    return m <= 64 ? 0 : (m - 65) / 32 + 1;
}

// The work list of one class at launch shape t: items of the class's
// problems in spatial order (problem, z, y, x), each with its residual slot,
// then arranged for the XCDs.  Block j of a launch runs on XCD j mod 8 and
// visits items j, j + grid, ... (grid a multiple of 8 when there are enough
// items): list position q goes to XCD q mod 8, so the spatial order is cut
// into eight contiguous chunks, chunk x filling positions x, x + 8, ...
// Tiles that share halo cells then run on one XCD at about the same time and
// the shared cells come from its L2.  seg (optional) receives each problem's
// [begin, end) slot range relative to the class.
std::vector<BatchItem> class_items(const std::vector<int> &members, const std::vector<Geom> &geoms, Tile t,
                                   std::vector<std::pair<int, int>> *seg) {
    std::vector<BatchItem> ci;
    for (int i : members) {
        const Geom &g = geoms[i];
        const int b0 = (int)ci.size();
        const int gx = (int)cdiv(g.nx, t.tx), gy = (int)cdiv(g.ny, t.ty), gz = (int)cdiv(g.nz, t.tz);
        for (int z = 0; z < gz; ++z)
            for (int y = 0; y < gy; ++y)
                for (int x = 0; x < gx; ++x) ci.push_back({i, x, y, z, (int)ci.size()});
        if (seg) seg->push_back({b0, (int)ci.size()});
    }
    const int n = (int)ci.size();
    if (n >= kXcdChunkItems) {
        const int chunk = (int)cdiv(n, 8);
        std::vector<BatchItem> perm;
        perm.reserve(n);
        for (int q = 0; q < 8 * chunk; ++q) {
            const int sidx = (q & 7) * chunk + (q >> 3);
            if (sidx < n) perm.push_back(ci[sidx]);
        }
        ci.swap(perm);
    }
    return ci;
}

// Tune one size class where it runs: every candidate form and shape is timed
// as the class's work-list kernel over all of the class's problems, on
// scratch grids of their extents.  The class's working set is the sum of its
// problems' and mostly leaves the Infinity Cache, which the largest problem
// timed alone does not show (its best shape can lose by 25 % in the batch).
stencil_status tune_class(const std::vector<int> &members, const std::vector<Geom> &geoms, double cc, double cn,
                          const TuneRequest &rq, TuneEntry *best) {
    int big = members[0];
    for (int i : members)
        if ((long long)geoms[i].nx * geoms[i].ny * geoms[i].nz >
            (long long)geoms[big].nx * geoms[big].ny * geoms[big].nz)
            big = i;
    TuneRequest r = rq;
    r.tile_map = 1;  // work lists fix the block order themselves
    const std::vector<Cand> cands = tune_candidates(&heat3d7_ops, STENCIL_HEAT3D7, geoms[big], r);
    if (cands.empty()) return fail(STENCIL_E_UNSUPPORTED, "no launch shape matches the requested tile fields");
    const int m = (int)members.size();
    struct Scratch {
        std::vector<void *> ptrs;
        hipStream_t s = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Scratch() {
            for (void *q : ptrs)
                if (q) (void)hipFree(q);
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            if (s) (void)hipStreamDestroy(s);
        }
    } sc;
    hipError_t e;
    if ((e = hipStreamCreate(&sc.s)) != hipSuccess) return hip_fail(e, "hipStreamCreate");
    if ((e = hipEventCreate(&sc.e0)) != hipSuccess || (e = hipEventCreate(&sc.e1)) != hipSuccess)
        return hip_fail(e, "hipEventCreate");
    std::vector<BatchProb> probs(m);
    std::vector<Geom> tg(geoms);  // dense copies of the members' layouts
    for (int k = 0; k < m; ++k) {
        Geom g = geoms[members[k]];
        g.py = g.nx + 2;
        g.pz = (long long)(g.nx + 2) * (g.ny + 2);
        tg[members[k]] = g;
        const long long n = g.pz * (g.nz + 2);
        for (int f = 0; f < 2; ++f) {
            void *q = nullptr;
            if ((e = hipMalloc(&q, sizeof(double) * (size_t)n)) != hipSuccess)
                return fail(STENCIL_E_NOMEM, "class tuning buffers: %s", hipGetErrorString(e));
            sc.ptrs.push_back(q);
            if ((e = launch_fill(q, n, 8, 1.0, sc.s)) != hipSuccess) return hip_fail(e, "fill");
            probs[k].f[f] = (double *)q;
        }
        probs[k].g = g;
        probs[k].cc = cc;
        probs[k].cn = cn;
    }
    // items refer to problems by their index in `probs`
    std::vector<int> local(m);
    std::vector<Geom> lg(m);
    for (int k = 0; k < m; ++k) {
        local[k] = k;
        lg[k] = tg[members[k]];
    }
    size_t max_items = 0;
    for (const Cand &c : cands) {
        long long n = 0;
        for (const Geom &g : lg) n += cdiv(g.nx, c.tile.tx) * cdiv(g.ny, c.tile.ty) * cdiv(g.nz, c.tile.tz);
        max_items = std::max(max_items, (size_t)n);
    }
    void *d_probs = nullptr, *d_items = nullptr;
    if ((e = hipMalloc(&d_probs, sizeof(BatchProb) * m)) != hipSuccess) return fail(STENCIL_E_NOMEM, "class tuning");
    sc.ptrs.push_back(d_probs);
    if ((e = hipMalloc(&d_items, sizeof(BatchItem) * max_items)) != hipSuccess)
        return fail(STENCIL_E_NOMEM, "class tuning");
    sc.ptrs.push_back(d_items);
    if ((e = hipMemcpyAsync(d_probs, probs.data(), sizeof(BatchProb) * m, hipMemcpyHostToDevice, sc.s)) != hipSuccess)
        return hip_fail(e, "problem table upload");
    auto time_cand = [&](const Cand &c, int T, int reps, double *us) -> hipError_t {
        const std::vector<BatchItem> items = class_items(local, lg, c.tile, nullptr);
        hipError_t err = hipMemcpyAsync(d_items, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice,
                                        sc.s);
        if (err != hipSuccess) return err;
        const int n = (int)items.size(), grid = std::min(n, kBatchGrid);
        std::vector<double> ts;
        for (int rp = 0; rp < reps + 1; ++rp) {  // the first repetition warms up
            if ((err = hipEventRecord(sc.e0, sc.s)) != hipSuccess) return err;
            for (int t = 0; t < T; ++t)
                if ((err = heat3d7_ops.batch_launch(c.variant, c.tile, (const BatchProb *)d_probs,
                                                    (const BatchItem *)d_items, n, t & 1, grid,
                                                    sweeps_per_launch(c.variant), nullptr, sc.s)) !=
                    hipSuccess)
                    return err;
            if ((err = hipEventRecord(sc.e1, sc.s)) != hipSuccess) return err;
            if ((err = hipEventSynchronize(sc.e1)) != hipSuccess) return err;
            float ms = 0;
            if ((err = hipEventElapsedTime(&ms, sc.e0, sc.e1)) != hipSuccess) return err;
            if (rp > 0) ts.push_back(1e3 * ms / (T * sweeps_per_launch(c.variant)));
        }
        std::sort(ts.begin(), ts.end());
        *us = ts[ts.size() / 2];
        return hipSuccess;
    };
    double probe = 0;
    if ((e = time_cand(cands[0], 2, 1, &probe)) != hipSuccess) return hip_fail(e, "class tuning launch");
    const int T = (int)std::min(50.0, std::max(2.0, 1000.0 / std::max(probe, 1.0)));
    TuneEntry bv{};
    bv.us = 1e300;
    std::vector<std::pair<double, size_t>> timed;
    for (size_t i = 0; i < cands.size(); ++i) {
        const Cand &c = cands[i];
        double us = 0;
        if ((e = time_cand(c, T, 3, &us)) != hipSuccess) return hip_fail(e, "class tuning launch");
        logf("tune batch class (%d problems) v=%d tile=(%d,%d,%d): %.2f us/sweep", m, c.variant, c.tile.tx, c.tile.ty,
             c.tile.tz, us);
        timed.push_back({us, i});
    }
    // as for single plans: the candidates within 5 % of the fastest (at most
    // eight) are timed again with more repetitions before the pick
    std::sort(timed.begin(), timed.end());
    for (size_t r = 0; r < timed.size() && r < 8 && timed[r].first <= 1.05 * timed[0].first; ++r) {
        const Cand &c = cands[timed[r].second];
        double us = 0;
        if ((e = time_cand(c, T, 9, &us)) != hipSuccess) return hip_fail(e, "class tuning launch");
        if (us < bv.us) {
            bv.us = us;
            bv.variant = c.variant;
            bv.tile = c.tile;
            bv.remap = 0;
        }
    }
    if ((e = hipStreamSynchronize(sc.s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    *best = bv;
    return STENCIL_OK;
}

// Cache key of a class: its problems' extents (in descriptor order) and the
// request's fixed fields.
std::string class_key(const std::vector<int> &members, const std::vector<Geom> &geoms, const TuneRequest &rq) {
    unsigned h = 2166136261u;
    for (int i : members)
        for (int v : {geoms[i].nx, geoms[i].ny, geoms[i].nz}) h = (h ^ (unsigned)v) * 16777619u;
    char buf[256];
    // "/c7": the candidate set of single plans' set 7 (entries of earlier sets
    // are not reused)
    std::snprintf(buf, sizeof buf, "batch/k%d/m%d/h%08x/v%d/t%d,%d,%d/c7", STENCIL_HEAT3D7, (int)members.size(), h,
                  rq.variant, rq.tile_x, rq.tile_y, rq.zblock);
    return buf;
}

void destroy_graph(BatchState *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_T = -1;
    b->graph_fields.clear();
}

stencil_status capture(stencil_plan_s *p, void *const *fields, int T, hipStream_t user) {
    BatchState *b = p->batch;
    hipError_t e;
    destroy_graph(b);
    // field pointers into the device problem table, ordered on the user stream
    for (int i = 0; i < b->count; ++i) {
        b->probs[i].f[0] = (double *)fields[2 * i];
        b->probs[i].f[1] = (double *)fields[2 * i + 1];
    }
    if ((e = hipMemcpyAsync(b->d_probs, b->probs.data(), sizeof(BatchProb) * b->count, hipMemcpyHostToDevice, user)) !=
        hipSuccess)
        return hip_fail(e, "problem table upload");
    if ((e = hipStreamSynchronize(user)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    hipStream_t cap = b->cap;
    if ((e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_fail(e, "hipStreamBeginCapture");
    auto abort_capture = [&](hipError_t err, const char *what) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(cap, &g);
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(err, what);
    };
    for (int i = 0; i < b->count; ++i)
        if ((e = launch_halo_copy(fields[2 * i], fields[2 * i + 1], 8, b->probs[i].g, 1, cap)) != hipSuccess)
            return abort_capture(e, "halo copy");
    const int nc = (int)b->classes.size();
    std::vector<int> launches(nc, 0);  // per class; each launch flips the problems' buffers
    if ((e = hipEventRecord(b->evs[0], cap)) != hipSuccess) return abort_capture(e, "fork");
    for (int c = 0; c < nc; ++c) {
        const BatchClass &C = b->classes[c];
        hipStream_t s = b->side[c];
        if ((e = hipStreamWaitEvent(s, b->evs[0], 0)) != hipSuccess) return abort_capture(e, "fork wait");
        // a two-sweep class starts an odd sweep count with one single sweep; a
        // three-sweep class starts with one launch of the remainder's sweeps
        const int per = sweeps_per_launch(C.variant), rem = T % per;
        for (int t = 0; t < T;) {
            const int v = (t == 0 && rem && C.variant != V_SAT3) ? V_SATURATED : C.variant;
            const int adv = (t == 0 && rem) ? (v == V_SAT3 ? rem : 1) : sweeps_per_launch(v);
            double *part = (t + adv == T) ? b->d_part + C.item_base : nullptr;
            if ((e = p->ops->batch_launch(v, C.tile, b->d_probs, b->d_items + C.item_base, C.n_items, launches[c] & 1,
                                          C.grid, adv, part, s)) != hipSuccess)
                return abort_capture(e, "batch sweep");
            t += adv;
            ++launches[c];
        }
        if ((e = hipEventRecord(b->evs[1 + c], s)) != hipSuccess) return abort_capture(e, "join");
        if ((e = hipStreamWaitEvent(cap, b->evs[1 + c], 0)) != hipSuccess) return abort_capture(e, "join wait");
    }
    for (int i = 0; i < b->count; ++i)
        if (launches[b->prob_class[i]] & 1)
            if ((e = launch_interior_copy(fields[2 * i + 1], fields[2 * i], 8, b->probs[i].g, 1, cap)) != hipSuccess)
                return abort_capture(e, "tail copy");
    if ((e = hipStreamEndCapture(cap, &b->graph)) != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess)
        return hip_fail(e, "hipGraphInstantiate");
    b->graph_T = T;
    b->graph_fields.assign(fields, fields + 2 * b->count);
    logf("batch graph captured: %d problems, %d classes, T=%d", b->count, nc, T);
    return STENCIL_OK;
}

}  // namespace

void free_batch(BatchState *b) {
    if (!b) return;
    destroy_graph(b);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_probs) (void)hipFree(b->d_probs);
    if (b->d_seg) (void)hipFree(b->d_seg);
    if (b->d_part) (void)hipFree(b->d_part);
    if (b->d_res) (void)hipFree(b->d_res);
    if (b->h_res) (void)hipHostFree(b->h_res);
    for (hipEvent_t ev : b->evs)
        if (ev) (void)hipEventDestroy(ev);
    for (hipStream_t s : b->side)
        if (s) (void)hipStreamDestroy(s);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
}

stencil_status batch_run(stencil_plan_s *p, void *const *fields, int T, hipStream_t s) {
    BatchState *b = p->batch;
    for (int i = 0; i < 2 * b->count; ++i) {
        if (!fields[i] || (uintptr_t)fields[i] % 8) return fail(STENCIL_E_INVAL, "batch field %d is NULL or misaligned", i);
        if ((i & 1) && fields[i] == fields[i - 1]) return fail(STENCIL_E_INVAL, "problem %d: fields must be distinct", i / 2);
    }
    if (T == 0) return STENCIL_OK;
    p->has_resid = false;
    const bool same = b->graph_T == T && b->exec &&
                      std::equal(b->graph_fields.begin(), b->graph_fields.end(), fields);
    stencil_status st;
    if (!same && (st = capture(p, fields, T, s)) != STENCIL_OK) return st;
    hipError_t e;
    if (p->profiling && (e = hipEventRecord(p->ev0, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    if ((e = hipGraphLaunch(b->exec, s)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    if (p->profiling) {
        if ((e = hipEventRecord(p->ev1, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        p->prof_sweeps = T;
        p->prof_valid = true;
    }
    p->has_resid = true;
    return STENCIL_OK;
}

stencil_status batch_residuals(stencil_plan_s *p, double *out, int count, hipStream_t s) {
    BatchState *b = p->batch;
    hipError_t e;
    if ((e = launch_segment_sums(b->d_part, b->d_seg, b->count, b->d_res, s)) != hipSuccess)
        return hip_fail(e, "segment sums");
    if ((e = hipMemcpyAsync(b->h_res, b->d_res, sizeof(double) * b->count, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (count == 1 && b->count != 1) {
        double t = 0.0;
        for (int i = 0; i < b->count; ++i) t += b->h_res[i];
        out[0] = t;
    } else {
        std::memcpy(out, b->h_res, sizeof(double) * b->count);
    }
    return STENCIL_OK;
}

}  // namespace stn

using namespace stn;

extern "C" stencil_status stencil_plan_batch(const stencil_desc *ds, int32_t count, stencil_plan_t *out) {
    if (!out) return fail(STENCIL_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!ds || count < 1 || count > (1 << 20)) return fail(STENCIL_E_INVAL, "need 1..2^20 descriptors");
    std::vector<Geom> geoms(count);
    for (int i = 0; i < count; ++i) {
        int rz = 0;
        stencil_status st = validate_desc(&ds[i], geoms[i], rz);
        if (st != STENCIL_OK) return fail(st, "descriptor %d: %s", i, stencil_last_error());
        if (ds[i].kind != STENCIL_HEAT3D7)
            return fail(STENCIL_E_UNSUPPORTED, "batched plans are offered for HEAT3D7 only (descriptor %d)", i);
        if (ds[i].bc != STENCIL_BC_DIRICHLET)
            return fail(STENCIL_E_UNSUPPORTED, "batched plans need Dirichlet boundaries (descriptor %d)", i);
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(STENCIL_E_DEVICE, "no HIP device available");
    stencil_plan_s *p = new (std::nothrow) stencil_plan_s();
    if (!p) return fail(STENCIL_E_NOMEM, "host allocation failed");
    p->kind = STENCIL_HEAT3D7;
    p->dtype = STENCIL_F64;
    p->ops = &heat3d7_ops;
    (void)hipGetDevice(&p->device);
    BatchState *b = new (std::nothrow) BatchState();
    if (!b) {
        delete p;
        return fail(STENCIL_E_NOMEM, "host allocation failed");
    }
    p->batch = b;
    b->count = count;
    b->probs.resize(count);
    b->prob_class.assign(count, 0);
    // classes and their forms: tuned (or default) on the class's largest problem
    std::vector<int> cls(count);
    int ncls = 0;
    for (int i = 0; i < count; ++i) ncls = std::max(ncls, (cls[i] = size_class(geoms[i])) + 1);
    std::vector<int> rep(ncls, -1);
    for (int i = 0; i < count; ++i) {
        b->probs[i].g = geoms[i];
        b->probs[i].cc = ds[i].coef[0];
        b->probs[i].cn = ds[i].coef[1];
        const long long v = (long long)geoms[i].nx * geoms[i].ny * geoms[i].nz;
        const int r = rep[cls[i]];
        if (r < 0 || v > (long long)geoms[r].nx * geoms[r].ny * geoms[r].nz) rep[cls[i]] = i;
    }
    std::vector<BatchItem> items;
    std::vector<int> seg(2 * count, 0);
    hipError_t e;
    stencil_status st = STENCIL_OK;
    for (int c = 0; c < ncls && st == STENCIL_OK; ++c) {
        if (rep[c] < 0) continue;
        std::vector<int> members;
        for (int i = 0; i < count; ++i)
            if (cls[i] == c) members.push_back(i);
        stencil_desc d = ds[rep[c]];
        d.variant = ds[0].variant;
        d.tune = STENCIL_TUNE_FIXED;  // validates the request and resolves the defaults
        d.tile_x = ds[0].tile_x;
        d.tile_y = ds[0].tile_y;
        d.zblock = ds[0].zblock;
        d.tile_map = 1;
        BatchClass C;
        const bool open = !is_point_form(d.variant) &&
                          (d.variant == STENCIL_AUTO || !d.tile_x || !d.tile_y || !d.zblock);
        bool tuned = false;
        if (ds[0].tune != STENCIL_TUNE_FIXED && open) {  // EXHAUSTIVE and MODEL: timed in place
            const TuneRequest rq{d.variant, d.tile_x, d.tile_y, d.zblock, 1};
            const std::string key = class_key(members, geoms, rq);
            TuneEntry te{};
            if (tune_lookup(key, &te)) {
                tuned = true;
            } else {
                st = tune_class(members, geoms, ds[rep[c]].coef[0], ds[rep[c]].coef[1], rq, &te);
                if (st == STENCIL_OK) {
                    tune_store(key, te);
                    tuned = true;
                } else if (st == STENCIL_E_NOMEM) {  // no room for the class's scratch grids
                    logf("%s; tuning class %d on its largest problem alone", stencil_last_error(), c);
                    d.tune = ds[0].tune;
                    st = STENCIL_OK;
                } else {
                    break;
                }
            }
            if (tuned) {
                C.variant = te.variant;
                C.tile = te.tile;
            }
        }
        if (!tuned) {
            stencil_plan_t rp = nullptr;
            if ((st = stencil_plan(&d, &rp)) != STENCIL_OK) break;
            C.variant = rp->variant;
            C.tile = rp->tile;
            free_plan(rp);
        }
        C.item_base = (int)items.size();
        std::vector<std::pair<int, int>> ranges;
        std::vector<BatchItem> ci = class_items(members, geoms, C.tile, &ranges);
        for (size_t k = 0; k < members.size(); ++k) {
            const int i = members[k];
            b->prob_class[i] = (int)b->classes.size();
            seg[i] = C.item_base + ranges[k].first;
            seg[count + i] = C.item_base + ranges[k].second;
        }
        C.n_items = (int)ci.size();
        C.grid = std::min(C.n_items, kBatchGrid);
        items.insert(items.end(), ci.begin(), ci.end());
        logf("batch class %d: rep %d variant=%d tile=(%d,%d,%d) items=%d", c, rep[c], C.variant, C.tile.tx, C.tile.ty,
             C.tile.tz, C.n_items);
        b->classes.push_back(C);
    }
    if (st != STENCIL_OK) {
        free_plan(p);
        return st;
    }
    b->n_items = (int)items.size();
    p->nblocks = b->n_items;
    p->variant = b->classes[0].variant;
    p->tile = b->classes[0].tile;
    if ((e = hipMalloc(&b->d_items, sizeof(BatchItem) * items.size())) != hipSuccess ||
        (e = hipMalloc(&b->d_probs, sizeof(BatchProb) * count)) != hipSuccess ||
        (e = hipMalloc(&b->d_seg, sizeof(int) * 2 * count)) != hipSuccess ||
        (e = hipMalloc(&b->d_part, sizeof(double) * items.size())) != hipSuccess ||
        (e = hipMalloc(&b->d_res, sizeof(double) * count)) != hipSuccess ||
        (e = hipHostMalloc(&b->h_res, sizeof(double) * count, hipHostMallocDefault)) != hipSuccess) {
        free_plan(p);
        return fail(STENCIL_E_NOMEM, "batch buffers: %s", hipGetErrorString(e));
    }
    if ((e = hipMemcpy(b->d_items, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (e = hipMemcpy(b->d_seg, seg.data(), sizeof(int) * 2 * count, hipMemcpyHostToDevice)) != hipSuccess) {
        free_plan(p);
        return hip_fail(e, "batch tables upload");
    }
    const int nc = (int)b->classes.size();
    b->side.assign(nc, nullptr);
    b->evs.assign(nc + 1, nullptr);
    bool ok = hipStreamCreate(&b->cap) == hipSuccess;
    for (int c = 0; c < nc && ok; ++c) ok = hipStreamCreate(&b->side[c]) == hipSuccess;
    for (int c = 0; c <= nc && ok; ++c) ok = hipEventCreateWithFlags(&b->evs[c], hipEventDisableTiming) == hipSuccess;
    if (ok) ok = hipEventCreate(&p->ev0) == hipSuccess && hipEventCreate(&p->ev1) == hipSuccess;
    if (!ok) {
        free_plan(p);
        return fail(STENCIL_E_DEVICE, "stream/event creation failed");
    }
    *out = p;
    return STENCIL_OK;
}
