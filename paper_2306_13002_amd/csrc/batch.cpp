// batch.cpp -- batched plans: many independent grids in one graph launch.
//
// Problems are grouped into size classes by their largest interior edge
// (<= 64, then buckets of 32).  Each class gets one form and launch shape
// (from the autotuner on the class's largest problem, or the defaults) and a
// work list of (problem, tile) items.  A run is one hipGraph: the halo copies,
// then per class a chain of T persistent work-list launches (classes are
// parallel branches of the graph), then the odd-T tail copies.  The graph is
// captured at the first run with a given (T, field pointers) and replayed
// afterwards.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/stencil.h"
#include "internal.hpp"
#include "plan.hpp"

namespace stn {

stencil_status fail(stencil_status st, const char *fmt, ...);
void logf(const char *fmt, ...);
stencil_status hip_fail(hipError_t e, const char *what);
stencil_status validate_desc(const stencil_desc *d, Geom &g, int &rz);
void free_plan(stencil_plan_s *p);

namespace {

int size_class(const Geom &g) {
    const int m = std::max(g.nx, std::max(g.ny, g.nz));
    return m <= 64 ? 0 : (m - 65) / 32 + 1;
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
        // a two-sweep class starts an odd sweep count with one single sweep
        const int per = sweeps_per_launch(C.variant);
        for (int t = 0; t < T;) {
            const int v = (t == 0 && (T % per)) ? V_SATURATED : C.variant;
            const int adv = sweeps_per_launch(v);
            double *part = (t + adv == T) ? b->d_part + C.item_base : nullptr;
            if ((e = p->ops->batch_launch(v, C.tile, b->d_probs, b->d_items + C.item_base, C.n_items, launches[c] & 1,
                                          C.grid, part, s)) != hipSuccess)
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
        stencil_desc d = ds[rep[c]];
        d.variant = ds[0].variant;
        d.tune = ds[0].tune;
        d.tile_x = ds[0].tile_x;
        d.tile_y = ds[0].tile_y;
        d.zblock = ds[0].zblock;
        d.tile_map = 1;
        stencil_plan_t rp = nullptr;
        if ((st = stencil_plan(&d, &rp)) != STENCIL_OK) break;
        BatchClass C;
        C.variant = rp->variant;
        C.tile = rp->tile;
        free_plan(rp);
        C.item_base = (int)items.size();
        for (int i = 0; i < count; ++i) {
            if (cls[i] != c) continue;
            b->prob_class[i] = (int)b->classes.size();
            const Geom &g = geoms[i];
            seg[i] = (int)items.size();
            const int gx = (int)cdiv(g.nx, C.tile.tx), gy = (int)cdiv(g.ny, C.tile.ty), gz = (int)cdiv(g.nz, C.tile.tz);
            for (int z = 0; z < gz; ++z)
                for (int y = 0; y < gy; ++y)
                    for (int x = 0; x < gx; ++x) items.push_back({i, x, y, z});
            seg[count + i] = (int)items.size();
        }
        C.n_items = (int)items.size() - C.item_base;
        C.grid = std::min(C.n_items, 2048);
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
