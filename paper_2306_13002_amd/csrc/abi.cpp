// abi.cpp -- the C ABI of libstencil.so (declared in include/stencil.h).
//
// Validation happens on the host before any HIP call; a plan owns only its
// residual partials, a one-double result slot, a pinned host double and two
// timing events.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/stencil.h"
#include "internal.hpp"
#include "plan.hpp"
#include "tune.hpp"
#include "rtc.hpp"

using namespace stn;

namespace {

thread_local char g_err[512] = "no error";  // fixed size: reporting an error allocates nothing

bool log_on() {
    static int v = -1;
    if (v < 0) {
        const char *e = std::getenv("STENCIL_LOG");
        v = (e && *e && std::strcmp(e, "0") != 0) ? 1 : 0;
    }
    return v == 1;
}

}  // namespace

namespace stn {

stencil_status fail(stencil_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::memcpy(g_err, buf, sizeof g_err);
    if (log_on()) std::fprintf(stderr, "[stencil] error %d: %s\n", (int)st, buf);
    // a failed allocation leaves its error as the runtime's last error; clear
    // it so that a later launch check does not report it as a launch failure
    if (st == STENCIL_E_NOMEM) (void)hipGetLastError();
    return st;
}

void logf(const char *fmt, ...) {
    if (!log_on()) return;
    va_list ap;
    va_start(ap, fmt);
    std::fprintf(stderr, "[stencil] ");
    std::vfprintf(stderr, fmt, ap);
    std::fprintf(stderr, "\n");
    va_end(ap);
}

stencil_status hip_fail(hipError_t e, const char *what) {
    return fail(STENCIL_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

const KindOps *ops_for(int kind) {
    switch (kind) {
    case STENCIL_HEAT2D5: return &heat2d5_ops;
    case STENCIL_HEAT3D7: return &heat3d7_ops;
    case STENCIL_POISSON19: return &poisson19_ops;
    case STENCIL_WAVE25: return &wave25_ops;
    case STENCIL_GENERIC: return &generic_ops;
    default: return nullptr;
    }
}

int elem_bytes(int dtype) { return dtype == STENCIL_F32 ? 4 : 8; }

// Library defaults (used when a field is left open and tuning is FIXED);
// picked from launch-shape sweeps on MI355X at the workload sizes.
Tile default_tile(int kind, int variant, const Geom &g) {
    if (variant == V_PLAIN) return kind == STENCIL_HEAT2D5 ? Tile{64, 4, 1} : Tile{128, 8, 1};
    if (variant == V_SAT2 && kind == STENCIL_POISSON19) return Tile{64, 8, g.nz < 32 ? g.nz : 32};
    if (variant == V_SAT3) return Tile{28, 28, g.nz < 32 ? g.nz : 32};
    switch (kind) {
    case STENCIL_HEAT3D7: return Tile{32, 8, g.nz < 8 ? g.nz : 8};
    case STENCIL_POISSON19: return Tile{128, 4, g.nz < 32 ? g.nz : 32};
    case STENCIL_WAVE25: return Tile{64, 32, g.nz < 256 ? g.nz : 256};
    default: return Tile{64, 4, 16};
    }
}

int default_remap(int) { return 1; }

// GENERIC: build the plain and saturated tap tables and upload them.
// Plain keeps the caller's order.  Saturated groups taps by (dz, coefficient
// id), groups ordered by dz slot then id, taps in a group by address.
stencil_status build_generic_tables(stencil_plan_s *p, const stencil_desc *d) {
    const int n = d->n_taps, r = p->g.r, ns = 2 * r + 1;
    std::vector<int> slot_g(ns + 1, 0), g_t, t_xy;
    std::vector<long long> off(n);  // 64-bit: a plane pitch may exceed INT_MAX / r
    std::vector<double> c(n), g_c;
    unsigned h = 2166136261u;
    for (int t = 0; t < n; ++t) {
        const int dx = d->tap_off[3 * t], dy = d->tap_off[3 * t + 1], dz = d->tap_off[3 * t + 2];
        off[t] = (long long)dz * p->g.pz + (long long)dy * p->g.py + dx;
        c[t] = d->coef[d->tap_cid[t]];
        for (int v : {dx, dy, dz, d->tap_cid[t]}) h = (h ^ (unsigned)v) * 16777619u;
    }
    p->taps_hash = h;
    for (int s = 0; s < ns; ++s) {
        slot_g[s] = (int)g_c.size();
        for (int id = 0; id < d->n_coef; ++id) {
            std::vector<std::pair<int, int>> mem;  // (dy, dx)
            for (int t = 0; t < n; ++t)
                if (d->tap_off[3 * t + 2] == s - r && d->tap_cid[t] == id)
                    mem.push_back({d->tap_off[3 * t + 1], d->tap_off[3 * t]});
            if (mem.empty()) continue;
            std::sort(mem.begin(), mem.end());
            g_t.push_back((int)t_xy.size());
            g_c.push_back(d->coef[id]);
            for (auto &m : mem) t_xy.push_back((int)(((unsigned)m.first << 16) | ((unsigned)m.second & 0xFFFFu)));
        }
    }
    slot_g[ns] = (int)g_c.size();
    g_t.push_back((int)t_xy.size());
    // one buffer: [slot_g ns+1][g_t ng+1][t_xy n] (ints), then 8-byte words
    // [off n] (int64), [c n][g_c ng] (doubles)
    const size_t ni = slot_g.size() + g_t.size() + t_xy.size();
    const size_t ib = ((ni * sizeof(int)) + 15) & ~size_t(15);
    const size_t total = ib + (off.size() + c.size() + g_c.size()) * 8;
    std::vector<char> host(total, 0);
    int *ip = (int *)host.data();
    size_t o = 0;
    auto put = [&](const std::vector<int> &v) { std::memcpy(ip + o, v.data(), v.size() * sizeof(int)); size_t at = o; o += v.size(); return at; };
    const size_t o_slot = put(slot_g), o_gt = put(g_t), o_xy = put(t_xy);
    std::memcpy(host.data() + ib, off.data(), off.size() * sizeof(long long));
    double *dp = (double *)(host.data() + ib + off.size() * sizeof(long long));
    std::memcpy(dp, c.data(), c.size() * sizeof(double));
    std::memcpy(dp + c.size(), g_c.data(), g_c.size() * sizeof(double));
    hipError_t e;
    if ((e = hipMalloc(&p->d_tab, total)) != hipSuccess)
        return fail(STENCIL_E_NOMEM, "hipMalloc tap tables: %s", hipGetErrorString(e));
    if ((e = hipMemcpy(p->d_tab, host.data(), total, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "hipMemcpy tap tables");
    const int *di = (const int *)p->d_tab;
    const long long *dl = (const long long *)((const char *)p->d_tab + ib);
    const double *dd = (const double *)(dl + off.size());
    GenTab &t = p->base_args.gen;
    t.off = dl;
    t.c = dd;
    t.n = n;
    t.slot_g = di + o_slot;
    t.g_t = di + o_gt;
    t.g_c = dd + c.size();
    t.t_xy = di + o_xy;
    t.corners = false;
    for (int k = 0; k < n; ++k)
        if (d->tap_off[3 * k] != 0 && d->tap_off[3 * k + 1] != 0) t.corners = true;
    // the same grouping, for the generated saturated kernels
    RtcSpec *sp = new (std::nothrow) RtcSpec();
    if (!sp) return fail(STENCIL_E_NOMEM, "host allocation failed");
    sp->R = r;
    sp->eb = elem_bytes(d->dtype);
    sp->corners = t.corners;
    sp->slots.resize(ns);
    for (int s = 0; s < ns; ++s)
        for (int gi = slot_g[s]; gi < slot_g[s + 1]; ++gi) {
            RtcGroup gr;
            gr.coef = g_c[gi];
            for (int ti = g_t[gi]; ti < g_t[gi + 1]; ++ti) {
                const int xy = t_xy[ti];
                gr.taps.push_back({(short)(xy & 0xFFFF), xy >> 16});
            }
            sp->slots[s].push_back(gr);
        }
    p->rtc = sp;
    const char *tbl = std::getenv("STENCIL_GENERIC_TABLE");
    p->base_args.rtc = (tbl && std::atoi(tbl) != 0) ? nullptr : sp;
    return STENCIL_OK;
}

// Validate the descriptor (host only).  Fills geometry on success.
stencil_status validate_desc(const stencil_desc *d, Geom &g, int &rz) {
    if (!d) return fail(STENCIL_E_INVAL, "descriptor is NULL");
    if (d->struct_size != sizeof(stencil_desc))
        return fail(STENCIL_E_INVAL, "struct_size %u != sizeof(stencil_desc) %zu", d->struct_size,
                    sizeof(stencil_desc));
    const int k = d->kind;
    if (k < STENCIL_HEAT2D5 || k > STENCIL_GENERIC) return fail(STENCIL_E_INVAL, "unknown kind %d", k);
    if (d->dtype != STENCIL_F32 && d->dtype != STENCIL_F64) return fail(STENCIL_E_INVAL, "unknown dtype %d", d->dtype);
    if (d->variant < STENCIL_PLAIN || d->variant > STENCIL_SATURATED_T3)
        return fail(STENCIL_E_INVAL, "unknown variant %d", d->variant);
    if (is_point_form(d->variant) && k != STENCIL_WAVE25 && k != STENCIL_POISSON19)
        return fail(STENCIL_E_UNSUPPORTED, "the per-point ablation forms are offered for WAVE25 and POISSON19");
    if (d->variant == STENCIL_SATURATED_T2 &&
        ((k != STENCIL_POISSON19 && k != STENCIL_HEAT3D7) || d->bc != STENCIL_BC_DIRICHLET))
        return fail(STENCIL_E_UNSUPPORTED, "the two-sweep saturated form is offered for POISSON19 and HEAT3D7 (Dirichlet)");
    if (d->variant == STENCIL_SATURATED_T3 && (k != STENCIL_HEAT3D7 || d->bc != STENCIL_BC_DIRICHLET))
        return fail(STENCIL_E_UNSUPPORTED, "the three-sweep saturated form is offered for HEAT3D7 (Dirichlet)");
    if (d->tune < STENCIL_TUNE_FIXED || d->tune > STENCIL_TUNE_MODEL)
        return fail(STENCIL_E_INVAL, "unknown tune mode %d", d->tune);
    if (d->bc != STENCIL_BC_DIRICHLET && d->bc != STENCIL_BC_PERIODIC)
        return fail(STENCIL_E_INVAL, "unknown boundary condition %d", d->bc);
    const int want_ndim = (k == STENCIL_HEAT2D5) ? 2 : 3;
    if (d->ndim != want_ndim) return fail(STENCIL_E_INVAL, "kind %d needs ndim %d, got %d", k, want_ndim, d->ndim);
    int want_r = (k == STENCIL_WAVE25) ? 4 : 1;
    if (k == STENCIL_GENERIC) {
        if (d->radius < 1 || d->radius > 4) return fail(STENCIL_E_INVAL, "generic radius %d not in 1..4", d->radius);
        want_r = d->radius;
    }
    if (d->radius != want_r) return fail(STENCIL_E_INVAL, "kind %d needs radius %d, got %d", k, want_r, d->radius);
    const int nd = d->ndim;
    for (int a = 0; a < nd; ++a)
        if (d->n[a] < 1 || d->n[a] > (1 << 24))
            return fail(STENCIL_E_INVAL, "interior extent n[%d] = %lld out of range [1, 2^24]", a, (long long)d->n[a]);
    const int r = want_r;
    const long long PX = d->n[0] + 2 * r, PY = d->n[1] + 2 * r, PZ = nd == 3 ? d->n[2] + 2 * r : 1;
    const long long py = d->pitch_y ? d->pitch_y : PX;
    const long long pz = nd == 3 ? (d->pitch_z ? d->pitch_z : py * PY) : py * PY;
    if (py < PX) return fail(STENCIL_E_INVAL, "pitch_y %lld < padded row length %lld", py, PX);
    if (nd == 3 && pz < py * PY) return fail(STENCIL_E_INVAL, "pitch_z %lld < pitch_y*padded rows %lld", pz, py * PY);
    if ((double)pz * (double)PZ > 9.0e18) return fail(STENCIL_E_INVAL, "grid too large");
    // dtype per kind
    if ((k == STENCIL_HEAT2D5 || k == STENCIL_HEAT3D7 || k == STENCIL_WAVE25) && d->dtype != STENCIL_F64)
        return fail(STENCIL_E_UNSUPPORTED, "kind %d is offered in F64 only", k);
    if (k == STENCIL_POISSON19 && d->dtype != STENCIL_F32)
        return fail(STENCIL_E_UNSUPPORTED, "POISSON19 is offered with F32 storage only");
    // coefficients
    if (k == STENCIL_HEAT2D5 || k == STENCIL_HEAT3D7) {
        if (!d->coef || d->n_coef != 2) return fail(STENCIL_E_INVAL, "heat kinds need coef = {centre, neighbour}");
    } else if (k == STENCIL_WAVE25) {
        if (!d->coef || d->n_coef != 5) return fail(STENCIL_E_INVAL, "WAVE25 needs 5 coefficients");
    } else if (k == STENCIL_POISSON19) {
        if (!std::isfinite(d->omega)) return fail(STENCIL_E_INVAL, "omega must be finite");
    } else {
        if (!d->coef || d->n_coef < 1) return fail(STENCIL_E_INVAL, "GENERIC needs n_coef >= 1 coefficients");
        if (d->n_taps < 1 || d->n_taps > 729 || !d->tap_off || !d->tap_cid)
            return fail(STENCIL_E_INVAL, "GENERIC needs 1..729 taps with tap_off and tap_cid");
        // the generated saturated kernels go through hipModuleLaunchKernel,
        // which refuses y or z grid dimensions above 65535 blocks
        if (d->variant != STENCIL_PLAIN && (d->n[1] > 65535 || d->n[2] > 65535))
            return fail(STENCIL_E_UNSUPPORTED, "GENERIC saturated kernels need ny, nz <= 65535 (PLAIN takes any extent)");
        for (int t = 0; t < d->n_taps; ++t) {
            for (int a = 0; a < 3; ++a)
                if (d->tap_off[3 * t + a] < -r || d->tap_off[3 * t + a] > r)
                    return fail(STENCIL_E_INVAL, "tap %d offset outside the radius", t);
            if (d->tap_cid[t] < 0 || d->tap_cid[t] >= d->n_coef)
                return fail(STENCIL_E_INVAL, "tap %d coefficient id %d out of range", t, d->tap_cid[t]);
        }
    }
    if (d->coef)
        for (int c = 0; c < d->n_coef; ++c)
            if (!std::isfinite(d->coef[c])) return fail(STENCIL_E_INVAL, "coefficient %d is not finite", c);
    if (d->bc == STENCIL_BC_PERIODIC && k != STENCIL_HEAT2D5 && k != STENCIL_HEAT3D7)
        return fail(STENCIL_E_UNSUPPORTED, "periodic boundaries are offered for the heat kinds only");
    if (d->tile_x < 0 || d->tile_y < 0 || d->zblock < 0) return fail(STENCIL_E_INVAL, "negative tile field");
    g.nx = (int)d->n[0];
    g.ny = (int)d->n[1];
    g.nz = nd == 3 ? (int)d->n[2] : 1;
    g.r = r;
    g.py = py;
    g.pz = pz;
    rz = nd == 3 ? r : 0;
    return STENCIL_OK;
}

// The host-side fields of a plan for a validated descriptor (no device call).
void init_plan_fields(stencil_plan_s *p, const stencil_desc *d, const Geom &g, int rz) {
    p->kind = d->kind;
    p->dtype = d->dtype;
    p->bc = d->bc;
    p->g = g;
    p->rz = rz;
    p->omega = d->omega;
    p->ops = ops_for(d->kind);
    for (int c = 0; c < 5; ++c) p->c[c] = (d->coef && c < d->n_coef) ? d->coef[c] : 0.0;
    p->info = stencil_info(d, g);
    p->base_args.g = g;
    for (int c = 0; c < 5; ++c) p->base_args.c[c] = p->c[c];
    p->base_args.omega = d->omega;
    p->base_args.elem_bytes = elem_bytes(d->dtype);
}

long long span_elems(const stencil_plan_s *p) {
    return (long long)(p->g.nz + 2 * p->rz - 1) * p->g.pz + (long long)(p->g.ny + 2 * p->g.r - 1) * p->g.py +
           (p->g.nx + 2 * p->g.r);
}

stencil_status alloc_plan_buffers(stencil_plan_s *p) {
    hipError_t e;
    p->nblocks = p->ops->nblocks(p->variant, p->tile, p->g);
    if ((e = hipMalloc(&p->d_part, sizeof(double) * (size_t)p->nblocks)) != hipSuccess)
        return fail(STENCIL_E_NOMEM, "hipMalloc residual partials (%lld blocks): %s", p->nblocks, hipGetErrorString(e));
    if ((e = hipMalloc(&p->d_red, sizeof(double) * kReduceBlocks)) != hipSuccess)
        return fail(STENCIL_E_NOMEM, "hipMalloc reduction scratch: %s", hipGetErrorString(e));
    // the reduction writes the residual straight into this pinned, coherent
    // host word (no device-to-host copy per residual)
    if ((e = hipHostMalloc(&p->h_result, sizeof(double), hipHostMallocCoherent)) != hipSuccess)
        return fail(STENCIL_E_NOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
    if ((e = hipEventCreate(&p->ev0)) != hipSuccess || (e = hipEventCreate(&p->ev1)) != hipSuccess)
        return hip_fail(e, "hipEventCreate");
    return STENCIL_OK;
}

void free_batch(BatchState *b);
stencil_status batch_run(stencil_plan_s *p, void *const *fields, int T, hipStream_t s);
stencil_status batch_residuals(stencil_plan_s *p, double *out, int count, hipStream_t s);

void free_plan(stencil_plan_s *p) {
    if (!p) return;
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (p->device >= 0) (void)hipSetDevice(p->device);
    if (p->d_part) (void)hipFree(p->d_part);
    if (p->d_red) (void)hipFree(p->d_red);
    if (p->d_tab) (void)hipFree(p->d_tab);
    free_batch(p->batch);
    if (p->rg) {
        for (hipGraphExec_t x : p->rg->x)
            if (x) (void)hipGraphExecDestroy(x);
        if (p->rg->cap) (void)hipStreamDestroy(p->rg->cap);
        delete p->rg;
    }
    delete p->rtc;
    if (p->h_result) (void)hipHostFree(p->h_result);
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    if (cur >= 0) (void)hipSetDevice(cur);
    delete p;
}

// Make the plan's device current for the lifetime of the guard.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) return;
        ok = (prev == dev) || hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        int now = -1;
        if (prev >= 0 && hipGetDevice(&now) == hipSuccess && now != prev) (void)hipSetDevice(prev);
    }
};

stencil_status choose_config(stencil_plan_s *p, const stencil_desc *d) {
    const KindOps *ops = p->ops;
    bool has_sat = ops->sat_tiles != nullptr;
    int dv = d->variant;
    // the saturated WAVE25 and POISSON19 kernels address a plane with 32-bit
    // byte offsets
    const long long plane_bytes = p->g.pz * (long long)elem_bytes(p->dtype);
    if ((p->kind == STENCIL_WAVE25 || p->kind == STENCIL_POISSON19) && plane_bytes > kMaxPlaneBytes32) {
        if (dv == STENCIL_SATURATED || dv == V_SAT2)
            return fail(STENCIL_E_UNSUPPORTED,
                        "kind %d: the saturated forms need pitch_z*%d <= %lld bytes (PLAIN takes any plane)", p->kind,
                        elem_bytes(p->dtype), kMaxPlaneBytes32);
        has_sat = false;
        if (dv == STENCIL_AUTO) dv = STENCIL_PLAIN;
    }
    if (d->tile_map < 0 || d->tile_map > 2) return fail(STENCIL_E_INVAL, "tile_map %d not in 0..2", d->tile_map);
    if (dv == STENCIL_SATURATED && !has_sat)
        return fail(STENCIL_E_UNSUPPORTED, "kind %d has no saturated form", p->kind);
    const bool open = !is_point_form(dv) && (dv == STENCIL_AUTO || !d->tile_x || !d->tile_y || !d->zblock || !d->tile_map);
    if (d->tune == STENCIL_TUNE_MODEL && open) {
        TuneRequest rq{has_sat ? dv : (int)STENCIL_PLAIN, d->tile_x, d->tile_y, d->zblock, d->tile_map, d->bc};
        TuneEntry e{};
        stencil_status st = tune_model(p, rq, &e);
        if (st == STENCIL_OK) {
            p->variant = e.variant;
            p->tile = e.tile;
            p->remap = e.remap;
            p->tuned = true;
            return STENCIL_OK;
        }
        if (st != STENCIL_E_STATE) return st;
        logf("%s; falling back to exhaustive tuning", stencil_last_error());
    }
    if ((d->tune == STENCIL_TUNE_EXHAUSTIVE || d->tune == STENCIL_TUNE_MODEL) && open) {
        TuneRequest rq{has_sat ? dv : (int)STENCIL_PLAIN, d->tile_x, d->tile_y, d->zblock, d->tile_map, d->bc};
        const std::string key = tune_key(p, rq);
        TuneEntry e{};
        if (!tune_lookup(key, &e)) {
            stencil_status st = tune_exhaustive(p, rq, &e);
            if (st != STENCIL_OK) return st;
            tune_store(key, e);
        }
        p->variant = e.variant;
        p->tile = e.tile;
        p->remap = e.remap;
        p->tuned = true;
        return STENCIL_OK;
    }
    int v = dv;
    if (v == STENCIL_AUTO) v = has_sat ? V_SATURATED : V_PLAIN;
    Tile t = default_tile(p->kind, is_point_form(v) ? V_PLAIN : v, p->g);
    if (d->tile_x) t.tx = d->tile_x;
    if (d->tile_y) t.ty = d->tile_y;
    if (d->zblock) t.tz = d->zblock;
    // HEAT2D5 PLAIN with fused sweeps: square 32 x 32 output tiles unless given
    if (p->kind == STENCIL_HEAT2D5 && t.tz > 1 && !d->tile_x && !d->tile_y) t.tx = t.ty = 32;
    if (!ops->tile_ok(v, t))
        return fail(STENCIL_E_UNSUPPORTED, "tile (%d, %d, %d) is not offered for kind %d variant %d", t.tx, t.ty, t.tz,
                    p->kind, v);
    if (p->kind == STENCIL_HEAT2D5 && t.tz > 1 && p->bc != STENCIL_BC_DIRICHLET)
        return fail(STENCIL_E_UNSUPPORTED, "HEAT2D5: fused sweeps (zblock > 1) need Dirichlet boundaries");
    p->variant = v;
    p->tile = t;
    p->remap = d->tile_map ? (d->tile_map == 2) : default_remap(p->kind);
    return STENCIL_OK;
}

// Check a single (non-batch) run's grid pointers against the plan and fill
// the launch arguments.  Host only; nothing is enqueued.
stencil_status prepare_run_args(const stencil_plan_s *p, void *const *fields, const void *const *coef_arrays,
                                SweepArgs &a) {
    if (!fields[0] || !fields[1]) return fail(STENCIL_E_INVAL, "fields[0] and fields[1] are required");
    if (fields[0] == fields[1]) return fail(STENCIL_E_INVAL, "fields[0] and fields[1] must be distinct");
    const int eb = elem_bytes(p->dtype);
    for (int f = 0; f < 2; ++f)
        if ((uintptr_t)fields[f] % eb) return fail(STENCIL_E_INVAL, "fields[%d] is not %d-byte aligned", f, eb);
    // Both fields are written, so their padded spans must be disjoint, and a
    // read-only coefficient grid must not overlap either of them.
    const uintptr_t span = (uintptr_t)span_elems(p) * (uintptr_t)eb;
    auto overlaps = [span](const void *x, const void *y, uintptr_t ybytes) {
        const uintptr_t a0 = (uintptr_t)x, b0 = (uintptr_t)y;
        return a0 < b0 + ybytes && b0 < a0 + span;
    };
    if (overlaps(fields[0], fields[1], span))
        return fail(STENCIL_E_INVAL, "fields[0] and fields[1] overlap (padded span %lld elements)", span_elems(p));
    a = p->base_args;
    a.remap = p->remap;
    if (p->kind == STENCIL_POISSON19) {
        if (!coef_arrays) return fail(STENCIL_E_INVAL, "POISSON19 needs 12 coefficient arrays");
        for (int c = 0; c < 12; ++c) {
            if (!coef_arrays[c] || (uintptr_t)coef_arrays[c] % 4)
                return fail(STENCIL_E_INVAL, "coefficient array %d is NULL or misaligned", c);
            a.coefs[c] = coef_arrays[c];
        }
    } else if (p->kind == STENCIL_WAVE25) {
        if (!coef_arrays || !coef_arrays[0] || (uintptr_t)coef_arrays[0] % 8)
            return fail(STENCIL_E_INVAL, "WAVE25 needs coef_arrays = {vsq} (F64, aligned)");
        a.coefs[0] = coef_arrays[0];
    }
    const int ncoef_arrays = p->kind == STENCIL_POISSON19 ? 12 : (p->kind == STENCIL_WAVE25 ? 1 : 0);
    for (int c = 0; c < ncoef_arrays; ++c)
        for (int f = 0; f < 2; ++f)
            if (overlaps(fields[f], coef_arrays[c], span))
                return fail(STENCIL_E_INVAL, "coefficient array %d overlaps fields[%d]", c, f);
    return STENCIL_OK;
}

// The three parts of a run on stream s (enqueued eagerly or under capture).
// Jacobi kinds first copy the state's halo into the scratch grid.
hipError_t run_pre(stencil_plan_s *p, void *const *fields, hipStream_t s) {
    if (p->kind == STENCIL_WAVE25 || p->bc != STENCIL_BC_DIRICHLET) return hipSuccess;
    // fused HEAT2D5 sweeps write the scratch grid's boundary ring themselves
    if (p->kind == STENCIL_HEAT2D5 && launch_sweeps(p->kind, p->variant, p->tile) > 1) return hipSuccess;
    return launch_halo_copy(fields[0], fields[1], elem_bytes(p->dtype), p->g, p->rz, s);
}

// Jacobi kinds read fields[0] first; the leapfrog reads the newer level
// fields[1] and overwrites the older fields[0] in place.  A launch of the
// two-sweep form advances two sweeps; an odd count starts with one single
// saturated sweep at the same shape, so the last launch (the one that leaves
// the residual partials) is always of the plan's form.
hipError_t run_sweeps(stencil_plan_s *p, void *const *fields, SweepArgs a, int iterations, hipStream_t s,
                      int *launches, double *part) {
    const bool wave = p->kind == STENCIL_WAVE25;
    const int eb = elem_bytes(p->dtype);
    void *src = wave ? fields[1] : fields[0], *dst = wave ? fields[0] : fields[1];
    // sweeps per launch: the two-sweep form does two (an odd count starts with
    // one single-sweep launch); fused HEAT2D5 sweeps do tile.tz and the
    // three-sweep form three (the first launch takes the remainder of the
    // count)
    const int per = launch_sweeps(p->kind, p->variant, p->tile);
    const bool fused = (p->kind == STENCIL_HEAT2D5 && per > 1) || p->variant == V_SAT3;
    hipError_t e;
    *launches = 0;
    for (int t = 0; t < iterations;) {
        if (p->bc == STENCIL_BC_PERIODIC && (e = launch_periodic_fill(src, eb, p->g, p->rz, s)) != hipSuccess)
            return e;
        const int first = iterations % per;
        const int v = (!fused && t == 0 && first) ? V_SATURATED : p->variant;
        const int adv = fused ? (t == 0 && first ? first : per) : sweeps_per_launch(v);
        a.sweeps = adv;
        a.src = src;
        a.dst = dst;
        a.part = (t + adv == iterations) ? part : nullptr;
        if ((e = p->ops->launch(v, p->tile, a, s)) != hipSuccess) return e;
        t += adv;
        ++*launches;
        std::swap(src, dst);
    }
    return hipSuccess;
}

// An odd launch count leaves a Jacobi result in the scratch grid: copy it back.
hipError_t run_post(stencil_plan_s *p, void *const *fields, int launches, hipStream_t s) {
    if (p->kind == STENCIL_WAVE25 || !(launches & 1)) return hipSuccess;
    return launch_interior_copy(fields[1], fields[0], elem_bytes(p->dtype), p->g, p->rz, s);
}

// Capture the three parts into p->rg->x (replacing earlier graphs).  Every
// node is a kernel launch.  On failure no graph is kept and no error is left.
hipError_t capture_run(stencil_plan_s *p, void *const *fields, const SweepArgs &a, int iterations) {
    RunGraphs *rg = p->rg;
    for (hipGraphExec_t &x : rg->x) {
        if (x) (void)hipGraphExecDestroy(x);
        x = nullptr;
    }
    rg->T = -1;
    hipError_t e = hipSuccess;
    if (!rg->cap && (e = hipStreamCreate(&rg->cap)) != hipSuccess) {
        (void)hipGetLastError();
        return e;
    }
    int launches = 0;
    for (int part = 0; part < 3 && e == hipSuccess; ++part) {
        if ((e = hipStreamBeginCapture(rg->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) break;
        const hipError_t le = part == 0 ? run_pre(p, fields, rg->cap)
                              : part == 1 ? run_sweeps(p, fields, a, iterations, rg->cap, &launches, p->d_part)
                                          : run_post(p, fields, launches, rg->cap);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(rg->cap, &g);
        if (le != hipSuccess) e = le;
        size_t n = 0;
        if (e == hipSuccess && g) e = hipGraphGetNodes(g, nullptr, &n);
        if (e == hipSuccess && n > 0) e = hipGraphInstantiate(&rg->x[part], g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
    }
    if (e != hipSuccess || !rg->x[1]) {
        for (hipGraphExec_t &x : rg->x) {
            if (x) (void)hipGraphExecDestroy(x);
            x = nullptr;
        }
        (void)hipGetLastError();
        return e != hipSuccess ? e : hipErrorUnknown;
    }
    return hipSuccess;
}

}  // namespace stn

extern "C" {

stencil_status stencil_plan(const stencil_desc *d, stencil_plan_t *out) {
    if (!out) return fail(STENCIL_E_INVAL, "out is NULL");
    *out = nullptr;
    Geom g{};
    int rz = 0;
    stencil_status st = validate_desc(d, g, rz);
    if (st != STENCIL_OK) return st;
    // device
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev < 1) return fail(STENCIL_E_DEVICE, "no HIP device available");
    stencil_plan_s *p = new (std::nothrow) stencil_plan_s();
    if (!p) return fail(STENCIL_E_NOMEM, "host allocation failed");
    init_plan_fields(p, d, g, rz);
    if ((e = hipGetDevice(&p->device)) != hipSuccess) {
        delete p;
        return hip_fail(e, "hipGetDevice");
    }
    if (p->kind == STENCIL_GENERIC && (st = build_generic_tables(p, d)) != STENCIL_OK) {
        free_plan(p);
        return st;
    }
    if ((st = choose_config(p, d)) != STENCIL_OK || (st = alloc_plan_buffers(p)) != STENCIL_OK) {
        free_plan(p);
        return st;
    }
    if (p->kind == STENCIL_GENERIC && p->variant == V_SATURATED && p->base_args.rtc &&
        !rtc_prepare(*p->rtc, {p->tile})) {
        logf("%s; using the table-driven generic kernel", stencil_last_error());
        p->base_args.rtc = nullptr;
    }
    logf("plan kind=%d variant=%d tile=(%d,%d,%d) map=%d tuned=%d n=(%d,%d,%d) blocks=%lld", p->kind, p->variant,
         p->tile.tx, p->tile.ty, p->tile.tz, p->remap ? 2 : 1, (int)p->tuned, g.nx, g.ny, g.nz, p->nblocks);
    *out = p;
    return STENCIL_OK;
}

stencil_status stencil_run(stencil_plan_t p, void *const *fields, const void *const *coef_arrays, int32_t iterations,
                           void *stream_) {
    if (!p) return fail(STENCIL_E_INVAL, "plan is NULL");
    if (!fields) return fail(STENCIL_E_INVAL, "fields is NULL");
    if (iterations < 0) return fail(STENCIL_E_INVAL, "iterations < 0");
    if (p->batch) {
        DeviceGuard guard(p->device);
        if (!guard.ok) return fail(STENCIL_E_DEVICE, "cannot make device %d current", p->device);
        return batch_run(p, fields, iterations, (hipStream_t)stream_);
    }
    SweepArgs a{};
    stencil_status st = prepare_run_args(p, fields, coef_arrays, a);
    if (st != STENCIL_OK) return st;
    if (iterations == 0) return STENCIL_OK;
    DeviceGuard guard(p->device);
    if (!guard.ok) return fail(STENCIL_E_DEVICE, "cannot make device %d current", p->device);
    hipStream_t s = (hipStream_t)stream_;
    hipError_t e;
    p->has_resid = false;
    std::vector<const void *> sig{fields[0], fields[1]};
    const int ncoef = p->kind == STENCIL_POISSON19 ? 12 : (p->kind == STENCIL_WAVE25 ? 1 : 0);
    for (int c = 0; c < ncoef; ++c) sig.push_back(coef_arrays[c]);
    RunGraphs *rg = (p->rg && p->rg->on && !p->rg->off) ? p->rg : nullptr;
    bool replay = false;
    if (rg) {
        if (rg->x[1] && rg->T == iterations && rg->sig == sig) {
            replay = true;
        } else if (rg->last_T == iterations && rg->last == sig) {
            if (capture_run(p, fields, a, iterations) == hipSuccess) {
                rg->T = iterations;
                rg->sig = sig;
                replay = true;
                logf("run graph captured: kind=%d T=%d", p->kind, iterations);
            } else {
                logf("run graph capture failed; running eagerly from now on");
                rg->off = true;
            }
        }
        rg->last_T = iterations;
        rg->last = sig;
    }
    if (replay) {
        if (rg->x[0] && (e = hipGraphLaunch(rg->x[0], s)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        if (p->profiling && (e = hipEventRecord(p->ev0, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        if ((e = hipGraphLaunch(rg->x[1], s)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
        if (p->profiling) {
            if ((e = hipEventRecord(p->ev1, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
            p->prof_sweeps = iterations;
            p->prof_valid = true;
        }
        if (rg->x[2] && (e = hipGraphLaunch(rg->x[2], s)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    } else {
        if ((e = run_pre(p, fields, s)) != hipSuccess) return hip_fail(e, "halo copy launch");
        if (p->profiling && (e = hipEventRecord(p->ev0, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        int launches = 0;
        if ((e = run_sweeps(p, fields, a, iterations, s, &launches, p->d_part)) != hipSuccess)
            return hip_fail(e, "sweep launch");
        if (p->profiling) {
            if ((e = hipEventRecord(p->ev1, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
            p->prof_sweeps = iterations;
            p->prof_valid = true;
        }
        if ((e = run_post(p, fields, launches, s)) != hipSuccess) return hip_fail(e, "tail copy launch");
    }
    p->has_resid = true;
    return STENCIL_OK;
}

// The sweeps of stencil_run, eagerly, with the residual partials in the
// library's device scratch and the reduced residual in the caller's memory.
// Nothing is allocated: no HIP allocation, no host heap (errors are written
// into a fixed thread-local buffer).
stencil_status stencil_run_noalloc(stencil_plan_t p, void *const *fields, const void *const *coef_arrays,
                                   int32_t iterations, double *residual_dev, void *stream_) {
    if (!p) return fail(STENCIL_E_INVAL, "plan is NULL");
    if (p->batch) return fail(STENCIL_E_UNSUPPORTED, "batched plans have no allocation-free run");
    if (p->kind == STENCIL_GENERIC && p->variant == V_SATURATED && p->base_args.rtc)
        return fail(STENCIL_E_UNSUPPORTED, "generated GENERIC kernels are looked up by their source text at launch; "
                                           "the allocation-free run takes the table-driven kernel only");
    if (p->nblocks > kNoallocPartials)
        return fail(STENCIL_E_UNSUPPORTED, "the plan's sweep launch has %lld blocks; the allocation-free run holds at most %lld",
                    p->nblocks, kNoallocPartials);
    if (!fields) return fail(STENCIL_E_INVAL, "fields is NULL");
    if (iterations < 0) return fail(STENCIL_E_INVAL, "iterations < 0");
    if ((uintptr_t)residual_dev % alignof(double)) return fail(STENCIL_E_INVAL, "residual_dev is not 8-byte aligned");
    SweepArgs a{};
    stencil_status st = prepare_run_args(p, fields, coef_arrays, a);
    if (st != STENCIL_OK) return st;
    if (iterations == 0) return STENCIL_OK;
    DeviceGuard guard(p->device);
    if (!guard.ok) return fail(STENCIL_E_DEVICE, "cannot make device %d current", p->device);
    hipStream_t s = (hipStream_t)stream_;
    hipError_t e;
    double *scr = nullptr;
    if ((e = noalloc_scratch(&scr)) != hipSuccess) return hip_fail(e, "device scratch address");
    if ((e = run_pre(p, fields, s)) != hipSuccess) return hip_fail(e, "halo copy launch");
    int launches = 0;
    if ((e = run_sweeps(p, fields, a, iterations, s, &launches, scr)) != hipSuccess) return hip_fail(e, "sweep launch");
    if ((e = run_post(p, fields, launches, s)) != hipSuccess) return hip_fail(e, "tail copy launch");
    if (residual_dev &&
        (e = launch_reduce_partials(scr, p->nblocks, scr + kNoallocPartials, residual_dev, s)) != hipSuccess)
        return hip_fail(e, "reduce launch");
    return STENCIL_OK;
}

stencil_status stencil_residual(stencil_plan_t p, double *host_out, void *stream_) {
    if (!p || !host_out) return fail(STENCIL_E_INVAL, "plan and host_out are required");
    if (!p->has_resid) return fail(STENCIL_E_STATE, "no sweep has run on this plan");
    DeviceGuard guard(p->device);
    if (!guard.ok) return fail(STENCIL_E_DEVICE, "cannot make device %d current", p->device);
    hipStream_t s = (hipStream_t)stream_;
    if (p->batch) return batch_residuals(p, host_out, 1, s);
    hipError_t e;
    if ((e = launch_reduce_partials(p->d_part, p->nblocks, p->d_red, p->h_result, s)) != hipSuccess)
        return hip_fail(e, "reduce launch");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    *host_out = *p->h_result;
    return STENCIL_OK;
}

stencil_status stencil_residuals(stencil_plan_t p, double *host_out, int32_t count, void *stream_) {
    if (!p || !host_out) return fail(STENCIL_E_INVAL, "plan and host_out are required");
    const int n = p->batch ? p->batch->count : 1;
    if (count != n) return fail(STENCIL_E_INVAL, "count %d != number of problems %d", count, n);
    if (!p->batch) return stencil_residual(p, host_out, stream_);
    if (!p->has_resid) return fail(STENCIL_E_STATE, "no sweep has run on this plan");
    DeviceGuard guard(p->device);
    if (!guard.ok) return fail(STENCIL_E_DEVICE, "cannot make device %d current", p->device);
    return batch_residuals(p, host_out, count, (hipStream_t)stream_);
}

stencil_status stencil_plan_config(stencil_plan_t p, int32_t *variant, int32_t *tile_x, int32_t *tile_y,
                                   int32_t *zblock, int32_t *tile_map) {
    if (!p) return fail(STENCIL_E_INVAL, "plan is NULL");
    if (variant) *variant = p->variant;
    if (tile_x) *tile_x = p->tile.tx;
    if (tile_y) *tile_y = p->tile.ty;
    if (zblock) *zblock = p->tile.tz;
    if (tile_map) *tile_map = p->remap ? 2 : 1;
    return STENCIL_OK;
}

stencil_status stencil_batch_problem_config(stencil_plan_t p, int32_t problem, int32_t *size_class, int32_t *variant,
                                            int32_t *tile_x, int32_t *tile_y, int32_t *zblock) {
    if (!p || !p->batch) return fail(STENCIL_E_INVAL, "not a batch plan");
    const BatchState *b = p->batch;
    if (problem < 0 || problem >= b->count) return fail(STENCIL_E_INVAL, "problem %d of %d", problem, b->count);
    const int c = b->prob_class[problem];
    const BatchClass &C = b->classes[c];
    if (size_class) *size_class = c;
    if (variant) *variant = C.variant;
    if (tile_x) *tile_x = C.tile.tx;
    if (tile_y) *tile_y = C.tile.ty;
    if (zblock) *zblock = C.tile.tz;
    return STENCIL_OK;
}

stencil_status stencil_plan_use_graphs(stencil_plan_t p, int32_t enable) {
    if (!p) return fail(STENCIL_E_INVAL, "plan is NULL");
    if (p->batch) return fail(STENCIL_E_UNSUPPORTED, "batched plans always run as graphs");
    // GENERIC launches generated kernels through the module API: always eager
    if (p->kind == STENCIL_GENERIC) return fail(STENCIL_E_UNSUPPORTED, "GENERIC plans run eagerly");
    if (!p->rg && !(p->rg = new (std::nothrow) RunGraphs())) return fail(STENCIL_E_NOMEM, "host allocation failed");
    p->rg->on = enable != 0;
    return STENCIL_OK;
}

stencil_status stencil_plan_graph(stencil_plan_t p, int32_t *iterations) {
    if (!p || !iterations) return fail(STENCIL_E_INVAL, "plan and iterations are required");
    *iterations = (p->rg && p->rg->x[1]) ? p->rg->T : 0;
    return STENCIL_OK;
}

stencil_status stencil_profile_enable(stencil_plan_t p, int32_t enable) {
    if (!p) return fail(STENCIL_E_INVAL, "plan is NULL");
    p->profiling = enable != 0;
    return STENCIL_OK;
}

stencil_status stencil_profile_read(stencil_plan_t p, double *sweep_ms, int32_t *sweeps) {
    if (!p || !sweep_ms) return fail(STENCIL_E_INVAL, "plan and sweep_ms are required");
    if (!p->prof_valid) return fail(STENCIL_E_STATE, "no profiled run on this plan");
    DeviceGuard guard(p->device);
    hipError_t e;
    if ((e = hipEventSynchronize(p->ev1)) != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float ms = 0.f;
    if ((e = hipEventElapsedTime(&ms, p->ev0, p->ev1)) != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    *sweep_ms = ms;
    if (sweeps) *sweeps = p->prof_sweeps;
    return STENCIL_OK;
}

stencil_status stencil_prepare(const stencil_desc *d) {
    if (!d) return fail(STENCIL_E_INVAL, "descriptor is NULL");
    Geom g{};
    int rz = 0;
    stencil_status st = validate_desc(d, g, rz);
    if (st != STENCIL_OK || d->kind != STENCIL_GENERIC) return st;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(STENCIL_E_DEVICE, "no HIP device available");
    stencil_plan_s tmp;
    tmp.kind = d->kind;
    tmp.dtype = d->dtype;
    tmp.g = g;
    tmp.rz = rz;
    tmp.base_args.g = g;
    tmp.base_args.elem_bytes = elem_bytes(d->dtype);
    if ((st = build_generic_tables(&tmp, d)) != STENCIL_OK) {
        if (tmp.d_tab) (void)hipFree(tmp.d_tab);
        delete tmp.rtc;
        return st;
    }
    TuneRequest rq{STENCIL_SATURATED, d->tile_x, d->tile_y, d->zblock, d->tile_map};
    std::vector<Tile> tiles;
    for (const Cand &c : tune_candidates(&generic_ops, STENCIL_GENERIC, g, rq)) tiles.push_back(c.tile);
    const bool ok = rtc_prepare(*tmp.rtc, tiles);
    (void)hipFree(tmp.d_tab);
    delete tmp.rtc;
    return ok ? STENCIL_OK : STENCIL_E_DEVICE;
}

stencil_status stencil_stream(int32_t op, const double *a, const double *b, const double *c, double *d, int64_t n,
                              int32_t width, int32_t flags, int32_t grid, void *stream) {
    if (op != 0 && op != 1) return fail(STENCIL_E_INVAL, "stream op %d not in {0, 1}", op);
    if (width != 1 && width != 2) return fail(STENCIL_E_INVAL, "stream width %d not in {1, 2}", width);
    if (flags < 0 || flags > 3) return fail(STENCIL_E_INVAL, "stream flags %d not in 0..3", flags);
    if (grid < 0) return fail(STENCIL_E_INVAL, "stream grid %d < 0", grid);
    if (n < 0) return fail(STENCIL_E_INVAL, "stream n < 0");
    if (!a || !d || (op == 1 && (!b || !c))) return fail(STENCIL_E_INVAL, "stream: a NULL array");
    const uintptr_t al = 8u * (uintptr_t)width;
    for (const void *q : {(const void *)a, (const void *)b, (const void *)c, (const void *)d})
        if (q && (uintptr_t)q % al) return fail(STENCIL_E_INVAL, "stream arrays must be %d-byte aligned", (int)al);
    // d is written: it must not overlap a read-only input (it may BE b, in place)
    const uintptr_t bytes = (uintptr_t)n * 8u;
    auto ov = [bytes](const void *x, const void *y) {
        return x && y && (uintptr_t)x < (uintptr_t)y + bytes && (uintptr_t)y < (uintptr_t)x + bytes;
    };
    if (ov(d, a) || (op == 1 && ov(d, c)) || (op == 1 && d != b && ov(d, b)))
        return fail(STENCIL_E_INVAL, "stream: d overlaps an input");
    if (n == 0) return STENCIL_OK;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(STENCIL_E_DEVICE, "no HIP device available");
    const hipError_t e = launch_stream(op, a, b, c, d, n, width, flags, grid, (hipStream_t)stream);
    return e == hipSuccess ? STENCIL_OK : hip_fail(e, "stream launch");
}

stencil_status stencil_destroy(stencil_plan_t p) {
    free_plan(p);
    return STENCIL_OK;
}

const char *stencil_last_error(void) { return g_err; }

const char *stencil_version(void) { return "0.1.0 gfx950"; }

}  // extern "C"
