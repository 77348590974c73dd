// program.cpp -- C ABI of the saturator (include/saturator.h): validation,
// generation, hipRTC compilation and launch of pointwise programs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "../../include/saturator.h"
#include "rtc.hpp"
#include "saturator.hpp"

namespace stn {
stencil_status fail(stencil_status st, const char *fmt, ...);
stencil_status hip_fail(hipError_t e, const char *what);
void logf(const char *fmt, ...);
}  // namespace stn

using namespace stn;

struct sat_plan_s {
    sat::Program prog;
    int form = 0, tx = 64, ty = 4, zb = 1, device = 0;
    hipFunction_t fn = nullptr;
    long long span = 0;  // elements of one padded array
    bool profiling = false, prof_valid = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace {

stencil_status read_desc(const sat_program_desc *d, sat::Program *p) {
    if (!d) return fail(STENCIL_E_INVAL, "program descriptor is NULL");
    if (d->struct_size != sizeof(sat_program_desc))
        return fail(STENCIL_E_INVAL, "struct_size %u does not match sizeof(sat_program_desc) = %zu", d->struct_size,
                    sizeof(sat_program_desc));
    if (d->n_insns < 1 || d->n_insns > 65536 || !d->insns) return fail(STENCIL_E_INVAL, "n_insns must be in [1, 65536]");
    if (d->n_consts < 0 || d->n_consts > 65536 || (d->n_consts > 0 && !d->consts))
        return fail(STENCIL_E_INVAL, "n_consts must be in [0, 65536] with a consts array");
    p->n_in = d->n_inputs;
    p->n_out = d->n_outputs;
    p->n_par = d->n_params;
    p->n_loc = d->n_locals;
    p->radius = d->radius;
    p->insns.resize(d->n_insns);
    for (int i = 0; i < d->n_insns; ++i)
        p->insns[i] = {d->insns[i].op, d->insns[i].a, d->insns[i].b, d->insns[i].c, d->insns[i].d};
    p->consts.assign(d->consts, d->consts + d->n_consts);
    for (int a = 0; a < 3; ++a) p->n[a] = d->n[a];
    p->py = d->pitch_y;
    p->pz = d->pitch_z;
    if (p->py < 0 || p->pz < 0) return fail(STENCIL_E_INVAL, "pitches must be >= 0");
    const std::string why = sat::validate(*p);
    if (!why.empty()) return fail(STENCIL_E_INVAL, "%s", why.c_str());
    return STENCIL_OK;
}

stencil_status check_shape(const sat::Program &p, int form, int *tx, int *ty, int *zb) {
    if (form < SAT_PLAIN || form > SAT_ACCSAT_Z) return fail(STENCIL_E_INVAL, "form %d is not a sat_form", form);
    if (*zb < 0) return fail(STENCIL_E_INVAL, "zblock must be >= 0");
    if (*zb == 0) *zb = form == SAT_ACCSAT_Z ? 32 : 1;
    if (*tx == 0 && *ty == 0) {
        *tx = 64;
        *ty = 4;
    }
    const long long nt = (long long)*tx * *ty;
    if (*tx < 1 || *ty < 1 || nt % 64 != 0 || nt > 1024)
        return fail(STENCIL_E_INVAL, "block %d x %d: threads must be a multiple of 64, at most 1024", *tx, *ty);
    if ((p.n[1] + *ty - 1) / *ty > 65535 || (p.n[2] + *zb - 1) / *zb > 65535)
        // generated kernels go through hipModuleLaunchKernel, which refuses y or
        // z grid dimensions above 65535 (the runtime launch path takes more)
        return fail(STENCIL_E_UNSUPPORTED, "grid too large for one launch (y blocks and z extent must be <= 65535)");
    return STENCIL_OK;
}

}  // namespace

extern "C" {

stencil_status sat_generate(const sat_program_desc *d, int32_t form, int32_t extract, int32_t tile_x, int32_t tile_y,
                            int32_t zblock, char *src, int64_t src_len, char *ssa, int64_t ssa_len, sat_stats *stats) {
    sat::Program p;
    stencil_status st = read_desc(d, &p);
    if (st != STENCIL_OK) return st;
    int tx = tile_x, ty = tile_y, zb = zblock;
    if ((st = check_shape(p, form, &tx, &ty, &zb)) != STENCIL_OK) return st;
    if (extract != SAT_EXTRACT_GREEDY && extract != SAT_EXTRACT_EXACT)
        return fail(STENCIL_E_INVAL, "extract must be SAT_EXTRACT_GREEDY or SAT_EXTRACT_EXACT");
    sat::Generated g;
    bool unsupported = false;
    const std::string err = sat::generate(p, form, extract, tx, ty, zb, sat::Limits{}, &g, &unsupported);
    if (!err.empty()) return fail(unsupported ? STENCIL_E_UNSUPPORTED : STENCIL_E_INVAL, "%s", err.c_str());
    if (src && (int64_t)g.src.size() + 1 > src_len)
        return fail(STENCIL_E_INVAL, "source buffer too small: %zu bytes needed", g.src.size() + 1);
    if (ssa && (int64_t)g.ssa.size() + 1 > ssa_len)
        return fail(STENCIL_E_INVAL, "ssa buffer too small: %zu bytes needed", g.ssa.size() + 1);
    if (src) std::memcpy(src, g.src.c_str(), g.src.size() + 1);
    if (ssa) std::memcpy(ssa, g.ssa.c_str(), g.ssa.size() + 1);
    if (stats) {
        stats->enodes = g.st.enodes;
        stats->eclasses = g.st.eclasses;
        stats->iterations = g.st.iterations;
        stats->saturated = g.st.saturated;
        stats->cost_input = g.st.cost_input;
        stats->cost_extracted = g.st.cost_extracted;
        stats->loads = g.st.loads;
        stats->ops = g.st.ops;
        stats->fmas = g.st.fmas;
        stats->saturate_ms = g.st.saturate_ms;
        stats->extract_ms = g.st.extract_ms;
    }
    return STENCIL_OK;
}

stencil_status sat_plan(const sat_program_desc *d, int32_t form, int32_t tile_x, int32_t tile_y, int32_t zblock,
                        sat_plan_t *out) {
    if (!out) return fail(STENCIL_E_INVAL, "out is NULL");
    *out = nullptr;
    sat::Program p;
    stencil_status st = read_desc(d, &p);
    if (st != STENCIL_OK) return st;
    int tx = tile_x, ty = tile_y, zb = zblock;
    if ((st = check_shape(p, form, &tx, &ty, &zb)) != STENCIL_OK) return st;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(STENCIL_E_DEVICE, "no HIP device");
    sat::Generated g;
    bool unsupported = false;
    const std::string err = sat::generate(p, form, SAT_EXTRACT_GREEDY, tx, ty, zb, sat::Limits{}, &g, &unsupported);
    if (!err.empty()) return fail(STENCIL_E_INVAL, "%s", err.c_str());
    logf("saturator form %d: %d e-nodes, %d e-classes, %d iterations, cost %.0f -> %.0f, %d loads %d ops", form,
         g.st.enodes, g.st.eclasses, g.st.iterations, g.st.cost_input, g.st.cost_extracted, g.st.loads, g.st.ops);
    hipFunction_t fn = rtc_function(g.src, sat::kernel_name(form));
    if (!fn) return STENCIL_E_DEVICE;  // error text set by rtc_function
    sat_plan_s *pl = new (std::nothrow) sat_plan_s;
    if (!pl) return fail(STENCIL_E_NOMEM, "plan allocation");
    pl->prog = std::move(p);
    pl->form = form;
    pl->tx = tx;
    pl->ty = ty;
    pl->zb = zb;
    pl->fn = fn;
    (void)hipGetDevice(&pl->device);
    const sat::Program &q = pl->prog;
    const long long PY = q.n[1] + 2 * q.radius, PZ = q.n[2] + 2 * q.radius, PX = q.n[0] + 2 * q.radius;
    pl->span = (PZ - 1) * q.pz + (PY - 1) * q.py + PX;
    hipError_t e;
    if ((e = hipEventCreate(&pl->ev0)) != hipSuccess || (e = hipEventCreate(&pl->ev1)) != hipSuccess) {
        sat_destroy(pl);
        return hip_fail(e, "hipEventCreate");
    }
    *out = pl;
    return STENCIL_OK;
}

stencil_status sat_run(sat_plan_t p, const void *const *inputs, void *const *outputs, const double *params,
                       void *stream) {
    if (!p) return fail(STENCIL_E_INVAL, "plan is NULL");
    const sat::Program &q = p->prog;
    if ((q.n_in > 0 && !inputs) || !outputs) return fail(STENCIL_E_INVAL, "inputs/outputs arrays are required");
    if (q.n_par > 0 && !params) return fail(STENCIL_E_INVAL, "params are required (n_params = %d)", q.n_par);
    const uintptr_t bytes = (uintptr_t)p->span * 8;
    std::vector<std::pair<uintptr_t, int>> iv;  // (start, is_output)
    for (int i = 0; i < q.n_in; ++i) {
        if (!inputs[i] || ((uintptr_t)inputs[i] & 7)) return fail(STENCIL_E_INVAL, "input %d is NULL or misaligned", i);
        iv.push_back({(uintptr_t)inputs[i], 0});
    }
    for (int i = 0; i < q.n_out; ++i) {
        if (!outputs[i] || ((uintptr_t)outputs[i] & 7))
            return fail(STENCIL_E_INVAL, "output %d is NULL or misaligned", i);
        iv.push_back({(uintptr_t)outputs[i], 1});
    }
    std::sort(iv.begin(), iv.end());
    for (size_t a = 0; a < iv.size(); ++a)
        for (size_t b = a + 1; b < iv.size() && iv[b].first < iv[a].first + bytes; ++b)
            if (iv[a].second || iv[b].second)
                return fail(STENCIL_E_INVAL, "an output array overlaps another array (padded span %lld elements)",
                            p->span);
    // kernel argument block: in[max(1,NI)] pointers, out[NO] pointers, prm[max(1,NP)] doubles
    const int NI = std::max(1, q.n_in), NP = std::max(1, q.n_par);
    std::vector<uint64_t> args((size_t)NI + q.n_out + NP, 0);
    for (int i = 0; i < q.n_in; ++i) args[i] = (uint64_t)(uintptr_t)inputs[i];
    for (int i = 0; i < q.n_out; ++i) args[NI + i] = (uint64_t)(uintptr_t)outputs[i];
    for (int i = 0; i < q.n_par; ++i) std::memcpy(&args[NI + q.n_out + i], &params[i], 8);
    size_t sz = args.size() * 8;
    void *extra[] = {HIP_LAUNCH_PARAM_BUFFER_POINTER, args.data(), HIP_LAUNCH_PARAM_BUFFER_SIZE, &sz,
                     HIP_LAUNCH_PARAM_END};
    int cur = 0;
    (void)hipGetDevice(&cur);
    if (cur != p->device) (void)hipSetDevice(p->device);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (p->profiling) e = hipEventRecord(p->ev0, s);
    if (e == hipSuccess)
        e = hipModuleLaunchKernel(p->fn, (unsigned)((q.n[0] + p->tx - 1) / p->tx), (unsigned)((q.n[1] + p->ty - 1) / p->ty),
                                  (unsigned)((q.n[2] + p->zb - 1) / p->zb), p->tx, p->ty, 1, 0, s, nullptr, extra);
    if (e == hipSuccess && p->profiling) e = hipEventRecord(p->ev1, s);
    if (cur != p->device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return hip_fail(e, "saturator kernel launch");
    if (p->profiling) p->prof_valid = true;
    return STENCIL_OK;
}

stencil_status sat_plan_info(sat_plan_t p, int32_t *regs, int32_t *private_bytes, int32_t *lds_bytes) {
    if (!p) return fail(STENCIL_E_INVAL, "plan is NULL");
    int v = 0;
    hipError_t e;
    if (regs) {
        if ((e = hipFuncGetAttribute(&v, HIP_FUNC_ATTRIBUTE_NUM_REGS, p->fn)) != hipSuccess)
            return hip_fail(e, "hipFuncGetAttribute");
        *regs = v;
    }
    if (private_bytes) {
        if ((e = hipFuncGetAttribute(&v, HIP_FUNC_ATTRIBUTE_LOCAL_SIZE_BYTES, p->fn)) != hipSuccess)
            return hip_fail(e, "hipFuncGetAttribute");
        *private_bytes = v;
    }
    if (lds_bytes) {
        if ((e = hipFuncGetAttribute(&v, HIP_FUNC_ATTRIBUTE_SHARED_SIZE_BYTES, p->fn)) != hipSuccess)
            return hip_fail(e, "hipFuncGetAttribute");
        *lds_bytes = v;
    }
    return STENCIL_OK;
}

stencil_status sat_profile_enable(sat_plan_t p, int32_t enable) {
    if (!p) return fail(STENCIL_E_INVAL, "plan is NULL");
    p->profiling = enable != 0;
    return STENCIL_OK;
}

stencil_status sat_profile_read(sat_plan_t p, double *run_ms, int32_t *runs) {
    if (!p || !run_ms) return fail(STENCIL_E_INVAL, "plan and run_ms are required");
    if (!p->prof_valid) return fail(STENCIL_E_STATE, "no profiled run on this plan");
    hipError_t e;
    if ((e = hipEventSynchronize(p->ev1)) != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float ms = 0.f;
    if ((e = hipEventElapsedTime(&ms, p->ev0, p->ev1)) != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    *run_ms = ms;
    if (runs) *runs = 1;
    return STENCIL_OK;
}

stencil_status sat_destroy(sat_plan_t p) {
    if (!p) return STENCIL_OK;
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    delete p;  // the compiled module stays in the process-wide cache
    return STENCIL_OK;
}

}  // extern "C"
