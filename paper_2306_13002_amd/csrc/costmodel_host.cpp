// costmodel_host.cpp -- cost-model features, model file, MODEL tuning and
// the cost model's C ABI entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <dlfcn.h>
#include <string>
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
const KindOps *ops_for(int kind);
int elem_bytes(int dtype);
int mlp_param_count();
stencil_status mlp_predict_device(const float *model, const float *X, int n, float *y_out, hipStream_t s);
stencil_status mlp_train_device(const float *X, const float *t, int n, const float *init, int epochs, float lr,
                                float *model_out, float *loss_out, int use_graph, hipStream_t s);

StencilInfo stencil_info(const stencil_desc *d, const Geom &g) {
    StencilInfo si{};
    si.kind = d->kind;
    si.dtype = d->dtype;
    si.eb = elem_bytes(d->dtype);
    si.r = g.r;
    si.g = g;
    switch (d->kind) {
    case STENCIL_HEAT2D5: si.n_taps = 5; si.n_coef = 2; si.n_groups = 2; si.box_frac = 0; break;
    case STENCIL_HEAT3D7: si.n_taps = 7; si.n_coef = 2; si.n_groups = 2; si.box_frac = 0; break;
    case STENCIL_POISSON19: si.n_taps = 19; si.n_coef = 12; si.n_groups = 12; si.box_frac = 12.0 / 19; break;
    case STENCIL_WAVE25: si.n_taps = 25; si.n_coef = 5; si.n_groups = 5; si.box_frac = 0; break;
    default: {
        si.n_taps = d->n_taps;
        std::vector<char> used(d->n_coef, 0);
        std::vector<long long> grp;
        int multi = 0;
        for (int t = 0; t < d->n_taps; ++t) {
            const int *o = d->tap_off + 3 * t;
            used[d->tap_cid[t]] = 1;
            multi += ((o[0] != 0) + (o[1] != 0) + (o[2] != 0)) >= 2;
            grp.push_back((long long)(o[2] + 8) * 1000000 + d->tap_cid[t]);
        }
        std::sort(grp.begin(), grp.end());
        si.n_groups = (int)(std::unique(grp.begin(), grp.end()) - grp.begin());
        si.n_coef = (int)std::count(used.begin(), used.end(), 1);
        si.box_frac = (double)multi / d->n_taps;
    }
    }
    return si;
}

// Features of one (stencil, candidate):
//  0 XCD-chunked tile map   1 radius            2 fraction of off-axis taps
//  3 taps                   4 distinct coefs    5 bytes per element
//  6-8 log2 nx, ny, nz      9 log2 points      10 form: 0 plain, 1 saturated,
//                                                 2 saturated, two sweeps per pass,
//                                                 3 saturated, three sweeps per pass
// 11-13 log2 tile x, y, z  14 read-footprint ratio of a tile incl. halo
// 15 LDS bytes per block   16 estimated VGPRs  17 estimated waves per SIMD
// 18 algorithmic bytes per point and sweep (halved by two sweeps per pass,
//    a third of it by three)
// 19 flops/pt of the form (several sweeps per pass: with the recomputed rings)
// 20 arithmetic intensity
// 21 the paper's static cost of the form's per-point expression (Sec. Cost
//    Model: constants 0, inputs 1, operations 10, memory accesses 100)
// 22 working set / 256 MB  23 blocks / 256 CUs
// The target the model learns is log(seconds per sweep) in every form.
void cost_features(const StencilInfo &si, const Cand &c, float out[24]) {
    const int r = si.r, tx = c.tile.tx, ty = c.tile.ty, tz = c.tile.tz;
    const bool t2 = c.variant == V_SAT2, t3 = c.variant == V_SAT3;
    const bool sat = c.variant == V_SATURATED || t2 || t3;
    const double pts = (double)si.g.nx * si.g.ny * si.g.nz;
    double bytes_pt, flops, loads, ops, inputs, lds = 0, vgpr, blocks;
    switch (si.kind) {
    case STENCIL_HEAT2D5:
    case STENCIL_HEAT3D7: {
        const int nb = si.kind == STENCIL_HEAT2D5 ? 4 : 6;
        bytes_pt = 2.0 * si.eb;
        flops = sat ? nb + 2 : 2 * nb + 1;
        loads = nb + 1;
        ops = sat ? nb + 1 : 2 * nb + 1;
        inputs = 2;
        if (sat) lds = 2.0 * (ty + 2) * (tx + 2) * 8;
        vgpr = sat ? 48 : 28;
        break;
    }
    case STENCIL_POISSON19:
        bytes_pt = 56;
        flops = sat ? 30 : 34;
        loads = 19 + 12;
        ops = sat ? 21 : 32;
        inputs = 1;
        if (sat) lds = 4.0 * (ty + 2) * (tx + 2) * 4;
        vgpr = sat ? 72 : 48;
        break;
    case STENCIL_WAVE25:
        bytes_pt = 32;
        flops = sat ? 33 : 57;
        loads = 25 + 2;
        ops = sat ? 24 : 56;
        inputs = 5;
        if (sat) lds = 2.0 * (ty + 8) * (tx + 8) * 8;
        vgpr = sat ? 60 + 9.0 * 2 * (ty >= 16 ? 4 : ty >= 8 ? 2 : 1) : 62;
        break;
    default: {
        const double n = si.n_taps, G = si.n_groups;
        bytes_pt = 2.0 * si.eb;
        flops = sat ? n + G : 2 * n - 1;
        loads = n;
        ops = sat ? n : 2 * n - 1;
        inputs = si.n_coef;
        if (sat) lds = 2.0 * (ty + 2 * r) * (tx + 2 * r) * 8;
        vgpr = sat ? 40 + 4.0 * (2 * r + 1) : 32;
    }
    }
    // two sweeps per pass (POISSON19, HEAT3D7; radius 1): the state tile carries a
    // two-cell ring and the first sweep is recomputed on a one-cell ring, four
    // LDS planes of each; the bytes of one pass serve two sweeps
    double ring1 = 1.0;
    if (t2) {
        ring1 = (double)(tx + 2) * (ty + 2) / ((double)tx * ty);
        bytes_pt *= 0.5;
        flops *= 0.5 * (1.0 + ring1);
        const double eb = si.kind == STENCIL_POISSON19 ? 4 : 8;
        lds = 4.0 * eb * ((ty + 4.0) * (tx + 5.0) + (ty + 2.0) * (tx + 3.0));
        vgpr = si.kind == STENCIL_POISSON19 ? 158 : 56;
    }
    // three sweeps per pass (HEAT3D7): one thread per column of a region two
    // cells wider than the tile on every side; sweeps 1 and 2 recomputed on
    // rings of two and one cells; three-plane rings of the state (region and a
    // one-cell halo) and of the two intermediate sweeps (the region)
    if (t3) {
        const double rx = tx + 4.0, ry = ty + 4.0;
        ring1 = rx * ry / ((double)tx * ty);
        bytes_pt /= 3.0;
        flops *= (rx * ry + (tx + 2.0) * (ty + 2.0) + (double)tx * ty) / (3.0 * tx * ty);
        lds = 3.0 * 8 * ((ry + 2) * (rx + 3) + 2 * ry * (rx + 1));
        vgpr = 56;
    }
    blocks = std::ceil((double)si.g.nx / tx) * std::ceil((double)si.g.ny / ty) * std::ceil((double)si.g.nz / tz);
    const double threads = (double)tx * ty * (sat ? ((t2 || t3) ? ring1 : 1.0) : tz);
    const double wpb = std::ceil(threads / 64);
    double waves = std::min(8.0, std::floor(512.0 / vgpr));
    if (lds > 0) waves = std::min(waves, std::floor(160.0 * 1024 / lds) * wpb / 4);
    const int rf = t3 ? 3 * r : (t2 ? 2 * r : r);
    const double foot = sat ? (double)(tx + 2 * rf) * (ty + 2 * rf) / ((double)tx * ty)
                            : (double)(tx + 2 * r) * (ty + 2 * r) * (tz + 2 * r) / ((double)tx * ty * tz);
    const double ws = (si.kind == STENCIL_POISSON19 ? 14.0 * 4 : (si.kind == STENCIL_WAVE25 ? 3.0 * 8 : 2.0 * si.eb)) *
                      (si.g.nx + 2.0 * r) * (si.g.ny + 2.0 * r) * (si.g.nz + 2.0 * r);
    const double cost = 100.0 * (loads + 1) + 10.0 * ops + 1.0 * inputs;
    const double f[24] = {(double)(sat && c.remap), (double)r, si.box_frac, (double)si.n_taps, (double)si.n_coef,
                          (double)si.eb, std::log2((double)si.g.nx), std::log2((double)si.g.ny),
                          std::log2((double)si.g.nz), std::log2(pts), t3 ? 3.0 : (t2 ? 2.0 : (double)sat), std::log2((double)tx),
                          std::log2((double)ty), std::log2((double)tz), foot, lds, vgpr, waves, bytes_pt, flops,
                          flops / bytes_pt, cost, ws / (256.0 * 1024 * 1024), blocks / 256.0};
    for (int i = 0; i < 24; ++i) out[i] = (float)f[i];
}

namespace {

// Model file: JSON with "mean" (24), "std" (24) and "params" (5825) arrays.
bool parse_array(const std::string &txt, const char *key, std::vector<float> &out) {
    const std::string k = std::string("\"") + key + "\"";
    size_t p = txt.find(k);
    if (p == std::string::npos) return false;
    p = txt.find('[', p);
    const size_t e = txt.find(']', p);
    if (p == std::string::npos || e == std::string::npos) return false;
    const char *s = txt.c_str() + p + 1, *end = txt.c_str() + e;
    out.clear();
    while (s < end) {
        char *nx = nullptr;
        const double v = std::strtod(s, &nx);
        if (nx == s) {
            ++s;
            continue;
        }
        out.push_back((float)v);
        s = nx;
    }
    return true;
}

std::string model_path() {
    if (const char *e = std::getenv("STENCIL_COST_MODEL")) return e;
    Dl_info info;
    if (dladdr((void *)&model_path, &info) && info.dli_fname) {
        std::string so = info.dli_fname;
        const size_t slash = so.rfind('/');
        return (slash == std::string::npos ? std::string(".") : so.substr(0, slash)) + "/cost_model.json";
    }
    return "cost_model.json";
}

bool load_model(std::vector<float> &model) {
    const std::string path = model_path();
    FILE *f = std::fopen(path.c_str(), "rb");
    if (!f) return false;
    std::string txt;
    char buf[65536];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, n);
    std::fclose(f);
    std::vector<float> mean, sd, params;
    if (!parse_array(txt, "mean", mean) || !parse_array(txt, "std", sd) || !parse_array(txt, "params", params) ||
        mean.size() != 24 || sd.size() != 24 || (int)params.size() != mlp_param_count())
        return false;
    model = mean;
    model.insert(model.end(), sd.begin(), sd.end());
    model.insert(model.end(), params.begin(), params.end());
    return true;
}

}  // namespace

// The cost model's candidates: the exhaustive tuner's, the two- and
// three-sweep forms included (feature 10 tells them apart, and the training
// campaign times them).
std::vector<Cand> model_candidates(const KindOps *ops, int kind, const Geom &g, const TuneRequest &rq) {
    // HEAT2D5's fused plain sweeps (tile.tz > 1) lie outside what the model was
    // trained on; exhaustive tuning weighs them
    std::vector<Cand> c = tune_candidates(ops, kind, g, rq);
    c.erase(std::remove_if(c.begin(), c.end(),
                           [kind](const Cand &x) { return kind == STENCIL_HEAT2D5 && x.tile.tz > 1; }),
            c.end());
    return c;
}

stencil_status tune_model(stencil_plan_s *p, const TuneRequest &rq, TuneEntry *best) {
    std::vector<float> model;
    if (!load_model(model)) return fail(STENCIL_E_STATE, "no usable cost model at %s", model_path().c_str());
    const std::vector<Cand> cands = model_candidates(p->ops, p->kind, p->g, rq);
    if (cands.empty()) return fail(STENCIL_E_UNSUPPORTED, "no launch shape matches the requested tile fields");
    std::vector<float> X(cands.size() * 24), y(cands.size());
    for (size_t i = 0; i < cands.size(); ++i) cost_features(p->info, cands[i], &X[i * 24]);
    hipStream_t s = nullptr;
    hipError_t e;
    if ((e = hipStreamCreate(&s)) != hipSuccess) return hip_fail(e, "hipStreamCreate");
    stencil_status st = mlp_predict_device(model.data(), X.data(), (int)cands.size(), y.data(), s);
    (void)hipStreamDestroy(s);
    if (st != STENCIL_OK) return st;
    const size_t k = std::min_element(y.begin(), y.end()) - y.begin();
    best->variant = cands[k].variant;
    best->tile = cands[k].tile;
    best->remap = cands[k].remap;
    best->us = std::exp((double)y[k]) * 1e6;
    logf("model pick kind=%d v=%d tile=(%d,%d,%d) map=%d predicted %.2f us/sweep of %zu candidates", p->kind,
         best->variant, best->tile.tx, best->tile.ty, best->tile.tz, best->remap ? 2 : 1, best->us, cands.size());
    return STENCIL_OK;
}

}  // namespace stn

using namespace stn;

extern "C" {

stencil_status stencil_candidates(const stencil_desc *d, int32_t max, int32_t *out, int32_t *n) {
    if (!d || !n || (max > 0 && !out)) return fail(STENCIL_E_INVAL, "descriptor, n and out are required");
    Geom g{};
    int rz = 0;
    stencil_status st = validate_desc(d, g, rz);
    if (st != STENCIL_OK) return st;
    TuneRequest rq{d->variant, d->tile_x, d->tile_y, d->zblock, d->tile_map, d->bc};
    const std::vector<Cand> c = model_candidates(ops_for(d->kind), d->kind, g, rq);
    *n = (int32_t)c.size();
    for (int i = 0; i < (int)c.size() && i < max; ++i) {
        int32_t *o = out + 5 * i;
        o[0] = c[i].variant;
        o[1] = c[i].tile.tx;
        o[2] = c[i].tile.ty;
        o[3] = c[i].tile.tz;
        o[4] = c[i].remap ? 2 : 1;
    }
    return STENCIL_OK;
}

stencil_status stencil_features(const stencil_desc *d, int32_t variant, int32_t tile_x, int32_t tile_y,
                                int32_t zblock, int32_t tile_map, float *out) {
    if (!d || !out) return fail(STENCIL_E_INVAL, "descriptor and out are required");
    Geom g{};
    int rz = 0;
    stencil_status st = validate_desc(d, g, rz);
    if (st != STENCIL_OK) return st;
    if ((variant != V_PLAIN && variant != V_SATURATED && variant != V_SAT2 && variant != V_SAT3) || tile_x < 1 ||
        tile_y < 1 || zblock < 1 ||
        (tile_map != 1 && tile_map != 2))
        return fail(STENCIL_E_INVAL, "bad candidate");
    cost_features(stencil_info(d, g), Cand{variant, Tile{tile_x, tile_y, zblock}, tile_map == 2}, out);
    return STENCIL_OK;
}

stencil_status stencil_mlp_train(const float *X, const float *y, int32_t n, const float *init, int32_t epochs,
                                 float lr, float *model_out, float *loss_out, void *stream) {
    if (!X || !y || !init || !model_out || n < 1 || epochs < 0 || !(lr > 0))
        return fail(STENCIL_E_INVAL, "X, y, init, model_out, n >= 1, epochs >= 0 and lr > 0 are required");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(STENCIL_E_DEVICE, "no HIP device available");
    const char *eg = std::getenv("STENCIL_MLP_GRAPH");
    const int use_graph = eg ? std::atoi(eg) != 0 : 1;
    return mlp_train_device(X, y, n, init, epochs, lr, model_out, loss_out, use_graph, (hipStream_t)stream);
}

stencil_status stencil_mlp_predict(const float *model, const float *X, int32_t n, float *y_out, void *stream) {
    if (!model || !X || !y_out || n < 1) return fail(STENCIL_E_INVAL, "model, X, y_out and n >= 1 are required");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(STENCIL_E_DEVICE, "no HIP device available");
    return mlp_predict_device(model, X, n, y_out, (hipStream_t)stream);
}

}  // extern "C"
