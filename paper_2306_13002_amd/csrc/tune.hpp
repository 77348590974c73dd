// tune.hpp -- autotuner interface (exhaustive search and its cache).
#pragma once

#include <string>
#include <vector>

#include "../../include/stencil.h"

#include "internal.hpp"

struct stencil_plan_s;

namespace stn {

// What the descriptor leaves open: variant STENCIL_AUTO and 0-valued fields
// are searched; other values restrict the candidates.
struct TuneRequest {
    int variant, tile_x, tile_y, zblock, tile_map;
    int bc = STENCIL_BC_DIRICHLET;  // fused HEAT2D5 sweeps are offered for Dirichlet plans only
};

// Sweeps one launch of (kind, variant, tile) performs: the two-sweep form
// does two; HEAT2D5 PLAIN with tile.tz > 1 fuses tile.tz sweeps per launch.
inline int launch_sweeps(int kind, int variant, const Tile &t) {
    if (kind == STENCIL_HEAT2D5 && variant == V_PLAIN && t.tz > 1) return t.tz;
    return sweeps_per_launch(variant);
}

struct TuneEntry {
    int variant;  // V_PLAIN, V_SATURATED, V_SAT2 or V_SAT3
    Tile tile;
    int remap;    // 0 natural, 1 XCD-chunked
    double us;    // median time per sweep of the winner
};

// One launch candidate: form, shape and tile map (remap 1 = XCD-chunked).
struct Cand {
    int variant;
    Tile tile;
    int remap;
};

// Static description of a stencil used by the cost model's features.
struct StencilInfo {
    int kind, dtype, eb, r;
    Geom g;
    int n_taps;        // points read per update from the state grid
    int n_coef;        // distinct coefficients (coefficient arrays for POISSON19)
    int n_groups;      // saturated tap groups (GENERIC), else distinct coefficients
    double box_frac;   // fraction of taps with two or more nonzero offsets
};

StencilInfo stencil_info(const stencil_desc *d, const Geom &g);
// Candidates the tuners consider for a plan's kind and geometry, restricted
// by the request's fixed fields.
std::vector<Cand> tune_candidates(const KindOps *ops, int kind, const Geom &g, const TuneRequest &rq);
void cost_features(const StencilInfo &si, const Cand &c, float out[24]);
stencil_status tune_model(stencil_plan_s *p, const TuneRequest &rq, TuneEntry *best);

std::string tune_key(const stencil_plan_s *p, const TuneRequest &rq);
bool tune_lookup(const std::string &key, TuneEntry *out);
void tune_store(const std::string &key, const TuneEntry &e);
stencil_status tune_exhaustive(stencil_plan_s *p, const TuneRequest &rq, TuneEntry *best);

}  // namespace stn
