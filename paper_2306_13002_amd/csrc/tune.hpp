// tune.hpp -- autotuner interface (exhaustive search and its cache).
#pragma once

#include <string>

#include "internal.hpp"

struct stencil_plan_s;

namespace stn {

// What the descriptor leaves open: variant STENCIL_AUTO and 0-valued fields
// are searched; other values restrict the candidates.
struct TuneRequest {
    int variant, tile_x, tile_y, zblock, tile_map;
};

struct TuneEntry {
    int variant;  // V_PLAIN / V_SATURATED
    Tile tile;
    int remap;    // 0 natural, 1 XCD-chunked
    double us;    // median time per sweep of the winner
};

std::string tune_key(const stencil_plan_s *p, const TuneRequest &rq);
bool tune_lookup(const std::string &key, TuneEntry *out);
void tune_store(const std::string &key, const TuneEntry &e);
stencil_status tune_exhaustive(stencil_plan_s *p, const TuneRequest &rq, TuneEntry *best);

}  // namespace stn
