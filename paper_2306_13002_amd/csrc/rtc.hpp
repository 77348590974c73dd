// rtc.hpp -- generated saturated generic kernels (hipRTC), see rtc.cpp.
#pragma once

#include <string>
#include <utility>
#include <vector>

#include "internal.hpp"

namespace stn {

// One coefficient group of one z slot: coefficient and its taps (dx, dy),
// in ascending address order.
struct RtcGroup {
    double coef;
    std::vector<std::pair<int, int>> taps;
};

// What a generated kernel depends on besides its tile.
struct RtcSpec {
    int R = 1, eb = 8;
    bool corners = false;
    std::vector<std::vector<RtcGroup>> slots;  // 2R+1 slots, slot s holds dz = s - R
};

// Compile (or fetch from the in-process and STENCIL_RTC_CACHE caches) kernel
// `kernel` of `src` for the current device; nullptr (error text set) on failure.
hipFunction_t rtc_function(const std::string &src, const char *kernel);

std::string rtc_generic_source(const RtcSpec &sp, int TX, int TY);
// Compile the generated kernels of the given tiles (concurrently); false if any failed.
bool rtc_prepare(const RtcSpec &sp, const std::vector<Tile> &tiles);
hipError_t rtc_generic_launch(const RtcSpec &sp, Tile t, const SweepArgs &a, hipStream_t s);

}  // namespace stn
