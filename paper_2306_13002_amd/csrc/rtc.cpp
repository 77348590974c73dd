// rtc.cpp -- saturated generic stencils generated for one stencil and
// compiled at plan time with hipRTC.
//
// This is the paper's code-generation step (Sec. Code Generation) done at
// run time for the taps a plan was given: the saturated expression -- taps
// grouped by coefficient id and z offset, each group summed as a balanced
// tree in ascending address order, one FMA per group -- is emitted as
// straight-line HIP with compile-time LDS offsets and exact coefficient
// literals, wrapped around the streaming body every generic kernel shares
// (generic_body.hpp), and compiled for the device.  Modules are cached per
// source text in-process and, when STENCIL_RTC_CACHE names a directory, as
// code-object files there.  rtc_function serves every generated kernel of
// the library (also the saturator's programs).
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/stencil.h"
#include "internal.hpp"
#include "rtc.hpp"
#include "rtc_headers.inc"  // kCommonHppText, kGenericBodyHppText (written by the build)

namespace stn {

stencil_status fail(stencil_status st, const char *fmt, ...);
void logf(const char *fmt, ...);

namespace {

std::mutex g_mu;
std::map<std::string, hipFunction_t> g_fn;  // hash of source and kernel name + device -> kernel

unsigned long long fnv64(const std::string &s) {
    unsigned long long h = 1469598103934665603ull;
    for (unsigned char c : s) h = (h ^ c) * 1099511628211ull;
    return h;
}

// Balanced-tree sum of LDS terms, in the given (ascending address) order.
std::string tree(const std::vector<std::string> &terms, size_t a, size_t b) {
    if (b - a == 1) return terms[a];
    const size_t m = a + (b - a + 1) / 2;
    return "(" + tree(terms, a, m) + " + " + tree(terms, m, b) + ")";
}

}  // namespace

std::string rtc_generic_source(const RtcSpec &sp, int TX, int TY) {
    const int R = sp.R, W = TX + 2 * R;
    std::string o;
    char buf[256];
    o += "#include \"generic_body.hpp\"\n\nnamespace {\nstruct GenSlots {\n";
    o += "    __device__ __forceinline__ void operator()(const double *__restrict__ t, int me, double *acc) const {\n";
    o += "        double a;\n";
    for (int s = 0; s < 2 * R + 1; ++s) {
        if (sp.slots[s].empty()) continue;
        std::snprintf(buf, sizeof buf, "        a = acc[%d];\n", s);
        o += buf;
        for (const RtcGroup &gr : sp.slots[s]) {
            std::vector<std::string> terms;
            for (const auto &xy : gr.taps) {
                std::snprintf(buf, sizeof buf, "t[me + %d]", xy.second * W + xy.first);
                terms.push_back(buf);
            }
            std::snprintf(buf, sizeof buf, "%a", gr.coef);
            o += "        a = fma(" + std::string(buf) + ", " + tree(terms, 0, terms.size()) + ", a);\n";
        }
        std::snprintf(buf, sizeof buf, "        acc[%d] = a;\n", s);
        o += buf;
    }
    o += "    }\n};\n}  // namespace\n\n";
    const char *T = sp.eb == 4 ? "float" : "double";
    std::snprintf(buf, sizeof buf,
                  "extern \"C\" __global__ __launch_bounds__(%d) void stencil_generic_gen(const %s *__restrict__ src, "
                  "%s *__restrict__ dst, stn::Geom g, int zb, int remap, double *__restrict__ part) {\n",
                  TX * TY, T, T);
    o += buf;
    std::snprintf(buf, sizeof buf, "    __shared__ double tile[2][%d];\n    __shared__ double red[16];\n",
                  (TY + 2 * R) * W);
    o += buf;
    o += "    int bx, by, bz;\n    stn::tile_coords(remap, bx, by, bz);\n";
    std::snprintf(buf, sizeof buf,
                  "    const double sacc = stn::generic_sat_body<%s, %d, %d, %d, %s>(src, dst, g, zb, bx, by, bz, "
                  "GenSlots{}, tile);\n",
                  T, R, TX, TY, sp.corners ? "true" : "false");
    o += buf;
    o += "    if (part) {\n        const double s = stn::block_sum_f64(sacc, red);\n";
    o += "        if (threadIdx.x == 0 && threadIdx.y == 0) part[stn::block_linear_id()] = s;\n    }\n}\n";
    return o;
}

// Compile (or fetch from the caches) kernel `kernel` of source `src`;
// returns nullptr and sets the error text on failure.
hipFunction_t rtc_function(const std::string &src, const char *kernel) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    char key[96];
    std::snprintf(key, sizeof key, "%016llx-%d", fnv64(src + '\n' + kernel), dev);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_fn.find(key);
        if (it != g_fn.end()) return it->second;
    }
    std::vector<char> code;
    const char *cache = std::getenv("STENCIL_RTC_CACHE");
    std::string path;
    if (cache && *cache) {
        path = std::string(cache) + "/" + key + ".co";
        if (FILE *f = std::fopen(path.c_str(), "rb")) {
            std::fseek(f, 0, SEEK_END);
            const long n = std::ftell(f);
            std::fseek(f, 0, SEEK_SET);
            code.resize(n > 0 ? n : 0);
            if (n <= 0 || std::fread(code.data(), 1, n, f) != (size_t)n) code.clear();
            std::fclose(f);
        }
    }
    if (code.empty()) {
        hiprtcProgram prog;
        const char *hdrs[] = {kCommonHppText, kGenericBodyHppText};
        const char *names[] = {"common.hpp", "generic_body.hpp"};
        if (hiprtcCreateProgram(&prog, src.c_str(), "generated.hip", 2, hdrs, names) != HIPRTC_SUCCESS) {
            fail(STENCIL_E_DEVICE, "hiprtcCreateProgram failed");
            return nullptr;
        }
        const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
                              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
        const hiprtcResult r = hiprtcCompileProgram(prog, 8, opts);
        if (r != HIPRTC_SUCCESS) {
            size_t ln = 0;
            hiprtcGetProgramLogSize(prog, &ln);
            std::string log(ln + 1, '\0');
            hiprtcGetProgramLog(prog, &log[0]);
            fail(STENCIL_E_DEVICE, "hipRTC compile of generated kernel %s failed: %.400s", kernel, log.c_str());
            hiprtcDestroyProgram(&prog);
            return nullptr;
        }
        size_t n = 0;
        hiprtcGetCodeSize(prog, &n);
        code.resize(n);
        hiprtcGetCode(prog, code.data());
        hiprtcDestroyProgram(&prog);
        if (!path.empty())
            if (FILE *f = std::fopen(path.c_str(), "wb")) {
                std::fwrite(code.data(), 1, code.size(), f);
                std::fclose(f);
            }
    }
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
    hipError_t e = hipModuleLoadData(&mod, code.data());
    if (e == hipSuccess) e = hipModuleGetFunction(&fn, mod, kernel);
    if (e != hipSuccess) {
        fail(STENCIL_E_DEVICE, "loading generated kernel %s: %s", kernel, hipGetErrorString(e));
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_fn.find(key);
    if (it != g_fn.end()) return it->second;  // another thread won; its module stays loaded too
    g_fn[key] = fn;
    return fn;
}

static hipFunction_t get_kernel(const RtcSpec &sp, int TX, int TY) {
    return rtc_function(rtc_generic_source(sp, TX, TY), "stencil_generic_gen");
}

bool rtc_prepare(const RtcSpec &sp, const std::vector<Tile> &tiles) {
    // compile the distinct tiles concurrently
    std::vector<Tile> uniq;
    for (const Tile &t : tiles) {
        bool seen = false;
        for (const Tile &u : uniq) seen |= (u.tx == t.tx && u.ty == t.ty);
        if (!seen) uniq.push_back(t);
    }
    std::vector<char> ok(uniq.size(), 0);
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::vector<std::thread> th;
    for (size_t i = 0; i < uniq.size(); ++i)
        th.emplace_back([&, i] {
            (void)hipSetDevice(dev);
            ok[i] = get_kernel(sp, uniq[i].tx, uniq[i].ty) != nullptr;
        });
    for (auto &t : th) t.join();
    return std::all_of(ok.begin(), ok.end(), [](char c) { return c != 0; });
}

hipError_t rtc_generic_launch(const RtcSpec &sp, Tile t, const SweepArgs &a, hipStream_t s) {
    hipFunction_t fn = get_kernel(sp, t.tx, t.ty);
    if (!fn) return hipErrorInvalidImage;
    const void *src = a.src;
    void *dst = a.dst;
    Geom g = a.g;
    int zb = t.tz, remap = a.remap;
    double *part = a.part;
    void *args[] = {&src, &dst, &g, &zb, &remap, &part};
    return hipModuleLaunchKernel(fn, (unsigned)cdiv(a.g.nx, t.tx), (unsigned)cdiv(a.g.ny, t.ty),
                                 (unsigned)cdiv(a.g.nz, t.tz), t.tx, t.ty, 1, 0, s, args, nullptr);
}

}  // namespace stn
