// plan.hpp -- the opaque plan object behind stencil_plan_t.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/stencil.h"
#include "internal.hpp"
#include "tune.hpp"
#include "rtc.hpp"

#include <vector>

// Batched plan state (see batch.cpp).
struct BatchClass {
    int variant = 0;
    stn::Tile tile{};
    int n_items = 0, item_base = 0, grid = 0;
};
struct BatchState {
    int count = 0, n_items = 0;
    std::vector<stn::BatchProb> probs;  // host copy of the problem table
    std::vector<BatchClass> classes;
    std::vector<int> prob_class;        // index into classes, per problem
    stn::BatchItem *d_items = nullptr;  // class-major, then problem, then tile (x fastest)
    stn::BatchProb *d_probs = nullptr;
    int *d_seg = nullptr;               // per problem: item begin [count], item end [count]
    double *d_part = nullptr;           // residual partial per item
    double *d_res = nullptr;            // residual per problem
    double *h_res = nullptr;            // pinned copy
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_T = -1;
    std::vector<void *> graph_fields;
    hipStream_t cap = nullptr;          // capture stream
    std::vector<hipStream_t> side;      // one per class (graph branches)
    std::vector<hipEvent_t> evs;        // fork + one join per class
};

// Graphs of one run of a single plan: the halo copy, the sweeps and the odd-T
// copy (an empty part has no graph), captured when the same iteration count
// and pointers arrive twice in a row and replayed while they keep arriving.
struct RunGraphs {
    hipStream_t cap = nullptr;                          // capture stream
    hipGraphExec_t x[3] = {nullptr, nullptr, nullptr};  // pre, sweeps, post
    int T = -1;
    std::vector<const void *> sig;   // pointers of the captured run
    std::vector<const void *> last;  // pointers of the previous run
    int last_T = -1;
    bool on = false;                 // enabled by stencil_plan_use_graphs
    bool off = false;                // a capture failed: eager runs only
};

struct stencil_plan_s {
    int kind = 0, dtype = 0, bc = 0;
    int variant = 0;            // resolved form (stn::Variant)
    stn::Tile tile{};           // resolved launch shape
    stn::Geom g{};
    int rz = 0;                 // z halo width (0 for 2-D)
    double c[5] = {0, 0, 0, 0, 0};
    double omega = 0;
    const stn::KindOps *ops = nullptr;
    int device = -1;
    long long nblocks = 0;      // blocks of one sweep launch = residual partial count
    double *d_part = nullptr;   // device: per-block residual partials of the last sweep
    double *d_red = nullptr;    // device: first-pass sums of the residual reduction
    int remap = 1;              // XCD-chunked tile order for the saturated forms
    double *h_result = nullptr; // pinned coherent host word: the reduced residual
    bool has_resid = false;
    bool profiling = false, prof_valid = false;
    int prof_sweeps = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    stn::SweepArgs base_args{};  // geometry and scalars shared by every launch of this plan
    unsigned taps_hash = 0;      // GENERIC: hash of the tap pattern (part of the tune key)
    void *d_tab = nullptr;       // GENERIC: device tap tables
    stn::RtcSpec *rtc = nullptr; // GENERIC: spec of the generated saturated kernels
    bool tuned = false;          // configuration came from the autotuner
    BatchState *batch = nullptr; // non-null for plans made by stencil_plan_batch
    RunGraphs *rg = nullptr;     // single plans: captured runs
    stn::StencilInfo info{};     // static description (cost-model features)
};

// Host-side steps of abi.cpp shared by the entry points (all host only unless
// noted; the run_* functions enqueue on s).
namespace stn {
stencil_status fail(stencil_status st, const char *fmt, ...);
stencil_status hip_fail(hipError_t e, const char *what);
stencil_status validate_desc(const stencil_desc *d, Geom &g, int &rz);
void init_plan_fields(stencil_plan_s *p, const stencil_desc *d, const Geom &g, int rz);
stencil_status choose_config(stencil_plan_s *p, const stencil_desc *d);
stencil_status prepare_run_args(const stencil_plan_s *p, void *const *fields, const void *const *coef_arrays,
                                SweepArgs &a);
hipError_t run_pre(stencil_plan_s *p, void *const *fields, hipStream_t s);
hipError_t run_sweeps(stencil_plan_s *p, void *const *fields, SweepArgs a, int iterations, hipStream_t s,
                      int *launches, double *part);
hipError_t run_post(stencil_plan_s *p, void *const *fields, int launches, hipStream_t s);
}  // namespace stn
