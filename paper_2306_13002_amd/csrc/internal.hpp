// internal.hpp -- host-side interface between the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace stn {

// Forms.  V_CSE_SAT, V_CSE_BULK and V_ACCSAT_POINT are the per-point forms of
// the paper's ablation (rewritten arithmetic only, bulk load only, both);
// V_SAT2 is the saturated form with two sweeps per pass (POISSON19, HEAT3D7),
// V_SAT3 with three (HEAT3D7).
enum Variant { V_PLAIN = 0, V_SATURATED = 1, V_CSE_SAT = 3, V_CSE_BULK = 4, V_ACCSAT_POINT = 5, V_SAT2 = 6, V_SAT3 = 7 };
inline bool is_point_form(int v) { return v == V_CSE_SAT || v == V_CSE_BULK || v == V_ACCSAT_POINT; }
// Sweeps one full launch performs (a V_SAT3 launch may be asked for fewer).
inline int sweeps_per_launch(int v) { return v == V_SAT2 ? 2 : (v == V_SAT3 ? 3 : 1); }

// Launch shape.  Plain forms: block = (tx, ty, tz) threads, one per point.
// Saturated forms: tx threads along x, a tile of ty rows, zblock planes
// streamed per block.
struct Tile {
    int tx, ty, tz;
};

struct RtcSpec;  // generated saturated generic kernels (rtc.hpp)

// GENERIC tap tables (device pointers, uniform over a launch).
struct GenTab {
    const long long *off;  // plain: linear offset dz*pz + dy*py + dx per tap, caller's order
    const double *c;    // plain: coefficient per tap
    int n;              // number of taps
    const int *slot_g;  // saturated: groups of z-offset slot s (dz = s - r) are [slot_g[s], slot_g[s+1])
    const int *g_t;     // saturated: taps of group g are [g_t[g], g_t[g+1])
    const double *g_c;  // saturated: coefficient of group g
    const int *t_xy;    // saturated: (dy << 16) | (dx & 0xffff) per tap, ascending address in a group
    bool corners;       // some tap has two nonzero in-plane offsets (the staged ring needs its corners)
};

// Arguments of one sweep launch.
struct SweepArgs {
    const void *src;          // Jacobi kinds: state read; WAVE25: u^n
    void *dst;                // Jacobi kinds: state written; WAVE25: u^{n-1} in, u^{n+1} out
    const void *coefs[12];    // POISSON19: a0 a1 a2 a3 b0 b1 b2 c0 c1 c2 bnd wrk1; WAVE25: vsq
    Geom g;
    double c[5];              // scalar coefficients (heat: cc, cn; wave: c0..c4)
    double omega;             // POISSON19
    double *part;             // residual partial per block, or nullptr
    const int *taps;          // GENERIC: device tap table
    const double *tap_coef;   // GENERIC: device coefficient table
    int n_taps, n_coef;
    int remap;                // saturated forms: XCD-chunked block -> tile map (1) or natural order (0)
    GenTab gen;               // GENERIC tap tables
    int elem_bytes;           // storage size (GENERIC: 4 or 8)
    const RtcSpec *rtc;       // GENERIC saturated: generated kernels (nullptr: table-driven kernel)
    int sweeps = 1;           // HEAT2D5 PLAIN with fused sweeps (tile.tz > 1): sweeps this launch performs
};

// Batched runs: one problem of a batch and one work item (a tile of a
// problem in its class's launch shape).
struct BatchProb {
    double *f[2];  // the problem's fields[0], fields[1]
    Geom g;
    double cc, cn;
};
struct BatchItem {
    int prob, bx, by, bz;
    int slot;  // index of its residual partial within the class (problem-major, then z, y, x)
};

struct KindOps {
    bool (*tile_ok)(int variant, Tile t);
    int (*sat_tiles)(Tile *out, int max);  // offered saturated (tx, ty) shapes; nullptr if none
    int (*sat2_tiles)(Tile *out, int max);  // shapes of the two-sweep saturated form; nullptr if none
    long long (*nblocks)(int variant, Tile t, const Geom &g);
    hipError_t (*launch)(int variant, Tile t, const SweepArgs &a, hipStream_t s);
    // Persistent work-list sweep over a batch (nullptr: kind not batchable).
    // Items [0, n_items) are visited by `grid` blocks in a fixed stride; the
    // residual partial of item i goes to part[i] when part is non-null.
    // sweeps: the sweeps this launch performs (V_SAT3: 1..3; others: their own).
    hipError_t (*batch_launch)(int variant, Tile t, const BatchProb *probs, const BatchItem *items, int n_items,
                               int parity, int grid, int sweeps, double *part, hipStream_t s);
    int (*sat3_tiles)(Tile *out, int max);  // output tiles of the three-sweep form; nullptr if none
};

extern KindOps heat2d5_ops, heat3d7_ops, poisson19_ops, wave25_ops, generic_ops;

// Support kernels (support.hip).
hipError_t launch_halo_copy(const void *src, void *dst, int elem_bytes, const Geom &g, int rz, hipStream_t s);
hipError_t launch_periodic_fill(void *buf, int elem_bytes, const Geom &g, int rz, hipStream_t s);
hipError_t launch_fill(void *buf, long long n, int elem_bytes, double value, hipStream_t s);
hipError_t launch_interior_copy(const void *src, void *dst, int elem_bytes, const Geom &g, int rz, hipStream_t s);
// Two fixed-order passes: up to kReduceBlocks blocks each sum a contiguous
// chunk of part[] into scratch[], then one block sums scratch[].
constexpr int kReduceBlocks = 256;
hipError_t launch_reduce_partials(const double *part, long long n, double *scratch, double *out, hipStream_t s);
// Allocation-free run: a file-scope device array of kNoallocPartials residual
// partials followed by kReduceBlocks first-pass sums.  noalloc_scratch gives
// its address on the current device (looked up once per device, then cached).
constexpr long long kNoallocPartials = 1LL << 17;
hipError_t noalloc_scratch(double **out);
// out[p] = sum of part[seg[p] .. seg[count+p]) in a fixed order, p < count.
hipError_t launch_segment_sums(const double *part, const int *seg, int count, double *out, hipStream_t s);

// Streaming kernels of known traffic (stream.hip): op 0 copies a to d, op 1
// writes d = fma(c, a, 2a - b) (three reads, one write; d may equal b).
hipError_t launch_stream(int op, const double *a, const double *b, const double *c, double *d, long long n,
                         int width, int flags, int grid, hipStream_t s);

inline long long cdiv(long long a, long long b) { return (a + b - 1) / b; }

// Largest plane (pitch_z * element size, bytes) that a kernel addressing a
// plane with 32-bit byte offsets through a buffer resource accepts.
constexpr long long kMaxPlaneBytes32 = 0xFFFFFFF0LL;

}  // namespace stn
