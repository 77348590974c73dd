// generic.hip -- generic 3-D linear stencils (star or box, radius 1..4).
//
//   u'(x) = sum_t coef[cid_t] * u(x + delta_t)
//
// F32 or F64 storage; arithmetic is FP64 in both (operands widened on load,
// the result rounded to the storage type on store).
//
// PLAIN: one thread per point; taps in the caller's order, each operand
// loaded from memory, products rounded and added left to right.  The tap
// table (linear offset, coefficient per tap) is uniform across the launch,
// so it is read through the scalar cache.
//
// SATURATED: the paper's rewrites on the tap sum.  COMM/ASSOC gather the
// taps that share a coefficient id AND a z offset into one group, summed
// first (taps in ascending address order) and multiplied once with an FMA
// (FMA1).  Loads: a block owns a TX x TY column tile and streams input
// planes; each plane is staged once in LDS (with its r-wide ring, corners
// included) and contributes to the 2r+1 output planes it touches, which
// wait in a register queue of FP64 accumulators (plane accumulation), so
// every input value is read from memory once per block.  The next plane's
// loads are issued before the current plane's arithmetic.
#include "generic_body.hpp"
#include "internal.hpp"
#include "rtc.hpp"

namespace stn {
namespace {

constexpr int kMaxWaves = 16;

template <typename T>
__global__ void generic_plain(const T *__restrict__ src, T *__restrict__ dst, Geom g, GenTab tab,
                             double *__restrict__ part) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    double d2 = 0.0;
    if (i < g.nx && j < g.ny && k < g.nz) {
        const long long q = (long long)(k + g.r) * g.pz + (long long)(j + g.r) * g.py + (i + g.r);
        double v = tab.c[0] * (double)src[q + tab.off[0]];
        for (int t = 1; t < tab.n; ++t) v = v + tab.c[t] * (double)src[q + tab.off[t]];
        const T out = (T)v;
        dst[q] = out;
        const double d = (double)out - (double)src[q];
        d2 = d * d;
    }
    if (part) {
        __shared__ double lds[kMaxWaves];
        const double s = block_sum_f64(d2, lds);
        if (threadIdx.x == 0 && threadIdx.y == 0 && threadIdx.z == 0) part[block_linear_id()] = s;
    }
}

// Table-driven tap sums: slot s's groups are read from the plan's tables.
template <typename T, int R, int TX, int TY, bool CORNERS>
struct TableSlotsW {
    GenTab tab;
    __device__ __forceinline__ void operator()(const double *__restrict__ t, int me, double *acc) const {
        constexpr int W = TX + 2 * R;
#pragma unroll
        for (int s = 0; s < 2 * R + 1; ++s) {
            const int g0 = tab.slot_g[s], g1 = tab.slot_g[s + 1];
            double a = acc[s];
            for (int gi = g0; gi < g1; ++gi) {
                const int t0 = tab.g_t[gi], t1 = tab.g_t[gi + 1];
                // the group's taps (ascending address): eight LDS reads in
                // flight, four independent partial sums, then one FMA
                double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
                int ti = t0;
                for (; ti + 8 <= t1; ti += 8) {
                    double v[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        const int xy = tab.t_xy[ti + q];
                        v[q] = t[me + (xy >> 16) * W + (short)(xy & 0xFFFF)];
                    }
                    s0 += v[0] + v[4];
                    s1 += v[1] + v[5];
                    s2 += v[2] + v[6];
                    s3 += v[3] + v[7];
                }
                for (; ti < t1; ++ti) {
                    const int xy = tab.t_xy[ti];
                    s0 += t[me + (xy >> 16) * W + (short)(xy & 0xFFFF)];
                }
                a = fma(tab.g_c[gi], (s0 + s1) + (s2 + s3), a);
            }
            acc[s] = a;
        }
    }
};

template <typename T, int R, int TX, int TY, bool CORNERS>
__global__ __launch_bounds__(TX *TY) void generic_sat(const T *__restrict__ src, T *__restrict__ dst, Geom g,
                                                      GenTab tab, int zb, int remap, double *__restrict__ part) {
    __shared__ double tile[2][(TY + 2 * R) * (TX + 2 * R)];
    __shared__ double red[kMaxWaves];
    int bx, by, bz;
    tile_coords(remap, bx, by, bz);
    const double sacc = generic_sat_body<T, R, TX, TY, CORNERS>(src, dst, g, zb, bx, by, bz,
                                                               TableSlotsW<T, R, TX, TY, CORNERS>{tab}, tile);
    if (part) {
        const double s = block_sum_f64(sacc, red);
        if (threadIdx.x == 0 && threadIdx.y == 0) part[block_linear_id()] = s;
    }
}

bool plain_tile_ok(Tile t) {
    const long long n = (long long)t.tx * t.ty * t.tz;
    return t.tx >= 1 && t.ty >= 1 && t.tz >= 1 && n % 64 == 0 && n <= 1024;
}

#define GEN_SAT_TILES(X) X(32, 4) X(32, 8) X(64, 2) X(64, 4) X(128, 2)

bool gen_tile_ok(int v, Tile t) {
    if (v == V_PLAIN) return plain_tile_ok(t);
    if (t.tz < 1) return false;
#define X(a, b) if (t.tx == a && t.ty == b) return true;
    GEN_SAT_TILES(X)
#undef X
    return false;
}

int gen_sat_tiles(Tile *out, int max) {
    int n = 0;
#define X(a, b) if (n < max) out[n++] = Tile{a, b, 0};
    GEN_SAT_TILES(X)
#undef X
    return n;
}

long long gen_nblocks(int, Tile t, const Geom &g) { return cdiv(g.nx, t.tx) * cdiv(g.ny, t.ty) * cdiv(g.nz, t.tz); }

template <typename T>
hipError_t gen_launch_t(int v, Tile t, const SweepArgs &a, hipStream_t s) {
    const T *src = (const T *)a.src;
    T *dst = (T *)a.dst;
    dim3 grid(cdiv(a.g.nx, t.tx), cdiv(a.g.ny, t.ty), cdiv(a.g.nz, t.tz));
    if (v == V_PLAIN) {
        hipLaunchKernelGGL(generic_plain<T>, grid, dim3(t.tx, t.ty, t.tz), 0, s, src, dst, a.g, a.gen, a.part);
        return hipGetLastError();
    }
#define GEN_LAUNCH(A_, B_, R_, C_)                                                                          \
    hipLaunchKernelGGL((generic_sat<T, R_, A_, B_, C_>), grid, dim3(A_, B_, 1), 0, s, src, dst, a.g, a.gen,   \
                       t.tz, a.remap, a.part)
#define X(A, B)                                                                                             \
    if (t.tx == A && t.ty == B) {                                                                           \
        const bool c = a.gen.corners;                                                                       \
        switch (a.g.r) {                                                                                    \
        case 1: if (c) GEN_LAUNCH(A, B, 1, true); else GEN_LAUNCH(A, B, 1, false); break;                               \
        case 2: if (c) GEN_LAUNCH(A, B, 2, true); else GEN_LAUNCH(A, B, 2, false); break;                               \
        case 3: if (c) GEN_LAUNCH(A, B, 3, true); else GEN_LAUNCH(A, B, 3, false); break;                               \
        case 4: if (c) GEN_LAUNCH(A, B, 4, true); else GEN_LAUNCH(A, B, 4, false); break;                               \
        default: return hipErrorInvalidValue;                                                               \
        }                                                                                                   \
        return hipGetLastError();                                                                           \
    }
    GEN_SAT_TILES(X)
#undef X
#undef GEN_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t gen_launch(int v, Tile t, const SweepArgs &a, hipStream_t s) {
    if (v == V_SATURATED && a.rtc) return rtc_generic_launch(*a.rtc, t, a, s);
    return a.elem_bytes == 4 ? gen_launch_t<float>(v, t, a, s) : gen_launch_t<double>(v, t, a, s);
}

}  // namespace

KindOps generic_ops = {gen_tile_ok, gen_sat_tiles, nullptr, gen_nblocks, gen_launch, nullptr};

}  // namespace stn
