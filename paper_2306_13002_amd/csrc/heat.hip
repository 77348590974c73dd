// heat.hip -- Jacobi heat sweeps: 2-D five-point and 3-D seven-point, FP64.
//
//   2-D:  dst = cc*u + cn*u(-x) + cn*u(+x) + cn*u(-y) + cn*u(+y)
//   3-D:  ... + cn*u(-z) + cn*u(+z)
//
// PLAIN: the loop body as written, one thread per interior point, every
// operand loaded from memory, products rounded and added left to right (the
// library is compiled with -ffp-contract=off, so no FMA is formed).  This
// is the paper's "original" code for its Jacobi class.
//
// SATURATED (3-D): the paper's rewrites applied by hand.  COMM/ASSOC regroup
// the six neighbour products so the shared coefficient is applied once,
// FMA1 fuses it with the centre term:  dst = fma(cn, (xm+xp)+(ym+yp)+(zm+zp), cc*u).
// Loads: each block owns a TX x TY column tile and streams z; the centre
// column lives in a three-deep register queue (each value loaded once), the
// in-plane neighbours come from an LDS tile, and the next plane's loads are
// all issued before the current plane is computed ("bulk load").
#include "internal.hpp"

namespace stn {
namespace {

constexpr int kMaxWaves = 16;  // blocks of at most 1024 threads

__global__ void heat2d5_plain(const double *__restrict__ src, double *__restrict__ dst, Geom g, double cc,
                              double cn, double *__restrict__ part) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    double d2 = 0.0;
    if (i < g.nx && j < g.ny) {
        const long long q = (long long)(j + 1) * g.py + (i + 1);
        const double u = src[q];
        double v = cc * u;
        v = v + cn * src[q - 1];
        v = v + cn * src[q + 1];
        v = v + cn * src[q - g.py];
        v = v + cn * src[q + g.py];
        dst[q] = v;
        const double d = v - u;
        d2 = d * d;
    }
    if (part) {
        __shared__ double lds[kMaxWaves];
        const double s = block_sum_f64(d2, lds);
        if (threadIdx.x == 0 && threadIdx.y == 0) part[block_linear_id()] = s;
    }
}

// Plain 3-D body for one block-shaped tile (bx, by, bz) of blockDim points;
// returns this thread's squared change.
__device__ __forceinline__ double heat3d7_plain_tile(const double *__restrict__ src, double *__restrict__ dst,
                                                     const Geom &g, double cc, double cn, int bx, int by, int bz) {
    const int i = bx * blockDim.x + threadIdx.x;
    const int j = by * blockDim.y + threadIdx.y;
    const int k = bz * blockDim.z + threadIdx.z;
    double d2 = 0.0;
    if (i < g.nx && j < g.ny && k < g.nz) {
        const long long q = (long long)(k + 1) * g.pz + (long long)(j + 1) * g.py + (i + 1);
        const double u = src[q];
        double v = cc * u;
        v = v + cn * src[q - 1];
        v = v + cn * src[q + 1];
        v = v + cn * src[q - g.py];
        v = v + cn * src[q + g.py];
        v = v + cn * src[q - g.pz];
        v = v + cn * src[q + g.pz];
        dst[q] = v;
        const double d = v - u;
        d2 = d * d;
    }
    return d2;
}

__global__ void heat3d7_plain(const double *__restrict__ src, double *__restrict__ dst, Geom g, double cc,
                              double cn, double *__restrict__ part) {
    const double d2 = heat3d7_plain_tile(src, dst, g, cc, cn, blockIdx.x, blockIdx.y, blockIdx.z);
    if (part) {
        __shared__ double lds[kMaxWaves];
        const double s = block_sum_f64(d2, lds);
        if (threadIdx.x == 0 && threadIdx.y == 0 && threadIdx.z == 0) part[block_linear_id()] = s;
    }
}

// Saturated 3-D body for one TX x TY column tile (bx, by) streaming planes
// [bz*zb, bz*zb + zb); block (TX, TY) threads, one column each.  Returns this
// thread's sum of squared changes.  Ends with every LDS read done before the
// caller's next barrier-protected use of `tile`.
template <int TX, int TY>
__device__ __forceinline__ double heat3d7_sat_tile(const double *__restrict__ src, double *__restrict__ dst,
                                                   const Geom &g, double cc, double cn, int zb, int bx, int by,
                                                   int bz, double (*tile)[(TY + 2) * (TX + 2)]) {
    constexpr int R = 1, W = TX + 2 * R, NT = TX * TY;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
    const int i = bx * TX + tx, j = by * TY + ty;
    const int xp = i + R, yp = j + R;
    const int PX = g.nx + 2 * R, PY = g.ny + 2 * R, PZ = g.nz + 2 * R;
    const bool in = i < g.nx && j < g.ny;
    const bool ld = xp < PX && yp < PY;  // column inside the padded array (ring included)
    const int k0 = bz * zb, k1 = min(k0 + zb, g.nz);
    const long long col = (long long)yp * g.py + xp;
    const int me = (ty + R) * W + (tx + R);

    HaloStager<double, TX, TY, R, false, NT> halo;
    halo.init(tid, bx * TX + R, by * TY + R, g.py, PX, PY);

    // padded z of the plane being computed: zc = k + R
    double prv = ld ? src[col + (long long)(k0)*g.pz] : 0.0;
    double cur = ld ? src[col + (long long)(k0 + 1) * g.pz] : 0.0;
    double nxt = ld ? src[col + (long long)(k0 + 2) * g.pz] : 0.0;
    halo.load(src + (long long)(k0 + 1) * g.pz);
    double acc = 0.0;

    for (int k = k0; k < k1; ++k) {
        const int zc = k + R;
        const int b = (k - k0) & 1;
        // stage plane zc: centre from the queue, ring from the stager
        tile[b][me] = cur;
        halo.store(tile[b]);
        // bulk load: every global load of the next plane before this plane's math
        const double nn = (ld && zc + 2 < PZ) ? src[col + (long long)(zc + 2) * g.pz] : 0.0;
        if (k + 1 < k1) halo.load(src + (long long)(zc + 1) * g.pz);
        __syncthreads();
        if (in) {
            const double *t = tile[b];
            const double s = ((t[me - 1] + t[me + 1]) + (t[me - W] + t[me + W])) + (prv + nxt);
            const double v = fma(cn, s, cc * cur);
            dst[col + (long long)zc * g.pz] = v;
            const double d = v - cur;
            acc = fma(d, d, acc);
        }
        prv = cur;
        cur = nxt;
        nxt = nn;
    }
    return acc;
}

template <int TX, int TY>
__global__ __launch_bounds__(TX *TY) void heat3d7_sat(const double *__restrict__ src, double *__restrict__ dst,
                                                      Geom g, double cc, double cn, int zb, int remap,
                                                      double *__restrict__ part) {
    __shared__ double tile[2][(TY + 2) * (TX + 2)];
    __shared__ double red[kMaxWaves];
    int bx, by, bz;
    tile_coords(remap, bx, by, bz);
    const double acc = heat3d7_sat_tile<TX, TY>(src, dst, g, cc, cn, zb, bx, by, bz, tile);
    if (part) {
        const double s = block_sum_f64(acc, red);
        if (threadIdx.x == 0 && threadIdx.y == 0) part[block_linear_id()] = s;
    }
}

// Persistent work-list forms: each block walks items blockIdx.x, +gridDim.x,
// ... and runs the same tile body as the single-problem kernel, so a batched
// problem is bit-identical to its own run with the same form and shape.
template <int TX, int TY>
__global__ __launch_bounds__(TX *TY) void heat3d7_sat_batch(const BatchProb *__restrict__ probs,
                                                            const BatchItem *__restrict__ items, int n_items,
                                                            int parity, int zb, double *__restrict__ part) {
    __shared__ double tile[2][(TY + 2) * (TX + 2)];
    __shared__ double red[kMaxWaves];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const BatchItem w = items[it];
        const BatchProb &P = probs[w.prob];
        const double acc = heat3d7_sat_tile<TX, TY>(P.f[parity], P.f[parity ^ 1], P.g, P.cc, P.cn, zb, w.bx, w.by,
                                                    w.bz, tile);
        if (part) {
            const double s = block_sum_f64(acc, red);
            if (threadIdx.x == 0 && threadIdx.y == 0) part[it] = s;
        }
        __syncthreads();  // LDS is reused by the next item
    }
}

__global__ void heat3d7_plain_batch(const BatchProb *__restrict__ probs, const BatchItem *__restrict__ items,
                                    int n_items, int parity, double *__restrict__ part) {
    __shared__ double red[kMaxWaves];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const BatchItem w = items[it];
        const BatchProb &P = probs[w.prob];
        const double d2 = heat3d7_plain_tile(P.f[parity], P.f[parity ^ 1], P.g, P.cc, P.cn, w.bx, w.by, w.bz);
        if (part) {
            const double s = block_sum_f64(d2, red);
            if (threadIdx.x == 0 && threadIdx.y == 0 && threadIdx.z == 0) part[it] = s;
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------
bool plain_tile_ok(Tile t) {
    const long long n = (long long)t.tx * t.ty * t.tz;
    return t.tx >= 1 && t.ty >= 1 && t.tz >= 1 && n % 64 == 0 && n <= 1024;
}

bool h2_tile_ok(int v, Tile t) { return v == V_PLAIN && plain_tile_ok(t) && t.tz == 1; }

long long h2_nblocks(int, Tile t, const Geom &g) { return cdiv(g.nx, t.tx) * cdiv(g.ny, t.ty); }

hipError_t h2_launch(int v, Tile t, const SweepArgs &a, hipStream_t s) {
    if (v != V_PLAIN) return hipErrorInvalidValue;
    dim3 grid(cdiv(a.g.nx, t.tx), cdiv(a.g.ny, t.ty), 1), block(t.tx, t.ty, 1);
    hipLaunchKernelGGL(heat2d5_plain, grid, block, 0, s, (const double *)a.src, (double *)a.dst, a.g, a.c[0],
                       a.c[1], a.part);
    return hipGetLastError();
}

// Saturated tiles offered: (TX, TY) with TX*TY a multiple of 64, <= 1024.
#define HEAT3D7_SAT_TILES(X) X(32, 2) X(32, 4) X(32, 8) X(64, 1) X(64, 2) X(64, 4) X(64, 8) X(128, 1) X(128, 2) \
    X(128, 4) X(256, 1) X(256, 2)

bool h3_tile_ok(int v, Tile t) {
    if (v == V_PLAIN) return plain_tile_ok(t);
    if (t.tz < 1) return false;
#define X(a, b) if (t.tx == a && t.ty == b) return true;
    HEAT3D7_SAT_TILES(X)
#undef X
    return false;
}

int h3_sat_tiles(Tile *out, int max) {
    int n = 0;
#define X(a, b) if (n < max) out[n++] = Tile{a, b, 0};
    HEAT3D7_SAT_TILES(X)
#undef X
    return n;
}

long long h3_nblocks(int v, Tile t, const Geom &g) {
    return cdiv(g.nx, t.tx) * cdiv(g.ny, t.ty) * cdiv(g.nz, t.tz);
}

hipError_t h3_launch(int v, Tile t, const SweepArgs &a, hipStream_t s) {
    const double *src = (const double *)a.src;
    double *dst = (double *)a.dst;
    dim3 grid(cdiv(a.g.nx, t.tx), cdiv(a.g.ny, t.ty), cdiv(a.g.nz, t.tz));
    if (v == V_PLAIN) {
        hipLaunchKernelGGL(heat3d7_plain, grid, dim3(t.tx, t.ty, t.tz), 0, s, src, dst, a.g, a.c[0], a.c[1],
                           a.part);
        return hipGetLastError();
    }
#define X(A, B)                                                                                        \
    if (t.tx == A && t.ty == B) {                                                                      \
        hipLaunchKernelGGL((heat3d7_sat<A, B>), grid, dim3(A, B, 1), 0, s, src, dst, a.g, a.c[0], a.c[1], \
                           t.tz, a.remap, a.part);                                                     \
        return hipGetLastError();                                                                      \
    }
    HEAT3D7_SAT_TILES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t h3_batch_launch(int v, Tile t, const BatchProb *probs, const BatchItem *items, int n_items, int parity,
                           int grid, double *part, hipStream_t s) {
    if (v == V_PLAIN) {
        hipLaunchKernelGGL(heat3d7_plain_batch, dim3(grid), dim3(t.tx, t.ty, t.tz), 0, s, probs, items, n_items, parity,
                           part);
        return hipGetLastError();
    }
#define X(A, B)                                                                                                \
    if (t.tx == A && t.ty == B) {                                                                              \
        hipLaunchKernelGGL((heat3d7_sat_batch<A, B>), dim3(grid), dim3(A, B, 1), 0, s, probs, items, n_items,   \
                           parity, t.tz, part);                                                                \
        return hipGetLastError();                                                                              \
    }
    HEAT3D7_SAT_TILES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace

KindOps heat2d5_ops = {h2_tile_ok, nullptr, nullptr, h2_nblocks, h2_launch, nullptr};
KindOps heat3d7_ops = {h3_tile_ok, h3_sat_tiles, nullptr, h3_nblocks, h3_launch, h3_batch_launch};

}  // namespace stn
