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

// PLAIN 2-D with fused sweeps: one launch performs k sweeps of the plain
// body.  A block owns an OT x OT output tile; it loads the tile and a k-cell
// ring around it into LDS, runs sweep s = 1..k on the cells within k - s of
// the tile (each from the previous sweep's values, ping-ponging two LDS
// buffers, one barrier per sweep), and writes the tile.  The ring is
// recomputed by every block that needs it, never exchanged.  Every value is
// computed with the plain body's operands and order, so the result equals k
// single launches bit for bit; cells that are not interior keep their value
// (Dirichlet), cells outside the padded array hold 0 and are read by none.
// The residual is the last sweep's, summed per block in the block's order.
// The launch also writes dst's boundary ring (the run needs no halo copy).
// Block 16 x 16 threads; k <= kFuseMax.
constexpr int kFuseMax = 16;

template <int OT>
__global__ __launch_bounds__(256) void heat2d5_fused(const double *__restrict__ src, double *__restrict__ dst, Geom g,
                                                     double cc, double cn, int k, double *__restrict__ part) {
    constexpr int S = OT + 2 * kFuseMax;
    __shared__ double buf[2][S * S];
    __shared__ double red[kMaxWaves];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int L = OT + 2 * k;                                           // region side (<= S)
    const int X0 = blockIdx.x * OT + 1 - k, Y0 = blockIdx.y * OT + 1 - k;  // padded coords of region cell (0, 0)
    const int PX = g.nx + 2, PY = g.ny + 2;
    for (int cy = ty; cy < L; cy += 16)
        for (int cx = tx; cx < L; cx += 16) {
            const int X = X0 + cx, Y = Y0 + cy;
            buf[0][cy * L + cx] = (X >= 0 && X < PX && Y >= 0 && Y < PY) ? src[(long long)Y * g.py + X] : 0.0;
        }
    __syncthreads();
    int a = 0;
    for (int s = 1; s <= k; ++s) {
        const double *A = buf[a];
        double *B = buf[a ^ 1];
        for (int cy = s + ty; cy < L - s; cy += 16)
            for (int cx = s + tx; cx < L - s; cx += 16) {
                const int X = X0 + cx, Y = Y0 + cy, e = cy * L + cx;
                const double u = A[e];
                double v = u;
                if (X >= 1 && X <= g.nx && Y >= 1 && Y <= g.ny) {
                    v = cc * u;
                    v = v + cn * A[e - 1];
                    v = v + cn * A[e + 1];
                    v = v + cn * A[e - L];
                    v = v + cn * A[e + L];
                }
                B[e] = v;
            }
        __syncthreads();
        a ^= 1;
    }
    const double *F = buf[a], *P = buf[a ^ 1];  // sweep k and sweep k-1 (the loaded values when k = 1)
    double d2 = 0.0;
    for (int cy = k + ty; cy < k + OT; cy += 16)
        for (int cx = k + tx; cx < k + OT; cx += 16) {
            const int X = X0 + cx, Y = Y0 + cy, e = cy * L + cx;
            if (X <= g.nx && Y <= g.ny) {
                dst[(long long)Y * g.py + X] = F[e];
                const double d = F[e] - P[e];
                d2 = d2 + d * d;
            }
        }
    // The boundary ring of dst (Dirichlet: the loaded values, unchanged by
    // every sweep; buf[0] holds them at every region cell), so no separate
    // halo copy has to precede the launch: each ring cell is written by the
    // block whose tile holds its nearest interior cell.
    for (int cy = k - 1 + ty; cy <= k + OT; cy += 16)
        for (int cx = k - 1 + tx; cx <= k + OT; cx += 16) {
            const int X = X0 + cx, Y = Y0 + cy;
            const bool ring = X >= 0 && X < PX && Y >= 0 && Y < PY && (X == 0 || X == PX - 1 || Y == 0 || Y == PY - 1);
            const int Xi = min(max(X, 1), g.nx), Yi = min(max(Y, 1), g.ny);
            if (ring && (Xi - 1) / OT == (int)blockIdx.x && (Yi - 1) / OT == (int)blockIdx.y)
                dst[(long long)Y * g.py + X] = buf[0][cy * L + cx];
        }
    if (part) {
        const double sum = block_sum_f64(d2, red);
        if (tx == 0 && ty == 0) part[block_linear_id()] = sum;
    }
}

// The same fused sweeps with one region cell per thread, for regions of at
// most 32 x 32 cells (OT + 2k <= 32): a 1-D block of L*L threads rounded up
// to whole waves, thread c holding region cell (c mod L, c div L).  Each
// thread keeps its own cell's value in a register from sweep to sweep and
// reads only its four neighbours from the previous sweep's LDS buffer, so a
// sweep is four independent LDS reads, the update, one LDS write and one
// barrier, with every lane of the block's waves at work.  Operands and order
// are the plain body's, as above; the padding threads past L*L take part in
// the barriers and the residual sum only.
__global__ __launch_bounds__(1024) void heat2d5_fused_cell(const double *__restrict__ src, double *__restrict__ dst,
                                                           Geom g, double cc, double cn, int OT, int k,
                                                           double *__restrict__ part) {
    __shared__ double buf[2][32 * 32];
    __shared__ double red[kMaxWaves];
    const int L = OT + 2 * k, c = threadIdx.x;
    const bool cell = c < L * L;
    const int cx = c % L, cy = c / L;
    const int X = blockIdx.x * OT + 1 - k + cx, Y = blockIdx.y * OT + 1 - k + cy;  // padded coords
    const int PX = g.nx + 2, PY = g.ny + 2;
    const bool inarr = cell && X >= 0 && X < PX && Y >= 0 && Y < PY;
    const bool interior = X >= 1 && X <= g.nx && Y >= 1 && Y <= g.ny;
    const long long q = (long long)Y * g.py + X;
    const double u0 = inarr ? src[q] : 0.0;
    double u = u0, prev = u0;  // this cell after the last sweep and the one before
    if (cell) buf[0][c] = u0;
    __syncthreads();
    for (int s = 1; s <= k; ++s) {
        const double *A = buf[(s - 1) & 1];
        if (cell && cx >= s && cx < L - s && cy >= s && cy < L - s) {  // within k - s of the tile
            double v = u;
            if (interior) {
                v = cc * u;
                v = v + cn * A[c - 1];
                v = v + cn * A[c + 1];
                v = v + cn * A[c - L];
                v = v + cn * A[c + L];
            }
            prev = u;
            u = v;
            buf[s & 1][c] = v;
        }
        __syncthreads();
    }
    double d2 = 0.0;
    if (cell && cx >= k && cx < k + OT && cy >= k && cy < k + OT && X <= g.nx && Y <= g.ny) {
        dst[q] = u;
        const double d = u - prev;
        d2 = d * d;
    }
    // dst's boundary ring, as in heat2d5_fused: the loaded values, each cell
    // written by the block whose tile holds its nearest interior cell
    if (inarr && cx >= k - 1 && cx <= k + OT && cy >= k - 1 && cy <= k + OT &&
        (X == 0 || X == PX - 1 || Y == 0 || Y == PY - 1)) {
        const int Xi = min(max(X, 1), g.nx), Yi = min(max(Y, 1), g.ny);
        if ((Xi - 1) / OT == (int)blockIdx.x && (Yi - 1) / OT == (int)blockIdx.y) dst[q] = u0;
    }
    if (part) {
        const double sum = block_sum_f64(d2, red);
        if (c == 0) part[block_linear_id()] = sum;
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
    // running offset of plane zc (one 64-bit add per plane instead of a
    // multiply per access)
    long long zo = (long long)(k0 + R) * g.pz;
    const long long pz = g.pz;

    for (int k = k0; k < k1; ++k, zo += pz) {
        const int zc = k + R;
        const int b = (k - k0) & 1;
        // stage plane zc: centre from the queue, ring from the stager
        tile[b][me] = cur;
        halo.store(tile[b]);
        // bulk load: every global load of the next plane before this plane's math
        const double nn = (ld && zc + 2 < PZ) ? src[col + zo + 2 * pz] : 0.0;
        if (k + 1 < k1) halo.load(src + zo + pz);
        __syncthreads();
        if (in) {
            const double *t = tile[b];
            const double s = ((t[me - 1] + t[me + 1]) + (t[me - W] + t[me + W])) + (prv + nxt);
            const double v = fma(cn, s, cc * cur);
            dst[col + zo] = v;
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

// Two sweeps per pass (SATURATED_T2): the block's TY rows of tile threads
// compute sweep 1 and sweep 2 of their own column; EY extra rows of ring
// threads compute sweep 1 on the one-cell ring around the tile (recomputed
// by every block that needs it).  p^t planes sit in a four-plane LDS ring
// with a two-cell halo, sweep-1 planes in a four-plane ring; sweep 2 runs two
// planes behind sweep 1, one barrier per plane.  Each value is computed with
// the same operations as heat3d7_sat_tile, so two sweeps equal two launches
// of the single-sweep form bit for bit.  In-plane neighbours come from the
// LDS rings; the centre values of the planes above and below from per-thread
// z-queues (sweep 2's from the thread's own sweep-1 values), which cuts the
// LDS reads per output column from 14 to 9.  Dirichlet only.
template <int TX, int TY>
struct H3Sat2Shape {
    // W0, W1: widths of the p^t and sweep-1 tiles; LS0, LS1: their LDS row
    // strides, odd numbers of doubles so that the ring threads' column
    // accesses spread over the banks
    static constexpr int W0 = TX + 4, LS0 = W0 + 1, PL0 = (TY + 4) * LS0;
    static constexpr int W1 = TX + 2, LS1 = W1 + 1, PL1 = (TY + 2) * LS1;
    static constexpr int RS = 2 * W1 + 2 * TY;
    static constexpr int EY0 = (RS + TX - 1) / TX;
    static constexpr int EY = (TX * (TY + EY0)) % 64 == 0 ? EY0 : EY0 + 1;
    static constexpr int NT = TX * (TY + EY);
};

template <int TX, int TY>
__device__ __forceinline__ double heat3d7_sat2_tile(const double *__restrict__ src, double *__restrict__ dst,
                                                    const Geom &g, double cc, double cn, int zb, int bx, int by,
                                                    int bz, double (*r0)[H3Sat2Shape<TX, TY>::PL0],
                                                    double (*r1)[H3Sat2Shape<TX, TY>::PL1]) {
    using S = H3Sat2Shape<TX, TY>;
    constexpr int W1 = S::W1, LS0 = S::LS0, LS1 = S::LS1, NT = S::NT, RS = S::RS;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
    const int PX = g.nx + 2, PY = g.ny + 2;
    const int k0 = bz * zb, k1 = min(k0 + zb, g.nz);
    const bool tile_t = ty < TY;
    const int xo = bx * TX + tx + 1, yo = by * TY + ty + 1;  // padded
    const bool in_o = tile_t && xo <= g.nx && yo <= g.ny;
    const bool ld_o = tile_t && xo < PX && yo < PY;
    const long long col_o = (long long)yo * g.py + xo;
    const int e0_o = (ty + 2) * LS0 + tx + 2, e1_o = (ty + 1) * LS1 + tx + 1;
    const int q = tid - TX * TY;
    const bool has_r = !tile_t && q < RS;
    int ex = 0, ey = 0;
    if (q < W1) {
        ex = q;
    } else if (q < 2 * W1) {
        ex = q - W1;
        ey = TY + 1;
    } else if (q < 2 * W1 + TY) {
        ey = q - 2 * W1 + 1;
    } else {
        ex = W1 - 1;
        ey = q - 2 * W1 - TY + 1;
    }
    const int xr = bx * TX + ex, yr = by * TY + ey;
    const bool in_r = has_r && xr >= 1 && xr <= g.nx && yr >= 1 && yr <= g.ny;
    const bool in_a = tile_t ? in_o : in_r, has_a = tile_t || has_r;
    const int e0_a = tile_t ? e0_o : (ey + 1) * LS0 + ex + 1, e1_a = tile_t ? e1_o : ey * LS1 + ex;

    HaloStager<double, TX, TY, 2, true, NT, LS0> halo;
    halo.init(tid, bx * TX + 1, by * TY + 1, g.py, PX, PY);
    const int zlo = k0, zhi = k1 + 1;
    for (int z = zlo - 1; z <= zlo; ++z) {
        if (z < 0) continue;
        const double *pl = src + (long long)z * g.pz;
        if (tile_t) r0[(z - zlo + 4) & 3][e0_o] = ld_o ? pl[col_o] : 0.0;
        halo.load(pl);
        halo.store(r0[(z - zlo + 4) & 3]);
    }
    double ctr = ld_o ? src[col_o + (long long)(zlo + 1) * g.pz] : 0.0;
    halo.load(src + (long long)(zlo + 1) * g.pz);
    double acc = 0.0;
    // z-queues of centre values: q1m, q1o = planes zA-1, zA of p^t at this
    // thread's sweep-1 cell; s1a, s1b, s1c = this thread's own sweep-1 values
    // of planes zA-1, zA-2, zA-3 (for a tile thread, the centres sweep 2 reads)
    double q1m = 0.0, q1o = 0.0, s1a = 0.0, s1b = 0.0, s1c = 0.0;
    __syncthreads();
    if (has_a) {
        q1m = r0[3][e0_a];  // plane zlo-1 (unused when zlo = 0: sweep 1 copies plane 0)
        q1o = r0[0][e0_a];
    }
    // ring slots relative to zlo: plane z sits in slot (z - zlo) mod 4; SM,
    // S0, SP, S2 are the slots of planes zA-1, zA, zA+1 and zA+2 (= zA-2)
    // running plane pointers (one 64-bit add per plane instead of a multiply)
    const double *pl_next = src + (long long)(zlo + 2) * g.pz;
    double *out_pl = dst + (long long)(zlo - 2) * g.pz;
    auto step = [&](const int zA, const int SM, const int S0, const int SP, const int S2) {
        if (zA <= zhi) {
            if (tile_t) r0[SP][e0_o] = ctr;
            halo.store(r0[SP]);
            if (zA < zhi && zA + 2 <= g.nz + 1) {
                ctr = ld_o ? pl_next[col_o] : 0.0;
                halo.load(pl_next);
            }
        }
        pl_next += g.pz;
        __syncthreads();
        double v1 = 0.0;
        if (zA <= zhi && has_a) {  // sweep 1 at plane zA
            const double *o = r0[S0];
            const int e = e0_a;
            const double uc = r0[SP][e];
            v1 = q1o;
            if (zA >= 1 && zA <= g.nz && in_a) {
                const double s = ((o[e - 1] + o[e + 1]) + (o[e - LS0] + o[e + LS0])) + (q1m + uc);
                v1 = fma(cn, s, cc * q1o);
            }
            r1[S0][e1_a] = v1;
            q1m = q1o;
            q1o = uc;
        }
        const int zc = zA - 2;  // sweep 2 at plane zc
        if (zc >= k0 + 1 && in_o) {
            const double *o = r1[S2];
            const int e = e1_o;
            const double s = ((o[e - 1] + o[e + 1]) + (o[e - LS1] + o[e + LS1])) + (s1c + s1a);
            const double v = fma(cn, s, cc * s1b);
            out_pl[col_o] = v;
            const double d = v - s1b;
            acc = fma(d, d, acc);
        }
        s1c = s1b;
        s1b = s1a;
        s1a = v1;
        out_pl += g.pz;
    };
    // four planes per trip, so that every slot is a compile-time constant
    // (7-10 % faster than slots computed per plane)
    for (int zA = zlo; zA <= zhi + 1; zA += 4) {
        step(zA, 3, 0, 1, 2);
        if (zA + 1 <= zhi + 1) step(zA + 1, 0, 1, 2, 3);
        if (zA + 2 <= zhi + 1) step(zA + 2, 1, 2, 3, 0);
        if (zA + 3 <= zhi + 1) step(zA + 3, 2, 3, 0, 1);
    }
    return acc;
}

template <int TX, int TY>
__global__ __launch_bounds__((H3Sat2Shape<TX, TY>::NT)) void heat3d7_sat2(const double *__restrict__ src,
                                                                           double *__restrict__ dst, Geom g,
                                                                           double cc, double cn, int zb, int remap,
                                                                           double *__restrict__ part) {
    using S = H3Sat2Shape<TX, TY>;
    __shared__ double r0[4][S::PL0];
    __shared__ double r1[4][S::PL1];
    __shared__ double red[kMaxWaves];
    int bx, by, bz;
    tile_coords(remap, bx, by, bz);
    const double acc = heat3d7_sat2_tile<TX, TY>(src, dst, g, cc, cn, zb, bx, by, bz, r0, r1);
    if (part) {
        const double s = block_sum_f64(acc, red);
        if (threadIdx.x == 0 && threadIdx.y == 0) part[block_linear_id()] = s;
    }
}

// Three sweeps per pass (SATURATED_T3): one thread per column of an RX x RY
// region around the (RX - 4) x (RY - 4) output tile.  Sweep j (1..k, k <= 3
// sweeps in this launch) runs on the region cells within k - j of the tile,
// two planes behind sweep j - 1, so the value it needs from sweep j - 1 one
// plane up was computed one step earlier, before the barrier that separates
// the steps.  In-plane neighbours come from three-plane LDS rings (p^t with a
// one-cell halo, then one ring per intermediate sweep); the column's centre
// values from the thread's own registers (the p^t column it loads, and
// per-sweep queues of its last three values).  Three slots suffice: a step
// writes a plane two planes ahead of the one it reads, and the previous
// step's reads are separated from this step's writes by the barrier.  Every
// value is computed with heat3d7_sat_tile's operations, so a pass equals k
// single-sweep launches bit for bit.  Dirichlet only.
template <int RX, int RY>
struct H3Sat3Shape {
    static constexpr int K = 3, TX = RX - 2 * (K - 1), TY = RY - 2 * (K - 1), NT = RX * RY;
    // row strides: odd numbers of doubles
    static constexpr int LSP = RX + 3, PLP = (RY + 2) * LSP;  // p^t: the region and a one-cell halo
    static constexpr int LSL = RX + 1, PLL = RY * LSL;        // intermediate sweeps: the region
};

// KK: the sweeps of this launch (3, or 1 or 2 for the remainder of a count),
// a compile-time constant so that every sweep's participation test and
// plane range fold.
template <int RX, int RY, int KK>
__device__ __forceinline__ double heat3d7_sat3_tile(const double *__restrict__ src, double *__restrict__ dst,
                                                    const Geom &g, double cc, double cn, int zb, int bx, int by, int bz,
                                                    double (*P)[H3Sat3Shape<RX, RY>::PLP],
                                                    double (*Lv)[3][H3Sat3Shape<RX, RY>::PLL]) {
    using S = H3Sat3Shape<RX, RY>;
    constexpr int k = KK;
    static_assert(KK >= 1 && KK <= S::K, "one to three sweeps per launch");
    constexpr int K = S::K, TX = S::TX, TY = S::TY, LSP = S::LSP, LSL = S::LSL, NT = S::NT;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * RX + tx;
    const int PX = g.nx + 2, PY = g.ny + 2;
    const int xr0 = bx * TX + 1 - (K - 1), yr0 = by * TY + 1 - (K - 1);  // padded coords of region cell (0, 0)
    const int X = xr0 + tx, Y = yr0 + ty;
    const int dx = max(max(bx * TX + 1 - X, X - bx * TX - TX), 0);
    const int dy = max(max(by * TY + 1 - Y, Y - by * TY - TY), 0);
    const int d = max(dx, dy);  // distance of this column from the output tile
    const bool col_ok = X >= 0 && X < PX && Y >= 0 && Y < PY;
    const bool inxy = X >= 1 && X <= g.nx && Y >= 1 && Y <= g.ny;
    const bool out_t = d == 0 && X <= g.nx && Y <= g.ny;
    const long long col = col_ok ? (long long)Y * g.py + X : 0;
    const int eP = (ty + 1) * LSP + tx + 1, eL = ty * LSL + tx;
    const int k0 = bz * zb, k1 = min(k0 + zb, g.nz);  // output planes k0+1 .. k1 (padded)
    const int hi0 = min(g.nz + 1, k1 + k);            // last p^t plane a sweep reads
    HaloStager<double, RX, RY, 1, false, NT, LSP> halo;
    halo.init(tid, xr0, yr0, g.py, PX, PY);
    auto pin = [&](int z) { return z >= 0 && z <= hi0; };
    auto ldp = [&](int z) { return (col_ok && pin(z)) ? src[col + (long long)z * g.pz] : 0.0; };
    auto hload = [&](int z) {
        if (pin(z)) {
            halo.load(src + (long long)z * g.pz);
        } else {
#pragma unroll
            for (int s = 0; s < decltype(halo)::HR; ++s) halo.val[s] = 0.0;
        }
    };
    // step t runs sweep j at plane t - 2(j - 1); plane z sits in ring slot (z - t0) mod 3
    const int t0 = k0 + 1 - (k - 1), tE = k1 + 2 * (k - 1);
    double pm1 = ldp(t0 - 1), p0 = ldp(t0);
    hload(t0);
    P[0][eP] = p0;
    halo.store(P[0]);
    double cA = ldp(t0 + 1), cB = 0.0;
    hload(t0 + 1);
    double qa[K], qb[K], qc[K];  // sweep j's values at the last three steps (j = 1, 2 used)
#pragma unroll
    for (int j = 0; j < K; ++j) qa[j] = qb[j] = qc[j] = 0.0;
    double acc = 0.0;
    // u = (t - t0) mod 6: ring slots and the staging register are compile-time
    auto step = [&](const int t, const int u, double &cur, double &nxt) {
        P[(u + 1) % 3][eP] = cur;  // p^t plane t + 1, loaded one step earlier
        halo.store(P[(u + 1) % 3]);
        if (pin(t + 2)) {
            nxt = ldp(t + 2);
            halo.load(src + (long long)(t + 2) * g.pz);
        }
        __syncthreads();
#pragma unroll
        for (int j = K; j >= 1; --j) {  // the last sweep first: each reads the queue before it advances
            if (j > k) continue;
            const int z = t - 2 * (j - 1);
            const int sl = (u + 6 - 2 * (j - 1)) % 3;
            const int lo = max(0, k0 + 1 - (k - j)), hi = min(g.nz + 1, k1 + (k - j));
            if (d <= k - j && z >= lo && z <= hi) {
                const double below = j == 1 ? pm1 : qc[j - 1];
                const double centre = j == 1 ? p0 : qb[j - 1];
                const double above = j == 1 ? cur : qa[j - 1];
                double v = centre;
                if (inxy && z >= 1 && z <= g.nz) {
                    const double *o = j == 1 ? P[u % 3] : Lv[j - 2 < 0 ? 0 : j - 2][sl];
                    const int e = j == 1 ? eP : eL, LS = j == 1 ? LSP : LSL;
                    const double sm = ((o[e - 1] + o[e + 1]) + (o[e - LS] + o[e + LS])) + (below + above);
                    v = fma(cn, sm, cc * centre);
                }
                if (j < k) {
                    Lv[j - 1][sl][eL] = v;
                    qc[j] = qb[j];
                    qb[j] = qa[j];
                    qa[j] = v;
                } else if (out_t) {
                    dst[col + (long long)z * g.pz] = v;
                    const double dd = v - centre;
                    acc = fma(dd, dd, acc);
                }
            } else if (j < k) {  // keep the queue aligned with the steps
                qc[j] = qb[j];
                qb[j] = qa[j];
                qa[j] = 0.0;
            }
        }
        pm1 = p0;
        p0 = cur;
    };
    for (int t = t0;; t += 6) {
        if (t > tE) break;
        step(t, 0, cA, cB);
        if (t + 1 > tE) break;
        step(t + 1, 1, cB, cA);
        if (t + 2 > tE) break;
        step(t + 2, 2, cA, cB);
        if (t + 3 > tE) break;
        step(t + 3, 3, cB, cA);
        if (t + 4 > tE) break;
        step(t + 4, 4, cA, cB);
        if (t + 5 > tE) break;
        step(t + 5, 5, cB, cA);
    }
    return acc;
}

template <int RX, int RY, int KK>
__global__ __launch_bounds__(RX *RY) void heat3d7_sat3(const double *__restrict__ src, double *__restrict__ dst,
                                                       Geom g, double cc, double cn, int zb, int remap,
                                                       double *__restrict__ part) {
    using S = H3Sat3Shape<RX, RY>;
    __shared__ double P[3][S::PLP];
    __shared__ double Lv[2][3][S::PLL];
    __shared__ double red[kMaxWaves];
    int bx, by, bz;
    tile_coords(remap, bx, by, bz);
    const double acc = heat3d7_sat3_tile<RX, RY, KK>(src, dst, g, cc, cn, zb, bx, by, bz, P, Lv);
    if (part) {
        const double s = block_sum_f64(acc, red);
        if (threadIdx.x == 0 && threadIdx.y == 0) part[block_linear_id()] = s;
    }
}

// Work-list forms: each block walks items blockIdx.x, +gridDim.x, ... (the
// batch launches one block per item up to 2^20 items) and runs the same tile
// body as the single-problem kernel, so a batched problem is bit-identical to
// its own run with the same form and shape.
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
            if (threadIdx.x == 0 && threadIdx.y == 0) part[w.slot] = s;
        }
        __syncthreads();  // LDS is reused by the next item
    }
}

template <int TX, int TY>
__global__ __launch_bounds__((H3Sat2Shape<TX, TY>::NT)) void heat3d7_sat2_batch(const BatchProb *__restrict__ probs,
                                                                                 const BatchItem *__restrict__ items,
                                                                                 int n_items, int parity, int zb,
                                                                                 double *__restrict__ part) {
    using S = H3Sat2Shape<TX, TY>;
    __shared__ double r0[4][S::PL0];
    __shared__ double r1[4][S::PL1];
    __shared__ double red[kMaxWaves];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const BatchItem w = items[it];
        const BatchProb &P = probs[w.prob];
        const double acc = heat3d7_sat2_tile<TX, TY>(P.f[parity], P.f[parity ^ 1], P.g, P.cc, P.cn, zb, w.bx, w.by,
                                                     w.bz, r0, r1);
        if (part) {
            const double s = block_sum_f64(acc, red);
            if (threadIdx.x == 0 && threadIdx.y == 0) part[w.slot] = s;
        }
        __syncthreads();  // LDS is reused by the next item
    }
}

template <int RX, int RY, int KK>
__global__ __launch_bounds__(RX *RY) void heat3d7_sat3_batch(const BatchProb *__restrict__ probs,
                                                             const BatchItem *__restrict__ items, int n_items,
                                                             int parity, int zb, double *__restrict__ part) {
    using S = H3Sat3Shape<RX, RY>;
    __shared__ double P[3][S::PLP];
    __shared__ double Lv[2][3][S::PLL];
    __shared__ double red[kMaxWaves];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const BatchItem w = items[it];
        const BatchProb &Q = probs[w.prob];
        const double acc = heat3d7_sat3_tile<RX, RY, KK>(Q.f[parity], Q.f[parity ^ 1], Q.g, Q.cc, Q.cn, zb, w.bx,
                                                         w.by, w.bz, P, Lv);
        if (part) {
            const double s = block_sum_f64(acc, red);
            if (threadIdx.x == 0 && threadIdx.y == 0) part[w.slot] = s;
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
            if (threadIdx.x == 0 && threadIdx.y == 0 && threadIdx.z == 0) part[w.slot] = s;
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------
bool plain_tile_ok(Tile t) {
    const long long n = (long long)t.tx * t.ty * t.tz;
    return t.tx >= 1 && t.ty >= 1 && t.tz >= 1 && n % 64 == 0 && n <= 1024;
}

// HEAT2D5 PLAIN tiles: (tx, ty, 1) threads, one point each, one sweep per
// launch; or (OT, OT, k): fused sweeps, up to k per launch, with one region
// cell per thread when OT + 2k <= 32, else from a 16 x 16-thread LDS tile
// (OT = 16 or 32)
bool h2_cell_tile(Tile t) { return t.tx + 2 * t.tz <= 32; }

bool h2_tile_ok(int v, Tile t) {
    if (v != V_PLAIN) return false;
    if (t.tz == 1) return plain_tile_ok(t);
    return t.tx == t.ty && t.tx >= 1 && t.tz >= 2 && t.tz <= kFuseMax &&
           (h2_cell_tile(t) || t.tx == 16 || t.tx == 32);
}

long long h2_nblocks(int, Tile t, const Geom &g) { return cdiv(g.nx, t.tx) * cdiv(g.ny, t.ty); }

hipError_t h2_launch(int v, Tile t, const SweepArgs &a, hipStream_t s) {
    if (v != V_PLAIN) return hipErrorInvalidValue;
    if (t.tz > 1) {
        if (a.sweeps < 1 || a.sweeps > t.tz) return hipErrorInvalidValue;
        dim3 grid(cdiv(a.g.nx, t.tx), cdiv(a.g.ny, t.ty), 1), block(16, 16, 1);
        if (h2_cell_tile(t)) {
            const int L = t.tx + 2 * a.sweeps;  // <= 32
            hipLaunchKernelGGL(heat2d5_fused_cell, grid, dim3((L * L + 63) / 64 * 64), 0, s, (const double *)a.src,
                               (double *)a.dst, a.g, a.c[0], a.c[1], t.tx, a.sweeps, a.part);
        } else if (t.tx == 16)
            hipLaunchKernelGGL(heat2d5_fused<16>, grid, block, 0, s, (const double *)a.src, (double *)a.dst, a.g,
                               a.c[0], a.c[1], a.sweeps, a.part);
        else
            hipLaunchKernelGGL(heat2d5_fused<32>, grid, block, 0, s, (const double *)a.src, (double *)a.dst, a.g,
                               a.c[0], a.c[1], a.sweeps, a.part);
        return hipGetLastError();
    }
    dim3 grid(cdiv(a.g.nx, t.tx), cdiv(a.g.ny, t.ty), 1), block(t.tx, t.ty, 1);
    hipLaunchKernelGGL(heat2d5_plain, grid, block, 0, s, (const double *)a.src, (double *)a.dst, a.g, a.c[0],
                       a.c[1], a.part);
    return hipGetLastError();
}

// Saturated tiles offered: (TX, TY) with TX*TY a multiple of 64, <= 1024.
#define HEAT3D7_SAT_TILES(X) X(32, 2) X(32, 4) X(32, 8) X(32, 16) X(32, 20) X(32, 24) X(32, 28) X(64, 1) X(64, 2) X(64, 4) X(64, 8) X(128, 1) X(128, 2) \
    X(128, 4) X(256, 1) X(256, 2)

// Two-sweep tiles (block = TX x (TY + ring rows) <= 1024 threads); each is
// also a single-sweep tile (an odd sweep count starts with one single sweep).
// Tall 32-wide tiles recompute the fewest ring cells per tile cell (1.20x at
// 32 x 16, 1.14x at 32 x 28): 32 x 16 is the fastest at 160^3, 32 x 28 on
// HBM-resident grids (400^3, the largest classes of the 64-grid batch).
#define HEAT3D7_SAT2_TILES(X) X(32, 4) X(32, 8) X(32, 16) X(32, 20) X(32, 24) X(32, 28) X(64, 4) X(64, 8) \
    X(128, 4)

// Three-sweep regions (RX, RY): one thread per region column; the output
// tile is (RX - 4) x (RY - 4).  Two blocks of the 32 x 32 region fit a CU's
// LDS.
#define HEAT3D7_SAT3_REGIONS(X) X(32, 32) X(32, 24) X(32, 16) X(64, 16)

bool h3_tile_ok(int v, Tile t) {
    if (v == V_PLAIN) return plain_tile_ok(t);
    if (t.tz < 1) return false;
    if (v == V_SAT3) {
#define X(a, b) if (t.tx == a - 4 && t.ty == b - 4) return true;
        HEAT3D7_SAT3_REGIONS(X)
#undef X
        return false;
    }
    if (v == V_SAT2) {
#define X(a, b) if (t.tx == a && t.ty == b) return true;
        HEAT3D7_SAT2_TILES(X)
#undef X
        return false;
    }
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

int h3_sat2_tiles(Tile *out, int max) {
    int n = 0;
#define X(a, b) if (n < max) out[n++] = Tile{a, b, 0};
    HEAT3D7_SAT2_TILES(X)
#undef X
    return n;
}

int h3_sat3_tiles(Tile *out, int max) {
    int n = 0;
#define X(a, b) if (n < max) out[n++] = Tile{a - 4, b - 4, 0};
    HEAT3D7_SAT3_REGIONS(X)
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
    if (v == V_SAT3) {
        if (a.sweeps < 1 || a.sweeps > 3) return hipErrorInvalidValue;
#define X(A, B)                                                                                                \
    if (t.tx == A - 4 && t.ty == B - 4) {                                                                      \
        if (a.sweeps == 3)                                                                                     \
            hipLaunchKernelGGL((heat3d7_sat3<A, B, 3>), grid, dim3(A, B, 1), 0, s, src, dst, a.g, a.c[0], a.c[1], \
                               t.tz, a.remap, a.part);                                                         \
        else if (a.sweeps == 2)                                                                                \
            hipLaunchKernelGGL((heat3d7_sat3<A, B, 2>), grid, dim3(A, B, 1), 0, s, src, dst, a.g, a.c[0], a.c[1], \
                               t.tz, a.remap, a.part);                                                         \
        else                                                                                                   \
            hipLaunchKernelGGL((heat3d7_sat3<A, B, 1>), grid, dim3(A, B, 1), 0, s, src, dst, a.g, a.c[0], a.c[1], \
                               t.tz, a.remap, a.part);                                                         \
        return hipGetLastError();                                                                              \
    }
        HEAT3D7_SAT3_REGIONS(X)
#undef X
        return hipErrorInvalidValue;
    }
    if (v == V_SAT2) {
#define X(A, B)                                                                                              \
    if (t.tx == A && t.ty == B) {                                                                            \
        hipLaunchKernelGGL((heat3d7_sat2<A, B>), grid, dim3(A, B + H3Sat2Shape<A, B>::EY, 1), 0, s, src, dst, a.g, \
                           a.c[0], a.c[1], t.tz, a.remap, a.part);                                            \
        return hipGetLastError();                                                                            \
    }
        HEAT3D7_SAT2_TILES(X)
#undef X
        return hipErrorInvalidValue;
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
                           int grid, int sweeps, double *part, hipStream_t s) {
    if (v == V_SAT3) {
        if (sweeps < 1 || sweeps > 3) return hipErrorInvalidValue;
#define X(A, B)                                                                                                 \
    if (t.tx == A - 4 && t.ty == B - 4) {                                                                       \
        if (sweeps == 3)                                                                                        \
            hipLaunchKernelGGL((heat3d7_sat3_batch<A, B, 3>), dim3(grid), dim3(A, B, 1), 0, s, probs, items,    \
                               n_items, parity, t.tz, part);                                                    \
        else if (sweeps == 2)                                                                                   \
            hipLaunchKernelGGL((heat3d7_sat3_batch<A, B, 2>), dim3(grid), dim3(A, B, 1), 0, s, probs, items,    \
                               n_items, parity, t.tz, part);                                                    \
        else                                                                                                    \
            hipLaunchKernelGGL((heat3d7_sat3_batch<A, B, 1>), dim3(grid), dim3(A, B, 1), 0, s, probs, items,    \
                               n_items, parity, t.tz, part);                                                    \
        return hipGetLastError();                                                                               \
    }
        HEAT3D7_SAT3_REGIONS(X)
#undef X
        return hipErrorInvalidValue;
    }
    if (v == V_PLAIN) {
        hipLaunchKernelGGL(heat3d7_plain_batch, dim3(grid), dim3(t.tx, t.ty, t.tz), 0, s, probs, items, n_items, parity,
                           part);
        return hipGetLastError();
    }
    if (v == V_SAT2) {
#define X(A, B)                                                                                                 \
    if (t.tx == A && t.ty == B) {                                                                               \
        hipLaunchKernelGGL((heat3d7_sat2_batch<A, B>), dim3(grid), dim3(A, B + H3Sat2Shape<A, B>::EY, 1), 0, s, probs, \
                           items, n_items, parity, t.tz, part);                                                  \
        return hipGetLastError();                                                                               \
    }
        HEAT3D7_SAT2_TILES(X)
#undef X
        return hipErrorInvalidValue;
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
KindOps heat3d7_ops = {h3_tile_ok, h3_sat_tiles, h3_sat2_tiles, h3_nblocks, h3_launch, h3_batch_launch, h3_sat3_tiles};

}  // namespace stn
