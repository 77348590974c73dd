// wave25.hip -- radius-4 25-point star, second order in time (leapfrog), FP64.
//
//   L(u)   = sum over axes x, y, z of [c0*u + sum_{q=1..4} c_q*(u(+q) + u(-q))]
//   u_next = 2u - u_prev + vsq*L(u)
//
// The newer level u^n is read-only; u_next overwrites u_prev in place (a
// point's update reads u_prev only at that point, so this is race-free).
// 32 algorithmic bytes per point: read u^n, u^{n-1}, vsq, write u^{n+1}.
//
// PLAIN: one thread per point, 27 products in one left-to-right chain (axis
// x, then y, then z; per axis c0*u, then q = 1..4 with +q before -q), no
// contraction -- the loop body as written.
//
// SATURATED: the paper's rewrites by hand.  Constant folding merges the three
// centre products into (3*c0)*u; COMM/ASSOC group the six taps at distance q
// so each shared coefficient multiplies once; FMA1 chains the four radii and
// the time update:  L = fma(c4,S4, fma(c3,S3, fma(c2,S2, fma(c1,S1, (3c0)*u)))),
// u_next = fma(vsq, L, 2u - u_prev).  Loads: a block owns a TX x TY column
// tile (BY thread rows, RY rows per thread) and streams z; each column keeps
// the nine planes z-4..z+4 in a register queue (one global load per point),
// the in-plane +-4 neighbours come from an LDS tile with a 4-cell ring (the
// ring loaded four planes ahead, together with the queue heads, and held in
// registers), and every load for the next plane (queue head, ring, u_prev,
// vsq) is issued before the current plane is computed ("bulk load").
#include "internal.hpp"

namespace stn {
namespace {

constexpr int kMaxWaves = 16;

struct W25C {
    double c0, c1, c2, c3, c4, c0x3;
};

__global__ void wave25_plain(const double *__restrict__ cur, double *__restrict__ pn, const double *__restrict__ vsq,
                             Geom g, W25C c, double *__restrict__ part) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    double d2 = 0.0;
    if (i < g.nx && j < g.ny && k < g.nz) {
        const long long q = (long long)(k + 4) * g.pz + (long long)(j + 4) * g.py + (i + 4);
        const long long X = 1, Y = g.py, Z = g.pz;
        const double u = cur[q];
        double L = c.c0 * u;
        L = L + c.c1 * cur[q + X];
        L = L + c.c1 * cur[q - X];
        L = L + c.c2 * cur[q + 2 * X];
        L = L + c.c2 * cur[q - 2 * X];
        L = L + c.c3 * cur[q + 3 * X];
        L = L + c.c3 * cur[q - 3 * X];
        L = L + c.c4 * cur[q + 4 * X];
        L = L + c.c4 * cur[q - 4 * X];
        L = L + c.c0 * u;
        L = L + c.c1 * cur[q + Y];
        L = L + c.c1 * cur[q - Y];
        L = L + c.c2 * cur[q + 2 * Y];
        L = L + c.c2 * cur[q - 2 * Y];
        L = L + c.c3 * cur[q + 3 * Y];
        L = L + c.c3 * cur[q - 3 * Y];
        L = L + c.c4 * cur[q + 4 * Y];
        L = L + c.c4 * cur[q - 4 * Y];
        L = L + c.c0 * u;
        L = L + c.c1 * cur[q + Z];
        L = L + c.c1 * cur[q - Z];
        L = L + c.c2 * cur[q + 2 * Z];
        L = L + c.c2 * cur[q - 2 * Z];
        L = L + c.c3 * cur[q + 3 * Z];
        L = L + c.c3 * cur[q - 3 * Z];
        L = L + c.c4 * cur[q + 4 * Z];
        L = L + c.c4 * cur[q - 4 * Z];
        const double nv = (2.0 * u - pn[q]) + vsq[q] * L;
        pn[q] = nv;
        const double d = nv - u;
        d2 = d * d;
    }
    if (part) {
        __shared__ double lds[kMaxWaves];
        const double s = block_sum_f64(d2, lds);
        if (threadIdx.x == 0 && threadIdx.y == 0 && threadIdx.z == 0) part[block_linear_id()] = s;
    }
}

// Per-point forms of the paper's ablation (Sec. Evaluation: CSE, CSE+SAT,
// CSE+BULK, ACCSAT), one thread per point with every operand from memory.
// The plain body already loads each address once, so CSE is the plain form.
//   FORM_SAT  : the rewritten arithmetic of the saturated form (3*c0 folded,
//               taps grouped by radius, FMA chain), loads where first used;
//   FORM_BULK : every load first, in ascending address order (previous level
//               and vsq, then z-4 .. z+4 of u^n with each plane's taps by
//               address), then the plain arithmetic order;
//   FORM_BOTH : the loads of FORM_BULK, then the arithmetic of FORM_SAT.
enum { FORM_SAT = 0, FORM_BULK = 1, FORM_BOTH = 2 };

template <int FORM>
__global__ void wave25_point(const double *__restrict__ cur, double *__restrict__ pn, const double *__restrict__ vsq,
                             Geom g, W25C c, double *__restrict__ part) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    double d2 = 0.0;
    if (i < g.nx && j < g.ny && k < g.nz) {
        const long long q = (long long)(k + 4) * g.pz + (long long)(j + 4) * g.py + (i + 4);
        const long long Y = g.py, Z = g.pz;
        double nv, u;
        if (FORM == FORM_SAT) {
            u = cur[q];
            const double s1 = ((cur[q - 1] + cur[q + 1]) + (cur[q - Y] + cur[q + Y])) + (cur[q - Z] + cur[q + Z]);
            const double s2 = ((cur[q - 2] + cur[q + 2]) + (cur[q - 2 * Y] + cur[q + 2 * Y])) +
                              (cur[q - 2 * Z] + cur[q + 2 * Z]);
            const double s3 = ((cur[q - 3] + cur[q + 3]) + (cur[q - 3 * Y] + cur[q + 3 * Y])) +
                              (cur[q - 3 * Z] + cur[q + 3 * Z]);
            const double s4 = ((cur[q - 4] + cur[q + 4]) + (cur[q - 4 * Y] + cur[q + 4 * Y])) +
                              (cur[q - 4 * Z] + cur[q + 4 * Z]);
            double L = c.c0x3 * u;
            L = fma(c.c1, s1, L);
            L = fma(c.c2, s2, L);
            L = fma(c.c3, s3, L);
            L = fma(c.c4, s4, L);
            nv = fma(vsq[q], L, 2.0 * u - pn[q]);
        } else {
            // bulk load in ascending address order
            const double up = pn[q], vv = vsq[q];
            double zm[4], ym[4], xm[4], xp[4], yp[4], zp[4];
#pragma unroll
            for (int r = 4; r >= 1; --r) zm[r - 1] = cur[q - r * Z];
#pragma unroll
            for (int r = 4; r >= 1; --r) ym[r - 1] = cur[q - r * Y];
#pragma unroll
            for (int r = 4; r >= 1; --r) xm[r - 1] = cur[q - r];
            u = cur[q];
#pragma unroll
            for (int r = 1; r <= 4; ++r) xp[r - 1] = cur[q + r];
#pragma unroll
            for (int r = 1; r <= 4; ++r) yp[r - 1] = cur[q + r * Y];
#pragma unroll
            for (int r = 1; r <= 4; ++r) zp[r - 1] = cur[q + r * Z];
            const double cr[5] = {c.c0, c.c1, c.c2, c.c3, c.c4};
            if (FORM == FORM_BULK) {  // the plain arithmetic order
                double L = c.c0 * u;
#pragma unroll
                for (int r = 1; r <= 4; ++r) {
                    L = L + cr[r] * xp[r - 1];
                    L = L + cr[r] * xm[r - 1];
                }
                L = L + c.c0 * u;
#pragma unroll
                for (int r = 1; r <= 4; ++r) {
                    L = L + cr[r] * yp[r - 1];
                    L = L + cr[r] * ym[r - 1];
                }
                L = L + c.c0 * u;
#pragma unroll
                for (int r = 1; r <= 4; ++r) {
                    L = L + cr[r] * zp[r - 1];
                    L = L + cr[r] * zm[r - 1];
                }
                nv = (2.0 * u - up) + vv * L;
            } else {  // the saturated arithmetic
                double L = c.c0x3 * u;
#pragma unroll
                for (int r = 1; r <= 4; ++r) {
                    const double sr = ((xm[r - 1] + xp[r - 1]) + (ym[r - 1] + yp[r - 1])) + (zm[r - 1] + zp[r - 1]);
                    L = fma(cr[r], sr, L);
                }
                nv = fma(vv, L, 2.0 * u - up);
            }
        }
        pn[q] = nv;
        const double d = nv - u;
        d2 = d * d;
    }
    if (part) {
        __shared__ double lds[kMaxWaves];
        const double s = block_sum_f64(d2, lds);
        if (threadIdx.x == 0 && threadIdx.y == 0 && threadIdx.z == 0) part[block_linear_id()] = s;
    }
}

template <int TX, int BY, int RY>
__global__ __launch_bounds__(TX *BY) void wave25_sat(const double *__restrict__ cur, double *__restrict__ pn,
                                                     const double *__restrict__ vsq, Geom g, W25C c, int zb,
                                                     int remap, double *__restrict__ part) {
    constexpr int R = 4, TY = BY * RY, W = TX + 2 * R, NT = TX * BY, PLANE = (TY + 2 * R) * W;
    __shared__ double tile[2][PLANE];
    __shared__ double red[kMaxWaves];
    int bx, by, bz;
    tile_coords(remap, bx, by, bz);
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
    const int i = bx * TX + tx, jb = by * TY + ty * RY;
    const int xp = i + R;
    const int PX = g.nx + 2 * R, PY = g.ny + 2 * R, PZ = g.nz + 2 * R;
    const int k0 = bz * zb, k1 = min(k0 + zb, g.nz);

    bool in[RY], ld[RY];
    long long col[RY];
    int me[RY];
#pragma unroll
    for (int m = 0; m < RY; ++m) {
        const int yp = jb + m + R;
        in[m] = i < g.nx && jb + m < g.ny;
        ld[m] = xp < PX && yp < PY;
        col[m] = (long long)yp * g.py + xp;
        me[m] = (ty * RY + m + R) * W + (tx + R);
    }
    HaloStager<double, TX, TY, R, false, NT> halo;
    halo.init(tid, bx * TX + R, by * TY + R, g.py, PX, PY);

    // q[m][s] = u^n at padded z = zc - 4 + s, zc = k + 4 the plane computed
    double q[RY][9], up[RY], vv[RY];
#pragma unroll
    for (int m = 0; m < RY; ++m) {
#pragma unroll
        for (int s = 0; s < 9; ++s) q[m][s] = ld[m] ? cur[col[m] + (long long)(k0 + s) * g.pz] : 0.0;
        const long long o = col[m] + (long long)(k0 + R) * g.pz;
        up[m] = in[m] ? pn[o] : 0.0;
        vv[m] = in[m] ? vsq[o] : 0.0;
    }
    // The ring cells of plane zc are loaded with the queue heads of plane
    // zc (four planes before the plane is computed), when the neighbouring
    // blocks load the same cells as their own queue heads, so the ring is
    // mostly served from L2; hq[s] holds the ring of plane zc + s.
    constexpr int HR = decltype(halo)::HR;
    double hq[R + 1][HR];
#pragma unroll
    for (int s = 0; s <= R; ++s) {
        halo.load(cur + (long long)(k0 + R + s) * g.pz);
#pragma unroll
        for (int h = 0; h < HR; ++h) hq[s][h] = halo.val[h];
    }
    double acc = 0.0;

    for (int k = k0; k < k1; ++k) {
        const int zc = k + R, b = (k - k0) & 1;
        double *t = tile[b];
#pragma unroll
        for (int m = 0; m < RY; ++m) t[me[m]] = q[m][4];
#pragma unroll
        for (int h = 0; h < HR; ++h) halo.val[h] = hq[0][h];
        halo.store(t);
        double upc[RY], vvc[RY], qn[RY];
#pragma unroll
        for (int m = 0; m < RY; ++m) {
            upc[m] = up[m];
            vvc[m] = vv[m];
            qn[m] = 0.0;
        }
        if (k + 1 < k1) {  // bulk load of plane zc+1 (queue head zc+5)
#pragma unroll
            for (int m = 0; m < RY; ++m) qn[m] = (ld[m] && zc + 5 < PZ) ? cur[col[m] + (long long)(zc + 5) * g.pz] : 0.0;
#pragma unroll
            for (int s = 0; s < R; ++s)
#pragma unroll
                for (int h = 0; h < HR; ++h) hq[s][h] = hq[s + 1][h];
            if (k + R + 1 < k1) {  // the ring of plane zc+5, computed at iteration k+5
                halo.load(cur + (long long)(zc + R + 1) * g.pz);
#pragma unroll
                for (int h = 0; h < HR; ++h) hq[R][h] = halo.val[h];
            }
#pragma unroll
            for (int m = 0; m < RY; ++m) {
                const long long o = col[m] + (long long)(zc + 1) * g.pz;
                up[m] = in[m] ? pn[o] : 0.0;
                vv[m] = in[m] ? vsq[o] : 0.0;
            }
        }
        __syncthreads();
        // y neighbours that are rows of this same thread come from its own
        // registers (the value in the LDS tile is the same number)
        auto yv = [&](int m, int d) -> double {
            const int mm = m + d;
            return (mm >= 0 && mm < RY) ? q[mm >= 0 && mm < RY ? mm : 0][4] : t[me[m] + d * W];
        };
#pragma unroll
        for (int m = 0; m < RY; ++m) {
            if (in[m]) {
                const int e = me[m];
                const double u = q[m][4];
                const double s1 = ((t[e - 1] + t[e + 1]) + (yv(m, -1) + yv(m, 1))) + (q[m][3] + q[m][5]);
                const double s2 = ((t[e - 2] + t[e + 2]) + (yv(m, -2) + yv(m, 2))) + (q[m][2] + q[m][6]);
                const double s3 = ((t[e - 3] + t[e + 3]) + (yv(m, -3) + yv(m, 3))) + (q[m][1] + q[m][7]);
                const double s4 = ((t[e - 4] + t[e + 4]) + (yv(m, -4) + yv(m, 4))) + (q[m][0] + q[m][8]);
                double L = c.c0x3 * u;
                L = fma(c.c1, s1, L);
                L = fma(c.c2, s2, L);
                L = fma(c.c3, s3, L);
                L = fma(c.c4, s4, L);
                const double nv = fma(vvc[m], L, 2.0 * u - upc[m]);
                pn[col[m] + (long long)zc * g.pz] = nv;
                const double d = nv - u;
                acc = fma(d, d, acc);
            }
        }
#pragma unroll
        for (int m = 0; m < RY; ++m) {
#pragma unroll
            for (int s = 0; s < 8; ++s) q[m][s] = q[m][s + 1];
            q[m][8] = qn[m];
        }
    }
    if (part) {
        const double s = block_sum_f64(acc, red);
        if (tid == 0) part[block_linear_id()] = s;
    }
}

bool plain_tile_ok(Tile t) {
    const long long n = (long long)t.tx * t.ty * t.tz;
    return t.tx >= 1 && t.ty >= 1 && t.tz >= 1 && n % 64 == 0 && n <= 1024;
}

// Saturated tiles: (TX, tile rows) -> (TX, BY thread rows, RY rows per thread)
// Taller tiles cut the share of y-halo rows (8 per tile): 64 x 32 and 256 x 8
// run ~6 % faster than 128 x 8 on a 512^3 grid; 1024-thread tiles with four
// rows per thread spill and are not offered.
#define W25_SAT_TILES(X) X(64, 4, 4, 1) X(64, 8, 4, 2) X(64, 16, 4, 4) X(64, 32, 8, 4) X(32, 8, 8, 1) \
    X(32, 16, 8, 2) X(128, 4, 4, 1) X(128, 8, 4, 2) X(128, 16, 8, 2) X(256, 4, 4, 1) X(256, 8, 4, 2)

bool w25_tile_ok(int v, Tile t) {
    if (v == V_PLAIN || is_point_form(v)) return plain_tile_ok(t);
    if (t.tz < 1) return false;
#define X(A_, TY_, BY_, RY_) if (t.tx == A_ && t.ty == TY_) return true;
    W25_SAT_TILES(X)
#undef X
    return false;
}

int w25_sat_tiles(Tile *out, int max) {
    int n = 0;
#define X(A_, TY_, BY_, RY_) if (n < max) out[n++] = Tile{A_, TY_, 0};
    W25_SAT_TILES(X)
#undef X
    return n;
}

long long w25_nblocks(int, Tile t, const Geom &g) { return cdiv(g.nx, t.tx) * cdiv(g.ny, t.ty) * cdiv(g.nz, t.tz); }

hipError_t w25_launch(int v, Tile t, const SweepArgs &a, hipStream_t s) {
    const double *cur = (const double *)a.src;
    double *pn = (double *)a.dst;
    const double *vsq = (const double *)a.coefs[0];
    W25C c{a.c[0], a.c[1], a.c[2], a.c[3], a.c[4], 3.0 * a.c[0]};
    dim3 grid(cdiv(a.g.nx, t.tx), cdiv(a.g.ny, t.ty), cdiv(a.g.nz, t.tz));
    if (v == V_PLAIN) {
        hipLaunchKernelGGL(wave25_plain, grid, dim3(t.tx, t.ty, t.tz), 0, s, cur, pn, vsq, a.g, c, a.part);
        return hipGetLastError();
    }
    if (is_point_form(v)) {
        const dim3 blk(t.tx, t.ty, t.tz);
        if (v == V_CSE_SAT) hipLaunchKernelGGL(wave25_point<FORM_SAT>, grid, blk, 0, s, cur, pn, vsq, a.g, c, a.part);
        else if (v == V_CSE_BULK) hipLaunchKernelGGL(wave25_point<FORM_BULK>, grid, blk, 0, s, cur, pn, vsq, a.g, c, a.part);
        else hipLaunchKernelGGL(wave25_point<FORM_BOTH>, grid, blk, 0, s, cur, pn, vsq, a.g, c, a.part);
        return hipGetLastError();
    }
#define X(A, TY, BY, RY)                                                                                   \
    if (t.tx == A && t.ty == TY) {                                                                         \
        hipLaunchKernelGGL((wave25_sat<A, BY, RY>), grid, dim3(A, BY, 1), 0, s, cur, pn, vsq, a.g, c, t.tz, \
                           a.remap, a.part);                                                               \
        return hipGetLastError();                                                                          \
    }
    W25_SAT_TILES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace

KindOps wave25_ops = {w25_tile_ok, w25_sat_tiles, nullptr, w25_nblocks, w25_launch, nullptr};

}  // namespace stn
