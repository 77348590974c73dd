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
// ring loaded five planes ahead, together with the queue heads, and held in
// registers), and every load for the next plane (queue head, ring, u_prev,
// vsq) is issued before the current plane is computed ("bulk load"), into
// staging registers first read one iteration later.
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

// Software pipeline: the loads of iteration k (queue head zc+5, u^{n-1} and
// vsq of zc+1, ring of zc+5) go into one of two staging sets, chosen by the
// parity of k - k0, and are first read -- used or moved -- at iteration k+1.
// The z loop is unrolled by two so that the parity is a compile-time
// constant; a single staging register moved into the queue at the end of its
// own iteration would make every iteration wait for the loads it issued.
// Every load is unconditional, so that no register is merged with an older
// value: a lane outside the padded array reads a clamped cell of its row, and
// a load for a plane past the block's range reads the current plane instead;
// neither value is ever used (an interior point reads only cells of the padded
// array).  Addresses: a wave-uniform pointer per plane stream, advanced one
// plane per iteration, plus a per-thread 32-bit byte offset within the plane
// (planes below 4 GiB, checked on the host), all loads and stores through
// scalar buffer resources.
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
    const int PX = g.nx + 2 * R, PY = g.ny + 2 * R;
    const int k0 = bz * zb, k1 = min(k0 + zb, g.nz);

    bool in[RY];
    unsigned colb[RY];  // byte offset of row m's column within a plane (clamped into the array)
    int me[RY];
#pragma unroll
    for (int m = 0; m < RY; ++m) {
        const int yp = min(jb + m + R, PY - 1), xp = min(i + R, PX - 1);
        in[m] = i < g.nx && jb + m < g.ny;
        colb[m] = (unsigned)(((long long)yp * g.py + xp) * (long long)sizeof(double));
        me[m] = (ty * RY + m + R) * W + (tx + R);
    }
    HaloStager<double, TX, TY, R, false, NT> halo;
    halo.init(tid, bx * TX + R, by * TY + R, g.py, PX, PY);
    constexpr int HR = decltype(halo)::HR;
    unsigned hb[HR];  // byte offsets of this thread's ring cells (cells outside the array: offset 0)
#pragma unroll
    for (int h = 0; h < HR; ++h) hb[h] = halo.ok[h] ? (unsigned)(halo.goff[h] * (long long)sizeof(double)) : 0u;
    const long long pzb = g.pz * (long long)sizeof(double);
    auto at = [](const void *plane, unsigned off) -> double { return buf_ld_f64(plane_rsrc(plane), off); };

    // Iteration k computes padded plane zc = k + 4.  q[m][s]: u^n of row m's
    // column at plane zc-4+s (s < 8); hd[P][m]: the queue head loaded at the
    // last iteration of parity P; uq / vq: u^{n-1} and vsq likewise; hq[s]:
    // this thread's ring cells of plane zc+s (s < 4), rg: the staged rings.
    // At iteration k of parity P the staging sets 1-P hold plane zc+4 (head,
    // ring) and plane zc (u^{n-1}, vsq), loaded at iteration k-1.
    double q[RY][8], hd[2][RY], uq[2][RY], vq[2][RY], hq[4][HR], rg[2][HR];
    const char *base = (const char *)cur + (long long)k0 * pzb;
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int m = 0; m < RY; ++m) q[m][s] = at(base + s * pzb, colb[m]);
#pragma unroll
    for (int m = 0; m < RY; ++m) {
        hd[1][m] = at(base + 2 * R * pzb, colb[m]);
        uq[1][m] = at((const char *)pn + (long long)(k0 + R) * pzb, colb[m]);
        vq[1][m] = at((const char *)vsq + (long long)(k0 + R) * pzb, colb[m]);
        hd[0][m] = uq[0][m] = vq[0][m] = 0.0;
    }
    // The ring cells of plane zc are loaded with the queue heads of plane zc,
    // when the neighbouring blocks load the same cells as their own queue
    // heads, so the ring is mostly served from L2.  Planes k0+4 .. k0+8 lie
    // inside the array.
#pragma unroll
    for (int h = 0; h < HR; ++h) {
#pragma unroll
        for (int s = 0; s < 4; ++s) hq[s][h] = at(base + (R + s) * pzb, hb[h]);
        rg[1][h] = at(base + 2 * R * pzb, hb[h]);
        rg[0][h] = 0.0;
    }
    double acc = 0.0;

    // plane zc of u^n, of u^{n-1} (overwritten by u^{n+1}) and of vsq
    const char *p_cur = (const char *)cur + (long long)(k0 + R) * pzb;
    char *p_out = (char *)pn + (long long)(k0 + R) * pzb;
    const char *p_vsq = (const char *)vsq + (long long)(k0 + R) * pzb;
    auto step = [&](const int k, const int P) {
        const int Q = 1 - P;
        double *t = tile[P];
#pragma unroll
        for (int m = 0; m < RY; ++m) t[me[m]] = q[m][4];
#pragma unroll
        for (int h = 0; h < HR; ++h)
            if (halo.has[h]) t[halo.lidx[h]] = hq[0][h];
        // bulk load into staging set P: head and ring of zc+5, u^{n-1} and vsq of zc+1
        {
            const long long o5 = k + 1 < k1 ? (R + 1) * pzb : 0;
            const long long r5 = k + R + 1 < k1 ? (R + 1) * pzb : 0;
            const long long o1 = k + 1 < k1 ? pzb : 0;
#pragma unroll
            for (int m = 0; m < RY; ++m) {
                hd[P][m] = at(p_cur + o5, colb[m]);
                uq[P][m] = at(p_out + o1, colb[m]);
                vq[P][m] = at(p_vsq + o1, colb[m]);
            }
#pragma unroll
            for (int h = 0; h < HR; ++h) rg[P][h] = at(p_cur + r5, hb[h]);
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
                const double uc = q[m][4];
                const double s1 = ((t[e - 1] + t[e + 1]) + (yv(m, -1) + yv(m, 1))) + (q[m][3] + q[m][5]);
                const double s2 = ((t[e - 2] + t[e + 2]) + (yv(m, -2) + yv(m, 2))) + (q[m][2] + q[m][6]);
                const double s3 = ((t[e - 3] + t[e + 3]) + (yv(m, -3) + yv(m, 3))) + (q[m][1] + q[m][7]);
                const double s4 = ((t[e - 4] + t[e + 4]) + (yv(m, -4) + yv(m, 4))) + (q[m][0] + hd[Q][m]);
                double L = c.c0x3 * uc;
                L = fma(c.c1, s1, L);
                L = fma(c.c2, s2, L);
                L = fma(c.c3, s3, L);
                L = fma(c.c4, s4, L);
                const double nv = fma(vq[Q][m], L, 2.0 * uc - uq[Q][m]);
                buf_st_f64(plane_rsrc(p_out), colb[m], nv);
                const double d = nv - uc;
                acc = fma(d, d, acc);
            }
        }
        // advance: the queue takes the head of plane zc+4, the ring that of zc+4
#pragma unroll
        for (int m = 0; m < RY; ++m) {
#pragma unroll
            for (int s = 0; s < 7; ++s) q[m][s] = q[m][s + 1];
            q[m][7] = hd[Q][m];
        }
#pragma unroll
        for (int h = 0; h < HR; ++h) {
#pragma unroll
            for (int s = 0; s < 3; ++s) hq[s][h] = hq[s + 1][h];
            hq[3][h] = rg[Q][h];
        }
        p_cur += pzb;
        p_out += pzb;
        p_vsq += pzb;
    };
    for (int k = k0;; k += 2) {
        if (k >= k1) break;
        step(k, 0);
        if (k + 1 >= k1) break;
        step(k + 1, 1);
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
