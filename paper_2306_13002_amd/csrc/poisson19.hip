// poisson19.hip -- 19-point variable-coefficient pressure relaxation.
//
// F32 storage, FP64 arithmetic: every operand is widened on load and the new
// p is rounded to F32 on store; the residual sum ss^2 is FP64.  (i,j,k) =
// (x,y,z) and every coefficient array is read at the point itself:
//
//   s0 = a0*p(i+1,j,k) + a1*p(i,j+1,k) + a2*p(i,j,k+1)
//      + b0*(p(i+1,j+1,k) - p(i+1,j-1,k) - p(i-1,j+1,k) + p(i-1,j-1,k))
//      + b1*(p(i,j+1,k+1) - p(i,j-1,k+1) - p(i,j+1,k-1) + p(i,j-1,k-1))
//      + b2*(p(i+1,j,k+1) - p(i-1,j,k+1) - p(i+1,j,k-1) + p(i-1,j,k-1))
//      + c0*p(i-1,j,k) + c1*p(i,j-1,k) + c2*p(i,j,k-1) + wrk1
//   ss = (s0*a3 - p)*bnd ;  p' = p + omega*ss ;  residual += ss^2
//
// This is the memory-bound halo-3D CFD loop-nest class of the paper's
// benchmark tables (NPB BT/LU/SP, SPEC csp/bt): 12 coefficient streams, one
// state stream read and one written, 56 algorithmic bytes per point.
//
// PLAIN: one thread per point, 19 + 12 loads, terms in the order above,
// products rounded and added left to right (no contraction): bit-identical
// to a plain FP64 loop nest that rounds stored p to F32.
//
// SATURATED: the cross terms are rewritten with COMM/ASSOC into differences
// of differences, e.g. b1*(D(k+1) - D(k-1)) with D(k') = p(i,j+1,k') -
// p(i,j-1,k') (a difference of two widened F32 values is exact in FP64),
// and the whole s0 becomes one FMA chain (FMA1/FMA3).  Each block streams a
// TX x TY column tile along z: the p planes k-1, k, k+1 sit in a four-deep
// LDS ring (one barrier per plane), and every global load of the next plane
// -- its p tile and the 12 coefficients -- is issued before the current
// plane is computed ("bulk load"), so each wave keeps ~13 loads in flight.
#include "internal.hpp"

namespace stn {
namespace {

constexpr int kMaxWaves = 16;

// a0 a1 a2 a3 b0 b1 b2 c0 c1 c2 bnd wrk1
enum { A0, A1, A2, A3, B0, B1, B2, C0, C1, C2, BND, WRK1 };
struct P19Coef {
    const float *f[12];
};

P19Coef pack(const SweepArgs &a) {
    P19Coef c;
    for (int i = 0; i < 12; ++i) c.f[i] = (const float *)a.coefs[i];
    return c;
}

__global__ void poisson19_plain(const float *__restrict__ p, float *__restrict__ pn, P19Coef c, Geom g,
                                double omega, double *__restrict__ part) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    double d2 = 0.0;
    if (i < g.nx && j < g.ny && k < g.nz) {
        const long long q = (long long)(k + 1) * g.pz + (long long)(j + 1) * g.py + (i + 1);
        const long long Y = g.py, Z = g.pz;
#define P(dx, dy, dz) ((double)p[q + (dx) + (dy)*Y + (dz)*Z])
        double s0 = (double)c.f[A0][q] * P(1, 0, 0);
        s0 = s0 + (double)c.f[A1][q] * P(0, 1, 0);
        s0 = s0 + (double)c.f[A2][q] * P(0, 0, 1);
        s0 = s0 + (double)c.f[B0][q] * (((P(1, 1, 0) - P(1, -1, 0)) - P(-1, 1, 0)) + P(-1, -1, 0));
        s0 = s0 + (double)c.f[B1][q] * (((P(0, 1, 1) - P(0, -1, 1)) - P(0, 1, -1)) + P(0, -1, -1));
        s0 = s0 + (double)c.f[B2][q] * (((P(1, 0, 1) - P(-1, 0, 1)) - P(1, 0, -1)) + P(-1, 0, -1));
        s0 = s0 + (double)c.f[C0][q] * P(-1, 0, 0);
        s0 = s0 + (double)c.f[C1][q] * P(0, -1, 0);
        s0 = s0 + (double)c.f[C2][q] * P(0, 0, -1);
        s0 = s0 + (double)c.f[WRK1][q];
        const double ss = (s0 * (double)c.f[A3][q] - P(0, 0, 0)) * (double)c.f[BND][q];
        pn[q] = (float)(P(0, 0, 0) + omega * ss);
#undef P
        d2 = ss * ss;
    }
    if (part) {
        __shared__ double lds[kMaxWaves];
        const double s = block_sum_f64(d2, lds);
        if (threadIdx.x == 0 && threadIdx.y == 0 && threadIdx.z == 0) part[block_linear_id()] = s;
    }
}

// Per-point forms of the paper's ablation (Sec. Evaluation), one thread per
// point with every operand from memory; CSE is the plain form (no address
// is loaded twice).  FORM_SAT: the saturated form's arithmetic (differences
// of differences, one FMA chain), loads where first used.  FORM_BULK: all 31
// loads first -- the 12 coefficients, then p in ascending address order --
// then the plain arithmetic order.  FORM_BOTH: those loads, then FORM_SAT's
// arithmetic.  FORM_SAT and FORM_BOTH compute exactly what the z-streaming
// saturated kernel computes; FORM_BULK exactly what the plain kernel does.
enum { FORM_SAT = 0, FORM_BULK = 1, FORM_BOTH = 2 };

__device__ __forceinline__ double p19_sat_math(const double *cf, double pc, double pE, double pW, double pN,
                                               double pS, double pU, double pD, double pNE, double pSE, double pNW,
                                               double pSW, double uN, double uS, double mN, double mS, double uE,
                                               double uW, double mE, double mW, double omega, float *out) {
    const double B0v = (pNE - pSE) - (pNW - pSW);
    const double B1v = (uN - uS) - (mN - mS);
    const double B2v = (uE - uW) - (mE - mW);
    double s0 = fma(cf[B0], B0v, cf[WRK1]);
    s0 = fma(cf[B1], B1v, s0);
    s0 = fma(cf[B2], B2v, s0);
    s0 = fma(cf[A0], pE, s0);
    s0 = fma(cf[C0], pW, s0);
    s0 = fma(cf[A1], pN, s0);
    s0 = fma(cf[C1], pS, s0);
    s0 = fma(cf[A2], pU, s0);
    s0 = fma(cf[C2], pD, s0);
    const double ss = fma(s0, cf[A3], -pc) * cf[BND];
    *out = (float)fma(omega, ss, pc);
    return ss;
}

template <int FORM>
__global__ void poisson19_point(const float *__restrict__ p, float *__restrict__ pn, P19Coef c, Geom g,
                                double omega, double *__restrict__ part) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    double d2 = 0.0;
    if (i < g.nx && j < g.ny && k < g.nz) {
        const long long q = (long long)(k + 1) * g.pz + (long long)(j + 1) * g.py + (i + 1);
        const long long Y = g.py, Z = g.pz;
        double ss;
        float out;
        if (FORM == FORM_SAT) {
            double cf[12];
#pragma unroll
            for (int a = 0; a < 12; ++a) cf[a] = c.f[a][q];
#define P(o) ((double)p[q + (o)])
            ss = p19_sat_math(cf, P(0), P(1), P(-1), P(Y), P(-Y), P(Z), P(-Z), P(Y + 1), P(-Y + 1), P(Y - 1), P(-Y - 1),
                              P(Z + Y), P(Z - Y), P(-Z + Y), P(-Z - Y), P(Z + 1), P(Z - 1), P(-Z + 1), P(-Z - 1), omega,
                              &out);
#undef P
        } else {
            // bulk load: coefficients, then p in ascending address order
            double cf[12];
#pragma unroll
            for (int a = 0; a < 12; ++a) cf[a] = c.f[a][q];
            const long long off[19] = {-Z - Y, -Z - 1, -Z, -Z + 1, -Z + Y, -Y - 1, -Y, -Y + 1, -1, 0,
                                       1,      Y - 1,  Y,  Y + 1,  Z - Y,  Z - 1,  Z,  Z + 1,  Z + Y};
            double v[19];
#pragma unroll
            for (int t = 0; t < 19; ++t) v[t] = (double)p[q + off[t]];
            // names by offset
            const double mS = v[0], mW = v[1], pD = v[2], mE = v[3], mN = v[4], pSW = v[5], pS = v[6], pSE = v[7],
                         pW = v[8], pc = v[9], pE = v[10], pNW = v[11], pN = v[12], pNE = v[13], uS = v[14],
                         uW = v[15], pU = v[16], uE = v[17], uN = v[18];
            if (FORM == FORM_BULK) {  // the plain arithmetic order
                double s0 = cf[A0] * pE;
                s0 = s0 + cf[A1] * pN;
                s0 = s0 + cf[A2] * pU;
                s0 = s0 + cf[B0] * (((pNE - pSE) - pNW) + pSW);
                s0 = s0 + cf[B1] * (((uN - uS) - mN) + mS);
                s0 = s0 + cf[B2] * (((uE - uW) - mE) + mW);
                s0 = s0 + cf[C0] * pW;
                s0 = s0 + cf[C1] * pS;
                s0 = s0 + cf[C2] * pD;
                s0 = s0 + cf[WRK1];
                ss = (s0 * cf[A3] - pc) * cf[BND];
                out = (float)(pc + omega * ss);
            } else {
                ss = p19_sat_math(cf, pc, pE, pW, pN, pS, pU, pD, pNE, pSE, pNW, pSW, uN, uS, mN, mS, uE, uW, mE, mW,
                                  omega, &out);
            }
        }
        pn[q] = out;
        d2 = ss * ss;
    }
    if (part) {
        __shared__ double lds[kMaxWaves];
        const double s = block_sum_f64(d2, lds);
        if (threadIdx.x == 0 && threadIdx.y == 0 && threadIdx.z == 0) part[block_linear_id()] = s;
    }
}

// F32 access to one plane through a scalar buffer resource (plane_rsrc: the
// base in 4 SGPRs, a 32-bit byte offset per lane; planes below 4 GiB).
__device__ __forceinline__ float buf_ld_f32(__amdgpu_buffer_rsrc_t r, unsigned off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ void buf_st_f32(__amdgpu_buffer_rsrc_t r, unsigned off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}

template <int TX, int TY>
__global__ __launch_bounds__(TX *TY) void poisson19_sat(const float *__restrict__ p, float *__restrict__ pn,
                                                        P19Coef c, Geom g, double omega, int zb, int remap,
                                                        double *__restrict__ part) {
    constexpr int R = 1, W = TX + 2 * R, NT = TX * TY, PLANE = (TY + 2 * R) * W;
    __shared__ float ring[4][PLANE];
    __shared__ double red[kMaxWaves];
    int bx, by, bz;
    tile_coords(remap, bx, by, bz);
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
    const int i = bx * TX + tx, j = by * TY + ty;
    const int xp = i + R, yp = j + R;
    const int PX = g.nx + 2 * R, PY = g.ny + 2 * R;
    const bool in = i < g.nx && j < g.ny;
    const bool ld = xp < PX && yp < PY;
    const int k0 = bz * zb, k1 = min(k0 + zb, g.nz);
    const long long col = (long long)yp * g.py + xp;
    const int me = (ty + R) * W + (tx + R);

    HaloStager<float, TX, TY, R, true, NT> halo;
    halo.init(tid, bx * TX + R, by * TY + R, g.py, PX, PY);
    constexpr int HR = decltype(halo)::HR;

    // prologue: planes zc0-1 and zc0 (zc = k + 1) into ring slots 0 and 1
    // (plane z sits in slot (z - k0) mod 4)
    for (int z = k0; z <= k0 + 1; ++z) {
        const float *pl = p + (long long)z * g.pz;
        ring[z - k0][me] = ld ? pl[col] : 0.0f;
        halo.load(pl);
        halo.store(ring[z - k0]);
    }
    // From here every load is unconditional and goes through a scalar buffer
    // resource per plane with a 32-bit byte offset per lane (planes below
    // 4 GiB, checked on the host): a lane with nothing to load reads the cell
    // of its own column (clamped into the padded array), which the tile loads
    // anyway; a ring cell outside the array is staged as 0; a load for a plane
    // the block does not need re-reads the last one it did.  None of those
    // values is used.
    const long long pzb = g.pz * (long long)sizeof(float);
    const unsigned ob =
        (unsigned)(((long long)min(yp, PY - 1) * g.py + min(xp, PX - 1)) * (long long)sizeof(float));
    unsigned hb[HR];
#pragma unroll
    for (int h = 0; h < HR; ++h) hb[h] = halo.ok[h] ? (unsigned)(halo.goff[h] * (long long)sizeof(float)) : ob;
    auto ldb = [](const void *plane, unsigned off) -> float { return buf_ld_f32(plane_rsrc(plane), off); };
    // registers for the plane after: p(zc+1) tile and the coefficients at zc,
    // in two sets by the parity of k - k0: set P is loaded at step k (plane
    // zc+1) and read at step k+1, so no set is ever copied
    float ctr = ldb((const char *)p + (long long)(k0 + 2) * pzb, ob);
    float hv[HR];
#pragma unroll
    for (int h = 0; h < HR; ++h) hv[h] = ldb((const char *)p + (long long)(k0 + 2) * pzb, hb[h]);
    float cf[2][12];
#pragma unroll
    for (int s = 0; s < 12; ++s) {
        cf[0][s] = 0.0f;
        cf[1][s] = ldb((const char *)c.f[s] + (long long)(k0 + 1) * pzb, ob);
    }
    double acc = 0.0;
    // running byte offsets of p plane zc+2 and coefficient plane zc+1, clamped
    // to the last plane each stream needs
    long long o_p = (long long)(k0 + 3) * pzb, o_c = (long long)(k0 + 2) * pzb;
    const long long p_max = (long long)(k1 + 1) * pzb, c_max = (long long)k1 * pzb;
    char *out_pl = (char *)pn + (long long)(k0 + 1) * pzb;

    // step k: plane zc = k + 1; M, O, U are the slots of planes zc-1, zc,
    // zc+1 and P the coefficient set loaded at this step
    auto step = [&](const int P, const int M, const int O, const int U) {
        // stage plane zc+1
        ring[U][me] = ctr;
#pragma unroll
        for (int h = 0; h < HR; ++h)
            if (halo.has[h]) ring[U][halo.lidx[h]] = halo.ok[h] ? hv[h] : 0.0f;
        // bulk-issue every load of the next plane
        {
            const char *pl = (const char *)p + min(o_p, p_max);
            ctr = ldb(pl, ob);
#pragma unroll
            for (int h = 0; h < HR; ++h) hv[h] = ldb(pl, hb[h]);
            const long long oc = min(o_c, c_max);
#pragma unroll
            for (int s = 0; s < 12; ++s) cf[P][s] = ldb((const char *)c.f[s] + oc, ob);
        }
        const float *cc = cf[1 - P];
        __syncthreads();
        if (in) {
            const float *m = ring[M], *o = ring[O], *u = ring[U];
            const double pc = o[me];
            const double pE = o[me + 1], pW = o[me - 1], pN = o[me + W], pS = o[me - W];
            const double B0v = ((double)o[me + W + 1] - (double)o[me - W + 1]) -
                              ((double)o[me + W - 1] - (double)o[me - W - 1]);
            const double B1v = ((double)u[me + W] - (double)u[me - W]) - ((double)m[me + W] - (double)m[me - W]);
            const double B2v = ((double)u[me + 1] - (double)u[me - 1]) - ((double)m[me + 1] - (double)m[me - 1]);
            const double pU = u[me], pD = m[me];
            double s0 = fma((double)cc[B0], B0v, (double)cc[WRK1]);
            s0 = fma((double)cc[B1], B1v, s0);
            s0 = fma((double)cc[B2], B2v, s0);
            s0 = fma((double)cc[A0], pE, s0);
            s0 = fma((double)cc[C0], pW, s0);
            s0 = fma((double)cc[A1], pN, s0);
            s0 = fma((double)cc[C1], pS, s0);
            s0 = fma((double)cc[A2], pU, s0);
            s0 = fma((double)cc[C2], pD, s0);
            const double ss = fma(s0, (double)cc[A3], -pc) * (double)cc[BND];
            buf_st_f32(plane_rsrc(out_pl), ob, (float)fma(omega, ss, pc));
            acc = fma(ss, ss, acc);
        }
        o_p += pzb;
        o_c += pzb;
        out_pl += pzb;
    };
    // Four planes per trip, so that every ring slot and coefficient set is a
    // compile-time constant; the loop leaves between steps, so no step is
    // skipped inside a trip and no value merges there.
    for (int k = k0;; k += 4) {
        if (k >= k1) break;
        step(0, 0, 1, 2);
        if (k + 1 >= k1) break;
        step(1, 1, 2, 3);
        if (k + 2 >= k1) break;
        step(0, 2, 3, 0);
        if (k + 3 >= k1) break;
        step(1, 3, 0, 1);
    }
    if (part) {
        const double s = block_sum_f64(acc, red);
        if (tid == 0) part[block_linear_id()] = s;
    }
}

// The saturated update of one point from three staged planes (m, o, u =
// planes zc-1, zc, zc+1 of an LDS tile of row width W) and the point's 12
// coefficients; returns ss and the new value rounded to F32.  The same
// operations in the same order as poisson19_sat.
template <int W, typename L>
__device__ __forceinline__ double p19_update(const L *m, const L *o, const L *u, int e, const float *cc, double omega,
                                             float *out) {
    const double pc = o[e];
    const double pE = o[e + 1], pW = o[e - 1], pN = o[e + W], pS = o[e - W];
    const double B0v = ((double)o[e + W + 1] - (double)o[e - W + 1]) - ((double)o[e + W - 1] - (double)o[e - W - 1]);
    const double B1v = ((double)u[e + W] - (double)u[e - W]) - ((double)m[e + W] - (double)m[e - W]);
    const double B2v = ((double)u[e + 1] - (double)u[e - 1]) - ((double)m[e + 1] - (double)m[e - 1]);
    const double pU = u[e], pD = m[e];
    double s0 = fma((double)cc[B0], B0v, (double)cc[WRK1]);
    s0 = fma((double)cc[B1], B1v, s0);
    s0 = fma((double)cc[B2], B2v, s0);
    s0 = fma((double)cc[A0], pE, s0);
    s0 = fma((double)cc[C0], pW, s0);
    s0 = fma((double)cc[A1], pN, s0);
    s0 = fma((double)cc[C1], pS, s0);
    s0 = fma((double)cc[A2], pU, s0);
    s0 = fma((double)cc[C2], pD, s0);
    const double ss = fma(s0, (double)cc[A3], -pc) * (double)cc[BND];
    *out = (float)fma(omega, ss, pc);
    return ss;
}

// p19_update with the plane-above and plane-below terms supplied: the centre
// values pc, pU, pD and the z-differences B1v, B2v (each the difference of
// a y- or x-difference of plane zc+1 and the same one of plane zc-1, kept
// from two planes earlier instead of being read again).  The same operands
// and operations as p19_update.
template <int W>
__device__ __forceinline__ double p19_update_zq(const float *o, int e, double pc, double pU, double pD, double B1v,
                                                double B2v, const float *cc, double omega, float *out) {
    const double pE = o[e + 1], pW = o[e - 1], pN = o[e + W], pS = o[e - W];
    const double B0v = ((double)o[e + W + 1] - (double)o[e - W + 1]) - ((double)o[e + W - 1] - (double)o[e - W - 1]);
    double s0 = fma((double)cc[B0], B0v, (double)cc[WRK1]);
    s0 = fma((double)cc[B1], B1v, s0);
    s0 = fma((double)cc[B2], B2v, s0);
    s0 = fma((double)cc[A0], pE, s0);
    s0 = fma((double)cc[C0], pW, s0);
    s0 = fma((double)cc[A1], pN, s0);
    s0 = fma((double)cc[C1], pS, s0);
    s0 = fma((double)cc[A2], pU, s0);
    s0 = fma((double)cc[C2], pD, s0);
    const double ss = fma(s0, (double)cc[A3], -pc) * (double)cc[BND];
    *out = (float)fma(omega, ss, pc);
    return ss;
}

// The centre value and the y- and x-differences of one plane at e.
struct ZTerms {
    float c;
    double dy, dx;
};
template <int W>
__device__ __forceinline__ ZTerms z_terms(const float *q, int e) {
    return ZTerms{q[e], (double)q[e + W] - (double)q[e - W], (double)q[e + 1] - (double)q[e - 1]};
}

// SATURATED, two sweeps per pass over memory (temporal blocking).  A block
// owns a TX x TY output tile and streams z.  Sweep 1 is computed on the tile
// plus a one-cell ring (its values are needed by sweep 2's neighbours and are
// recomputed by every block that needs them, never exchanged), from an LDS
// ring of p^t planes with a two-cell halo; sweep 2 is computed on the tile
// from an LDS ring of the sweep-1 planes and written out.  The 12 coefficient
// streams and p are read once per two sweeps: 56 algorithmic bytes per two
// point updates.  Every value is the one two launches of poisson19_sat would
// produce (same operations, sweep-1 values rounded to F32 as if stored), so
// the result and the residual (sum of ss^2 of the second sweep) match it bit
// for bit.  Cells of the ring that are boundary cells keep their fixed value.
//
// Threads: TY rows of TX "tile" threads (one output cell each: its sweep-1
// and sweep-2 values) and EY extra rows of "ring" threads (one ring cell of
// sweep 1 each), so that no wave carries two sweep-1 cells.
template <int TX, int TY>
struct Sat2Shape {
    static constexpr int W1 = TX + 2;
    static constexpr int RS = 2 * W1 + 2 * TY;  // ring cells of the sweep-1 tile
    static constexpr int EY0 = (RS + TX - 1) / TX;
    static constexpr int EY = (TX * (TY + EY0)) % 64 == 0 ? EY0 : EY0 + 1;  // whole waves
    static constexpr int NT = TX * (TY + EY);
    // z-queues (each thread keeps the centre values and y-/x-differences of
    // the two planes below the one it reads): 19 -> 13 LDS reads and
    // conversions per update for about 20 more VGPRs.  Measured faster at
    // 64 x 8, 128 x 4 and 32 x 4; at 64 x 4 (7 waves) they cost the second
    // block per CU, and at 32 x 8 they measured slower at the z-blocks that
    // matter (16, 32).
    static constexpr bool ZQ = (TX == 64 && TY == 8) || (TX == 128 && TY == 4) || (TX == 32 && TY == 4);
};

template <int TX, int TY>
__global__ __launch_bounds__((Sat2Shape<TX, TY>::NT)) void poisson19_sat2(const float *__restrict__ p,
                                                                         float *__restrict__ pn, P19Coef c, Geom g,
                                                                         double omega, int zb, int remap,
                                                                         double *__restrict__ part) {
    using S = Sat2Shape<TX, TY>;
    constexpr int W0 = TX + 4, PL0 = (TY + 4) * W0;  // p^t tile, two-cell halo
    constexpr int W1 = S::W1, PL1 = (TY + 2) * W1;   // sweep-1 tile, one-cell ring
    constexpr int NT = S::NT, RS = S::RS;
    static_assert(RS <= TX * S::EY && NT <= 1024, "ring threads");
    // The LDS rings hold the F32 values (widened at each read: FP64 rings
    // double the LDS traffic and measured slower).
    __shared__ float r0[4][PL0];
    __shared__ float r1[4][PL1];
    __shared__ double red[kMaxWaves];
    int bx, by, bz;
    tile_coords(remap, bx, by, bz);
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
    const int PX = g.nx + 2, PY = g.ny + 2;
    const int k0 = bz * zb, k1 = min(k0 + zb, g.nz);  // output planes zc = k0+1 .. k1 (padded)

    // tile thread: sweep-1 cell (tx+1, ty+1) of the ring tile and output cell of sweep 2
    const bool tile_t = ty < TY;
    const int xo = bx * TX + tx + 1, yo = by * TY + ty + 1;  // padded coordinates
    const bool in_o = tile_t && xo <= g.nx && yo <= g.ny;
    const bool ld_o = tile_t && xo < PX && yo < PY;
    const long long col_o = (long long)yo * g.py + xo;
    const int e0_o = (ty + 2) * W0 + tx + 2, e1_o = (ty + 1) * W1 + tx + 1;
    // ring thread: ring cell q of the sweep-1 tile
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
    const int xr = bx * TX + ex, yr = by * TY + ey;  // padded
    const bool in_r = has_r && xr >= 1 && xr <= g.nx && yr >= 1 && yr <= g.ny;
    const int e0_r = (ey + 1) * W0 + ex + 1, e1_r = ey * W1 + ex;
    // the cell this thread computes in sweep 1
    const bool in_a = tile_t ? in_o : in_r;
    const bool has_a = tile_t || has_r;
    const int e0_a = tile_t ? e0_o : e0_r, e1_a = tile_t ? e1_o : e1_r;

    HaloStager<float, TX, TY, 2, true, NT> halo;
    halo.init(tid, bx * TX + 1, by * TY + 1, g.py, PX, PY);
    constexpr int HR = decltype(halo)::HR;

    const int zlo = k0, zhi = k1 + 1;  // sweep-1 planes computed: zlo .. zhi (padded)
    // prologue: p^t planes zlo-1 (if any) and zlo into LDS
    for (int z = zlo - 1; z <= zlo; ++z) {
        if (z < 0) continue;
        const float *pl = p + (long long)z * g.pz;
        if (tile_t) r0[(z - zlo + 4) & 3][e0_o] = ld_o ? pl[col_o] : 0.0f;
        halo.load(pl);
        halo.store(r0[(z - zlo + 4) & 3]);
    }
    // From here every load is unconditional and goes through a scalar buffer
    // resource per plane with a 32-bit byte offset per lane (planes below
    // 4 GiB, checked on the host).  A lane with nothing to load reads the
    // cell of its own tile column (the tile's first row for ring threads),
    // which the tile loads anyway, so the request coalesces with real ones;
    // a cell outside the padded array reads the clamped cell of its row, a
    // ring cell outside it is stored as 0, and a load for a plane the block
    // does not need reads one it does.  None of those values is used.  No
    // register is then merged with an older value or zeroed while a load
    // into it is in flight.
    const long long pzb = g.pz * (long long)sizeof(float);
    auto cb = [&](int y, int x) -> unsigned {
        return (unsigned)(((long long)min(max(y, 0), PY - 1) * g.py + min(max(x, 0), PX - 1)) * (long long)sizeof(float));
    };
    const unsigned ob = tile_t ? cb(yo, xo) : cb(by * TY + 1, xo);  // centre of p (own column)
    const unsigned ab = has_r ? cb(yr, xr) : ob;                     // coefficients of the sweep-1 cell
    unsigned hb[HR];
#pragma unroll
    for (int h = 0; h < HR; ++h) hb[h] = halo.ok[h] ? (unsigned)(halo.goff[h] * (long long)sizeof(float)) : ob;
    auto ld = [](const void *plane, unsigned off) -> float { return buf_ld_f32(plane_rsrc(plane), off); };
    float ctr = ld((const char *)p + (long long)(zlo + 1) * pzb, ob);
    float hv[HR];
#pragma unroll
    for (int h = 0; h < HR; ++h) hv[h] = ld((const char *)p + (long long)(zlo + 1) * pzb, hb[h]);
    // Coefficients of this thread's sweep-1 cell, in four sets, one per plane
    // mod 4: set P = (zA - zlo) mod 4 is loaded at step zA (plane zA+1), read
    // by sweep 1 at step zA+1 and (tile threads: the own cell) by sweep 2 at
    // step zA+3, two planes behind, and reloaded at step zA+4, so no set is
    // ever copied.  Set 3 starts with plane zlo.
    float cf[4][12];
    {
        const long long zo = (long long)max(zlo, 1) * pzb;
#pragma unroll
        for (int s = 0; s < 12; ++s) {
            cf[0][s] = cf[1][s] = cf[2][s] = 0.0f;
            cf[3][s] = ld((const char *)c.f[s] + zo, ab);
        }
    }
    // z-queues: the terms of planes zA-1 and zA for sweep 1 (from the p^t
    // ring) and of planes zc-1 and zc for sweep 2 (from the sweep-1 ring)
    ZTerms q1m{}, q1o{}, q2m{}, q2o{};
    if constexpr (S::ZQ) {
        __syncthreads();
        if (has_a) {
            q1m = z_terms<W0>(r0[3], e0_a);  // plane zlo-1 (unused when zlo = 0: sweep 1 copies plane 0)
            q1o = z_terms<W0>(r0[0], e0_a);
        }
    }
    double acc = 0.0;

    // Iteration zA: sweep 1 at plane zA, sweep 2 at plane zA-2 (its inputs,
    // sweep-1 planes zA-3 .. zA-1, were written in earlier iterations), so one
    // barrier per plane separates every LDS write from its readers.  Ring
    // slots are relative to zlo: plane z sits in slot (z - zlo) mod 4; SM,
    // S0, SP, S2 are the slots of planes zA-1, zA, zA+1 and zA+2 (= zA-2).
    // running byte offsets of planes zA+2 (p), zA+1 (coefficients) and zA-2 (output)
    // (clamped to the last plane each stream needs: the loads of the last
    // steps re-read a plane just read, from L2)
    long long o_p = (long long)(zlo + 2) * pzb, o_c = (long long)(zlo + 1) * pzb;
    const long long p_max = (long long)min(zhi + 1, g.nz + 1) * pzb, c_max = (long long)min(zhi, g.nz) * pzb;
    long long o_out = (long long)(zlo - 2) * pzb;  // >= pzb whenever a store happens
    auto step = [&](const int zA, const int P, const int SM, const int S0, const int SP, const int S2) {
        // the coefficients of plane zA (sweep 1) and of plane zA-2 (sweep 2)
        const float *cc = cf[(P + 3) & 3], *cs = cf[(P + 1) & 3];
        if (zA <= zhi) {
            // stage p^t plane zA+1
            if (tile_t) r0[SP][e0_o] = ctr;
#pragma unroll
            for (int h = 0; h < HR; ++h)
                if (halo.has[h]) r0[SP][halo.lidx[h]] = halo.ok[h] ? hv[h] : 0.0f;
        }
        {
            // every load of the next plane: p^t plane zA+2 (needed if zA < zhi and
            // inside the array) and the coefficients of plane zA+1 (if interior)
            const long long op = min(o_p, p_max);
            ctr = ld((const char *)p + op, ob);
#pragma unroll
            for (int h = 0; h < HR; ++h) hv[h] = ld((const char *)p + op, hb[h]);
            const long long oc = max(min(o_c, c_max), pzb);
#pragma unroll
            for (int s = 0; s < 12; ++s) cf[P][s] = ld((const char *)c.f[s] + oc, ab);
        }
        __syncthreads();
        const int zc = zA - 2;  // sweep 2 at plane zc, from sweep-1 planes zc-1 .. zc+1
        if constexpr (S::ZQ) {
            if (zA <= zhi && has_a) {  // sweep 1 at plane zA: own cell or ring cell
                const bool zin = zA >= 1 && zA <= g.nz;
                const ZTerms t = z_terms<W0>(r0[SP], e0_a);  // plane zA+1
                float v;
                if (zin && in_a)
                    p19_update_zq<W0>(r0[S0], e0_a, q1o.c, t.c, q1m.c, t.dy - q1m.dy, t.dx - q1m.dx, cc, omega, &v);
                else v = q1o.c;
                r1[S0][e1_a] = v;
                q1m = q1o;
                q1o = t;
            }
            if (zA > zlo && tile_t) {
                const ZTerms t = z_terms<W1>(r1[SM], e1_o);  // plane zc+1
                if (zc >= k0 + 1 && in_o) {
                    float v;
                    const double ss = p19_update_zq<W1>(r1[S2], e1_o, q2o.c, t.c, q2m.c, t.dy - q2m.dy,
                                                        t.dx - q2m.dx, cs, omega, &v);
                    buf_st_f32(plane_rsrc((char *)pn + o_out), ob, v);
                    acc = fma(ss, ss, acc);
                }
                q2m = q2o;
                q2o = t;
            }
        } else {
            if (zA <= zhi && has_a) {  // sweep 1 at plane zA: own cell or ring cell
                const bool zin = zA >= 1 && zA <= g.nz;
                const float *m = r0[SM], *o = r0[S0], *u = r0[SP];
                float v;
                if (zin && in_a) p19_update<W0>(m, o, u, e0_a, cc, omega, &v);
                else v = o[e0_a];
                r1[S0][e1_a] = v;
            }
            if (zc >= k0 + 1 && in_o) {
                const float *m = r1[SP], *o = r1[S2], *u = r1[SM];
                float v;
                const double ss = p19_update<W1>(m, o, u, e1_o, cs, omega, &v);
                buf_st_f32(plane_rsrc((char *)pn + o_out), ob, v);
                acc = fma(ss, ss, acc);
            }
        }
        o_p += pzb;
        o_c += pzb;
        o_out += pzb;
    };
    // Four planes per trip: every ring slot and coefficient set is a
    // compile-time constant.  The loop leaves between steps, so no step is
    // skipped inside a trip and no value merges there (a merge would copy
    // registers whose loads are still in flight, and wait for them).
    for (int zA = zlo;; zA += 4) {
        if (zA > zhi + 1) break;
        step(zA, 0, 3, 0, 1, 2);
        if (zA + 1 > zhi + 1) break;
        step(zA + 1, 1, 0, 1, 2, 3);
        if (zA + 2 > zhi + 1) break;
        step(zA + 2, 2, 1, 2, 3, 0);
        if (zA + 3 > zhi + 1) break;
        step(zA + 3, 3, 2, 3, 0, 1);
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

#define P19_SAT_TILES(X) X(32, 2) X(32, 4) X(32, 8) X(64, 1) X(64, 2) X(64, 4) X(64, 8) X(128, 1) X(128, 2) \
    X(128, 4) X(128, 8) X(256, 1) X(256, 4)
// Two-sweep tiles (block = TX x (TY + ring rows) <= 1024 threads); each is
// also a single-sweep tile (an odd sweep count starts with one single sweep
// at the same shape).
#define P19_SAT2_TILES(X) X(32, 4) X(32, 8) X(64, 4) X(64, 8) X(128, 4)

bool p19_tile_ok(int v, Tile t) {
    if (v == V_PLAIN || is_point_form(v)) return plain_tile_ok(t);
    if (t.tz < 1) return false;
    if (v == V_SAT2) {
#define X(a, b) if (t.tx == a && t.ty == b) return true;
        P19_SAT2_TILES(X)
#undef X
        return false;
    }
#define X(a, b) if (t.tx == a && t.ty == b) return true;
    P19_SAT_TILES(X)
#undef X
    return false;
}

int p19_sat_tiles(Tile *out, int max) {
    int n = 0;
#define X(a, b) if (n < max) out[n++] = Tile{a, b, 0};
    P19_SAT_TILES(X)
#undef X
    return n;
}

int p19_sat2_tiles(Tile *out, int max) {
    int n = 0;
#define X(a, b) if (n < max) out[n++] = Tile{a, b, 0};
    P19_SAT2_TILES(X)
#undef X
    return n;
}

long long p19_nblocks(int, Tile t, const Geom &g) { return cdiv(g.nx, t.tx) * cdiv(g.ny, t.ty) * cdiv(g.nz, t.tz); }

hipError_t p19_launch(int v, Tile t, const SweepArgs &a, hipStream_t s) {
    const float *src = (const float *)a.src;
    float *dst = (float *)a.dst;
    const P19Coef c = pack(a);
    dim3 grid(cdiv(a.g.nx, t.tx), cdiv(a.g.ny, t.ty), cdiv(a.g.nz, t.tz));
    if (v == V_PLAIN) {
        hipLaunchKernelGGL(poisson19_plain, grid, dim3(t.tx, t.ty, t.tz), 0, s, src, dst, c, a.g, a.omega, a.part);
        return hipGetLastError();
    }
    if (is_point_form(v)) {
        const dim3 blk(t.tx, t.ty, t.tz);
        if (v == V_CSE_SAT) hipLaunchKernelGGL(poisson19_point<FORM_SAT>, grid, blk, 0, s, src, dst, c, a.g, a.omega, a.part);
        else if (v == V_CSE_BULK) hipLaunchKernelGGL(poisson19_point<FORM_BULK>, grid, blk, 0, s, src, dst, c, a.g, a.omega, a.part);
        else hipLaunchKernelGGL(poisson19_point<FORM_BOTH>, grid, blk, 0, s, src, dst, c, a.g, a.omega, a.part);
        return hipGetLastError();
    }
    if (v == V_SAT2) {
#define X(A, B)                                                                                           \
    if (t.tx == A && t.ty == B) {                                                                         \
        hipLaunchKernelGGL((poisson19_sat2<A, B>), grid, dim3(A, B + Sat2Shape<A, B>::EY, 1), 0, s, src, dst, c, a.g, \
                           a.omega, t.tz,                                                                          \
                           a.remap, a.part);                                                              \
        return hipGetLastError();                                                                         \
    }
        P19_SAT2_TILES(X)
#undef X
        return hipErrorInvalidValue;
    }
#define X(A, B)                                                                                          \
    if (t.tx == A && t.ty == B) {                                                                        \
        hipLaunchKernelGGL((poisson19_sat<A, B>), grid, dim3(A, B, 1), 0, s, src, dst, c, a.g, a.omega, t.tz, \
                           a.remap, a.part);                                                             \
        return hipGetLastError();                                                                        \
    }
    P19_SAT_TILES(X)
#undef X
    return hipErrorInvalidValue;
}

}  // namespace

KindOps poisson19_ops = {p19_tile_ok, p19_sat_tiles, p19_sat2_tiles, p19_nblocks, p19_launch, nullptr};

}  // namespace stn
