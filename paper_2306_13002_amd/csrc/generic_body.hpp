// generic_body.hpp -- the saturated generic stencil's streaming body, shared
// by the table-driven kernel (generic.hip) and the kernels generated for one
// stencil at plan time (rtc.cpp).
//
// A block owns a TX x TY column tile and streams input planes
// zp = bz*zb .. bz*zb + zb - 1 + 2R (padded z).  Each plane is staged once in
// LDS with its R-wide ring (corners when CORNERS) and contributes to the 2R+1
// output planes it touches; their FP64 accumulators wait in a register queue
// (acc[s] holds output plane m + R - s after input plane m).  `slots(t, me,
// acc)` adds the plane's taps to every slot: slot s takes the taps with
// dz = s - R.  The next plane's loads are issued before this plane's
// arithmetic.  Returns the thread's sum of squared changes.
#pragma once

#include "common.hpp"

namespace stn {

template <typename T, int R, int TX, int TY, bool CORNERS, class Slots>
__device__ __forceinline__ double generic_sat_body(const T *__restrict__ src, T *__restrict__ dst, const Geom &g,
                                                   int zb, int bx, int by, int bz, const Slots &slots,
                                                   double (*tile)[(TY + 2 * R) * (TX + 2 * R)]) {
    constexpr int W = TX + 2 * R, NT = TX * TY, NQ = 2 * R + 1;
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * TX + tx;
    const int i = bx * TX + tx, j = by * TY + ty;
    const int xp = i + R, yp = j + R;
    const int PX = g.nx + 2 * R, PY = g.ny + 2 * R;
    const bool in = i < g.nx && j < g.ny;
    const bool ld = xp < PX && yp < PY;
    const int k0 = bz * zb, k1 = min(k0 + zb, g.nz);
    const long long col = (long long)yp * g.py + xp;
    const int me = (ty + R) * W + (tx + R);

    HaloStager<T, TX, TY, R, CORNERS, NT> halo;
    halo.init(tid, bx * TX + R, by * TY + R, g.py, PX, PY);

    // ctr[s]: the old value of the output in slot s (for the residual)
    double acc[NQ], ctr[NQ];
#pragma unroll
    for (int s = 0; s < NQ; ++s) {
        acc[s] = 0.0;
        ctr[s] = 0.0;
    }
    int zp = k0;
    T cval = ld ? src[col + (long long)zp * g.pz] : T(0);
    halo.load(src + (long long)zp * g.pz);
    double sacc = 0.0;
    const int zend = k1 - 1 + 2 * R;
    for (int b = 0; zp <= zend; ++zp, b ^= 1) {
        double *t = tile[b];
        t[me] = (double)cval;
#pragma unroll
        for (int s = 0; s < decltype(halo)::HR; ++s)
            if (halo.has[s]) t[halo.lidx[s]] = (double)halo.val[s];
        const double cur_ctr = (double)cval;
        if (zp < zend) {  // bulk load of the next plane
            cval = ld ? src[col + (long long)(zp + 1) * g.pz] : T(0);
            halo.load(src + (long long)(zp + 1) * g.pz);
        }
        __syncthreads();
        // input plane m = zp - R: slot s now holds output plane m + R - s
#pragma unroll
        for (int s = NQ - 1; s > 0; --s) {
            acc[s] = acc[s - 1];
            ctr[s] = ctr[s - 1];
        }
        acc[0] = 0.0;
        ctr[0] = 0.0;
        ctr[R] = cur_ctr;  // this plane's centre is the old value of output m
        slots(t, me, acc);
        // output m - R (slot 2R) is complete
        const int kout = zp - 2 * R;
        if (in && kout >= k0 && kout < k1) {
            const T out = (T)acc[2 * R];
            dst[col + (long long)(kout + R) * g.pz] = out;
            const double d = (double)out - ctr[2 * R];
            sacc = fma(d, d, sacc);
        }
    }
    return sacc;
}

}  // namespace stn
