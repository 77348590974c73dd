/*
 * oracle.c -- plain CPU FP64 definition of every stencil sweep in this library.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the tests, the package smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no source with the HIP library.
 *
 * What it computes.  The paper (ACC Saturator, arXiv 2306.13002) optimizes the
 * sequential body of the innermost parallel loop of directive-based codes
 * (Sec. "E-Graph Creation"; its benchmark tables list Jacobi and halo-3D CFD
 * loop nests as the memory-bound class).  Every method here is an exact,
 * deterministic Jacobi/leapfrog iteration, so the oracle is simply the loop
 * body written out once, in the "plain" order below, with no blocking, fusion
 * or reordering:
 *
 *   - each product is rounded, then the terms are added left to right;
 *   - the build uses -O2 -fno-fast-math -ffp-contract=off, so no FMA is formed;
 *   - every array is a dense row-major padded grid, x contiguous, with a halo
 *     of width r on every side: element (x,y,z) of the padded grid sits at
 *     ((z*PY)+y)*PX+x with PX = nx+2r, PY = ny+2r, PZ = nz+2r; interior point
 *     (i,j,k), 0 <= i < nx, sits at padded (i+r, j+r, k+r);
 *   - Dirichlet: the halo holds fixed boundary values and is never written;
 *     periodic (heat only, used by the conservation check): neighbours wrap
 *     inside the interior and the halo is ignored;
 *   - residual of a run = sum over the interior of (new - old)^2 of the LAST
 *     sweep, accumulated in FP64 in z, y, x order (for the pressure kind the
 *     residual is the sum of ss^2 of the last sweep, see below).
 *
 * Storage modes for FP32-storage kinds: mode 0 (F64) keeps the state in FP64;
 * mode 1 (F32STORE) computes in FP64 but rounds every stored state value to
 * FP32, exactly as a kernel that widens on load and narrows on store does.
 *
 * Return value of every entry: 0 on success, -1 on bad arguments or
 * allocation failure.  All pointers are host pointers owned by the caller.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PIDX(x, y, z, PX, PY) ((((int64_t)(z) * (PY)) + (y)) * (PX) + (x))

static double store_round(double v, int mode) { return mode == 1 ? (double)(float)v : v; }

static int64_t wrap(int64_t i, int64_t n) {
    i %= n;
    return i < 0 ? i + n : i;
}

/* ------------------------------------------------------------------------- */
/* 2-D five-point heat (Jacobi) sweep.
 * dst = cc*u + cn*u(-x) + cn*u(+x) + cn*u(-y) + cn*u(+y).                  */
static void heat2d5_sweep(int64_t nx, int64_t ny, const double *src, double *dst,
                          double cc, double cn, int periodic) {
    const int64_t PX = nx + 2, PY = ny + 2;
    for (int64_t j = 0; j < ny; ++j)
        for (int64_t i = 0; i < nx; ++i) {
            int64_t xm = i - 1, xp = i + 1, ym = j - 1, yp = j + 1;
            if (periodic) {
                xm = wrap(xm, nx); xp = wrap(xp, nx); ym = wrap(ym, ny); yp = wrap(yp, ny);
            }
            const double u = src[PIDX(i + 1, j + 1, 0, PX, PY)];
            double v = cc * u;
            v = v + cn * src[PIDX(xm + 1, j + 1, 0, PX, PY)];
            v = v + cn * src[PIDX(xp + 1, j + 1, 0, PX, PY)];
            v = v + cn * src[PIDX(i + 1, ym + 1, 0, PX, PY)];
            v = v + cn * src[PIDX(i + 1, yp + 1, 0, PX, PY)];
            dst[PIDX(i + 1, j + 1, 0, PX, PY)] = v;
        }
}

/* 3-D seven-point heat sweep: centre, -x, +x, -y, +y, -z, +z.               */
static void heat3d7_sweep(int64_t nx, int64_t ny, int64_t nz, const double *src,
                          double *dst, double cc, double cn, int periodic) {
    const int64_t PX = nx + 2, PY = ny + 2;
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t xm = i - 1, xp = i + 1, ym = j - 1, yp = j + 1, zm = k - 1, zp = k + 1;
                if (periodic) {
                    xm = wrap(xm, nx); xp = wrap(xp, nx);
                    ym = wrap(ym, ny); yp = wrap(yp, ny);
                    zm = wrap(zm, nz); zp = wrap(zp, nz);
                }
                const double u = src[PIDX(i + 1, j + 1, k + 1, PX, PY)];
                double v = cc * u;
                v = v + cn * src[PIDX(xm + 1, j + 1, k + 1, PX, PY)];
                v = v + cn * src[PIDX(xp + 1, j + 1, k + 1, PX, PY)];
                v = v + cn * src[PIDX(i + 1, ym + 1, k + 1, PX, PY)];
                v = v + cn * src[PIDX(i + 1, yp + 1, k + 1, PX, PY)];
                v = v + cn * src[PIDX(i + 1, j + 1, zm + 1, PX, PY)];
                v = v + cn * src[PIDX(i + 1, j + 1, zp + 1, PX, PY)];
                dst[PIDX(i + 1, j + 1, k + 1, PX, PY)] = v;
            }
}

/* Sum over the interior of (a-b)^2, z,y,x order, FP64. */
static double diff_sq_sum(int64_t nx, int64_t ny, int64_t nz, int r, const double *a,
                          const double *b) {
    const int64_t PX = nx + 2 * r, PY = ny + 2 * r;
    double s = 0.0;
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                const int64_t p = PIDX(i + r, j + r, k + r, PX, PY);
                const double d = a[p] - b[p];
                s = s + d * d;
            }
    return s;
}

static double diff_sq_sum_2d(int64_t nx, int64_t ny, const double *a, const double *b) {
    const int64_t PX = nx + 2, PY = ny + 2;
    double s = 0.0;
    for (int64_t j = 0; j < ny; ++j)
        for (int64_t i = 0; i < nx; ++i) {
            const int64_t p = PIDX(i + 1, j + 1, 0, PX, PY);
            const double d = a[p] - b[p];
            s = s + d * d;
        }
    return s;
}

/*
 * oracle_heat_run: T Jacobi sweeps of the 2-D 5-point (ndim=2) or 3-D 7-point
 * (ndim=3) heat operator on u, in place (ping-pong through an internal copy).
 * u: padded grid ((ny+2)*(nx+2) for 2-D, (nz+2)*(ny+2)*(nx+2) for 3-D).
 * resid (may be NULL): residual of the last sweep; 0 when T == 0.
 */
int oracle_heat_run(int ndim, int64_t nx, int64_t ny, int64_t nz, double *u, double cc,
                    double cn, int T, int periodic, double *resid) {
    if (!u || nx < 1 || ny < 1 || (ndim == 3 && nz < 1) || T < 0 || (ndim != 2 && ndim != 3))
        return -1;
    const int64_t total = (ndim == 2) ? (nx + 2) * (ny + 2) : (nx + 2) * (ny + 2) * (nz + 2);
    double *a = (double *)malloc(sizeof(double) * total);
    double *b = (double *)malloc(sizeof(double) * total);
    if (!a || !b) { free(a); free(b); return -1; }
    memcpy(a, u, sizeof(double) * total);
    memcpy(b, u, sizeof(double) * total); /* halo of the second buffer = halo of u */
    double *src = a, *dst = b;
    double r = 0.0;
    for (int t = 0; t < T; ++t) {
        if (ndim == 2) heat2d5_sweep(nx, ny, src, dst, cc, cn, periodic);
        else heat3d7_sweep(nx, ny, nz, src, dst, cc, cn, periodic);
        if (t == T - 1)
            r = (ndim == 2) ? diff_sq_sum_2d(nx, ny, dst, src) : diff_sq_sum(nx, ny, nz, 1, dst, src);
        double *tmp = src; src = dst; dst = tmp;
    }
    memcpy(u, src, sizeof(double) * total);
    free(a); free(b);
    if (resid) *resid = r;
    return 0;
}

/* ------------------------------------------------------------------------- */
/*
 * 19-point variable-coefficient pressure relaxation (Jacobi with relaxation
 * factor omega), the halo-3D CFD loop-nest class.  Logical (i,j,k) = (x,y,z);
 * every coefficient array is read at the point itself:
 *
 *   s0 = a0*p(i+1,j,k) + a1*p(i,j+1,k) + a2*p(i,j,k+1)
 *      + b0*(p(i+1,j+1,k) - p(i+1,j-1,k) - p(i-1,j+1,k) + p(i-1,j-1,k))
 *      + b1*(p(i,j+1,k+1) - p(i,j-1,k+1) - p(i,j+1,k-1) + p(i,j-1,k-1))
 *      + b2*(p(i+1,j,k+1) - p(i-1,j,k+1) - p(i+1,j,k-1) + p(i-1,j,k-1))
 *      + c0*p(i-1,j,k) + c1*p(i,j-1,k) + c2*p(i,j,k-1) + wrk1
 *   ss = (s0*a3 - p)*bnd ;  p' = p + omega*ss ;  residual += ss^2
 *
 * coef: 12 padded arrays in the order a0 a1 a2 a3 b0 b1 b2 c0 c1 c2 bnd wrk1
 * (values at halo cells are never read).  p: padded state, updated in place.
 * mode 0 = F64, 1 = F32STORE.  gosa (may be NULL): sum of ss^2 of the last
 * sweep, FP64, z,y,x order.
 */
int oracle_poisson19_run(int64_t nx, int64_t ny, int64_t nz, double *p,
                         const double *const *coef, double omega, int T, int mode,
                         double *gosa) {
    if (!p || !coef || nx < 1 || ny < 1 || nz < 1 || T < 0 || (mode != 0 && mode != 1)) return -1;
    for (int c = 0; c < 12; ++c) if (!coef[c]) return -1;
    const int64_t PX = nx + 2, PY = ny + 2, total = (nx + 2) * (ny + 2) * (nz + 2);
    const double *a0 = coef[0], *a1 = coef[1], *a2 = coef[2], *a3 = coef[3];
    const double *b0 = coef[4], *b1 = coef[5], *b2 = coef[6];
    const double *c0 = coef[7], *c1 = coef[8], *c2 = coef[9], *bnd = coef[10], *wrk1 = coef[11];
    double *a = (double *)malloc(sizeof(double) * total);
    double *b = (double *)malloc(sizeof(double) * total);
    if (!a || !b) { free(a); free(b); return -1; }
    for (int64_t q = 0; q < total; ++q) a[q] = store_round(p[q], mode);
    memcpy(b, a, sizeof(double) * total);
    double *src = a, *dst = b, g = 0.0;
#define P(di, dj, dk) src[PIDX(x + (di), y + (dj), z + (dk), PX, PY)]
    for (int t = 0; t < T; ++t) {
        g = 0.0;
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t i = 0; i < nx; ++i) {
                    const int64_t x = i + 1, y = j + 1, z = k + 1;
                    const int64_t c = PIDX(x, y, z, PX, PY);
                    double s0 = a0[c] * P(1, 0, 0);
                    s0 = s0 + a1[c] * P(0, 1, 0);
                    s0 = s0 + a2[c] * P(0, 0, 1);
                    s0 = s0 + b0[c] * (((P(1, 1, 0) - P(1, -1, 0)) - P(-1, 1, 0)) + P(-1, -1, 0));
                    s0 = s0 + b1[c] * (((P(0, 1, 1) - P(0, -1, 1)) - P(0, 1, -1)) + P(0, -1, -1));
                    s0 = s0 + b2[c] * (((P(1, 0, 1) - P(-1, 0, 1)) - P(1, 0, -1)) + P(-1, 0, -1));
                    s0 = s0 + c0[c] * P(-1, 0, 0);
                    s0 = s0 + c1[c] * P(0, -1, 0);
                    s0 = s0 + c2[c] * P(0, 0, -1);
                    s0 = s0 + wrk1[c];
                    const double ss = (s0 * a3[c] - P(0, 0, 0)) * bnd[c];
                    g = g + ss * ss;
                    dst[c] = store_round(P(0, 0, 0) + omega * ss, mode);
                }
        double *tmp = src; src = dst; dst = tmp;
    }
#undef P
    memcpy(p, src, sizeof(double) * total);
    free(a); free(b);
    if (gosa) *gosa = g;
    return 0;
}

/* ------------------------------------------------------------------------- */
/*
 * Radius-4 25-point star, second order in time (leapfrog wave update):
 *   L(u) = sum over axes x, y, z of [ c0*u + c1*u(+1) + c1*u(-1) + ... + c4*u(-4) ]
 *          evaluated as ONE left-to-right chain of 27 products (axis x, then y,
 *          then z; per axis c0*u first, then r = 1..4 with +r before -r);
 *   u_next = (2*u - u_prev) + vsq*L(u),  vsq = (v*dt/h)^2 given per point.
 * a, b: the two time-level buffers (padded, halo 4); on entry a = u^{n-1},
 * b = u^n.  Each step overwrites the interior of the OLDER level in place
 * (u_next at a point needs u_prev only at that same point), then the roles
 * swap.  Each buffer keeps its own halo, which is never written.  After T
 * steps the newest level u^{n+T} is in a when T is odd and in b when T is
 * even; the other buffer holds u^{n+T-1}.
 * resid (may be NULL): sum over the interior of (u^{n+T} - u^{n+T-1})^2.
 */
int oracle_wave25_run(int64_t nx, int64_t ny, int64_t nz, double *a, double *b,
                      const double *vsq, const double *c, int T, double *resid) {
    if (!a || !b || !vsq || !c || nx < 1 || ny < 1 || nz < 1 || T < 0) return -1;
    const int64_t PX = nx + 8, PY = ny + 8;
    double *prev = a, *cur = b, r = 0.0;
    for (int t = 0; t < T; ++t) {
        r = 0.0;
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t i = 0; i < nx; ++i) {
                    const int64_t x = i + 4, y = j + 4, z = k + 4;
                    const int64_t q = PIDX(x, y, z, PX, PY);
                    double L = c[0] * cur[q];
                    for (int rr = 1; rr <= 4; ++rr) {
                        L = L + c[rr] * cur[PIDX(x + rr, y, z, PX, PY)];
                        L = L + c[rr] * cur[PIDX(x - rr, y, z, PX, PY)];
                    }
                    L = L + c[0] * cur[q];
                    for (int rr = 1; rr <= 4; ++rr) {
                        L = L + c[rr] * cur[PIDX(x, y + rr, z, PX, PY)];
                        L = L + c[rr] * cur[PIDX(x, y - rr, z, PX, PY)];
                    }
                    L = L + c[0] * cur[q];
                    for (int rr = 1; rr <= 4; ++rr) {
                        L = L + c[rr] * cur[PIDX(x, y, z + rr, PX, PY)];
                        L = L + c[rr] * cur[PIDX(x, y, z - rr, PX, PY)];
                    }
                    const double nv = (2.0 * cur[q] - prev[q]) + vsq[q] * L;
                    const double d = nv - cur[q];
                    r = r + d * d;
                    prev[q] = nv;
                }
        double *tmp = prev; prev = cur; cur = tmp;
    }
    if (resid) *resid = r;
    return 0;
}

/* ------------------------------------------------------------------------- */
/*
 * Generic 3-D linear stencil: u'(x) = sum_t coef[cid_t] * u(x + delta_t),
 * evaluated in tap-list order, left to right, from the first product.
 * tap_off: n_taps triples (dx, dy, dz) with |d| <= r; tap_cid: coefficient
 * index per tap, 0 <= cid < n_coef.  u: padded grid with halo r, updated in
 * place (Dirichlet: halo fixed).  mode 0 = F64, 1 = F32STORE.
 * resid (may be NULL): residual of the last sweep.
 */
int oracle_generic_run(int64_t nx, int64_t ny, int64_t nz, int r, double *u, int n_taps,
                       const int32_t *tap_off, const int32_t *tap_cid, const double *coef,
                       int n_coef, int T, int mode, double *resid) {
    if (!u || !tap_off || !tap_cid || !coef || nx < 1 || ny < 1 || nz < 1 || r < 1 || n_taps < 1 ||
        n_coef < 1 || T < 0 || (mode != 0 && mode != 1))
        return -1;
    for (int t = 0; t < n_taps; ++t) {
        if (tap_cid[t] < 0 || tap_cid[t] >= n_coef) return -1;
        for (int d = 0; d < 3; ++d)
            if (tap_off[3 * t + d] < -r || tap_off[3 * t + d] > r) return -1;
    }
    const int64_t PX = nx + 2 * r, PY = ny + 2 * r, total = PX * PY * (nz + 2 * r);
    double *a = (double *)malloc(sizeof(double) * total);
    double *b = (double *)malloc(sizeof(double) * total);
    if (!a || !b) { free(a); free(b); return -1; }
    for (int64_t q = 0; q < total; ++q) a[q] = store_round(u[q], mode);
    memcpy(b, a, sizeof(double) * total);
    double *src = a, *dst = b, rs = 0.0;
    for (int t = 0; t < T; ++t) {
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t i = 0; i < nx; ++i) {
                    const int64_t x = i + r, y = j + r, z = k + r;
                    double v = 0.0;
                    for (int s = 0; s < n_taps; ++s) {
                        const double term = coef[tap_cid[s]] *
                            src[PIDX(x + tap_off[3 * s], y + tap_off[3 * s + 1], z + tap_off[3 * s + 2], PX, PY)];
                        v = (s == 0) ? term : v + term;
                    }
                    dst[PIDX(x, y, z, PX, PY)] = store_round(v, mode);
                }
        if (t == T - 1) rs = diff_sq_sum(nx, ny, nz, r, dst, src);
        double *tmp = src; src = dst; dst = tmp;
    }
    memcpy(u, src, sizeof(double) * total);
    free(a); free(b);
    if (resid) *resid = rs;
    return 0;
}

/* ------------------------------------------------------------------------- */
/*
 * Pointwise multi-statement program (the loop body the paper rewrites, Sec.
 * "E-Graph Creation": straight-line assignments inside the innermost
 * parallel loop).  For every interior point, in z, y, x order, the
 * statements run in program order; each statement's expression is given in
 * postfix form and evaluated with a value stack, one IEEE operation per
 * instruction (so products and sums round in the written order):
 *   op 1 CONST a      push consts[a]
 *   op 2 PARAM a      push params[a]
 *   op 3 LOAD a,b,c,d push in[a] at (i+b, j+c, k+d)
 *   op 4 ADD, 5 SUB, 6 MUL: pop y, pop x, push x+y / x-y / x*y
 *   op 7 NEG          pop x, push -x
 *   op 8 STORE a      pop x, out[a] at (i,j,k) = x
 *   op 9 SET a        pop x, local a = x
 *   op 10 GET a       push local a
 * insns: n_insns groups of 5 int32 (op, a, b, c, d).  Every array is a
 * padded grid of this file's layout with halo r; outputs are written at
 * interior points only.  Returns -1 on a malformed program.
 */
int oracle_program_run(int64_t nx, int64_t ny, int64_t nz, int r, const int32_t *insns, int n_insns,
                       const double *consts, int n_consts, int n_in, const double *const *in, int n_out,
                       double *const *out, int n_par, const double *params, int n_loc) {
    if (!insns || n_insns < 1 || nx < 1 || ny < 1 || nz < 1 || r < 0 || n_in < 0 || n_out < 1 || n_par < 0 ||
        n_loc < 0 || (n_in > 0 && !in) || !out || (n_par > 0 && !params) || (n_consts > 0 && !consts))
        return -1;
    /* check the program once: operand ranges and stack depth */
    int depth = 0, max_depth = 0;
    for (int q = 0; q < n_insns; ++q) {
        const int32_t *s = insns + 5 * q;
        switch (s[0]) {
        case 1: if (s[1] < 0 || s[1] >= n_consts) return -1; ++depth; break;
        case 2: if (s[1] < 0 || s[1] >= n_par) return -1; ++depth; break;
        case 3:
            if (s[1] < 0 || s[1] >= n_in) return -1;
            for (int d = 2; d < 5; ++d)
                if (s[d] < -r || s[d] > r) return -1;
            ++depth;
            break;
        case 4: case 5: case 6: if (depth < 2) return -1; --depth; break;
        case 7: if (depth < 1) return -1; break;
        case 8: if (depth != 1 || s[1] < 0 || s[1] >= n_out) return -1; depth = 0; break;
        case 9: if (depth != 1 || s[1] < 0 || s[1] >= n_loc) return -1; depth = 0; break;
        case 10: if (s[1] < 0 || s[1] >= n_loc) return -1; ++depth; break;
        default: return -1;
        }
        if (depth > max_depth) max_depth = depth;
    }
    if (depth != 0) return -1;
    const int64_t PX = nx + 2 * r, PY = ny + 2 * r;
    double *stack = (double *)malloc(sizeof(double) * (size_t)(max_depth + 1));
    double *loc = (double *)calloc((size_t)(n_loc + 1), sizeof(double));
    if (!stack || !loc) { free(stack); free(loc); return -1; }
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                const int64_t x = i + r, y = j + r, z = k + r;
                int sp = 0;
                for (int q = 0; q < n_insns; ++q) {
                    const int32_t *s = insns + 5 * q;
                    switch (s[0]) {
                    case 1: stack[sp++] = consts[s[1]]; break;
                    case 2: stack[sp++] = params[s[1]]; break;
                    case 3: stack[sp++] = in[s[1]][PIDX(x + s[2], y + s[3], z + s[4], PX, PY)]; break;
                    case 4: --sp; stack[sp - 1] = stack[sp - 1] + stack[sp]; break;
                    case 5: --sp; stack[sp - 1] = stack[sp - 1] - stack[sp]; break;
                    case 6: --sp; stack[sp - 1] = stack[sp - 1] * stack[sp]; break;
                    case 7: stack[sp - 1] = -stack[sp - 1]; break;
                    case 8: out[s[1]][PIDX(x, y, z, PX, PY)] = stack[--sp]; break;
                    case 9: loc[s[1]] = stack[--sp]; break;
                    case 10: stack[sp++] = loc[s[1]]; break;
                    }
                }
            }
    free(stack);
    free(loc);
    return 0;
}
