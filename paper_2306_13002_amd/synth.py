"""Seeded synthetic inputs for the stencil workloads.

This module only draws numbers and lays them out; it holds none of the
stencils' arithmetic, so both the HIP path (tests, benchmark) and the CPU
oracle can be fed from it without sharing any computation.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used in counter form: the value
for linear index ``idx`` of stream ``stream`` under ``seed`` is the SplitMix64
output function applied to ``key + (idx + 1) * GAMMA`` with
``key = seed * 2**16 + stream`` and GAMMA the golden-ratio increment.  A
uniform double in [0, 1) is ``(x >> 11) * 2**-53``.  Linear indices run over
the PADDED array, so a value does not depend on the chunking used here.

Workload recipes (padded layout: x contiguous, halo r on every side):

* heat2d5: 256 x 256 interior, 1-cell ring fixed at 0, u0 = U[0,1)
  (seed 1, stream 0), coefficients 0.6 centre / 0.1 per neighbour, T = 10.
* poisson19: 129 x 129 x 257 grid INCLUDING its 1-cell boundary (interior
  127 x 127 x 255), FP32 arrays a0..a2 = 1, a3 = fl32(1/6), b0..b2 = 0,
  c0..c2 = 1, bnd = 1, wrk1 = 0; p = k^2 / 256^2 with k the z storage index
  (boundary included); omega = 0.8; T = 20.
* wave25: 512^3 interior + 4-cell halo; v = 1.5 + 3 U (seed 3, stream 0),
  vsq = (v * 0.4 / 4.5)^2 (Courant number at most 0.4); both time levels
  u^{-1} = u^0 = 1 + 0.1 U (seed 3, stream 1) over the whole padded array;
  per-axis coefficients (-2.847222, 1.6, -0.2, 0.025397, -0.001786); T = 10.
* heat3d7 batch: 64 problems, interior edges nx, ny, nz each drawn
  independently as 32 + floor(129 U) (seed 4, stream 0, problem-major), fields
  U[0,1) (seed 4, stream 1 + b) with a 0 ring; coefficients 0.4 / 0.1; T = 50.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_CHUNK = 1 << 22


def _mix64(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    """Raw 64-bit outputs for linear indices start .. start+count-1."""
    key = np.uint64((int(seed) << 16) + int(stream))
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix64(key + idx * GAMMA)


def uniform_f64(seed: int, stream: int, shape) -> np.ndarray:
    """U[0,1) doubles, (x >> 11) * 2^-53, filled in index order."""
    n = int(np.prod(shape))
    out = np.empty(n, dtype=np.float64)
    for s in range(0, n, _CHUNK):
        c = min(_CHUNK, n - s)
        out[s:s + c] = (splitmix64(seed, stream, s, c) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return out.reshape(shape)


def uniform_f32(seed: int, stream: int, shape) -> np.ndarray:
    """U[0,1) floats, (x >> 40) * 2^-24 (exact in FP32)."""
    n = int(np.prod(shape))
    out = np.empty(n, dtype=np.float32)
    for s in range(0, n, _CHUNK):
        c = min(_CHUNK, n - s)
        out[s:s + c] = ((splitmix64(seed, stream, s, c) >> np.uint64(40)).astype(np.float64)
                        * (2.0 ** -24)).astype(np.float32)
    return out.reshape(shape)


def zero_halo(a: np.ndarray, r: int) -> np.ndarray:
    """Set the halo of width r of a padded array to 0 (in place)."""
    for ax in range(a.ndim):
        sl = [slice(None)] * a.ndim
        sl[ax] = slice(0, r)
        a[tuple(sl)] = 0
        sl[ax] = slice(a.shape[ax] - r, a.shape[ax])
        a[tuple(sl)] = 0
    return a


# --------------------------------------------------------------------------
# heat2d5: 2-D five-point Jacobi heat sweep
HEAT2D5 = dict(n=256, T=10, cc=0.6, cn=0.1, seed=1)


def heat2d5_input(n: int = 256, seed: int = 1, stream: int = 0, ny: int | None = None) -> np.ndarray:
    ny = n if ny is None else ny
    u = uniform_f64(seed, stream, (ny + 2, n + 2))
    return zero_halo(u, 1)


# --------------------------------------------------------------------------
# heat3d7: 3-D seven-point Jacobi heat sweep, batch of uneven grids
HEAT3D7 = dict(count=64, lo=32, hi=160, T=50, cc=0.4, cn=0.1, seed=4)


def heat3d7_batch_sizes(count: int = 64, seed: int = 4, lo: int = 32, hi: int = 160):
    """Interior (nx, ny, nz) per problem, each edge lo + floor((hi-lo+1) U)."""
    u = uniform_f64(seed, 0, (count * 3,))
    e = lo + np.floor(u * (hi - lo + 1)).astype(np.int64)
    return [tuple(int(v) for v in e[3 * b:3 * b + 3]) for b in range(count)]


def heat3d7_input(nx: int, ny: int, nz: int, seed: int = 4, stream: int = 1) -> np.ndarray:
    u = uniform_f64(seed, stream, (nz + 2, ny + 2, nx + 2))
    return zero_halo(u, 1)


# --------------------------------------------------------------------------
# poisson19: 19-point variable-coefficient pressure relaxation (FP32 storage)
POISSON19 = dict(shape_total=(257, 129, 129), omega=0.8, T=20)
POISSON_COEF_ORDER = ("a0", "a1", "a2", "a3", "b0", "b1", "b2", "c0", "c1", "c2", "bnd", "wrk1")
POISSON_COEF_VALUES = dict(a0=1.0, a1=1.0, a2=1.0, a3=1.0 / 6.0, b0=0.0, b1=0.0, b2=0.0,
                           c0=1.0, c1=1.0, c2=1.0, bnd=1.0, wrk1=0.0)


def poisson19_inputs(shape_total=(257, 129, 129), values=None):
    """p and the 12 coefficient arrays as FP32 padded grids (z, y, x), the
    given shape including the 1-cell boundary.  p = k^2/(K-1)^2 with k the z
    storage index and K the z extent (exact in FP32 for K = 257)."""
    vals = dict(POISSON_COEF_VALUES)
    if values:
        vals.update(values)
    K = shape_total[0]
    k = np.arange(K, dtype=np.float64)
    prof = (k * k / float((K - 1) ** 2)).astype(np.float32)
    p = np.empty(shape_total, dtype=np.float32)
    p[...] = prof[:, None, None]
    coefs = [np.full(shape_total, np.float32(vals[name]), dtype=np.float32) for name in POISSON_COEF_ORDER]
    return p, coefs


def poisson19_random_inputs(shape_total, seed: int = 7):
    """A dense variant with every coefficient array random (for parity of
    every term, including the b cross terms that are 0 in the workload above):
    a*, c* in [0.5, 1.5), b* in [-0.25, 0.25), a3 in [0.1, 0.2), bnd in
    {0, 1}, wrk1 in [-0.01, 0.01), p in [0, 1).  Streams 0..12."""
    p = uniform_f32(seed, 0, shape_total)
    coefs = []
    for s, name in enumerate(POISSON_COEF_ORDER):
        u = uniform_f32(seed, 1 + s, shape_total)
        if name in ("a0", "a1", "a2", "c0", "c1", "c2"):
            c = np.float32(0.5) + u
        elif name in ("b0", "b1", "b2"):
            c = (u - np.float32(0.5)) * np.float32(0.5)
        elif name == "a3":
            c = np.float32(0.1) + u * np.float32(0.1)
        elif name == "bnd":
            c = (u < np.float32(0.9)).astype(np.float32)
        else:
            c = (u - np.float32(0.5)) * np.float32(0.02)
        coefs.append(np.ascontiguousarray(c, dtype=np.float32))
    return p, coefs


# --------------------------------------------------------------------------
# wave25: radius-4 25-point leapfrog wave update
WAVE25 = dict(n=512, T=10, seed=3)
WAVE25_COEF = (-2.847222, 1.6, -0.2, 0.025397, -0.001786)
WAVE25_COURANT_DT_OVER_H = 0.4 / 4.5


def wave25_inputs(nx: int, ny: int | None = None, nz: int | None = None, seed: int = 3):
    """(u_prev, u_cur, vsq) float64 padded grids with a 4-cell halo."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    shape = (nz + 8, ny + 8, nx + 8)
    v = 1.5 + 3.0 * uniform_f64(seed, 0, shape)
    vsq = v * WAVE25_COURANT_DT_OVER_H
    vsq *= vsq
    del v
    u = 1.0 + 0.1 * uniform_f64(seed, 1, shape)
    return u, u.copy(), vsq


# --------------------------------------------------------------------------
# generic stencils: seeded random corpus (star or box, radius 1..4)
GENERIC_CORPUS = dict(count=250, train=200, seed=5, edge_lo=64, edge_hi=512, T=4)
SHARING = ("distinct", "reflection", "symmetric", "partition")


def star_taps(r: int):
    """Centre, then for x, y, z: +q, -q for q = 1..r."""
    taps = [(0, 0, 0)]
    for ax in range(3):
        for q in range(1, r + 1):
            for s in (q, -q):
                d = [0, 0, 0]
                d[ax] = s
                taps.append(tuple(d))
    return taps


def box_taps(r: int):
    """All (dx, dy, dz) in [-r, r]^3, dz slowest, dx fastest."""
    return [(dx, dy, dz) for dz in range(-r, r + 1) for dy in range(-r, r + 1) for dx in range(-r, r + 1)]


def sharing_ids(taps, pattern: str, u_iter):
    """Coefficient id per tap for a sharing pattern (ids are dense 0..m-1)."""
    if pattern == "distinct":
        return list(range(len(taps))), len(taps)
    if pattern in ("reflection", "symmetric"):
        keys = {}
        ids = []
        for d in taps:
            if pattern == "reflection":
                k = max(d, tuple(-v for v in d))
            else:
                k = tuple(sorted(abs(v) for v in d))
            ids.append(keys.setdefault(k, len(keys)))
        return ids, len(keys)
    m = 1 + int(next(u_iter) * len(taps))
    m = min(m, len(taps))
    ids = [min(m - 1, int(next(u_iter) * m)) for _ in taps]
    used = sorted(set(ids))
    remap = {v: i for i, v in enumerate(used)}
    return [remap[v] for v in ids], len(used)


def generic_stencil(index: int, seed: int = 5, max_edge: int | None = None):
    """Stencil number `index` of the seeded corpus: a dict with radius, shape,
    dtype, interior n (x, y, z), taps, cids, coef.  Every draw comes from
    stream `index`: radius 1 + floor(4u); box if u < 0.5; F32 if u < 0.5;
    each edge 64 + floor(449u); sharing pattern floor(4u); coefficient values
    U(0.1, 1) per id, normalized so the taps' coefficients sum to 1.
    max_edge caps the grid (parity runs use a shrunken grid)."""
    u = iter(uniform_f64(seed, index, (4096,)))
    r = 1 + int(next(u) * 4)
    box = next(u) < 0.5
    dtype = "f32" if next(u) < 0.5 else "f64"
    n = [64 + int(next(u) * 449) for _ in range(3)]
    pattern = SHARING[int(next(u) * 4)]
    taps = box_taps(r) if box else star_taps(r)
    cids, m = sharing_ids(taps, pattern, u)
    vals = [0.1 + 0.9 * next(u) for _ in range(m)]
    total = sum(vals[c] for c in cids)
    coef = [v / total for v in vals]
    if max_edge is not None:
        n = [min(e, max_edge) for e in n]
    return dict(index=index, radius=r, shape="box" if box else "star", dtype=dtype, n=tuple(n),
                pattern=pattern, taps=taps, cids=cids, coef=coef)


def generic_input(n, r: int, dtype: str, seed: int = 5, stream: int = 1000):
    """U[0,1) padded grid (halo included) for a generic stencil."""
    shape = (n[2] + 2 * r, n[1] + 2 * r, n[0] + 2 * r)
    if dtype == "f32":
        return uniform_f32(seed, stream, shape)
    return uniform_f64(seed, stream, shape)


def mlp_init(seed: int = 5, stream: int = 7000):
    """Initial cost-model parameters (5825): weights U(-sqrt(6/fan_in),
    sqrt(6/fan_in)) in the layout W1 (64x24), b1, W2 (64x64), b2, w3, b3;
    biases 0."""
    u = uniform_f64(seed, stream, (24 * 64 + 64 * 64 + 64,))
    w1 = (2 * u[:1536] - 1) * np.sqrt(6 / 24)
    w2 = (2 * u[1536:1536 + 4096] - 1) * np.sqrt(6 / 64)
    w3 = (2 * u[1536 + 4096:] - 1) * np.sqrt(6 / 64)
    z = np.zeros(64)
    return np.concatenate([w1, z, w2, z, w3, [0.0]]).astype(np.float32)


# ---------------------------------------------------------------------------
# Pointwise programs (the saturator's input) and their inputs.
#
# A program is a dict: n_inputs, n_outputs, n_params, n_locals, radius, insns
# (postfix instructions (op, a, b, c, d), op codes as in include/saturator.h:
# 1 CONST, 2 PARAM, 3 LOAD, 4 ADD, 5 SUB, 6 MUL, 7 NEG, 8 STORE, 9 SET,
# 10 GET) and consts.  Written out by hand here: these are inputs, not
# arithmetic.

_CONST, _PARAM, _LOAD, _ADD, _SUB, _MUL, _NEG, _STORE, _SET, _GET = range(1, 11)

# Block-tridiagonal assembly of an implicit line solve along z (the shape of
# the paper's Listing lst:zsolve): for 5 x 5 blocks, with flux Jacobian F and
# viscous Jacobian N given per point, t1 = dt*tz1 and t2 = dt*tz2,
#   A[m][n] = -t2*F(k-1) - t1*N(k-1)            (- t1*dz[m]  on the diagonal)
#   B[m][n] = 2*t1*N(k)                         (+ 1 + 2*t1*dz[m] on the diagonal)
#   C[m][n] =  t2*F(k+1) - t1*N(k+1)            (- t1*dz[m]  on the diagonal)
# 75 statements, 125 loads.  Inputs: F[m][n] = array 5m+n, N[m][n] = array
# 25+5m+n; outputs A, B, C = arrays 5m+n, 25+5m+n, 50+5m+n; params dt, tz1,
# tz2, dz[0..4]; locals t1, t2.
LHS_PARAMS = (0.5, 1.0, 4.0, 0.1, 0.2, 0.3, 0.4, 0.5)  # dt, tz1, tz2, dz[0..4]
LHS_N = (162, 162, 162)


# The heat3d7 loop body as a program, written as the plain kernel reads it:
# u' = cc*u + cn*u(-x) + cn*u(+x) + cn*u(-y) + cn*u(+y) + cn*u(-z) + cn*u(+z),
# added left to right; params cc, cn; one input, one output.
def heat3d7_program():
    op = lambda o: (o, 0, 0, 0, 0)  # noqa: E731
    ins = [(_PARAM, 0, 0, 0, 0), (_LOAD, 0, 0, 0, 0), op(_MUL)]
    for d in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
        ins += [(_PARAM, 1, 0, 0, 0), (_LOAD, 0) + d, op(_MUL), op(_ADD)]
    ins.append((_STORE, 0, 0, 0, 0))
    return dict(n_inputs=1, n_outputs=1, n_params=2, n_locals=0, radius=1, insns=ins, consts=[])


def lhs_program():
    ins = [(_PARAM, 0, 0, 0, 0), (_PARAM, 1, 0, 0, 0), (_MUL, 0, 0, 0, 0), (_SET, 0, 0, 0, 0),
           (_PARAM, 0, 0, 0, 0), (_PARAM, 2, 0, 0, 0), (_MUL, 0, 0, 0, 0), (_SET, 1, 0, 0, 0)]
    t1, t2 = (_GET, 0, 0, 0, 0), (_GET, 1, 0, 0, 0)
    two, one = (_CONST, 0, 0, 0, 0), (_CONST, 1, 0, 0, 0)
    op = lambda o: (o, 0, 0, 0, 0)  # noqa: E731
    for m in range(5):  # A
        for n in range(5):
            ins += [t2, op(_NEG), (_LOAD, 5 * m + n, 0, 0, -1), op(_MUL),
                    t1, (_LOAD, 25 + 5 * m + n, 0, 0, -1), op(_MUL), op(_SUB)]
            if m == n:
                ins += [t1, (_PARAM, 3 + m, 0, 0, 0), op(_MUL), op(_SUB)]
            ins.append((_STORE, 5 * m + n, 0, 0, 0))
    for m in range(5):  # B
        for n in range(5):
            ins += [two, t1, op(_MUL), (_LOAD, 25 + 5 * m + n, 0, 0, 0), op(_MUL)]
            if m == n:
                ins += [one, two, t1, op(_MUL), (_PARAM, 3 + m, 0, 0, 0), op(_MUL), op(_ADD), op(_ADD)]
            ins.append((_STORE, 25 + 5 * m + n, 0, 0, 0))
    for m in range(5):  # C
        for n in range(5):
            ins += [t2, (_LOAD, 5 * m + n, 0, 0, 1), op(_MUL), t1, (_LOAD, 25 + 5 * m + n, 0, 0, 1), op(_MUL),
                    op(_SUB)]
            if m == n:
                ins += [t1, (_PARAM, 3 + m, 0, 0, 0), op(_MUL), op(_SUB)]
            ins.append((_STORE, 50 + 5 * m + n, 0, 0, 0))
    return dict(n_inputs=50, n_outputs=75, n_params=8, n_locals=2, radius=1, insns=ins, consts=[2.0, 1.0])


def lhs_inputs(n=LHS_N, seed: int = 11):
    """F = 1 + U[0,1) (streams 0..24), N = U[0,1) (streams 25..49) over the
    padded arrays (halo 1).  With tz2 = 4 tz1 every output is a sum of terms
    that cannot cancel by more than a factor of about 4."""
    nx, ny, nz = n
    shape = (nz + 2, ny + 2, nx + 2)
    out = []
    for s in range(50):
        u = uniform_f64(seed, s, shape)
        out.append(u + 1.0 if s < 25 else u)
    return out


def random_program(index: int, seed: int = 13, n_inputs: int = 4, n_outputs: int = 3, n_params: int = 3,
                   max_terms: int = 6, radius: int = 1):
    """A seeded random program: each output is a sum of products of two or
    three factors (loads at offsets within `radius`, parameters, constants
    from {2, 0.5, 3}), some sharing subexpressions with earlier statements;
    every value positive when inputs and parameters are, so no statement
    cancels.  Used to exercise the rewriting on shapes beyond the fixed
    workload."""
    u = splitmix64(seed, 9000 + index, 0, 4096)
    it = iter(((u >> np.uint64(11)).astype(np.float64) * 2.0 ** -53).tolist())
    pick = lambda k: min(k - 1, int(next(it) * k))  # noqa: E731
    consts = [2.0, 0.5, 3.0]
    ins = []

    def leaf():
        c = pick(3)
        if c == 0:
            return [(_LOAD, pick(n_inputs), pick(2 * radius + 1) - radius, pick(2 * radius + 1) - radius,
                     pick(2 * radius + 1) - radius)]
        if c == 1:
            return [(_PARAM, pick(n_params), 0, 0, 0)]
        return [(_CONST, pick(3), 0, 0, 0)]

    shared = leaf() + leaf() + [(_MUL, 0, 0, 0, 0)]
    for o in range(n_outputs):
        terms = 1 + pick(max_terms)
        for t in range(terms):
            f = (shared if pick(3) == 0 else leaf() + leaf() + [(_MUL, 0, 0, 0, 0)])
            if pick(2):
                f = f + leaf() + [(_MUL, 0, 0, 0, 0)]
            ins += f
            if t > 0:
                ins.append((_ADD, 0, 0, 0, 0))
        ins.append((_STORE, o, 0, 0, 0))
    return dict(n_inputs=n_inputs, n_outputs=n_outputs, n_params=n_params, n_locals=0, radius=radius, insns=ins,
                consts=consts)


# A VALU-bound generic stencil for measurement: FP64 box of radius 3 (343 taps)
# with the fully symmetric sharing pattern (one coefficient per sorted |delta|
# triple: 20 ids), coefficients U(0.1, 1) per id (seed 5, stream 900)
# normalized to sum 1 over the taps, on a 256^3 interior, 4 sweeps.
GENERIC_BOX_N = (256, 256, 256)


def generic_box_workload(r: int = 3):
    taps = box_taps(r)
    cids, m = sharing_ids(taps, "symmetric", iter(()))
    u = uniform_f64(5, 900, (m,))
    vals = [0.1 + 0.9 * float(v) for v in u]
    total = sum(vals[c] for c in cids)
    return dict(radius=r, taps=taps, cids=cids, coef=[v / total for v in vals], dtype="f64", n=GENERIC_BOX_N)
