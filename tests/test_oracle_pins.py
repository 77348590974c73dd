"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test targets a class of plausible mistakes (a dropped term, a wrong sign,
a wrong or transposed index, a wrong coefficient, a wrong update order):

* closed forms (harmonic fixed points, quadratic light cones, the pressure
  sweep's first-iteration residual, the leapfrog polynomial solution);
* library routines the special cases reduce to (scipy.ndimage.correlate,
  uniform_filter, a Kronecker-sum sparse operator built from 1-D matrices);
* invariants (periodic conservation, the maximum principle);
* exact rational arithmetic (fractions) on small inputs;
* impulse responses that expose every tap's offset and weight.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.ndimage as ndi
import scipy.sparse as sp

import oracle
from paper_2306_13002_amd import synth

EPS = np.finfo(np.float64).eps


def interior(a, r):
    return a[tuple(slice(r, s - r) for s in a.shape)]


def light_cone_mask(shape_interior, t, reach=1):
    """True where the point's distance to the halo d >= reach*(t-1)."""
    idx = np.indices(shape_interior)
    d = np.min([np.minimum(idx[a], shape_interior[a] - 1 - idx[a]) for a in range(len(shape_interior))], axis=0)
    return d >= reach * (t - 1)


# ---------------------------------------------------------------- heat
@pytest.mark.parametrize("T", [1, 4])
def test_heat2d5_harmonic_fixed_point(T):
    # x^2 - y^2 has zero discrete Laplacian, so a weighted average with weights
    # summing to 1 leaves it unchanged (halo = the same field).
    y, x = np.indices((14, 19)).astype(np.float64)
    u = x * x - y * y
    out, _ = oracle.heat(u, T, 0.6, 0.1)
    assert np.max(np.abs(out - u)) <= 8 * T * EPS * np.max(np.abs(u))


@pytest.mark.parametrize("field", ["xyz", "x2+y2-2z2"])
def test_heat3d7_harmonic_fixed_point(field):
    z, y, x = np.indices((9, 11, 13)).astype(np.float64)
    u = x * y * z if field == "xyz" else x * x + y * y - 2 * z * z
    out, _ = oracle.heat(u, 3, 0.4, 0.1)
    assert np.max(np.abs(out - u)) <= 8 * 3 * EPS * np.max(np.abs(u))


@pytest.mark.parametrize("ndim,cc,step", [(2, 0.6, 0.4), (3, 0.4, 0.6)])
def test_heat_quadratic_light_cone(ndim, cc, step):
    # u = x^2 + y^2 (+ z^2): sum of face neighbours = 2*ndim*u + 2*ndim, so one
    # sweep adds 2*ndim*cn exactly where no stale halo value was seen.
    shape = (12, 15) if ndim == 2 else (10, 11, 12)
    idx = np.indices(shape).astype(np.float64)
    u = sum(c * c for c in idx)
    for T in (1, 2, 3, 4):
        out, _ = oracle.heat(u, T, cc, 0.1)
        m = light_cone_mask(tuple(s - 2 for s in shape), T)
        got = interior(out, 1)[m]
        want = interior(u, 1)[m] + T * step
        np.testing.assert_allclose(got, want, rtol=1e-14, atol=0)
        # and outside the cone the stale halo must have been seen somewhere
        if T >= 3:
            assert not np.allclose(interior(out, 1)[~m], interior(u, 1)[~m] + T * step, rtol=1e-14)


def test_heat2d5_impulse_response():
    u = np.zeros((9, 9))
    u[4, 4] = 1.0
    out, _ = oracle.heat(u, 1, 0.6, 0.1)
    want = np.zeros((9, 9))
    want[4, 4] = 0.6
    for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
        want[4 + dy, 4 + dx] = 0.1
    assert np.array_equal(out, want)


def test_heat3d7_impulse_response():
    u = np.zeros((7, 8, 9))
    u[3, 4, 5] = 1.0
    out, _ = oracle.heat(u, 1, 0.4, 0.1)
    want = np.zeros_like(u)
    want[3, 4, 5] = 0.4
    for d in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        want[3 + d[0], 4 + d[1], 5 + d[2]] = 0.1
    assert np.array_equal(out, want)


@pytest.mark.parametrize("ndim", [2, 3])
def test_heat_matches_scipy_correlate(ndim):
    # One sweep is a correlation with the 3^ndim weight kernel; T sweeps with a
    # fixed halo re-impose the halo after each correlation.
    shape = (21, 17) if ndim == 2 else (11, 13, 10)
    rng = np.random.default_rng(3)
    u0 = rng.random(shape)
    cc = 0.6 if ndim == 2 else 0.4
    w = np.zeros((3,) * ndim)
    c = (1,) * ndim
    w[c] = cc
    for a in range(ndim):
        for s in (0, 2):
            i = list(c)
            i[a] = s
            w[tuple(i)] = 0.1
    ref = u0.copy()
    for _ in range(5):
        nxt = ndi.correlate(ref, w, mode="constant", cval=0.0)
        ref_int = interior(ref, 1)
        ref_int[...] = interior(nxt, 1)
    out, res = oracle.heat(u0, 5, cc, 0.1)
    np.testing.assert_allclose(interior(out, 1), interior(ref, 1), rtol=1e-13)
    assert np.array_equal(out[0], u0[0])  # halo untouched


def _kron_sum_operator(n_int, cc, cn):
    """Sparse matrix of one Dirichlet-0 heat sweep on the interior, built as
    cc*I + cn*(sum over axes of I (x) S (x) I) with S the 1-D neighbour-sum
    matrix (ones on the first off-diagonals).  Axis order follows the C-order
    flattening (z, y, x)."""
    mats = [sp.identity(n, format="csr") for n in n_int]
    ops = []
    for a, n in enumerate(n_int):
        S = sp.diags([np.ones(n - 1), np.ones(n - 1)], [-1, 1], format="csr")
        facs = [S if b == a else mats[b] for b in range(len(n_int))]
        k = facs[0]
        for f in facs[1:]:
            k = sp.kron(k, f, format="csr")
        ops.append(k)
    N = int(np.prod(n_int))
    return cc * sp.identity(N, format="csr") + cn * sum(ops)


@pytest.mark.parametrize("n_int", [(4, 4), (3, 4, 5)])
def test_heat_exact_rational_small(n_int):
    # Brute force on tiny grids: apply the Kronecker-sum operator T times in
    # exact rationals (coefficients = their FP64 values) and compare.
    ndim = len(n_int)
    cc = 0.6 if ndim == 2 else 0.4
    A = _kron_sum_operator(n_int, cc, 0.1).toarray()
    Afrac = [[Fraction(v) for v in row] for row in A]
    rng = np.random.default_rng(11)
    u0 = np.zeros(tuple(n + 2 for n in n_int))
    interior(u0, 1)[...] = rng.random(n_int)
    vec = [Fraction(v) for v in interior(u0, 1).ravel()]
    T = 3
    for _ in range(T):
        vec = [sum((a * b for a, b in zip(row, vec)), Fraction(0)) for row in Afrac]
    out, _ = oracle.heat(u0, T, cc, 0.1)
    got = interior(out, 1).ravel()
    want = np.array([float(v) for v in vec])
    np.testing.assert_allclose(got, want, rtol=8 * T * EPS * 7)


def test_heat_periodic_conservation():
    rng = np.random.default_rng(5)
    for shape, cc in (((12, 18), 0.6), ((8, 10, 12), 0.4)):
        u0 = rng.random(shape)
        T = 7
        out, _ = oracle.heat(u0, T, cc, 0.1, periodic=True)
        s0, s1 = interior(u0, 1).sum(), interior(out, 1).sum()
        N = interior(u0, 1).size
        assert abs(s1 - s0) <= T * N * EPS * 4
        # periodic run is a circular correlation of the interior
        w = np.zeros((3,) * len(shape))
        c = (1,) * len(shape)
        w[c] = cc
        for a in range(len(shape)):
            for s in (0, 2):
                i = list(c)
                i[a] = s
                w[tuple(i)] = 0.1
        ref = interior(u0, 1).copy()
        for _ in range(T):
            ref = ndi.correlate(ref, w, mode="wrap")
        np.testing.assert_allclose(interior(out, 1), ref, rtol=1e-13)


def test_heat2d5_maximum_principle_workload():
    u0 = synth.heat2d5_input(64)
    mx = u0.max()
    for T in (1, 5, 10):
        out, _ = oracle.heat(u0, T, 0.6, 0.1)
        assert out.min() >= 0.0 and out.max() <= mx


def test_heat_residual_definition():
    rng = np.random.default_rng(9)
    u0 = rng.random((8, 9, 10))
    u3, r3 = oracle.heat(u0, 3, 0.4, 0.1)
    u4, r4 = oracle.heat(u0, 4, 0.4, 0.1)
    d = interior(u4, 1) - interior(u3, 1)
    np.testing.assert_allclose(r4, np.sum(d * d), rtol=1e-12)
    _, r0 = oracle.heat(u0, 0, 0.4, 0.1)
    assert r0 == 0.0


# ---------------------------------------------------------------- poisson19
def _poisson_ss_closed_form(k):
    """First sweep on the workload inputs, derived by hand: a = c = 1, b = 0,
    wrk1 = 0, p = k^2/2^16, a3 = fl32(1/6) = 11184811*2^-26 give
    s0 = (6k^2 + 2)/2^16 and, since 6*11184811 = 2^26 + 2,
    ss(k) = (2k^2 + 22369622) * 2^-42 exactly."""
    return Fraction(2 * k * k + 22369622, 2 ** 42)


def test_poisson19_first_iteration_closed_form():
    p, coefs = synth.poisson19_inputs((257, 9, 9))
    assert float(coefs[3][0, 0, 0]) == 11184811 * 2.0 ** -26
    out, gosa = oracle.poisson19(p, coefs, 0.8, 1, mode="F64")
    ks = np.arange(1, 256)
    ss = np.array([float(_poisson_ss_closed_form(int(k))) for k in ks])
    want_p = (ks * ks / 65536.0)[:, None, None] + 0.8 * ss[:, None, None]
    np.testing.assert_allclose(interior(out, 1), np.broadcast_to(want_p, (255, 7, 7)), rtol=1e-15)
    exact = 49 * sum(_poisson_ss_closed_form(int(k)) ** 2 for k in ks)
    assert abs(gosa - float(exact)) <= 1e-10 * float(exact)


def test_poisson19_first_iteration_closed_form_full_size():
    # the full 129 x 129 x 257 workload: gosa_1 = 127^2 * sum_k ss(k)^2
    p, coefs = synth.poisson19_inputs()
    _, gosa = oracle.poisson19(p, coefs, 0.8, 1, mode="F64")
    exact = 127 * 127 * sum(_poisson_ss_closed_form(k) ** 2 for k in range(1, 256))
    assert abs(gosa - float(exact)) <= 1e-10 * float(exact)
    assert abs(float(exact) - 1.0681643715818605e-4) <= 1e-16


def test_poisson19_one_dimensional_reduction_exact():
    # Where the i/j boundary has not been felt (light cone), p depends on k
    # only and follows q_t(k) = q(k) + w*(a3*(4q(k) + q(k+1) + q(k-1)) - q(k)),
    # computed here in exact rationals.
    K, nxy, T = 65, 21, 8
    p, coefs = synth.poisson19_inputs((K, nxy, nxy))
    a3 = Fraction(float(coefs[3][0, 0, 0]))
    w = Fraction(0.8)
    q = [Fraction(k * k, (K - 1) ** 2) for k in range(K)]
    for t in range(1, T + 1):
        q = [q[0]] + [q[k] + w * (a3 * (4 * q[k] + q[k + 1] + q[k - 1]) - q[k]) for k in range(1, K - 1)] + [q[-1]]
        out, _ = oracle.poisson19(p, coefs, 0.8, t, mode="F64")
        inner = interior(out, 1)  # (K-2, nxy-2, nxy-2)
        n = nxy - 2
        for j in range(n):
            for i in range(n):
                if min(i, j, n - 1 - i, n - 1 - j) >= t - 1:
                    got = inner[:, j, i]
                    want = np.array([float(v) for v in q[1:K - 1]])
                    np.testing.assert_allclose(got, want, rtol=1e-13)


# tap table of the pressure operator: (dx, dy, dz, coefficient name, sign)
_P19_TAPS = [
    (1, 0, 0, "a0", 1), (0, 1, 0, "a1", 1), (0, 0, 1, "a2", 1),
    (1, 1, 0, "b0", 1), (1, -1, 0, "b0", -1), (-1, 1, 0, "b0", -1), (-1, -1, 0, "b0", 1),
    (0, 1, 1, "b1", 1), (0, -1, 1, "b1", -1), (0, 1, -1, "b1", -1), (0, -1, -1, "b1", 1),
    (1, 0, 1, "b2", 1), (-1, 0, 1, "b2", -1), (1, 0, -1, "b2", -1), (-1, 0, -1, "b2", 1),
    (-1, 0, 0, "c0", 1), (0, -1, 0, "c1", 1), (0, 0, -1, "c2", 1),
]


def test_poisson19_impulse_response():
    # Distinct power-of-two coefficients make every response exact and
    # different, so a wrong offset, sign or coefficient is visible.
    shape = (9, 9, 9)
    vals = dict(a0=2.0 ** -1, a1=2.0 ** -2, a2=2.0 ** -3, a3=2.0 ** -4, b0=2.0 ** -5, b1=2.0 ** -6,
                b2=2.0 ** -7, c0=2.0 ** -8, c1=2.0 ** -9, c2=2.0 ** -10, bnd=1.0, wrk1=0.0)
    p = np.zeros(shape, dtype=np.float32)
    p[4, 4, 4] = 1.0
    coefs = [np.full(shape, vals[n], dtype=np.float32) for n in synth.POISSON_COEF_ORDER]
    w = 0.5
    out, gosa = oracle.poisson19(p, coefs, w, 1, mode="F64")
    want = np.zeros(shape)
    want[4, 4, 4] = 1.0 - w  # s0 = 0 at the impulse, ss = -1
    ss2 = 1.0
    for dx, dy, dz, name, sgn in _P19_TAPS:
        # point x reads p(x + d) = impulse  =>  x = impulse - d
        v = sgn * vals[name] * vals["a3"]
        want[4 - dz, 4 - dy, 4 - dx] = w * v
        ss2 += v * v
    assert np.array_equal(out, want)
    assert gosa == ss2


def test_poisson19_boundary_mask_and_source_term():
    # p = 0: s0 = wrk1, so ss = wrk1*a3*bnd and p' = w*ss exactly (powers of
    # two); where bnd = 0 the point must keep its value whatever the
    # neighbours are.
    shape = (8, 9, 10)
    rng = np.random.default_rng(21)
    bnd = (rng.random(shape) < 0.5).astype(np.float32)
    wrk = np.float32(2.0 ** -3) * (1 + (rng.random(shape) < 0.5)).astype(np.float32)
    vals = dict(a0=0.5, a1=0.5, a2=0.5, a3=0.25, b0=0.125, b1=0.125, b2=0.125, c0=0.5, c1=0.5, c2=0.5)
    coefs = []
    for n in synth.POISSON_COEF_ORDER:
        coefs.append(bnd if n == "bnd" else wrk if n == "wrk1" else np.full(shape, vals[n], np.float32))
    out, gosa = oracle.poisson19(np.zeros(shape, np.float32), coefs, 0.5, 1, mode="F64")
    want = 0.5 * (wrk.astype(np.float64) * 0.25 * bnd)
    np.testing.assert_array_equal(interior(out, 1), interior(want, 1))
    ss = interior(wrk.astype(np.float64) * 0.25 * bnd, 1)
    assert gosa == pytest.approx(np.sum(ss * ss), rel=1e-15)
    # random field, bnd mask: masked points are unchanged after many sweeps
    p = synth.uniform_f32(5, 0, shape)
    coefs2 = [np.full(shape, vals.get(n, 0.0), np.float32) for n in synth.POISSON_COEF_ORDER]
    coefs2[10] = bnd
    out2, _ = oracle.poisson19(p, coefs2, 0.8, 4, mode="F64")
    m = interior(bnd, 1) == 0
    assert np.array_equal(interior(out2, 1)[m], interior(p, 1).astype(np.float64)[m])
    assert not np.array_equal(interior(out2, 1)[~m], interior(p, 1).astype(np.float64)[~m])


def test_poisson19_f32store_rounds_state():
    p, coefs = synth.poisson19_random_inputs((12, 11, 10), seed=3)
    o64, g64 = oracle.poisson19(p, coefs, 0.8, 3, mode="F64")
    o32, g32 = oracle.poisson19(p, coefs, 0.8, 3, mode="F32STORE")
    assert np.array_equal(o32, o32.astype(np.float32).astype(np.float64))
    np.testing.assert_allclose(interior(o32, 1), interior(o64, 1), rtol=1e-6, atol=1e-7)
    assert abs(g32 - g64) <= 1e-4 * g64


def _round_f32(x: Fraction) -> Fraction:
    """x rounded to the nearest float32 (ties to even), as an exact rational:
    the float32 candidates around a first guess are compared exactly, so no
    double rounding through float64 can creep in."""
    f = np.float32(float(x))
    cands = [f, np.nextafter(f, np.float32(np.inf)), np.nextafter(f, np.float32(-np.inf))]
    best = None
    for c in cands:
        d = abs(Fraction(float(c)) - x)
        even = (int(np.array(c, np.float32).view(np.uint32)) & 1) == 0
        if best is None or d < best[0] or (d == best[0] and even):
            best = (d, c)
    return Fraction(float(best[1]))


def test_poisson19_f32store_one_dimensional_reduction_exact():
    # F32 storage rounds the state after EVERY sweep: inside the light cone
    # the F32STORE run follows q_t = fl32(q + w*(a3*(4q(k) + q(k+1) + q(k-1)) - q)),
    # fl32 a correct rounding to float32 of the exact rational.  With a3 = 1/8
    # and w = 3/4 every FP64 operation of a sweep on float32 data is exact
    # (at most ~30 significant bits), so FP64 arithmetic followed by the store
    # rounding IS that correct rounding.  (With w = 0.8 the exact value can sit
    # on a float32 tie that FP64 rounding of w*ss breaks differently.)  A state
    # rounded only once at the end, or only on input, drifts off this
    # recurrence by float32 ulps from the second sweep on.
    K, nxy, T = 65, 13, 6
    p, coefs = synth.poisson19_inputs((K, nxy, nxy), values=dict(a3=0.125))
    a3 = Fraction(1, 8)
    w = Fraction(3, 4)
    q = [Fraction(k * k, (K - 1) ** 2) for k in range(K)]
    assert all(_round_f32(v) == v for v in q)  # the initial state is exact in float32
    n = nxy - 2
    rounded = 0
    for t in range(1, T + 1):
        nq = [q[0]]
        for k in range(1, K - 1):
            v = q[k] + w * (a3 * (4 * q[k] + q[k + 1] + q[k - 1]) - q[k])
            nq.append(_round_f32(v))
            rounded += nq[-1] != v
        q = nq + [q[-1]]
        out, _ = oracle.poisson19(p, coefs, 0.75, t, mode="F32STORE")
        want = np.array([float(v) for v in q[1:K - 1]])
        inner = interior(out, 1)
        for j in range(n):
            for i in range(n):
                if min(i, j, n - 1 - i, n - 1 - j) >= t - 1:
                    assert np.array_equal(inner[:, j, i], want), (t, j, i)
    assert rounded > (K - 2) * T // 4  # the store rounding really acts (136 of 378 updates)


@pytest.mark.parametrize("T", [1, 2, 3, 4])
def test_poisson19_f32store_is_one_rounding_per_sweep(T):
    # T sweeps in F32STORE mode = T times (one FP64 sweep, then round the
    # state to float32), and the residual is that of the last such sweep.
    # Random coefficients, b terms nonzero.
    p, coefs = synth.poisson19_random_inputs((12, 11, 10), seed=4)
    assert any(np.any(coefs[i] != 0) for i in (4, 5, 6))
    state = p.astype(np.float64)
    g1 = None
    for _ in range(T):
        one, g1 = oracle.poisson19(state, coefs, 0.8, 1, mode="F64")
        state = one.astype(np.float32).astype(np.float64)
    o32, g32 = oracle.poisson19(p, coefs, 0.8, T, mode="F32STORE")
    assert np.array_equal(o32, state)
    assert g32 == g1


def _dyadic_generic(r, box, seed):
    """Taps, ids and coefficients for the float32-storage pins: coefficients
    are multiples of 2^-8 summing to about 1, the field lies in [0.5, 1] and
    is float32.  Every product then has at most 32 significant bits and every
    partial sum stays far inside float64's 53, so any summation order gives
    the exact value and only the float32 store rounds."""
    rng = np.random.default_rng(seed)
    taps = synth.box_taps(r) if box else synth.star_taps(r)
    m = max(1, len(taps) // 3)
    cid = rng.integers(0, m, size=len(taps)).astype(np.int32)
    n_c = rng.integers(1, 9, size=m)
    total = sum(int(n_c[c]) for c in cid)
    coef = np.array([max(1, round(int(v) * 256 / total)) / 256.0 for v in n_c])
    shape = (2 * r + 6, 2 * r + 5, 2 * r + 7)
    u0 = (0.5 + 0.5 * synth.uniform_f32(seed, 0, shape)).astype(np.float32)
    return np.array(taps, np.int32), cid, coef, u0


@pytest.mark.parametrize("r,box", [(2, True), (4, False)])
def test_generic_f32store_matches_correlate_rounded_per_sweep(r, box):
    # Independent of the oracle: scipy's correlate (exact here, see
    # _dyadic_generic) followed by a float32 rounding of the interior after
    # every sweep; the halo keeps its float32 values.
    taps, cid, coef, u0 = _dyadic_generic(r, box, 40 + r)
    k = np.zeros((2 * r + 1,) * 3)
    for (dx, dy, dz), c in zip(taps, cid):
        k[dz + r, dy + r, dx + r] += coef[c]
    ref = u0.astype(np.float64)
    for T in (1, 2, 3):
        nxt = ndi.correlate(ref, k, mode="constant")
        interior(ref, r)[...] = interior(nxt, r).astype(np.float32).astype(np.float64)
        out, res = oracle.generic(u0, r, taps, cid, coef, T, mode="F32STORE")
        assert np.array_equal(out, ref), T


@pytest.mark.parametrize("r,box", [(2, True), (4, False)])
@pytest.mark.parametrize("T", [1, 2, 3, 4])
def test_generic_f32store_is_one_rounding_per_sweep(r, box, T):
    # T sweeps in F32STORE mode = T times (one FP64 sweep, then round to
    # float32), with random (non-dyadic) coefficients; the residual is that of
    # the stored (rounded) states of the last sweep.
    rng = np.random.default_rng(60 + r)
    taps = np.array(synth.box_taps(r) if box else synth.star_taps(r), np.int32)
    m = max(1, len(taps) // 4)
    cid = rng.integers(0, m, size=len(taps)).astype(np.int32)
    coef = rng.random(m)
    coef = coef / sum(coef[c] for c in cid)
    u0 = synth.uniform_f32(7, r, (2 * r + 5, 2 * r + 6, 2 * r + 4))
    state = u0.astype(np.float64)
    prev = state
    for _ in range(T):
        one, _ = oracle.generic(state, r, taps, cid, coef, 1, mode="F64")
        prev, state = state, one.astype(np.float32).astype(np.float64)
    out, res = oracle.generic(u0, r, taps, cid, coef, T, mode="F32STORE")
    assert np.array_equal(out, state)
    d = interior(state, r) - interior(prev, r)
    assert abs(res - np.sum(d * d)) <= 1e-13 * res


# ---------------------------------------------------------------- wave25
def test_wave25_impulse_response():
    c = synth.WAVE25_COEF
    shape = (19, 18, 17)
    o = (9, 9, 8)
    a = np.zeros(shape)
    b = np.zeros(shape)
    b[o] = 1.0
    v = np.ones(shape)
    A, B, _ = oracle.wave25(a, b, v, c, 1)
    want = np.zeros(shape)
    want[o] = 2.0 + ((c[0] + c[0]) + c[0])
    for r in range(1, 5):
        for d in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
            for s in (1, -1):
                want[o[0] + s * r * d[0], o[1] + s * r * d[1], o[2] + s * r * d[2]] = c[r]
    assert np.array_equal(A, want)
    assert np.array_equal(B, b)


def test_wave25_polynomial_closed_form():
    # u^{-1} = u^0 = P quadratic, vsq constant: L(P) is the constant
    # M2 * (sum of the quadratic's axis weights) (up to the tiny FP64 residue
    # of c0 + 2 sum c_r), so u^n = P + vsq*L(P)*n(n+1)/2 inside the light cone
    # d >= 4(n-1) of the fixed halo.
    c = synth.WAVE25_COEF
    cr = [Fraction(str(x)) for x in c]
    M2 = 2 * sum(cr[r] * r * r for r in range(1, 5))
    assert M2 == Fraction("1.999994")
    shape = (30, 29, 28)
    z, y, x = np.indices(shape).astype(np.float64)
    P = x * x + 2 * y * y + 3 * z * z
    vsq = 0.01
    V = np.full(shape, vsq)
    LP = float(M2 * 6)
    for T in (1, 2, 3):
        A, B, _ = oracle.wave25(P, P, V, c, T)
        newest = A if T % 2 == 1 else B
        m = light_cone_mask((22, 21, 20), T, reach=4)
        got = interior(newest, 4)[m]
        want = interior(P, 4)[m] + vsq * LP * T * (T + 1) / 2
        np.testing.assert_allclose(got, want, rtol=2e-14)


def test_wave25_constant_field():
    shape = (14, 15, 16)
    u = np.full(shape, 1.25)
    A, B, res = oracle.wave25(u, u, np.full(shape, 0.02), synth.WAVE25_COEF, 4)
    np.testing.assert_allclose(A, 1.25, rtol=1e-14)
    np.testing.assert_allclose(B, 1.25, rtol=1e-14)
    assert res < 1e-25


def test_wave25_laplacian_matches_scipy():
    # the 25-point operator is a correlation with an axis-cross kernel
    c = synth.WAVE25_COEF
    rng = np.random.default_rng(4)
    shape = (18, 19, 20)
    a = rng.random(shape)
    b = rng.random(shape)
    vsq = rng.random(shape) * 0.02
    k = np.zeros((9, 9, 9))
    k[4, 4, 4] = 3 * c[0]
    for r in range(1, 5):
        for s in (-r, r):
            k[4 + s, 4, 4] = c[r]
            k[4, 4 + s, 4] = c[r]
            k[4, 4, 4 + s] = c[r]
    L = ndi.correlate(b, k, mode="constant")
    want = interior(2 * b - a + vsq * L, 4)
    A, B, res = oracle.wave25(a, b, vsq, c, 1)
    np.testing.assert_allclose(interior(A, 4), want, rtol=1e-13)
    assert np.array_equal(B, b)
    assert np.array_equal(A[:4], a[:4]) and np.array_equal(A[:, :, -4:], a[:, :, -4:])
    d = want - interior(b, 4)
    np.testing.assert_allclose(res, np.sum(d * d), rtol=1e-12)


def test_wave25_restart_composes():
    rng = np.random.default_rng(8)
    shape = (14, 14, 14)
    a = 1 + 0.1 * rng.random(shape)
    b = 1 + 0.1 * rng.random(shape)
    v = 0.02 * np.ones(shape)
    A5, B5, r5 = oracle.wave25(a, b, v, synth.WAVE25_COEF, 5)
    A2, B2, _ = oracle.wave25(a, b, v, synth.WAVE25_COEF, 2)
    A3, B3, r3 = oracle.wave25(A2, B2, v, synth.WAVE25_COEF, 3)
    assert np.array_equal(A5, A3) and np.array_equal(B5, B3) and r5 == r3


# ---------------------------------------------------------------- generic
def _random_taps(rng, r, box):
    offs = []
    for dz in range(-r, r + 1):
        for dy in range(-r, r + 1):
            for dx in range(-r, r + 1):
                nz = (dx != 0) + (dy != 0) + (dz != 0)
                if box or nz <= 1:
                    offs.append((dx, dy, dz))
    offs = np.array(offs, dtype=np.int32)
    rng.shuffle(offs)
    return offs


@pytest.mark.parametrize("r,box", [(1, False), (2, True), (3, False), (4, False), (1, True)])
def test_generic_matches_scipy_correlate(r, box):
    rng = np.random.default_rng(100 + r)
    offs = _random_taps(rng, r, box)
    m = max(1, len(offs) // 3)
    cid = rng.integers(0, m, size=len(offs)).astype(np.int32)
    coef = rng.random(m) * 0.1
    k = np.zeros((2 * r + 1,) * 3)
    for (dx, dy, dz), c in zip(offs, cid):
        k[dz + r, dy + r, dx + r] += coef[c]
    shape = (2 * r + 7, 2 * r + 6, 2 * r + 9)
    u0 = rng.random(shape)
    ref = u0.copy()
    T = 2
    for _ in range(T):
        nxt = ndi.correlate(ref, k, mode="constant")
        interior(ref, r)[...] = interior(nxt, r)
    out, res = oracle.generic(u0, r, offs, cid, coef, T)
    np.testing.assert_allclose(interior(out, r), interior(ref, r), rtol=1e-12)
    assert np.array_equal(out[:r], u0[:r])


def test_generic_box_single_coefficient_is_box_sum():
    r = 2
    rng = np.random.default_rng(6)
    offs = _random_taps(rng, r, True)
    shape = (13, 12, 11)
    u0 = rng.random(shape)
    out, _ = oracle.generic(u0, r, offs, np.zeros(len(offs), np.int32), [0.25], 1)
    box = ndi.uniform_filter(u0, size=2 * r + 1, mode="constant") * (2 * r + 1) ** 3 * 0.25
    np.testing.assert_allclose(interior(out, r), interior(box, r), rtol=1e-12)


def test_generic_star1_equals_heat3d7():
    offs = np.array([(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)], np.int32)
    cid = np.array([0, 1, 1, 1, 1, 1, 1], np.int32)
    rng = np.random.default_rng(12)
    u0 = rng.random((9, 10, 11))
    g, rg = oracle.generic(u0, 1, offs, cid, [0.4, 0.1], 4)
    h, rh = oracle.heat(u0, 4, 0.4, 0.1)
    assert np.array_equal(g, h) and rg == rh


# ---------------------------------------------------------------- generator
def test_splitmix64_matches_sequential_definition():
    # the counter form equals the sequential generator (state += gamma, then
    # the output mix) started from state = seed*2^16 + stream
    M = (1 << 64) - 1

    def seq(state, n):
        out = []
        for _ in range(n):
            state = (state + 0x9E3779B97F4A7C15) & M
            z = state
            z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
            z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
            out.append(z ^ (z >> 31))
        return out

    for seed, stream in ((1, 0), (3, 1), (4, 17)):
        got = synth.splitmix64(seed, stream, 0, 50)
        assert [int(v) for v in got] == seq((seed << 16) + stream, 50)
        assert [int(v) for v in synth.splitmix64(seed, stream, 20, 5)] == seq((seed << 16) + stream, 25)[20:]


def test_uniform_ranges_and_moments():
    u = synth.uniform_f64(2, 0, (1 << 16,))
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.01 and abs(u.var() - 1 / 12) < 0.005
    f = synth.uniform_f32(2, 0, (1 << 12,))
    assert f.dtype == np.float32 and f.min() >= 0 and f.max() < 1
