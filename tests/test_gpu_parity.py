"""GPU parity: every kind x form x launch shape against the CPU oracle, through
the C ABI (libstencil.so), on seeded inputs.

Bars: plain forms are bit-identical to the oracle (same operations, same
order, no contraction).  Saturated F64 forms: max relative error <= 1e-12.
POISSON19 (F32 storage): p within 1e-5 of the F64 oracle, residual within
1e-5 of the F32STORE oracle.  Residuals of F64 kinds: relative 1e-10
(different summation order).  The halo is bit-identical to the input; the
scratch grid starts as NaN so any read of an unsynchronised cell shows.
"""
import numpy as np
import pytest

import oracle
from paper_2306_13002_amd import synth
from gpu_util import compare_region, crop_box, inner, maxrel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PLAIN_TILES = [(64, 4, 1), (64, 2, 2), (128, 2, 1), (256, 1, 1), (32, 8, 1), (64, 8, 1)]
HEAT_SAT_TILES = [(32, 2), (32, 4), (32, 8), (32, 16), (32, 20), (32, 24), (32, 28), (64, 1), (64, 2), (64, 4), (64, 8), (128, 1), (128, 2), (128, 4),
                  (256, 1), (256, 2)]
P19_SAT_TILES = [(32, 2), (32, 4), (32, 8), (64, 1), (64, 2), (64, 4), (64, 8), (128, 1), (128, 2), (128, 4), (128, 8),
                 (256, 1), (256, 4)]
P19_SAT2_TILES = [(32, 4), (32, 8), (64, 4), (64, 8), (128, 4)]
W25_SAT_TILES = [(64, 4), (64, 8), (64, 16), (64, 32), (32, 8), (32, 16), (128, 4), (128, 8), (128, 16), (256, 4),
                 (256, 8)]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def Plan(*a, **k):
    from paper_2306_13002_amd.stencil import Plan as P
    return P(*a, **k)


def _dev(a, dev):
    return torch.tensor(np.ascontiguousarray(a), device=dev)


def _nan_like(a, dev):
    return torch.full(a.shape, float("nan"), dtype=torch.float64 if a.dtype == np.float64 else torch.float32,
                      device=dev)


def run_jacobi(kind, u0, n, dev, T, coef=None, coefs=None, **kw):
    p = Plan(kind, n, coef=coef, **kw)
    f = [_dev(u0, dev), _nan_like(u0, dev)]
    cs = [_dev(c, dev) for c in coefs] if coefs is not None else None
    p.run(f, cs, iterations=T)
    res = p.residual() if T > 0 else None
    out = f[0].cpu().numpy()
    p.close()
    return out, res


# ---------------------------------------------------------------- heat2d5
@pytest.mark.parametrize("n,T", [((37, 29), 3), ((1, 1), 2), ((256, 256), 10), ((65, 3), 5)])
@pytest.mark.parametrize("tile", [(64, 4, 1), (256, 1, 1), (32, 8, 1)])
def test_heat2d5_plain_bitwise(dev, n, T, tile):
    u0 = synth.heat2d5_input(n[0], ny=n[1])
    want, wr = oracle.heat(u0, T, 0.6, 0.1)
    got, gr = run_jacobi("heat2d5", u0, n, dev, T, coef=(0.6, 0.1), variant="plain", tile=tile)
    assert np.array_equal(got, want)
    assert abs(gr - wr) <= 1e-10 * wr


def test_heat2d5_workload_full(dev):
    # the 256 x 256, T = 10 workload at its launch configuration
    u0 = synth.heat2d5_input(256)
    want, wr = oracle.heat(u0, 10, 0.6, 0.1)
    got, gr = run_jacobi("heat2d5", u0, (256, 256), dev, 10, coef=(0.6, 0.1), variant="plain")
    assert np.array_equal(got, want)
    assert abs(gr - wr) <= 1e-10 * wr
    assert got.min() >= 0 and got.max() <= u0.max()


@pytest.mark.parametrize("n", [(37, 29), (256, 256), (1, 1), (65, 3), (33, 17)])
@pytest.mark.parametrize("tile", [(16, 16, 2), (16, 16, 5), (16, 16, 8), (12, 12, 10), (22, 22, 5), (28, 28, 2),
                                  (3, 3, 4), (32, 32, 3), (32, 32, 10), (32, 32, 16), (16, 16, 9)])
def test_heat2d5_fused_sweeps_bitwise(dev, n, tile):
    # k sweeps per launch over a k-cell ring (one region cell per thread when
    # OT + 2k <= 32, else from a 16 x 16-thread LDS tile): the grid equals the
    # oracle bit for bit for sweep counts below, at and above k (the first
    # launch takes the remainder), the residual within rounding of its order
    u0 = synth.heat2d5_input(n[0], ny=n[1])
    k = tile[2]
    for T in sorted({1, max(1, k - 1), k, 2 * k + 1}):
        want, wr = oracle.heat(u0, T, 0.6, 0.1)
        got, gr = run_jacobi("heat2d5", u0, n, dev, T, coef=(0.6, 0.1), variant="plain", tile=tile)
        assert np.array_equal(got, want), T
        assert abs(gr - wr) <= 1e-10 * wr, T


@pytest.mark.parametrize("n,tile,T", [((37, 29), (16, 16, 4), 9), ((64, 33), (32, 32, 3), 6), ((1, 1), (16, 16, 2), 3),
                                      ((37, 29), (12, 12, 10), 23), ((1, 1), (28, 28, 2), 3), ((64, 33), (16, 16, 12), 13)])
def test_heat2d5_fused_sweeps_write_the_scratch_ring(dev, n, tile, T):
    # fused runs make no halo copy: each launch writes its destination's
    # boundary ring, so a NaN-filled scratch grid ends with the state's ring
    # and every launch reads only finite cells
    u0 = synth.heat2d5_input(n[0], ny=n[1])
    p = Plan("heat2d5", n, variant="plain", coef=(0.6, 0.1), tile=tile)
    f = [_dev(u0, dev), _nan_like(u0, dev)]
    p.run(f, iterations=T)
    p.close()
    a, b = f[0].cpu().numpy(), f[1].cpu().numpy()
    ring = np.ones(u0.shape, bool)
    ring[1:-1, 1:-1] = False
    assert np.array_equal(b[ring], u0[ring]) and np.array_equal(a[ring], u0[ring])
    assert np.all(np.isfinite(b))
    want, _ = oracle.heat(u0, T, 0.6, 0.1)
    assert np.array_equal(a, want)


@pytest.mark.parametrize("tile", [(64, 4, 1), (16, 16, 5), (12, 12, 10), (32, 32, 6)])
def test_heat2d5_pitched_rows(dev, tile):
    # rows padded beyond the grid (row pitch 301 > 258): one launch per sweep
    # and both fused kernels equal the oracle bit for bit, the gaps untouched
    n, T = (256, 61), 11
    PX, PY, py = n[0] + 2, n[1] + 2, 301
    u0 = synth.heat2d5_input(n[0], ny=n[1])
    want, wr = oracle.heat(u0, T, 0.6, 0.1)
    buf = np.full(PY * py, -7.0)
    for y in range(PY):
        buf[y * py: y * py + PX] = u0[y]
    p = Plan("heat2d5", n, variant="plain", coef=(0.6, 0.1), tile=tile, pitch=(py, 0))
    f = [_dev(buf, dev), torch.full((PY * py,), float("nan"), dtype=torch.float64, device=dev)]
    p.run(f, iterations=T)
    gr = p.residual()
    p.close()
    out = f[0].cpu().numpy()
    got = np.stack([out[y * py: y * py + PX] for y in range(PY)])
    assert np.array_equal(got, want)
    gaps = np.concatenate([out[y * py + PX: (y + 1) * py] for y in range(PY - 1)])
    assert np.all(gaps == -7.0)
    assert abs(gr - wr) <= 1e-10 * wr


def test_heat2d5_fused_sweeps_rules(dev):
    # zblock alone picks the 32 x 32 fused tile; periodic boundaries and
    # tiles outside the offered set are refused before anything runs
    # (20 + 2*7 > 32 and 20 is not an LDS-tile size; 12 x 12 x 1 is not a
    # one-sweep thread block of whole waves)
    from paper_2306_13002_amd.stencil import E_INVAL, E_UNSUPPORTED, StencilError

    with Plan("heat2d5", (64, 64), variant="plain", coef=(0.6, 0.1), tile=(0, 0, 8)) as p:
        assert tuple(p.config()["tile"]) == (32, 32, 8)
    with Plan("heat2d5", (64, 64), variant="plain", coef=(0.6, 0.1), tile=(22, 22, 5)) as p:
        assert tuple(p.config()["tile"]) == (22, 22, 5)
    for kw in (dict(tile=(32, 32, 4), bc="periodic"), dict(tile=(64, 4, 4)), dict(tile=(32, 32, 17)),
               dict(tile=(16, 32, 4)), dict(tile=(20, 20, 7)), dict(tile=(12, 12, 1))):
        with pytest.raises(StencilError) as e:
            Plan("heat2d5", (64, 64), variant="plain", coef=(0.6, 0.1), **kw)
        assert e.value.status in (E_UNSUPPORTED, E_INVAL), kw


# ---------------------------------------------------------------- heat3d7
N3 = (70, 37, 29)


@pytest.mark.parametrize("tile", PLAIN_TILES)
def test_heat3d7_plain_bitwise(dev, tile):
    u0 = synth.heat3d7_input(*N3, stream=3)
    for T in (3, 4):
        want, wr = oracle.heat(u0, T, 0.4, 0.1)
        got, gr = run_jacobi("heat3d7", u0, N3, dev, T, coef=(0.4, 0.1), variant="plain", tile=tile)
        assert np.array_equal(got, want)
        assert abs(gr - wr) <= 1e-10 * wr


@pytest.mark.parametrize("tile", HEAT_SAT_TILES)
@pytest.mark.parametrize("zb", [1, 5, 64])
def test_heat3d7_saturated(dev, tile, zb):
    u0 = synth.heat3d7_input(*N3, stream=4)
    T = 3
    want, wr = oracle.heat(u0, T, 0.4, 0.1)
    got, gr = run_jacobi("heat3d7", u0, N3, dev, T, coef=(0.4, 0.1), variant="saturated", tile=(tile[0], tile[1], zb))
    assert maxrel(inner(got, 1), inner(want, 1)) <= 1e-12
    assert np.array_equal(got[0], u0[0]) and np.array_equal(got[:, :, -1], u0[:, :, -1])
    assert abs(gr - wr) <= 1e-10 * wr


H3_SAT2_TILES = [(32, 4), (32, 8), (32, 16), (32, 20), (32, 24), (32, 28), (64, 4), (64, 8), (128, 4)]


@pytest.mark.parametrize("tile", H3_SAT2_TILES)
@pytest.mark.parametrize("zb", [1, 5, 64])
@pytest.mark.parametrize("remap", ["natural", "xcd"])
def test_heat3d7_two_sweep_equals_saturated_bitwise(dev, tile, zb, remap):
    u0 = synth.heat3d7_input(*N3, stream=6)
    for T in (1, 2, 3, 4, 5):
        ref, gr = run_jacobi("heat3d7", u0, N3, dev, T, coef=(0.4, 0.1), variant="saturated",
                             tile=(tile[0], tile[1], zb), tile_map=remap)
        got, gg = run_jacobi("heat3d7", u0, N3, dev, T, coef=(0.4, 0.1), variant="saturated_t2",
                             tile=(tile[0], tile[1], zb), tile_map=remap)
        assert np.array_equal(got, ref), T
        assert gg == gr, T


H3_SAT3_TILES = [(28, 28), (28, 20), (28, 12), (60, 12)]


@pytest.mark.parametrize("tile", H3_SAT3_TILES)
@pytest.mark.parametrize("zb", [1, 5, 64])
@pytest.mark.parametrize("remap", ["natural", "xcd"])
def test_heat3d7_three_sweep_equals_saturated_bitwise(dev, tile, zb, remap):
    # three sweeps per pass (a remainder of one or two sweeps first): the grid
    # equals single sweeps bit for bit; residuals to rounding (another tile)
    u0 = synth.heat3d7_input(*N3, stream=6)
    for T in (1, 2, 3, 4, 5, 7):
        ref, gr = run_jacobi("heat3d7", u0, N3, dev, T, coef=(0.4, 0.1), variant="saturated", tile=(32, 8, 4))
        got, gg = run_jacobi("heat3d7", u0, N3, dev, T, coef=(0.4, 0.1), variant="saturated_t3",
                             tile=(tile[0], tile[1], zb), tile_map=remap)
        assert np.array_equal(got, ref), T
        assert abs(gg - gr) <= 1e-12 * gr, T


@pytest.mark.parametrize("n", [(1, 1, 1), (3, 40, 2), (29, 29, 29), (61, 13, 7)])
def test_heat3d7_three_sweep_small_grids(dev, n):
    u0 = synth.heat3d7_input(*n, stream=8)
    for T in (3, 4, 8):
        want, wr = oracle.heat(u0, T, 0.4, 0.1)
        got, gr = run_jacobi("heat3d7", u0, n, dev, T, coef=(0.4, 0.1), variant="saturated_t3", tile=(28, 12, 4))
        assert maxrel(inner(got, 1), inner(want, 1)) <= 1e-12, T
        assert np.array_equal(got[0], u0[0]) and np.array_equal(got[:, :, -1], u0[:, :, -1])
        assert abs(gr - wr) <= 1e-10 * wr


def test_heat3d7_three_sweep_vs_oracle(dev):
    u0 = synth.heat3d7_input(*N3, stream=7)
    want, wr = oracle.heat(u0, 9, 0.4, 0.1)
    got, gr = run_jacobi("heat3d7", u0, N3, dev, 9, coef=(0.4, 0.1), variant="saturated_t3", tile=(28, 20, 8))
    assert maxrel(inner(got, 1), inner(want, 1)) <= 1e-12
    assert np.array_equal(got[0], u0[0]) and np.array_equal(got[:, :, -1], u0[:, :, -1])
    assert abs(gr - wr) <= 1e-10 * wr


def test_heat3d7_three_sweep_rules(dev):
    # the default shape, and tiles outside the offered set refused
    from paper_2306_13002_amd.stencil import E_UNSUPPORTED, StencilError
    with Plan("heat3d7", (64, 64, 64), variant="saturated_t3", coef=(0.4, 0.1)) as p:
        assert tuple(p.config()["tile"]) == (28, 28, 32)
    for t in ((32, 8, 4), (28, 16, 4), (32, 32, 8)):
        with pytest.raises(StencilError) as e:
            Plan("heat3d7", (64, 64, 64), variant="saturated_t3", coef=(0.4, 0.1), tile=t)
        assert e.value.status == E_UNSUPPORTED, t


def test_heat3d7_two_sweep_vs_oracle(dev):
    u0 = synth.heat3d7_input(*N3, stream=7)
    want, wr = oracle.heat(u0, 6, 0.4, 0.1)
    got, gr = run_jacobi("heat3d7", u0, N3, dev, 6, coef=(0.4, 0.1), variant="saturated_t2", tile=(64, 4, 8))
    assert maxrel(inner(got, 1), inner(want, 1)) <= 1e-12
    assert np.array_equal(got[0], u0[0]) and np.array_equal(got[:, :, -1], u0[:, :, -1])
    assert abs(gr - wr) <= 1e-10 * wr


@pytest.mark.parametrize("variant", ["plain", "saturated", "saturated_t2", "saturated_t3"])
def test_heat3d7_workload_full(dev, variant):
    """The 160^3 grid, T = 50, at the tuned launch shape the benchmark times."""
    n = (160, 160, 160)
    print(f"heat3d7 160^3 {variant}", flush=True)
    u0 = synth.heat3d7_input(*n)
    want, wr = oracle.heat(u0, 50, 0.4, 0.1)
    got, gr = run_jacobi("heat3d7", u0, n, dev, 50, coef=(0.4, 0.1), variant=variant, tune="exhaustive")
    if variant == "plain":
        assert np.array_equal(got, want)
    else:
        assert maxrel(inner(got, 1), inner(want, 1)) <= 1e-12
    assert np.array_equal(got[0], u0[0]) and np.array_equal(got[:, -1], u0[:, -1])
    assert abs(gr - wr) <= 1e-10 * wr


@pytest.mark.parametrize("variant", ["plain", "saturated"])
def test_heat3d7_periodic(dev, variant):
    u0 = synth.heat3d7_input(33, 20, 17, stream=5)
    T = 6
    want, wr = oracle.heat(u0, T, 0.4, 0.1, periodic=True)
    got, gr = run_jacobi("heat3d7", u0, (33, 20, 17), dev, T, coef=(0.4, 0.1), variant=variant, bc="periodic")
    assert maxrel(inner(got, 1), inner(want, 1)) <= (0 if variant == "plain" else 1e-12)
    assert abs(inner(got, 1).sum() - inner(u0, 1).sum()) <= 1e-10 * inner(u0, 1).sum()
    assert abs(gr - wr) <= 1e-10 * wr


def test_heat2d5_periodic(dev):
    u0 = synth.heat2d5_input(40, ny=23)
    want, wr = oracle.heat(u0, 5, 0.6, 0.1, periodic=True)
    got, gr = run_jacobi("heat2d5", u0, (40, 23), dev, 5, coef=(0.6, 0.1), variant="plain", bc="periodic")
    assert np.array_equal(inner(got, 1), inner(want, 1))
    assert abs(gr - wr) <= 1e-10 * wr


# ---------------------------------------------------------------- poisson19
NP = (70, 19, 23)  # interior; padded (25, 21, 72)


def _p19_inputs(seed=2):
    return synth.poisson19_random_inputs((NP[2] + 2, NP[1] + 2, NP[0] + 2), seed=seed)


@pytest.mark.parametrize("tile", PLAIN_TILES)
def test_poisson19_plain_bitwise(dev, tile):
    p0, cf = _p19_inputs()
    for T in (2, 3):
        want, wg = oracle.poisson19(p0, cf, 0.8, T, mode="F32STORE")
        got, gg = run_jacobi("poisson19", p0, NP, dev, T, coefs=cf, variant="plain", tile=tile, omega=0.8)
        assert np.array_equal(got.astype(np.float64), want)
        assert abs(gg - wg) <= 1e-10 * wg


@pytest.mark.parametrize("tile", P19_SAT_TILES)
@pytest.mark.parametrize("zb", [1, 4, 16, 64])
def test_poisson19_saturated(dev, tile, zb):
    p0, cf = _p19_inputs(seed=3)
    T = 3
    w64, _ = oracle.poisson19(p0, cf, 0.8, T, mode="F64")
    w32, g32 = oracle.poisson19(p0, cf, 0.8, T, mode="F32STORE")
    got, gg = run_jacobi("poisson19", p0, NP, dev, T, coefs=cf, variant="saturated", tile=(tile[0], tile[1], zb),
                         omega=0.8)
    assert maxrel(inner(got, 1), inner(w64, 1)) <= 1e-5
    # FP64 arithmetic on F32 storage: rounding flips of stored p are rare
    assert np.mean(inner(got, 1).astype(np.float64) != inner(w32, 1)) < 1e-3
    assert abs(gg - g32) <= 1e-5 * g32
    assert np.array_equal(got[0], p0[0]) and np.array_equal(got[:, 0], p0[:, 0])


@pytest.mark.parametrize("tile", P19_SAT2_TILES)
@pytest.mark.parametrize("zb", [1, 5, 64])
@pytest.mark.parametrize("remap", ["natural", "xcd"])
def test_poisson19_two_sweep_equals_saturated_bitwise(dev, tile, zb, remap):
    """Two sweeps per pass give exactly what the single-sweep saturated
    kernel gives, for even and odd sweep counts, residual included."""
    p0, cf = _p19_inputs(seed=4)
    for T in (1, 2, 3, 4, 5):
        ref, gr = run_jacobi("poisson19", p0, NP, dev, T, coefs=cf, variant="saturated",
                             tile=(tile[0], tile[1], zb), omega=0.8, tile_map=remap)
        got, gg = run_jacobi("poisson19", p0, NP, dev, T, coefs=cf, variant="saturated_t2",
                             tile=(tile[0], tile[1], zb), omega=0.8, tile_map=remap)
        assert np.array_equal(got, ref), T
        assert gg == gr, T


TINY = [(1, 1, 1), (3, 2, 1), (5, 1, 2), (2, 7, 3), (70, 1, 1), (1, 40, 5), (65, 9, 2)]


@pytest.mark.parametrize("n", TINY)
@pytest.mark.parametrize("zb", [1, 2, 64])
def test_two_sweep_forms_on_degenerate_grids(dev, n, zb):
    """One- and two-cell extents, single planes, grids smaller than a tile:
    both two-sweep forms equal their single-sweep forms bit for bit and the
    oracle within tolerance, for T = 1..4."""
    u0 = synth.heat3d7_input(*n, stream=40)
    pp, cf = synth.poisson19_random_inputs((n[2] + 2, n[1] + 2, n[0] + 2), seed=40)
    for T in (1, 2, 3, 4):
        print(f"degenerate n={n} zb={zb} T={T}", flush=True)
        ref, gr = run_jacobi("heat3d7", u0, n, dev, T, coef=(0.4, 0.1), variant="saturated", tile=(32, 8, zb))
        got, gg = run_jacobi("heat3d7", u0, n, dev, T, coef=(0.4, 0.1), variant="saturated_t2", tile=(32, 8, zb))
        assert np.array_equal(got, ref) and gg == gr, ("heat3d7", T)
        want, wr = oracle.heat(u0, T, 0.4, 0.1)
        assert maxrel(inner(got, 1), inner(want, 1)) <= 1e-12
        assert abs(gg - wr) <= 1e-10 * wr or (wr == 0 and gg == 0)
        ref, gr = run_jacobi("poisson19", pp, n, dev, T, coefs=cf, variant="saturated", tile=(64, 8, zb), omega=0.8)
        got, gg = run_jacobi("poisson19", pp, n, dev, T, coefs=cf, variant="saturated_t2", tile=(64, 8, zb),
                             omega=0.8)
        assert np.array_equal(got, ref) and gg == gr, ("poisson19", T)
        w64, _ = oracle.poisson19(pp, cf, 0.8, T, mode="F64")
        assert maxrel(inner(got.astype(np.float64), 1), inner(w64, 1)) <= 1e-5


@pytest.mark.parametrize("tile", [(128, 4), (64, 8), (32, 4)])
def test_poisson19_two_sweep_vs_oracle(dev, tile):
    p0, cf = _p19_inputs(seed=6)
    T = 4
    w64, _ = oracle.poisson19(p0, cf, 0.8, T, mode="F64")
    w32, g32 = oracle.poisson19(p0, cf, 0.8, T, mode="F32STORE")
    got, gg = run_jacobi("poisson19", p0, NP, dev, T, coefs=cf, variant="saturated_t2", tile=(tile[0], tile[1], 8),
                         omega=0.8)
    assert maxrel(inner(got, 1), inner(w64, 1)) <= 1e-5
    assert np.mean(inner(got, 1).astype(np.float64) != inner(w32, 1)) < 1e-3
    assert abs(gg - g32) <= 1e-5 * g32
    assert np.array_equal(got[0], p0[0]) and np.array_equal(got[:, 0], p0[:, 0])


@pytest.mark.parametrize("variant,tile", [("plain", (0, 0, 0)), ("saturated", (0, 0, 0)), ("saturated_t2", (0, 0, 0)),
                                          ("saturated_t2", (64, 8, 32)), ("saturated_t2", (128, 4, 32))])
def test_poisson19_workload_full(dev, variant, tile):
    # the 129 x 129 x 257 (boundary included) workload, T = 20, as benchmarked
    # (default shape, and the two-sweep shapes the tuner picks)
    p0, cf = synth.poisson19_inputs()
    n = (127, 127, 255)
    w64, g64 = oracle.poisson19(p0, cf, 0.8, 20, mode="F64")
    w32, g32 = oracle.poisson19(p0, cf, 0.8, 20, mode="F32STORE")
    got, gg = run_jacobi("poisson19", p0, n, dev, 20, coefs=cf, variant=variant, omega=0.8, tile=tile)
    assert maxrel(inner(got, 1), inner(w64, 1)) <= 1e-5
    assert abs(gg - g32) <= 1e-5 * g32
    if variant == "plain":
        assert np.array_equal(got.astype(np.float64), w32)
    # first sweep: closed form of the residual
    p1 = Plan("poisson19", n, variant=variant, omega=0.8, tile=tile)
    f = [_dev(p0, dev), _nan_like(p0, dev)]
    p1.run(f, [_dev(c, dev) for c in cf], iterations=1)
    g1 = p1.residual()
    p1.close()
    assert abs(g1 - 1.0681643715818605e-4) <= 1e-5 * 1.0681643715818605e-4


# ---------------------------------------------------------------- wave25
NW = (45, 22, 19)


def run_wave(n, a, b, vsq, T, dev, **kw):
    p = Plan("wave25", n, coef=synth.WAVE25_COEF, **kw)
    f = [_dev(a, dev), _dev(b, dev)]
    p.run(f, [_dev(vsq, dev)], iterations=T)
    res = p.residual() if T > 0 else None
    out = (f[0].cpu().numpy(), f[1].cpu().numpy())
    p.close()
    return out, res


@pytest.mark.parametrize("tile", PLAIN_TILES)
def test_wave25_plain_bitwise(dev, tile):
    a, b, v = synth.wave25_inputs(*NW)
    for T in (1, 2, 3):
        A, B, wr = oracle.wave25(a, b, v, synth.WAVE25_COEF, T)
        (ga, gb), gr = run_wave(NW, a, b, v, T, dev, variant="plain", tile=tile)
        assert np.array_equal(ga, A) and np.array_equal(gb, B)
        assert abs(gr - wr) <= 1e-10 * wr


@pytest.mark.parametrize("tile", W25_SAT_TILES)
@pytest.mark.parametrize("zb", [1, 6, 64])
def test_wave25_saturated(dev, tile, zb):
    a, b, v = synth.wave25_inputs(*NW, seed=5)
    T = 3
    A, B, wr = oracle.wave25(a, b, v, synth.WAVE25_COEF, T)
    (ga, gb), gr = run_wave(NW, a, b, v, T, dev, variant="saturated", tile=(tile[0], tile[1], zb))
    assert maxrel(inner(ga, 4), inner(A, 4)) <= 1e-12 and maxrel(inner(gb, 4), inner(B, 4)) <= 1e-12
    assert np.array_equal(ga[:4], a[:4]) and np.array_equal(gb[:, :, -4:], b[:, :, -4:])
    assert abs(gr - wr) <= 1e-10 * wr


@pytest.fixture(scope="module")
def wave_full():
    return synth.wave25_inputs(512)


@pytest.mark.parametrize("variant", ["plain", "saturated"])
def test_wave25_workload_full_sampled(dev, variant, wave_full):
    # 512^3 interior, T = 10, at the benchmark's launch configuration.  The
    # oracle runs on light-cone crops: after T steps a point depends only on
    # cells within 4T, so a crop with a 4(T-1) margin reproduces it exactly.
    n, T = (512, 512, 512), 10
    a, b, v = wave_full
    p = Plan("wave25", n, variant=variant, coef=synth.WAVE25_COEF)
    f = [_dev(a, dev), _dev(b, dev)]
    vs = _dev(v, dev)
    p.run(f, [vs], iterations=T)
    gr = p.residual()
    ga = f[0].cpu().numpy()
    gb = f[1].cpu().numpy()
    del f, vs
    p.close()
    tol = 0 if variant == "plain" else 1e-12
    boxes = [((0, 0, 0), (12, 9, 7)), ((250, 251, 249), (262, 259, 257)), ((500, 3, 505), (512, 11, 512)),
             ((100, 506, 0), (108, 512, 6))]
    for lo, hi in boxes:
        sl, off = crop_box(n, lo, hi, 4, 4 * (T - 1))
        A, B, _ = oracle.wave25(a[sl], b[sl], v[sl], synth.WAVE25_COEF, T)
        gsl = tuple(slice(s.start + o0 + 4, s.start + o1 + 4) for s, (o0, o1) in zip(sl, off))
        assert maxrel(ga[gsl], compare_region(A, off, 4)) <= tol
        assert maxrel(gb[gsl], compare_region(B, off, 4)) <= tol
    # halo untouched
    assert np.array_equal(ga[:4], a[:4]) and np.array_equal(gb[-4:], b[-4:])
    # the residual (two-pass reduction over the benchmarked launch's block
    # partials) against the returned fields: T even, so the newest level is
    # fields[1]
    d = inner(gb, 4) - inner(ga, 4)
    want = float(np.sum(d * d))
    del d
    assert want > 0 and abs(gr - want) <= 1e-10 * want


# ---------------------------------------------------------------- contracts
def test_determinism_and_restart(dev):
    a, b, v = synth.wave25_inputs(*NW, seed=8)
    for variant in ("plain", "saturated"):
        (a5, b5), r5 = run_wave(NW, a, b, v, 5, dev, variant=variant)
        (a5b, b5b), r5b = run_wave(NW, a, b, v, 5, dev, variant=variant)
        assert np.array_equal(a5, a5b) and np.array_equal(b5, b5b) and r5 == r5b
        (a2, b2), _ = run_wave(NW, a, b, v, 2, dev, variant=variant)
        (a3, b3), r3 = run_wave(NW, a2, b2, v, 3, dev, variant=variant)
        assert np.array_equal(a3, a5) and np.array_equal(b3, b5) and r3 == r5
    u0 = synth.heat3d7_input(*N3, stream=6)
    for variant in ("plain", "saturated"):
        g5, r5 = run_jacobi("heat3d7", u0, N3, dev, 5, coef=(0.4, 0.1), variant=variant)
        g2, _ = run_jacobi("heat3d7", u0, N3, dev, 2, coef=(0.4, 0.1), variant=variant)
        g3, r3 = run_jacobi("heat3d7", g2, N3, dev, 3, coef=(0.4, 0.1), variant=variant)
        assert np.array_equal(g5, g3) and r5 == r3


def test_zero_iterations_and_state(dev):
    from paper_2306_13002_amd.stencil import StencilError, E_STATE
    u0 = synth.heat3d7_input(9, 8, 7)
    p = Plan("heat3d7", (9, 8, 7), coef=(0.4, 0.1))
    f = [_dev(u0, dev), _nan_like(u0, dev)]
    p.run(f, iterations=0)
    torch.cuda.synchronize()
    assert np.array_equal(f[0].cpu().numpy(), u0)
    with pytest.raises(StencilError) as e:
        p.residual()
    assert e.value.status == E_STATE
    p.close()


@pytest.mark.parametrize("kind,variant", [("heat3d7", "plain"), ("heat3d7", "saturated"), ("heat3d7", "saturated_t2"),
                                          ("heat3d7", "saturated_t3"),
                                          ("wave25", "plain"), ("wave25", "saturated")])
def test_pitched_layout(dev, kind, variant):
    # rows and planes padded beyond the grid: same result, gaps untouched
    n = (37, 13, 11)
    r = 1 if kind == "heat3d7" else 4
    PX, PY, PZ = n[0] + 2 * r, n[1] + 2 * r, n[2] + 2 * r
    py, pz = PX + 7, (PX + 7) * PY + 19
    if kind == "heat3d7":
        u0 = synth.heat3d7_input(*n, stream=7)
        want, _ = oracle.heat(u0, 3, 0.4, 0.1)
        grids = [u0]
    else:
        a, b, v = synth.wave25_inputs(*n, seed=9)
        A, B, _ = oracle.wave25(a, b, v, synth.WAVE25_COEF, 3)
        grids = [a, b, v]

    def pitched(g):
        buf = np.full(PZ * pz, -7.0)
        for z in range(PZ):
            for y in range(PY):
                buf[z * pz + y * py: z * pz + y * py + PX] = g[z, y]
        return buf

    def unpitched(buf):
        out = np.empty((PZ, PY, PX))
        for z in range(PZ):
            for y in range(PY):
                out[z, y] = buf[z * pz + y * py: z * pz + y * py + PX]
        return out

    p = Plan(kind, n, coef=(0.4, 0.1) if kind == "heat3d7" else synth.WAVE25_COEF, variant=variant, pitch=(py, pz))
    if kind == "heat3d7":
        f = [_dev(pitched(u0), dev), torch.full((PZ * pz,), float("nan"), dtype=torch.float64, device=dev)]
        p.run(f, iterations=3)
        buf = f[0].cpu().numpy()
        assert maxrel(inner(unpitched(buf), 1), inner(want, 1)) <= (0 if variant == "plain" else 1e-12)
    else:
        f = [_dev(pitched(a), dev), _dev(pitched(b), dev)]
        p.run(f, [_dev(pitched(v), dev)], iterations=3)
        buf = f[0].cpu().numpy()
        assert maxrel(inner(unpitched(buf), 4), inner(A, 4)) <= (0 if variant == "plain" else 1e-12)
    mask = np.ones(PZ * pz, bool)
    for z in range(PZ):
        for y in range(PY):
            mask[z * pz + y * py: z * pz + y * py + PX] = False
    assert np.all(buf[mask] == -7.0)


@pytest.mark.parametrize("variant,tile", [("plain", (64, 4, 1)), ("saturated", (64, 8, 4)), ("saturated", (128, 4, 64)),
                                          ("saturated_t2", (64, 8, 4)), ("saturated_t2", (128, 4, 64)),
                                          ("saturated_t2", (32, 8, 3))])
def test_pitched_layout_poisson19(dev, variant, tile):
    # p and all 12 coefficient grids with rows and planes padded beyond the
    # grid (the saturated kernels address cells by byte offsets built from the
    # pitches): plain equals the F32-store oracle bit for bit, the saturated
    # forms equal their own unpitched runs bit for bit, and the gaps of the
    # state grid are left alone
    n = (37, 13, 11)
    PX, PY, PZ = n[0] + 2, n[1] + 2, n[2] + 2
    py, pz = PX + 7, (PX + 7) * PY + 19
    p0, cf = synth.poisson19_random_inputs((PZ, PY, PX), seed=12)
    T = 3

    def pitched(g):
        buf = np.full(PZ * pz, -7.0, dtype=np.float32)
        for z in range(PZ):
            for y in range(PY):
                buf[z * pz + y * py: z * pz + y * py + PX] = g[z, y]
        return buf

    def unpitched(buf):
        out = np.empty((PZ, PY, PX), dtype=np.float32)
        for z in range(PZ):
            for y in range(PY):
                out[z, y] = buf[z * pz + y * py: z * pz + y * py + PX]
        return out

    p = Plan("poisson19", n, variant=variant, tile=tile, omega=0.8, pitch=(py, pz))
    f = [_dev(pitched(p0), dev), torch.full((PZ * pz,), float("nan"), dtype=torch.float32, device=dev)]
    p.run(f, [_dev(pitched(c), dev) for c in cf], iterations=T)
    gg = p.residual()
    p.close()
    buf = f[0].cpu().numpy()
    got = unpitched(buf)
    if variant == "plain":
        want, wg = oracle.poisson19(p0, cf, 0.8, T, mode="F32STORE")
        assert np.array_equal(got.astype(np.float64), want)
        assert abs(gg - wg) <= 1e-10 * wg
    else:
        ref, gr = run_jacobi("poisson19", p0, n, dev, T, coefs=cf, variant=variant, tile=tile, omega=0.8)
        assert np.array_equal(got, ref)
        assert gg == gr
    mask = np.ones(PZ * pz, bool)
    for z in range(PZ):
        for y in range(PY):
            mask[z * pz + y * py: z * pz + y * py + PX] = False
    assert np.all(buf[mask] == -7.0)
    p.close()
