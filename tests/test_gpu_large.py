"""Grids with more than 2^31 elements per array: every index and offset on
the path is 64-bit.  One pass of each form on grids of 2.2e9 padded
elements (17-18 GB per FP64 array), checked at sampled boxes -- the highest
planes, whose element indices pass 2^31, among them -- against the oracle
on the light-cone crop around each box (the crop's outer ring is either the
grid's real halo or interior cells the sampled values cannot see).

Inputs are integer patterns scaled by powers of two, exact in FP32 and
FP64, generated on the device plane block by plane block and read back
only inside the crops."""
import numpy as np
import pytest

import oracle
from paper_2306_13002_amd import synth
from gpu_util import compare_region, crop_box, maxrel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N_HEAT = (1024, 1024, 2100)  # padded 1026 x 1026 x 2102 = 2.21e9 elements
N_WAVE = (1024, 1024, 2100)  # padded 1032 x 1032 x 2108 = 2.25e9 elements


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


@pytest.fixture(autouse=True)
def _free_memory():
    yield
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def pattern(shape, dev, dtype, mult, mod, scale, base=0.0):
    """base + ((mult_x*i + mult_y*j + mult_z*k) mod `mod`) * scale over a
    padded (z, y, x) array, built in blocks of planes."""
    out = torch.empty(shape, dtype=dtype, device=dev)
    PZ, PY, PX = shape
    ji = (torch.arange(PY, device=dev, dtype=torch.int64)[:, None] * mult[1] +
          torch.arange(PX, device=dev, dtype=torch.int64)[None, :] * mult[0])
    for z0 in range(0, PZ, 64):
        z1 = min(z0 + 64, PZ)
        k = torch.arange(z0, z1, device=dev, dtype=torch.int64)[:, None, None] * mult[2]
        out[z0:z1] = ((ji[None] + k) % mod).to(dtype) * scale + base
    return out


def boxes(n):
    """Sample boxes (lo, hi) in interior coordinates (x, y, z): the last
    corner (highest addresses), the top planes at other x/y, the first
    corner, and the middle."""
    nx, ny, nz = n
    return [((nx - 6, ny - 5, nz - 4), (nx, ny, nz)),
            ((0, ny // 2, nz - 3), (7, ny // 2 + 4, nz)),
            ((nx // 3, 0, nz - 70), (nx // 3 + 5, 3, nz - 66)),
            ((0, 0, 0), (5, 4, 3)),
            ((nx // 2, ny // 2, nz // 2), (nx // 2 + 4, ny // 2 + 4, nz // 2 + 4))]


def host(t, sl):
    return t[sl].cpu().numpy()


@pytest.mark.parametrize("variant,T", [("plain", 1), ("saturated", 1), ("saturated_t2", 2)])
def test_heat3d7_beyond_2_31_elements(dev, variant, T):
    from paper_2306_13002_amd.stencil import Plan
    n = N_HEAT
    print(f"large heat3d7 {variant} T={T} n={n}", flush=True)
    shape = (n[2] + 2, n[1] + 2, n[0] + 2)
    assert shape[0] * shape[1] * shape[2] > 2 ** 31
    u0 = pattern(shape, dev, torch.float64, (7, 13, 29), 1024, 1.0 / 1024)
    f = [u0.clone(), torch.empty_like(u0)]
    p = Plan("heat3d7", n, variant=variant, coef=(0.4, 0.1), tune="fixed")
    p.run(f, iterations=T)
    torch.cuda.synchronize()
    r = p.residual()
    p.close()
    del f[1]
    assert np.isfinite(r) and r > 0
    for lo, hi in boxes(n):
        sl, off = crop_box(n, lo, hi, 1, T - 1)
        want, _ = oracle.heat(host(u0, sl), T, 0.4, 0.1)
        gsl = tuple(slice(s.start + o0 + 1, s.start + o1 + 1) for s, (o0, o1) in zip(sl, off))
        got = host(f[0], gsl)
        err = maxrel(got, compare_region(want, off, 1))
        assert err <= (0 if variant == "plain" else 1e-12), (lo, err)
    # the halo is never written
    assert torch.equal(f[0][-1], u0[-1]) and torch.equal(f[0][:, :, 0], u0[:, :, 0])


# coefficient patterns: (base, x/y/z multipliers, modulus, scale); every
# value a multiple of 2^-10, exact in FP32; b-terms nonzero
P19_COEF = dict(a0=(1.0, (3, 5, 7), 16, 2.0 ** -8), a1=(1.0, (5, 7, 3), 16, 2.0 ** -8),
                a2=(1.0, (7, 3, 5), 16, 2.0 ** -8), a3=(1.0 / 8, (1, 2, 3), 8, 2.0 ** -10),
                b0=(0.0, (2, 3, 5), 8, 2.0 ** -8), b1=(0.0, (3, 5, 2), 8, 2.0 ** -8),
                b2=(0.0, (5, 2, 3), 8, 2.0 ** -8), c0=(1.0, (11, 1, 2), 16, 2.0 ** -8),
                c1=(1.0, (1, 11, 2), 16, 2.0 ** -8), c2=(1.0, (2, 1, 11), 16, 2.0 ** -8),
                bnd=(1.0, (0, 0, 0), 1, 0.0), wrk1=(0.0, (1, 1, 1), 4, 2.0 ** -10))


@pytest.mark.parametrize("variant,T", [("plain", 1), ("saturated_t2", 2)])
def test_poisson19_beyond_2_31_elements(dev, variant, T):
    from paper_2306_13002_amd.stencil import Plan
    n = N_HEAT
    print(f"large poisson19 {variant} T={T} n={n}", flush=True)
    shape = (n[2] + 2, n[1] + 2, n[0] + 2)
    assert shape[0] * shape[1] * shape[2] > 2 ** 31
    p0 = pattern(shape, dev, torch.float32, (7, 13, 29), 256, 2.0 ** -8)
    cs = [pattern(shape, dev, torch.float32, P19_COEF[k][1], P19_COEF[k][2], P19_COEF[k][3], P19_COEF[k][0])
          for k in synth.POISSON_COEF_ORDER]
    f = [p0.clone(), torch.empty_like(p0)]
    p = Plan("poisson19", n, variant=variant, omega=0.8, tune="fixed")
    p.run(f, cs, iterations=T)
    torch.cuda.synchronize()
    r = p.residual()
    p.close()
    del f[1]
    assert np.isfinite(r) and r > 0
    for lo, hi in boxes(n):
        sl, off = crop_box(n, lo, hi, 1, T - 1)
        cc = [host(c, sl) for c in cs]
        gsl = tuple(slice(s.start + o0 + 1, s.start + o1 + 1) for s, (o0, o1) in zip(sl, off))
        got = host(f[0], gsl).astype(np.float64)
        if variant == "plain":  # the plain body is the oracle's, rounded to F32 on store
            want, _ = oracle.poisson19(host(p0, sl), cc, 0.8, T, mode="F32STORE")
            assert np.array_equal(got, compare_region(want, off, 1)), lo
        else:
            want, _ = oracle.poisson19(host(p0, sl), cc, 0.8, T, mode="F64")
            assert maxrel(got, compare_region(want, off, 1)) <= 1e-5, lo
    assert torch.equal(f[0][-1], p0[-1]) and torch.equal(f[0][:, 0], p0[:, 0])


@pytest.mark.parametrize("variant", ["plain", "saturated"])
def test_wave25_beyond_2_31_elements(dev, variant):
    from paper_2306_13002_amd.stencil import Plan
    n = N_WAVE
    print(f"large wave25 {variant} n={n}", flush=True)
    shape = (n[2] + 8, n[1] + 8, n[0] + 8)
    assert shape[0] * shape[1] * shape[2] > 2 ** 31
    a = pattern(shape, dev, torch.float64, (7, 13, 29), 64, 2.0 ** -10, 1.0)
    b = pattern(shape, dev, torch.float64, (13, 7, 3), 64, 2.0 ** -10, 1.0)
    v = pattern(shape, dev, torch.float64, (3, 5, 11), 32, 2.0 ** -8, 0.125)
    f = [a.clone(), b]
    p = Plan("wave25", n, variant=variant, coef=synth.WAVE25_COEF, tune="fixed")
    p.run(f, [v], iterations=1)
    torch.cuda.synchronize()
    r = p.residual()
    p.close()
    assert np.isfinite(r) and r > 0
    for lo, hi in boxes(n):
        sl, off = crop_box(n, lo, hi, 4, 0)
        A, _, _ = oracle.wave25(host(a, sl), host(b, sl), host(v, sl), synth.WAVE25_COEF, 1)
        gsl = tuple(slice(s.start + o0 + 4, s.start + o1 + 4) for s, (o0, o1) in zip(sl, off))
        err = maxrel(host(f[0], gsl), compare_region(A, off, 4))
        assert err <= (0 if variant == "plain" else 1e-12), (lo, err)
    assert torch.equal(f[0][-4:], a[-4:]) and torch.equal(f[0][:, :, :4], a[:, :, :4])


@pytest.mark.parametrize("variant", ["plain", "saturated", "saturated_t2", "saturated_t3"])
def test_tall_grids_beyond_65535_planes(dev, variant):
    """Thin columns taller than 65 535 planes: the plain kernels launch one
    block row per plane (a z grid dimension above 65 535), the saturated
    forms block z; every form against the oracle on the whole grid."""
    from paper_2306_13002_amd.stencil import Plan
    n, T = (3, 2, 70001), 3
    print(f"tall heat3d7 {variant} n={n}", flush=True)
    u0 = synth.heat3d7_input(*n, stream=44)
    p = Plan("heat3d7", n, variant=variant, coef=(0.4, 0.1), tune="fixed")
    f = [torch.tensor(u0, device=dev), torch.full(u0.shape, float("nan"), dtype=torch.float64, device=dev)]
    p.run(f, iterations=T)
    gr = p.residual()
    p.close()
    want, wr = oracle.heat(u0, T, 0.4, 0.1)
    got = f[0].cpu().numpy()
    assert maxrel(got[1:-1, 1:-1, 1:-1], want[1:-1, 1:-1, 1:-1]) <= (0 if variant == "plain" else 1e-12)
    assert abs(gr - wr) <= 1e-10 * wr
    if variant == "saturated_t3":  # a heat3d7 form only
        return
    print(f"tall poisson19 {variant} n={n}", flush=True)
    pp, cf = synth.poisson19_random_inputs((n[2] + 2, n[1] + 2, n[0] + 2), seed=44)
    p = Plan("poisson19", n, variant=variant, omega=0.8, tune="fixed")
    f = [torch.tensor(pp, device=dev), torch.zeros(pp.shape, dtype=torch.float32, device=dev)]
    p.run(f, [torch.tensor(c, device=dev) for c in cf], iterations=T)
    p.close()
    w64, _ = oracle.poisson19(pp, cf, 0.8, T, mode="F64")
    assert maxrel(f[0].cpu().numpy().astype(np.float64)[1:-1, 1:-1, 1:-1], w64[1:-1, 1:-1, 1:-1]) <= 1e-5



def test_generic_plain_plane_pitch_beyond_int32_offsets(dev):
    from paper_2306_13002_amd.stencil import Plan

    # A plane pitch of 6e8 elements: the z taps of a radius-4 star reach
    # +-4 planes = +-2.4e9 elements, past the 32-bit range, so every tap
    # offset must be 64-bit.  F32 storage, one interior plane, 19 GB per
    # array (only the grid's rows are written; the gaps are never read).
    r, n = 4, (40, 6, 1)
    PX, PY, PZ = n[0] + 2 * r, n[1] + 2 * r, n[2] + 2 * r
    py, pz = PX, 600_000_000
    assert 4 * pz > 2 ** 31
    taps = synth.star_taps(r)
    cids = [0] + [1 + (i // 2) % 4 for i in range(len(taps) - 1)]
    coef = [0.4, 0.05, 0.04, 0.03, 0.03]
    dense = synth.uniform_f32(23, 0, (PZ, PY, PX))
    want, wr = oracle.generic(dense, r, taps, cids, coef, 2, mode="F32STORE")
    span = (PZ - 1) * pz + PY * py
    f = [torch.empty(span, dtype=torch.float32, device=dev) for _ in range(2)]
    for z in range(PZ):
        f[0][z * pz: z * pz + PY * py] = torch.from_numpy(dense[z].ravel()).to(dev)
    p = Plan("generic", n, variant="plain", dtype="f32", radius=r, coef=coef, taps=taps, cids=cids,
             pitch=(py, pz))
    p.run(f, iterations=2)
    gr = p.residual()
    p.close()
    got = np.stack([f[0][z * pz: z * pz + PY * py].cpu().numpy().reshape(PY, PX) for z in range(PZ)])
    del f
    assert np.array_equal(got.astype(np.float64), want)
    assert abs(gr - wr) <= 1e-10 * wr


@pytest.mark.parametrize("kind,kw,eb,form", [
    ("wave25", dict(coef=synth.WAVE25_COEF), 8, "saturated"),
    ("poisson19", dict(omega=0.8), 4, "saturated"),
    ("poisson19", dict(omega=0.8), 4, "saturated_t2"),
])
def test_saturated_plane_limit(dev, kind, kw, eb, form):
    # The saturated leapfrog and Poisson kernels address a plane with 32-bit
    # byte offsets: a plane pitch above 0xFFFFFFF0 bytes is refused for those
    # forms, and AUTO picks PLAIN.  Only plans are made here (no grid is
    # allocated).
    from paper_2306_13002_amd.stencil import E_UNSUPPORTED, Plan, StencilError

    n = (8, 8, 8)
    big, fits = 0xFFFFFFF0 // eb + 1, 0xFFFFFFF0 // eb
    with pytest.raises(StencilError) as e:
        Plan(kind, n, variant=form, pitch=(0, big), **kw)
    assert e.value.status == E_UNSUPPORTED
    with Plan(kind, n, variant=form, pitch=(0, fits), **kw) as p:
        assert p.config()["variant"] == form
    with Plan(kind, n, variant="auto", pitch=(0, big), **kw) as p:
        assert p.config()["variant"] == "plain"
