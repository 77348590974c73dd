"""The allocation-free run (stencil_run_noalloc) against stencil_run +
stencil_residual on the same inputs, through the C ABI: the same kernels and
the same fixed-order reduction, so fields and residual must agree bit for
bit.  Every kind's form is called twice in a row on one GPU, the second
call on a smaller grid (the scratch keeps the first call's partials beyond
the second call's block count; the reduction must read only its own).
Also: the host-side refusals, which happen before anything is enqueued."""
import numpy as np
import pytest

from paper_2306_13002_amd import synth
from paper_2306_13002_amd.stencil import E_INVAL, E_UNSUPPORTED, Plan, StencilError

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def _both_ways(kind, n, fields_host, coef_host, T, dev, **kw):
    """(fields, residual) of stencil_run + stencil_residual and of
    stencil_run_noalloc, each from its own copy of the inputs."""
    out = []
    with Plan(kind, n, **kw) as p:
        for way in ("run", "noalloc"):
            f = [torch.tensor(a, device=dev) for a in fields_host]
            c = [torch.tensor(a, device=dev) for a in coef_host] if coef_host else None
            if way == "run":
                p.run(f, c, iterations=T)
                r = p.residual()
            else:
                res = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
                p.run_noalloc(f, c, iterations=T, residual=res)
                torch.cuda.synchronize()
                r = float(res.cpu()[0])
            out.append(([t.cpu().numpy() for t in f], r))
        cfg = p.config()
    return out, cfg


def _check_equal(out):
    (fa, ra), (fb, rb) = out
    for a, b in zip(fa, fb):
        assert np.array_equal(a, b)
    assert np.isfinite(ra) and ra > 0
    assert ra == rb  # same partials, same fixed reduction order


def _wave_case(n):
    a, b, v = synth.wave25_inputs(*n, seed=11)
    return [a, b], [v]


def _heat3_case(n):
    u = synth.heat3d7_input(*n, seed=12)
    return [u, np.zeros_like(u)], None


def _p19_case(n):
    p, cf = synth.poisson19_random_inputs((n[2] + 2, n[1] + 2, n[0] + 2), seed=13)
    return [p, np.zeros_like(p)], cf


def _heat2_case(n):
    u = synth.heat2d5_input(n[0], seed=14, ny=n[1])
    return [u, np.zeros_like(u)], None


# (kind, plan kwargs, input builder, larger grid, smaller grid, sweeps)
CASES = [
    ("wave25", dict(variant="saturated", coef=synth.WAVE25_COEF, tile=(64, 32, 64)), _wave_case,
     (97, 70, 150), (40, 33, 21), 3),
    ("wave25", dict(variant="plain", coef=synth.WAVE25_COEF), _wave_case, (97, 70, 60), (40, 33, 21), 2),
    ("heat3d7", dict(variant="saturated_t2", coef=(0.4, 0.1)), _heat3_case, (130, 61, 77), (33, 20, 9), 5),
    ("heat3d7", dict(variant="saturated", coef=(0.4, 0.1)), _heat3_case, (130, 61, 77), (33, 20, 9), 4),
    ("heat3d7", dict(variant="saturated_t3", coef=(0.4, 0.1)), _heat3_case, (130, 61, 77), (33, 20, 9), 5),
    ("poisson19", dict(variant="saturated_t2", omega=0.8), _p19_case, (127, 40, 66), (30, 11, 17), 3),
    ("poisson19", dict(variant="plain", omega=0.8), _p19_case, (127, 40, 66), (30, 11, 17), 2),
    ("heat2d5", dict(variant="plain", coef=(0.6, 0.1)), _heat2_case, (300, 211), (37, 29), 3),
    ("heat2d5", dict(variant="plain", coef=(0.6, 0.1), tile=(32, 32, 4)), _heat2_case, (300, 211), (37, 29), 7),
    ("heat2d5", dict(variant="plain", coef=(0.6, 0.1), tile=(16, 16, 4)), _heat2_case, (300, 211), (37, 29), 7),
]


@pytest.mark.parametrize("kind,kw,build,n_big,n_small,T", CASES,
                         ids=[f"{c[0]}-{c[1]['variant']}" + ("-fused" if c[1].get("tile", (0, 0, 1))[2] > 1 and c[0] == "heat2d5"
                                                            else "") for c in CASES])
def test_noalloc_matches_run_twice_second_smaller(dev, kind, kw, build, n_big, n_small, T):
    print(f"[noalloc] {kind} {kw['variant']} {n_big} then {n_small}, T={T}", flush=True)
    for n in (n_big, n_small):
        fields, coefs = build(n)
        out, cfg = _both_ways(kind, n, fields, coefs, T, dev, **kw)
        assert cfg["variant"] == kw["variant"]
        _check_equal(out)


def test_noalloc_without_residual_output(dev):
    n = (50, 41, 33)
    fields, coefs = _wave_case(n)
    with Plan("wave25", n, variant="saturated", coef=synth.WAVE25_COEF) as p:
        f1 = [torch.tensor(a, device=dev) for a in fields]
        f2 = [torch.tensor(a, device=dev) for a in fields]
        vs = torch.tensor(coefs[0], device=dev)
        p.run(f1, [vs], iterations=2)
        p.run_noalloc(f2, [vs], iterations=2, residual=None)
        torch.cuda.synchronize()
        for a, b in zip(f1, f2):
            assert torch.equal(a, b)


def test_noalloc_refusals_before_enqueue(dev):
    import ctypes

    from paper_2306_13002_amd.stencil import lib

    # more blocks than the scratch holds (1 x 256 x 520 blocks of 64 x 1 x 1):
    # refused before the grid pointers are even looked at
    with Plan("wave25", (64, 256, 520), variant="plain", coef=synth.WAVE25_COEF, tile=(64, 1, 1)) as p:
        assert lib().stencil_run_noalloc(p._h, None, None, 1, None, None) == E_UNSUPPORTED
    # a misaligned residual pointer
    n = (20, 20, 20)
    fields, coefs = _wave_case(n)
    with Plan("wave25", n, variant="saturated", coef=synth.WAVE25_COEF) as p:
        f = [torch.tensor(a, device=dev) for a in fields]
        vs = torch.tensor(coefs[0], device=dev)
        buf = torch.zeros(2, dtype=torch.float64, device=dev)
        fp = (ctypes.c_void_p * 2)(f[0].data_ptr(), f[1].data_ptr())
        cp = (ctypes.c_void_p * 1)(vs.data_ptr())
        st = lib().stencil_run_noalloc(p._h, fp, cp, 1, ctypes.c_void_p(buf.data_ptr() + 4), None)
        assert st == E_INVAL
    # GENERIC plans running generated kernels
    s = synth.generic_stencil(3, max_edge=24)
    with Plan("generic", s["n"], variant="saturated", dtype=s["dtype"], radius=s["radius"], coef=s["coef"],
              taps=s["taps"], cids=s["cids"]) as p:
        u = synth.generic_input(s["n"], s["radius"], s["dtype"])
        f = [torch.tensor(u, device=dev), torch.tensor(u, device=dev)]
        with pytest.raises(StencilError) as e:
            p.run_noalloc(f, None, iterations=1)
        assert e.value.status == E_UNSUPPORTED
