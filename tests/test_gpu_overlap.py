"""stencil_run refuses grids whose padded spans overlap where one is
written (both fields; a read-only coefficient grid against either field),
before anything is enqueued; coefficient grids may alias each other."""
import numpy as np
import pytest

import oracle
from paper_2306_13002_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def test_overlapping_fields_rejected(dev):
    from paper_2306_13002_amd.stencil import E_INVAL, Plan, StencilError

    n = (10, 9, 8)
    span = 12 * 11 * 10
    buf = torch.zeros(2 * span, dtype=torch.float64, device=dev)
    with Plan("heat3d7", n, variant="plain", coef=(0.4, 0.1)) as p:
        for shift in (1, span - 1):
            with pytest.raises(StencilError) as e:
                p.run([buf[:span], buf[shift:shift + span]], iterations=1)
            assert e.value.status == E_INVAL and "overlap" in str(e.value)
        p.run([buf[:span], buf[span:]], iterations=1)  # adjacent, disjoint: fine
        torch.cuda.synchronize()


def test_wave25_vsq_overlapping_a_field_rejected(dev):
    from paper_2306_13002_amd.stencil import E_INVAL, Plan, StencilError

    n = (9, 8, 7)
    a, b, v = synth.wave25_inputs(*n)
    span = a.size
    buf = torch.zeros(3 * span, dtype=torch.float64, device=dev)
    with Plan("wave25", n, variant="saturated", coef=synth.WAVE25_COEF) as p:
        with pytest.raises(StencilError) as e:
            p.run([buf[:span], buf[span:2 * span]], [buf[span + 8:2 * span + 8]], iterations=1)
        assert e.value.status == E_INVAL and "overlap" in str(e.value)


def test_poisson19_aliased_coefficients_allowed(dev):
    # a0 = a1 = a2 = c0 = c1 = c2 (one grid of ones): read-only aliases are fine
    from paper_2306_13002_amd.stencil import Plan

    shape = (12, 11, 10)
    p0, cf = synth.poisson19_inputs(shape)
    want, wg = oracle.poisson19(p0, cf, 0.8, 2, mode="F32STORE")
    ones = torch.tensor(cf[0], device=dev)
    cs = [ones if i in (0, 1, 2, 7, 8, 9, 10) else torch.tensor(c, device=dev) for i, c in enumerate(cf)]
    f = [torch.tensor(p0, device=dev), torch.empty(p0.shape, dtype=torch.float32, device=dev)]
    with Plan("poisson19", (shape[2] - 2, shape[1] - 2, shape[0] - 2), variant="plain", omega=0.8) as p:
        p.run(f, cs, iterations=2)
        g = p.residual()
    assert np.array_equal(f[0].cpu().numpy().astype(np.float64), want)
    assert abs(g - wg) <= 1e-10 * wg
