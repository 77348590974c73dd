"""The paper's ablation forms (CSE+SAT, CSE+BULK, per-point ACCSAT) for the
leapfrog and pressure kernels.  Exact relations: CSE+BULK reorders only the
loads, so it is bit-identical to PLAIN; CSE+SAT, ACCSAT_POINT and SATURATED
evaluate the same rewritten arithmetic, so they are bit-identical to each
other; all match the oracle within the form's bar."""
import numpy as np
import pytest

import oracle
from paper_2306_13002_amd import synth
from gpu_util import inner, maxrel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
FORMS = ["plain", "cse_sat", "cse_bulk", "accsat_point", "saturated"]


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_wave25_forms(dev):
    from paper_2306_13002_amd.stencil import Plan
    n = (45, 22, 19)
    a, b, v = synth.wave25_inputs(*n, seed=11)
    out = {}
    for form in FORMS:
        p = Plan("wave25", n, variant=form, coef=synth.WAVE25_COEF)
        f = [torch.tensor(a, device=dev), torch.tensor(b, device=dev)]
        p.run(f, [torch.tensor(v, device=dev)], iterations=3)
        out[form] = (f[0].cpu().numpy(), f[1].cpu().numpy(), p.residual())
        p.close()
    A, B, wr = oracle.wave25(a, b, v, synth.WAVE25_COEF, 3)
    assert np.array_equal(out["cse_bulk"][0], out["plain"][0]) and np.array_equal(out["cse_bulk"][1], out["plain"][1])
    assert np.array_equal(out["plain"][0], A)
    for form in ("accsat_point", "saturated"):
        assert np.array_equal(out[form][0], out["cse_sat"][0]) and np.array_equal(out[form][1], out["cse_sat"][1])
    assert maxrel(inner(out["cse_sat"][0], 4), inner(A, 4)) <= 1e-12
    for form in FORMS:
        assert abs(out[form][2] - wr) <= 1e-10 * wr


def test_poisson19_forms(dev):
    from paper_2306_13002_amd.stencil import Plan
    n = (70, 19, 23)
    p0, cf = synth.poisson19_random_inputs((n[2] + 2, n[1] + 2, n[0] + 2), seed=12)
    out = {}
    for form in FORMS:
        p = Plan("poisson19", n, variant=form, omega=0.8)
        f = [torch.tensor(p0, device=dev), torch.zeros(p0.shape, dtype=torch.float32, device=dev)]
        p.run(f, [torch.tensor(c, device=dev) for c in cf], iterations=3)
        out[form] = (f[0].cpu().numpy(), p.residual())
        p.close()
    w32, g32 = oracle.poisson19(p0, cf, 0.8, 3, mode="F32STORE")
    w64, _ = oracle.poisson19(p0, cf, 0.8, 3, mode="F64")
    assert np.array_equal(out["cse_bulk"][0], out["plain"][0])
    assert np.array_equal(out["plain"][0].astype(np.float64), w32)
    for form in ("accsat_point", "saturated"):
        assert np.array_equal(out[form][0], out["cse_sat"][0])
    assert maxrel(inner(out["cse_sat"][0], 1), inner(w64, 1)) <= 1e-5
    for form in FORMS:
        assert abs(out[form][1] - g32) <= 1e-5 * g32
