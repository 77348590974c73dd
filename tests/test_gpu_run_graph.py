"""Runs replayed from captured HIP graphs (enabled per plan): the second
identical run of a single plan is captured, later identical runs replay it.  Every replay is
checked against the eager run and the oracle, with eager runs of other
iteration counts, host copies and synchronizations between the replays."""
import numpy as np
import pytest
import torch

import oracle
from paper_2306_13002_amd import synth
from paper_2306_13002_amd.stencil import Plan

from gpu_util import inner, maxrel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def _state(p, f):
    torch.cuda.synchronize()
    return [x.cpu().numpy().copy() for x in f], p.residual()


def _check_replays(p, f, init, coefs, T, other_T):
    """Run T from `init` six times, with an eager run of other_T in between;
    returns the first (eager) result after checking the others equal it."""
    def reset():
        for x, v in zip(f, init):
            x.copy_(v)

    p.use_graphs(True)
    reset()
    p.run(f, coefs, iterations=T)  # eager
    first = _state(p, f)
    assert p.graph_iterations() == 0
    for k in range(5):
        reset()
        p.run(f, coefs, iterations=T)  # k = 0 captures, then replays
        got = _state(p, f)
        assert p.graph_iterations() == T, k
        for a, b in zip(got[0], first[0]):
            assert np.array_equal(a, b), k
        assert got[1] == first[1], k
        if k == 2:  # eager work in between: another iteration count, twice
            for _ in range(2):
                reset()
                p.run(f, coefs, iterations=other_T)
                torch.cuda.synchronize()
            assert p.graph_iterations() == other_T  # the second one was captured
            reset()
            p.run(f, coefs, iterations=T)  # eager again (the previous run differed)
            got = _state(p, f)
            for a, b in zip(got[0], first[0]):
                assert np.array_equal(a, b)
    return first


@pytest.mark.parametrize("variant,T", [("plain", 4), ("saturated", 5), ("saturated_t2", 5), ("saturated_t2", 6),
                                       ("saturated_t3", 5), ("saturated_t3", 6)])
def test_heat3d7_replay(dev, variant, T):
    n = (45, 19, 23)
    u0 = synth.heat3d7_input(*n, stream=31)
    p = Plan("heat3d7", n, variant=variant, coef=(0.4, 0.1))
    f = [torch.tensor(u0, device=dev), torch.full(u0.shape, float("nan"), dtype=torch.float64, device=dev)]
    init = [torch.tensor(u0, device=dev), torch.full(u0.shape, float("nan"), dtype=torch.float64, device=dev)]
    (g, _), gr = _check_replays(p, f, init, None, T, T + 3)
    p.close()
    want, wr = oracle.heat(u0, T, 0.4, 0.1)
    assert maxrel(inner(g, 1), inner(want, 1)) <= 1e-12
    assert abs(gr - wr) <= 1e-10 * wr


@pytest.mark.parametrize("tile", [(64, 4, 1), (16, 16, 4)])
def test_heat2d5_replay(dev, tile):
    # one sweep per launch, and fused sweeps (10 = 2 + 4 + 4; 3 = 3)
    u0 = synth.heat2d5_input(256)
    p = Plan("heat2d5", (256, 256), variant="plain", coef=(0.6, 0.1), tile=tile)
    f = [torch.tensor(u0, device=dev), torch.zeros(u0.shape, dtype=torch.float64, device=dev)]
    init = [torch.tensor(u0, device=dev), torch.zeros(u0.shape, dtype=torch.float64, device=dev)]
    (g, _), gr = _check_replays(p, f, init, None, 10, 3)
    p.close()
    want, wr = oracle.heat(u0, 10, 0.6, 0.1)
    assert np.array_equal(g, want)
    assert abs(gr - wr) <= 1e-10 * wr


def test_heat3d7_periodic_replay(dev):
    n = (33, 20, 17)
    u0 = synth.heat3d7_input(*n, stream=32)
    p = Plan("heat3d7", n, variant="saturated", coef=(0.4, 0.1), bc="periodic")
    f = [torch.tensor(u0, device=dev), torch.zeros(u0.shape, dtype=torch.float64, device=dev)]
    init = [torch.tensor(u0, device=dev), torch.zeros(u0.shape, dtype=torch.float64, device=dev)]
    (g, _), _ = _check_replays(p, f, init, None, 4, 2)
    p.close()
    want, _ = oracle.heat(u0, 4, 0.4, 0.1, periodic=True)
    assert maxrel(inner(g, 1), inner(want, 1)) <= 1e-12


@pytest.mark.parametrize("variant,T", [("saturated", 3), ("saturated_t2", 4), ("plain", 3)])
def test_poisson19_replay(dev, variant, T):
    pp, cf = synth.poisson19_random_inputs((21, 13, 70), seed=4)  # padded (z, y, x)
    n = (68, 11, 19)
    p = Plan("poisson19", n, variant=variant, omega=0.8)
    f = [torch.tensor(pp, device=dev), torch.zeros(pp.shape, dtype=torch.float32, device=dev)]
    init = [torch.tensor(pp, device=dev), torch.zeros(pp.shape, dtype=torch.float32, device=dev)]
    cs = [torch.tensor(c, device=dev) for c in cf]
    (g, _), gr = _check_replays(p, f, init, cs, T, T + 1)
    p.close()
    w64, _ = oracle.poisson19(pp, cf, 0.8, T, mode="F64")
    assert maxrel(inner(g.astype(np.float64), 1), inner(w64, 1)) <= 1e-5


def test_wave25_replay(dev):
    n = (40, 21, 17)
    a, b, v = synth.wave25_inputs(*n, seed=6)
    p = Plan("wave25", n, variant="saturated", coef=synth.WAVE25_COEF)
    f = [torch.tensor(a, device=dev), torch.tensor(b, device=dev)]
    init = [torch.tensor(a, device=dev), torch.tensor(b, device=dev)]
    vs = [torch.tensor(v, device=dev)]
    (ga, gb), gr = _check_replays(p, f, init, vs, 3, 2)
    p.close()
    A, B, wr = oracle.wave25(a, b, v, synth.WAVE25_COEF, 3)
    assert maxrel(inner(ga, 4), inner(A, 4)) <= 1e-12 and maxrel(inner(gb, 4), inner(B, 4)) <= 1e-12
    assert abs(gr - wr) <= 1e-10 * wr


def test_new_pointers_run_eagerly(dev):
    """Other buffers never replay a graph made for different pointers."""
    n = (45, 19, 23)
    u0 = synth.heat3d7_input(*n, stream=33)
    p = Plan("heat3d7", n, variant="saturated", coef=(0.4, 0.1))
    p.use_graphs(True)
    f1 = [torch.tensor(u0, device=dev), torch.zeros(u0.shape, dtype=torch.float64, device=dev)]
    f2 = [torch.tensor(u0, device=dev), torch.zeros(u0.shape, dtype=torch.float64, device=dev)]
    p.run(f1, iterations=3)
    p.run(f1, iterations=3)  # captured (f1 now holds 6 sweeps)
    assert p.graph_iterations() == 3
    p.run(f2, iterations=3)  # other pointers: eager
    torch.cuda.synchronize()
    want, _ = oracle.heat(u0, 3, 0.4, 0.1)
    assert maxrel(inner(f2[0].cpu().numpy(), 1), inner(want, 1)) <= 1e-12
    want6, _ = oracle.heat(u0, 6, 0.4, 0.1)
    assert maxrel(inner(f1[0].cpu().numpy(), 1), inner(want6, 1)) <= 1e-12
    p.close()


def test_graphs_off_by_default_and_refused_for_generic(dev):
    from paper_2306_13002_amd.stencil import StencilError
    n = (45, 19, 23)
    u0 = synth.heat3d7_input(*n, stream=34)
    p = Plan("heat3d7", n, variant="saturated", coef=(0.4, 0.1))
    f = [torch.tensor(u0, device=dev), torch.zeros(u0.shape, dtype=torch.float64, device=dev)]
    for _ in range(3):
        p.run(f, iterations=2)
    assert p.graph_iterations() == 0
    p.close()
    g = Plan("generic", (20, 20, 20), dtype="f64", radius=1, coef=(0.5, 0.5), taps=[(0, 0, 0), (1, 0, 0)], cids=[0, 1])
    with pytest.raises(StencilError, match="eagerly"):
        g.use_graphs(True)
    g.close()
