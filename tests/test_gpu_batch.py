"""Batched plans: many uneven HEAT3D7 grids in one graph launch.

Each problem is bit-identical to its own single plan with the same form
and launch shape (same tile body, same operation order); single plans are
pinned to the oracle elsewhere, and a few problems are checked against the
oracle directly.  Graph replays are interleaved with eager work and each is
checked against the eager single-plan result."""
import numpy as np
import pytest

import oracle
from paper_2306_13002_amd import synth
from gpu_util import inner, maxrel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


SIZES = [(9, 7, 5), (33, 12, 70), (64, 64, 64), (65, 20, 11), (17, 97, 40), (100, 30, 31), (1, 1, 1), (40, 41, 129)]


def fields_for(sizes, dev, stream0=20):
    us = [synth.heat3d7_input(*n, stream=stream0 + i) for i, n in enumerate(sizes)]
    fs = [(torch.tensor(u, device=dev), torch.full(u.shape, float("nan"), dtype=torch.float64, device=dev))
          for u in us]
    return us, fs


def single(n, u0, T, dev, **kw):
    from paper_2306_13002_amd.stencil import Plan
    p = Plan("heat3d7", n, coef=(0.4, 0.1), **kw)
    f = [torch.tensor(u0, device=dev), torch.full(u0.shape, float("nan"), dtype=torch.float64, device=dev)]
    p.run(f, iterations=T)
    r = p.residual()
    p.close()
    return f[0].cpu().numpy(), r


@pytest.mark.parametrize("variant,tile", [("saturated", (32, 8, 8)), ("saturated", (64, 4, 16)),
                                          ("plain", (64, 4, 1)), ("plain", (128, 2, 1)),
                                          ("saturated_t2", (32, 8, 8)), ("saturated_t2", (64, 4, 16)),
                                          ("saturated_t3", (28, 28, 32)), ("saturated_t3", (60, 12, 8))])
@pytest.mark.parametrize("T", [3, 4, 5])
def test_batch_bitwise_equals_single(dev, variant, tile, T):
    from paper_2306_13002_amd.stencil import BatchPlan
    us, fs = fields_for(SIZES, dev)
    bp = BatchPlan(SIZES, variant=variant, tile=tile)
    bp.run(fs, iterations=T)
    res = bp.residuals()
    tot = bp.residual()
    bp.close()
    for i, (n, u0) in enumerate(zip(SIZES, us)):
        want, wr = single(n, u0, T, dev, variant=variant, tile=tile)
        got = fs[i][0].cpu().numpy()
        assert np.array_equal(got, want), f"problem {i} {n}"
        assert abs(res[i] - wr) <= 1e-12 * wr
    assert abs(tot - sum(res)) <= 1e-12 * tot


def test_batch_against_oracle(dev):
    from paper_2306_13002_amd.stencil import BatchPlan
    sizes = SIZES[:4]
    us, fs = fields_for(sizes, dev, stream0=40)
    bp = BatchPlan(sizes, variant="saturated", tile=(32, 8, 8))
    bp.run(fs, iterations=5)
    res = bp.residuals()
    bp.close()
    for i, (n, u0) in enumerate(zip(sizes, us)):
        want, wr = oracle.heat(u0, 5, 0.4, 0.1)
        got = fs[i][0].cpu().numpy()
        assert maxrel(inner(got, 1), inner(want, 1)) <= 1e-12
        assert np.array_equal(got[0], u0[0])
        assert abs(res[i] - wr) <= 1e-10 * wr


def test_graph_replays_with_eager_work_between(dev):
    from paper_2306_13002_amd.stencil import BatchPlan
    sizes = SIZES[:5]
    us, fs = fields_for(sizes, dev, stream0=60)
    bp = BatchPlan(sizes, variant="saturated", tile=(64, 4, 16))
    state = [u.copy() for u in us]
    for rep in range(4):
        bp.run(fs, iterations=3)  # replays the same graph after the first capture
        res = bp.residuals()
        # eager work of the program between replays
        junk = torch.randn(1 << 20, device=dev)
        junk.mul_(2.0).sum().item()
        torch.cuda.synchronize()
        for i, n in enumerate(sizes):
            want, wr = single(n, state[i], 3, dev, variant="saturated", tile=(64, 4, 16))
            got = fs[i][0].cpu().numpy()
            assert np.array_equal(got, want), f"replay {rep} problem {i}"
            assert abs(res[i] - wr) <= 1e-12 * wr
            state[i] = want
    bp.close()


def test_batch_tuned_workload(dev):
    # the 64-problem workload (edges 32..160, T = 50) with tuned classes,
    # against 64 separate plain runs
    from paper_2306_13002_amd.stencil import BatchPlan
    sizes = synth.heat3d7_batch_sizes()
    us, fs = fields_for(sizes, dev, stream0=1)
    bp = BatchPlan(sizes, tune="exhaustive")
    bp.run(fs, iterations=50)
    res = bp.residuals()
    bp.close()
    for i, n in enumerate(sizes):
        want, wr = single(n, us[i], 50, dev, variant="plain")
        got = fs[i][0].cpu().numpy()
        assert maxrel(inner(got, 1), inner(want, 1)) <= 1e-12, f"problem {i}"
        assert abs(res[i] - wr) <= 1e-10 * wr
    # two problems fully against the oracle
    for i in sorted(range(len(sizes)), key=lambda b: np.prod(sizes[b]))[:2]:
        want, _ = oracle.heat(us[i], 50, 0.4, 0.1)
        assert maxrel(inner(fs[i][0].cpu().numpy(), 1), inner(want, 1)) <= 1e-12


def test_batch_two_sweep_tuned_workload(dev):
    """The 64-problem workload with two-sweep classes tuned in place (the
    benchmark's configuration), against 64 separate plain runs."""
    from paper_2306_13002_amd.stencil import BatchPlan, StencilError
    sizes = synth.heat3d7_batch_sizes()
    us, fs = fields_for(sizes, dev, stream0=1)
    bp = BatchPlan(sizes, tune="exhaustive", variant="saturated_t2")
    bp.run(fs, iterations=50)
    res = bp.residuals()
    # classes: edge buckets (<= 64, then 32 wide), numbered from the smallest,
    # each problem in exactly one, every class with a two-sweep launch shape
    classes = bp.classes()
    bucket = lambda n: 0 if max(n) <= 64 else (max(n) - 65) // 32 + 1
    assert sorted(i for c in classes for i in c["problems"]) == list(range(len(sizes)))
    keys = [bucket(sizes[c["problems"][0]]) for c in classes]
    assert keys == sorted(set(keys))
    for c in classes:
        assert {bucket(sizes[i]) for i in c["problems"]} == {bucket(sizes[c["problems"][0]])}
        assert c["variant"] == "saturated_t2" and min(c["tile"]) >= 1
    with pytest.raises(StencilError, match="problem"):
        bp.problem_config(len(sizes))
    bp.close()
    for i, n in enumerate(sizes):
        want, wr = single(n, us[i], 50, dev, variant="plain")
        got = fs[i][0].cpu().numpy()
        assert maxrel(inner(got, 1), inner(want, 1)) <= 1e-12, f"problem {i}"
        assert abs(res[i] - wr) <= 1e-10 * wr
    for i in sorted(range(len(sizes)), key=lambda b: np.prod(sizes[b]))[:2]:
        want, _ = oracle.heat(us[i], 50, 0.4, 0.1)
        assert maxrel(inner(fs[i][0].cpu().numpy(), 1), inner(want, 1)) <= 1e-12


def test_batch_three_sweep_equals_single_sweep_batch(dev):
    """A batch whose classes run three sweeps per launch gives the
    single-sweep batch's grids bit for bit (T not a multiple of three: one
    launch of the remainder first); the residuals agree to rounding (the
    forms sum different block partitions)."""
    from paper_2306_13002_amd.stencil import BatchPlan
    for T in (4, 5, 6):
        out = []
        for variant, tile in (("saturated", (64, 4, 16)), ("saturated_t3", (28, 12, 16))):
            us, fs = fields_for(SIZES, dev)
            bp = BatchPlan(SIZES, variant=variant, tile=tile)
            bp.run(fs, iterations=T)
            out.append(([f[0].cpu().numpy() for f in fs], bp.residuals()))
            bp.close()
        for a, b in zip(out[0][0], out[1][0]):
            assert np.array_equal(a, b), T
        for a, b in zip(out[0][1], out[1][1]):
            assert abs(a - b) <= 1e-12 * a, T


def test_batch_two_sweep_equals_single_sweep_batch(dev):
    """A batch whose classes run two sweeps per launch gives the single-sweep
    batch's result bit for bit (odd T: one single sweep first)."""
    from paper_2306_13002_amd.stencil import BatchPlan
    for T in (5, 6):
        out = []
        for variant in ("saturated", "saturated_t2"):
            us, fs = fields_for(SIZES, dev)
            bp = BatchPlan(SIZES, variant=variant, tile=(64, 4, 16))
            bp.run(fs, iterations=T)
            out.append(([f[0].cpu().numpy() for f in fs], bp.residuals()))
            bp.close()
        for a, b in zip(out[0][0], out[1][0]):
            assert np.array_equal(a, b)
        assert list(out[0][1]) == list(out[1][1])
