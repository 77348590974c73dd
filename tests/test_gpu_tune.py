"""Exhaustive autotuner: the chosen launch shape is an offered one, results
under it match the oracle, and the cache (in-process and JSON-lines file)
returns the same choice without re-timing.

The pick itself has no oracle: the exhaustive timing is the reference, and
several shapes within timing noise are equally correct."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2306_13002_amd import synth
from gpu_util import inner, maxrel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_tuned_heat3d7_matches_oracle_and_caches(dev):
    from paper_2306_13002_amd.stencil import Plan
    n = (61, 35, 47)
    u0 = synth.heat3d7_input(*n, stream=11)
    p = Plan("heat3d7", n, coef=(0.4, 0.1), tune="exhaustive")
    cfg = p.config()
    assert cfg["variant"] in ("plain", "saturated", "saturated_t2", "saturated_t3")  # exhaustive AUTO weighs all four
    f = [torch.tensor(u0, device=dev), torch.full(u0.shape, float("nan"), dtype=torch.float64, device=dev)]
    p.run(f, iterations=4)
    got = f[0].cpu().numpy()
    want, wr = oracle.heat(u0, 4, 0.4, 0.1)
    assert maxrel(inner(got, 1), inner(want, 1)) <= 1e-12
    assert abs(p.residual() - wr) <= 1e-10 * wr
    p.close()
    q = Plan("heat3d7", n, coef=(0.4, 0.1), tune="exhaustive")
    assert q.config() == cfg
    q.close()


@pytest.mark.parametrize("variant", ["plain", "saturated"])
def test_tuned_variant_restriction(dev, variant):
    from paper_2306_13002_amd.stencil import Plan
    n = (70, 19, 23)
    p0, cf = synth.poisson19_random_inputs((n[2] + 2, n[1] + 2, n[0] + 2), seed=4)
    p = Plan("poisson19", n, variant=variant, tune="exhaustive", omega=0.8)
    assert p.config()["variant"] == variant
    f = [torch.tensor(p0, device=dev), torch.zeros(p0.shape, dtype=torch.float32, device=dev)]
    p.run(f, [torch.tensor(c, device=dev) for c in cf], iterations=3)
    w64, _ = oracle.poisson19(p0, cf, 0.8, 3, mode="F64")
    assert maxrel(inner(f[0].cpu().numpy(), 1), inner(w64, 1)) <= 1e-5
    p.close()


def test_tuned_partial_request_keeps_given_fields(dev):
    from paper_2306_13002_amd.stencil import Plan
    p = Plan("wave25", (40, 24, 30), variant="saturated", coef=synth.WAVE25_COEF, tune="exhaustive",
             tile=(64, 0, 0))
    cfg = p.config()
    assert cfg["tile"][0] == 64 and cfg["variant"] == "saturated"
    p.close()


def test_tune_cache_file_roundtrip(tmp_path):
    cache = tmp_path / "tune.jsonl"
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2306_13002_amd.stencil import Plan\n"
            "p = Plan('heat3d7', (33, 29, 31), coef=(0.4, 0.1), tune='exhaustive')\n"
            "print('CFG', p.config())\n") % ROOT
    env = dict(os.environ, STENCIL_TUNE_CACHE=str(cache), STENCIL_LOG="1")
    r1 = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert r1.returncode == 0, r1.stderr
    lines = cache.read_text().strip().splitlines()
    assert len(lines) == 1
    e = json.loads(lines[0])
    assert e["key"].startswith("k2/") and e["us"] > 0
    assert "tune kind=2" in r1.stderr
    r2 = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert r2.returncode == 0, r2.stderr
    assert "tune kind=2" not in r2.stderr  # served from the file, not re-timed
    cfg1 = [l for l in r1.stdout.splitlines() if l.startswith("CFG")]
    cfg2 = [l for l in r2.stdout.splitlines() if l.startswith("CFG")]
    assert cfg1 == cfg2
    assert len(cache.read_text().strip().splitlines()) == 1


def test_batch_class_tuning_cache_roundtrip(tmp_path):
    """Batch classes are timed in place once per class (one cache line each,
    keyed by the class's extents) and served from the file afterwards."""
    cache = tmp_path / "tune.jsonl"
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2306_13002_amd.stencil import BatchPlan\n"
            "b = BatchPlan([(40, 33, 35), (30, 41, 37), (90, 70, 66)], tune='exhaustive', variant='saturated')\n"
            "print('CFG', b.config())\n") % ROOT
    env = dict(os.environ, STENCIL_TUNE_CACHE=str(cache), STENCIL_LOG="1")
    r1 = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert r1.returncode == 0, r1.stderr
    keys = [json.loads(l)["key"] for l in cache.read_text().strip().splitlines()]
    assert len(keys) == 2 and all(k.startswith("batch/k2/") for k in keys)  # two size classes
    assert "tune batch class (2 problems)" in r1.stderr and "tune batch class (1 problems)" in r1.stderr
    r2 = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert r2.returncode == 0, r2.stderr
    assert "tune batch class" not in r2.stderr
    cfg1 = [l for l in r1.stdout.splitlines() if l.startswith("CFG")]
    cfg2 = [l for l in r2.stdout.splitlines() if l.startswith("CFG")]
    assert cfg1 == cfg2
    assert len(cache.read_text().strip().splitlines()) == 2


@pytest.mark.parametrize("tune", ["exhaustive", "model"])
def test_tuned_three_sweep_heat3d7(dev, tune):
    """Both tuners, asked for the three-sweep form with the shape open, pick
    one of its tiles; the tuned run matches the oracle (T = 7: a one-sweep
    launch, then two three-sweep passes)."""
    from paper_2306_13002_amd.stencil import Plan
    n = (61, 35, 47)
    u0 = synth.heat3d7_input(*n, stream=12)
    p = Plan("heat3d7", n, variant="saturated_t3", coef=(0.4, 0.1), tune=tune)
    cfg = p.config()
    assert cfg["variant"] == "saturated_t3"
    assert tuple(cfg["tile"][:2]) in [(28, 28), (28, 20), (28, 12), (60, 12)]
    f = [torch.tensor(u0, device=dev), torch.full(u0.shape, float("nan"), dtype=torch.float64, device=dev)]
    p.run(f, iterations=7)
    want, wr = oracle.heat(u0, 7, 0.4, 0.1)
    assert maxrel(inner(f[0].cpu().numpy(), 1), inner(want, 1)) <= 1e-12
    assert abs(p.residual() - wr) <= 1e-10 * wr
    p.close()


def test_tuned_two_sweep_poisson19(dev):
    """The two-sweep form's tuned pick is one of its own shapes and its result
    equals the single-sweep form at that shape."""
    from paper_2306_13002_amd.stencil import Plan
    n = (50, 21, 30)
    p0, cf = synth.poisson19_random_inputs((n[2] + 2, n[1] + 2, n[0] + 2), seed=9)
    p = Plan("poisson19", n, variant="saturated_t2", omega=0.8, tune="exhaustive")
    cfg = p.config()
    assert cfg["variant"] == "saturated_t2"
    assert tuple(cfg["tile"][:2]) in [(32, 4), (32, 8), (64, 4), (64, 8), (128, 4)]
    outs = []
    for plan in (p, Plan("poisson19", n, variant="saturated", omega=0.8, tile=cfg["tile"], tile_map=cfg["tile_map"])):
        f = [torch.tensor(p0, device=dev), torch.full(p0.shape, float("nan"), dtype=torch.float32, device=dev)]
        plan.run(f, [torch.tensor(c, device=dev) for c in cf], iterations=6)
        outs.append((f[0].cpu().numpy(), plan.residual()))
        plan.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1] == outs[1][1]
    # exhaustive and model tuning of AUTO weigh it against the other forms
    # (poisson19 has no three-sweep form)
    a = Plan("poisson19", n, variant="auto", omega=0.8, tune="exhaustive")
    assert a.config()["variant"] in ("plain", "saturated", "saturated_t2")
    a.close()
    m = Plan("poisson19", n, variant="auto", omega=0.8, tune="model")
    assert m.config()["variant"] in ("plain", "saturated", "saturated_t2")
    m.close()
