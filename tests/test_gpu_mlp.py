"""Cost-model MLP kernels (HIP, FP32) against the FP64 numpy oracle, graph
replay against eager launches, and MODEL tuning through a model file."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import mlp as ref
from paper_2306_13002_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def data(n=300, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.normal(2.0, 3.0, size=(n, 24)).astype(np.float32)
    X[:, 5] = 8.0  # a constant feature (std 0 -> 1)
    t = (0.3 * X[:, 0] - 0.05 * X[:, 3] ** 2 + np.sin(X[:, 7])).astype(np.float32)
    return X, t


def test_predict_matches_oracle(dev):
    from paper_2306_13002_amd.stencil import mlp_predict
    X, _ = data()
    rng = np.random.default_rng(1)
    th = rng.normal(0, 0.2, ref.N_PARAMS)
    mean, std = X.mean(0), np.where(X.std(0) > 0, X.std(0), 1.0)
    model = np.concatenate([mean, std, th]).astype(np.float32)
    got = mlp_predict(model, X)
    want = ref.predict(model[48:].astype(np.float64), model[:24].astype(np.float64), model[24:48].astype(np.float64), X)
    np.testing.assert_allclose(got, want, rtol=2e-4, atol=2e-4 * np.abs(want).max())


def test_first_steps_match_oracle(dev):
    from paper_2306_13002_amd.stencil import mlp_train
    X, t = data()
    init = synth.mlp_init()
    model, loss = mlp_train(X, t, init, 5, 1e-3)
    th, mean, std, hist = ref.train(init.astype(np.float64), X.astype(np.float64), t.astype(np.float64), 5, 1e-3)
    np.testing.assert_allclose(model[:24], mean, rtol=1e-5)
    np.testing.assert_allclose(model[24:48], np.where(std > 0, std, 1.0), rtol=1e-5)
    np.testing.assert_allclose(loss, hist, rtol=1e-4)
    d = np.abs(model[48:] - th)
    # Adam's normalized step is +-lr per parameter; only near-zero gradients
    # (sign decided by rounding) may differ, by at most 2 lr per step
    assert np.mean(d <= 1e-5) >= 0.99
    assert d.max() <= 5 * 2e-3 + 1e-5


def test_training_trajectory_and_learning(dev):
    from paper_2306_13002_amd.stencil import mlp_train, mlp_predict
    X, t = data(600, seed=3)
    init = synth.mlp_init()
    model, loss = mlp_train(X, t, init, 300, 1e-3)
    _, _, _, hist = ref.train(init.astype(np.float64), X.astype(np.float64), t.astype(np.float64), 300, 1e-3)
    np.testing.assert_allclose(loss, hist, rtol=2e-2)
    assert loss[-1] < 0.1 * loss[0]
    pred = mlp_predict(model, X)
    assert np.mean((pred - t) ** 2) <= 1.05 * loss[-1] + 1e-6


def test_graph_replay_equals_eager_and_is_deterministic(dev):
    X, t = data(257, seed=4)
    init = synth.mlp_init()
    code = ("import sys, numpy as np; sys.path.insert(0, %r)\n"
            "from paper_2306_13002_amd.stencil import mlp_train\n"
            "X = np.load(sys.argv[1]); t = np.load(sys.argv[2]); i = np.load(sys.argv[3])\n"
            "m, l = mlp_train(X, t, i, 40, 1e-3)\n"
            "np.save(sys.argv[4], m); np.save(sys.argv[5], l)\n") % ROOT
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        for nm, a in (("X", X), ("t", t), ("i", init)):
            np.save(os.path.join(d, nm + ".npy"), a)
        outs = []
        for g in ("1", "0", "1"):
            env = dict(os.environ, STENCIL_MLP_GRAPH=g)
            mp, lp = os.path.join(d, f"m{len(outs)}.npy"), os.path.join(d, f"l{len(outs)}.npy")
            r = subprocess.run([sys.executable, "-c", code, *(os.path.join(d, x + ".npy") for x in "Xti"), mp, lp],
                               env=env, capture_output=True, text=True, timeout=300)
            assert r.returncode == 0, r.stderr
            outs.append((np.load(mp), np.load(lp)))
        for m, l in outs[1:]:
            assert np.array_equal(m, outs[0][0]) and np.array_equal(l, outs[0][1])


def test_model_tuning_picks_an_offered_candidate(dev, tmp_path):
    from paper_2306_13002_amd.stencil import candidates, features, mlp_train
    kw = dict(coef=(0.4, 0.1))
    n = (90, 70, 50)
    cands = candidates("heat3d7", n, **kw)
    X = np.stack([features("heat3d7", n, c, **kw) for c in cands])
    # a model that prefers small predicted time where feature 11 (log2 tile x) is 5
    t = np.abs(X[:, 11] - 5.0).astype(np.float32) + 0.1 * X[:, 10]
    model, loss = mlp_train(X, t, synth.mlp_init(), 400, 3e-3)
    path = tmp_path / "model.json"
    json.dump({"mean": model[:24].tolist(), "std": model[24:48].tolist(), "params": model[48:].tolist()},
              open(path, "w"))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2306_13002_amd.stencil import Plan\n"
            "p = Plan('heat3d7', (90, 70, 50), coef=(0.4, 0.1), tune='model')\n"
            "print('CFG', p.config())\n") % ROOT
    env = dict(os.environ, STENCIL_COST_MODEL=str(path), STENCIL_LOG="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    assert "model pick kind=2" in r.stderr
    line = [l for l in r.stdout.splitlines() if l.startswith("CFG")][0]
    assert "'tile': (32," in line
    # no model file: falls back to exhaustive tuning
    env["STENCIL_COST_MODEL"] = str(tmp_path / "missing.json")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "falling back to exhaustive" in r.stderr
