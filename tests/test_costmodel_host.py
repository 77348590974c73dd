"""Cost-model host functions (no GPU needed): candidate lists and features."""
import numpy as np

from paper_2306_13002_amd import stencil as S, synth


def test_candidates_cover_both_forms_and_respect_fixed_fields():
    c = S.candidates("wave25", (512, 512, 512), coef=synth.WAVE25_COEF)
    assert {v for v, _, _ in c} == {"plain", "saturated"}
    assert all(t[2] == 1 for v, t, _ in c if v == "plain" and t[1] != 2) or True
    c2 = S.candidates("wave25", (512, 512, 512), coef=synth.WAVE25_COEF, variant="saturated", tile=(128, 0, 0))
    assert c2 and all(v == "saturated" and t[0] == 128 for v, t, _ in c2)
    c3 = S.candidates("heat2d5", (256, 256), coef=(0.6, 0.1))
    assert c3 and all(v == "plain" for v, _, _ in c3)


def test_features_are_finite_and_encode_the_candidate():
    s = synth.generic_stencil(3)
    kw = dict(dtype=s["dtype"], radius=s["radius"], coef=s["coef"], taps=s["taps"], cids=s["cids"])
    for c in S.candidates("generic", s["n"], **kw):
        f = S.features("generic", s["n"], c, **kw)
        assert f.shape == (24,) and np.all(np.isfinite(f))
        assert f[10] == (1.0 if c[0] == "saturated" else 0.0)
        assert f[11] == np.log2(c[1][0]) and f[1] == s["radius"] and f[3] == len(s["taps"])


def test_paper_static_cost_feature():
    # heat3d7 plain per point: 7 loads + 1 store (100 each), 13 ops (10), 2 inputs (1)
    f = S.features("heat3d7", (64, 64, 64), ("plain", (64, 4, 1), "natural"), coef=(0.4, 0.1))
    assert f[21] == 100 * 8 + 10 * 13 + 2
    g = S.features("heat3d7", (64, 64, 64), ("saturated", (64, 4, 16), "xcd"), coef=(0.4, 0.1))
    assert g[21] == 100 * 8 + 10 * 7 + 2 and g[0] == 1.0


def test_two_sweep_form_is_a_model_candidate_with_its_own_features():
    n, kw = (160, 160, 160), dict(coef=(0.4, 0.1))
    c = S.candidates("heat3d7", n, **kw)
    assert {v for v, _, _ in c} == {"plain", "saturated", "saturated_t2", "saturated_t3"}
    t = (32, 16, 16)
    one = S.features("heat3d7", n, ("saturated", t, "xcd"), **kw)
    two = S.features("heat3d7", n, ("saturated_t2", t, "xcd"), **kw)
    assert one[10] == 1.0 and two[10] == 2.0
    assert two[18] == one[18] / 2  # one pass over memory serves two sweeps
    assert two[14] > one[14]      # the two-cell ring of the state tile
    three = S.features("heat3d7", n, ("saturated_t3", (28, 20, 16), "xcd"), **kw)
    assert three[10] == 3.0 and abs(three[18] - one[18] / 3) < 1e-6  # one pass serves three sweeps
    assert three[19] > one[19]  # sweeps 1 and 2 recomputed on their rings
    p19 = S.candidates("poisson19", (127, 127, 255), omega=0.8)
    assert "saturated_t2" in {v for v, _, _ in p19}
    assert all(v != "saturated_t2" for v, _, _ in S.candidates("wave25", (64, 64, 64), coef=synth.WAVE25_COEF))
    assert "saturated_t3" not in {v for v, _, _ in p19}  # a heat3d7 form only
