"""Host-side tests of the saturator (include/saturator.h), no GPU needed.

The e-graph rewriting is checked against mathematics, not against itself:
every extracted program is evaluated in exact rational arithmetic and must
equal the program as written (the rules of Table tab:rule are identities of
real arithmetic); the forms that apply no rule must evaluate bitwise like
the oracle's plain interpreter; costs follow the paper's cost model; the
greedy extraction is compared with the exhaustive one on small e-graphs;
and the paper's own example (Listings lst:zsolve / lst:zsolvegen) is
reproduced.
"""
import ctypes
import os
import re
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2306_13002_amd import saturator as X
from paper_2306_13002_amd import stencil as S
from paper_2306_13002_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FORMS = ["plain", "cse", "cse_sat", "cse_bulk", "accsat", "accsat_z"]


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "saturator.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sat_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = S.lib()
    syms = header_symbols()
    assert {"sat_generate", "sat_plan", "sat_run", "sat_destroy"} <= set(syms)
    for name in syms:
        assert hasattr(L, name), name


def test_desc_struct_size_checked():
    p = synth.lhs_program()
    d, keep = X.Program.from_dict(p).desc((8, 8, 8))
    d.struct_size -= 8
    st = X._lib().sat_generate(ctypes.byref(d), 0, 0, 0, 0, 0, None, 0, None, 0, None)
    assert st == S.E_INVAL and "struct_size" in S.last_error()


# ---------------------------------------------------------------------------
# evaluation of programs and of extracted SSA


def eval_rpn(prog, load, params, num=Fraction):
    """Plain postfix evaluation at one point; load(a, dx, dy, dz) gives an
    input value.  Returns {output: value}."""
    st, loc, out = [], {}, {}
    for op, a, b, c, d in prog["insns"]:
        if op == 1:
            st.append(num(prog["consts"][a]))
        elif op == 2:
            st.append(params[a])
        elif op == 3:
            st.append(load(a, b, c, d))
        elif op in (4, 5, 6):
            y, x = st.pop(), st.pop()
            st.append(x + y if op == 4 else (x - y if op == 5 else x * y))
        elif op == 7:
            st.append(-st.pop())
        elif op == 8:
            out[a] = st.pop()
        elif op == 9:
            loc[a] = st.pop()
        elif op == 10:
            st.append(loc[a])
    return out


def eval_ssa(ssa, load, params, num=Fraction, fma=None):
    v, out = {}, {}
    for line in ssa.strip().splitlines():
        t = line.split()
        if t[0] == "store":
            out[int(t[1])] = v[t[2]]
            continue
        if t[0] == "set":
            continue
        name, op, args = t[0], t[2], t[3:]
        if op == "const":
            val = num(float.fromhex(args[0]))
        elif op == "param":
            val = params[int(args[0])]
        elif op == "load":
            val = load(*(int(s) for s in args))
        elif op == "neg":
            val = -v[args[0]]
        elif op == "fma":  # fma A B C = A + B*C
            a, b, c = (v[s] for s in args)
            val = fma(b, c, a) if fma else a + b * c
        else:
            x, y = v[args[0]], v[args[1]]
            val = {"add": x + y, "sub": x - y, "mul": x * y}[op]
        v[name] = val
    return out


def rational_inputs(prog, seed):
    rng = np.random.default_rng(seed)
    vals = {}

    def load(a, dx, dy, dz):
        key = (a, dx, dy, dz)
        if key not in vals:
            vals[key] = Fraction(int(rng.integers(1, 1000)), int(rng.integers(1, 97)))
        return vals[key]

    params = [Fraction(int(rng.integers(1, 1000)), int(rng.integers(1, 97))) for _ in range(prog["n_params"])]
    return load, params


def programs():
    out = [("lhs", synth.lhs_program())]
    out += [(f"rand{i}", synth.random_program(i)) for i in range(6)]
    return out


@pytest.mark.parametrize("name,prog", programs())
@pytest.mark.parametrize("form", FORMS)
def test_extracted_program_equals_written_program_exactly(name, prog, form):
    src, ssa, st = X.generate(prog, (8, 8, 8), form)
    for seed in range(2):
        load, params = rational_inputs(prog, seed)
        want = eval_rpn(prog, load, params)
        got = eval_ssa(ssa, load, params)
        assert got == want
    assert st["cost_extracted"] <= st["cost_input"]


@pytest.mark.parametrize("name,prog", programs())
@pytest.mark.parametrize("form", ["plain", "cse", "cse_bulk"])
def test_forms_without_rules_are_bitwise_the_plain_evaluation(name, prog, form):
    """PLAIN, CSE and CSE+BULK perform exactly the written operations: their
    SSA evaluated in FP64 equals the oracle's interpreter bit for bit."""
    n = (3, 2, 2)
    r = prog["radius"]
    shape = (n[2] + 2 * r, n[1] + 2 * r, n[0] + 2 * r)
    ins = [synth.uniform_f64(21, s, shape) + (1.0 if s % 2 else 0.0) for s in range(prog["n_inputs"])]
    params = [0.5 + 0.25 * i for i in range(prog["n_params"])]
    outs = oracle.program(prog, ins, params, n)
    src, ssa, st = X.generate(prog, n, form)
    for k in range(n[2]):
        for j in range(n[1]):
            for i in range(n[0]):
                load = lambda a, dx, dy, dz: float(ins[a][k + r + dz, j + r + dy, i + r + dx])  # noqa: E731
                got = eval_ssa(ssa, load, params, num=float)
                for o, val in got.items():
                    assert val == outs[o][k + r, j + r, i + r]


# ---------------------------------------------------------------------------
# the rules, the cost model, code generation


def single(expr_builder, n_in=3, n_par=0):
    p = X.Program(n_inputs=n_in, n_outputs=1, n_params=n_par, radius=1)
    p.store(0, expr_builder([X.In(a).at() for a in range(n_in)], [X.Param(i) for i in range(n_par)]))
    return p


def ssa_ops(ssa):
    return [ln.split()[2] for ln in ssa.strip().splitlines() if " = " in ln]


def test_fma1_rule():
    """A + B*C -> FMA(A, B, C) saves one operation (cost 10)."""
    for builder in (lambda v: v[0] + v[1] * v[2], lambda v: v[1] * v[2] + v[0]):  # the second needs COMM-ADD
        p = X.Program(n_inputs=3, n_outputs=1, radius=1)
        p.store(0, builder([X.In(a).at() for a in range(3)]))
        _, _, st0 = X.generate(p, (4, 4, 4), "cse")
        _, ssa, st = X.generate(p, (4, 4, 4), "cse_sat")
        assert st["fmas"] == 1 and st["ops"] == 1
        assert "mul" not in ssa_ops(ssa) and "add" not in ssa_ops(ssa)
        assert st["cost_extracted"] == st0["cost_extracted"] - 10


@pytest.mark.parametrize("rule", ["FMA2", "FMA3"])
def test_fma2_fma3_rules(rule):
    """A - B*C -> FMA(A, -B, C) and B*C - A -> FMA(-A, B, C) cost a negation,
    so under the cost model they tie with the written form for one statement
    and win once two statements share the negated operand."""
    v = [X.In(a).at() for a in range(5)]
    p = X.Program(n_inputs=5, n_outputs=2, radius=1)
    if rule == "FMA2":
        p.store(0, v[0] - v[1] * v[2])
        p.store(1, v[3] - v[1] * v[4])
    else:
        p.store(0, v[1] * v[2] - v[0])
        p.store(1, v[3] * v[4] - v[0])
    _, _, st0 = X.generate(p, (4, 4, 4), "cse")
    _, ssa, st = X.generate(p, (4, 4, 4), "cse_sat")
    assert st["fmas"] == 2 and ssa_ops(ssa).count("neg") == 1
    assert st["cost_extracted"] == st0["cost_extracted"] - 10
    one = X.Program(n_inputs=5, n_outputs=1, radius=1)
    one.store(0, v[0] - v[1] * v[2] if rule == "FMA2" else v[1] * v[2] - v[0])
    assert X.generate(one, (4, 4, 4), "cse_sat")[2]["cost_extracted"] == X.generate(one, (4, 4, 4), "cse")[2][
        "cost_extracted"]


def test_constant_folding():
    p = single(lambda v, p: (X.Const(2.0) * X.Const(3.0)) * v[0] + X.Const(0.5) * X.Const(4.0), n_in=1)
    _, ssa, st = X.generate(p, (4, 4, 4), "cse_sat")
    consts = [float.fromhex(ln.split()[3]) for ln in ssa.splitlines() if " const " in ln]
    assert 6.0 in consts and 2.0 in consts
    assert st["ops"] == 1 and st["fmas"] == 1  # fma(6, x, 2)
    # without the rules nothing is folded
    _, ssa0, st0 = X.generate(p, (4, 4, 4), "cse")
    assert st0["ops"] == 4


def test_comm_assoc_expose_common_subexpressions():
    """x*y*z written two ways in two statements: COMM/ASSOC put both in one
    e-class, so the saturated form computes the product once."""
    p = X.Program(n_inputs=3, n_outputs=2, radius=1)
    x, y, z = (X.In(a).at() for a in range(3))
    p.store(0, (x * y) * z)
    p.store(1, z * (y * x))
    _, _, st0 = X.generate(p, (4, 4, 4), "cse")
    _, ssa, st = X.generate(p, (4, 4, 4), "cse_sat")
    assert st0["ops"] == 4 and st["ops"] == 2
    assert st["cost_extracted"] == st0["cost_extracted"] - 20


def test_cse_shares_loads_and_subexpressions():
    p = X.Program(n_inputs=2, n_outputs=2, radius=1)
    a, b = X.In(0).at(0, 0, 1), X.In(1).at()
    p.store(0, a * b + a)
    p.store(1, a * b)
    _, ssa_p, stp = X.generate(p, (4, 4, 4), "plain")
    _, ssa_c, stc = X.generate(p, (4, 4, 4), "cse")
    assert stp["loads"] == 5 and stc["loads"] == 2
    assert stp["ops"] == 3 and stc["ops"] == 2


def test_bulk_forms_issue_every_load_first_in_address_order():
    prog = synth.lhs_program()
    for form in ("cse_bulk", "accsat"):
        _, ssa, st = X.generate(prog, (8, 8, 8), form)
        lines = [ln for ln in ssa.strip().splitlines() if " = " in ln]
        kinds = [ln.split()[2] for ln in lines]
        n_loads = kinds.count("load")
        assert n_loads == 125 == st["loads"]
        assert all(k == "load" for k in kinds[:n_loads])
        keys = [tuple(int(s) for s in ln.split()[3:]) for ln in lines[:n_loads]]
        order = [(a, dz, dy, dx) for a, dx, dy, dz in keys]
        assert order == sorted(order)
    # the non-bulk forms place each load right before its first use
    _, ssa, _ = X.generate(prog, (8, 8, 8), "cse_sat")
    kinds = [ln.split()[2] for ln in ssa.strip().splitlines() if " = " in ln]
    assert kinds.index("mul") < kinds.index("load") + 3


def test_generated_source_shape():
    src, _, st = X.generate(synth.lhs_program(), (162, 162, 162), "accsat", tile=(64, 4))
    assert 'extern "C" __global__ __launch_bounds__(256) void sat_kernel_accsat(SatArgs A)' in src
    assert src.count("A.in[") == 125 and src.count("A.out[") == 75
    assert "fma(" in src and "__restrict__" not in src  # the program's arrays may alias, as written


def test_lhs_program_statistics():
    """The fixed workload: 75 statements, 125 loads; saturation turns most
    products into FMAs and lowers the cost-model cost."""
    prog = synth.lhs_program()
    stats = {f: X.generate(prog, (16, 16, 16), f)[2] for f in FORMS}
    assert stats["plain"]["loads"] == 125 and stats["plain"]["ops"] == 267
    assert stats["cse"]["ops"] < stats["plain"]["ops"]
    assert stats["accsat"]["fmas"] >= 60
    assert stats["accsat"]["ops"] < stats["cse"]["ops"]
    assert stats["accsat"]["cost_extracted"] < stats["cse"]["cost_extracted"] < stats["plain"]["cost_input"]
    assert stats["accsat"]["saturated"] == 1 and stats["accsat"]["enodes"] <= 10000


def tiny_programs():
    out = []
    for i in range(12):
        p = synth.random_program(100 + i, n_inputs=2, n_outputs=1, n_params=1, max_terms=2)
        out.append(p)
    return out


@pytest.mark.parametrize("idx", range(12))
def test_greedy_extraction_matches_exhaustive_on_small_egraphs(idx):
    prog = tiny_programs()[idx]
    try:
        _, _, ex = X.generate(prog, (4, 4, 4), "cse_sat", extract="exact")
    except S.StencilError as e:
        assert e.status == S.E_UNSUPPORTED
        pytest.skip("e-graph too large for the exhaustive extraction")
    _, _, gr = X.generate(prog, (4, 4, 4), "cse_sat", extract="greedy")
    assert gr["cost_extracted"] == ex["cost_extracted"]


def listing_program():
    """The statement of the paper's Listing lst:zsolve:
    temp1 = dt*tz1; temp2 = dt*tz2;
    lhs = -temp2*fjac[k-1] - temp1*njac[k-1] - temp1*dz1."""
    F, N = X.In(0), X.In(1)
    t1, t2 = X.Local(0), X.Local(1)
    dt, tz1, tz2, dz1 = (X.Param(i) for i in range(4))
    p = X.Program(n_inputs=2, n_outputs=1, n_params=4, n_locals=2, radius=1)
    p.set(t1, dt * tz1)
    p.set(t2, dt * tz2)
    p.store(0, -t2 * F.at(0, 0, -1) - t1 * N.at(0, 0, -1) - t1 * dz1)
    return p


def test_paper_listing_example():
    """Listing lst:zsolvegen is the tool's output for that statement: two
    loads, the products dt*tz1 and dt*tz2, and five operations (-temp2,
    temp1*njac, its negation, then an add of a product and a subtract of a
    product, i.e. two FMAs).  Under the cost model (loads 100, inputs 1,
    operations 10) that is 2*100 + 4*1 + 2*10 + 5*10 = 274.  The extraction
    here reaches the same cost, the exhaustive optimum, with an equal
    expression."""
    p = listing_program()
    _, ssa, st = X.generate(p, (8, 8, 8), "accsat")
    assert st["cost_extracted"] == 274.0
    assert st["fmas"] == 2 and st["loads"] == 2
    _, _, ex = X.generate(p, (8, 8, 8), "accsat", extract="exact")
    assert ex["cost_extracted"] == 274.0
    d = p.to_dict()
    load, params = rational_inputs(d, 3)
    assert eval_ssa(ssa, load, params) == eval_rpn(d, load, params)
    # the program as written costs 2 loads, 5 parameter/local reads and 8 operations
    assert st["cost_input"] == 2 * 100 + 8 * 1 + 8 * 10


def test_expression_lowering_is_postfix_in_written_order():
    p = listing_program()
    ins = p.to_dict()["insns"]
    want = [(2, 0, 0, 0, 0), (2, 1, 0, 0, 0), (6, 0, 0, 0, 0), (9, 0, 0, 0, 0),
            (2, 0, 0, 0, 0), (2, 2, 0, 0, 0), (6, 0, 0, 0, 0), (9, 1, 0, 0, 0),
            (10, 1, 0, 0, 0), (7, 0, 0, 0, 0), (3, 0, 0, 0, -1), (6, 0, 0, 0, 0),
            (10, 0, 0, 0, 0), (3, 1, 0, 0, -1), (6, 0, 0, 0, 0), (5, 0, 0, 0, 0),
            (10, 0, 0, 0, 0), (2, 3, 0, 0, 0), (6, 0, 0, 0, 0), (5, 0, 0, 0, 0), (8, 0, 0, 0, 0)]
    assert ins == want


def test_saturation_limits():
    """A 60-term sum explodes under COMM/ASSOC: the e-node limit stops the
    saturation (reported as not saturated) and the result stays exact."""
    p = X.Program(n_inputs=60, n_outputs=1, radius=1)
    e = X.In(0).at()
    for a in range(1, 60):
        e = e + X.In(a).at()
    p.store(0, e)
    _, ssa, st = X.generate(p, (4, 4, 4), "cse_sat")
    assert st["saturated"] == 0 and st["enodes"] < 10000 + 5000
    d = p.to_dict()
    load, params = rational_inputs(d, 0)
    assert eval_ssa(ssa, load, params) == eval_rpn(d, load, params)


BAD = [
    ([(4, 0, 0, 0, 0), (8, 0, 0, 0, 0)], "underflow"),
    ([(3, 5, 0, 0, 0), (8, 0, 0, 0, 0)], "input index"),
    ([(3, 0, 2, 0, 0), (8, 0, 0, 0, 0)], "radius"),
    ([(10, 0, 0, 0, 0), (8, 0, 0, 0, 0)], "before it is set"),
    ([(3, 0, 0, 0, 0), (3, 0, 0, 0, 0), (8, 0, 0, 0, 0)], "exactly one value"),
    ([(3, 0, 0, 0, 0), (8, 3, 0, 0, 0)], "output index"),
    ([(3, 0, 0, 0, 0)], "not terminated"),
    ([(3, 0, 0, 0, 0), (9, 0, 0, 0, 0)], "stores nothing"),
    ([(1, 4, 0, 0, 0), (8, 0, 0, 0, 0)], "constant index"),
    ([(2, 0, 0, 0, 0), (8, 0, 0, 0, 0)], "parameter index"),
    ([(42, 0, 0, 0, 0), (8, 0, 0, 0, 0)], "unknown op"),
]


@pytest.mark.parametrize("insns,msg", BAD)
def test_malformed_programs_rejected(insns, msg):
    prog = dict(n_inputs=1, n_outputs=1, n_params=0, n_locals=1, radius=1, insns=insns, consts=[1.0])
    with pytest.raises(S.StencilError) as ei:
        X.generate(prog, (4, 4, 4), "cse")
    assert ei.value.status == S.E_INVAL and msg in str(ei.value)


def test_bad_shapes_rejected():
    prog = synth.lhs_program()
    with pytest.raises(S.StencilError, match="multiple of 64"):
        X.generate(prog, (8, 8, 8), "cse", tile=(10, 3))
    with pytest.raises(S.StencilError, match="extents"):
        X.generate(prog, (8, 0, 8), "cse")
    with pytest.raises(S.StencilError, match="pitch_y"):
        X.generate(prog, (8, 8, 8), "cse", pitch=(9, 0))
    # the module launch API takes at most 65535 blocks in y and z
    with pytest.raises(S.StencilError, match="65535"):
        X.generate(prog, (4, 4, 70000), "cse")


def _stencil_program(taps, cids, coef, grouped):
    """One output: the generic stencil sum_t coef[cid_t] * u(x + delta_t),
    written tap by tap (plain) or as the hand-grouped saturated form (taps
    sharing a coefficient and a z offset summed, then one product per group)."""
    p = X.Program(n_inputs=1, n_outputs=1, radius=max(max(abs(v) for v in t) for t in taps))
    u = X.In(0)
    if not grouped:
        e = None
        for t, c in zip(taps, cids):
            term = X.Const(coef[c]) * u.at(*t)
            e = term if e is None else e + term
    else:
        groups = {}
        for t, c in zip(taps, cids):
            groups.setdefault((t[2], c), []).append(tuple(t))
        e = None
        for (dz, c), ts in sorted(groups.items()):
            s = None
            for t in sorted(ts, key=lambda q: (q[1], q[0])):
                s = u.at(*t) if s is None else s + u.at(*t)
            term = X.Const(coef[c]) * s
            e = term if e is None else e + term
    p.store(0, e)
    return p


@pytest.mark.parametrize("idx", [2, 3, 4, 5, 7])
def test_engine_on_generic_stencils_matches_or_beats_the_hand_grouping(idx):
    """The generic stencils' saturated kernels use a hand rule (group sums,
    one product per group).  Under the paper's cost model the e-graph,
    started from the plain tap-by-tap sum, finds a form at least as cheap
    (FMA chains tie with factoring: both need one operation per tap), and
    every form is the same polynomial."""
    s = synth.generic_stencil(idx, max_edge=16)
    taps, cids, coef = [tuple(t) for t in s["taps"]], list(s["cids"]), list(s["coef"])
    plain = _stencil_program(taps, cids, coef, grouped=False)
    grouped = _stencil_program(taps, cids, coef, grouped=True)
    _, ssa_e, st_e = X.generate(plain, (8, 8, 8), "cse_sat")
    _, ssa_g, st_g = X.generate(grouped, (8, 8, 8), "cse")
    assert st_e["cost_extracted"] <= st_g["cost_extracted"]
    assert st_e["ops"] <= len(taps)
    d = plain.to_dict()
    load, params = rational_inputs(d, idx)
    want = eval_rpn(d, load, params)
    assert eval_ssa(ssa_e, load, params) == want and eval_ssa(ssa_g, load, params) == want
