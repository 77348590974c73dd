"""GPU parity of the saturator's generated kernels against the oracle's
program interpreter (plain FP64 evaluation in the written order).

PLAIN, CSE and CSE+BULK perform exactly the written operations and must be
bit-identical to the oracle; CSE+SAT and ACCSAT reassociate and fuse, and
must be within 1e-12 relative (the workloads' terms are positive or cancel
by at most a factor of about 4, so a handful of roundings stay near 1e-15).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2306_13002_amd import saturator as X
from paper_2306_13002_amd import stencil as S
from paper_2306_13002_amd import synth

from gpu_util import maxrel

pytestmark = pytest.mark.gpu

FORMS = ["plain", "cse", "cse_sat", "cse_bulk", "accsat", "accsat_z"]
EXACT = {"plain", "cse", "cse_bulk"}
TOL = 1e-12


def dev(a):
    return torch.tensor(a, dtype=torch.float64, device="cuda")


def run(prog, n, ins_dev, params, form, tile=(0, 0), shape=None, pitch=(0, 0), zblock=0):
    shape = shape or tuple(ins_dev[0].shape)
    outs = [torch.zeros(shape, dtype=torch.float64, device="cuda") for _ in range(prog["n_outputs"])]
    plan = X.ProgramPlan(prog, n, form, tile=tile, pitch=pitch, zblock=zblock)
    plan.run(ins_dev, outs, params)
    torch.cuda.synchronize()
    plan.close()
    return [o.cpu().numpy() for o in outs]


def check(form, got, want, r):
    for o, (g, w) in enumerate(zip(got, want)):
        gi, wi = g[r:-r, r:-r, r:-r] if r else g, w[r:-r, r:-r, r:-r] if r else w
        if form in EXACT:
            assert np.array_equal(gi, wi), (form, o)
        else:
            assert maxrel(gi, wi) <= TOL, (form, o, maxrel(gi, wi))
        if r:  # the halo of every output is never written
            h = g.copy()
            h[r:-r, r:-r, r:-r] = 0.0
            assert not np.any(h), (form, o)


@pytest.mark.parametrize("form", FORMS)
def test_lhs_assembly_ragged_grid(form):
    n = (37, 13, 11)  # ragged against every block shape
    print(f"lhs {form} n={n}", flush=True)
    prog = synth.lhs_program()
    ins = synth.lhs_inputs(n)
    want = oracle.program(prog, ins, synth.LHS_PARAMS, n)
    got = run(prog, n, [dev(a) for a in ins], synth.LHS_PARAMS, form)
    check(form, got, want, 1)


@pytest.mark.parametrize("form", FORMS)
def test_heat3d7_program_forms(form):
    """The heat3d7 loop body through the saturator in every form of the
    paper's ablation, against the oracle's heat sweep (the same arithmetic
    as the program for the forms without rules)."""
    n = (37, 13, 11)
    print(f"heat3d7 program {form}", flush=True)
    u0 = synth.heat3d7_input(*n, stream=12)
    want, _ = oracle.heat(u0, 1, 0.4, 0.1)
    got = run(synth.heat3d7_program(), n, [dev(u0)], [0.4, 0.1], form, zblock=4 if form == "accsat_z" else 0)
    check(form, got, [want], 1)


@pytest.mark.parametrize("idx", range(8))
@pytest.mark.parametrize("form", FORMS)
def test_random_programs(idx, form):
    prog = synth.random_program(idx)
    n = (19, 7, 5)
    print(f"random program {idx} {form}", flush=True)
    shape = (n[2] + 2, n[1] + 2, n[0] + 2)
    ins = [synth.uniform_f64(41, s, shape) + 0.5 for s in range(prog["n_inputs"])]
    params = [0.5, 1.25, 2.0]
    want = oracle.program(prog, ins, params, n)
    got = run(prog, n, [dev(a) for a in ins], params, form)
    check(form, got, want, 1)


@pytest.mark.parametrize("zb", [1, 3, 4, 11, 64])
def test_z_streaming_equals_accsat_bitwise(zb):
    """Reusing loads along z changes where values come from, not the
    arithmetic: every z-block depth (ragged against nz = 11) gives ACCSAT's
    result bit for bit."""
    prog = synth.lhs_program()
    n = (37, 13, 11)
    d = [dev(a) for a in synth.lhs_inputs(n)]
    base = run(prog, n, d, synth.LHS_PARAMS, "accsat")
    got = run(prog, n, d, synth.LHS_PARAMS, "accsat_z", zblock=zb)
    for g, b in zip(got, base):
        assert np.array_equal(g, b)


@pytest.mark.parametrize("form", ["plain", "cse", "cse_sat", "cse_bulk", "accsat"])
@pytest.mark.parametrize("zb", [2, 3, 64])
def test_z_loop_equals_one_plane_per_thread_bitwise(form, zb):
    """The non-streaming forms with several planes per thread (a z loop that
    issues every load again) give the one-plane-per-thread result bit for
    bit, ragged z-blocks included (nz = 11)."""
    prog = synth.lhs_program()
    n = (37, 13, 11)
    d = [dev(a) for a in synth.lhs_inputs(n)]
    base = run(prog, n, d, synth.LHS_PARAMS, form)
    got = run(prog, n, d, synth.LHS_PARAMS, form, zblock=zb)
    for g, b in zip(got, base):
        assert np.array_equal(g, b)


@pytest.mark.parametrize("idx", range(4))
def test_z_streaming_random_programs_with_radius_two(idx):
    """Programs reading z offsets -2..2 (windows of up to five planes)."""
    prog = synth.random_program(200 + idx, radius=2)
    n = (21, 6, 9)
    shape = (n[2] + 4, n[1] + 4, n[0] + 4)
    ins = [synth.uniform_f64(47, s, shape) + 0.5 for s in range(prog["n_inputs"])]
    params = [0.5, 1.25, 2.0]
    want = oracle.program(prog, ins, params, n)
    d = [dev(a) for a in ins]
    got = run(prog, n, d, params, "accsat_z", zblock=4)
    check("accsat_z", got, want, 2)
    base = run(prog, n, d, params, "accsat")
    for g, b in zip(got, base):
        assert np.array_equal(g, b)


@pytest.mark.parametrize("tile", [(64, 4), (128, 2), (256, 1), (32, 8), (64, 16), (1024, 1)])
def test_block_shapes_agree_bitwise(tile):
    prog = synth.lhs_program()
    n = (70, 9, 4)
    ins = synth.lhs_inputs(n)
    d = [dev(a) for a in ins]
    base = run(prog, n, d, synth.LHS_PARAMS, "accsat", tile=(64, 4))
    got = run(prog, n, d, synth.LHS_PARAMS, "accsat", tile=tile)
    for g, b in zip(got, base):
        assert np.array_equal(g, b)


def test_pitched_arrays():
    """Rows padded to pitch_y = 48 and planes to one extra row: the kernel
    indexes with the pitches and leaves the padding alone."""
    prog = synth.random_program(3)
    n = (30, 6, 4)
    PX, PY, PZ = n[0] + 2, n[1] + 2, n[2] + 2
    py, pz = 48, 48 * (PY + 1)
    dense = [synth.uniform_f64(43, s, (PZ, PY, PX)) + 0.5 for s in range(prog["n_inputs"])]
    pitched = []
    for a in dense:
        b = np.full((PZ, PY + 1, py), np.nan)
        b[:, :PY, :PX] = a
        pitched.append(b)
    params = [0.5, 1.25, 2.0]
    want = oracle.program(prog, dense, params, n)
    got = run(prog, n, [dev(a) for a in pitched], params, "plain", shape=(PZ, PY + 1, py), pitch=(py, pz))
    for g, w in zip(got, want):
        assert np.array_equal(g[1:-1, 1:PY - 1, 1:PX - 1], w[1:-1, 1:-1, 1:-1])
        g2 = g.copy()
        g2[1:-1, 1:PY - 1, 1:PX - 1] = 0.0
        assert not np.any(g2)  # padding and halo untouched (zero-initialized)


@pytest.mark.parametrize("form,zblock", [("plain", 0), ("accsat", 0), ("accsat", 16), ("accsat_z", 0)])
def test_lhs_full_size_sampled_slabs(form, zblock):
    """The 162^3 workload at the benchmark's launch shape; the outputs of a
    point depend only on planes k-1..k+1, so the oracle runs on z-slabs of
    the inputs and is compared with the matching planes."""
    n = synth.LHS_N
    print(f"lhs full size {form}", flush=True)
    prog = synth.lhs_program()
    ins = synth.lhs_inputs(n)
    got = run(prog, n, [dev(a) for a in ins], synth.LHS_PARAMS, form, zblock=zblock)
    for k0, k1 in ((0, 2), (80, 82), (160, 162)):
        sub = [a[k0:k1 + 2] for a in ins]  # padded planes k0 .. k1+1 = interior k0-1 .. k1
        want = oracle.program(prog, sub, synth.LHS_PARAMS, (n[0], n[1], k1 - k0))
        for o in range(75):
            g = got[o][k0 + 1:k1 + 1, 1:-1, 1:-1]
            w = want[o][1:-1, 1:-1, 1:-1]
            if form in EXACT:
                assert np.array_equal(g, w), (k0, o)
            else:
                assert maxrel(g, w) <= TOL, (k0, o)


def test_overlapping_outputs_rejected():
    prog = synth.random_program(0)
    n = (8, 8, 8)
    shape = (10, 10, 10)
    ins = [torch.ones(shape, dtype=torch.float64, device="cuda") for _ in range(prog["n_inputs"])]
    outs = [torch.zeros(shape, dtype=torch.float64, device="cuda") for _ in range(prog["n_outputs"])]
    plan = X.ProgramPlan(prog, n, "cse")
    with pytest.raises(S.StencilError, match="overlaps"):
        plan.run(ins, [ins[0]] + outs[1:], [1.0, 1.0, 1.0])
    big = torch.zeros((2 * 1000 + 5,), dtype=torch.float64, device="cuda")
    with pytest.raises(S.StencilError, match="overlaps"):
        plan.run(ins, [big[0:1000], big[5:1005], outs[2]], [1.0, 1.0, 1.0])
    plan.run(ins, outs, [1.0, 1.0, 1.0])
    torch.cuda.synchronize()
    plan.close()


def test_plan_info_and_profile():
    prog = synth.lhs_program()
    n = (64, 8, 4)
    ins = [dev(a) for a in synth.lhs_inputs(n)]
    for form in ("plain", "accsat"):
        plan = X.ProgramPlan(prog, n, form)
        info = plan.info()
        assert info["regs"] > 0 and info["private_bytes"] >= 0 and info["lds_bytes"] == 0
        outs = [torch.zeros_like(ins[0]) for _ in range(75)]
        plan.profile(True)
        plan.run(ins, outs, synth.LHS_PARAMS)
        assert plan.profile_read() > 0.0
        plan.close()
