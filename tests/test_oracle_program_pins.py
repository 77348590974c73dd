"""Pins of the oracle's program interpreter (oracle_program_run).

It is checked against an independent evaluation (a pure-Python stack
machine written here, one IEEE operation per instruction, so the results
must agree bit for bit) and against closed forms of the block-tridiagonal
assembly: with zero Jacobians only the diagonal terms remain, and with
Jacobians constant along z the three blocks of a row sum to the identity
(the centred difference of a constant vanishes and the dissipation terms
-1, +2, -1 cancel), both up to rounding of a few terms.
"""
import numpy as np
import pytest

import oracle
from paper_2306_13002_amd import synth


def py_eval(prog, ins, params, n):
    r = prog["radius"]
    nx, ny, nz = n
    outs = [np.zeros_like(ins[0]) if ins else None for _ in range(prog["n_outputs"])]
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                st, loc = [], {}
                for op, a, b, c, d in prog["insns"]:
                    if op == 1:
                        st.append(float(prog["consts"][a]))
                    elif op == 2:
                        st.append(float(params[a]))
                    elif op == 3:
                        st.append(float(ins[a][k + r + d, j + r + c, i + r + b]))
                    elif op in (4, 5, 6):
                        y, x = st.pop(), st.pop()
                        st.append(x + y if op == 4 else (x - y if op == 5 else x * y))
                    elif op == 7:
                        st.append(-st.pop())
                    elif op == 8:
                        outs[a][k + r, j + r, i + r] = st.pop()
                    elif op == 9:
                        loc[a] = st.pop()
                    elif op == 10:
                        st.append(loc[a])
    return outs


@pytest.mark.parametrize("which", ["lhs", "rand0", "rand1", "rand2"])
def test_interpreter_matches_independent_evaluation_bitwise(which):
    prog = synth.lhs_program() if which == "lhs" else synth.random_program(int(which[4:]))
    n = (3, 2, 3)
    r = prog["radius"]
    shape = (n[2] + 2 * r, n[1] + 2 * r, n[0] + 2 * r)
    ins = [synth.uniform_f64(31, s, shape) * (1 + s % 3) for s in range(prog["n_inputs"])]
    params = [0.25 + 0.5 * i for i in range(prog["n_params"])]
    got = oracle.program(prog, ins, params, n)
    want = py_eval(prog, ins, params, n)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)


def lhs_blocks(outs, r=1):
    """(A, B, C) as arrays [m][n] of interior fields."""
    inner = lambda a: a[r:-r, r:-r, r:-r]  # noqa: E731
    return [[[inner(outs[25 * b + 5 * m + n]) for n in range(5)] for m in range(5)] for b in range(3)]


def test_lhs_zero_jacobians_leave_the_diagonal_terms():
    prog = synth.lhs_program()
    n = (4, 3, 5)
    shape = (n[2] + 2, n[1] + 2, n[0] + 2)
    ins = [np.zeros(shape) for _ in range(50)]
    dt, tz1, tz2, *dz = synth.LHS_PARAMS
    A, B, C = lhs_blocks(oracle.program(prog, ins, synth.LHS_PARAMS, n))
    t1 = dt * tz1
    for m in range(5):
        for q in range(5):
            if m == q:
                assert np.all(A[m][q] == -(t1 * dz[m])) and np.all(C[m][q] == -(t1 * dz[m]))
                assert np.all(B[m][q] == 1.0 + (2.0 * t1) * dz[m])
            else:
                assert np.all(A[m][q] == 0.0) and np.all(B[m][q] == 0.0) and np.all(C[m][q] == 0.0)


def test_lhs_rows_sum_to_identity_for_z_constant_jacobians():
    prog = synth.lhs_program()
    n = (5, 4, 6)
    shape = (n[2] + 2, n[1] + 2, n[0] + 2)
    rng = np.random.default_rng(5)
    ins = []
    for s in range(50):
        plane = rng.uniform(0.0, 2.0, size=(1, shape[1], shape[2]))
        ins.append(np.repeat(plane, shape[0], axis=0))
    A, B, C = lhs_blocks(oracle.program(prog, ins, synth.LHS_PARAMS, n))
    for m in range(5):
        for q in range(5):
            s = A[m][q] + B[m][q] + C[m][q]
            assert np.max(np.abs(s - (1.0 if m == q else 0.0))) < 1e-14


def test_lhs_depends_on_the_neighbour_planes():
    """A reads k-1 and C reads k+1: a change of plane z of one input moves A
    on the plane above it and C on the plane below it only."""
    prog = synth.lhs_program()
    n = (3, 3, 5)
    shape = (n[2] + 2, n[1] + 2, n[0] + 2)
    ins = synth.lhs_inputs(n)
    base = oracle.program(prog, ins, synth.LHS_PARAMS, n)
    ins2 = [a.copy() for a in ins]
    ins2[0][3] += 1.0  # F[0][0] on padded plane 3 (interior k = 2)
    moved = oracle.program(prog, ins2, synth.LHS_PARAMS, n)
    diff = [np.nonzero(np.any(moved[o] != base[o], axis=(1, 2)))[0].tolist() for o in range(75)]
    assert diff[0] == [4] and diff[50] == [2]  # A[0][0] at k = 3, C[0][0] at k = 1 (padded 4 and 2)
    assert all(d == [] for o, d in enumerate(diff) if o not in (0, 50))


def test_heat3d7_program_is_the_heat_sweep():
    """The heat3d7 loop body written as a program, run by the interpreter,
    gives the oracle's heat sweep bit for bit (same operations, same order),
    and leaves the halo at zero."""
    prog = synth.heat3d7_program()
    n = (9, 7, 5)
    u0 = synth.heat3d7_input(*n, stream=3)
    got = oracle.program(prog, [u0], [0.4, 0.1], n)[0]
    want, _ = oracle.heat(u0, 1, 0.4, 0.1)
    assert np.array_equal(got[1:-1, 1:-1, 1:-1], want[1:-1, 1:-1, 1:-1])
    h = got.copy()
    h[1:-1, 1:-1, 1:-1] = 0.0
    assert not np.any(h)


def test_malformed_program_rejected_by_the_oracle():
    bad = dict(n_inputs=1, n_outputs=1, n_params=0, n_locals=0, radius=1, insns=[(4, 0, 0, 0, 0), (8, 0, 0, 0, 0)],
               consts=[])
    with pytest.raises(ValueError):
        oracle.program(bad, [np.zeros((3, 3, 3))], [], (1, 1, 1))
