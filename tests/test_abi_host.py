"""Host-side contract of the C ABI (runs without a GPU): the library loads,
exports every entry point include/stencil.h declares, and rejects bad
descriptors on the host before touching a device."""
import ctypes
import os
import re

import pytest

from paper_2306_13002_amd import stencil as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "stencil.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(stencil_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = S.lib()
    syms = header_symbols()
    assert "stencil_plan" in syms and "stencil_run" in syms and "stencil_residual" in syms
    for name in syms:
        assert hasattr(L, name), name


def test_struct_layout_matches_header():
    # the library checks struct_size == sizeof(stencil_desc): a descriptor that
    # passes every check reaches the device probe (E_DEVICE without a GPU)
    d, keep = S.make_desc("heat3d7", (10, 10, 10), coef=(0.4, 0.1))
    st, h = S.plan_status(d)
    if st == S.OK:
        S.lib().stencil_destroy(ctypes.c_void_p(h))
    assert st in (S.OK, S.E_DEVICE), S.last_error()
    d.struct_size = ctypes.sizeof(S.StencilDesc) - 8
    assert S.plan_status(d)[0] == S.E_INVAL
    assert "struct_size" in S.last_error()


BAD = [
    (dict(kind="heat3d7", n=(10, 10, 0), coef=(0.4, 0.1)), S.E_INVAL, "n[2]"),
    (dict(kind="heat3d7", n=(10, 10, 10)), S.E_INVAL, "coef"),
    (dict(kind="heat3d7", n=(10, 10, 10), coef=(0.4, 0.1), radius=2), S.E_INVAL, "radius"),
    (dict(kind="wave25", n=(10, 10, 10), coef=(1, 2, 3)), S.E_INVAL, "5 coefficients"),
    (dict(kind="wave25", n=(10, 10, 10), coef=(1, 2, 3, 4, 5), dtype="f32"), S.E_UNSUPPORTED, "F64"),
    (dict(kind="poisson19", n=(10, 10, 10), dtype="f64"), S.E_UNSUPPORTED, "F32"),
    (dict(kind="poisson19", n=(10, 10, 10), omega=float("nan")), S.E_INVAL, "omega"),
    (dict(kind="heat3d7", n=(10, 10, 10), coef=(0.4, 0.1), pitch=(11, 0)), S.E_INVAL, "pitch_y"),
    (dict(kind="heat3d7", n=(10, 10, 10), coef=(0.4, 0.1), pitch=(12, 100)), S.E_INVAL, "pitch_z"),
    (dict(kind="wave25", n=(10, 10, 10), coef=(1, 2, 3, 4, 5), bc="periodic"), S.E_UNSUPPORTED, "periodic"),
    (dict(kind="heat3d7", n=(10, 10, 10), coef=(0.4, float("inf"))), S.E_INVAL, "finite"),
    (dict(kind="generic", n=(10, 10, 10), coef=(1.0,), taps=[(5, 0, 0)], cids=[0], radius=4), S.E_INVAL, "radius"),
    (dict(kind="generic", n=(10, 10, 10), coef=(1.0,), taps=[(1, 0, 0)], cids=[3], radius=1), S.E_INVAL, "id"),
    (dict(kind="wave25", n=(10, 10, 10), coef=(1, 2, 3, 4, 5), variant="saturated_t2"), S.E_UNSUPPORTED, "two-sweep"),
    (dict(kind="heat3d7", n=(10, 10, 10), coef=(0.4, 0.1), variant="saturated_t2", bc="periodic"), S.E_UNSUPPORTED,
     "two-sweep"),
    (dict(kind="generic", n=(10, 10, 10), coef=(1.0,), taps=[(1, 0, 0)], cids=[0], radius=1, variant="saturated_t2"),
     S.E_UNSUPPORTED, "two-sweep"),
    (dict(kind="poisson19", n=(10, 10, 10), variant="saturated_t3"), S.E_UNSUPPORTED, "three-sweep"),
    (dict(kind="heat3d7", n=(10, 10, 10), coef=(0.4, 0.1), variant="saturated_t3", bc="periodic"), S.E_UNSUPPORTED,
     "three-sweep"),
]


@pytest.mark.parametrize("kw,status,msg", BAD)
def test_bad_descriptors_rejected_on_host(kw, status, msg):
    kw = dict(kw)
    kind, n = kw.pop("kind"), kw.pop("n")
    d, keep = S.make_desc(kind, n, **kw)
    st, h = S.plan_status(d)
    assert st == status, (st, S.last_error())
    assert h is None
    assert msg in S.last_error()


def test_generated_kernels_refuse_grids_the_module_launch_cannot_take():
    """Saturated GENERIC kernels and generated programs are launched through
    hipModuleLaunchKernel (y and z grid dimensions up to 65535): taller
    grids are refused on the host, before any device call."""
    L = S.lib()
    taps = [(0, 0, 0), (1, 0, 0), (0, 0, -1)]
    for variant, status in (("saturated", S.E_UNSUPPORTED), ("auto", S.E_UNSUPPORTED)):
        d, keep = S.make_desc("generic", (4, 4, 70000), dtype="f64", radius=1, coef=(0.5, 0.25), taps=taps,
                              cids=[0, 1, 1], variant=variant)
        h = ctypes.c_void_p()
        assert L.stencil_plan(ctypes.byref(d), ctypes.byref(h)) == status
        assert "65535" in S.last_error()


def test_null_arguments():
    L = S.lib()
    h = ctypes.c_void_p()
    assert L.stencil_plan(None, ctypes.byref(h)) == S.E_INVAL
    d, keep = S.make_desc("heat3d7", (4, 4, 4), coef=(0.4, 0.1))
    assert L.stencil_plan(ctypes.byref(d), None) == S.E_INVAL
    assert L.stencil_run(None, None, None, 1, None) == S.E_INVAL
    out = ctypes.c_double()
    assert L.stencil_residual(None, ctypes.byref(out), None) == S.E_INVAL
    assert L.stencil_destroy(None) == S.OK
    c = ctypes.c_int32()
    assert L.stencil_batch_problem_config(None, 0, ctypes.byref(c), None, None, None, None) == S.E_INVAL
    assert "batch" in S.last_error()
    assert isinstance(S.last_error(), str)
    assert L.stencil_version().decode().endswith("gfx950")


def test_ablation_forms_only_for_wave_and_pressure():
    d, keep = S.make_desc("heat3d7", (10, 10, 10), coef=(0.4, 0.1), variant="cse_sat")
    assert S.plan_status(d)[0] == S.E_UNSUPPORTED and "ablation" in S.last_error()
    d, keep = S.make_desc("wave25", (10, 10, 10), coef=(1, 2, 3, 4, 5), variant="cse_bulk")
    assert S.plan_status(d)[0] in (S.OK, S.E_DEVICE)
