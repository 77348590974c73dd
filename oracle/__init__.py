"""CPU FP64 oracle for the stencil sweeps -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP library never imports, links or
calls it, and this package never imports the HIP library.

Every function takes padded numpy grids (x contiguous, halo of width r on all
sides, see ``oracle.c``), widens FP32 inputs to FP64 exactly, runs the plain C
loop nests of ``oracle.c`` and returns new arrays (inputs are not modified).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

# Plain FP64: no fast-math, no contraction, round-to-nearest-even.
CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-std=c11", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain flags above)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        i64, dp, cint, dbl = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_double
        lib.oracle_heat_run.argtypes = [cint, i64, i64, i64, dp, dbl, dbl, cint, cint, dp]
        lib.oracle_poisson19_run.argtypes = [i64, i64, i64, dp, ctypes.POINTER(dp), dbl, cint, cint, dp]
        lib.oracle_wave25_run.argtypes = [i64, i64, i64, dp, dp, dp, dp, cint, dp]
        lib.oracle_generic_run.argtypes = [i64, i64, i64, cint, dp, cint,
                                           ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                           dp, cint, cint, cint, dp]
        lib.oracle_program_run.argtypes = [i64, i64, i64, cint, ctypes.POINTER(ctypes.c_int32), cint, dp, cint, cint,
                                           ctypes.POINTER(dp), cint, ctypes.POINTER(dp), cint, dp, cint]
        for f in (lib.oracle_heat_run, lib.oracle_poisson19_run, lib.oracle_wave25_run, lib.oracle_generic_run,
                  lib.oracle_program_run):
            f.restype = cint
        _lib = lib
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.float64).copy()


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int, name: str):
    if rc != 0:
        raise ValueError(f"oracle {name}: invalid arguments")


def heat(u, T: int, cc: float, cn: float, periodic: bool = False):
    """T sweeps of the 2-D 5-point (u.ndim == 2) or 3-D 7-point (u.ndim == 3)
    heat operator: new = cc*u + cn*(sum of face neighbours).  u is padded with
    a 1-cell halo.  Returns (u_T, residual of the last sweep)."""
    a = _f64(u)
    if a.ndim == 2:
        ny, nx = a.shape[0] - 2, a.shape[1] - 2
        nz, nd = 1, 2
    elif a.ndim == 3:
        nz, ny, nx = a.shape[0] - 2, a.shape[1] - 2, a.shape[2] - 2
        nd = 3
    else:
        raise ValueError("heat: u must be 2-D or 3-D")
    r = ctypes.c_double(0.0)
    _check(_load().oracle_heat_run(nd, nx, ny, nz, _ptr(a), cc, cn, int(T), int(bool(periodic)),
                                   ctypes.byref(r)), "heat")
    return a, r.value


POISSON_COEF_ORDER = ("a0", "a1", "a2", "a3", "b0", "b1", "b2", "c0", "c1", "c2", "bnd", "wrk1")


def poisson19(p, coefs, omega: float, T: int, mode: str = "F64"):
    """T relaxation sweeps of the 19-point variable-coefficient pressure
    operator (formula in oracle.c).  p and the 12 coefficient arrays (list in
    POISSON_COEF_ORDER order) are padded 3-D grids with a 1-cell halo.
    mode "F64" keeps p in FP64; "F32STORE" rounds every stored p to FP32.
    Returns (p_T as float64, residual = sum ss^2 of the last sweep)."""
    a = _f64(p)
    if a.ndim != 3 or len(coefs) != 12:
        raise ValueError("poisson19: p must be 3-D and coefs must hold 12 arrays")
    cs = [_f64(c) for c in coefs]
    for c in cs:
        if c.shape != a.shape:
            raise ValueError("poisson19: coefficient shape mismatch")
    arr = (ctypes.POINTER(ctypes.c_double) * 12)(*[_ptr(c) for c in cs])
    nz, ny, nx = a.shape[0] - 2, a.shape[1] - 2, a.shape[2] - 2
    g = ctypes.c_double(0.0)
    m = {"F64": 0, "F32STORE": 1}[mode]
    _check(_load().oracle_poisson19_run(nx, ny, nz, _ptr(a), arr, float(omega), int(T), m, ctypes.byref(g)),
           "poisson19")
    return a, g.value


def wave25(a, b, vsq, c, T: int):
    """T leapfrog steps of the radius-4 25-point wave update.  a = u^{n-1},
    b = u^n, vsq: padded grids with a 4-cell halo; c = (c0, c1, c2, c3, c4).
    Each step overwrites the older buffer's interior in place.  Returns
    (a_T, b_T, residual): after T steps the newest level is in a when T is
    odd and in b when T is even."""
    A, B, V = _f64(a), _f64(b), _f64(vsq)
    if A.ndim != 3 or A.shape != B.shape or A.shape != V.shape:
        raise ValueError("wave25: three padded 3-D grids of equal shape are required")
    cc = np.ascontiguousarray(np.asarray(c, dtype=np.float64))
    if cc.shape != (5,):
        raise ValueError("wave25: 5 coefficients required")
    nz, ny, nx = A.shape[0] - 8, A.shape[1] - 8, A.shape[2] - 8
    r = ctypes.c_double(0.0)
    _check(_load().oracle_wave25_run(nx, ny, nz, _ptr(A), _ptr(B), _ptr(V), _ptr(cc), int(T), ctypes.byref(r)),
           "wave25")
    return A, B, r.value


def generic(u, radius: int, tap_off, tap_cid, coef, T: int, mode: str = "F64"):
    """T sweeps of u'(x) = sum_t coef[cid_t] * u(x + delta_t) in tap-list
    order.  u: padded 3-D grid with halo `radius`; tap_off: (n_taps, 3) ints
    (dx, dy, dz); tap_cid: n_taps ints.  Returns (u_T, residual)."""
    a = _f64(u)
    off = np.ascontiguousarray(np.asarray(tap_off, dtype=np.int32).reshape(-1, 3))
    cid = np.ascontiguousarray(np.asarray(tap_cid, dtype=np.int32).reshape(-1))
    cf = np.ascontiguousarray(np.asarray(coef, dtype=np.float64).reshape(-1))
    if a.ndim != 3 or off.shape[0] != cid.shape[0]:
        raise ValueError("generic: bad shapes")
    r = int(radius)
    nz, ny, nx = a.shape[0] - 2 * r, a.shape[1] - 2 * r, a.shape[2] - 2 * r
    res = ctypes.c_double(0.0)
    m = {"F64": 0, "F32STORE": 1}[mode]
    i32p = ctypes.POINTER(ctypes.c_int32)
    _check(_load().oracle_generic_run(nx, ny, nz, r, _ptr(a), int(cid.shape[0]), off.ctypes.data_as(i32p),
                                      cid.ctypes.data_as(i32p), _ptr(cf), int(cf.shape[0]), int(T), m,
                                      ctypes.byref(res)), "generic")
    return a, res.value


def program(prog: dict, inputs, params, n):
    """Run a pointwise program once (see oracle_program_run in oracle.c).

    prog: dict with n_inputs, n_outputs, n_params, n_locals, radius, insns
    (list of (op, a, b, c, d)) and consts; inputs: padded 3-D arrays (halo
    radius); params: n_params floats; n: interior (nx, ny, nz).  Returns the
    n_outputs padded output arrays (halo 0, interior written)."""
    r = int(prog["radius"])
    nx, ny, nz = (int(v) for v in n)
    shape = (nz + 2 * r, ny + 2 * r, nx + 2 * r)
    ins = [_f64(a) for a in inputs]
    for a in ins:
        if a.shape != shape:
            raise ValueError("program: input shape does not match n and radius")
    outs = [np.zeros(shape, dtype=np.float64) for _ in range(int(prog["n_outputs"]))]
    code = np.ascontiguousarray(np.asarray(prog["insns"], dtype=np.int32).reshape(-1, 5))
    cs = np.ascontiguousarray(np.asarray(list(prog["consts"]) + [0.0], dtype=np.float64))
    pr = np.ascontiguousarray(np.asarray(list(params) + [0.0], dtype=np.float64))
    dp = ctypes.POINTER(ctypes.c_double)
    in_arr = (dp * max(1, len(ins)))(*[_ptr(a) for a in ins])
    out_arr = (dp * len(outs))(*[_ptr(a) for a in outs])
    _check(_load().oracle_program_run(nx, ny, nz, r, code.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      int(code.shape[0]), _ptr(cs), len(prog["consts"]), len(ins), in_arr,
                                      len(outs), out_arr, int(prog["n_params"]), _ptr(pr), int(prog["n_locals"])),
           "program")
    return outs
