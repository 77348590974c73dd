"""Python binding of the saturator (include/saturator.h): pointwise
multi-statement programs rewritten by an e-graph and run as generated HIP.

Programs are built from expression objects::

    F, N = In(0), In(1)
    t1 = Local(0)
    prog = Program(n_inputs=2, n_outputs=1, n_params=2, n_locals=1, radius=1)
    prog.set(t1, Param(0) * Param(1))
    prog.store(0, -t1 * F.at(0, 0, -1) - t1 * N.at(0, 0, 1))

and lowered to the library's postfix instruction list.  Only argument
marshalling happens here; rewriting, generation and compilation run in
libstencil.so.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

from . import stencil as S

OP_CONST, OP_PARAM, OP_LOAD, OP_ADD, OP_SUB, OP_MUL, OP_NEG, OP_STORE, OP_SET, OP_GET = range(1, 11)
FORMS = {"plain": 0, "cse": 1, "cse_sat": 2, "cse_bulk": 3, "accsat": 4, "accsat_z": 5}
FORM_NAMES = {v: k for k, v in FORMS.items()}
EXTRACT = {"greedy": 0, "exact": 1}


class SatInsn(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("a", ctypes.c_int32), ("b", ctypes.c_int32), ("c", ctypes.c_int32),
                ("d", ctypes.c_int32)]


class SatProgramDesc(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("n_inputs", ctypes.c_int32),
        ("n_outputs", ctypes.c_int32),
        ("n_params", ctypes.c_int32),
        ("n_locals", ctypes.c_int32),
        ("n_insns", ctypes.c_int32),
        ("insns", ctypes.POINTER(SatInsn)),
        ("n_consts", ctypes.c_int32),
        ("consts", ctypes.POINTER(ctypes.c_double)),
        ("radius", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3),
        ("pitch_y", ctypes.c_int64),
        ("pitch_z", ctypes.c_int64),
    ]


class SatStats(ctypes.Structure):
    _fields_ = [
        ("enodes", ctypes.c_int32), ("eclasses", ctypes.c_int32), ("iterations", ctypes.c_int32),
        ("saturated", ctypes.c_int32), ("cost_input", ctypes.c_double), ("cost_extracted", ctypes.c_double),
        ("loads", ctypes.c_int32), ("ops", ctypes.c_int32), ("fmas", ctypes.c_int32),
        ("saturate_ms", ctypes.c_double), ("extract_ms", ctypes.c_double),
    ]


# ---------------------------------------------------------------------------
# expressions

class Expr:
    def __add__(self, o):
        return Op(OP_ADD, self, _wrap(o))

    def __radd__(self, o):
        return Op(OP_ADD, _wrap(o), self)

    def __sub__(self, o):
        return Op(OP_SUB, self, _wrap(o))

    def __rsub__(self, o):
        return Op(OP_SUB, _wrap(o), self)

    def __mul__(self, o):
        return Op(OP_MUL, self, _wrap(o))

    def __rmul__(self, o):
        return Op(OP_MUL, _wrap(o), self)

    def __neg__(self):
        return Op(OP_NEG, self)


def _wrap(v):
    return v if isinstance(v, Expr) else Const(float(v))


class Const(Expr):
    def __init__(self, v: float):
        self.v = float(v)


class Param(Expr):
    def __init__(self, i: int):
        self.i = int(i)


class Load(Expr):
    def __init__(self, a: int, dx: int = 0, dy: int = 0, dz: int = 0):
        self.a, self.off = int(a), (int(dx), int(dy), int(dz))


class In:
    """Input array a; .at(dx, dy, dz) is its load at an offset."""

    def __init__(self, a: int):
        self.a = int(a)

    def at(self, dx: int = 0, dy: int = 0, dz: int = 0) -> Load:
        return Load(self.a, dx, dy, dz)


class Local(Expr):
    def __init__(self, i: int):
        self.i = int(i)


class Op(Expr):
    def __init__(self, op: int, *args: Expr):
        self.op, self.args = op, args


class Program:
    """An ordered list of statements over one padded geometry."""

    def __init__(self, n_inputs: int, n_outputs: int, n_params: int = 0, n_locals: int = 0, radius: int = 1):
        self.n_inputs, self.n_outputs, self.n_params, self.n_locals = n_inputs, n_outputs, n_params, n_locals
        self.radius = radius
        self.insns: list[tuple[int, int, int, int, int]] = []
        self.consts: list[float] = []
        self._cidx: dict[int, int] = {}

    def _const(self, v: float) -> int:
        key = ctypes.c_uint64.from_buffer_copy(ctypes.c_double(v)).value
        if key not in self._cidx:
            self._cidx[key] = len(self.consts)
            self.consts.append(v)
        return self._cidx[key]

    def _emit(self, e: Expr):
        stack = [(e, False)]
        while stack:
            x, done = stack.pop()
            if isinstance(x, Const):
                self.insns.append((OP_CONST, self._const(x.v), 0, 0, 0))
            elif isinstance(x, Param):
                self.insns.append((OP_PARAM, x.i, 0, 0, 0))
            elif isinstance(x, Load):
                self.insns.append((OP_LOAD, x.a, *x.off))
            elif isinstance(x, Local):
                self.insns.append((OP_GET, x.i, 0, 0, 0))
            elif isinstance(x, Op):
                if done:
                    self.insns.append((x.op, 0, 0, 0, 0))
                else:
                    stack.append((x, True))
                    for a in reversed(x.args):
                        stack.append((a, False))
            else:
                raise TypeError(f"not an expression: {x!r}")

    def store(self, out: int, e: Expr):
        self._emit(_wrap(e))
        self.insns.append((OP_STORE, int(out), 0, 0, 0))

    def set(self, loc: Local, e: Expr):
        self._emit(_wrap(e))
        self.insns.append((OP_SET, loc.i, 0, 0, 0))

    @classmethod
    def from_dict(cls, d: dict) -> "Program":
        """A program given directly as postfix instructions (keys n_inputs,
        n_outputs, n_params, n_locals, radius, insns, consts)."""
        p = cls(d["n_inputs"], d["n_outputs"], d.get("n_params", 0), d.get("n_locals", 0), d.get("radius", 1))
        p.insns = [tuple(int(v) for v in t) for t in d["insns"]]
        p.consts = [float(v) for v in d.get("consts", [])]
        return p

    def to_dict(self) -> dict:
        return dict(n_inputs=self.n_inputs, n_outputs=self.n_outputs, n_params=self.n_params, n_locals=self.n_locals,
                    radius=self.radius, insns=list(self.insns), consts=list(self.consts))

    def desc(self, n: Sequence[int], pitch: Sequence[int] = (0, 0)):
        """(SatProgramDesc, keepalive)."""
        ins = (SatInsn * len(self.insns))(*[SatInsn(*t) for t in self.insns])
        cs = (ctypes.c_double * max(1, len(self.consts)))(*self.consts)
        d = SatProgramDesc()
        d.struct_size = ctypes.sizeof(SatProgramDesc)
        d.n_inputs, d.n_outputs, d.n_params, d.n_locals = self.n_inputs, self.n_outputs, self.n_params, self.n_locals
        d.n_insns = len(self.insns)
        d.insns = ctypes.cast(ins, ctypes.POINTER(SatInsn))
        d.n_consts = len(self.consts)
        d.consts = ctypes.cast(cs, ctypes.POINTER(ctypes.c_double))
        d.radius = self.radius
        nn = list(n) + [1] * (3 - len(n))
        for a in range(3):
            d.n[a] = int(nn[a])
        d.pitch_y, d.pitch_z = int(pitch[0]), int(pitch[1])
        return d, (ins, cs)


def _lib():
    L = S.lib()
    if not getattr(L, "_sat_sigs", False):
        P = ctypes.POINTER
        L.sat_generate.argtypes = [P(SatProgramDesc), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_char_p, ctypes.c_int64, ctypes.c_char_p, ctypes.c_int64,
                                   P(SatStats)]
        L.sat_plan.argtypes = [P(SatProgramDesc), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                               P(ctypes.c_void_p)]
        L.sat_run.argtypes = [ctypes.c_void_p, P(ctypes.c_void_p), P(ctypes.c_void_p), P(ctypes.c_double),
                              ctypes.c_void_p]
        L.sat_plan_info.argtypes = [ctypes.c_void_p, P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_int32)]
        L.sat_profile_enable.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        L.sat_profile_read.argtypes = [ctypes.c_void_p, P(ctypes.c_double), P(ctypes.c_int32)]
        L.sat_destroy.argtypes = [ctypes.c_void_p]
        for f in ("sat_generate", "sat_plan", "sat_run", "sat_plan_info", "sat_profile_enable", "sat_profile_read",
                  "sat_destroy"):
            getattr(L, f).restype = ctypes.c_int32
        L._sat_sigs = True
    return L


def _stats(st: SatStats) -> dict:
    return {f: getattr(st, f) for f, _ in SatStats._fields_}


def _as_program(prog) -> Program:
    return prog if isinstance(prog, Program) else Program.from_dict(prog)


def generate(prog, n: Sequence[int], form: str = "accsat", extract: str = "greedy",
             tile: Sequence[int] = (0, 0), pitch: Sequence[int] = (0, 0), zblock: int = 0):
    """Rewrite and generate on the host: (HIP source, SSA text, stats dict).
    prog: a Program or its dict form."""
    d, keep = _as_program(prog).desc(n, pitch)
    L = _lib()
    size = 1 << 16
    while True:
        src = ctypes.create_string_buffer(size)
        ssa = ctypes.create_string_buffer(size)
        st = SatStats()
        r = L.sat_generate(ctypes.byref(d), FORMS[form], EXTRACT[extract], int(tile[0]), int(tile[1]), int(zblock),
                           src, size, ssa, size, ctypes.byref(st))
        if r == S.OK:
            del keep
            return src.value.decode(), ssa.value.decode(), _stats(st)
        if r == S.E_INVAL and "buffer too small" in S.last_error() and size < (1 << 28):
            size *= 4
            continue
        raise S.StencilError(r, S.last_error())


class ProgramPlan:
    """A program compiled for one form; run() takes torch tensors."""

    def __init__(self, prog, n: Sequence[int], form: str = "accsat", tile: Sequence[int] = (0, 0),
                 pitch: Sequence[int] = (0, 0), zblock: int = 0):
        self.prog, self.form = _as_program(prog), form
        d, keep = self.prog.desc(n, pitch)
        h = ctypes.c_void_p()
        S._check(_lib().sat_plan(ctypes.byref(d), FORMS[form], int(tile[0]), int(tile[1]), int(zblock),
                                 ctypes.byref(h)))
        del keep
        self._h = h

    def run(self, inputs, outputs, params: Optional[Sequence[float]] = None, stream=None):
        for t in list(inputs) + list(outputs):
            if not t.is_cuda or t.dtype.itemsize != 8 or not t.is_contiguous():
                raise ValueError("arrays must be contiguous FP64 device tensors")
        ip = (ctypes.c_void_p * max(1, len(inputs)))(*[t.data_ptr() for t in inputs])
        op = (ctypes.c_void_p * len(outputs))(*[t.data_ptr() for t in outputs])
        pr = (ctypes.c_double * max(1, len(params or [])))(*(params or []))
        S._check(_lib().sat_run(self._h, ip, op, pr, S._stream_handle(stream)))

    def info(self) -> dict:
        r, p, l = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        S._check(_lib().sat_plan_info(self._h, ctypes.byref(r), ctypes.byref(p), ctypes.byref(l)))
        return {"regs": r.value, "private_bytes": p.value, "lds_bytes": l.value}

    def profile(self, enable: bool = True):
        S._check(_lib().sat_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self) -> float:
        ms, n = ctypes.c_double(), ctypes.c_int32()
        S._check(_lib().sat_profile_read(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib().sat_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
